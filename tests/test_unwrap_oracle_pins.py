"""Pins of the phase-unwrap oracle (eqs. (9)-(10) and the unwrapping it uses) against
what the mathematics fixes, independently of the oracle's own formulas:

* wrap: range, 2 pi periodicity, closed values;
* reliability: closed forms of the second differences of quadratic phases (each of the
  four directions contributes 2c, 8c or 0 depending on the quadratic's orientation);
* edge order: a strict total order, ties broken by a bijective hash;
* merging: on tiny grids the edges that join groups are the maximum spanning tree under
  that order (brute force over every spanning tree), and the unwrapped phase is the sum of
  wrapped differences along that tree;
* residue-free maps: the unwrapped phase equals numpy's one-dimensional unwrapping along
  the first column and then along every row (a library routine), up to one 2 pi multiple;
* the global offset rounds the mean wrap count, halves up;
* Pi_U: leaves a smooth field unchanged, removes lattice-translation artefacts exactly,
  is idempotent, and with coplanar Bragg vectors keeps the component no peak sees.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import unwrap_oracle as U
from synth import get_config, lattice_jump, make_problem, unwrap_field
from synth.inputs import LATTICE_A_NM, bragg_vector

TWO_PI = 2.0 * math.pi


def test_wrap_range_and_period():
    rng = np.random.default_rng(1)
    phi = rng.uniform(-60, 60, 4000).astype(np.float32)
    psi, q = U.wrap(phi)
    assert psi.dtype == np.float32 and q.dtype == np.int64
    assert np.all(np.abs(psi) <= math.pi * (1 + 1e-6))
    np.testing.assert_allclose(phi.astype(np.float64), psi + TWO_PI * q, atol=2e-5)
    assert U.wrap(np.float32(1.5 * math.pi))[0] == pytest.approx(-0.5 * math.pi, abs=1e-6)
    assert U.wrap(np.float32(-7.0))[0] == pytest.approx(-7.0 + TWO_PI, abs=1e-6)
    assert U.wrap(np.float32(0.25))[0] == np.float32(0.25)


@pytest.mark.parametrize("kind, expect", [
    ("ii", 2.0 * math.sqrt(3.0)),      # H = 0, V = D1 = D2 = 2c
    ("jj", 2.0 * math.sqrt(3.0)),      # V = 0, H = D1 = D2 = 2c
    ("i+j", 6.0 * math.sqrt(2.0)),     # H = V = 2c, D1 = 8c, D2 = 0
    ("i-j", 6.0 * math.sqrt(2.0)),     # H = V = 2c, D1 = 0, D2 = 8c
])
def test_reliability_quadratic_closed_form(kind, expect):
    c = 0.02          # first differences stay below pi; the values wrap several times
    i, j = np.meshgrid(np.arange(14.0), np.arange(11.0), indexing="ij")
    t = {"ii": i, "jj": j, "i+j": i + j, "i-j": i - j}[kind]
    phi = (c * t * t).astype(np.float32)
    R = U.reliability(U.wrap(phi)[0])
    np.testing.assert_allclose(R[1:-1, 1:-1], 1.0 / (expect * c), rtol=2e-4)
    assert (R[0] == 0).all() and (R[-1] == 0).all() and (R[:, 0] == 0).all() and (R[:, -1] == 0).all()


def test_reliability_is_wrap_invariant():
    # the measure sees only wrapped first differences: adding 2 pi multiples changes nothing
    rng = np.random.default_rng(2)
    phi = (np.cumsum(rng.uniform(-1, 1, (9, 12)), axis=1)).astype(np.float32)
    psi = U.wrap(phi)[0]
    k = rng.integers(-3, 4, phi.shape)
    psi2 = U.wrap((psi + TWO_PI * k).astype(np.float32))[0]
    np.testing.assert_allclose(U.reliability(psi2), U.reliability(psi), rtol=1e-4)


def test_edge_reliability_is_the_sum_of_its_pixels():
    # The method's edge reliability is the sum of the two pixels' reliabilities; on a 2 x 2
    # map the edges are (0,1), (2,3) (rows) then (0,2), (1,3) (columns).
    R = np.array([[0.1, 5.0], [2.0, 2.0]], dtype=np.float32)
    p, q = U.edge_list(2, 2)
    np.testing.assert_array_equal(p, [0, 2, 0, 1])
    np.testing.assert_array_equal(q, [1, 3, 2, 3])
    np.testing.assert_allclose(U.edge_keys(R, p, q), [5.1, 4.0, 2.1, 7.0], rtol=1e-6)
    np.testing.assert_array_equal(U.edge_order(U.edge_keys(R, p, q)), [3, 0, 1, 2])


def test_fmix32_bijective_and_order_total():
    h = U.fmix32(np.arange(1 << 16))
    assert len(np.unique(h)) == 1 << 16 and int(U.fmix32(0)) == 0
    rng = np.random.default_rng(3)
    keys = rng.integers(0, 5, 300).astype(np.float32)      # many ties
    keys[::7] = np.inf
    o = U.edge_order(keys)
    assert sorted(o.tolist()) == list(range(300))
    tie = U.fmix32(np.arange(300))
    for a, b in zip(o[:-1], o[1:]):
        assert keys[a] > keys[b] or (keys[a] == keys[b] and tie[a] < tie[b])


def _spanning_trees(ny, nx, p, q):
    npx, ne = ny * nx, len(p)
    for sub in itertools.combinations(range(ne), npx - 1):
        parent = list(range(npx))

        def find(x):
            while parent[x] != x:
                x = parent[x]
            return x
        ok = True
        for e in sub:
            a, b = find(int(p[e])), find(int(q[e]))
            if a == b:
                ok = False
                break
            parent[a] = b
        if ok:
            yield sub


@pytest.mark.parametrize("ny, nx, seed", [(3, 3, 0), (3, 3, 1), (3, 4, 2), (2, 5, 3)])
def test_merging_follows_maximum_spanning_tree(ny, nx, seed):
    rng = np.random.default_rng(seed)
    p, q = U.edge_list(ny, nx)
    keys = rng.integers(0, 4, len(p)).astype(np.float32)   # ties on purpose
    order = U.edge_order(keys)
    rank = np.empty(len(p), dtype=np.int64)
    rank[order] = np.arange(len(p))
    # the maximum spanning tree of the strict order = the tree whose edges, weighted
    # 2^(E - rank), have the largest sum (brute force)
    best = max(_spanning_trees(ny, nx, p, q), key=lambda t: sum(1 << int(len(p) - rank[e]) for e in t))
    psi = rng.uniform(-math.pi, math.pi, (ny, nx)).astype(np.float32)
    n, joined = U.merge_groups(psi, order, p, q, record=True)
    assert sorted(joined) == sorted(best)
    # the unwrapped phase along each tree edge steps by the wrapped difference
    unw = psi.ravel().astype(np.float64) + TWO_PI * n
    for e in best:
        a, b = int(p[e]), int(q[e])
        d = float(np.float32(psi.ravel()[b] - psi.ravel()[a]))
        step = d - TWO_PI * round(d / TWO_PI)
        assert unw[b] - unw[a] == pytest.approx(step, abs=1e-5)


@pytest.mark.parametrize("shape", [(40, 40), (23, 57)])
def test_residue_free_map_matches_numpy_unwrap(shape):
    ny, nx = shape
    i, j = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    phi = (0.9 * j + 0.02 * (i - ny / 2) ** 2 + 3.0 * np.sin(i / 7.0) * np.cos(j / 9.0)).astype(np.float32)
    psi, q = U.wrap(phi)
    n = U.unwrap_map(psi)
    got = psi.astype(np.float64) + TWO_PI * n
    col = np.unwrap(psi[:, 0].astype(np.float64))
    ref = np.stack([np.unwrap(psi[r].astype(np.float64)) + (col[r] - psi[r, 0]) for r in range(ny)])
    d = got - ref
    assert np.allclose(d, d.flat[0], atol=1e-4)
    assert abs(d.flat[0] / TWO_PI - round(d.flat[0] / TWO_PI)) < 1e-6
    # with the map's own wrap counts, the mean rule recovers phi itself
    n2 = U.unwrap_map(psi, q)
    np.testing.assert_array_equal(n2, q)


def test_global_offset_rounds_half_up():
    assert U.global_offset([0, 1], [0, 0]) == 1       # mean 0.5
    assert U.global_offset([-1, 0], [0, 0]) == 0      # mean -0.5
    assert U.global_offset([3, 3, 4], [0, 0, 0]) == 3  # mean 3.33
    assert U.global_offset([0, 0, 0], [2, 2, 1]) == -2  # mean -1.67


@pytest.fixture(scope="module")
def g3():
    return make_problem(get_config("c1_tiny")).g       # (111), (-111), (1-11): full rank


def test_projector_leaves_smooth_field_unchanged(g3):
    u = unwrap_field(2, 40, 36, seed=11)
    phi = U.phase_maps(u, g3)
    assert np.abs(phi).max() > 3 * math.pi              # the maps do wrap
    out, wraps = U.unwrap_projector(u, g3, return_wraps=True)
    assert not wraps.any()
    np.testing.assert_allclose(out, u, atol=2e-6)


def test_projector_removes_lattice_jump(g3):
    u = unwrap_field(2, 40, 36, seed=12)
    bad = lattice_jump(u, 5, 19, 8, 22, cells=1)
    out, wraps = U.unwrap_projector(bad, g3, return_wraps=True)
    np.testing.assert_allclose(out, u, atol=2e-6)
    h = np.round(np.asarray(g3)[:, 0] * LATTICE_A_NM / TWO_PI).astype(int)   # h of each peak
    for m in range(3):
        exp = np.zeros((2, 40, 36), dtype=np.int64)
        exp[:, 5:19, 8:22] = -h[m]
        np.testing.assert_array_equal(wraps[m], exp)


def test_projector_idempotent_with_residues(g3):
    u = unwrap_field(1, 32, 32, seed=13, noise_nm=0.08)
    v = U.unwrap_projector(u, g3).astype(np.float32)
    w, wraps = U.unwrap_projector(v, g3, return_wraps=True)
    assert not wraps.any()
    np.testing.assert_allclose(w, v, atol=2e-6)


def test_projector_coplanar_peaks_keep_unseen_component():
    g = np.stack([bragg_vector(h) for h in ((2, 0, 0), (0, 2, 0), (1, 1, 0))])
    u = unwrap_field(1, 30, 30, seed=14)
    bad = lattice_jump(u, 4, 15, 6, 20, cells=1)
    out = U.unwrap_projector(bad, g)
    np.testing.assert_allclose(out[:2], u[:2], atol=2e-6)
    np.testing.assert_array_equal(out[2], bad[2].astype(np.float64))
