"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Every test here runs on the CPU.  Each one is chosen so that a plausible slip in the
oracle (a dropped term, a sign, a conjugate, a transposed index, an off-by-one in the
window or the shear) fails at least one of them:

* hand-computed index tables of the tiny workload, rounding of halves;
* the Fourier transform against a brute-force double sum, Parseval and the inverse;
* the projection against brute-force loops, its adjoint by the dot-product test and the
  textbook special case (no shear, one slice: psi = P * O);
* a closed-form single Bragg spot for the whole forward model;
* zero loss and zero gradient at the truth, a hand value of the amplitude metric;
* invariances of eq. (6) / eq. (7) (lattice vectors, the per-peak 2*pi family, a
  constant shift) and their consequence sum(df/du) = 0;
* Euler homogeneity of f in chi and alpha;
* central finite differences of the full objective;
* the minibatch sum of eq. (11) over a partition of the frames;
* the optimiser of Algorithm 1: Adam against closed forms (constant gradient, sign
  steps, a two-step worked example, invariance to gradient scale), the eq. (8) chain
  rule against finite differences in the log variables, and the loops' invariants.
"""
import math

import numpy as np
import pytest

from oracle import mpbp_oracle as O
from synth import get_config, make_problem, make_fields
from tests.conftest import tiny_problem, random_fields, ragged


# ----------------------------------------------------------------- index tables ---

@pytest.mark.parametrize("v,expect", [
    (0.5, 1), (-0.5, -1), (1.5, 2), (-1.5, -2), (2.5, 3), (-2.5, -3),
    (0.49999999999999994, 0), (-0.49999999999999994, 0), (0.0, 0), (-0.0, 0),
    (1e-300, 0), (0.5000000000000001, 1), (2.4999999999999996, 2), (-7.2, -7), (6.6, 7),
])
def test_round_half_away(v, expect):
    assert O.round_half_away(v) == expect


def test_tiny_workload_tables_by_hand():
    # Workload c1_tiny: nz = 8 (reference slice 4), 5 x 5 raster at step 4 from (0, 0),
    # window 32, probe 16.  Shear per slice worked out by hand from
    # t = tan(theta) * (G_y, G_x)/|G_xy| and round-half-away((z - 4) * t).
    prob = make_problem(get_config("c1_tiny"))
    tab = O.tables(prob)
    s111 = [-1, -1, 0, 0, 0, 0, 0, 1]
    sm111_y = [-1, -1, -1, 0, 0, 0, 1, 1]
    s1m11_y = [1, 1, 1, 0, 0, 0, -1, -1]
    np.testing.assert_array_equal(tab["shear"][0, :, 0], s111)
    np.testing.assert_array_equal(tab["shear"][0, :, 1], s111)
    np.testing.assert_array_equal(tab["shear"][1, :, 0], sm111_y)
    np.testing.assert_array_equal(tab["shear"][1, :, 1], [-v for v in sm111_y])
    np.testing.assert_array_equal(tab["shear"][2, :, 0], s1m11_y)
    np.testing.assert_array_equal(tab["shear"][2, :, 1], [-v for v in s1m11_y])
    assert tab["scan"].shape == (75, 2)
    for m in range(3):
        for iy in range(5):
            for ix in range(5):
                f = 25 * m + 5 * iy + ix
                assert tuple(tab["scan"][f]) == (4 * iy, 4 * ix)
    np.testing.assert_array_equal(tab["y_off"], [0, 25600, 51200, 76800])
    np.testing.assert_array_equal(tab["offset"], [8, 8, 8])


def test_raster_with_unequal_steps_by_hand():
    # Raster scan (section 4): frame (iy, ix) at origin + (iy step_y, ix step_x), raster
    # order; a 2 x 3 raster with steps (3, 5) from (-1, 2), written out.
    got = O.scan_positions((2, 3), (3, 5), (-1, 2))
    np.testing.assert_array_equal(got, [[-1, 2], [-1, 7], [-1, 12], [2, 2], [2, 7], [2, 12]])


def test_large_workload_geometry_readings():
    # Raster origins / steps and footprint spans of the larger workloads, worked out by
    # hand from the centring rule (N - ((n-1) step + Np)) // 2.
    c4 = make_problem(get_config("c4_batch"))
    np.testing.assert_array_equal(c4.scan_step, [[11, 11], [9, 8], [7, 7], [6, 7], [5, 5], [8, 8]])
    np.testing.assert_array_equal(c4.scan_origin, [[7, 7], [8, 4], [3, 3], [7, 10], [14, 14], [4, 4]])
    tab = O.tables(c4)
    spans = [(tab["shear"][m].min(axis=0).tolist(), tab["shear"][m].max(axis=0).tolist())
             for m in range(6)]
    assert spans[3] == ([0, -10], [0, 9])       # (200): 32 x 51 footprint
    assert spans[4] == ([-6, 0], [5, 0])        # (020): 43 x 32 footprint
    c5 = make_problem(get_config("c5_full"))
    np.testing.assert_array_equal(c5.scan_origin, [[-12, -12]] * 3)
    assert c5.n_frames() == 12288


def test_footprint_outside_window_is_rejected():
    prob = tiny_problem(dets=(8, 9), shears=((3.0, 0.0), (0.0, 0.0)))
    with pytest.raises(O.FootprintError):
        O.tables(prob)
    prob = tiny_problem(dets=(3, 9))
    with pytest.raises(O.FootprintError):
        O.tables(prob)


# ---------------------------------------------------------- Fourier transform ---

def _dft2_bruteforce(x):
    d0, d1 = x.shape
    out = np.zeros_like(x, dtype=np.complex128)
    for k0 in range(d0):
        for k1 in range(d1):
            s = 0j
            for n0 in range(d0):
                for n1 in range(d1):
                    s += x[n0, n1] * complex(math.cos(-2 * math.pi * (k0 * n0 / d0 + k1 * n1 / d1)),
                                             math.sin(-2 * math.pi * (k0 * n0 / d0 + k1 * n1 / d1)))
            out[k0, k1] = s / math.sqrt(d0 * d1)
    return out


@pytest.mark.parametrize("d", [4, 6, 8, 12, 16])
def test_far_field_is_orthonormal_dft(d):
    rng = np.random.default_rng(d)
    x = rng.normal(size=(d, d)) + 1j * rng.normal(size=(d, d))
    ref = _dft2_bruteforce(x)
    got = O.far_field(x)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
    # Parseval and the inverse
    assert abs(np.sum(np.abs(got) ** 2) - np.sum(np.abs(x) ** 2)) <= 1e-12 * np.sum(np.abs(x) ** 2)
    back = O.far_field_adjoint(got)
    assert np.max(np.abs(back - x)) <= 1e-12 * np.max(np.abs(x))


# ----------------------------------------------------------------- projection ---

def _exit_wave_bruteforce(o_m, probe_m, py, px, shear_m, det):
    nz, ny, nx = o_m.shape
    n = probe_m.shape[0]
    c = (det - n) // 2
    psi = np.zeros((det, det), dtype=np.complex128)
    for z in range(nz):
        for a in range(n):
            for b in range(n):
                yy, xx = py + a, px + b
                if 0 <= yy < ny and 0 <= xx < nx:
                    psi[a + c + shear_m[z, 0], b + c + shear_m[z, 1]] += probe_m[a, b] * o_m[z, yy, xx]
    return psi


def test_exit_wave_matches_bruteforce_loops():
    prob = tiny_problem()
    tab = O.tables(prob)
    u, chi, alpha, probe = random_fields(prob, seed=3)
    obj = O.objects(u, chi, alpha, prob)
    nonzero_shear = False
    for fid in range(prob.n_frames()):
        m = tab["peak_of_frame"][fid]
        py, px = tab["scan"][fid]
        det = int(prob.det[m])
        got = O.exit_wave(obj[m], probe[m], py, px, tab["shear"][m], det)
        ref = _exit_wave_bruteforce(obj[m], probe[m], py, px, tab["shear"][m], det)
        assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))
        nonzero_shear |= bool(np.any(tab["shear"][m] != 0))
    assert nonzero_shear


def test_projection_adjoint_dot_product():
    prob = tiny_problem()
    tab = O.tables(prob)
    rng = np.random.default_rng(7)
    shape = (prob.nz, prob.ny, prob.nx)
    for fid in range(prob.n_frames()):
        m = tab["peak_of_frame"][fid]
        py, px = tab["scan"][fid]
        det = int(prob.det[m])
        p = rng.normal(size=(prob.probe_n,) * 2) + 1j * rng.normal(size=(prob.probe_n,) * 2)
        o = rng.normal(size=shape) + 1j * rng.normal(size=shape)
        w = rng.normal(size=(det, det)) + 1j * rng.normal(size=(det, det))
        ao = O.exit_wave(o, p, py, px, tab["shear"][m], det)
        ahw = np.zeros(shape, dtype=np.complex128)
        O.back_project(w, p, py, px, tab["shear"][m], ahw)
        lhs = np.vdot(w, ao)          # <w, A o>
        rhs = np.vdot(ahw, o)         # <A^H w, o>
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_projection_textbook_case():
    # No shear, one slice: the exit wave is P * O on the window (2D ptychography).
    prob = tiny_problem(nz=1, shears=((0.0, 0.0), (0.0, 0.0)))
    tab = O.tables(prob)
    u, chi, alpha, probe = random_fields(prob, seed=5)
    obj = O.objects(u, chi, alpha, prob)
    fid = 1                      # peak 0, frame (0, 1): py = -1 (one row off-grid), px = 4
    py, px = tab["scan"][fid]
    assert (py, px) == (-1, 4)
    psi = O.exit_wave(obj[0], probe[0], py, px, tab["shear"][0], 8)
    c = 2
    ref = np.zeros((8, 8), dtype=np.complex128)
    ref[c + 1:c + 4, c:c + 4] = probe[0][1:4, :] * obj[0][0, 0:3, 4:8]
    np.testing.assert_allclose(psi, ref, rtol=0, atol=1e-15)


# --------------------------------------------------------- closed-form spot ---

@pytest.mark.parametrize("k0", [0, 3, 5])
def test_single_bragg_spot(k0):
    # Flat probe filling the window (Np = D), no shear, chi = 1 on T slices, and a
    # displacement ramp making G.u = 2 pi k0 x / D: every slice adds the same plane wave,
    # so the far field is one spot of modulus alpha * D * T at (0, k0).
    from synth.inputs import Problem
    d, nz, t = 8, 4, 3
    gx = 7.5
    prob = Problem("spot", nz, d, d, d, np.array([[gx, 0.0, 0.0]]), np.zeros((1, 2)),
                   np.array([d]), np.array([[1, 1]]), np.array([[1, 1]]), np.array([[0, 0]]))
    x = np.arange(d, dtype=np.float64)
    u = np.zeros((3, nz, d, d))
    u[0] = (2 * math.pi * k0 * x / d / gx)[None, None, :]
    chi = np.zeros((nz, d, d))
    chi[:t] = 1.0
    alpha = np.array([1.7])
    probe = np.ones((1, d, d), dtype=np.complex128)
    inten = O.model_intensity(u, chi, alpha, probe, prob)[0]
    ref = np.zeros((d, d))
    ref[0, k0] = (alpha[0] * d * t) ** 2
    np.testing.assert_allclose(inten, ref, rtol=1e-12, atol=1e-9)


# ----------------------------------------------------------- amplitude metric ---

def test_amplitude_metric_hand_value():
    f, r = O.amplitude_residual(np.array([[3 + 4j, 0j]]), np.array([[16.0, 4.0]]))
    # (5 - 4)^2 / 2 + (0 - 2)^2 / 2 ; residual 0 where |Psi| = 0
    assert f == pytest.approx(0.5 + 2.0, rel=1e-15)
    assert r[0, 0] == pytest.approx((3 + 4j) / 5, rel=1e-15)
    assert r[0, 1] == 0


def _noiseless(prob, u, chi, alpha, probe):
    return ragged(O.model_intensity(u, chi, alpha, probe, prob))


def test_zero_loss_and_gradient_at_truth():
    prob = tiny_problem()
    u, chi, alpha, probe = random_fields(prob, seed=11)
    y = _noiseless(prob, u, chi, alpha, probe)
    r = O.loss_grad(u, chi, alpha, probe, y, prob)
    assert r["loss"] <= 1e-24 * np.sum(y)
    for k in ("grad_u", "grad_chi", "grad_alpha"):
        assert np.max(np.abs(r[k])) <= 1e-10


# ------------------------------------------------------------- invariances ---

def _c1_like():
    cfg = get_config("c1_tiny")
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    return prob, f


def test_lattice_vector_and_per_peak_invariance():
    prob, f = _c1_like()
    u = f["u"].astype(np.float64)
    chi, alpha, probe = f["chi"], f["alpha"], f["probe"]
    base = O.model_intensity(u, chi, alpha, probe, prob)
    rng = np.random.default_rng(2)
    # u + a * n, n integer per voxel: every G_m . (a n) is a multiple of 2 pi.
    a = 0.2 * math.sqrt(3.0)
    n = rng.integers(-1, 2, size=u.shape).astype(np.float64)
    moved = O.model_intensity(u + a * n, chi, alpha, probe, prob)
    for b, mv in zip(base, moved):
        np.testing.assert_allclose(mv, b, rtol=1e-9, atol=1e-9 * b.max())
    # Per-peak family: u + 2 pi m G_1 / |G_1|^2 with m in {-1, 0, 1} per voxel (Fig. 2)
    # and the alternating +-5 pattern (eq. (7)) keep peak 1's data, not the others'.
    g1 = prob.g[0]
    for mfield in (rng.integers(-1, 2, size=u.shape[1:]).astype(np.float64),
                   5.0 * (-1.0) ** np.indices(u.shape[1:]).sum(axis=0)):
        shift = 2 * math.pi * mfield[None] * (g1 / np.dot(g1, g1))[:, None, None, None]
        moved = O.model_intensity(u + shift, chi, alpha, probe, prob)
        for fid in range(prob.n_frames()):
            b, mv = base[fid], moved[fid]
            if fid < 25:
                np.testing.assert_allclose(mv, b, rtol=1e-9, atol=1e-9 * b.max())
        assert max(np.max(np.abs(moved[f] - base[f])) for f in range(25, 75)) > 1e-3 * base[30].max()


def test_constant_shift_invariance_and_zero_gradient_sum():
    prob = tiny_problem()
    u, chi, alpha, probe = random_fields(prob, seed=13)
    rng = np.random.default_rng(14)
    y = ragged(O.model_intensity(u + rng.normal(0, 0.05, size=u.shape), chi, alpha, probe, prob))
    l0, _ = O.loss(u, chi, alpha, probe, y, prob)
    l1, _ = O.loss(u + np.array([0.3, -0.7, 1.1])[:, None, None, None], chi, alpha, probe, y, prob)
    assert abs(l1 - l0) <= 1e-11 * l0
    r = O.loss_grad(u, chi, alpha, probe, y, prob)
    for c in range(3):
        assert abs(r["grad_u"][c].sum()) <= 1e-10 * np.abs(r["grad_u"][c]).sum()


# ------------------------------------------------------------ homogeneity ---

def test_euler_homogeneity_chi_and_alpha():
    prob = tiny_problem()
    u, chi, alpha, probe = random_fields(prob, seed=17)
    rng = np.random.default_rng(18)
    y = ragged(O.model_intensity(u + rng.normal(0, 0.05, size=u.shape), chi * 1.1, alpha, probe, prob))
    r = O.loss_grad(u, chi, alpha, probe, y, prob)
    tab = O.tables(prob)
    inten = O.model_intensity(u, chi, alpha, probe, prob)
    per_peak = np.zeros(prob.n_peaks)
    for fid, it in enumerate(inten):
        a = np.sqrt(it)
        yy = O.frame_data(y, tab, prob, fid)
        per_peak[tab["peak_of_frame"][fid]] += np.sum((a - np.sqrt(yy)) * a)
    assert np.sum(chi * r["grad_chi"]) == pytest.approx(per_peak.sum(), rel=1e-10)
    np.testing.assert_allclose(alpha * r["grad_alpha"], per_peak, rtol=1e-10)


# ----------------------------------------------------------------- support ---

def test_gradient_support():
    prob = tiny_problem()
    u, chi, alpha, probe = random_fields(prob, seed=19, chi_zero_frac=0.3)
    rng = np.random.default_rng(20)
    y = ragged(O.model_intensity(u + rng.normal(0, 0.05, size=u.shape), chi, alpha, probe, prob))
    r = O.loss_grad(u, chi, alpha, probe, y, prob)
    zero = chi == 0
    assert zero.any()
    for c in range(3):
        assert np.all(r["grad_u"][c][zero] == 0.0)
    # voxels no window covers get nothing
    tab = O.tables(prob)
    covered = np.zeros((prob.ny, prob.nx), dtype=bool)
    for py, px in tab["scan"]:
        covered[max(py, 0):max(py + prob.probe_n, 0), max(px, 0):max(px + prob.probe_n, 0)] = True
    assert (~covered).any()
    assert np.all(r["grad_chi"][:, ~covered] == 0.0)
    assert np.all(r["grad_u"][:, :, ~covered] == 0.0)


def test_in_plane_peaks_give_no_out_of_plane_gradient():
    # Bragg vectors in the membrane plane (l = 0, the paper's setting): df/du_z = 0.
    prob = tiny_problem(gs=[(9.0, -4.0, 0.0), (-3.0, 7.0, 0.0)])
    u, chi, alpha, probe = random_fields(prob, seed=21)
    rng = np.random.default_rng(22)
    y = ragged(O.model_intensity(u + rng.normal(0, 0.05, size=u.shape), chi, alpha, probe, prob))
    r = O.loss_grad(u, chi, alpha, probe, y, prob)
    assert np.all(r["grad_u"][2] == 0.0)
    assert np.abs(r["grad_u"][0]).max() > 0


# ------------------------------------------------------- finite differences ---

def test_gradient_matches_central_differences():
    prob = tiny_problem()
    u, chi, alpha, probe = random_fields(prob, seed=23)
    rng = np.random.default_rng(24)
    y = ragged(O.model_intensity(u + rng.normal(0, 0.05, size=u.shape), chi * 0.9, alpha * 1.2,
                                 probe, prob))
    r = O.loss_grad(u, chi, alpha, probe, y, prob)

    def f(uu, cc, aa):
        return O.loss(uu, cc, aa, probe, y, prob)[0]

    scale_u = np.abs(r["grad_u"]).max()
    for _ in range(12):
        c = int(rng.integers(3))
        idx = tuple(int(rng.integers(s)) for s in u.shape[1:])
        h = 1e-6
        up, um = u.copy(), u.copy()
        up[(c,) + idx] += h
        um[(c,) + idx] -= h
        fd = (f(up, chi, alpha) - f(um, chi, alpha)) / (2 * h)
        assert fd == pytest.approx(r["grad_u"][(c,) + idx], abs=1e-6 * scale_u)
    scale_c = np.abs(r["grad_chi"]).max()
    for _ in range(8):
        idx = tuple(int(rng.integers(s)) for s in chi.shape)
        h = 1e-6
        cp, cm = chi.copy(), chi.copy()
        cp[idx] += h
        cm[idx] -= h
        fd = (f(u, cp, alpha) - f(u, cm, alpha)) / (2 * h)
        assert fd == pytest.approx(r["grad_chi"][idx], abs=1e-6 * scale_c)
    for m in range(prob.n_peaks):
        h = 1e-6
        ap, am = alpha.copy(), alpha.copy()
        ap[m] += h
        am[m] -= h
        fd = (f(u, chi, ap) - f(u, chi, am)) / (2 * h)
        assert fd == pytest.approx(r["grad_alpha"][m], rel=1e-6)


def test_tied_membrane_gradient_matches_central_differences():
    # Unknowns per lateral pixel, constant along x3 (section 3): perturbing one tied
    # variable moves the whole voxel column.
    prob = tiny_problem()
    rng = np.random.default_rng(25)
    u2 = rng.normal(0, 0.1, size=(3, 1, prob.ny, prob.nx))
    chi2 = rng.uniform(0.5, 1.5, size=(1, prob.ny, prob.nx))
    _, _, alpha, probe = random_fields(prob, seed=26)
    y = ragged(O.model_intensity(np.broadcast_to(u2 + rng.normal(0, 0.05, size=u2.shape),
                                                 (3, prob.nz, prob.ny, prob.nx)),
                                 np.broadcast_to(chi2, (prob.nz, prob.ny, prob.nx)), alpha, probe, prob))
    r = O.loss_grad_ztied(u2, chi2, alpha, probe, y, prob)

    def f(uu, cc):
        return O.loss(np.broadcast_to(uu, (3, prob.nz, prob.ny, prob.nx)),
                      np.broadcast_to(cc, (prob.nz, prob.ny, prob.nx)), alpha, probe, y, prob)[0]

    scale = np.abs(r["grad_u"]).max()
    for _ in range(6):
        c, yy, xx = int(rng.integers(3)), int(rng.integers(prob.ny)), int(rng.integers(prob.nx))
        h = 1e-6
        up, um = u2.copy(), u2.copy()
        up[c, 0, yy, xx] += h
        um[c, 0, yy, xx] -= h
        fd = (f(up, chi2) - f(um, chi2)) / (2 * h)
        assert fd == pytest.approx(r["grad_u"][c, 0, yy, xx], abs=1e-6 * scale)


# ------------------------------------------------------------------ subsets ---

def test_minibatch_partition_sums():
    prob = tiny_problem()
    u, chi, alpha, probe = random_fields(prob, seed=27)
    rng = np.random.default_rng(28)
    y = ragged(O.model_intensity(u + rng.normal(0, 0.05, size=u.shape), chi, alpha, probe, prob))
    full = O.loss_grad(u, chi, alpha, probe, y, prob)
    perm = rng.permutation(prob.n_frames())
    parts = [perm[:4], perm[4:7], perm[7:]]
    acc = {k: 0.0 for k in ("loss", "grad_u", "grad_chi", "grad_alpha")}
    for p in parts:
        r = O.loss_grad(u, chi, alpha, probe, y, prob, frames=p)
        for k in acc:
            acc[k] = acc[k] + r[k]
    assert acc["loss"] == pytest.approx(full["loss"], rel=1e-12)
    for k in ("grad_u", "grad_chi", "grad_alpha"):
        np.testing.assert_allclose(acc[k], full[k], rtol=1e-10, atol=1e-12 * np.abs(full[k]).max())
    with pytest.raises(ValueError):
        O.loss(u, chi, alpha, probe, y, prob, frames=[0, 0])


# --------------------------------------------------------- paper geometry ---

def test_exit_wave_pixel_matches_table_1_voxel():
    # Table 1: lambda = 1.377 A, 150 px of 55 um at 0.35 m.  The far-field sampling
    # lambda z / (D p) reproduces the 5.84 nm voxel of section 4, the reading that the
    # exit-wave pixel equals the object voxel.
    pitch_nm = 1.377e-10 * 0.35 / (150 * 55e-6) * 1e9
    assert pitch_nm == pytest.approx(5.84, abs=0.005)


# ------------------------------------------------------------------ optimiser ---
def test_adam_constant_gradient_closed_form():
    """With a constant gradient the bias-corrected moments are g and g^2 at every step,
    so each Adam update is exactly lr g / (|g| + eps)."""
    g = np.array([2.5, -0.3, 1e-3, -40.0])
    p, m, v = np.zeros(4), np.zeros(4), np.zeros(4)
    for t in range(1, 8):
        q, m, v = O.adam_update(p, g, m, v, t, lr=0.1, beta1=0.9, beta2=0.999, eps=1e-8)
        np.testing.assert_allclose(q - p, -0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)
        p = q


def test_adam_two_step_worked_example():
    """beta1 = 1/2, beta2 = 3/4, lr = 1, eps = 0, gradients 1 then 3:
    m = 1/2, 7/4; v = 1/4, 39/16; corrected m = 1, 7/3; corrected v = 1, 39/7;
    steps 1 and (7/3) / sqrt(39/7)."""
    p, m, v = np.zeros(1), np.zeros(1), np.zeros(1)
    p1, m, v = O.adam_update(p, [1.0], m, v, 1, lr=1.0, beta1=0.5, beta2=0.75, eps=0.0)
    assert p1[0] == pytest.approx(-1.0, rel=1e-15)
    assert (m[0], v[0]) == (0.5, 0.25)
    p2, m, v = O.adam_update(p1, [3.0], m, v, 2, lr=1.0, beta1=0.5, beta2=0.75, eps=0.0)
    assert (m[0], v[0]) == (1.75, 2.4375)
    assert p2[0] - p1[0] == pytest.approx(-(7.0 / 3.0) / math.sqrt(39.0 / 7.0), rel=1e-14)


def test_adam_scale_invariance_and_sign_steps():
    rng = np.random.default_rng(5)
    gs = rng.normal(size=(6, 10))
    pa = pb = np.zeros(10)
    ma = va = mb = vb = np.zeros(10)
    for t, g in enumerate(gs, start=1):
        pa, ma, va = O.adam_update(pa, g, ma, va, t, lr=0.01, eps=0.0)
        pb, mb, vb = O.adam_update(pb, 1e4 * g, mb, vb, t, lr=0.01, eps=0.0)
    np.testing.assert_allclose(pa, pb, rtol=1e-12, atol=1e-15)
    # no momentum, no averaging: a pure sign step of size lr
    q, _, _ = O.adam_update(np.zeros(10), gs[0], np.zeros(10), np.zeros(10), 1, lr=0.2, beta1=0.0, beta2=0.0,
                            eps=0.0)
    np.testing.assert_allclose(q, -0.2 * np.sign(gs[0]), rtol=1e-15)


def test_log_variables_chain_rule_matches_finite_differences():
    """eq. (8): with chi = exp(chi~), alpha = exp(alpha~), df/dchi~ = chi df/dchi."""
    prob = tiny_problem()
    u, chi, alpha, probe = random_fields(prob, seed=41)
    rng = np.random.default_rng(42)
    y = ragged(O.model_intensity(u + rng.normal(0, 0.05, size=u.shape), chi * 1.1, alpha * 0.8, probe, prob))
    cl, al = np.log(chi), np.log(alpha)
    r = O.loss_grad(u, chi, alpha, probe, y, prob)
    gcl = O.log_param_grad(chi, r["grad_chi"])
    gal = O.log_param_grad(alpha, r["grad_alpha"])

    def f(c, a):
        return O.loss(u, np.exp(c), np.exp(a), probe, y, prob)[0]

    h = 1e-6
    for _ in range(6):
        idx = tuple(int(rng.integers(s)) for s in chi.shape)
        cp, cm = cl.copy(), cl.copy()
        cp[idx] += h
        cm[idx] -= h
        assert (f(cp, al) - f(cm, al)) / (2 * h) == pytest.approx(gcl[idx], abs=1e-6 * np.abs(gcl).max())
    for m in range(prob.n_peaks):
        ap, am = al.copy(), al.copy()
        ap[m] += h
        am[m] -= h
        assert (f(cl, ap) - f(cl, am)) / (2 * h) == pytest.approx(gal[m], rel=1e-6)


def test_adam_reconstruct_invariants():
    """Algorithm 1 (no unwrap projection) on a tiny noiseless problem started near the
    truth: the loss falls, the reference alpha stays fixed, every minibatch is b
    consecutive frames of the shuffled order."""
    prob = tiny_problem()
    u, chi, alpha, probe = random_fields(prob, seed=51)
    y = ragged(O.model_intensity(u, chi, alpha, probe, prob))
    rng = np.random.default_rng(52)
    order = np.concatenate([rng.permutation(prob.n_frames()) for _ in range(12)])
    u0 = u + rng.normal(0, 0.02, size=u.shape)
    out_u, cl, al, losses = O.adam_reconstruct(u0, np.log(chi), np.log(alpha) + 0.05, probe, y, prob, order,
                                               batch=prob.n_frames(), iterations=12, lr=(0.002, 0.01, 0.01),
                                               fixed_alpha=0)
    assert al[0] == pytest.approx(np.log(alpha[0]) + 0.05, abs=0.0)
    assert losses[-1] < 0.5 * losses[0]
    full = O.loss(u0, chi, alpha * np.exp(0.05), probe, y, prob)[0]
    assert losses[0] == pytest.approx(full, rel=1e-12)      # batch = all frames: the full loss


def test_line_search_descent_invariants():
    prob = tiny_problem()
    u, chi, alpha, probe = random_fields(prob, seed=61)
    y = ragged(O.model_intensity(u, chi, alpha, probe, prob))
    u0 = u + np.random.default_rng(62).normal(0, 0.03, size=u.shape)
    out, losses, etas = O.line_search_descent(u0, chi, alpha, probe, y, prob, iterations=8)
    assert len(etas) == len(losses) == 8
    assert all(b < a for a, b in zip(losses, losses[1:]))
    assert O.loss(out, chi, alpha, probe, y, prob)[0] < losses[-1]


# ---------------------------------------------------------- background (eq. (2)) ---

def _background(prob, seed, scale):
    rng = np.random.default_rng(seed)
    n = sum(int(prob.det[m]) ** 2 * int(prob.scan_n[m].prod()) for m in range(prob.n_peaks))
    return rng.uniform(0.0, scale, n)


def test_background_zero_is_no_background():
    prob = tiny_problem()
    u, chi, alpha, probe = random_fields(prob, seed=61)
    rng = np.random.default_rng(62)
    y = ragged(O.model_intensity(u + rng.normal(0, 0.05, size=u.shape), chi, alpha, probe, prob))
    a = O.loss_grad(u, chi, alpha, probe, y, prob)
    b = O.loss_grad(u, chi, alpha, probe, y, prob, background=np.zeros_like(y))
    for k in ("loss", "grad_u", "grad_chi", "grad_alpha"):
        np.testing.assert_array_equal(a[k], b[k])


def test_background_closed_form_without_object():
    # chi = 0: the exit wave vanishes, I = b, f = 1/2 sum (sqrt(b) - sqrt(y))^2 and every
    # gradient is 0 (the residual's direction Psi / sqrt(I) is 0)
    prob = tiny_problem()
    u, chi, alpha, probe = random_fields(prob, seed=63)
    bg = _background(prob, 64, 3.0)
    y = np.random.default_rng(65).uniform(0.0, 5.0, bg.size)
    r = O.loss_grad(u, np.zeros_like(chi), alpha, probe, y, prob, background=bg)
    assert r["loss"] == pytest.approx(0.5 * np.sum((np.sqrt(bg) - np.sqrt(y)) ** 2), rel=1e-12)
    assert not r["grad_u"].any() and not r["grad_chi"].any()
    inten = O.model_intensity(u, np.zeros_like(chi), alpha, probe, prob, background=bg)
    np.testing.assert_array_equal(np.concatenate([i.ravel() for i in inten]), bg)


def test_background_zero_loss_at_truth_and_central_differences():
    prob = tiny_problem()
    u, chi, alpha, probe = random_fields(prob, seed=66)
    rng = np.random.default_rng(67)
    bg = _background(prob, 68, 2.0)
    y0 = ragged(O.model_intensity(u, chi, alpha, probe, prob, background=bg))
    r0 = O.loss_grad(u, chi, alpha, probe, y0, prob, background=bg)
    assert r0["loss"] < 1e-20 and np.abs(r0["grad_u"]).max() < 1e-9
    y = ragged(O.model_intensity(u + rng.normal(0, 0.05, size=u.shape), chi * 0.9, alpha, probe, prob,
                                 background=bg))
    r = O.loss_grad(u, chi, alpha, probe, y, prob, background=bg)
    f = lambda uu, cc: O.loss(uu, cc, alpha, probe, y, prob, background=bg)[0]
    scale_u, scale_c = np.abs(r["grad_u"]).max(), np.abs(r["grad_chi"]).max()
    for _ in range(8):
        c = int(rng.integers(3))
        idx = tuple(int(rng.integers(s)) for s in u.shape[1:])
        up, um = u.copy(), u.copy()
        up[(c,) + idx] += 1e-6
        um[(c,) + idx] -= 1e-6
        assert (f(up, chi) - f(um, chi)) / 2e-6 == pytest.approx(r["grad_u"][(c,) + idx], abs=1e-6 * scale_u)
    for _ in range(6):
        idx = tuple(int(rng.integers(s)) for s in chi.shape)
        cp, cm = chi.copy(), chi.copy()
        cp[idx] += 1e-6
        cm[idx] -= 1e-6
        assert (f(u, cp) - f(u, cm)) / 2e-6 == pytest.approx(r["grad_chi"][idx], abs=1e-6 * scale_c)


# -------------------------------------------------- 3D illumination (section 2) ---

def _exit_wave_bruteforce_3d(o_m, probe3, py, px, shear_m, det):
    nz, ny, nx = o_m.shape
    n = probe3.shape[-1]
    c = (det - n) // 2
    psi = np.zeros((det, det), dtype=np.complex128)
    for z in range(nz):
        for a in range(n):
            for b in range(n):
                yy, xx = py + a, px + b
                if 0 <= yy < ny and 0 <= xx < nx:
                    psi[a + c + shear_m[z, 0], b + c + shear_m[z, 1]] += probe3[z, a, b] * o_m[z, yy, xx]
    return psi


def _probe3(prob, seed):
    rng = np.random.default_rng(seed)
    s = (prob.n_peaks, prob.nz, prob.probe_n, prob.probe_n)
    return rng.normal(size=s) + 1j * rng.normal(size=s)


def test_3d_probe_projection_bruteforce_and_adjoint():
    prob = tiny_problem()
    tab = O.tables(prob)
    u, chi, alpha, _ = random_fields(prob, seed=81)
    p3 = _probe3(prob, 82)
    obj = O.objects(u, chi, alpha, prob)
    rng = np.random.default_rng(83)
    for fid in range(prob.n_frames()):
        m = tab["peak_of_frame"][fid]
        py, px = tab["scan"][fid]
        det = int(prob.det[m])
        got = O.exit_wave(obj[m], p3[m], py, px, tab["shear"][m], det)
        ref = _exit_wave_bruteforce_3d(obj[m], p3[m], py, px, tab["shear"][m], det)
        assert np.max(np.abs(got - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))
        w = rng.normal(size=(det, det)) + 1j * rng.normal(size=(det, det))
        ahw = np.zeros(obj[m].shape, dtype=np.complex128)
        O.back_project(w, p3[m], py, px, tab["shear"][m], ahw)
        assert abs(np.vdot(w, got) - np.vdot(ahw, obj[m])) <= 1e-12 * max(1.0, abs(np.vdot(w, got)))


def test_3d_probe_constant_along_x3_is_the_2d_probe():
    prob = tiny_problem()
    u, chi, alpha, probe = random_fields(prob, seed=84)
    p3 = np.repeat(probe[:, None], prob.nz, axis=1)
    rng = np.random.default_rng(85)
    y = ragged(O.model_intensity(u + rng.normal(0, 0.05, size=u.shape), chi, alpha, probe, prob))
    a = O.loss_grad(u, chi, alpha, probe, y, prob)
    b = O.loss_grad(u, chi, alpha, p3, y, prob)
    for k in ("loss", "grad_u", "grad_chi", "grad_alpha"):
        np.testing.assert_array_equal(a[k], b[k])


def test_3d_probe_gradient_matches_central_differences():
    prob = tiny_problem()
    u, chi, alpha, _ = random_fields(prob, seed=86)
    p3 = _probe3(prob, 87) * 0.3
    rng = np.random.default_rng(88)
    y = ragged(O.model_intensity(u + rng.normal(0, 0.05, size=u.shape), chi, alpha, p3, prob))
    r = O.loss_grad(u, chi, alpha, p3, y, prob)
    f = lambda uu, cc: O.loss(uu, cc, alpha, p3, y, prob)[0]
    scale_u, scale_c = np.abs(r["grad_u"]).max(), np.abs(r["grad_chi"]).max()
    for _ in range(8):
        c = int(rng.integers(3))
        idx = tuple(int(rng.integers(s)) for s in u.shape[1:])
        up, um = u.copy(), u.copy()
        up[(c,) + idx] += 1e-6
        um[(c,) + idx] -= 1e-6
        assert (f(up, chi) - f(um, chi)) / 2e-6 == pytest.approx(r["grad_u"][(c,) + idx], abs=1e-6 * scale_u)
    for _ in range(6):
        idx = tuple(int(rng.integers(s)) for s in chi.shape)
        cp, cm = chi.copy(), chi.copy()
        cp[idx] += 1e-6
        cm[idx] -= 1e-6
        assert (f(u, cp) - f(u, cm)) / 2e-6 == pytest.approx(r["grad_chi"][idx], abs=1e-6 * scale_c)


# ------------------------------------------- interpolating exit-beam offsets (R) ---

def _linear(prob):
    import dataclasses
    return dataclasses.replace(prob, shear_linear=True)


def _exit_wave_tent(o_m, probe_m, py, px, shear_t, det, nz):
    # bilinear sampling written with the tent kernel of the continuous offset
    # s(z) = (z - nz//2) t: psi[q] = sum_z sum_e W_z[e] K(q - c - e - s(z)),
    # K(d) = max(0, 1 - |d_y|) max(0, 1 - |d_x|)
    ny, nx = o_m.shape[1:]
    n = probe_m.shape[0]
    c = (det - n) // 2
    psi = np.zeros((det, det), dtype=np.complex128)
    for z in range(nz):
        s = ((z - nz // 2) * shear_t[0], (z - nz // 2) * shear_t[1])
        for a in range(n):
            for b in range(n):
                yy, xx = py + a, px + b
                if not (0 <= yy < ny and 0 <= xx < nx):
                    continue
                w = probe_m[a, b] * o_m[z, yy, xx]
                for qy in range(det):
                    ky = max(0.0, 1.0 - abs(qy - c - a - s[0]))
                    if ky == 0.0:
                        continue
                    for qx in range(det):
                        kx = max(0.0, 1.0 - abs(qx - c - b - s[1]))
                        if kx:
                            psi[qy, qx] += ky * kx * w
    return psi


def test_linear_offsets_match_the_tent_kernel_and_adjoint():
    prob = _linear(tiny_problem())
    tab = O.tables(prob)
    assert (tab["shear_frac"] > 0).any()
    u, chi, alpha, probe = random_fields(prob, seed=101)
    obj = O.objects(u, chi, alpha, prob)
    rng = np.random.default_rng(102)
    for fid in range(prob.n_frames()):
        m = tab["peak_of_frame"][fid]
        py, px = tab["scan"][fid]
        det = int(prob.det[m])
        got = O.exit_wave(obj[m], probe[m], py, px, tab["shear"][m], det, tab["shear_frac"][m])
        ref = _exit_wave_tent(obj[m], probe[m], py, px, prob.shear[m], det, prob.nz)
        assert np.max(np.abs(got - ref)) <= 1e-12 * max(1.0, np.max(np.abs(ref)))
        w = rng.normal(size=(det, det)) + 1j * rng.normal(size=(det, det))
        ahw = np.zeros(obj[m].shape, dtype=np.complex128)
        O.back_project(w, probe[m], py, px, tab["shear"][m], ahw, tab["shear_frac"][m])
        assert abs(np.vdot(w, got) - np.vdot(ahw, obj[m])) <= 1e-12 * max(1.0, abs(np.vdot(w, got)))


def test_linear_offsets_conserve_each_slice_and_reduce_to_integer_shears():
    # the bilinear weights of a slice sum to 1: the exit wave's sum is sum_z sum P O_z
    prob = _linear(tiny_problem())
    tab = O.tables(prob)
    u, chi, alpha, probe = random_fields(prob, seed=103)
    obj = O.objects(u, chi, alpha, prob)
    py, px = 2, 2                 # support inside the grid
    det = int(prob.det[0])
    psi = O.exit_wave(obj[0], probe[0], py, px, tab["shear"][0], det, tab["shear_frac"][0])
    n = prob.probe_n
    assert psi.sum() == pytest.approx(np.sum(probe[0][None] * obj[0][:, py:py + n, px:px + n]), rel=1e-12)
    # integral offsets: the interpolating projection is the rounded one
    pint = tiny_problem(shears=((1.0, -1.0), (0.0, 1.0)))
    a = O.loss_grad(u, chi, alpha, probe, _y(pint, u, chi, alpha, probe), pint)
    b = O.loss_grad(u, chi, alpha, probe, _y(pint, u, chi, alpha, probe), _linear(pint))
    for k in ("loss", "grad_u", "grad_chi", "grad_alpha"):
        np.testing.assert_allclose(b[k], a[k], rtol=1e-13, atol=1e-13 * np.abs(a[k]).max())


def _y(prob, u, chi, alpha, probe):
    rng = np.random.default_rng(104)
    return ragged(O.model_intensity(u + rng.normal(0, 0.05, size=u.shape), chi, alpha, probe, prob))


def test_linear_offsets_gradient_matches_central_differences():
    prob = _linear(tiny_problem())
    u, chi, alpha, probe = random_fields(prob, seed=105)
    y = _y(prob, u, chi, alpha, probe)
    r = O.loss_grad(u, chi, alpha, probe, y, prob)
    f = lambda uu, cc: O.loss(uu, cc, alpha, probe, y, prob)[0]
    rng = np.random.default_rng(106)
    scale_u, scale_c = np.abs(r["grad_u"]).max(), np.abs(r["grad_chi"]).max()
    for _ in range(8):
        c = int(rng.integers(3))
        idx = tuple(int(rng.integers(s)) for s in u.shape[1:])
        up, um = u.copy(), u.copy()
        up[(c,) + idx] += 1e-6
        um[(c,) + idx] -= 1e-6
        assert (f(up, chi) - f(um, chi)) / 2e-6 == pytest.approx(r["grad_u"][(c,) + idx], abs=1e-6 * scale_u)
    for _ in range(6):
        idx = tuple(int(rng.integers(s)) for s in chi.shape)
        cp, cm = chi.copy(), chi.copy()
        cp[idx] += 1e-6
        cm[idx] -= 1e-6
        assert (f(u, cp) - f(u, cm)) / 2e-6 == pytest.approx(r["grad_chi"][idx], abs=1e-6 * scale_c)
