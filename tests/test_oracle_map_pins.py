"""Pins of the oracle's detector-frame map of R (section 2: R rotates and interpolates the
illuminated object into each peak's detector frame, whose exit-wave pixel size may differ
per peak), CPU only.

With problem.lateral_map[m] = M, slice z's probe-window point (a, b) lands on the exit-wave
point q = M ((a, b) - n/2) + (c + n/2) + (z - nz//2) t_m, and each exit-wave pixel takes the
bilinear interpolation of the illuminated slice at its pre-image.  Checked against:
  * M = identity: the interpolated-offset model (problem.shear_linear) exactly, and with
    integral offsets the rounded model;
  * a brute-force sum with the tent kernel, written independently of the tap code;
  * the adjoint dot product of the projection and the back-projection;
  * closed forms: a quarter turn and a factor-2 scale put every sample on a pixel;
  * central differences of the objective;
  * the window check.
"""
import dataclasses
import math

import numpy as np
import pytest

from oracle import mpbp_oracle as O
from synth.inputs import detector_map
from tests.conftest import random_fields, ragged, tiny_problem


def _mapped(prob, maps):
    return dataclasses.replace(prob, lateral_map=np.asarray(maps, dtype=np.float64))


def _prob(shears=((0.37, -0.21), (-0.45, 0.18)), dets=(14, 16)):
    return tiny_problem(nz=3, dets=dets, shears=shears)


def test_identity_map_is_the_interpolated_offset_model():
    prob = _prob()
    u, chi, alpha, probe = random_fields(prob, seed=201)
    lin = dataclasses.replace(prob, shear_linear=True)
    mp = _mapped(prob, [np.eye(2)] * prob.n_peaks)
    a = O.model_intensity(u, chi, alpha, probe, lin)
    b = O.model_intensity(u, chi, alpha, probe, mp)
    for x, y in zip(a, b):
        np.testing.assert_allclose(y, x, rtol=1e-12, atol=1e-12 * x.max())
    y = ragged(O.model_intensity(u + np.random.default_rng(2010).normal(0, 0.05, size=u.shape), chi, alpha, probe,
                                 lin))
    ra, rb = O.loss_grad(u, chi, alpha, probe, y, lin), O.loss_grad(u, chi, alpha, probe, y, mp)
    assert rb["loss"] == pytest.approx(ra["loss"], rel=1e-12)
    for k in ("grad_u", "grad_chi", "grad_alpha"):
        np.testing.assert_allclose(rb[k], ra[k], rtol=1e-10, atol=1e-12 * np.abs(ra[k]).max())


def test_identity_map_with_integral_offsets_is_the_rounded_model():
    prob = _prob(shears=((1.0, -2.0), (0.0, 1.0)))        # (z - 1) t integral for nz = 3
    u, chi, alpha, probe = random_fields(prob, seed=202)
    mp = _mapped(prob, [np.eye(2)] * prob.n_peaks)
    for x, y in zip(O.model_intensity(u, chi, alpha, probe, prob), O.model_intensity(u, chi, alpha, probe, mp)):
        np.testing.assert_allclose(y, x, rtol=1e-12, atol=1e-12 * x.max())


def _brute_force_psi(o_m, probe_m, py, px, prob, m):
    """psi[q] = sum_z sum_{a,b} tent(p_y - a) tent(p_x - b) ill_z[a, b], with
    p = M^-1 (q - centre - (z - nz//2) t) + n/2 and tent(d) = max(0, 1 - |d|)."""
    mat = np.asarray(prob.lateral_map[m], dtype=np.float64)
    minv = np.linalg.inv(mat)
    n, det, nz = prob.probe_n, int(prob.det[m]), prob.nz
    centre = (det - n) // 2 + n / 2.0
    psi = np.zeros((det, det), dtype=np.complex128)
    for z in range(nz):
        off = (z - nz // 2) * np.asarray(prob.shear[m], dtype=np.float64)
        for qy in range(det):
            for qx in range(det):
                r = np.array([qy - centre - off[0], qx - centre - off[1]])
                p = minv @ r + n / 2.0
                total = 0.0 + 0.0j
                for a in range(n):
                    for b in range(n):
                        w = max(0.0, 1 - abs(p[0] - a)) * max(0.0, 1 - abs(p[1] - b))
                        oy, ox = py + a, px + b
                        if w and 0 <= oy < o_m.shape[1] and 0 <= ox < o_m.shape[2]:
                            total += w * probe_m[a, b] * o_m[z, oy, ox]
                psi[qy, qx] += total
    return psi


def test_mapped_projection_against_brute_force_tent_sum():
    prob = tiny_problem(nz=2, ny=9, nx=8, probe_n=4, dets=(12,), shears=((0.35, -0.6),), scan_n=((2, 2),),
                        steps=((3, 3),), origins=((-1, 1),), gs=[(3.0, -2.0, 1.5)])
    prob = _mapped(prob, [detector_map(1.2, 0.3)])
    u, chi, alpha, probe = random_fields(prob, seed=203)
    obj = O.objects(u, chi, alpha, prob)
    tab = O.tables(prob)
    for fid in range(prob.n_frames()):
        py, px = (int(v) for v in tab["scan"][fid])
        got = O.exit_wave_mapped(obj[0], probe[0], py, px, prob, 0)
        ref = _brute_force_psi(obj[0], probe[0], py, px, prob, 0)
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
        assert np.abs(ref).max() > 0


def test_mapped_adjoint_dot_product():
    prob = _mapped(_prob(), [detector_map(1.3, 0.4), detector_map(0.8, -1.1)])
    rng = np.random.default_rng(204)
    u, chi, alpha, probe = random_fields(prob, seed=204)
    tab = O.tables(prob)
    for m in range(prob.n_peaks):
        det = int(prob.det[m])
        fid = int(np.flatnonzero(tab["peak_of_frame"] == m)[0])
        py, px = (int(v) for v in tab["scan"][fid])
        x = rng.normal(size=(prob.nz, prob.ny, prob.nx)) + 1j * rng.normal(size=(prob.nz, prob.ny, prob.nx))
        w = rng.normal(size=(det, det)) + 1j * rng.normal(size=(det, det))
        ax = O.exit_wave_mapped(x, probe[m], py, px, prob, m)
        aw = np.zeros_like(x)
        O.back_project_mapped(w, probe[m], py, px, prob, m, aw)
        lhs, rhs = np.vdot(w, ax), np.vdot(aw, x)
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_quarter_turn_and_factor_two_place_every_sample_on_a_pixel():
    n, det = 4, 16
    prob = tiny_problem(nz=1, ny=6, nx=6, probe_n=n, dets=(det, det), shears=((0.0, 0.0), (0.0, 0.0)),
                        scan_n=((1, 1), (1, 1)), steps=((1, 1), (1, 1)), origins=((1, 1), (1, 1)))
    prob = _mapped(prob, [[[0.0, -1.0], [1.0, 0.0]], [[2.0, 0.0], [0.0, 2.0]]])
    u, chi, alpha, probe = random_fields(prob, seed=205)
    obj = O.objects(u, chi, alpha, prob)
    centre = (det - n) // 2 + n / 2.0
    ill = [probe[m] * obj[m][0, 1:1 + n, 1:1 + n] for m in range(2)]
    turn = O.exit_wave_mapped(obj[0], probe[0], 1, 1, prob, 0)
    twice = O.exit_wave_mapped(obj[1], probe[1], 1, 1, prob, 1)
    for a in range(n):
        for b in range(n):
            # quarter turn: (a, b) - n/2 -> (-(b - n/2), a - n/2)
            qy, qx = int(centre - (b - n / 2)), int(centre + (a - n / 2))
            assert turn[qy, qx] == pytest.approx(ill[0][a, b], abs=1e-14)
            qy, qx = int(centre + 2 * (a - n / 2)), int(centre + 2 * (b - n / 2))
            assert twice[qy, qx] == pytest.approx(ill[1][a, b], abs=1e-14)
            if a + 1 < n:   # half way between two samples: their mean
                assert twice[qy + 1, qx] == pytest.approx(0.5 * (ill[1][a, b] + ill[1][a + 1, b]), abs=1e-14)
    assert np.count_nonzero(np.abs(turn) > 1e-15) == n * n


def test_mapped_gradient_matches_central_differences():
    prob = _mapped(_prob(), [detector_map(1.15, 0.5), detector_map(0.9, -0.7)])
    u, chi, alpha, probe = random_fields(prob, seed=206)
    rng = np.random.default_rng(207)
    y = ragged(O.model_intensity(u + rng.normal(0, 0.05, size=u.shape), chi, alpha, probe, prob))
    r = O.loss_grad(u, chi, alpha, probe, y, prob)
    h = 1e-6
    for _ in range(8):
        c = int(rng.integers(3))
        idx = tuple(int(rng.integers(s)) for s in u.shape[1:])
        up, um = u.copy(), u.copy()
        up[(c,) + idx] += h
        um[(c,) + idx] -= h
        fd = (O.loss(up, chi, alpha, probe, y, prob)[0] - O.loss(um, chi, alpha, probe, y, prob)[0]) / (2 * h)
        assert fd == pytest.approx(r["grad_u"][(c,) + idx], rel=1e-5, abs=1e-6 * np.abs(r["grad_u"]).max())


def test_mapped_support_must_stay_in_the_window():
    prob = _mapped(_prob(dets=(14, 16)), [detector_map(3.5, 0.0), np.eye(2)])
    with pytest.raises(O.FootprintError):
        O.tables(prob)
    lo, hi = O.mapped_extent(_mapped(_prob(), [detector_map(1.0, math.pi / 4)] * 2), 0)
    assert (lo >= 0).all() and (hi <= 13).all()
