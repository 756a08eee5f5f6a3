"""GPU parity of R with a detector-frame map (MPBP_DETECTOR_MAP, section 2: each peak's
exit wave lives in its own detector frame, turned against the object's frame and sampled
at its own pixel size) against the oracle's mapped R.

Slice z's probe-window point (a, b) lands on q = M_m ((a, b) - n/2) + centre + (z - nz/2) t_m
and each exit-wave pixel interpolates the illuminated slice bilinearly at its pre-image.
Checked: loss, per-frame losses, model intensities and gradients on c1 with a different
map per peak (turns, magnifications and a reduction); the z-tied parameterisation; 3D
illumination volumes with a background; c2 minibatches; a c5 minibatch (the full
geometry); identity maps against the interpolated-offset model (MPBP_SHEAR_LINEAR) on the
GPU; the plain path's refusal.
Tolerances as in the other parity tests.
"""
import dataclasses
import math

import numpy as np
import pytest

from oracle import mpbp_oracle as O
from synth import get_config, incident_probe_3d, make_fields, make_problem
from synth.inputs import detector_map
from tests.conftest import ragged
from tests.gpu_util import assert_grad_close, assert_loss_close, dev, gpu_forward, gpu_loss_grad, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
B = pytest.importorskip("paper_2312_14907_amd.binding")

# per peak: (pixel ratio, detector-frame angle); the mapped supports stay in the windows
C1_MAPS = [(1.1, 0.4), (0.85, -1.0), (1.0, math.pi / 2 + 0.2)]
C2_MAPS = [(1.2, 0.4), (0.9, 2.5), (1.05, -0.7)]


def _case(name, maps):
    cfg = get_config(name)
    base = make_problem(cfg)
    prob = dataclasses.replace(base, lateral_map=np.stack([detector_map(r, a) for r, a in maps]))
    f = make_fields(cfg, prob)
    y = ragged(O.model_intensity(f["u"], f["chi"], f["alpha"], f["probe"], prob)).astype(np.float32)
    return prob, f, y


@pytest.fixture(scope="module")
def c1():
    return _case("c1_tiny", C1_MAPS)


def _check(got, ref):
    assert_loss_close(got["loss"], ref["loss"])
    for c in range(3):
        assert_grad_close(got["grad_u"][c], ref["grad_u"][c], f"grad_u[{c}]")
    assert_grad_close(got["grad_chi"], ref["grad_chi"], "grad_chi")
    assert_grad_close(got["grad_alpha"], ref["grad_alpha"], "grad_alpha")


def test_c1_detector_map(c1):
    prob, f, y = c1
    say("detector map c1")
    u = (f["u"] + f["delta"]).astype(np.float32)
    plan = B.Plan(prob, 0, flags=B.MPBP_DETECTOR_MAP)
    got = gpu_loss_grad(plan, u, f["chi"], f["alpha"], f["probe"], y)
    ref = O.loss_grad(u, f["chi"], f["alpha"], f["probe"], y, prob)
    np.testing.assert_allclose(got["frame_loss"], ref["frame_loss"], rtol=1e-5, atol=1e-5 * ref["frame_loss"].max())
    _check(got, ref)


def test_c1_detector_map_intensity(c1):
    prob, f, _ = c1
    say("detector map c1 model intensity")
    u = (f["u"] + f["delta"]).astype(np.float32)
    plan = B.Plan(prob, 0, flags=B.MPBP_DETECTOR_MAP)
    got = gpu_forward(plan, u, f["chi"], f["alpha"], f["probe"], intensity=True)["intensity"]
    ref = ragged(O.model_intensity(u, f["chi"], f["alpha"], f["probe"], prob))
    np.testing.assert_allclose(got, ref, rtol=1e-4, atol=1e-5 * ref.max())


def test_c1_detector_map_z_tied(c1):
    prob, f, y = c1
    say("detector map c1 z-tied")
    u2 = (f["u"] + f["delta"])[:, :1].astype(np.float32)
    chi2 = f["chi"].max(axis=0, keepdims=True).astype(np.float32)
    plan = B.Plan(prob, 0, flags=B.MPBP_DETECTOR_MAP | B.MPBP_Z_TIED)
    got = gpu_loss_grad(plan, u2, chi2, f["alpha"], f["probe"], y)
    _check(got, O.loss_grad_ztied(u2, chi2, f["alpha"], f["probe"], y, prob))


def test_c1_detector_map_probe3_background(c1):
    prob, f, _ = c1
    say("detector map + 3D probe + background c1")
    rng = np.random.default_rng(131)
    p3 = np.stack([incident_probe_3d(f["probe"][m], prob.nz, rng.uniform(-0.3, 0.3, 2))
                   for m in range(prob.n_peaks)]).astype(np.complex64)
    inten = ragged(O.model_intensity(f["u"], f["chi"], f["alpha"], p3, prob))
    bg = rng.uniform(0.0, 0.2 * float(inten.mean()), inten.size).astype(np.float32)
    y = ragged(O.model_intensity(f["u"], f["chi"], f["alpha"], p3, prob, background=bg)).astype(np.float32)
    u = (f["u"] + f["delta"]).astype(np.float32)
    plan = B.Plan(prob, 0, flags=B.MPBP_DETECTOR_MAP | B.MPBP_PROBE_3D)
    plan.mpbp_set_background(dev(bg))
    got = gpu_loss_grad(plan, u, f["chi"], f["alpha"], p3, y)
    _check(got, O.loss_grad(u, f["chi"], f["alpha"], p3, y, prob, background=bg))


def test_c2_minibatch_detector_map():
    prob, f, y = _case("c2_forward", C2_MAPS)
    say("detector map c2 minibatch")
    u = (f["u"] + f["delta"]).astype(np.float32)
    plan = B.Plan(prob, 0, flags=B.MPBP_DETECTOR_MAP)
    frames = np.random.default_rng(132).choice(prob.n_frames(), 40, replace=False)
    got = gpu_loss_grad(plan, u, f["chi"], f["alpha"], f["probe"], y, frames=frames)
    _check(got, O.loss_grad(u, f["chi"], f["alpha"], f["probe"], y, prob, frames=frames))


def test_identity_map_is_the_interpolated_offset_model():
    cfg = get_config("c1_tiny")
    base = make_problem(cfg)
    f = make_fields(cfg, base)
    lin = dataclasses.replace(base, shear_linear=True)
    y = ragged(O.model_intensity(f["u"], f["chi"], f["alpha"], f["probe"], lin)).astype(np.float32)
    ident = dataclasses.replace(base, lateral_map=np.stack([np.eye(2)] * base.n_peaks))
    say("identity detector map vs interpolated offsets c1")
    u = (f["u"] + f["delta"]).astype(np.float32)
    a = gpu_loss_grad(B.Plan(lin, 0, flags=B.MPBP_SHEAR_LINEAR), u, f["chi"], f["alpha"], f["probe"], y)
    b = gpu_loss_grad(B.Plan(ident, 0, flags=B.MPBP_DETECTOR_MAP), u, f["chi"], f["alpha"], f["probe"], y)
    _check(b, a)


def test_plain_path_refuses_the_map(c1):
    prob, _, _ = c1
    plan = B.Plan(prob, 0, flags=B.MPBP_DETECTOR_MAP)
    with pytest.raises(B.MPBPError) as e:
        plan.mpbp_set_option(B.MPBP_OPT_PATH, 1)
    assert e.value.status == 6                            # MPBP_ERR_UNSUPPORTED


def test_c2_minibatch_detector_map_z_tied():
    prob, f, y = _case("c2_forward", C2_MAPS)
    say("detector map c2 minibatch z-tied")
    u2 = (f["u"] + f["delta"])[:, :1].astype(np.float32)
    chi2 = f["chi"].max(axis=0, keepdims=True).astype(np.float32)
    plan = B.Plan(prob, 0, flags=B.MPBP_DETECTOR_MAP | B.MPBP_Z_TIED)
    frames = np.random.default_rng(133).choice(prob.n_frames(), 40, replace=False)
    got = gpu_loss_grad(plan, u2, chi2, f["alpha"], f["probe"], y, frames=frames)
    _check(got, O.loss_grad_ztied(u2, chi2, f["alpha"], f["probe"], y, prob, frames=frames))


def test_c5_minibatch_detector_map_sampled():
    """The detector map at the full c5 geometry (32 x 512 x 512 voxels, 256 x 256 windows,
    16 colours of frames, mapped footprints up to 62 x 62): a minibatch of 4 frames per
    peak, spread over each raster, against the oracle on the same frames.  The counts are
    the oracle's model intensities at the true fields on those frames (zero elsewhere:
    no listed frame reads them)."""
    cfg = get_config("c5_full")
    base = make_problem(cfg)
    prob = dataclasses.replace(base, lateral_map=np.stack([detector_map(r, a) for r, a in C2_MAPS]))
    f = make_fields(cfg, base)
    tab = O.tables(prob)
    rng = np.random.default_rng(134)
    frames, start = [], 0
    for m in range(prob.n_peaks):
        nfr = int(prob.scan_n[m][0]) * int(prob.scan_n[m][1])
        frames += [start + int(j) for j in rng.choice(nfr, 4, replace=False)]
        start += nfr
    frames = sorted(frames)
    say("detector map c5 minibatch (oracle on 12 frames)")
    y = np.zeros(int(tab["y_off"][-1]), dtype=np.float32)
    for fid, inten in zip(frames, O.model_intensity(f["u"], f["chi"], f["alpha"], f["probe"], prob, frames=frames)):
        m, j = int(tab["peak_of_frame"][fid]), int(tab["local_index"][fid])
        d2 = int(prob.det[m]) ** 2
        y[int(tab["y_off"][m]) + j * d2:int(tab["y_off"][m]) + (j + 1) * d2] = inten.ravel()
    u = (f["u"] + f["delta"]).astype(np.float32)
    plan = B.Plan(prob, 0, flags=B.MPBP_DETECTOR_MAP)
    got = gpu_loss_grad(plan, u, f["chi"], f["alpha"], f["probe"], y, frames=frames)
    ref = O.loss_grad(u, f["chi"], f["alpha"], f["probe"], y, prob, frames=frames)
    _check(got, ref)
    assert np.allclose(got["frame_loss"], ref["frame_loss"], rtol=1e-4, atol=0)
