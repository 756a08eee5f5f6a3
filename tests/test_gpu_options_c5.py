"""GPU parity of the forward-model options at the full c5 geometry (3 peaks,
32 x 512 x 512 voxels, 256 x 256 windows, 64 x 64 rasters): for each option a minibatch
of 4 frames per peak, spread over each raster, against the oracle on the same frames
(eq. (11): a minibatch's loss and gradients are sums over its frames).  The counts are
the oracle's model intensities at the true fields on the listed frames and zero
elsewhere (no listed frame reads them).  Options: interpolated exit-beam offsets with
3D illumination volumes (the per-slice projection and walk), the z-tied
parameterisation (the run path with tied chain rule) and the background of eq. (2).
The detector map has its own c5 case in test_gpu_detector_map.py."""
import dataclasses

import numpy as np
import pytest

from oracle import mpbp_oracle as O
from synth import get_config, incident_probe_3d, make_fields, make_problem
from tests.gpu_util import assert_grad_close, assert_loss_close, dev, gpu_loss_grad, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
B = pytest.importorskip("paper_2312_14907_amd.binding")


def _frames(prob, seed, per_peak=4):
    rng = np.random.default_rng(seed)
    frames, start = [], 0
    for m in range(prob.n_peaks):
        nfr = int(prob.scan_n[m][0]) * int(prob.scan_n[m][1])
        frames += [start + int(j) for j in rng.choice(nfr, per_peak, replace=False)]
        start += nfr
    return sorted(frames)


def _ragged_on(prob, frames, per_frame):
    """A ragged array (the layout of y) holding per_frame[k] on frames[k], zero elsewhere."""
    tab = O.tables(prob)
    out = np.zeros(int(tab["y_off"][-1]), dtype=np.float32)
    for fid, a in zip(frames, per_frame):
        m, j = int(tab["peak_of_frame"][fid]), int(tab["local_index"][fid])
        d2 = int(prob.det[m]) ** 2
        out[int(tab["y_off"][m]) + j * d2:int(tab["y_off"][m]) + (j + 1) * d2] = np.asarray(a).ravel()
    return out


def _check(got, ref):
    assert_loss_close(got["loss"], ref["loss"])
    assert np.allclose(got["frame_loss"], ref["frame_loss"], rtol=1e-4, atol=0)
    for c in range(got["grad_u"].shape[0]):
        assert_grad_close(got["grad_u"][c], ref["grad_u"][c], f"grad_u[{c}]")
    assert_grad_close(got["grad_chi"], ref["grad_chi"], "grad_chi")
    assert_grad_close(got["grad_alpha"], ref["grad_alpha"], "grad_alpha")


def test_c5_interpolated_offsets_and_3d_probes():
    cfg = get_config("c5_full")
    prob = dataclasses.replace(make_problem(cfg), shear_linear=True)
    f = make_fields(cfg, prob)
    rng = np.random.default_rng(141)
    p3 = np.stack([incident_probe_3d(f["probe"][m], prob.nz, rng.uniform(-0.4, 0.4, 2))
                   for m in range(prob.n_peaks)]).astype(np.complex64)
    frames = _frames(prob, 142)
    say("c5 minibatch: interpolated offsets and 3D probes (oracle on 12 frames)")
    y = _ragged_on(prob, frames, O.model_intensity(f["u"], f["chi"], f["alpha"], p3, prob, frames=frames))
    u = (f["u"] + f["delta"]).astype(np.float32)
    plan = B.Plan(prob, 0, flags=B.MPBP_SHEAR_LINEAR | B.MPBP_PROBE_3D)
    got = gpu_loss_grad(plan, u, f["chi"], f["alpha"], p3, y, frames=frames)
    _check(got, O.loss_grad(u, f["chi"], f["alpha"], p3, y, prob, frames=frames))


def test_c5_z_tied():
    cfg = get_config("c5_full")
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    u2 = np.ascontiguousarray(f["u"][:, :1])            # the fields are z-invariant already
    up = (u2 + f["delta"][:, :1]).astype(np.float32)
    chi2 = np.full((1, prob.ny, prob.nx), float(f["chi"].max()), dtype=np.float32)
    full = lambda a, lead: np.broadcast_to(a, lead + (prob.nz, prob.ny, prob.nx))
    frames = _frames(prob, 143)
    say("c5 minibatch: z-tied (oracle on 12 frames)")
    inten = O.model_intensity(full(u2, (3,)).astype(np.float64), full(chi2, ()), f["alpha"], f["probe"], prob,
                              frames=frames)
    y = _ragged_on(prob, frames, inten)
    plan = B.Plan(prob, 0, flags=B.MPBP_Z_TIED)
    got = gpu_loss_grad(plan, up, chi2, f["alpha"], f["probe"], y, frames=frames)
    ref = O.loss_grad_ztied(up, chi2, f["alpha"], f["probe"], y, prob, frames=frames)
    assert got["grad_u"].shape == (3, 1, prob.ny, prob.nx)
    _check(got, ref)


def test_c5_background():
    cfg = get_config("c5_full")
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    frames = _frames(prob, 144)
    rng = np.random.default_rng(145)
    say("c5 minibatch: background (oracle on 12 frames)")
    bg = _ragged_on(prob, frames, [rng.uniform(0.0, 0.5, int(prob.det[0]) ** 2) for _ in frames])
    inten = O.model_intensity(f["u"], f["chi"], f["alpha"], f["probe"], prob, frames=frames, background=bg)
    y = _ragged_on(prob, frames, inten)
    u = (f["u"] + f["delta"]).astype(np.float32)
    plan = B.Plan(prob, 0)
    plan.mpbp_set_background(dev(bg))
    got = gpu_loss_grad(plan, u, f["chi"], f["alpha"], f["probe"], y, frames=frames)
    _check(got, O.loss_grad(u, f["chi"], f["alpha"], f["probe"], y, prob, frames=frames, background=bg))
