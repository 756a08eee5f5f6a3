"""GPU parity at the full workload sizes.

c3_grad runs whole against the oracle.  c4_batch (six peaks, windows 64..256, uneven
rasters) and c5_full (three peaks, 256 windows, 12288 frames) run the full batch on the
GPU in the benchmark's launch configuration; the oracle then recomputes sampled outputs
one by one: per-frame losses of sampled frames, and the gradient on sampled voxel
columns from exactly the frames whose windows cover them (other frames contribute
nothing there).  The frames the oracle checks carry Poisson counts of the oracle's own
forward model at the true fields (as measured data would); every other frame carries
model-free speckle counts drawn on the device, which the GPU path processes all the
same.  (Speckle unrelated to the model puts counts where the model's far field sits at
the FP32 rounding floor, where the direction of the amplitude residual is undefined in
FP32; model-consistent data keeps the checked outputs well conditioned.)
"""
import numpy as np
import pytest

from oracle import mpbp_oracle as O
from synth import get_config, make_fields, make_problem, photon_rng, poisson_counts
from tests.conftest import ragged
from tests.gpu_util import (assert_grad_close, assert_loss_close, dev, gpu_loss_grad, host, say,
                            speckle_y)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
B = pytest.importorskip("paper_2312_14907_amd.binding")


class DeviceY:
    """Slices of a device intensity array fetched on demand (for the oracle)."""

    def __init__(self, t):
        self.t = t

    def __getitem__(self, sl):
        return self.t[sl].cpu().numpy()


def covering_frames(prob, tab, yy, xx):
    out = []
    for fid in range(prob.n_frames()):
        py, px = tab["scan"][fid]
        if py <= yy < py + prob.probe_n and px <= xx < px + prob.probe_n:
            out.append(fid)
    return out


def _check_sampled(name, seed, columns, frames_per_peak=3):
    cfg = get_config(name)
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    u = (f["u"] + f["delta"]).astype(np.float32)
    tab = O.tables(prob)
    sample = []
    for m in range(prob.n_peaks):
        base = int(np.sum(prob.frames_per_peak()[:m]))
        nfr = prob.frames_per_peak()[m]
        sample += [base, base + nfr // 2 + int(prob.scan_n[m, 1]) // 2, base + nfr - 1][:frames_per_peak]
    cover = {col: covering_frames(prob, tab, *col) for col in columns}
    checked = sorted(set(sample).union(*cover.values()))
    say(f"{name}: intensities on device; oracle data for {len(checked)} checked frames")
    y = speckle_y(prob, seed)
    inten = O.model_intensity(f["u"], f["chi"], f["alpha"], f["probe"], prob, frames=checked)
    rng = np.random.default_rng(seed)
    for fid, it in zip(checked, inten):
        m = int(tab["peak_of_frame"][fid])
        d = int(prob.det[m])
        start = int(tab["y_off"][m]) + int(tab["local_index"][fid]) * d * d
        y[start:start + d * d] = dev(poisson_counts(rng, it).ravel())
    plan = B.Plan(prob, 0)
    say(f"{name}: full-batch loss_grad")
    got = gpu_loss_grad(plan, u, f["chi"], f["alpha"], f["probe"], y)
    assert np.isfinite(got["loss"])
    assert got["loss"] == pytest.approx(float(np.sum(got["frame_loss"].astype(np.float64))), rel=1e-6)
    ylazy = DeviceY(y)
    say(f"{name}: oracle on {len(sample)} sampled frames")
    _, per = O.loss(u, f["chi"], f["alpha"], f["probe"], ylazy, prob, frames=sample)
    np.testing.assert_allclose(got["frame_loss"][sample], per, rtol=1e-5)
    for (yy, xx) in columns:
        fr = cover[(yy, xx)]
        say(f"{name}: oracle gradient at column ({yy}, {xx}) from {len(fr)} frames")
        ref = O.loss_grad(u, f["chi"], f["alpha"], f["probe"], ylazy, prob, frames=fr)
        for c in range(3):
            assert_grad_close(got["grad_u"][c][:, yy, xx], ref["grad_u"][c][:, yy, xx], f"grad_u[{c}]")
        assert_grad_close(got["grad_chi"][:, yy, xx], ref["grad_chi"][:, yy, xx], "grad_chi")
    plan.close()


def test_c3_full_batch_against_oracle():
    cfg = get_config("c3_grad")
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    say("c3: oracle intensities")
    inten = O.model_intensity(f["u"], f["chi"], f["alpha"], f["probe"], prob)
    y = poisson_counts(photon_rng(cfg), ragged(inten))
    del inten
    u = (f["u"] + f["delta"]).astype(np.float32)
    plan = B.Plan(prob, 0)
    say("c3: gpu")
    got = gpu_loss_grad(plan, u, f["chi"], f["alpha"], f["probe"], y)
    say("c3: oracle loss_grad")
    ref = O.loss_grad(u, f["chi"], f["alpha"], f["probe"], y, prob)
    assert_loss_close(got["loss"], ref["loss"])
    np.testing.assert_allclose(got["frame_loss"], ref["frame_loss"], rtol=1e-5,
                               atol=1e-6 * ref["frame_loss"].max())
    for c in range(3):
        assert_grad_close(got["grad_u"][c], ref["grad_u"][c], f"grad_u[{c}]")
    assert_grad_close(got["grad_chi"], ref["grad_chi"], "grad_chi")
    assert_grad_close(got["grad_alpha"], ref["grad_alpha"], "grad_alpha")


def test_c4_full_batch_sampled():
    _check_sampled("c4_batch", 404, columns=[(3, 5), (128, 131), (250, 17)])


def test_c5_full_batch_sampled():
    _check_sampled("c5_full", 505, columns=[(0, 0), (255, 300), (511, 498)])
