"""Voxels that no frame's window reaches.

A copy of c1_tiny on a 44 x 56 object: the centred 5 x 5 rasters (step 4, 16-pixel
probe) cover only rows 6..37 and columns 12..43, so the gradient kernel has voxel tiles
whose range of covering raster columns is empty after clamping to the raster (right of
the rasters, the frames it would name lie past the end of a raster row).  Their gradient must be exactly zero, and everything
must match the oracle, for the full batch and for a minibatch, on both paths.
"""
import numpy as np
import pytest

from oracle import mpbp_oracle as O
from synth import get_config, make_fields, make_problem
from tests.conftest import ragged
from tests.gpu_util import assert_grad_close, assert_loss_close, gpu_loss_grad, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
B = pytest.importorskip("paper_2312_14907_amd.binding")


@pytest.fixture(scope="module")
def wide():
    cfg = dict(get_config("c1_tiny"), ny=44, nx=56)
    prob = make_problem(cfg)
    assert (prob.ny, prob.nx) == (44, 56)
    f = make_fields(cfg, prob)
    y = ragged(O.model_intensity(f["u"], f["chi"], f["alpha"], f["probe"], prob)).astype(np.float32)
    u = (f["u"] + f["delta"]).astype(np.float32)
    return prob, f, y, u


@pytest.mark.parametrize("path", [0, 1])
@pytest.mark.parametrize("subset", [False, True])
def test_uncovered_voxels(wide, path, subset):
    prob, f, y, u = wide
    frames = list(range(0, prob.n_frames(), 3)) if subset else None
    say(f"uncovered voxels: path={path} subset={subset}")
    plan = B.Plan(prob, 0)
    plan.mpbp_set_option(B.MPBP_OPT_PATH, path)
    got = gpu_loss_grad(plan, u, f["chi"], f["alpha"], f["probe"], y, frames=frames)
    ref = O.loss_grad(u, f["chi"], f["alpha"], f["probe"], y, prob, frames=frames)
    lo = prob.scan_origin.min(axis=0)
    hi = (prob.scan_origin + (prob.scan_n - 1) * prob.scan_step).max(axis=0) + prob.probe_n
    out = np.ones((prob.ny, prob.nx), dtype=bool)
    out[lo[0]:hi[0], lo[1]:hi[1]] = False
    assert out[:, hi[1]:].all() and out.sum() > 0.4 * out.size
    assert np.all(ref["grad_u"][:, :, out] == 0)
    assert np.all(got["grad_u"][:, :, out] == 0) and np.all(got["grad_chi"][:, out] == 0)
    assert np.abs(got["grad_u"][:, :, ~out]).max() > 0
    assert_loss_close(got["loss"], ref["loss"])
    for c in range(3):
        assert_grad_close(got["grad_u"][c], ref["grad_u"][c], f"grad_u[{c}]")
    assert_grad_close(got["grad_chi"], ref["grad_chi"], "grad_chi")
    assert_grad_close(got["grad_alpha"], ref["grad_alpha"], "grad_alpha")
    plan.close()


def test_minibatch_of_every_frame_equals_full_batch():
    """All frames listed as a minibatch (staged lists, the flagged walk of the gradient
    kernel) against the full-batch call (the unflagged walk): the same sums in the same
    order, so bitwise equal (c4_batch: six detector-size classes)."""
    cfg = get_config("c4_batch")
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    from tests.gpu_util import speckle_y
    y = speckle_y(prob, cfg["seed"])
    u = (f["u"] + f["delta"]).astype(np.float32)
    plan = B.Plan(prob, 0)
    say("minibatch of every frame vs full batch, c4_batch")
    full = gpu_loss_grad(plan, u, f["chi"], f["alpha"], f["probe"], y)
    every = gpu_loss_grad(plan, u, f["chi"], f["alpha"], f["probe"], y, frames=list(range(prob.n_frames())))
    for k in ("grad_u", "grad_chi", "frame_loss"):
        np.testing.assert_array_equal(every[k], full[k], err_msg=k)
    np.testing.assert_allclose(every["grad_alpha"], full["grad_alpha"], rtol=1e-6)
    assert abs(every["loss"] - full["loss"]) <= 1e-12 * abs(full["loss"])
    plan.close()
