"""GPU parity of the membrane (z-tied) parameterisation against the oracle.

Under MPBP_Z_TIED the unknowns are given per lateral pixel and hold for every slice
(sections 3-4); the gradients are the z-sums of the per-voxel gradients.  The oracle's
loss_grad_ztied broadcasts the fields and sums its per-voxel gradients.  The film
fills the whole grid here: chi is the workload's slab amplitude on every slice.
Tolerances as in the other parity tests.
"""
import numpy as np
import pytest

from oracle import mpbp_oracle as O
from synth import get_config, make_fields, make_problem, photon_rng, poisson_counts
from tests.conftest import ragged
from tests.gpu_util import assert_grad_close, assert_loss_close, gpu_forward, gpu_loss_grad, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
B = pytest.importorskip("paper_2312_14907_amd.binding")


def _tied_workload(name):
    cfg = get_config(name)
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    u2 = np.ascontiguousarray(f["u"][:, :1])           # the fields are z-invariant already
    d2 = np.ascontiguousarray(f["delta"][:, :1])
    chi2 = np.full((1, prob.ny, prob.nx), float(f["chi"].max()), dtype=np.float32)
    nz = prob.nz
    full = lambda a, lead: np.broadcast_to(a, lead + (nz, prob.ny, prob.nx))
    inten = O.model_intensity(full(u2, (3,)).astype(np.float64), full(chi2, ()), f["alpha"], f["probe"], prob)
    y = poisson_counts(photon_rng(cfg), ragged(inten)) if cfg["noise"] else ragged(inten).astype(np.float32)
    return prob, f, u2, (u2 + d2).astype(np.float32), chi2, y


@pytest.mark.parametrize("path", [0, 1])
def test_c1_ztied_loss_and_gradient(path):
    say(f"z-tied c1_tiny, path {path}")
    prob, f, u2, up, chi2, y = _tied_workload("c1_tiny")
    plan = B.Plan(prob, 0, flags=B.MPBP_Z_TIED)
    plan.mpbp_set_option(B.MPBP_OPT_PATH, path)
    got = gpu_loss_grad(plan, up, chi2, f["alpha"], f["probe"], y)
    ref = O.loss_grad_ztied(up, chi2, f["alpha"], f["probe"], y, prob)
    assert got["grad_u"].shape == (3, 1, prob.ny, prob.nx) and got["grad_chi"].shape == (1, prob.ny, prob.nx)
    assert_loss_close(got["loss"], ref["loss"])
    np.testing.assert_allclose(got["frame_loss"], ref["frame_loss"], rtol=1e-4, atol=1e-6 * ref["frame_loss"].max())
    assert_grad_close(got["grad_u"], ref["grad_u"], "grad_u")
    assert_grad_close(got["grad_chi"], ref["grad_chi"], "grad_chi")
    assert_grad_close(got["grad_alpha"], ref["grad_alpha"], "grad_alpha")
    # at the truth the noiseless data is matched: zero loss up to FP32 rounding
    zero = gpu_forward(plan, u2, chi2, f["alpha"], f["probe"], y)
    assert zero["loss"] <= 1e-9 * float(np.sum(y))


def test_c2_ztied_gradient_and_step():
    say("z-tied c2_forward gradient, fused path, and the plain step on tied fields")
    prob, f, u2, up, chi2, y = _tied_workload("c2_forward")
    plan = B.Plan(prob, 0, flags=B.MPBP_Z_TIED)
    frames = list(range(0, prob.n_frames(), 7))
    got = gpu_loss_grad(plan, up, chi2, f["alpha"], f["probe"], y, frames=frames)
    ref = O.loss_grad_ztied(up, chi2, f["alpha"], f["probe"], y, prob, frames=frames)
    assert_loss_close(got["loss"], ref["loss"])
    assert_grad_close(got["grad_u"], ref["grad_u"], "grad_u")
    assert_grad_close(got["grad_chi"], ref["grad_chi"], "grad_chi")
    assert_grad_close(got["grad_alpha"], ref["grad_alpha"], "grad_alpha")
    # mpbp_step updates the tied fields (3 ny nx and ny nx elements), nothing beyond
    du = torch.from_numpy(up.copy()).cuda()
    dc = torch.from_numpy(chi2.copy()).cuda()
    da = torch.from_numpy(f["alpha"].copy()).cuda()
    gu = torch.from_numpy(got["grad_u"]).cuda()
    gc = torch.from_numpy(got["grad_chi"]).cuda()
    ga = torch.from_numpy(got["grad_alpha"]).cuda()
    plan.mpbp_step(du, dc, da, gu, gc, ga, (1e-9, 1e-9, 1e-9))
    torch.cuda.synchronize()
    new = O.step((up, chi2, f["alpha"]), (got["grad_u"], got["grad_chi"], got["grad_alpha"]), (1e-9,) * 3)
    for a, b in zip((du, dc, da), new):
        np.testing.assert_allclose(a.cpu().numpy(), b, rtol=1e-6, atol=1e-7)
