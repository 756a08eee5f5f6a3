"""Degenerate shapes of c1_tiny against the oracle, on both paths:

* one slice (nz = 1: no projection sum, the shear offsets are all zero, the method
  reduces to two-dimensional Bragg ptychography);
* five slices (fewer slices than one pass of the gradient kernel, and not a multiple of
  the slices a lane holds or of the projection's slices in flight);
* one peak with a single scan position (one frame in all);
* full batch and a minibatch of one frame.
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


def _case(name):
    cfg = dict(get_config("c1_tiny"))
    if name == "one_slice":
        cfg.update(nz=1, slab=1)
    elif name == "five_slices":
        cfg.update(nz=5, slab=4)
    elif name == "one_frame":
        cfg["peaks"] = [dict(cfg["peaks"][1], scan_n=(1, 1))]
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    # model-consistent data at the true field, evaluated at u + delta (counts added where
    # the model's far field is at the FP32 floor would make the residual's direction
    # rounding noise in any FP32 code)
    y = ragged(O.model_intensity(f["u"], f["chi"], f["alpha"], f["probe"], prob)).astype(np.float32)
    return prob, f, y, (f["u"] + f["delta"]).astype(np.float32)


@pytest.mark.parametrize("name", ["one_slice", "five_slices", "one_frame"])
@pytest.mark.parametrize("path", [0, 1])
def test_degenerate_shapes(name, path):
    prob, f, y, u = _case(name)
    assert prob.n_frames() >= 1
    for frames in (None, [prob.n_frames() - 1]):
        say(f"degenerate {name}: path={path} frames={frames} (nz={prob.nz}, peaks={prob.n_peaks}, frames={prob.n_frames()})")
        plan = B.Plan(prob, 0)
        plan.mpbp_set_option(B.MPBP_OPT_PATH, path)
        got = gpu_loss_grad(plan, u, f["chi"], f["alpha"], f["probe"], y, frames=frames)
        ref = O.loss_grad(u, f["chi"], f["alpha"], f["probe"], y, prob, frames=frames)
        assert ref["loss"] > 0
        assert_loss_close(got["loss"], ref["loss"])
        for c in range(3):
            assert_grad_close(got["grad_u"][c], ref["grad_u"][c], f"grad_u[{c}]")
        assert_grad_close(got["grad_chi"], ref["grad_chi"], "grad_chi")
        assert_grad_close(got["grad_alpha"], ref["grad_alpha"], "grad_alpha")
        plan.close()
