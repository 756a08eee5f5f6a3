"""Phases far beyond +-20 rad (GPU against the oracle).

Adding a lattice vector a n (n integer per voxel) to u changes every phase G_hkl . u by
2 pi (h, k, l) . n, a multiple of 2 pi (eq. (6)-(7): intensities unchanged).  With n up
to 5 per component the phases reach about 90 rad; the object build and the gradient
kernel both reduce these arguments (by multiples of pi/2) and must match the oracle there, and the
loss must equal the loss at the unshifted field.
"""
import numpy as np
import pytest

from oracle import mpbp_oracle as O
from synth import get_config, make_fields, make_problem
from synth.inputs import LATTICE_A_NM
from tests.conftest import ragged
from tests.gpu_util import assert_grad_close, assert_loss_close, gpu_loss_grad, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
B = pytest.importorskip("paper_2312_14907_amd.binding")


@pytest.mark.parametrize("path", [0, 1])
def test_lattice_shifted_field_c1(path):
    cfg = get_config("c1_tiny")
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    y = ragged(O.model_intensity(f["u"], f["chi"], f["alpha"], f["probe"], prob)).astype(np.float32)
    u0 = (f["u"] + f["delta"]).astype(np.float32)
    n = np.random.default_rng(cfg["seed"] + 77).integers(-5, 6, size=u0.shape)
    u = (u0.astype(np.float64) + LATTICE_A_NM * n).astype(np.float32)
    phase = np.max(np.abs(np.einsum("mc,c...->m...", prob.g, u.astype(np.float64))))
    say(f"large phases, path {path}: max |G . u| = {phase:.1f} rad")
    assert phase > 60.0
    plan = B.Plan(prob, 0)
    plan.mpbp_set_option(B.MPBP_OPT_PATH, path)
    got = gpu_loss_grad(plan, u, f["chi"], f["alpha"], f["probe"], y)
    ref = O.loss_grad(u, f["chi"], f["alpha"], f["probe"], y, prob)
    assert_loss_close(got["loss"], ref["loss"])
    for c in range(3):
        assert_grad_close(got["grad_u"][c], ref["grad_u"][c], f"grad_u[{c}]")
    assert_grad_close(got["grad_chi"], ref["grad_chi"], "grad_chi")
    assert_grad_close(got["grad_alpha"], ref["grad_alpha"], "grad_alpha")
    base = gpu_loss_grad(plan, u0, f["chi"], f["alpha"], f["probe"], y)
    assert_loss_close(got["loss"], base["loss"], "loss against the unshifted field", rtol=1e-4)
    plan.close()
