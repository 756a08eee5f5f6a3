"""GPU parity on the paper-shaped workload c6_paper against the oracle: 150 x 150
detector windows (mixed radix 2 * 3 * 5^2: rows as 10 x 15, column chunks of 50), the four
in-plane peaks [100], [110], [120], [210] of a 0.3905 nm cubic lattice, a 9 x 9 raster at
a step of 6 and the paper's count rates (section 4).

Checked: loss, per-frame losses and gradients on both paths, per voxel and in the membrane
(z-tied) parameterisation, the model intensities, and the unwrap projector on the four
coplanar peaks (H H^T of rank 2: the component of u no peak sees is kept).  c6_paper100
takes the paper's 100-voxel window along x3 (Table 1) with a 17-voxel film: its sheared
footprints reach 70 x 51 pixels, and it is checked whole on both paths, per slice and
per run of equal offsets, and through Poisson counts.
"""
import numpy as np
import pytest

from oracle import mpbp_oracle as O
from oracle import unwrap_oracle as UW
from synth import get_config, lattice_jump, make_fields, make_problem, unwrap_field
from tests.conftest import ragged
from tests.gpu_util import assert_grad_close, assert_loss_close, dev, gpu_forward, gpu_loss_grad, host, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
B = pytest.importorskip("paper_2312_14907_amd.binding")


@pytest.fixture(scope="module")
def c6():
    cfg = get_config("c6_paper")
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    y = ragged(O.model_intensity(f["u"], f["chi"], f["alpha"], f["probe"], prob)).astype(np.float32)
    return prob, f, y


def _check(got, ref):
    assert_loss_close(got["loss"], ref["loss"])
    for c in range(3):
        assert_grad_close(got["grad_u"][c], ref["grad_u"][c], f"grad_u[{c}]")
    assert_grad_close(got["grad_chi"], ref["grad_chi"], "grad_chi")
    assert_grad_close(got["grad_alpha"], ref["grad_alpha"], "grad_alpha")


@pytest.mark.parametrize("path", [0, 1])
def test_c6_loss_and_gradient(c6, path):
    prob, f, y = c6
    say(f"c6_paper loss_grad path={path}")
    u = (f["u"] + f["delta"]).astype(np.float32)
    plan = B.Plan(prob, 0)
    plan.mpbp_set_option(B.MPBP_OPT_PATH, path)
    got = gpu_loss_grad(plan, u, f["chi"], f["alpha"], f["probe"], y)
    ref = O.loss_grad(u, f["chi"], f["alpha"], f["probe"], y, prob)
    np.testing.assert_allclose(got["frame_loss"], ref["frame_loss"], rtol=1e-5, atol=1e-5 * ref["frame_loss"].max())
    _check(got, ref)
    assert not got["grad_u"][2].any()          # in-plane peaks: u_z is unseen
    fw = gpu_forward(plan, u, f["chi"], f["alpha"], f["probe"], intensity=True)
    ri = ragged(O.model_intensity(u, f["chi"], f["alpha"], f["probe"], prob))
    np.testing.assert_allclose(fw["intensity"], ri, rtol=1e-5, atol=1e-5 * ri.max())


def test_c6_every_footprint_bound(c6):
    prob, f, y = c6
    u = (f["u"] + f["delta"]).astype(np.float32)
    ref = O.loss_grad(u, f["chi"], f["alpha"], f["probe"], y, prob)
    for fb in (48, 64, 150):
        say(f"c6_paper footprint bound {fb}")
        plan = B.Plan(prob, 0)
        plan.mpbp_set_variant(0, fb, 4, 1)
        _check(gpu_loss_grad(plan, u, f["chi"], f["alpha"], f["probe"], y), ref)


def test_c6_membrane(c6):
    prob, f, y = c6
    u2 = (f["u"] + f["delta"])[:, :1].astype(np.float32)
    chi2 = f["chi"].max(axis=0, keepdims=True).astype(np.float32)
    plan = B.Plan(prob, 0, flags=B.MPBP_Z_TIED)
    got = gpu_loss_grad(plan, u2, chi2, f["alpha"], f["probe"], y)
    _check(got, O.loss_grad_ztied(u2, chi2, f["alpha"], f["probe"], y, prob))


def test_c6_unwrap_coplanar_peaks(c6):
    prob, _, _ = c6
    plan = B.Plan(prob, 0, flags=B.MPBP_Z_TIED)
    u = lattice_jump(unwrap_field(1, prob.ny, prob.nx, seed=121, noise_nm=0.02), 40, 120, 30, 110)
    du = dev(u)
    wraps = torch.zeros((prob.n_peaks, 1, prob.ny, prob.nx), dtype=torch.int32, device="cuda:0")
    plan.mpbp_unwrap_project(du, wraps)
    torch.cuda.synchronize()
    ref_u, ref_w = UW.unwrap_projector(u, prob.g, return_wraps=True)
    np.testing.assert_array_equal(host(wraps), ref_w)
    np.testing.assert_allclose(host(du), ref_u, atol=2e-6, rtol=0)
    np.testing.assert_array_equal(host(du)[2], u[2])       # u_z: no peak sees it


@pytest.fixture(scope="module")
def c6_100():
    from synth import photon_rng, poisson_counts
    cfg = get_config("c6_paper100")
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    say("c6_paper100: oracle intensities (100 slices)")
    y = poisson_counts(photon_rng(cfg), ragged(O.model_intensity(f["u"], f["chi"], f["alpha"], f["probe"], prob)))
    u = (f["u"] + f["delta"]).astype(np.float32)
    say("c6_paper100: oracle loss and gradient")
    return prob, f, y, u, O.loss_grad(u, f["chi"], f["alpha"], f["probe"], y, prob)


@pytest.mark.parametrize("path,runs", [(0, 1), (0, 0), (1, 1)])
def test_c6_hundred_slices(c6_100, path, runs):
    prob, f, y, u, ref = c6_100
    say(f"c6_paper100 path={path} runs={runs}")
    plan = B.Plan(prob, 0)
    t = plan.mpbp_tuning()
    assert max(max(c["fy"], c["fx"]) for c in t["classes"]) == 70
    plan.mpbp_set_option(B.MPBP_OPT_PATH, path)
    plan.mpbp_set_option(B.MPBP_OPT_RUNS, runs)
    got = gpu_loss_grad(plan, u, f["chi"], f["alpha"], f["probe"], y)
    np.testing.assert_allclose(got["frame_loss"], ref["frame_loss"], rtol=1e-5, atol=1e-5 * ref["frame_loss"].max())
    _check(got, ref)
    plan.close()
