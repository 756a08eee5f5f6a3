"""GPU parity of per-peak 3D illumination volumes (MPBP_PROBE_3D, section 2) against the
oracle.

The probe of every peak is built as the paper builds its 3D probes: the workload's 2D
beam profile carried along an inclined incident beam (synth.incident_probe_3d), with a
per-slice phase so that no two slices are equal.  Checked on both paths: loss, per-frame
losses and gradients on c1 (tolerances as in the other parity tests), the z-tied
parameterisation, a c2 minibatch, and a volume constant along x3 against the 2D probe.
"""
import numpy as np
import pytest

from oracle import mpbp_oracle as O
from synth import get_config, incident_probe_3d, make_fields, make_problem
from tests.conftest import ragged
from tests.gpu_util import assert_grad_close, assert_loss_close, gpu_loss_grad, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
B = pytest.importorskip("paper_2312_14907_amd.binding")


def _volumes(prob, probe2d, seed):
    rng = np.random.default_rng(seed)
    vols = []
    for m in range(prob.n_peaks):
        t_in = rng.uniform(-0.4, 0.4, 2)
        v = incident_probe_3d(probe2d[m], prob.nz, t_in).astype(np.complex128)
        v *= np.exp(1j * rng.uniform(-np.pi, np.pi, prob.nz))[:, None, None]
        vols.append(v)
    return np.stack(vols).astype(np.complex64)


def _case(name, seed):
    cfg = get_config(name)
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    p3 = _volumes(prob, f["probe"], seed)
    y = ragged(O.model_intensity(f["u"], f["chi"], f["alpha"], p3, prob)).astype(np.float32)
    return prob, f, p3, y


@pytest.fixture(scope="module")
def c1():
    return _case("c1_tiny", 91)


def _check(got, ref):
    assert_loss_close(got["loss"], ref["loss"])
    for c in range(3):
        assert_grad_close(got["grad_u"][c], ref["grad_u"][c], f"grad_u[{c}]")
    assert_grad_close(got["grad_chi"], ref["grad_chi"], "grad_chi")
    assert_grad_close(got["grad_alpha"], ref["grad_alpha"], "grad_alpha")


@pytest.mark.parametrize("path", [0, 1])
def test_c1_3d_probe(c1, path):
    prob, f, p3, y = c1
    say(f"3D probe c1 path={path}")
    u = (f["u"] + f["delta"]).astype(np.float32)
    plan = B.Plan(prob, 0, flags=B.MPBP_PROBE_3D)
    plan.mpbp_set_option(B.MPBP_OPT_PATH, path)
    got = gpu_loss_grad(plan, u, f["chi"], f["alpha"], p3, y)
    ref = O.loss_grad(u, f["chi"], f["alpha"], p3, y, prob)
    np.testing.assert_allclose(got["frame_loss"], ref["frame_loss"], rtol=1e-5, atol=1e-5 * ref["frame_loss"].max())
    _check(got, ref)


@pytest.mark.parametrize("path", [0, 1])
def test_c1_3d_probe_z_tied(c1, path):
    prob, f, p3, y = c1
    say(f"3D probe z-tied c1 path={path}")
    u2 = (f["u"] + f["delta"])[:, :1].astype(np.float32)
    chi2 = f["chi"].max(axis=0, keepdims=True).astype(np.float32)
    plan = B.Plan(prob, 0, flags=B.MPBP_PROBE_3D | B.MPBP_Z_TIED)
    plan.mpbp_set_option(B.MPBP_OPT_PATH, path)
    got = gpu_loss_grad(plan, u2, chi2, f["alpha"], p3, y)
    ref = O.loss_grad_ztied(u2, chi2, f["alpha"], p3, y, prob)
    _check(got, ref)


def test_c2_minibatch_3d_probe():
    prob, f, p3, y = _case("c2_forward", 92)
    say("3D probe c2 minibatch")
    u = (f["u"] + f["delta"]).astype(np.float32)
    plan = B.Plan(prob, 0, flags=B.MPBP_PROBE_3D)
    frames = np.random.default_rng(93).choice(prob.n_frames(), 40, replace=False)
    got = gpu_loss_grad(plan, u, f["chi"], f["alpha"], p3, y, frames=frames)
    ref = O.loss_grad(u, f["chi"], f["alpha"], p3, y, prob, frames=frames)
    _check(got, ref)


def test_volume_constant_along_x3_is_the_2d_probe(c1):
    # data consistent with this probe (with counts unrelated to the model, last-bit
    # differences decide the residual's direction where |Psi| is at the FP32 floor)
    prob, f, _, _ = c1
    y = ragged(O.model_intensity(f["u"], f["chi"], f["alpha"], f["probe"], prob)).astype(np.float32)
    u = (f["u"] + f["delta"]).astype(np.float32)
    p3 = np.repeat(f["probe"][:, None], prob.nz, axis=1)
    a = gpu_loss_grad(B.Plan(prob, 0), u, f["chi"], f["alpha"], f["probe"], y)
    b = gpu_loss_grad(B.Plan(prob, 0, flags=B.MPBP_PROBE_3D), u, f["chi"], f["alpha"], p3, y)
    assert b["loss"] == pytest.approx(a["loss"], rel=1e-6)
    for k in ("grad_u", "grad_chi", "grad_alpha"):
        np.testing.assert_allclose(b[k], a[k], rtol=1e-5, atol=1e-6 * np.abs(a[k]).max())
