"""GPU parity of the optimiser around the objective (Algorithm 1 and the Armijo loop).

* mpbp_adam_step against the oracle's Adam update and eq. (8) chain rule, elementwise,
  over several steps, in both parameterisations and with a fixed reference alpha;
* Algorithm 1 on c1_tiny with the same shuffled frame order on both sides, without and
  with its unwrap projection (eq. (10)): per-iteration minibatch losses, the oracle's
  objective at the two final fields, and the removal of a lattice-translation artefact;
* the Armijo line-search loop on c1_tiny: losses and accepted steps of the first
  iterations, and a monotone decrease.
Adam scales every step to the learning rate, so a gradient element whose sign is
decided by rounding moves by a full step either way; the loops are therefore compared
through the objective (an aggregate), not element by element.
"""
import numpy as np
import pytest

from oracle import mpbp_oracle as O
from synth import get_config, make_fields, make_problem
from synth.inputs import LATTICE_A_NM as LATTICE, frame_order
from tests.conftest import ragged
from tests.gpu_util import dev, host, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
B = pytest.importorskip("paper_2312_14907_amd.binding")
from paper_2312_14907_amd import optim  # noqa: E402


@pytest.fixture(scope="module")
def c1():
    cfg = get_config("c1_tiny")
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    y = ragged(O.model_intensity(f["u"], f["chi"], f["alpha"], f["probe"], prob)).astype(np.float32)
    return cfg, prob, f, y


@pytest.mark.parametrize("log_params", [1, 0])
def test_adam_kernel_matches_oracle(c1, log_params):
    cfg, prob, f, y = c1
    say(f"adam kernel, log_params={log_params}")
    plan = B.Plan(prob, 0)
    rng = np.random.default_rng(7)
    nf = prob.nz * prob.ny * prob.nx
    M = prob.n_peaks
    u = rng.normal(0, 0.05, (3, prob.nz, prob.ny, prob.nx))
    xl = rng.normal(-0.5, 0.3, (prob.nz, prob.ny, prob.nx))      # chi~ (or chi itself)
    al = rng.normal(0.0, 0.2, M)
    if not log_params:
        xl = np.abs(xl) * 0.05                                      # small chi: the clamp at 0 acts
        al = np.exp(al)
    lr, b1, b2, eps = (0.01, 0.1, 0.1), 0.9, 0.999, 1e-8
    cfgd = {"lr": lr, "beta1": b1, "beta2": b2, "eps": eps, "log_params": log_params, "fixed_alpha": 0}
    du, dxl, dal = dev(u.astype(np.float32)), dev(xl.astype(np.float32)), dev(al.astype(np.float32))
    dchi = torch.empty_like(dxl) if log_params else dxl
    dalpha = torch.empty_like(dal) if log_params else dal
    state = torch.full((2 * (4 * nf + M),), float("nan"), device="cuda:0")
    plan.mpbp_adam_step(cfgd, 0, du, dchi, dalpha, dxl if log_params else None, dal if log_params else None,
                        state, None, None, None)
    # oracle state, starting from the float32 values the device holds
    p = [u.astype(np.float32).astype(np.float64), xl.astype(np.float32).astype(np.float64),
         al.astype(np.float32).astype(np.float64)]
    mom = [np.zeros_like(q) for q in p]
    sec = [np.zeros_like(q) for q in p]
    for t in range(1, 4):
        gu = rng.normal(0, 1e3, u.shape).astype(np.float32)
        gx = rng.normal(0, 10.0, xl.shape).astype(np.float32)
        ga = rng.normal(0, 50.0, M).astype(np.float32)
        plan.mpbp_adam_step(cfgd, t, du, dchi, dalpha, dxl if log_params else None, dal if log_params else None,
                            state, dev(gu), dev(gx), dev(ga))
        if log_params:
            gx64, ga64 = O.log_param_grad(np.exp(p[1]), gx), O.log_param_grad(np.exp(p[2]), ga)
        else:
            gx64, ga64 = gx.astype(np.float64), ga.astype(np.float64)
        p[0], mom[0], sec[0] = O.adam_update(p[0], gu, mom[0], sec[0], t, lr[0], b1, b2, eps)
        p[1], mom[1], sec[1] = O.adam_update(p[1], gx64, mom[1], sec[1], t, lr[1], b1, b2, eps)
        keep = (p[2][0], mom[2][0], sec[2][0])
        p[2], mom[2], sec[2] = O.adam_update(p[2], ga64, mom[2], sec[2], t, lr[2], b1, b2, eps)
        p[2][0], mom[2][0], sec[2][0] = keep
        if not log_params:
            p[1] = np.maximum(p[1], 0.0)
            p[2] = np.maximum(p[2], 0.0)
    torch.cuda.synchronize()
    np.testing.assert_allclose(host(du), p[0], rtol=1e-5, atol=1e-6 * lr[0])
    np.testing.assert_allclose(host(dxl), p[1], rtol=1e-5, atol=1e-6 * lr[1])
    np.testing.assert_allclose(host(dal), p[2], rtol=1e-5, atol=1e-6 * lr[2])
    assert host(dal)[0] == np.float32(al[0])
    if log_params:
        np.testing.assert_allclose(host(dchi), np.exp(p[1]), rtol=2e-5)
        np.testing.assert_allclose(host(dalpha), np.exp(p[2]), rtol=2e-5)
    else:
        assert (host(dxl) >= 0).all() and (host(dxl) == 0).any()


def test_algorithm1_c1_matches_oracle(c1):
    cfg, prob, f, y = c1
    say("Algorithm 1 (no unwrap projection), c1_tiny")
    plan = B.Plan(prob, 0)
    order = frame_order(prob.n_frames(), cfg["seed"], epochs=3)
    u0 = (f["u"] + f["delta"]).astype(np.float32)
    chi0 = np.maximum(f["chi"], 1e-3).astype(np.float32)
    cl0 = np.log(chi0).astype(np.float32)
    al0 = (np.log(f["alpha"]) + 0.1).astype(np.float32)
    # 75 frames, b = 20: three minibatches per shuffle (15 frames left), six iterations
    # cross into the second shuffle
    lr, batch, iters = (0.002, 0.02, 0.02), 20, 6
    du, dcl, dal = dev(u0), dev(cl0), dev(al0)
    chi, alpha, losses = optim.adam_reconstruct(plan, dev(f["probe"]), dev(y), du, dcl, dal, order, batch=batch,
                                                iterations=iters, lr=lr, fixed_alpha=0)
    ou, ocl, oal, olosses = O.adam_reconstruct(u0, cl0, al0, f["probe"], y, prob, order, batch, iters, lr=lr,
                                               fixed_alpha=0)
    np.testing.assert_allclose(losses, olosses, rtol=1e-3)
    assert host(dal)[0] == al0[0]
    np.testing.assert_allclose(host(chi), np.exp(host(dcl)), rtol=2e-5)
    f_gpu = O.loss(host(du), np.exp(host(dcl).astype(np.float64)), np.exp(host(dal).astype(np.float64)),
                   f["probe"], y, prob)[0]
    f_ora = O.loss(ou, np.exp(ocl), np.exp(oal), f["probe"], y, prob)[0]
    f_start = O.loss(u0, chi0, np.exp(al0), f["probe"], y, prob)[0]
    assert f_gpu == pytest.approx(f_ora, rel=1e-3)
    assert f_gpu < f_start


def test_algorithm1_with_unwrap_c1_matches_oracle(c1):
    # Algorithm 1 with its last step, the unwrap projection Pi_U of eq. (10), starting
    # from a field with a lattice-translation artefact on a patch
    from synth import lattice_jump
    cfg, prob, f, y = c1
    say("Algorithm 1 with the unwrap projection, c1_tiny")
    plan = B.Plan(prob, 0)
    order = frame_order(prob.n_frames(), cfg["seed"], epochs=3)
    u0 = lattice_jump((f["u"] + f["delta"]).astype(np.float32), 6, 20, 4, 18, cells=1)
    chi0 = np.maximum(f["chi"], 1e-3).astype(np.float32)
    cl0 = np.log(chi0).astype(np.float32)
    al0 = (np.log(f["alpha"]) + 0.1).astype(np.float32)
    lr, batch, iters = (0.002, 0.02, 0.02), 25, 6
    du, dcl, dal = dev(u0), dev(cl0), dev(al0)
    _, _, losses = optim.adam_reconstruct(plan, dev(f["probe"]), dev(y), du, dcl, dal, order, batch=batch,
                                          iterations=iters, lr=lr, fixed_alpha=0, unwrap=True)
    ou, ocl, oal, olosses = O.adam_reconstruct(u0, cl0, al0, f["probe"], y, prob, order, batch, iters, lr=lr,
                                               fixed_alpha=0, unwrap=True)
    np.testing.assert_allclose(losses, olosses, rtol=1e-3)
    # the projection removed the artefact: the field is back near the smooth one
    smooth = (f["u"] + f["delta"]).astype(np.float64)
    assert np.abs(host(du) - smooth).max() < 0.1 * LATTICE
    assert np.abs(ou - smooth).max() < 0.1 * LATTICE


def test_line_search_c1_matches_oracle(c1):
    cfg, prob, f, y = c1
    say("Armijo line search, c1_tiny")
    plan = B.Plan(prob, 0)
    u0 = (f["u"] + f["delta"]).astype(np.float32)
    du = dev(u0)
    out = optim.line_search_descent(plan, dev(f["probe"]), dev(y), du, dev(f["chi"]), dev(f["alpha"]), iterations=8)
    _, olosses, oetas = O.line_search_descent(u0, f["chi"], f["alpha"], f["probe"], y, prob, iterations=8)
    assert len(out["losses"]) == 8
    np.testing.assert_allclose(out["losses"][:3], olosses[:3], rtol=1e-4)
    np.testing.assert_allclose(out["etas"][:3], oetas[:3], rtol=1e-3)
    assert all(b < a for a, b in zip(out["losses"], out["losses"][1:]))
    assert out["losses"][-1] < 0.5 * out["losses"][0]
    # the GPU loop's own trials follow the line search's definition
    c, step0 = 1e-4, 0.01
    for k, tr in enumerate(out["trials"]):
        n2, tried = tr["norm2"], tr["tried"]
        first = tried[0][0]
        if k == 0:
            assert first == pytest.approx(step0 / np.sqrt(n2 / u0.size), rel=1e-12)
        else:
            assert first == pytest.approx(2.0 * out["etas"][k - 1], rel=1e-15)
        for (e0, _), (e1, _) in zip(tried, tried[1:]):
            assert e1 == pytest.approx(0.5 * e0, rel=1e-15)
        for e, f1 in tried[:-1]:
            assert f1 > out["losses"][k] - c * e * n2
        assert tried[-1][0] == out["etas"][k]
        assert tried[-1][1] <= out["losses"][k] - c * tried[-1][0] * n2
