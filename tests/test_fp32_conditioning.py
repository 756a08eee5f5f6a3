"""How far FP32 arithmetic itself is from the FP64 oracle at the evaluation points the
GPU tests use (CPU; tests/fp32_model.py performs the oracle's steps in complex64).

At a perturbed point (u_true + delta, or delta alone) every output of an FP32 evaluation
is within a few 1e-6 of the oracle.  At u = 0 (the paper's initial guess) the loss and
df/dalpha still are, but df/du and df/dchi are a few percent off: the slab at u = 0
gives a far field that falls to the FP32 rounding floor at detector pixels where the
data (taken at the true, strained field) have counts; there the residual's direction
Psi/|Psi| is rounding noise in any FP32 evaluation, and each such pixel adds a term of
size sqrt(y) in that direction to the gradient.  The GPU tests at u = 0 take their
tolerance from this measurement.
"""
import numpy as np
import pytest

from oracle import mpbp_oracle as O
from synth import get_config, make_fields, make_problem
from tests.conftest import ragged, random_fields, tiny_problem
from tests.fp32_model import loss_grad_fp32, rel_errors


def _c1():
    cfg = get_config("c1_tiny")
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    y = ragged(O.model_intensity(f["u"], f["chi"], f["alpha"], f["probe"], prob)).astype(np.float32)
    return prob, f, y


def test_fp32_steps_match_oracle_on_random_problem():
    prob = tiny_problem()
    u, chi, alpha, probe = random_fields(prob, seed=81)
    rng = np.random.default_rng(82)
    y = ragged(O.model_intensity(u + rng.normal(0, 0.05, size=u.shape), chi, alpha, probe, prob)).astype(np.float32)
    u32 = u.astype(np.float32)
    err = rel_errors(loss_grad_fp32(u32, chi, alpha, probe, y, prob), O.loss_grad(u32, chi, alpha, probe, y, prob))
    assert max(err.values()) < 2e-5, err


@pytest.mark.parametrize("point", ["u_true+delta", "delta"])
def test_fp32_is_accurate_at_perturbed_points(point):
    prob, f, y = _c1()
    u = (f["u"] + f["delta"] if point == "u_true+delta" else f["delta"]).astype(np.float32)
    err = rel_errors(loss_grad_fp32(u, f["chi"], f["alpha"], f["probe"], y, prob),
                     O.loss_grad(u, f["chi"], f["alpha"], f["probe"], y, prob))
    assert err["loss"] < 1e-6
    assert max(v for k, v in err.items() if k != "loss") < 2e-5, err


def test_fp32_floor_at_zero_displacement():
    prob, f, y = _c1()
    u = np.zeros_like(f["u"])
    err = rel_errors(loss_grad_fp32(u, f["chi"], f["alpha"], f["probe"], y, prob),
                     O.loss_grad(u, f["chi"], f["alpha"], f["probe"], y, prob))
    assert err["loss"] < 1e-6 and err["grad_alpha"] < 1e-4, err
    worst = max(err["grad_chi"], *(err[f"grad_u[{c}]"] for c in range(3)))
    assert 5e-3 < worst < 0.1, err          # far above 1e-3, and bounded
