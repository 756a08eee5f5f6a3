"""The Python binding validates every device buffer before calling the library (CPU).

The library reads and writes the caller's buffers from its kernels and cannot check a
device address, so the binding rejects, with ValueError naming the argument: anything
that is not a torch tensor (a numpy array would pass a host address), a wrong dtype (a
float32 loss would receive an 8-byte store), a non-contiguous view, a wrong element
count, and a tensor that is not on the plan's GPU.  Without a GPU every correct-looking
tensor fails the last check, so each case here changes one property of an otherwise
well-formed CPU tensor and expects the message of that property.
"""
import numpy as np
import pytest

from synth import get_config, make_problem

torch = pytest.importorskip("torch")
B = pytest.importorskip("paper_2312_14907_amd.binding")


@pytest.fixture(scope="module")
def plan():
    return B.Plan(make_problem(get_config("c1_tiny")), device=-1)


def _good(plan):
    nf = plan.field_size
    return {
        "u": torch.zeros(3 * nf), "chi": torch.zeros(nf), "alpha": torch.zeros(plan.n_peaks),
        "probe": torch.zeros(plan.probe_size, dtype=torch.complex64), "y": torch.zeros(plan.intensity_size),
        "grad_u": torch.zeros(3 * nf), "grad_chi": torch.zeros(nf), "grad_alpha": torch.zeros(plan.n_peaks),
        "loss": torch.zeros((), dtype=torch.float64), "frame_loss": torch.zeros(plan.n_frames),
    }


def _bad_variants(t):
    yield "numpy", t.numpy() if t.dtype != torch.complex64 else t.numpy(), "torch CUDA tensor"
    wrong = torch.float64 if t.dtype != torch.float64 else torch.float32
    yield "dtype", t.to(wrong), "must be"
    if t.numel() > 1:
        big = torch.zeros(2 * t.numel(), dtype=t.dtype)
        yield "strided", big[::2], "contiguous"
    yield "size", torch.zeros(t.numel() + 1, dtype=t.dtype), "elements"
    yield "cpu", t, "must be on cuda"


LOSS_GRAD_ARGS = ("u", "chi", "alpha", "probe", "y", "grad_u", "grad_chi", "grad_alpha", "loss")


@pytest.mark.parametrize("name", LOSS_GRAD_ARGS)
def test_loss_grad_rejects_each_bad_buffer(plan, name):
    g = _good(plan)
    for kind, bad, msg in _bad_variants(g[name]):
        if name == "loss" and kind == "size":
            bad = torch.zeros(2, dtype=torch.float64)
        a = dict(g, **{name: bad})
        with pytest.raises(ValueError, match=msg) as e:
            plan.mpbp_loss_grad(a["u"], a["chi"], a["alpha"], a["probe"], a["y"], a["grad_u"], a["grad_chi"],
                                a["grad_alpha"], loss=a["loss"])
        if kind != "cpu":     # (every buffer here is on the CPU: the first one is named)
            assert str(e.value).startswith(name + " "), (kind, str(e.value))


def test_a_float32_loss_is_rejected(plan):
    g = _good(plan)
    with pytest.raises(ValueError, match="loss must be float64"):
        plan.mpbp_forward(g["u"], g["chi"], g["alpha"], g["probe"], g["y"], loss=torch.zeros((), dtype=torch.float32))


def test_forward_checks_outputs(plan):
    g = _good(plan)
    with pytest.raises(ValueError, match="frame_loss must hold at least 4"):
        plan.mpbp_forward(g["u"], g["chi"], g["alpha"], g["probe"], g["y"], frames=[0, 1, 2, 3],
                          frame_loss=torch.zeros(3))
    with pytest.raises(ValueError, match="model_intensity"):
        plan.mpbp_forward(g["u"], g["chi"], g["alpha"], g["probe"], None,
                          model_intensity=torch.zeros(plan.intensity_size - 1))
    with pytest.raises(ValueError, match="y is required"):
        plan.mpbp_forward(g["u"], g["chi"], g["alpha"], g["probe"], None, loss=g["loss"])


def test_step_adam_norm_check_buffers(plan):
    g = _good(plan)
    with pytest.raises(ValueError, match="grad_chi"):
        plan.mpbp_step(g["u"], g["chi"], g["alpha"], g["grad_u"], g["grad_chi"][:-1], g["grad_alpha"], (1, 1, 1))
    state = torch.zeros(2 * (4 * plan.field_size + plan.n_peaks))
    with pytest.raises(ValueError, match="state"):
        plan.mpbp_adam_step({"lr": (1, 1, 1)}, 1, g["u"], g["chi"], g["alpha"], g["chi"], g["alpha"], state[:-1],
                            g["grad_u"], g["grad_chi"], g["grad_alpha"])
    with pytest.raises(ValueError, match="chi_log is required"):
        plan.mpbp_adam_step({"lr": (1, 1, 1), "log_params": 1}, 1, g["u"], g["chi"], g["alpha"], None, g["alpha"],
                            state, g["grad_u"], g["grad_chi"], g["grad_alpha"])
    with pytest.raises(ValueError, match="out must be float64"):
        plan.mpbp_norm2(g["u"], torch.zeros(1))
    with pytest.raises(ValueError, match="b must"):
        plan.mpbp_set_background(torch.zeros(plan.intensity_size, dtype=torch.float64))
