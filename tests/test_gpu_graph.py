"""Graph replay of full-batch calls (MPBP_OPT_GRAPH) against direct launches.

A full-batch fused call is captured into a hipGraph on first use for a given set of
buffer addresses and replayed afterwards; the detector-size classes become parallel
graph branches.  The kernels and their arguments are those of the direct launches and
the path has no atomics, so every replay must match the direct launches bit for bit.
Each check replays several times, with the program's own device work and
synchronisations between replays, and with the inputs rewritten in place between
replays (a replay must read the buffers' current contents).  Also with detector maps
(one back-projection launch per colour of frames in the graph) and interpolated offsets.
"""
import dataclasses

import numpy as np
import pytest

from synth import get_config, make_fields, make_problem
from synth.inputs import detector_map
from tests.gpu_util import dev, say, speckle_y

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
B = pytest.importorskip("paper_2312_14907_amd.binding")


def _setup(name, option=None):
    cfg = get_config(name)
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    flags = 0
    if option == "detector_map":       # a turned and scaled detector frame per peak
        prob = dataclasses.replace(prob, lateral_map=np.stack(
            [detector_map(r, a) for r, a in [(1.2, 0.4), (0.9, 2.5), (1.05, -0.7)]][:prob.n_peaks]))
        flags = B.MPBP_DETECTOR_MAP
    elif option == "interpolated_offsets":
        prob = dataclasses.replace(prob, shear_linear=True)
        flags = B.MPBP_SHEAR_LINEAR
    plan = B.Plan(prob, 0, flags=flags)
    y = speckle_y(prob, cfg["seed"])
    ua = dev((f["u"] + f["delta"]).astype(np.float32))
    ub = dev((f["u"] - 0.5 * f["delta"]).astype(np.float32))
    return plan, prob, f, y, ua, ub


def _loss_grad(plan, u, chi, alpha, probe, y, out):
    loss, fl, gu, gc, ga = out
    plan.mpbp_loss_grad(u, chi, alpha, probe, y, gu, gc, ga, loss=loss, frame_loss=fl)
    torch.cuda.synchronize()
    return [t.clone() for t in out]


def _outputs(plan, u):
    return (torch.zeros((), dtype=torch.float64, device="cuda:0"),
            torch.zeros(plan.n_frames, dtype=torch.float32, device="cuda:0"),
            torch.empty_like(u), torch.empty(u.shape[1:], dtype=torch.float32, device="cuda:0"),
            torch.empty(plan.n_peaks, dtype=torch.float32, device="cuda:0"))


def _same(a, b, what):
    for i, (x, y) in enumerate(zip(a, b)):
        assert torch.equal(x, y), f"{what}: output {i} differs (max {(x - y).abs().max().item():.3e})"


@pytest.mark.parametrize("name, option", [("c1_tiny", None), ("c4_batch", None), ("c2_forward", "detector_map"),
                                          ("c2_forward", "interpolated_offsets")])
def test_loss_grad_replays_match_direct(name, option):
    say(f"graph replay vs direct launches, loss_grad, {name} {option or ''}")
    plan, prob, f, y, ua, ub = _setup(name, option)
    chi, alpha, probe = dev(f["chi"]), dev(f["alpha"]), dev(f["probe"])
    u = ua.clone()
    out = _outputs(plan, u)

    plan.mpbp_set_option(B.MPBP_OPT_GRAPH, 0)
    ref_a = _loss_grad(plan, u, chi, alpha, probe, y, out)
    u.copy_(ub)
    ref_b = _loss_grad(plan, u, chi, alpha, probe, y, out)
    assert not torch.equal(ref_a[0], ref_b[0])

    plan.mpbp_set_option(B.MPBP_OPT_GRAPH, 1)
    for rep, (src, ref) in enumerate([(ua, ref_a), (ua, ref_a), (ub, ref_b), (ua, ref_a), (ub, ref_b)]):
        u.copy_(src)                                  # same buffer, new contents
        for t in out:
            t.fill_(float("nan"))                     # the replay must overwrite every output
        junk = torch.randn(1 << 20, device="cuda:0").sum()   # the program's own work
        got = _loss_grad(plan, u, chi, alpha, probe, y, out)
        assert torch.isfinite(junk)
        _same(got, ref, f"{name} replay {rep}")

    # new output buffers: a second graph, same results
    out2 = _outputs(plan, u)
    u.copy_(ua)
    _same(_loss_grad(plan, u, chi, alpha, probe, y, out2), ref_a, f"{name} new buffers")
    _same(_loss_grad(plan, u, chi, alpha, probe, y, out), ref_a, f"{name} first buffers again")


def test_forward_replays_match_direct():
    say("graph replay vs direct launches, forward with model intensity, c4_batch")
    plan, prob, f, y, ua, ub = _setup("c4_batch")
    chi, alpha, probe = dev(f["chi"]), dev(f["alpha"]), dev(f["probe"])
    u = ua.clone()
    loss = torch.zeros((), dtype=torch.float64, device="cuda:0")
    fl = torch.zeros(plan.n_frames, dtype=torch.float32, device="cuda:0")
    mi = torch.zeros(plan.intensity_size, dtype=torch.float32, device="cuda:0")

    def run():
        plan.mpbp_forward(u, chi, alpha, probe, y, loss=loss, frame_loss=fl, model_intensity=mi)
        torch.cuda.synchronize()
        return [loss.clone(), fl.clone(), mi.clone()]

    plan.mpbp_set_option(B.MPBP_OPT_GRAPH, 0)
    ref_a = run()
    u.copy_(ub)
    ref_b = run()
    plan.mpbp_set_option(B.MPBP_OPT_GRAPH, 1)
    for rep, (src, ref) in enumerate([(ua, ref_a), (ub, ref_b), (ub, ref_b), (ua, ref_a)]):
        u.copy_(src)
        for t in (loss, fl, mi):
            t.fill_(float("nan"))
        got = run()
        _same(got, ref, f"forward replay {rep}")


def test_graph_then_subset_and_profile_calls():
    """Subset calls and profiled calls launch directly; they interleave with replays."""
    say("graph replays interleaved with subset and profiled calls, c1_tiny")
    plan, prob, f, y, ua, ub = _setup("c1_tiny")
    chi, alpha, probe = dev(f["chi"]), dev(f["alpha"]), dev(f["probe"])
    out = _outputs(plan, ua)
    plan.mpbp_set_option(B.MPBP_OPT_GRAPH, 0)
    ref = _loss_grad(plan, ua, chi, alpha, probe, y, out)
    plan.mpbp_set_option(B.MPBP_OPT_GRAPH, 1)
    sub = [3, 10, 40, 74]
    gu, gc, ga = torch.empty_like(ua), torch.empty_like(chi), torch.empty_like(alpha)
    sl = torch.zeros((), dtype=torch.float64, device="cuda:0")
    for rep in range(3):
        _same(_loss_grad(plan, ua, chi, alpha, probe, y, out), ref, f"replay {rep}")
        plan.mpbp_loss_grad(ua, chi, alpha, probe, y, gu, gc, ga, frames=sub, loss=sl)
        torch.cuda.synchronize()
        assert abs(sl.item() - float(ref[1][sub].double().sum())) <= 1e-5 * abs(sl.item())
    plan.mpbp_set_option(B.MPBP_OPT_PROFILE, 1)
    _same(_loss_grad(plan, ua, chi, alpha, probe, y, out), ref, "profiled call")
    st = plan.mpbp_stage_times()
    assert st["frames"][1] == 1 and st["grad"][1] == 1
