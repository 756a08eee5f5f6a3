"""Launch variants and the autotuner.

Every compiled variant of the frame kernel (footprint bound, projection depth,
XCD-aware order) and of the back-projection kernel (frames per step) computes the same
result as the default launch parameters, which the oracle parity tests cover.  The XCD
order and the frame batch leave every operation as it is, so those results are bitwise
equal.  The projection depth (object slices in flight) and a larger footprint bound
keep every sum (the bound only adds exact zeros), but in another instance the compiler
may contract products into FMAs in another order, so those results agree to rounding:
1e-5 of each output's largest magnitude.  The autotuner picks the fastest projection
depth, then the fastest footprint bound and XCD order, leaves the results unchanged, and
its cache file restores the choice in a new plan.
"""
import os

import numpy as np
import pytest

from synth import get_config, make_fields, make_problem
from tests.gpu_util import dev, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
B = pytest.importorskip("paper_2312_14907_amd.binding")


@pytest.fixture(scope="module")
def c4():
    """c4_batch at u_true + delta.  The counts are Poisson draws of the library's own
    model intensities at the true fields: a comparison between launch variants needs
    well-conditioned data (counts unrelated to the model put counts where the model's
    far field is at the FP32 rounding floor, and there the direction of the residual,
    hence the gradient, follows last-bit rounding differences)."""
    cfg = get_config("c4_batch")
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    chi, alpha, probe = dev(f["chi"]), dev(f["alpha"]), dev(f["probe"])
    plan = B.Plan(prob, 0)
    inten = torch.zeros(plan.intensity_size, dtype=torch.float32, device="cuda:0")
    plan.mpbp_forward(dev(f["u"]), chi, alpha, probe, model_intensity=inten)
    g = torch.Generator(device="cuda:0")
    g.manual_seed(cfg["seed"])
    y = torch.poisson(inten, generator=g)
    plan.close()
    args = (dev((f["u"] + f["delta"]).astype(np.float32)), chi, alpha, probe, y)
    return prob, args


def _run(plan, args):
    u, chi, alpha, probe, y = args
    gu, gc, ga = torch.empty_like(u), torch.empty_like(chi), torch.empty_like(alpha)
    loss = torch.zeros((), dtype=torch.float64, device="cuda:0")
    fl = torch.zeros(plan.n_frames, dtype=torch.float32, device="cuda:0")
    plan.mpbp_loss_grad(u, chi, alpha, probe, y, gu, gc, ga, loss=loss, frame_loss=fl)
    torch.cuda.synchronize()
    return [loss, fl, gu, gc, ga]


def _equal(got, ref, what):
    for i, (a, b) in enumerate(zip(got, ref)):
        assert torch.equal(a, b), f"{what}: output {i} differs by {(a - b).abs().max().item():.3e}"


def _close(got, ref, what, rtol=1e-5):
    for i, (a, b) in enumerate(zip(got, ref)):
        a, b = a.double(), b.double()
        scale = b.abs().max().item()
        assert (a - b).abs().max().item() <= rtol * scale, f"{what}: output {i}"


def test_every_variant_matches_default(c4):
    prob, args = c4
    plan = B.Plan(prob, 0)
    ref = _run(plan, args)
    classes = plan.mpbp_tuning()["classes"]
    n = 0
    for k, c in enumerate(classes):
        for fb in sorted({48, 64, c["D"], 32} - {x for x in (32, 48, 64) if x < c["key"]}):
            for g in (2, 4, 8):
                for xcd in (0, 1):
                    try:
                        plan.mpbp_set_variant(k, fb, g, xcd)
                    except B.MPBPError as e:
                        assert e.status == 6, str(e)      # not compiled for this D
                        continue
                    say(f"variant class {k} (D={c['D']}): FB={fb} G={g} xcd={xcd}")
                    got = _run(plan, args)
                    if fb == c["key"] and g == 4:
                        _equal(got, ref, f"class {k} FB={fb} G={g} xcd={xcd}")
                    else:
                        _close(got, ref, f"class {k} FB={fb} G={g} xcd={xcd}")
                    n += 1
        plan.mpbp_set_variant(k, c["key"], 4, 1)
    assert n >= 2 * 2 * len(classes)
    # per run of equal exit-beam offset (default) and per slice: the projection rounds the
    # regrouped sums differently (close), every gradient batch size of one setting sums
    # the frames in the same order with the same fused multiply-adds (bit for bit)
    for runs in (0, 1):
        plan.mpbp_set_option(B.MPBP_OPT_RUNS, runs)
        first = None
        for b in (1, 2, 4, 8, 16):
            say(f"runs={runs}, gradient batch {b}")
            plan.mpbp_set_option(B.MPBP_OPT_GRAD_BATCH, b)
            got = _run(plan, args)
            if first is None:
                first = got
                _close(got, ref, f"runs={runs}")
            _equal(got, first, f"runs={runs} batch {b}")
    plan.mpbp_set_option(B.MPBP_OPT_RUNS, 1)
    plan.mpbp_set_option(B.MPBP_OPT_GRAD_BATCH, 8)
    for tx in (8, 16):
        # another tile grid sums the alpha partials over other voxel sets
        say(f"gradient kernel tile width {tx}")
        plan.mpbp_set_option(B.MPBP_OPT_GRAD_TILE, tx)
        got = _run(plan, args)
        _equal(got[:4], ref[:4], f"grad tile {tx}")
        _close(got[4:], ref[4:], f"grad tile {tx}")


def test_autotune_and_cache(c4, tmp_path):
    prob, args = c4
    cache = tmp_path / "tune.txt"
    old = os.environ.get("MPBP_TUNE_CACHE")
    os.environ["MPBP_TUNE_CACHE"] = str(cache)
    try:
        plan = B.Plan(prob, 0)
        assert plan.mpbp_tuning()["source"] == "default"
        ref = _run(plan, args)
        say("autotune c4_batch")
        plan.mpbp_autotune(*args)
        t = plan.mpbp_tuning()
        assert t["source"] == "autotune"
        for k, c in enumerate(t["classes"]):
            # projection depth: the fastest projection for the chosen XCD order
            proj = [x for x in t["candidates"] if x.get("class") == k and x.get("kernel") == "project"]
            assert sorted((x["G"], x["xcd"]) for x in proj) == [(g, x) for g in (2, 4, 8) for x in (0, 1)]
            at_x = [x for x in proj if x["xcd"] == c["xcd"]]
            assert [x for x in at_x if x["G"] == c["G"]][0]["us"] <= min(x["us"] for x in at_x) + 0.01
            # footprint bound and XCD order: the fastest projection + frame kernel pair
            cand = [x for x in t["candidates"] if x.get("class") == k and "FB" in x]
            assert cand, f"class {k} not timed"
            best = min(x["us"] for x in cand)       # (the report rounds to 0.01 us)
            chosen = [x for x in cand if (x["FB"], x["G"], x["xcd"]) == (c["FB"], c["G"], c["xcd"])]
            assert chosen and chosen[0]["us"] <= best + 0.01
            assert c["us"] == pytest.approx(best, abs=0.01)
        gb = [x for x in t["candidates"] if "grad_batch" in x]
        assert sorted((x["grad_batch"], x["grad_tile"]) for x in gb) == [(b, tx) for b in (4, 8, 16) for tx in (8, 16)]
        chosen = [x for x in gb if (x["grad_batch"], x["grad_tile"]) == (t["grad_batch"], t["grad_tile"])]
        assert chosen and chosen[0]["us"] <= min(x["us"] for x in gb) + 0.01
        _close(_run(plan, args), ref, "autotuned")
        lines = cache.read_text().splitlines()
        assert len(lines) == len(t["classes"]) + 1 and all(" | " in ln for ln in lines)
        plan2 = B.Plan(prob, 0)
        t2 = plan2.mpbp_tuning()
        assert t2["source"] == "cache" and (t2["grad_batch"], t2["grad_tile"]) == (t["grad_batch"], t["grad_tile"])
        for a, b in zip(t["classes"], t2["classes"]):
            assert (a["FB"], a["G"], a["xcd"]) == (b["FB"], b["G"], b["xcd"])
        _close(_run(plan2, args), ref, "from cache")
    finally:
        if old is None:
            os.environ.pop("MPBP_TUNE_CACHE", None)
        else:
            os.environ["MPBP_TUNE_CACHE"] = old
