"""GPU parity at the full workload sizes, every output against the FP64 oracle.

c3_grad runs whole against the oracle in one process.  c4_batch (six peaks, windows
64..256, uneven rasters) and c5_full (three peaks, 256 windows, 12288 frames: the
benchmark's workload) run whole against the oracle evaluated band by band in parallel
CPU processes (tests/oracle_pool.py): model-consistent Poisson counts for every frame
(the oracle's forward model at the true fields), then every frame loss, the total loss,
df/dalpha and the whole df/du and df/dchi fields at u_true + delta.  c5 is checked in
three launch configurations: the defaults, the autotuner's choice (what the benchmark
times), and the benchmark's recorded choice set by hand (footprint bound 48, projection
depth 2, gradient batch 4 over 8 x 8 tiles).
"""
import numpy as np
import pytest

from oracle import mpbp_oracle as O
from synth import get_config, make_fields, make_problem, photon_rng, poisson_counts
from tests.conftest import ragged
from tests.gpu_util import assert_grad_close, assert_loss_close, dev, gpu_loss_grad, say
from tests.oracle_pool import oracle_whole, workers

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
B = pytest.importorskip("paper_2312_14907_amd.binding")


def _compare(got, ref, what):
    assert_loss_close(got["loss"], ref["loss"], f"{what}: loss")
    np.testing.assert_allclose(got["frame_loss"], ref["frame_loss"], rtol=1e-5,
                               atol=1e-6 * ref["frame_loss"].max(), err_msg=f"{what}: frame losses")
    for c in range(3):
        assert_grad_close(got["grad_u"][c], ref["grad_u"][c], f"{what}: grad_u[{c}]")
    assert_grad_close(got["grad_chi"], ref["grad_chi"], f"{what}: grad_chi")
    assert_grad_close(got["grad_alpha"], ref["grad_alpha"], f"{what}: grad_alpha")


def test_c3_full_batch_against_oracle():
    cfg = get_config("c3_grad")
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    say("c3: oracle intensities")
    inten = O.model_intensity(f["u"], f["chi"], f["alpha"], f["probe"], prob)
    y = poisson_counts(photon_rng(cfg), ragged(inten))
    del inten
    u = (f["u"] + f["delta"]).astype(np.float32)
    plan = B.Plan(prob, 0)
    say("c3: gpu")
    got = gpu_loss_grad(plan, u, f["chi"], f["alpha"], f["probe"], y)
    say("c3: oracle loss_grad")
    ref = O.loss_grad(u, f["chi"], f["alpha"], f["probe"], y, prob)
    _compare(got, ref, "c3")


def _whole(name, rows):
    say(f"{name}: oracle data and loss/gradient over every frame, {workers()} CPU processes")
    ref = oracle_whole(name, rows_per_band=rows)
    say(f"{name}: oracle loss {ref['loss']:.9e}")
    cfg = get_config(name)
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    return prob, f, ref


def test_c4_full_batch_against_oracle():
    prob, f, ref = _whole("c4_batch", 4)
    u = (f["u"] + f["delta"]).astype(np.float32)
    plan = B.Plan(prob, 0)
    dy = dev(ref.pop("y"))
    say("c4: gpu, default launch parameters")
    _compare(gpu_loss_grad(plan, u, f["chi"], f["alpha"], f["probe"], dy), ref, "c4 default")
    say("c4: gpu, autotuned")
    plan.mpbp_autotune(dev(u), dev(f["chi"]), dev(f["alpha"]), dev(f["probe"]), dy)
    say(f"c4: tuned {[(c['D'], c['FB'], c['G']) for c in plan.mpbp_tuning()['classes']]}")
    _compare(gpu_loss_grad(plan, u, f["chi"], f["alpha"], f["probe"], dy), ref, "c4 autotuned")
    plan.close()


def test_c5_full_batch_against_oracle():
    prob, f, ref = _whole("c5_full", 4)
    u = (f["u"] + f["delta"]).astype(np.float32)
    dy = dev(ref.pop("y"))
    plan = B.Plan(prob, 0)
    say("c5: gpu, default launch parameters")
    _compare(gpu_loss_grad(plan, u, f["chi"], f["alpha"], f["probe"], dy), ref, "c5 default")
    say("c5: gpu, autotuned (the benchmark's path)")
    plan.mpbp_autotune(dev(u), dev(f["chi"]), dev(f["alpha"]), dev(f["probe"]), dy)
    t = plan.mpbp_tuning()
    say(f"c5: tuned {[(c['D'], c['FB'], c['G'], c['xcd']) for c in t['classes']]}, grad batch {t['grad_batch']}, "
        f"tile {t.get('grad_tile')}")
    _compare(gpu_loss_grad(plan, u, f["chi"], f["alpha"], f["probe"], dy), ref, "c5 autotuned")
    say("c5: gpu, footprint bound 48, projection depth 2, gradient batch 4, 8 x 8 tiles")
    plan.mpbp_set_variant(0, 48, 2, 1)
    plan.mpbp_set_option(B.MPBP_OPT_GRAD_BATCH, 4)
    plan.mpbp_set_option(B.MPBP_OPT_GRAD_TILE, 8)
    _compare(gpu_loss_grad(plan, u, f["chi"], f["alpha"], f["probe"], dy), ref, "c5 FB48 G2 B4 T8")
    plan.close()
