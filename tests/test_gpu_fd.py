"""Central finite differences of the GPU objective against the gradient that the
torch.autograd.Function returns (recompute mode: the backward pass re-runs the forward
model and the hand-written adjoint), on c3_grad: h = 1e-4 nm on each displacement
component of 64 seeded voxels inside the slab.

Each voxel's differences and gradient are evaluated over exactly the frames whose
windows cover it (a minibatch, eq. (11)): the other frames do not depend on that voxel,
so the restriction is exact and keeps the loss small enough for FP32 rounding not to
swamp the difference.

Tolerance.  The objective is a sum of FP32 per-pixel terms (about 80 frames of 128 x 128
pixels here); their rounding changes between u + h and u - h, which puts noise of about
1e-4 on each loss and, divided by 2h, about 0.75 on a difference (measured by performing
the oracle's steps in complex64 on this workload, against FP64 differences that match
the analytic gradient to 1e-6).  The gradients range over about 50 to 1000.  So each
difference must be within 5 + 1e-2 |g| of the gradient (over six times the noise), and
over all 192 values ||FD - g||_2 <= 1e-2 ||g||_2.  The oracle's own differences are
pinned at 1e-5 on the CPU (tests/test_oracle_pins.py).
"""
import numpy as np
import pytest

from oracle import mpbp_oracle as O
from synth import get_config, make_fields, make_problem, photon_rng, poisson_counts
from tests.conftest import ragged
from tests.gpu_util import dev, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
B = pytest.importorskip("paper_2312_14907_amd.binding")
from paper_2312_14907_amd.autograd import MPBPLoss  # noqa: E402

H = 1e-4
ABS_TOL, REL_TOL = 5.0, 1e-2


def test_central_differences_c3():
    cfg = get_config("c3_grad")
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    say("c3 FD: oracle intensities")
    y = poisson_counts(photon_rng(cfg), ragged(O.model_intensity(f["u"], f["chi"], f["alpha"], f["probe"], prob)))
    tab = O.tables(prob)
    scan = tab["scan"]
    u = (f["u"] + f["delta"]).astype(np.float32)
    rng = np.random.default_rng(cfg["seed"] + 1000)
    voxels = []
    while len(voxels) < 64:
        v = (int(rng.integers(prob.nz)), int(rng.integers(prob.ny)), int(rng.integers(prob.nx)))
        if f["chi"][v] > 0 and v not in voxels:
            voxels.append(v)
    du, dchi, dal, dpr, dy = dev(u), dev(f["chi"]), dev(f["alpha"]), dev(f["probe"]), dev(y)
    plan = B.Plan(prob, 0)
    lp = torch.zeros((), dtype=torch.float64, device="cuda:0")
    lm = torch.zeros((), dtype=torch.float64, device="cuda:0")
    fd, an = [], []
    for k, (z, yy, xx) in enumerate(voxels):
        cover = [i for i in range(prob.n_frames())
                 if scan[i, 0] <= yy < scan[i, 0] + prob.probe_n and scan[i, 1] <= xx < scan[i, 1] + prob.probe_n]
        if k % 16 == 0:
            say(f"c3 FD: voxel {k} ({z}, {yy}, {xx}), {len(cover)} frames")
        uu = du.clone().requires_grad_(True)
        loss = MPBPLoss.apply(uu, dchi, dal, plan, dpr, dy, cover, "recompute")
        loss.backward()
        g = uu.grad[:, z, yy, xx].double().cpu().numpy()
        for c in range(3):
            up, um = du.clone(), du.clone()
            up[c, z, yy, xx] += H
            um[c, z, yy, xx] -= H
            step = (float(up[c, z, yy, xx]) - float(um[c, z, yy, xx])) / 2.0
            plan.mpbp_forward(up, dchi, dal, dpr, dy, frames=cover, loss=lp)
            plan.mpbp_forward(um, dchi, dal, dpr, dy, frames=cover, loss=lm)
            fd.append((lp.item() - lm.item()) / (2.0 * step))
            an.append(g[c])
    fd, an = np.array(fd), np.array(an)
    err = np.abs(fd - an)
    say(f"c3 FD: max |FD - g| {err.max():.3f}, rms {np.sqrt(np.mean(err ** 2)):.3f}, "
        f"|g| in [{np.abs(an).min():.1f}, {np.abs(an).max():.1f}], "
        f"||FD - g|| / ||g|| = {np.linalg.norm(fd - an) / np.linalg.norm(an):.2e}")
    assert np.all(err <= ABS_TOL + REL_TOL * np.abs(an)), np.max(err - REL_TOL * np.abs(an))
    assert np.linalg.norm(fd - an) <= REL_TOL * np.linalg.norm(an)
    plan.close()
