"""Helpers of the GPU parity tests: device transfer, library calls, tolerance checks."""
import sys

import numpy as np

LOSS_RTOL = 1e-5      # relative tolerance on the loss (FP32 path vs FP64 oracle)
GRAD_RTOL = 1e-3      # relative tolerance on the gradients


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0").contiguous()


def host(t):
    return t.detach().to("cpu").numpy()


def gpu_loss_grad(plan, u, chi, alpha, probe, y, frames=None, frame_loss=True):
    """Run mpbp_loss_grad; numpy results (float64 loss)."""
    import torch
    du, dchi, dal = dev(u), dev(chi), dev(alpha)
    dpr = dev(probe)
    dy = y if isinstance(y, torch.Tensor) else dev(y)
    gu, gc, ga = torch.empty_like(du), torch.empty_like(dchi), torch.empty_like(dal)
    loss = torch.zeros((), dtype=torch.float64, device="cuda:0")
    nfl = plan.n_frames if frames is None else len(frames)
    fl = torch.zeros(max(nfl, 1), dtype=torch.float32, device="cuda:0") if frame_loss else None
    plan.mpbp_loss_grad(du, dchi, dal, dpr, dy, gu, gc, ga, frames=frames, loss=loss, frame_loss=fl)
    torch.cuda.synchronize()
    out = {"loss": float(loss.item()), "grad_u": host(gu), "grad_chi": host(gc), "grad_alpha": host(ga)}
    if frame_loss:
        out["frame_loss"] = host(fl)[:nfl]
    return out


def gpu_forward(plan, u, chi, alpha, probe, y=None, frames=None, intensity=False):
    import torch
    du, dchi, dal, dpr = dev(u), dev(chi), dev(alpha), dev(probe)
    dy = None if y is None else (y if isinstance(y, torch.Tensor) else dev(y))
    nfl = plan.n_frames if frames is None else len(frames)
    loss = torch.zeros((), dtype=torch.float64, device="cuda:0") if y is not None else None
    fl = torch.zeros(max(nfl, 1), dtype=torch.float32, device="cuda:0") if y is not None else None
    mi = torch.zeros(plan.intensity_size, dtype=torch.float32, device="cuda:0") if intensity else None
    plan.mpbp_forward(du, dchi, dal, dpr, dy, frames=frames, loss=loss, frame_loss=fl, model_intensity=mi)
    torch.cuda.synchronize()
    out = {}
    if y is not None:
        out["loss"] = float(loss.item())
        out["frame_loss"] = host(fl)[:nfl]
    if intensity:
        out["intensity"] = host(mi)
    return out


def assert_grad_close(got, ref, name, rtol=GRAD_RTOL, mask=None):
    """Per field: ||d||_2 <= rtol ||ref||_2 and |d| <= rtol max|ref| + rtol |ref| elementwise."""
    g = np.asarray(got, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    if mask is not None:
        g, r = g[..., mask], r[..., mask]
    d = g - r
    nr = np.linalg.norm(r)
    assert np.linalg.norm(d) <= rtol * nr + 1e-30, f"{name}: |d|={np.linalg.norm(d):.3e} |ref|={nr:.3e}"
    bound = rtol * np.abs(r).max() + rtol * np.abs(r)
    worst = np.max(np.abs(d) - bound)
    assert worst <= 0, f"{name}: elementwise excess {worst:.3e} (max|ref| {np.abs(r).max():.3e})"


def assert_loss_close(got, ref, name="loss", rtol=LOSS_RTOL):
    assert abs(got - ref) <= rtol * abs(ref), f"{name}: {got!r} vs {ref!r} (rel {abs(got - ref) / abs(ref):.3e})"


def speckle_y(prob, seed):
    """Speckle-like Poisson counts under a centred envelope, ragged over peaks."""
    import torch
    g = torch.Generator(device="cuda:0")
    g.manual_seed(seed)
    parts = []
    for m in range(prob.n_peaks):
        d = int(prob.det[m])
        nfr = int(prob.scan_n[m, 0] * prob.scan_n[m, 1])
        k = torch.fft.fftfreq(d, device="cuda:0") * d
        env = torch.exp(-(k[:, None] ** 2 + k[None, :] ** 2) / (2.0 * (d / 10.0) ** 2))
        env = env * (1e5 / d ** 2) / env.mean()
        lam = torch.empty((nfr, d, d), device="cuda:0").exponential_(1.0, generator=g) * env
        parts.append(torch.poisson(lam, generator=g).reshape(-1))
        del lam
    return torch.cat(parts).contiguous()
