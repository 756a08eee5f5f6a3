"""The FP64 oracle over a whole workload in parallel CPU processes.

TEST INFRASTRUCTURE.  The frames are split into bands of scan rows (synth.band_problem:
the rows of every peak's raster in the band, and only the object rows those frames
reach).  A CPU-only worker process (numpy; no torch, no GPU library) evaluates each
band with the unchanged oracle: the model intensities at the true fields with seeded
Poisson counts per frame (a counter-based seed (workload seed, global frame id), so the
counts do not depend on the split), then the loss and gradient at the evaluation point.
The band results add up to the whole workload's (eq. (11): the objective and its
gradient are sums over frames; a band's frames touch only its object rows).
"""
import os

import numpy as np


def _band_worker(args):
    name, row0, row1, eval_key, noise = args
    from oracle import mpbp_oracle as O
    from synth import band_problem, get_config, make_fields, make_problem
    cfg = get_config(name)
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    band, lo, hi, gids = band_problem(prob, row0, row1)
    if not gids:
        return None
    sl = np.s_[..., lo:hi, :]
    u_true = f["u"][sl]
    chi, alpha, probe = f["chi"][sl], f["alpha"], f["probe"]
    inten = O.model_intensity(u_true, chi, alpha, probe, band)
    ys = []
    for gid, it in zip(gids, inten):
        if noise:
            rng = np.random.default_rng([cfg["seed"], gid])
            ys.append(rng.poisson(np.clip(it, 0.0, None)).astype(np.float32))
        else:
            ys.append(it.astype(np.float32))
    y = np.concatenate([a.ravel() for a in ys])
    u = np.zeros_like(f["u"][sl]) if eval_key == "zero" else (f["u"] + f["delta"]).astype(np.float32)[sl]
    ref = O.loss_grad(u, chi, alpha, probe, y, band)
    return {"frames": gids, "y": ys, "lo": lo, "hi": hi, "frame_loss": ref["frame_loss"],
            "grad_u": ref["grad_u"], "grad_chi": ref["grad_chi"], "grad_alpha": ref["grad_alpha"]}


def workers():
    """CPU processes to use: the cores this process may run on, at most 16."""
    return max(1, min(len(os.sched_getaffinity(0)), 16))


def oracle_whole(name, rows_per_band, eval_key="delta", noise=True, n_workers=None):
    """Model-consistent data and the FP64 oracle's loss and gradient over every frame of
    workload `name`, computed band by band in parallel.

    eval_key: "delta" (u_true + delta) or "zero" (u = 0).  Returns dict with y (ragged
    float32 in the workload's frame order), frame_loss [F], loss, grad_u, grad_chi,
    grad_alpha.
    """
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor
    from synth import get_config, make_problem
    cfg = get_config(name)
    prob = make_problem(cfg)
    rmax = int(prob.scan_n[:, 0].max())
    jobs = [(name, r, r + rows_per_band, eval_key, noise) for r in range(0, rmax, rows_per_band)]
    # spawned (not forked) workers: the parent may hold a GPU context; a worker that dies
    # fails the call (BrokenProcessPool) instead of being replaced
    with ProcessPoolExecutor(max_workers=min(n_workers or workers(), len(jobs)),
                             mp_context=mp.get_context("spawn")) as pool:
        parts = [p for p in pool.map(_band_worker, jobs) if p is not None]
    nf = prob.n_frames()
    dets = [int(prob.det[m]) for m in range(prob.n_peaks)]
    fpp = prob.frames_per_peak()
    peak_of = np.repeat(np.arange(prob.n_peaks), fpp)
    y_off = np.concatenate([[0], np.cumsum([fpp[m] * dets[m] ** 2 for m in range(prob.n_peaks)])])
    first = np.concatenate([[0], np.cumsum(fpp)])
    y = np.empty(int(y_off[-1]), dtype=np.float32)
    frame_loss = np.full(nf, np.nan)
    grad_u = np.zeros((3, prob.nz, prob.ny, prob.nx))
    grad_chi = np.zeros((prob.nz, prob.ny, prob.nx))
    grad_alpha = np.zeros(prob.n_peaks)
    for p in parts:
        for k, gid in enumerate(p["frames"]):
            m = int(peak_of[gid])
            d = dets[m]
            s = int(y_off[m]) + (gid - int(first[m])) * d * d
            y[s:s + d * d] = p["y"][k].ravel()
            frame_loss[gid] = p["frame_loss"][k]
        grad_u[:, :, p["lo"]:p["hi"], :] += p["grad_u"]
        grad_chi[:, p["lo"]:p["hi"], :] += p["grad_chi"]
        grad_alpha += p["grad_alpha"]
    assert not np.isnan(frame_loss).any(), "a frame was not covered by any band"
    return {"y": y, "frame_loss": frame_loss, "loss": float(np.sum(frame_loss)), "grad_u": grad_u,
            "grad_chi": grad_chi, "grad_alpha": grad_alpha}
