"""Reconstruction loops around the library's objective and gradient.

Host-side control only: every arithmetic step (object build, forward model, gradient,
Adam update, eq. (8) exponentials, sums of squares, gradient steps) runs in the
library's kernels; the loops choose frames and step sizes.  Device buffers are torch
CUDA tensors.

  adam_reconstruct      Algorithm 1: shuffled minibatches (JD/b per shuffle), minibatch gradients
                        (eq. (11)), Adam on u and the log variables chi~ = log chi,
                        alpha~ = log alpha (eq. (8)), and with unwrap=True the
                        phase-unwrap projection Pi_U of eq. (10) after every update
                        (without it: the concurrent-wrapped variant).
  line_search_descent   full-batch gradient descent on u with a backtracking (Armijo)
                        step-size search.
"""
import math
import time

import numpy as np
import torch


def minibatch_frames(order, n_frames, batch, it):
    """The frame ids of iteration `it` of Algorithm 1 (section 3.3).

    A pass over the data draws a new shuffle of all n_frames patterns and takes
    floor(n_frames / batch) minibatches of `batch` consecutive entries from it; the
    n_frames mod batch entries at its end are not visited in that pass.  `order` is the
    concatenation of the shuffles (whole shuffles only), reused cyclically when the
    iterations outrun it.
    """
    if not 1 <= batch <= n_frames:
        raise ValueError(f"batch must be in [1, {n_frames}] (got {batch})")
    n_shuffles, rest = divmod(len(order), n_frames)
    if n_shuffles == 0 or rest:
        raise ValueError(f"order must concatenate whole shuffles of {n_frames} frames (got {len(order)} ids)")
    per_pass = n_frames // batch
    shuffle = (it // per_pass) % n_shuffles
    first = shuffle * n_frames + (it % per_pass) * batch
    return order[first:first + batch]


def adam_reconstruct(plan, probe, y, u, chi_log, alpha_log, order, batch=50, iterations=None,
                     lr=(0.01, 0.1, 0.1), fixed_alpha=0, beta1=0.9, beta2=0.999, eps=1e-8, unwrap=False):
    """Run `iterations` minibatch iterations (default: every minibatch of every shuffle
    in `order`).

    u, chi_log, alpha_log: device float32 tensors updated in place (u in the layout of
    the plan; chi_log like chi; alpha_log [n_peaks]).  order: host int array, shuffles
    of all the plan's frame ids concatenated; iteration `it` uses
    minibatch_frames(order, n_frames, batch, it).
    Returns (chi, alpha, losses): the model variables exp(chi_log), exp(alpha_log) and
    the minibatch loss of every iteration (before its update), as a float64 array.
    """
    order = np.ascontiguousarray(np.asarray(order, dtype=np.int32))
    n_frames = plan.n_frames
    n_iter = iterations if iterations is not None else (len(order) // n_frames) * (n_frames // batch)
    minibatch_frames(order, n_frames, batch, 0)          # validates order and batch
    dev = u.device
    chi = torch.empty_like(chi_log)
    alpha = torch.empty_like(alpha_log)
    nf = chi.numel()
    state = torch.empty(2 * (4 * nf + alpha.numel()), dtype=torch.float32, device=dev)
    gu, gc, ga = torch.empty_like(u), torch.empty_like(chi), torch.empty_like(alpha)
    hist = torch.zeros(max(n_iter, 1), dtype=torch.float64, device=dev)
    cfg = {"lr": lr, "beta1": beta1, "beta2": beta2, "eps": eps, "log_params": 1, "fixed_alpha": fixed_alpha}
    plan.mpbp_adam_step(cfg, 0, u, chi, alpha, chi_log, alpha_log, state, None, None, None)
    for it in range(n_iter):
        frames = minibatch_frames(order, n_frames, batch, it)
        plan.mpbp_loss_grad(u, chi, alpha, probe, y, gu, gc, ga, frames=frames, loss=hist[it:it + 1])
        plan.mpbp_adam_step(cfg, it + 1, u, chi, alpha, chi_log, alpha_log, state, gu, gc, ga)
        if unwrap:
            plan.mpbp_unwrap_project(u)
    torch.cuda.synchronize(dev)
    return chi, alpha, hist[:n_iter].cpu().numpy()


def line_search_descent(plan, probe, y, u, chi, alpha, iterations=200, step0=0.01, c=1e-4, shrink=0.5,
                        grow=2.0, max_backtracks=30):
    """Full-batch gradient descent on u (chi and alpha held) with Armijo backtracking.

    Each iteration evaluates f and g = df/du at u, then tries u - eta g, with eta the
    previous accepted step grown by `grow` (first: step0 over the RMS of g), shrinking
    it by `shrink` until f(u - eta g) <= f(u) - c eta |g|^2.  u is updated in place.
    Returns a dict: losses (before each iteration), etas (accepted steps), evaluations
    (objective evaluations per iteration), seconds (wall time per iteration), and trials:
    per iteration, the (eta, f(u - eta g)) pairs tried in order and |g|^2.
    """
    dev = u.device
    gu, gc, ga = torch.empty_like(u), torch.empty_like(chi), torch.empty_like(alpha)
    zc, za = torch.zeros_like(chi), torch.zeros_like(alpha)
    trial = torch.empty_like(u)
    chi_t, alpha_t = chi.clone(), alpha.clone()
    f0 = torch.zeros((), dtype=torch.float64, device=dev)
    f1 = torch.zeros((), dtype=torch.float64, device=dev)
    n2 = torch.zeros((), dtype=torch.float64, device=dev)
    out = {"losses": [], "etas": [], "evaluations": [], "seconds": [], "trials": []}
    eta = None
    for _ in range(iterations):
        t0 = time.perf_counter()
        plan.mpbp_loss_grad(u, chi, alpha, probe, y, gu, gc, ga, loss=f0)
        plan.mpbp_norm2(gu, n2)
        F, N = float(f0.item()), float(n2.item())
        out["losses"].append(F)
        if N == 0.0:
            break
        eta = step0 / math.sqrt(N / gu.numel()) if eta is None else eta * grow
        evals, accepted = 1, False
        tried = []
        out["trials"].append({"norm2": N, "tried": tried})
        for _ in range(max_backtracks):
            trial.copy_(u)
            plan.mpbp_step(trial, chi_t, alpha_t, gu, zc, za, (eta, 0.0, 0.0))
            plan.mpbp_forward(trial, chi, alpha, probe, y, loss=f1)
            evals += 1
            F1 = float(f1.item())
            tried.append((eta, F1))
            if F1 <= F - c * eta * N:
                u.copy_(trial)
                out["etas"].append(eta)
                accepted = True
                break
            eta *= shrink
        torch.cuda.synchronize(dev)
        out["evaluations"].append(evals)
        out["seconds"].append(time.perf_counter() - t0)
        if not accepted:
            break
    return out
