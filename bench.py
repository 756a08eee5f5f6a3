"""Benchmark of the MPBP loss-and-gradient evaluation on one MI355X.

One step = one mpbp_loss_grad call over every frame (all Bragg peaks, all scan
positions) of the workload, inputs resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c5_full]
                    [--no-cpu-baseline] [--no-plain] [--no-extras]
    python bench.py --loop 200     # the full-batch descent loop from u = 0 (loss curve)
    python bench.py --options-only # the forward-model options alone (profiling their kernels)
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# FP32 vector peak without packed-FP32 instructions (the device code is compiled without them):
# 256 CUs x 4 SIMDs x 16 lanes x 2 flop (FMA) x 2.4 GHz.
ALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
METRIC = "loss+gradient scan-positions/s at stated tol; batched-fused vs plain, % HBM peak"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", default="c5_full")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-plain", action="store_true")
    p.add_argument("--no-extras", action="store_true",
                   help="skip the unwrap projector, paper-shaped workload and option timings (profiling runs)")
    p.add_argument("--options-only", action="store_true",
                   help="instead of the step benchmark: only the forward-model option timings of the "
                        "workload (one JSON line; profiling runs of the option kernels)")
    p.add_argument("--no-autotune", action="store_true", help="keep the default launch parameters")
    p.add_argument("--loop", type=int, default=0,
                   help="instead of the step benchmark: this many iterations of full-batch gradient "
                        "descent on u with an Armijo line search from u = 0, and the oracle's iteration "
                        "time on a one-eighth crop of the workload")
    p.add_argument("--calib-copy-mib", type=int, default=0,
                   help="first run a plain elementwise copy (out = -in) of this many MiB, the "
                        "known-size reference for HBM byte counters")
    return p.parse_args()


def frame_kernel_work(prob, tab_shear):
    """Algorithmic HBM bytes and nominal FLOPs of the per-frame transform kernel
    (k_frames) for all frames.

    Bytes per frame: the measured intensities, 4 D^2 (read once).  FLOPs per frame
    (5 N log2 N per complex N-point transform): forward and adjoint transforms of the
    F_x footprint columns and of all D rows, and 12 per detector pixel for the modulus
    residual.  (The sheared projection, 8 Np^2 Nz per frame, runs in k_project.)
    """
    import math
    import numpy as np
    nbytes, flops = 0.0, 0.0
    for m in range(prob.n_peaks):
        d = int(prob.det[m])
        nfr = int(prob.scan_n[m, 0] * prob.scan_n[m, 1])
        span_x = int(tab_shear[m, :, 1].max() - tab_shear[m, :, 1].min())
        fx = prob.probe_n + span_x
        fft = 5.0 * d * math.log2(d)
        per = 2 * fx * fft + 2 * d * fft + 12.0 * d * d
        nbytes += nfr * 4.0 * d * d
        flops += nfr * per
    return nbytes, flops


def measured_copy_gbps(torch, mib=1024, reps=10):
    """Bandwidth of a plain device-to-device copy of `mib` MiB (bytes read + written per
    second, median of `reps`): the HBM rate a streaming kernel reaches on this GPU."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        ts.append(a.elapsed_time(b) / 1e3)
    del src, dst
    return 2 * n * 4 / sorted(ts)[len(ts) // 2] / 1e9


def step_bytes(prob):
    """Algorithmic HBM bytes of one loss+gradient step: y once, plus 32 B per voxel
    (read u and chi, write their gradients), plus the probe."""
    nvox = prob.nz * prob.ny * prob.nx
    y = sum(4.0 * int(prob.det[m]) ** 2 * int(prob.scan_n[m, 0] * prob.scan_n[m, 1])
            for m in range(prob.n_peaks))
    return y + 32.0 * nvox + 8.0 * prob.n_peaks * prob.probe_n ** 2


def code_text(src):
    """A source file's code without its comments and with runs of white space made one
    space (edits to comments leave it unchanged)."""
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return re.sub(r"\s+", " ", src).strip()


def frame_kernel_sources(root=ROOT):
    """The frame kernel's translation units (mpbp_frames_<D>.hip) and every header of the
    library they include, directly or through other headers, in name order."""
    csrc = os.path.join(root, "paper_2312_14907_amd", "csrc")
    todo = [f for f in os.listdir(csrc) if re.fullmatch(r"mpbp_frames_\d+\.hip", f)]
    seen = set()
    while todo:
        f = todo.pop()
        if f in seen or not os.path.exists(os.path.join(csrc, f)):
            continue
        seen.add(f)
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            todo += re.findall(r'#include\s+"([^"]+)"', fh.read())
    return sorted(seen)


def kernel_source_hash(root=ROOT):
    """sha256 (first 16 hex digits) of the code of the frame kernel's sources
    (frame_kernel_sources(), comments left out): a committed counter summary of the
    frame kernel applies while it matches."""
    h = hashlib.sha256()
    csrc = os.path.join(root, "paper_2312_14907_amd", "csrc")
    for f in frame_kernel_sources(root):
        with open(os.path.join(csrc, f), encoding="utf-8") as fh:
            h.update(f.encode() + b"\0" + code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload):
    """HBM bytes per launch of the frame kernel from the committed counter summary, if it
    was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"k_frames_{workload}_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel source sha256\[:16\]:\s*([0-9a-f]{16})", text)
    t = re.search(r"HBM bytes per launch \(scaled\):\s*([0-9.eE+]+)", text)
    if not m or not t or m.group(1) != kernel_source_hash():
        return None
    return float(t.group(1))


def make_inputs(name, torch):
    """Seeded synthetic workload on the device; y = Poisson counts of the library's
    own forward model at the true fields."""
    import numpy as np
    from paper_2312_14907_amd.binding import Plan
    from synth import get_config, make_fields, make_problem
    cfg = get_config(name)
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    plan = Plan(prob, 0)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    u_true, chi, alpha, probe = d(f["u"]), d(f["chi"]), d(f["alpha"]), d(f["probe"])
    inten = torch.zeros(plan.intensity_size, dtype=torch.float32, device="cuda:0")
    plan.mpbp_forward(u_true, chi, alpha, probe, model_intensity=inten)
    g = torch.Generator(device="cuda:0")
    g.manual_seed(cfg["seed"])
    y = torch.poisson(inten, generator=g) if cfg["noise"] else inten.clone()
    del inten
    u = d((f["u"] + f["delta"]).astype(np.float32))
    torch.cuda.synchronize()
    return cfg, prob, f, plan, (u, chi, alpha, probe, y)


def time_steps(plan, args_t, steps, warmup, torch):
    u, chi, alpha, probe, y = args_t
    gu, gc, ga = torch.empty_like(u), torch.empty_like(chi), torch.empty_like(alpha)
    loss = torch.zeros((), dtype=torch.float64, device="cuda:0")
    for _ in range(warmup):
        plan.mpbp_loss_grad(u, chi, alpha, probe, y, gu, gc, ga, loss=loss)
    torch.cuda.synchronize()
    plan.mpbp_stage_times()                      # reset accumulators
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.mpbp_loss_grad(u, chi, alpha, probe, y, gu, gc, ga, loss=loss)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return dt, plan.mpbp_stage_times(), float(loss.item())


def baseline_band(prob):
    """The oracle's sample of the workload: one band of 8 scan rows of every peak's
    raster (all columns), in the middle of the rasters, with only the object rows those
    frames reach (one eighth of c5_full's 12288 frames)."""
    r0 = max(0, int(prob.scan_n[:, 0].max()) // 2 - 4)
    return r0, r0 + 8


def cpu_baseline(name, plan, args_t, torch):
    """The FP64 oracle on the band crop (single process, one thread), and the accuracy
    of the timed launch configuration on the same frames.

    The band's intensities are replaced on the device by Poisson counts of the oracle's
    own forward model at the true fields (seeded per frame); the oracle's loss and
    gradient on the cropped band are timed; the plan, as tuned for the timed steps,
    then evaluates the same frames as a minibatch, and its loss, frame losses and
    gradients are compared with the oracle's (loss relative 1e-5; every gradient field
    ||d||_2 <= 1e-3 ||ref||_2, on the band's object rows; zero elsewhere)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import mpbp_oracle as O
    from synth import band_problem, get_config, make_fields, make_problem
    cfg = get_config(name)
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    r0, r1 = baseline_band(prob)
    band, lo, hi, gids = band_problem(prob, r0, r1)
    crop = np.s_[..., lo:hi, :]
    inten = O.model_intensity(f["u"][crop], f["chi"][crop], f["alpha"], f["probe"], band)
    ys = [np.random.default_rng([cfg["seed"], g]).poisson(np.clip(i, 0, None)).astype(np.float32) for g, i in
          zip(gids, inten)]
    u = (f["u"] + f["delta"]).astype(np.float32)
    with threadpool_limits(limits=1):      # one core: the figure is per host core
        t0 = time.perf_counter()
        ref = O.loss_grad(u[crop], f["chi"][crop], f["alpha"], f["probe"], np.concatenate([a.ravel() for a in ys]),
                          band)
        dt = time.perf_counter() - t0
    # the band's counts into the device intensities, then the plan on the band's frames
    du, dchi, dal, dpr, dy = args_t
    _, _, y_off = plan.mpbp_tables()
    fpp = prob.frames_per_peak()
    first = np.concatenate([[0], np.cumsum(fpp)])
    for g, a in zip(gids, ys):
        m = int(np.searchsorted(first, g, side="right") - 1)
        d = int(prob.det[m])
        s = int(y_off[m]) + (g - int(first[m])) * d * d
        dy[s:s + d * d] = torch.from_numpy(a.ravel()).to(dy.device)
    du.copy_(torch.from_numpy(u))
    gu, gc, ga = torch.empty_like(du), torch.empty_like(dchi), torch.empty_like(dal)
    loss = torch.zeros((), dtype=torch.float64, device=du.device)
    fl = torch.zeros(len(gids), dtype=torch.float32, device=du.device)
    plan.mpbp_loss_grad(du, dchi, dal, dpr, dy, gu, gc, ga, frames=gids, loss=loss, frame_loss=fl)
    torch.cuda.synchronize()
    gu, gc, ga = gu.cpu().numpy(), gc.cpu().numpy(), ga.cpu().numpy().astype(np.float64)

    def rel(a, b):
        return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))

    acc = {"frames": len(gids), "loss_rel": abs(loss.item() - ref["loss"]) / abs(ref["loss"]),
           "frame_loss_max_rel": float(np.max(np.abs(fl.cpu().numpy() - ref["frame_loss"]) /
                                              np.abs(ref["frame_loss"]))),
           "grad_u_rel": max(rel(gu[c][crop], ref["grad_u"][c]) for c in range(3)),
           "grad_chi_rel": rel(gc[crop], ref["grad_chi"]), "grad_alpha_rel": rel(ga, ref["grad_alpha"]),
           "outside_band_max_abs": float(max(np.abs(gu[..., :lo, :]).max(initial=0), np.abs(gu[..., hi:, :]).max(initial=0),
                                             np.abs(gc[..., :lo, :]).max(initial=0), np.abs(gc[..., hi:, :]).max(initial=0)))}
    acc["tolerance"] = {"loss_rel": 1e-5, "grad_rel": 1e-3}
    acc["ok"] = bool(acc["loss_rel"] <= 1e-5 and max(acc["grad_u_rel"], acc["grad_chi_rel"], acc["grad_alpha_rel"]) <= 1e-3
                     and acc["outside_band_max_abs"] == 0.0)
    sample = (f"FP64 oracle loss+gradient on one band of {name}: raster rows {r0}-{r1 - 1} of each of the "
              f"{prob.n_peaks} peaks ({len(gids)} frames), object rows {lo}-{hi - 1} ({hi - lo} of {prob.ny}): "
              f"{dt:.1f} s")
    return len(gids) / dt, sample, acc


def cpu_baseline_all_cores(workload, n_frames, total_frames):
    """The same oracle call in W concurrent CPU-only child processes (W = the host cores
    this process may use, at most 16), each on its own band of 8 scan rows (with the
    object rows it reaches) and one thread; set-up happens before a common start, so the
    wall time from the start to the last finish covers W oracle calls."""
    import subprocess
    import tempfile
    from synth import get_config, make_problem
    prob = make_problem(get_config(workload))
    rows = int(prob.scan_n[:, 0].max())
    w_count = max(1, min(len(os.sched_getaffinity(0)), 16))
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
               HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="")
    go = os.path.join(tempfile.mkdtemp(prefix="mpbp_cpu_"), "go")
    procs = [subprocess.Popen([sys.executable, "-m", "oracle.time_worker", workload,
                               str((8 * w) % max(rows - 7, 1)), "8", go],
                              cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                              text=True) for w in range(w_count)]
    try:
        for p in procs:
            if p.stdout.readline().strip() != "ready":
                raise RuntimeError("oracle timing worker failed: " + p.stderr.read()[-2000:])
        t0 = time.perf_counter()
        open(go, "w").close()
        outs = [p.communicate(timeout=900) for p in procs]
        wall = time.perf_counter() - t0
    finally:
        for p in procs:
            if p.poll() is None:
                p.kill()
    for p, (out, err) in zip(procs, outs):
        if p.returncode != 0:
            raise RuntimeError("oracle timing worker failed: " + err[-2000:])
    lines = [o.strip().splitlines()[-1].split() for o, _ in outs]
    frames = sum(int(a) for a, _ in lines)
    calls = [float(b) for _, b in lines]
    return {"value": round(frames / wall, 2), "unit": "scan-positions/s", "cores": w_count,
            "kind": "oracle",
            "sample": f"{w_count} concurrent single-thread processes, each the FP64 oracle's "
                      f"loss+gradient on its own band of 8 scan rows of every peak of {workload} "
                      f"({frames // w_count} frames, with the object rows they reach): "
                      f"{wall:.1f} s wall (calls {min(calls):.1f}-{max(calls):.1f} s)"}


def unwrap_inputs(prob, nz):
    """Seeded displacement field on the workload's grid for the unwrap projector: a
    smooth strain field with noise and one lattice-translation artefact on a patch."""
    from synth import lattice_jump, unwrap_field
    u = unwrap_field(nz, prob.ny, prob.nx, seed=5, noise_nm=0.03)
    return lattice_jump(u, prob.ny // 5, 3 * prob.ny // 5, prob.nx // 10, prob.nx // 2)


def time_unwrap(prob, torch, calls):
    """ms per mpbp_unwrap_project call on the workload's lateral grid, z-tied (one map per
    peak, the paper's 2D unwrapping) and per slice (one map per peak and slice)."""
    from paper_2312_14907_amd.binding import MPBP_Z_TIED, Plan
    out = {}
    for name, flags, nz in (("tied", MPBP_Z_TIED, 1), ("slices", 0, prob.nz)):
        plan = Plan(prob, 0, flags=flags)
        u0 = torch.from_numpy(unwrap_inputs(prob, nz)).to("cuda:0")
        u = u0.clone()
        plan.mpbp_unwrap_project(u)            # workspace allocation, warm-up
        ts = []
        for _ in range(calls):
            u.copy_(u0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            plan.mpbp_unwrap_project(u)        # synchronous
            ts.append(time.perf_counter() - t0)
        ms = 1e3 * sorted(ts)[len(ts) // 2]
        px = prob.n_peaks * nz * prob.ny * prob.nx
        out[name] = {"maps": prob.n_peaks * nz, "map": [prob.ny, prob.nx], "ms_per_call": round(ms, 3),
                     "map_pixels_per_s": round(px / ms * 1e3, 1)}
        plan.close()
    return out


def time_paper_shape(torch, name="c6_paper", steps=20):
    """A paper-shaped workload (150 x 150 detectors, four in-plane peaks, 9 x 9 rasters; 32
    slices, or the paper's 100-voxel window with c6_paper100): loss+gradient steps after
    autotuning."""
    cfg, prob, f, plan, args_t = make_inputs(name, torch)
    plan.mpbp_autotune(*args_t)
    dt, _, _ = time_steps(plan, args_t, steps, 3, torch)
    nfr = prob.n_frames()
    t = plan.mpbp_tuning()
    plan.close()
    return {"workload": name, "frames": nfr, "detector": 150, "peaks": prob.n_peaks, "slices": prob.nz,
            "ms_per_step": round(1e3 * dt / steps, 4), "value": round(nfr * steps / dt, 1),
            "unit": "scan-positions/s",
            "launch": [{k: c[k] for k in ("fy", "fx", "FB", "G", "xcd")} for c in t["classes"]]}


# Per peak: (ratio of voxel pitch to exit-wave pixel pitch, detector-frame angle in rad)
# of the detector maps timed in the option extras.
OPTION_MAPS = [(1.2, 0.4), (0.9, 2.5), (1.05, -0.7)]


def time_options(torch, name, steps=10):
    """The forward-model options on workload `name` (not part of `value`): interpolated
    exit-beam offsets, 3D illumination volumes, detector maps, the z-tied
    parameterisation and the background, each autotuned and timed over `steps`
    loss+gradient steps with every stage timed (HIP events per stage).  Counts are
    Poisson draws of the library's own model intensities at the true fields of each
    option's model."""
    import dataclasses
    import numpy as np
    from paper_2312_14907_amd import binding as B
    from synth import get_config, incident_probe_3d, make_fields, make_problem
    from synth.inputs import detector_map
    cfg = get_config(name)
    base = make_problem(cfg)
    f = make_fields(cfg, base)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    rng = np.random.default_rng(cfg["seed"] + 1)
    p3 = np.stack([incident_probe_3d(f["probe"][m], base.nz, rng.uniform(-0.4, 0.4, 2))
                   for m in range(base.n_peaks)]).astype(np.complex64)
    u_t, u_e = f["u"], (f["u"] + f["delta"]).astype(np.float32)
    chi2 = np.full((1, base.ny, base.nx), float(f["chi"].max()), dtype=np.float32)
    cases = [
        ("interpolated_offsets", dataclasses.replace(base, shear_linear=True), B.MPBP_SHEAR_LINEAR, f["probe"],
         u_t, u_e, f["chi"], False),
        ("probe_3d", base, B.MPBP_PROBE_3D, p3, u_t, u_e, f["chi"], False),
        ("detector_map", dataclasses.replace(base, lateral_map=np.stack([detector_map(r, a) for r, a in OPTION_MAPS])),
         B.MPBP_DETECTOR_MAP, f["probe"], u_t, u_e, f["chi"], False),
        ("z_tied", base, B.MPBP_Z_TIED, f["probe"], np.ascontiguousarray(u_t[:, :1]),
         np.ascontiguousarray(u_e[:, :1]), chi2, False),
        ("background", base, 0, f["probe"], u_t, u_e, f["chi"], True),
    ]
    out = {}
    for key, prob, flags, probe, ut, ue, chi, with_bg in cases:
        plan = B.Plan(prob, 0, flags=flags)
        dchi, alpha, dprobe = d(chi), d(f["alpha"]), d(probe)
        if with_bg:
            g = torch.Generator(device="cuda:0")
            g.manual_seed(cfg["seed"] + 2)
            bg = 0.5 * torch.rand(plan.intensity_size, generator=g, device="cuda:0")
            plan.mpbp_set_background(bg)
        inten = torch.zeros(plan.intensity_size, dtype=torch.float32, device="cuda:0")
        plan.mpbp_forward(d(ut), dchi, alpha, dprobe, model_intensity=inten)
        g = torch.Generator(device="cuda:0")
        g.manual_seed(cfg["seed"])
        y = torch.poisson(inten, generator=g)
        del inten
        args_t = (d(ue), dchi, alpha, dprobe, y)
        plan.mpbp_autotune(*args_t)
        plan.mpbp_set_option(B.MPBP_OPT_PROFILE, 1)
        dt, st, _ = time_steps(plan, args_t, steps, 3, torch)
        plan.close()
        del y, args_t
        out[key] = {"ms_per_step": round(1e3 * dt / steps, 4),
                    "stages_ms_per_step": {k: round(v[0] / steps, 4) for k, v in st.items() if v[1]}}
    out["note"] = (f"{name}, every stage timed (its events add a few percent); detector maps per peak "
                   f"(pixel ratio, angle in rad): {OPTION_MAPS}")
    return out


def cpu_unwrap(prob):
    """The unwrap oracle on the z-tied maps of the workload (one per peak), seconds."""
    from threadpoolctl import threadpool_limits
    from oracle import unwrap_oracle as U
    u = unwrap_inputs(prob, 1)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        U.unwrap_projector(u, prob.g)
        return time.perf_counter() - t0


def run_loop(args, torch):
    """Full-batch descent on u from u = 0 (chi and alpha at the truth) with an Armijo
    line search; the loss curve and the time per iteration, beside the oracle's time per
    iteration of the same loop on a one-eighth crop (c5_crop8 for c5_full)."""
    import numpy as np
    from paper_2312_14907_amd import optim
    cfg, prob, f, plan, (u, chi, alpha, probe, y) = make_inputs(args.workload, torch)
    if not args.no_autotune:
        plan.mpbp_autotune(u, chi, alpha, probe, y)
    u0 = torch.zeros_like(u)
    t0 = time.perf_counter()
    r = optim.line_search_descent(plan, probe, y, u0, chi, alpha, iterations=args.loop)
    total = time.perf_counter() - t0
    losses = r["losses"]
    n = len(r["seconds"])
    marks = sorted(set(list(range(0, len(losses), max(1, len(losses) // 20))) + [len(losses) - 1]))
    out = {
        "loop": "full-batch gradient descent on u with Armijo line search, u0 = 0",
        "workload": args.workload,
        "frames": prob.n_frames(),
        "iterations": n,
        "seconds_total": round(total, 3),
        "ms_per_iteration": round(1e3 * float(np.mean(r["seconds"])), 3) if n else None,
        "evaluations_per_iteration": round(float(np.mean(r["evaluations"])), 3) if n else None,
        "loss_first": losses[0],
        "loss_last": losses[-1],
        "loss_curve": {str(i): losses[i] for i in marks},
        "launch": plan.mpbp_tuning()["classes"],
    }
    if not args.no_cpu_baseline:
        from oracle import mpbp_oracle as O
        from synth import make_fields as mf, make_problem as mp
        from synth.inputs import speckle_counts
        crop = "c5_crop8" if args.workload == "c5_full" else args.workload
        ccfg = get_config_named(crop)
        cprob = mp(ccfg)
        cf = mf(ccfg, cprob)
        rng = np.random.default_rng(ccfg["seed"])
        cy = np.concatenate([speckle_counts(rng, int(cprob.det[m]), int(cprob.scan_n[m].prod()), 1e5).ravel()
                             for m in range(cprob.n_peaks)])
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1):
            t1 = time.perf_counter()
            _, cl, _ = O.line_search_descent(np.zeros_like(cf["u"]), cf["chi"], cf["alpha"], cf["probe"], cy,
                                             cprob, iterations=1)
            cdt = time.perf_counter() - t1
        out["cpu_baseline"] = {"kind": "oracle", "cores": 1, "workload": crop, "frames": cprob.n_frames(),
                               "seconds_per_iteration": round(cdt, 2),
                               "note": "one iteration of the same loop (one loss+gradient evaluation and the "
                                       "line-search objective evaluations) on model-free speckle counts"}
    print(json.dumps(out), flush=True)


def get_config_named(name):
    from synth import get_config
    return get_config(name)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (got --gpus {args.gpus}); "
              "sharding over several GPUs (bands of scan rows with a halo reduction of the gradient) is designed but not built", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2312_14907_amd.binding import MPBP_OPT_PATH, MPBP_OPT_PROFILE

    if args.loop > 0:
        run_loop(args, torch)
        return
    if args.options_only:
        print(json.dumps({"workload": args.workload, "options": time_options(torch, args.workload, args.steps)}),
              flush=True)
        return

    cfg, prob, f, plan, args_t = make_inputs(args.workload, torch)
    calib = None
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.empty(n, dtype=torch.float32, device="cuda:0").fill_(1.0)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)          # reads and writes n * 4 bytes
        torch.cuda.synchronize()
        del src, dst
        calib = {"kernel": "torch neg (elementwise)", "bytes_read": 4 * n, "bytes_written": 4 * n}
    copy_gbps = measured_copy_gbps(torch)
    if not args.no_autotune:
        plan.mpbp_autotune(*args_t)
    tuning = plan.mpbp_tuning()
    # The timed steps: direct launches with HIP events around the frame stage only (the
    # dominant kernel's duration for the roofline; the least the events add to a step).
    plan.mpbp_set_option(MPBP_OPT_PROFILE, 2)
    dt, stages, loss = time_steps(plan, args_t, args.steps, args.warmup, torch)
    # every stage timed, in a pass of its own (the breakdown; its events cost a few
    # percent of the step)
    plan.mpbp_set_option(MPBP_OPT_PROFILE, 1)
    sdt, all_stages, _ = time_steps(plan, args_t, args.steps, 1, torch)
    nfr = prob.n_frames()
    value = nfr * args.steps / dt
    ms_step = 1e3 * dt / args.steps

    _, shear_tab, _ = plan.mpbp_tables()
    fk_bytes, fk_flops = frame_kernel_work(prob, shear_tab)
    fk_ms, fk_n = stages["frames"]
    fk_avg_s = fk_ms / max(fk_n, 1) / 1e3
    achieved_tflops = fk_flops / fk_avg_s / 1e12
    achieved_gbps = fk_bytes / fk_avg_s / 1e9
    traffic = measured_traffic(args.workload)

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "scan-positions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "peaks": prob.n_peaks,
            "object_zyx": [prob.nz, prob.ny, prob.nx],
            "frames": nfr,
            "detector": sorted(set(int(d) for d in prob.det)),
            "probe": prob.probe_n,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_frames",
            "achieved": round(achieved_tflops, 3),
            "peak": round(ALU_PEAK_TFLOPS, 2),
            "unit": "TFLOP/s",
            "frac": round(achieved_tflops / ALU_PEAK_TFLOPS, 4),
            "traffic": traffic,
            "hbm_achieved_GBps": round(achieved_gbps, 1),
            "hbm_frac": round(achieved_gbps / HBM_PEAK_GBPS, 4),
            "avg_launch_ms": round(fk_avg_s * 1e3, 4),
        },
        "hbm_step": {
            "algorithmic_bytes": step_bytes(prob),
            "achieved_GBps": round(step_bytes(prob) / (dt / args.steps) / 1e9, 1),
            "frac": round(step_bytes(prob) / (dt / args.steps) / 1e9 / HBM_PEAK_GBPS, 4),
            "measured_copy_GBps": round(copy_gbps, 1),
            "frac_of_measured_copy": round(step_bytes(prob) / (dt / args.steps) / 1e9 / copy_gbps, 4),
        },
        "stages_ms_per_step": {k: round(v[0] / max(args.steps, 1), 4) for k, v in all_stages.items() if v[1]},
        "stages_pass_ms_per_step": round(1e3 * sdt / args.steps, 4),
        "loss": loss,
        "launch": {"source": tuning["source"], "grad_batch": tuning["grad_batch"],
                   "frame_classes": [{k: c[k] for k in ("D", "frames", "FB", "G", "xcd", "us")}
                                     for c in tuning["classes"]]},
    }
    if calib:
        out["calibration"] = calib

    # the same steps replayed from the captured graph (no stage events)
    plan.mpbp_set_option(MPBP_OPT_PROFILE, 0)
    gdt, _, _ = time_steps(plan, args_t, args.steps, 1, torch)
    out["graph_replay"] = {"ms_per_step": round(1e3 * gdt / args.steps, 4),
                           "value": round(nfr * args.steps / gdt, 1)}

    if not args.no_plain:
        plan.mpbp_set_option(MPBP_OPT_PATH, 1)
        pdt, _, ploss = time_steps(plan, args_t, 1, 1, torch)
        plan.mpbp_set_option(MPBP_OPT_PATH, 0)
        out["plain"] = {"value": round(nfr / pdt, 1), "ms_per_step": round(1e3 * pdt, 2),
                        "speedup_fused_vs_plain": round((nfr / pdt and value / (nfr / pdt)), 2),
                        "loss_rel_diff": abs(ploss - loss) / abs(loss)}

    if not args.no_extras:
        # the unwrap projector of eq. (10), the last step of Algorithm 1, and the
        # paper-shaped workload (neither is part of `value`)
        out["unwrap"] = time_unwrap(prob, torch, 10)
        out["paper_shape"] = time_paper_shape(torch)
        out["paper_shape_100_slices"] = time_paper_shape(torch, "c6_paper100")
        out["options"] = time_options(torch, args.workload)

    if not args.no_cpu_baseline:
        rate, sample, acc = cpu_baseline(args.workload, plan, args_t, torch)
        out["cpu_baseline"] = {"value": round(rate, 2), "unit": "scan-positions/s", "cores": 1, "kind": "oracle",
                               "sample": sample}
        out["accuracy"] = acc
        out["cpu_baseline"]["all_cores"] = cpu_baseline_all_cores(args.workload, 0, prob.n_frames())
        if "unwrap" in out:
            usec = cpu_unwrap(prob)
            out["cpu_baseline"]["unwrap_tied_s_per_call"] = round(usec, 3)
            out["unwrap"]["tied"]["speedup_vs_oracle"] = round(usec / (out["unwrap"]["tied"]["ms_per_call"] / 1e3), 1)
    print(json.dumps(out), flush=True)
    if "accuracy" in out and not out["accuracy"]["ok"]:
        print("bench.py: the timed launch configuration is outside the stated tolerance against the oracle",
              file=sys.stderr)
        sys.exit(1)


if __name__ == "__main__":
    main()
