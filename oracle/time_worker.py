"""Timing worker of the benchmark's CPU-baseline leg on all host cores.

TEST INFRASTRUCTURE.  Only the benchmark's CPU-baseline leg runs this module, as a
CPU-only child process (it imports neither torch nor the GPU library).  It times one
call of the FP64 oracle's loss and gradient (`mpbp_oracle.loss_grad`, unchanged) on a
band of a workload's scan rows with the object rows they reach (synth.band_problem), as
the single-core baseline does; several copies released together give the oracle's
throughput on all host cores.

Usage: python -m oracle.time_worker WORKLOAD ROW0 ROWS GO_FILE

The worker builds the band's problem and fields, and seeded synthetic counts for its
frames (the oracle's cost does not depend on their values), prints "ready", waits until
GO_FILE exists, then prints the band's frame count and the seconds the oracle call took.
"""
import os
import sys
import time

import numpy as np

from oracle import mpbp_oracle as O
from synth import band_problem, get_config, make_fields, make_problem


class FrameCounts:
    """Ragged intensities served by element offset, precomputed for the listed frames."""

    def __init__(self, tab, frames, seed):
        self.parts = {}
        y_off = tab["y_off"]
        for fid in frames:
            m = int(tab["peak_of"][fid])
            det = int(tab["det"][m])
            start = int(y_off[m]) + int(tab["frame_index"][fid]) * det * det
            rng = np.random.default_rng(seed + fid)
            self.parts[start] = rng.poisson(20.0, det * det).astype(np.float32)

    def __getitem__(self, sl):
        return self.parts[sl.start][: sl.stop - sl.start]


def main():
    workload, row0, rows, go = sys.argv[1], int(sys.argv[2]), int(sys.argv[3]), sys.argv[4]
    cfg = get_config(workload)
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    band, lo, hi, _ = band_problem(prob, row0, row0 + rows)
    crop = np.s_[..., lo:hi, :]
    u = (f["u"] + f["delta"]).astype(np.float32)[crop]
    frames = list(range(band.n_frames()))
    tab = O.tables(band)
    y = FrameCounts(_frame_table(band, tab), frames, cfg["seed"])
    print("ready", flush=True)
    while not os.path.exists(go):
        time.sleep(0.002)
    t0 = time.perf_counter()
    O.loss_grad(u, f["chi"][crop], f["alpha"], f["probe"], y, band)
    print(f"{len(frames)} {time.perf_counter() - t0:.6f}", flush=True)


def _frame_table(prob, tab):
    """Peak and index within the peak of every global frame id (peak-major order)."""
    counts = [int(c) for c in prob.frames_per_peak()]
    peak_of = np.repeat(np.arange(len(counts)), counts)
    frame_index = np.concatenate([np.arange(c) for c in counts])
    return {"y_off": tab["y_off"], "peak_of": peak_of, "frame_index": frame_index,
            "det": np.asarray(prob.det)}


if __name__ == "__main__":
    main()
