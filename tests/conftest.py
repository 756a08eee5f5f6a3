import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def tiny_problem(nz=3, ny=11, nx=9, probe_n=4, dets=(8, 9), shears=((0.6, -1.2), (-1.6, 0.5)),
                 gs=None, scan_n=((3, 2), (2, 3)), steps=((3, 4), (4, 4)),
                 origins=((-1, 0), (2, -2))):
    """A small hand-made geometry with off-grid windows, odd sizes and both shear signs."""
    from synth.inputs import Problem
    m = len(dets)
    if gs is None:
        gs = [(9.0, -4.0, 2.5), (-3.0, 7.0, -5.5), (1.0, 1.0, 1.0)][:m]
    return Problem("tiny", nz, ny, nx, probe_n,
                   np.array(gs, dtype=np.float64), np.array(shears, dtype=np.float64),
                   np.array(dets, dtype=np.int64), np.array(scan_n, dtype=np.int64),
                   np.array(steps, dtype=np.int64), np.array(origins, dtype=np.int64))


def random_fields(problem, seed=0, chi_zero_frac=0.0):
    rng = np.random.default_rng(seed)
    nz, ny, nx, n = problem.nz, problem.ny, problem.nx, problem.probe_n
    u = rng.normal(0.0, 0.1, size=(3, nz, ny, nx))
    chi = rng.uniform(0.5, 1.5, size=(nz, ny, nx))
    if chi_zero_frac > 0:
        chi[rng.uniform(size=chi.shape) < chi_zero_frac] = 0.0
    alpha = rng.uniform(0.5, 2.0, size=problem.n_peaks)
    probe = (rng.normal(size=(problem.n_peaks, n, n)) + 1j * rng.normal(size=(problem.n_peaks, n, n)))
    return u, chi, alpha, probe


def ragged(frames):
    return np.concatenate([np.asarray(f, dtype=np.float64).ravel() for f in frames])
