"""The bounds-checked debug library (libmpbp_debug.so, MPBP_DEBUG): every code path of
the projection and the back-projection on c1 (fused per run and per slice, plain, a
minibatch, z-tied, 3D probes, interpolated offsets, detector maps, the allocation-free
call, graph off),
c2, c4 and the 100-slice paper-shaped workload, with no device-side check firing
(a check that fires makes the call return MPBP_ERR_INTERNAL), and the c1 results within
the parity tolerances of the oracle.  Runs in a child process that loads the debug
library."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DEBUG_LIB = os.path.join(ROOT, "paper_2312_14907_amd", "libmpbp_debug.so")


def test_debug_library_checks_stay_silent():
    assert os.path.exists(DEBUG_LIB), "build the debug library (paper_2312_14907_amd.build.build_debug)"
    env = dict(os.environ, MPBP_LIBRARY=DEBUG_LIB)
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "tests", "debug_lib_run.py")], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=240)
    print(r.stdout[-3000:], flush=True)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-3000:]
    assert r.stdout.strip().splitlines()[-1] == "ok"
