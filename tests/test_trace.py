"""MPBP_TRACE=1: the library logs its plan choices on stderr (CPU, a host-only plan in a
child process)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SNIPPET = """
from synth import get_config, make_problem
from paper_2312_14907_amd.binding import Plan
Plan(make_problem(get_config("c4_batch")), device=-1).close()
"""


def _run(trace):
    env = dict(os.environ, MPBP_TRACE=trace, HIP_VISIBLE_DEVICES="")
    return subprocess.run([sys.executable, "-c", SNIPPET], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=120)


def test_trace_lists_the_plan_choices():
    r = _run("1")
    assert r.returncode == 0, r.stderr
    lines = [ln for ln in r.stderr.splitlines() if ln.startswith("mpbp: ")]
    assert any("created" in ln and "6 peaks" in ln and "5560 frames" in ln for ln in lines), r.stderr
    assert sum("  peak " in ln for ln in lines) == 6
    classes = [ln for ln in lines if "  class " in ln]
    assert len(classes) == 6 and all("footprint bound" in ln and "projection depth" in ln for ln in classes)
    assert any("objects summed per run" in ln and "tuning source default" in ln for ln in lines)
    assert any("LDS bytes" in ln for ln in lines)


def test_no_trace_by_default():
    r = _run("0")
    assert r.returncode == 0, r.stderr
    assert "mpbp: " not in r.stderr
