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


MAP_SNIPPET = """
import dataclasses, numpy as np
from synth import get_config, make_problem
from synth.inputs import detector_map
from paper_2312_14907_amd.binding import Plan, MPBP_DETECTOR_MAP
base = make_problem(get_config("c2_forward"))
prob = dataclasses.replace(base, lateral_map=np.stack([detector_map(r, a) for r, a in
                                                       [(1.2, 0.4), (0.9, 2.5), (1.05, -0.7)]]))
Plan(prob, device=-1, flags=MPBP_DETECTOR_MAP).close()
"""


def test_trace_reports_the_detector_map_colours():
    # frame (iy, ix) of a peak takes colour (iy mod cy) cx + (ix mod cx) with
    # cy = ceil(Np / step_y), cx = ceil(Np / step_x); every frame has one colour
    import math
    sys.path.insert(0, ROOT)
    from synth import get_config, make_problem
    prob = make_problem(get_config("c2_forward"))
    np_ = int(prob.probe_n)
    ncol = max(math.ceil(np_ / int(prob.scan_step[m][0])) * math.ceil(np_ / int(prob.scan_step[m][1]))
               for m in range(prob.n_peaks))
    nfr = sum(int(prob.scan_n[m][0]) * int(prob.scan_n[m][1]) for m in range(prob.n_peaks))
    env = dict(os.environ, MPBP_TRACE="1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([sys.executable, "-c", MAP_SNIPPET], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    line = [ln for ln in r.stderr.splitlines() if "back-projection:" in ln]
    assert len(line) == 1, r.stderr
    assert f" {ncol} colours" in line[0] and line[0].endswith(f"{nfr} in all"), (line[0], ncol, nfr)
    assert sum("detector map [" in ln for ln in r.stderr.splitlines()) == prob.n_peaks
