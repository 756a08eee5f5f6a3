"""CPU checks of the C-ABI library: it loads, exports every declared symbol, builds the
integer tables bit-exactly as the oracle does, and rejects bad descriptors with the
documented status codes.  No compute call runs here (no GPU)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from synth import CONFIG_NAMES, get_config, make_problem
from synth.inputs import Problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
B = pytest.importorskip("paper_2312_14907_amd.binding")
from oracle import mpbp_oracle as O  # noqa: E402


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "mpbp.h")).read()
    declared = set(re.findall(r"\b(mpbp_[a-z0-9_]+)\s*\(", header))
    assert declared == set(B.EXPORTED)
    lib = ctypes.CDLL(B.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(lib, name), name


def _supported_problem(shears, dets=(32, 64), nz=7):
    return Problem("abi", nz, 40, 37, 12, np.array([[3.0, -2.0, 1.0], [0.5, 4.0, -1.5]]),
                   np.array(shears, dtype=np.float64), np.array(dets), np.array([[4, 3], [3, 5]]),
                   np.array([[7, 9], [11, 6]]), np.array([[-3, 2], [1, -4]]))


@pytest.mark.parametrize("name", CONFIG_NAMES)
def test_tables_bit_exact_against_oracle(name):
    prob = make_problem(get_config(name))
    plan = B.Plan(prob, device=-1)
    scan, shear, y_off = plan.mpbp_tables()
    tab = O.tables(prob)
    np.testing.assert_array_equal(scan, tab["scan"])
    np.testing.assert_array_equal(shear, tab["shear"])
    np.testing.assert_array_equal(y_off, tab["y_off"])
    assert plan.n_frames == prob.n_frames()
    assert plan.intensity_size == int(tab["y_off"][-1])
    plan.close()


@pytest.mark.parametrize("shears", [
    ((0.5, -0.5), (1.5, 2.5)),               # exact halves round away from zero
    ((0.49999999999999994, -1.0 / 3.0), (0.7, -0.35)),
    ((0.0, 0.0), (-1.25, 0.75)),
])
def test_tables_half_cases(shears):
    prob = _supported_problem(shears)
    plan = B.Plan(prob, device=-1)
    scan, shear, y_off = plan.mpbp_tables()
    tab = O.tables(prob)
    np.testing.assert_array_equal(shear, tab["shear"])
    np.testing.assert_array_equal(scan, tab["scan"])
    np.testing.assert_array_equal(y_off, tab["y_off"])


def _status_of(problem_struct, device=-1):
    h = ctypes.c_void_p()
    st = B.lib.mpbp_plan_create(ctypes.byref(problem_struct) if problem_struct is not None else None,
                                device, ctypes.byref(h))
    if st == 0:
        B.lib.mpbp_plan_destroy(h)
    return st, B.mpbp_last_error()


def test_descriptor_validation_codes():
    good = _supported_problem(((0.3, 0.2), (0.1, -0.4)))
    assert _status_of(B.make_problem_struct(good))[0] == 0
    assert _status_of(None)[0] == 1                       # NULL problem
    s = B.make_problem_struct(good)
    s.flags = 16
    assert _status_of(s)[0] == 1                          # undefined flag
    s.flags = B.MPBP_DETECTOR_MAP | B.MPBP_SHEAR_LINEAR
    assert _status_of(s)[0] == 1                          # the map includes the interpolated offsets
    s.flags = B.MPBP_DETECTOR_MAP | B.MPBP_Z_TIED | B.MPBP_PROBE_3D
    assert _status_of(s)[0] == 0                          # identity maps
    s.flags = B.MPBP_Z_TIED
    assert _status_of(s)[0] == 0                          # membrane parameterisation
    s.flags = B.MPBP_Z_TIED | B.MPBP_PROBE_3D | B.MPBP_SHEAR_LINEAR
    assert _status_of(s)[0] == 0                          # every defined flag together
    bad = _supported_problem(((0.3, 0.2), (0.1, -0.4)), dets=(32, 48))
    st, msg = _status_of(B.make_problem_struct(bad))
    assert st == 2 and "48" in msg                        # unsupported detector size
    bad = _supported_problem(((4.0, 0.2), (0.1, -0.4)))   # shear of 12 px leaves a 32 window
    st, msg = _status_of(B.make_problem_struct(bad))
    assert st == 3 and "window" in msg
    s = B.make_problem_struct(good)
    s.probe_n = 40                                        # above the kernels' 32 x 32 support
    st, msg = _status_of(s)
    assert st == 6 and "probe_n" in msg
    s = B.make_problem_struct(good)
    s.n_peaks = 0
    assert _status_of(s)[0] == 2
    s = B.make_problem_struct(good)
    s.nz = 0
    assert _status_of(s)[0] == 2
    s = B.make_problem_struct(good)
    s.peaks[1].scan_step[0] = 0
    assert _status_of(s)[0] == 2
    s = B.make_problem_struct(good)
    s.peaks[0].g[1] = float("nan")
    assert _status_of(s)[0] == 1
    assert _status_of(B.make_problem_struct(good), device=-2)[0] == 1


def test_host_only_plan_refuses_compute_and_options():
    plan = B.Plan(_supported_problem(((0.3, 0.2), (0.1, -0.4))), device=-1)
    z = np.zeros(1, np.float32)
    with pytest.raises(B.MPBPError) as e:      # the library's own refusal (no device)
        B._check(B.lib.mpbp_forward(plan.handle, z.ctypes.data, z.ctypes.data, z.ctypes.data, z.ctypes.data,
                                    None, None, 0, None, None, None, None))
    assert e.value.status == 4
    with pytest.raises(B.MPBPError) as e:
        plan.mpbp_set_option(99, 0)
    assert e.value.status == 1
    with pytest.raises(B.MPBPError):
        plan.mpbp_set_option(B.MPBP_OPT_PATH, 2)
    plan.mpbp_set_option(B.MPBP_OPT_PATH, 1)
    assert plan.mpbp_get_option(B.MPBP_OPT_PATH) == 1
    assert plan.mpbp_get_option(B.MPBP_OPT_GRAPH) == 1
    assert B.lib.mpbp_num_frames(None) == -1
    assert B.lib.mpbp_intensity_size(None) == -1
    B.lib.mpbp_plan_destroy(None)


def test_launch_parameter_api_on_host_plan():
    """Size classes, variant selection and its validation (no kernel runs)."""
    prob = make_problem(get_config("c4_batch"))
    plan = B.Plan(prob, device=-1)
    t = plan.mpbp_tuning()
    assert t["source"] == "default" and t["grad_batch"] == 8 and t["runs"] == 1 and t["candidates"] == []
    # one class per (detector size, smallest footprint bound); frames add up
    assert sum(c["frames"] for c in t["classes"]) == plan.n_frames
    assert [c["D"] for c in t["classes"]] == sorted([c["D"] for c in t["classes"]], reverse=True)
    for c in t["classes"]:
        assert c["FB"] == c["key"] and c["G"] == 4 and c["xcd"] == 1
        assert max(c["fy"], c["fx"]) <= c["key"]
    k = next(i for i, c in enumerate(t["classes"]) if c["D"] == 256)
    plan.mpbp_set_variant(k, 256, 8, 0)
    c = plan.mpbp_tuning()["classes"][k]
    assert (c["FB"], c["G"], c["xcd"]) == (256, 8, 0)
    assert plan.mpbp_tuning()["source"] == "manual"
    for args, status in (((len(t["classes"]), 48, 4, 1), 1),   # class out of range
                         ((k, 32, 4, 1), 6),                  # bound below the footprint
                         ((k, 48, 3, 1), 6),                  # slab depth not compiled
                         ((k, 48, 4, 2), 1)):                 # bad xcd flag
        with pytest.raises(B.MPBPError) as e:
            plan.mpbp_set_variant(*args)
        assert e.value.status == status
    for v in (1, 2, 4, 8, 16):
        plan.mpbp_set_option(B.MPBP_OPT_GRAD_BATCH, v)
        assert plan.mpbp_get_option(B.MPBP_OPT_GRAD_BATCH) == v
    for v in (3, 32):
        with pytest.raises(B.MPBPError):
            plan.mpbp_set_option(B.MPBP_OPT_GRAD_BATCH, v)
    assert plan.mpbp_get_option(B.MPBP_OPT_RUNS) == 1
    plan.mpbp_set_option(B.MPBP_OPT_RUNS, 0)
    assert plan.mpbp_get_option(B.MPBP_OPT_RUNS) == 0
    with pytest.raises(B.MPBPError):
        plan.mpbp_set_option(B.MPBP_OPT_RUNS, 2)
    assert plan.mpbp_tuning()["grad_tile"] == 16
    for v in (8, 16):
        plan.mpbp_set_option(B.MPBP_OPT_GRAD_TILE, v)
        assert plan.mpbp_get_option(B.MPBP_OPT_GRAD_TILE) == v
    with pytest.raises(B.MPBPError):
        plan.mpbp_set_option(B.MPBP_OPT_GRAD_TILE, 4)
    with pytest.raises(B.MPBPError) as e:     # autotuning needs a device plan
        z = np.zeros(1, np.float32)
        B._check(B.lib.mpbp_autotune(plan.handle, *(5 * [z.ctypes.data]), None))
    assert e.value.status == 4
    n = ctypes.c_int64()
    assert B.lib.mpbp_tuning(plan.handle, None, 0, ctypes.byref(n)) == 0 and n.value > 2
    small = ctypes.create_string_buffer(8)
    assert B.lib.mpbp_tuning(plan.handle, small, 8, ctypes.byref(n)) == 1
    assert len(small.value) == 7


def test_package_lazy_attributes():
    # the package resolves its submodules on first attribute access (regression: the
    # lookup once recursed into itself before the submodule was loaded)
    import importlib
    import paper_2312_14907_amd as P
    P = importlib.reload(P)
    assert P.Plan is B.Plan and P.binding is B and P.MPBPError is B.MPBPError


def test_unwrap_needs_a_device_plan():
    plan = B.Plan(make_problem(get_config("c1_tiny")), device=-1)
    with pytest.raises(B.MPBPError) as e:
        B._check(B.lib.mpbp_unwrap_project(plan.handle, None, None, None))
    assert e.value.status == 4


@pytest.mark.parametrize("name", ["c1_tiny", "c4_batch", "c5_full"])
def test_linear_offset_tables_against_oracle(name):
    # MPBP_SHEAR_LINEAR: the floors of the fractional offsets, bit-exact
    import dataclasses
    prob = dataclasses.replace(make_problem(get_config(name)), shear_linear=True)
    plan = B.Plan(prob, device=-1, flags=B.MPBP_SHEAR_LINEAR)
    scan, shear, y_off = plan.mpbp_tables()
    tab = O.tables(prob)
    np.testing.assert_array_equal(shear, tab["shear"])
    np.testing.assert_array_equal(scan, tab["scan"])
    assert (tab["shear_frac"] > 0).any()


def test_detector_map_window_check_matches_the_oracle():
    """MPBP_DETECTOR_MAP: the host's footprint check (the mapped support's bounding box,
    widened by one sample, inside the window) agrees with the oracle's on a sweep of maps
    near the window's edge; a singular map is an invalid descriptor."""
    import dataclasses
    from synth.inputs import detector_map
    rng = np.random.default_rng(301)
    base = _supported_problem(((0.3, 0.2), (0.1, -0.4)))
    agree = {True: 0, False: 0}
    for _ in range(60):
        maps = np.stack([detector_map(rng.uniform(0.5, 3.0), rng.uniform(-math.pi, math.pi)) for _ in range(2)])
        prob = dataclasses.replace(base, lateral_map=maps)
        try:
            O.tables(prob)
            fits = True
        except O.FootprintError:
            fits = False
        st, msg = _status_of(B.make_problem_struct(prob, B.MPBP_DETECTOR_MAP))
        assert st == (0 if fits else 3), (st, msg, maps)
        agree[fits] += 1
    assert agree[True] >= 5 and agree[False] >= 5
    prob = dataclasses.replace(base, lateral_map=np.stack([np.eye(2), [[1.0, 2.0], [0.5, 1.0]]]))
    assert _status_of(B.make_problem_struct(prob, B.MPBP_DETECTOR_MAP))[0] == 1


def test_detector_map_footprint_matches_the_oracle():
    """The footprint the host derives for each peak (origin and size, read from the trace)
    is the oracle's mapped extent."""
    import subprocess
    import sys
    snippet = """
import dataclasses, math
import numpy as np
from synth import get_config, make_problem
from synth.inputs import detector_map
from paper_2312_14907_amd.binding import Plan, MPBP_DETECTOR_MAP
base = make_problem(get_config("c2_forward"))
maps = np.stack([detector_map(r, a) for r, a in [(1.2, 0.4), (0.9, 2.5), (1.05, -0.7)]])
Plan(dataclasses.replace(base, lateral_map=maps), device=-1, flags=MPBP_DETECTOR_MAP).close()
"""
    env = dict(os.environ, MPBP_TRACE="1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([sys.executable, "-c", snippet], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    got = [tuple(int(v) for v in m.groups())
           for m in re.finditer(r"footprint (\d+)x(\d+) at \((\d+), (\d+)\)", r.stderr)]
    import dataclasses
    from synth.inputs import detector_map
    base = make_problem(get_config("c2_forward"))
    prob = dataclasses.replace(base, lateral_map=np.stack(
        [detector_map(a, b) for a, b in [(1.2, 0.4), (0.9, 2.5), (1.05, -0.7)]]))
    want = []
    for m in range(prob.n_peaks):
        lo, hi = O.mapped_extent(prob, m)
        want.append((int(hi[0] - lo[0] + 1), int(hi[1] - lo[1] + 1), int(lo[0]), int(lo[1])))
    assert got == want, r.stderr
    assert "detector-map" in r.stderr
