"""Mutation check of the oracle's pins (CPU): each entry below plants one plausible mistake
in a copy of `oracle/` (a dropped term, a wrong sign, index or operand, a wrong constant
or rounding) and runs the pin tests that should notice it against the copy.  Every
planted mistake must make those pins fail, and the unmodified copy must pass them.

The copies live in a temporary folder (oracle/, synth/, tests/ and pytest.ini); the
repository's own files are never changed.  Each mutant runs in a child process, several
at a time.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PINS = "tests/test_oracle_pins.py"
MAP = "tests/test_oracle_map_pins.py"
OPT = "tests/test_optim_pins.py"
UW = "tests/test_unwrap_oracle_pins.py"
ORA = "oracle/mpbp_oracle.py"
UWO = "oracle/unwrap_oracle.py"

# (name, file, text, replacement, pin files).  The text must occur in the file; its first
# occurrence is replaced.
MUTANTS = [
    # integer tables (section 2: S and R)
    ("halves rounded toward zero", ORA, "r = f + (1 if (a - f) >= 0.5 else 0)", "r = f + (1 if (a - f) > 0.5 else 0)",
     [PINS]),
    ("shear from slice 0", ORA, "    zref = nz // 2\n    out = np.zeros((nz, 2), dtype=np.int64)",
     "    zref = 0\n    out = np.zeros((nz, 2), dtype=np.int64)", [PINS]),
    ("shear axes swapped", ORA, "out[z, 0] = round_half_away(dz * float(shear[0]))",
     "out[z, 0] = round_half_away(dz * float(shear[1]))", [PINS]),
    ("raster step axes swapped", ORA, "int(scan_origin[0]) + iy * int(scan_step[0])",
     "int(scan_origin[0]) + iy * int(scan_step[1])", [PINS]),
    ("interpolated offsets rounded up", ORA, "            s0[z, a] = math.floor(v)",
     "            s0[z, a] = math.ceil(v)", [PINS]),
    # object, eq. (1) / (3)
    ("phase sign", ORA, "out[m] = float(alpha[m]) * chi * np.exp(1j * phases(u, problem.g[m]))",
     "out[m] = float(alpha[m]) * chi * np.exp(-1j * phases(u, problem.g[m]))", [PINS]),
    ("alpha dropped from the object", ORA, "out[m] = float(alpha[m]) * chi * np.exp(",
     "out[m] = chi * np.exp(", [PINS]),
    ("phase reads u_y for u_z", ORA, "g[0] * u[0] + g[1] * u[1] + g[2] * u[2]", "g[0] * u[0] + g[1] * u[1] + g[2] * u[1]",
     [PINS]),
    # projection and back-projection, eq. (2)
    ("support clipped one row late", ORA, "    a1 = min(n, size - p0)\n", "    a1 = min(n, size - p0 + 1)\n", [PINS]),
    ("shear applied with the wrong sign", ORA,
     "sy, sx = int(shear_m[z, 0]) + dy, int(shear_m[z, 1]) + dx\n            psi[",
     "sy, sx = -int(shear_m[z, 0]) + dy, int(shear_m[z, 1]) + dx\n            psi[", [PINS]),
    ("back-projection without conj(P)", ORA, "pc = np.conj(_probe_slice(probe_m, z)[a0:a1, b0:b1])",
     "pc = _probe_slice(probe_m, z)[a0:a1, b0:b1]", [PINS]),
    ("back-projection taps transposed", ORA,
     "sy, sx = int(shear_m[z, 0]) + dy, int(shear_m[z, 1]) + dx\n            g_o_m",
     "sy, sx = int(shear_m[z, 0]) + dx, int(shear_m[z, 1]) + dy\n            g_o_m", [PINS]),
    ("bilinear weights swapped", ORA, "(0, 1, (1 - fy) * fx), (1, 0, fy * (1 - fx))",
     "(0, 1, fy * (1 - fx)), (1, 0, (1 - fy) * fx)", [PINS]),
    ("3D probe slice ignored", ORA, "return probe_m[z] if probe_m.ndim == 3 else probe_m",
     "return probe_m[0] if probe_m.ndim == 3 else probe_m", [PINS]),
    # far field and residual, eq. (2) / (4)
    ("unnormalised transform", ORA, 'return np.fft.fft2(psi, norm="ortho")', "return np.fft.fft2(psi)", [PINS]),
    ("adjoint is the forward transform", ORA, 'return np.fft.ifft2(g, norm="ortho")',
     'return np.fft.fft2(g, norm="ortho")', [PINS]),
    ("loss without the half", ORA, "f = 0.5 * float(np.sum(r * r))", "f = float(np.sum(r * r))", [PINS]),
    ("residual on intensities", ORA, "r = a - np.sqrt(np.asarray(y, dtype=np.float64))",
     "r = a * a - np.asarray(y, dtype=np.float64)", [PINS]),
    ("residual direction not normalised", ORA, "grad = np.where(a > 0.0, r * psi_ff / safe, 0.0)",
     "grad = np.where(a > 0.0, r * psi_ff, 0.0)", [PINS]),
    ("background added to the amplitude", ORA,
     "a = np.sqrt(np.abs(psi_ff) ** 2 + np.asarray(b, dtype=np.float64))",
     "a = np.abs(psi_ff) + np.asarray(b, dtype=np.float64)", [PINS]),
    # chain rule
    ("phase gradient sign", ORA, "dphi = np.imag(g_obj[m] * np.conj(obj[m]))",
     "dphi = np.imag(np.conj(g_obj[m]) * obj[m])", [PINS]),
    ("chi gradient without alpha", ORA, "grad_chi += np.real(np.conj(g_obj[m]) * float(alpha[m]) * e)",
     "grad_chi += np.real(np.conj(g_obj[m]) * e)", [PINS]),
    ("alpha gradient without chi", ORA, "grad_alpha[m] = float(np.sum(np.real(np.conj(g_obj[m]) * chi * e)))",
     "grad_alpha[m] = float(np.sum(np.real(np.conj(g_obj[m]) * e)))", [PINS]),
    ("u gradient from the wrong G component", ORA, "grad_u[c] += problem.g[m][c] * dphi",
     "grad_u[c] += problem.g[m][2 - c] * dphi", [PINS]),
    ("tied gradient not summed over z", ORA, 'r["grad_u"] = r["grad_u"].sum(axis=1, keepdims=True)',
     'r["grad_u"] = r["grad_u"][:, :1]', [PINS]),
    # R with a detector-frame map (section 2)
    ("transposed inverse map", ORA, "py = minv[0, 0] * ry + minv[0, 1] * rx + n / 2.0",
     "py = minv[0, 0] * ry + minv[1, 0] * rx + n / 2.0", [MAP]),
    ("no half-support shift", ORA, "px = minv[1, 0] * ry + minv[1, 1] * rx + n / 2.0",
     "px = minv[1, 0] * ry + minv[1, 1] * rx", [MAP]),
    ("mapped tap weights swapped", ORA,
     "w = np.stack([(1 - fy) * (1 - fx), (1 - fy) * fx, fy * (1 - fx), fy * fx])",
     "w = np.stack([(1 - fy) * (1 - fx), fy * (1 - fx), (1 - fy) * fx, fy * fx])", [MAP]),
    ("mapped offset sign", ORA, "ry, rx = qy - centre - offs[z, 0], qx - centre - offs[z, 1]",
     "ry, rx = qy - centre + offs[z, 0], qx - centre - offs[z, 1]", [MAP]),
    ("mapped adjoint without conj(P)", ORA,
     "np.conj(_probe_slice(probe_m, z)[a0:a1, b0:b1]) * acc[a0:a1, b0:b1])",
     "(_probe_slice(probe_m, z)[a0:a1, b0:b1]) * acc[a0:a1, b0:b1])", [MAP]),
    ("mapped centre off by half a pixel", ORA, "centre = window_offset(int(problem.det[m]), n) + n / 2.0",
     "centre = window_offset(int(problem.det[m]), n) + (n - 1) / 2.0", [MAP]),
    # optimiser (Algorithm 1, eq. (8))
    ("Adam without bias correction", ORA, "mhat = m / (1.0 - beta1 ** t)", "mhat = m", [PINS, OPT]),
    ("Adam epsilon inside the root", ORA, "return p - lr * mhat / (np.sqrt(vhat) + eps), m, v",
     "return p - lr * mhat / np.sqrt(vhat + eps), m, v", [PINS, OPT]),
    ("log-variable gradient divides", ORA,
     "return np.asarray(x, dtype=np.float64) * np.asarray(grad_x, dtype=np.float64)",
     "return np.asarray(grad_x, dtype=np.float64) / np.asarray(x, dtype=np.float64)", [PINS, OPT]),
    ("short last minibatch kept", ORA, "per_pass = n_frames // batch", "per_pass = -(-n_frames // batch)",
     [OPT]),
    ("no reshuffle between passes", ORA, "perm = order[(e % shuffles) * n_frames:(e % shuffles + 1) * n_frames]",
     "perm = order[:n_frames]", [OPT]),
    ("Armijo test without sufficient decrease", ORA, "if f1 <= f0 - c * eta * n2:", "if f1 < f0:", [OPT]),
    ("line search does not grow the step", ORA, "if eta is None else eta * grow", "if eta is None else eta",
     [OPT]),
    ("first step not scaled by the RMS", ORA, "eta = step0 / math.sqrt(n2 / g.size)", "eta = step0 / math.sqrt(n2)",
     [OPT]),
    # unwrap projector (eqs. (9)-(10))
    ("wrap to [0, 2 pi)", UWO, "qf = np.rint(phi / TWO_PI_32).astype(np.float32)",
     "qf = np.floor(phi / TWO_PI_32).astype(np.float32)", [UW]),
    ("second difference with a plus", UWO,
     "return (gamma((a - c).astype(np.float32)) - gamma((c - b).astype(np.float32))).astype(np.float32)",
     "return (gamma((a - c).astype(np.float32)) + gamma((c - b).astype(np.float32))).astype(np.float32)", [UW]),
    ("one diagonal dropped", UWO, "+ D1 * D1).astype(np.float32) + D2 * D2)", "+ D1 * D1).astype(np.float32) + D1 * D1)",
     [UW]),
    ("edge key is a product", UWO, "return (r[p] + r[q]).astype(np.float32)", "return (r[p] * r[q]).astype(np.float32)",
     [UW]),
    ("least reliable edges first", UWO, "return np.lexsort((tie, -keys.astype(np.float64)))",
     "return np.lexsort((tie, keys.astype(np.float64)))", [UW]),
    ("edge wrap count sign", UWO, "k = n[a] - w - n[b]", "k = n[a] + w - n[b]", [UW]),
    ("global offset truncated", UWO, "return (2 * s + cnt) // (2 * cnt)", "return s // cnt", [UW]),
    ("projector uses H instead of its pseudo-inverse", UWO, "A = H.T @ np.linalg.inv(HHt)               # M x 3",
     "A = H.T                                      # M x 3", [UW]),
]


def _copy_tree(dst):
    for d in ("oracle", "synth", "tests"):
        shutil.copytree(os.path.join(ROOT, d), os.path.join(dst, d),
                        ignore=shutil.ignore_patterns("__pycache__", "host_sanitize", "test_gpu_*", "*.so"))
    shutil.copy(os.path.join(ROOT, "pytest.ini"), dst)


def _run_pins(dst, pins):
    env = {k: v for k, v in os.environ.items() if k != "PYTHONPATH"}
    env["OMP_NUM_THREADS"] = "1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        *pins], cwd=dst, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, (r.stdout + r.stderr).strip().splitlines()[-1:] or [""]


def _mutant(tmp, k, entry):
    name, path, old, new, pins = entry
    dst = os.path.join(tmp, f"m{k:02d}")
    _copy_tree(dst)
    f = os.path.join(dst, path)
    text = open(f).read()
    if old not in text:
        return name, None, "text not found"
    with open(f, "w") as fh:
        fh.write(text.replace(old, new, 1))
    rc, tail = _run_pins(dst, pins)
    shutil.rmtree(dst, ignore_errors=True)
    return name, rc, tail[0]


def test_every_planted_mistake_fails_a_pin(tmp_path):
    base = os.path.join(str(tmp_path), "base")
    _copy_tree(base)
    rc, tail = _run_pins(base, sorted({p for e in MUTANTS for p in e[4]}))
    assert rc == 0, f"the unmodified oracle fails its pins: {tail}"
    workers = max(1, min(8, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        results = list(ex.map(lambda ke: _mutant(str(tmp_path), *ke), enumerate(MUTANTS)))
    missing = [n for n, rc, why in results if rc is None]
    assert not missing, f"planted text no longer in the oracle: {missing}"
    survived = [(n, why) for n, rc, why in results if rc == 0]
    assert not survived, f"mistakes no pin noticed: {survived}"
    # a pin run that could not start (collection error) is not a pin failing
    broken = [(n, why) for n, rc, why in results if rc not in (0, 1)]
    assert not broken, f"pin runs that did not complete: {broken}"
