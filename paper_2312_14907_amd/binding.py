"""ctypes binding of libmpbp.so (include/mpbp.h).

Argument marshalling only: every computation runs in the library's HIP kernels.  Device
buffers are torch CUDA tensors (PyTorch provides device memory and streams); the
functions keep the C names.  A missing library raises at import: there is no fallback.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmpbp.so")

MPBP_OK = 0
STATUS_NAMES = {0: "MPBP_OK", 1: "MPBP_ERR_INVALID", 2: "MPBP_ERR_SHAPE", 3: "MPBP_ERR_FOOTPRINT",
                4: "MPBP_ERR_DEVICE", 5: "MPBP_ERR_NOMEM", 6: "MPBP_ERR_UNSUPPORTED", 7: "MPBP_ERR_INTERNAL"}
MPBP_OPT_PATH = 1
MPBP_OPT_GRAPH = 2
MPBP_OPT_XCD_ORDER = 3
MPBP_OPT_PROFILE = 4
MPBP_OPT_GRAD_BATCH = 5
MPBP_OPT_GRAD_TILE = 6
MPBP_Z_TIED = 1
MPBP_PROBE_3D = 2
MPBP_SHEAR_LINEAR = 4
STAGES = ("object", "frames", "grad", "finalize", "plain", "project")

EXPORTED = ("mpbp_plan_create", "mpbp_plan_destroy", "mpbp_num_frames", "mpbp_intensity_size",
            "mpbp_tables", "mpbp_forward", "mpbp_loss_grad", "mpbp_step", "mpbp_set_option",
            "mpbp_get_option", "mpbp_stage_times", "mpbp_autotune", "mpbp_set_variant", "mpbp_tuning",
            "mpbp_adam_step", "mpbp_norm2", "mpbp_set_background", "mpbp_unwrap_project",
            "mpbp_last_error")


class mpbp_peak(ctypes.Structure):
    _fields_ = [("g", ctypes.c_double * 3), ("shear", ctypes.c_double * 2), ("det", ctypes.c_int32),
                ("scan_n", ctypes.c_int32 * 2), ("scan_step", ctypes.c_int32 * 2),
                ("scan_origin", ctypes.c_int32 * 2)]


class mpbp_adam(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float * 3), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("log_params", ctypes.c_int32), ("fixed_alpha", ctypes.c_int32)]


class mpbp_problem(ctypes.Structure):
    _fields_ = [("nz", ctypes.c_int32), ("ny", ctypes.c_int32), ("nx", ctypes.c_int32),
                ("probe_n", ctypes.c_int32), ("n_peaks", ctypes.c_int32),
                ("peaks", ctypes.POINTER(mpbp_peak)), ("flags", ctypes.c_uint32)]


class MPBPError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2312_14907_amd.build`")
    # torch first: its HIP runtime is then the one the library binds to.  Loaded the other
    # way round, the process holds the system runtime and torch's build of it side by
    # side, and neither sees the GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32p, st = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), ctypes.c_int
    lib.mpbp_plan_create.argtypes = [ctypes.POINTER(mpbp_problem), ctypes.c_int, ctypes.POINTER(vp)]
    lib.mpbp_plan_create.restype = st
    lib.mpbp_plan_destroy.argtypes = [vp]
    lib.mpbp_plan_destroy.restype = None
    lib.mpbp_num_frames.argtypes = [vp]
    lib.mpbp_num_frames.restype = i64
    lib.mpbp_intensity_size.argtypes = [vp]
    lib.mpbp_intensity_size.restype = i64
    lib.mpbp_tables.argtypes = [vp, vp, vp, vp]
    lib.mpbp_tables.restype = st
    lib.mpbp_forward.argtypes = [vp, vp, vp, vp, vp, vp, i32p, i64, vp, vp, vp, vp]
    lib.mpbp_forward.restype = st
    lib.mpbp_loss_grad.argtypes = [vp, vp, vp, vp, vp, vp, i32p, i64, vp, vp, vp, vp, vp, vp]
    lib.mpbp_loss_grad.restype = st
    lib.mpbp_step.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(ctypes.c_float), vp]
    lib.mpbp_step.restype = st
    lib.mpbp_set_option.argtypes = [vp, ctypes.c_int, i64]
    lib.mpbp_set_option.restype = st
    lib.mpbp_get_option.argtypes = [vp, ctypes.c_int, ctypes.POINTER(i64)]
    lib.mpbp_get_option.restype = st
    lib.mpbp_stage_times.argtypes = [vp, vp, vp]
    lib.mpbp_stage_times.restype = st
    lib.mpbp_autotune.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    lib.mpbp_autotune.restype = st
    lib.mpbp_set_variant.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.mpbp_set_variant.restype = st
    lib.mpbp_tuning.argtypes = [vp, ctypes.c_char_p, i64, ctypes.POINTER(i64)]
    lib.mpbp_tuning.restype = st
    lib.mpbp_adam_step.argtypes = [vp, ctypes.POINTER(mpbp_adam), i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.mpbp_adam_step.restype = st
    lib.mpbp_norm2.argtypes = [vp, vp, i64, vp, vp]
    lib.mpbp_norm2.restype = st
    lib.mpbp_set_background.argtypes = [vp, vp]
    lib.mpbp_set_background.restype = st
    lib.mpbp_unwrap_project.argtypes = [vp, vp, vp, vp]
    lib.mpbp_unwrap_project.restype = st
    lib.mpbp_last_error.argtypes = []
    lib.mpbp_last_error.restype = ctypes.c_char_p
    return lib


lib = _load()


def mpbp_last_error():
    return lib.mpbp_last_error().decode()


def _check(status):
    if status != MPBP_OK:
        raise MPBPError(status, mpbp_last_error())


def _ptr(t):
    """Device (or host) address of a tensor / array, or None."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def make_problem_struct(problem, flags=0):
    """mpbp_problem for a geometry object with attributes nz, ny, nx, probe_n, g, shear,
    det, scan_n, scan_step, scan_origin (as built by synth.make_problem)."""
    m = int(np.asarray(problem.g).shape[0])
    peaks = (mpbp_peak * m)()
    for k in range(m):
        pk = peaks[k]
        for c in range(3):
            pk.g[c] = float(problem.g[k][c])
        for c in range(2):
            pk.shear[c] = float(problem.shear[k][c])
            pk.scan_n[c] = int(problem.scan_n[k][c])
            pk.scan_step[c] = int(problem.scan_step[k][c])
            pk.scan_origin[c] = int(problem.scan_origin[k][c])
        pk.det = int(problem.det[k])
    prob = mpbp_problem(int(problem.nz), int(problem.ny), int(problem.nx), int(problem.probe_n), m,
                        ctypes.cast(peaks, ctypes.POINTER(mpbp_peak)), int(flags))
    prob._peaks_keepalive = peaks
    return prob


class Plan:
    """A library plan (mpbp_plan) for one workload geometry on one device (-1: host only);
    flags = MPBP_Z_TIED for fields given per lateral pixel."""

    def __init__(self, problem, device=0, flags=0):
        self._struct = make_problem_struct(problem, flags)
        self.flags = int(flags)
        h = ctypes.c_void_p()
        _check(lib.mpbp_plan_create(ctypes.byref(self._struct), int(device), ctypes.byref(h)))
        self.handle = h
        self.device = device
        self.nz, self.ny, self.nx = int(problem.nz), int(problem.ny), int(problem.nx)
        self.probe_n = int(problem.probe_n)
        self.n_peaks = int(np.asarray(problem.g).shape[0])
        self.n_frames = int(lib.mpbp_num_frames(h))
        self.intensity_size = int(lib.mpbp_intensity_size(h))

    def close(self):
        if getattr(self, "handle", None):
            lib.mpbp_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def mpbp_tables(self):
        scan = np.zeros((self.n_frames, 2), dtype=np.int32)
        shear = np.zeros((self.n_peaks, self.nz, 2), dtype=np.int32)
        y_off = np.zeros(self.n_peaks + 1, dtype=np.int64)
        _check(lib.mpbp_tables(self.handle, scan.ctypes.data, shear.ctypes.data, y_off.ctypes.data))
        return scan, shear, y_off

    @staticmethod
    def _frames(frames):
        if frames is None:
            return None, 0, None
        arr = np.ascontiguousarray(np.asarray(frames, dtype=np.int32))
        return arr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), int(arr.size), arr

    def mpbp_forward(self, u, chi, alpha, probe, y=None, frames=None, loss=None, frame_loss=None,
                     model_intensity=None, stream=None):
        fp, n, keep = self._frames(frames)
        _check(lib.mpbp_forward(self.handle, _ptr(u), _ptr(chi), _ptr(alpha), _ptr(probe), _ptr(y),
                                fp, n, _ptr(loss), _ptr(frame_loss), _ptr(model_intensity),
                                _stream(stream)))
        del keep

    def mpbp_loss_grad(self, u, chi, alpha, probe, y, grad_u, grad_chi, grad_alpha, frames=None,
                       loss=None, frame_loss=None, stream=None):
        fp, n, keep = self._frames(frames)
        _check(lib.mpbp_loss_grad(self.handle, _ptr(u), _ptr(chi), _ptr(alpha), _ptr(probe), _ptr(y),
                                  fp, n, _ptr(loss), _ptr(frame_loss), _ptr(grad_u), _ptr(grad_chi),
                                  _ptr(grad_alpha), _stream(stream)))
        del keep

    def mpbp_step(self, u, chi, alpha, grad_u, grad_chi, grad_alpha, eta, stream=None):
        e = (ctypes.c_float * 3)(*[float(v) for v in eta])
        _check(lib.mpbp_step(self.handle, _ptr(u), _ptr(chi), _ptr(alpha), _ptr(grad_u),
                             _ptr(grad_chi), _ptr(grad_alpha), e, _stream(stream)))

    def mpbp_adam_step(self, cfg, t, u, chi, alpha, chi_log, alpha_log, state, grad_u, grad_chi, grad_alpha,
                       stream=None):
        """cfg: dict with lr (3), beta1, beta2, eps, log_params, fixed_alpha."""
        c = mpbp_adam((ctypes.c_float * 3)(*[float(v) for v in cfg["lr"]]), float(cfg.get("beta1", 0.9)),
                      float(cfg.get("beta2", 0.999)), float(cfg.get("eps", 1e-8)), int(cfg.get("log_params", 1)),
                      int(cfg.get("fixed_alpha", -1)))
        _check(lib.mpbp_adam_step(self.handle, ctypes.byref(c), int(t), _ptr(u), _ptr(chi), _ptr(alpha),
                                  _ptr(chi_log), _ptr(alpha_log), _ptr(state), _ptr(grad_u), _ptr(grad_chi),
                                  _ptr(grad_alpha), _stream(stream)))

    def mpbp_norm2(self, a, out, n=None, stream=None):
        _check(lib.mpbp_norm2(self.handle, _ptr(a), int(a.numel() if n is None else n), _ptr(out), _stream(stream)))

    def mpbp_set_background(self, b):
        """Background b of eq. (2) (device float, ragged like y) for later calls; None clears
        it.  The plan keeps a reference to the tensor while it is set."""
        if b is not None and (b.numel() != self.intensity_size or b.element_size() != 4 or not b.is_contiguous()):
            raise ValueError(f"b must be a contiguous float32 tensor of {self.intensity_size} elements")
        _check(lib.mpbp_set_background(self.handle, _ptr(b)))
        self._background = b

    def mpbp_unwrap_project(self, u, wraps=None, stream=None):
        """Pi_U of eq. (10) in place on u (float32, the layout of mpbp_loss_grad); wraps:
        optional int32 [n_peaks][nz or 1][ny][nx] receiving the 2 pi multiples added."""
        lat = (1 if self.flags & MPBP_Z_TIED else self.nz) * self.ny * self.nx
        if u.numel() != 3 * lat or u.element_size() != 4 or not u.is_contiguous():
            raise ValueError(f"u must be a contiguous float32 tensor of {3 * lat} elements")
        if wraps is not None and (wraps.numel() != self.n_peaks * lat or wraps.element_size() != 4
                                  or not wraps.is_contiguous()):
            raise ValueError(f"wraps must be a contiguous int32 tensor of {self.n_peaks * lat} elements")
        _check(lib.mpbp_unwrap_project(self.handle, _ptr(u), _ptr(wraps), _stream(stream)))

    def mpbp_set_option(self, option, value):
        _check(lib.mpbp_set_option(self.handle, int(option), int(value)))

    def mpbp_stage_times(self):
        """{stage: (total_ms, launches)} accumulated since the previous call."""
        ms = np.zeros(len(STAGES), dtype=np.float64)
        n = np.zeros(len(STAGES), dtype=np.int64)
        _check(lib.mpbp_stage_times(self.handle, ms.ctypes.data, n.ctypes.data))
        return {name: (float(ms[i]), int(n[i])) for i, name in enumerate(STAGES)}

    def mpbp_autotune(self, u, chi, alpha, probe, y, stream=None):
        _check(lib.mpbp_autotune(self.handle, _ptr(u), _ptr(chi), _ptr(alpha), _ptr(probe), _ptr(y),
                                 _stream(stream)))

    def mpbp_set_variant(self, size_class, footprint_bound, slab, xcd_order):
        _check(lib.mpbp_set_variant(self.handle, int(size_class), int(footprint_bound), int(slab),
                                    int(xcd_order)))

    def mpbp_tuning(self):
        """The plan's launch parameters (dict, from the library's JSON text)."""
        import json
        n = ctypes.c_int64()
        _check(lib.mpbp_tuning(self.handle, None, 0, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(int(n.value))
        _check(lib.mpbp_tuning(self.handle, buf, int(n.value), ctypes.byref(n)))
        return json.loads(buf.value.decode())

    def mpbp_get_option(self, option):
        v = ctypes.c_int64()
        _check(lib.mpbp_get_option(self.handle, int(option), ctypes.byref(v)))
        return int(v.value)
