"""ctypes binding of libmpbp.so (include/mpbp.h).

Argument marshalling only: every computation runs in the library's HIP kernels.  Device
buffers are torch CUDA tensors (PyTorch provides device memory and streams); the
functions keep the C names.  A missing library raises at import: there is no fallback.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# MPBP_LIBRARY may name another build of the library (the bounds-checked libmpbp_debug.so)
LIB_PATH = os.environ.get("MPBP_LIBRARY") or os.path.join(_PKG, "libmpbp.so")

MPBP_OK = 0
STATUS_NAMES = {0: "MPBP_OK", 1: "MPBP_ERR_INVALID", 2: "MPBP_ERR_SHAPE", 3: "MPBP_ERR_FOOTPRINT",
                4: "MPBP_ERR_DEVICE", 5: "MPBP_ERR_NOMEM", 6: "MPBP_ERR_UNSUPPORTED", 7: "MPBP_ERR_INTERNAL"}
MPBP_OPT_PATH = 1
MPBP_OPT_GRAPH = 2
MPBP_OPT_XCD_ORDER = 3
MPBP_OPT_PROFILE = 4
MPBP_OPT_GRAD_BATCH = 5
MPBP_OPT_GRAD_TILE = 6
MPBP_OPT_RUNS = 7
MPBP_Z_TIED = 1
MPBP_PROBE_3D = 2
MPBP_SHEAR_LINEAR = 4
MPBP_DETECTOR_MAP = 8
STAGES = ("object", "frames", "grad", "finalize", "plain", "project")

EXPORTED = ("mpbp_plan_create", "mpbp_plan_destroy", "mpbp_num_frames", "mpbp_intensity_size",
            "mpbp_tables", "mpbp_forward", "mpbp_loss_grad", "mpbp_step", "mpbp_set_option",
            "mpbp_get_option", "mpbp_stage_times", "mpbp_autotune", "mpbp_set_variant", "mpbp_tuning",
            "mpbp_adam_step", "mpbp_norm2", "mpbp_set_background", "mpbp_unwrap_project",
            "mpbp_last_error", "mpbp_loss_grad_static")


class mpbp_peak(ctypes.Structure):
    _fields_ = [("g", ctypes.c_double * 3), ("shear", ctypes.c_double * 2), ("det", ctypes.c_int32),
                ("scan_n", ctypes.c_int32 * 2), ("scan_step", ctypes.c_int32 * 2),
                ("scan_origin", ctypes.c_int32 * 2), ("map", ctypes.c_double * 4)]


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
    lib.mpbp_loss_grad_static.argtypes = [vp, vp, vp, vp, vp, vp, i32p, i64, vp, vp, vp, vp, vp, vp]
    lib.mpbp_loss_grad_static.restype = st
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
    """Device address of a tensor, or None."""
    if t is None:
        return None
    return t.data_ptr()


_DTYPES = {"f32": ("float32", 4), "f64": ("float64", 8), "c64": ("complex64", 8)}


def _dev_bufs(device, *specs):
    """Validate the device buffers of one compute call and return their addresses.

    Each spec is (tensor, name, kind, numel[, flags]) with flags a string of "o"
    (optional: None allowed) and "+" (at least numel elements).  A buffer must be a
    contiguous torch tensor of dtype `kind` and `numel` elements, on the plan's GPU.
    The library reads and writes these addresses from its kernels and cannot check
    them itself.  Every buffer's type, dtype, layout and size are checked before any
    buffer's device, so the first error names the argument that is wrong."""
    import torch
    for t, name, kind, numel, *fl in specs:
        fl = fl[0] if fl else ""
        if t is None:
            if "o" in fl:
                continue
            raise ValueError(f"{name} is required")
        if not isinstance(t, torch.Tensor):
            raise ValueError(f"{name} must be a torch CUDA tensor (got {type(t).__name__})")
        dt, _ = _DTYPES[kind]
        if t.dtype != getattr(torch, dt):
            raise ValueError(f"{name} must be {dt} (got {t.dtype})")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        n = t.numel()
        if (n < numel) if "+" in fl else (n != numel):
            raise ValueError(f"{name} must hold {'at least ' if '+' in fl else ''}{numel} elements (got {n})")
    for t, name, *_ in specs:
        if t is not None and (not t.is_cuda or t.device.index != device):
            raise ValueError(f"{name} must be on cuda:{device} (got {t.device})")
    return tuple(None if t is None else t.data_ptr() for t, *_ in specs)


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
        lm = getattr(problem, "lateral_map", None)
        mk = np.eye(2) if lm is None else np.asarray(lm[k], dtype=np.float64)
        for c in range(4):
            pk.map[c] = float(mk.reshape(4)[c])
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
        # element counts of the device buffers
        self.field_size = (1 if self.flags & MPBP_Z_TIED else self.nz) * self.ny * self.nx
        self.probe_size = self.n_peaks * (self.nz if self.flags & MPBP_PROBE_3D else 1) * self.probe_n ** 2

    def _input_specs(self, u, chi, alpha, probe, y, y_required=True):
        return ((u, "u", "f32", 3 * self.field_size), (chi, "chi", "f32", self.field_size),
                (alpha, "alpha", "f32", self.n_peaks), (probe, "probe", "c64", self.probe_size),
                (y, "y", "f32", self.intensity_size, "" if y_required else "o"))

    def _grad_specs(self, grad_u, grad_chi, grad_alpha, flags=""):
        return ((grad_u, "grad_u", "f32", 3 * self.field_size, flags),
                (grad_chi, "grad_chi", "f32", self.field_size, flags),
                (grad_alpha, "grad_alpha", "f32", self.n_peaks, flags))

    @staticmethod
    def _output_specs(n, loss, frame_loss):
        return ((loss, "loss", "f64", 1, "o"), (frame_loss, "frame_loss", "f32", max(n, 1), "o+"))

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
        n_out = self.n_frames if frames is None else n
        pu, pc, pa, pp, py, pl, pf, pm = _dev_bufs(
            self.device, *self._input_specs(u, chi, alpha, probe, y, loss is not None or frame_loss is not None),
            *self._output_specs(n_out, loss, frame_loss),
            (model_intensity, "model_intensity", "f32", self.intensity_size, "o"))
        _check(lib.mpbp_forward(self.handle, pu, pc, pa, pp, py, fp, n, pl, pf, pm, _stream(stream)))
        del keep

    def mpbp_loss_grad(self, u, chi, alpha, probe, y, grad_u, grad_chi, grad_alpha, frames=None,
                       loss=None, frame_loss=None, stream=None):
        fp, n, keep = self._frames(frames)
        n_out = self.n_frames if frames is None else n
        pu, pc, pa, pp, py, pl, pf, gu, gc, ga = _dev_bufs(
            self.device, *self._input_specs(u, chi, alpha, probe, y), *self._output_specs(n_out, loss, frame_loss),
            *self._grad_specs(grad_u, grad_chi, grad_alpha))
        _check(lib.mpbp_loss_grad(self.handle, pu, pc, pa, pp, py, fp, n, pl, pf, gu, gc, ga, _stream(stream)))
        del keep

    def mpbp_loss_grad_static(self, u, chi, alpha, probe, y, grad_u, grad_chi, grad_alpha, frames=None,
                              loss=None, frame_loss=None, stream=None):
        """mpbp_loss_grad with the library's fixed device workspace (allocates nothing)."""
        fp, n, keep = self._frames(frames)
        n_out = self.n_frames if frames is None else n
        pu, pc, pa, pp, py, pl, pf, gu, gc, ga = _dev_bufs(
            self.device, *self._input_specs(u, chi, alpha, probe, y), *self._output_specs(n_out, loss, frame_loss),
            *self._grad_specs(grad_u, grad_chi, grad_alpha))
        _check(lib.mpbp_loss_grad_static(self.handle, pu, pc, pa, pp, py, fp, n, pl, pf, gu, gc, ga,
                                         _stream(stream)))
        del keep

    def mpbp_step(self, u, chi, alpha, grad_u, grad_chi, grad_alpha, eta, stream=None):
        e = (ctypes.c_float * 3)(*[float(v) for v in eta])
        pu, pc, pa, gu, gc, ga = _dev_bufs(
            self.device, (u, "u", "f32", 3 * self.field_size), (chi, "chi", "f32", self.field_size),
            (alpha, "alpha", "f32", self.n_peaks), *self._grad_specs(grad_u, grad_chi, grad_alpha))
        _check(lib.mpbp_step(self.handle, pu, pc, pa, gu, gc, ga, e, _stream(stream)))

    def mpbp_adam_step(self, cfg, t, u, chi, alpha, chi_log, alpha_log, state, grad_u, grad_chi, grad_alpha,
                       stream=None):
        """cfg: dict with lr (3), beta1, beta2, eps, log_params, fixed_alpha."""
        c = mpbp_adam((ctypes.c_float * 3)(*[float(v) for v in cfg["lr"]]), float(cfg.get("beta1", 0.9)),
                      float(cfg.get("beta2", 0.999)), float(cfg.get("eps", 1e-8)), int(cfg.get("log_params", 1)),
                      int(cfg.get("fixed_alpha", -1)))
        nf, lf = self.field_size, "" if c.log_params else "o"
        pu, pc, pa, pcl, pal, ps, gu, gc, ga = _dev_bufs(
            self.device, (u, "u", "f32", 3 * nf), (chi, "chi", "f32", nf), (alpha, "alpha", "f32", self.n_peaks),
            (chi_log, "chi_log", "f32", nf, lf), (alpha_log, "alpha_log", "f32", self.n_peaks, lf),
            (state, "state", "f32", 2 * (4 * nf + self.n_peaks)),
            *self._grad_specs(grad_u, grad_chi, grad_alpha, "o" if int(t) == 0 else ""))
        _check(lib.mpbp_adam_step(self.handle, ctypes.byref(c), int(t), pu, pc, pa, pcl, pal, ps, gu, gc, ga,
                                  _stream(stream)))

    def mpbp_norm2(self, a, out, n=None, stream=None):
        n = int(a.numel() if n is None else n)
        pa, po = _dev_bufs(self.device, (a, "a", "f32", n, "+"), (out, "out", "f64", 1))
        _check(lib.mpbp_norm2(self.handle, pa, n, po, _stream(stream)))

    def mpbp_set_background(self, b):
        """Background b of eq. (2) (device float, ragged like y) for later calls; None clears
        it.  The plan keeps a reference to the tensor while it is set."""
        (pb,) = _dev_bufs(self.device, (b, "b", "f32", self.intensity_size, "o"))
        _check(lib.mpbp_set_background(self.handle, pb))
        self._background = b

    def mpbp_unwrap_project(self, u, wraps=None, stream=None):
        """Pi_U of eq. (10) in place on u (float32, the layout of mpbp_loss_grad); wraps:
        optional int32 [n_peaks][nz or 1][ny][nx] receiving the 2 pi multiples added."""
        import torch
        lat = self.field_size
        (pu,) = _dev_bufs(self.device, (u, "u", "f32", 3 * lat))
        if wraps is not None and (not isinstance(wraps, torch.Tensor) or wraps.dtype != torch.int32
                                  or not wraps.is_cuda or wraps.device.index != self.device
                                  or wraps.numel() != self.n_peaks * lat or not wraps.is_contiguous()):
            raise ValueError(f"wraps must be a contiguous int32 tensor of {self.n_peaks * lat} elements "
                             f"on cuda:{self.device}")
        _check(lib.mpbp_unwrap_project(self.handle, pu, _ptr(wraps), _stream(stream)))

    def mpbp_set_option(self, option, value):
        _check(lib.mpbp_set_option(self.handle, int(option), int(value)))

    def mpbp_stage_times(self):
        """{stage: (total_ms, launches)} accumulated since the previous call."""
        ms = np.zeros(len(STAGES), dtype=np.float64)
        n = np.zeros(len(STAGES), dtype=np.int64)
        _check(lib.mpbp_stage_times(self.handle, ms.ctypes.data, n.ctypes.data))
        return {name: (float(ms[i]), int(n[i])) for i, name in enumerate(STAGES)}

    def mpbp_autotune(self, u, chi, alpha, probe, y, stream=None):
        pu, pc, pa, pp, py = _dev_bufs(self.device, *self._input_specs(u, chi, alpha, probe, y))
        _check(lib.mpbp_autotune(self.handle, pu, pc, pa, pp, py, _stream(stream)))

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
