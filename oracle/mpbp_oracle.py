"""Plain FP64 CPU oracle of the multi-peak Bragg ptychography objective and gradient.

TEST INFRASTRUCTURE.  This module is the slow, obviously correct reference that the GPU
library is checked against.  Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.  It shares no
code with the GPU library: it computes its own index tables, in numpy float64 /
complex128, with plain loops over peaks, frames and z-slices.

What it computes (Kandel et al., "Imaging extended single crystal lattice distortion
fields with multi-peak Bragg ptychography"):

* eq. (1) and eq. (3): the per-peak object O_m = alpha_m * chi * exp(i G_m . u), with
  G_m in rad/nm (the paper's 2*pi folded into G) and alpha given for every peak;
* eq. (2): intensity I_{m,j} = |F R_m diag(P_m) S_{m,j} O_m|^2 + b_{m,j}; P_m is the probe,
  [M][Np][Np] constant along x3 or a 3D illumination volume [M][nz][Np][Np]; the background
  b given per frame and detector pixel in the layout of y (None: b = 0).
  S_{m,j} selects the probe window of scan position j (section 4: raster scan), the
  probe is constant along the incident beam x3 (section 4), and R_m projects the
  illuminated slices along the exit beam: slice z lands s_m(z) pixels over, an integer
  lateral shear, inside a D_m x D_m window centred on the probe support (with
  problem.shear_linear the offset stays fractional and the slice is spread over the four
  neighbouring integer offsets with bilinear weights: R interpolating, section 2; with
  problem.lateral_map, R rotates and scales each slice into the peak's detector frame and
  interpolates it bilinearly onto the exit-wave pixels, see exit_wave_mapped).  F is the
  orthonormal 2D DFT with kernel exp(-2 pi i k.x / D), DC at index 0;
* eq. (4): f = 1/2 sum_{m,j} || I^{1/2} - y^{1/2} ||^2, summed (not averaged) over the
  listed frames as in the minibatch sums of eq. (11);
* the gradient of f with respect to u (3 components), chi and alpha: the exact adjoint of
  the chain above (the paper obtains it by automatic differentiation).

Complex gradients use the convention g = df/dRe + i df/dIm.
"""
import math

import numpy as np


# ---------------------------------------------------------------------------------
# Index tables (the shift operator S and the exit-beam projection R of eq. (2)).
# ---------------------------------------------------------------------------------

def round_half_away(v):
    """Round a double to the nearest integer, halves away from zero.

    Written with floor and an exact fractional part so that 0.49999999999999994 rounds
    to 0 (floor(v + 0.5) would give 1).
    """
    a = abs(float(v))
    f = math.floor(a)
    r = f + (1 if (a - f) >= 0.5 else 0)
    return int(-r if v < 0 else r)


def window_offset(det, probe_n):
    """Top-left of the probe support inside the D x D exit-wave window (centred)."""
    return (det - probe_n) // 2


def shear_table(nz, shear):
    """s_m(z) = (rha((z - nz//2) * t_y), rha((z - nz//2) * t_x)) for z = 0..nz-1."""
    zref = nz // 2
    out = np.zeros((nz, 2), dtype=np.int64)
    for z in range(nz):
        dz = float(z - zref)
        out[z, 0] = round_half_away(dz * float(shear[0]))
        out[z, 1] = round_half_away(dz * float(shear[1]))
    return out


def shear_table_linear(nz, shear):
    """Interpolated exit-beam offsets: s(z) = (z - nz//2) * t per axis, split into
    s0 = floor(s) and the fraction f = s - s0 in [0, 1).  A slice's illuminated object
    then lands on offsets s0 (weight 1 - f) and s0 + 1 (weight f) along each axis:
    linear interpolation of the slice sampled at q - s(z)."""
    zref = nz // 2
    s0 = np.zeros((nz, 2), dtype=np.int64)
    fr = np.zeros((nz, 2), dtype=np.float64)
    for z in range(nz):
        for a in range(2):
            v = float(z - zref) * float(shear[a])
            s0[z, a] = math.floor(v)
            fr[z, a] = v - s0[z, a]
    return s0, fr


def scan_positions(scan_n, scan_step, scan_origin):
    """Top-left object voxel (py, px) of the probe support for each raster frame."""
    rows, cols = int(scan_n[0]), int(scan_n[1])
    out = np.zeros((rows * cols, 2), dtype=np.int64)
    for iy in range(rows):
        for ix in range(cols):
            out[iy * cols + ix, 0] = int(scan_origin[0]) + iy * int(scan_step[0])
            out[iy * cols + ix, 1] = int(scan_origin[1]) + ix * int(scan_step[1])
    return out


def _lateral_map(problem):
    lm = getattr(problem, "lateral_map", None)
    return None if lm is None else np.asarray(lm, dtype=np.float64)


def mapped_geometry(problem, m):
    """R with a detector map (problem.lateral_map[m] = M, 2 x 2): the probe window's
    lateral point (a, b) of slice z lands on the exit-wave point
        q = M ((a, b) - n/2) + (c + n/2) + (z - nz//2) t_m
    (n the probe support, c the window offset of the support, t_m the exit-beam offset per
    slice, in exit-wave pixels), so the support's centre lands where the unmapped model
    puts it, and M = identity gives the interpolated-offset model.  Returns (M, M^-1, the
    centre c + n/2, the offsets (z - nz//2) t_m [nz][2])."""
    mat = _lateral_map(problem)[m]
    n = problem.probe_n
    centre = window_offset(int(problem.det[m]), n) + n / 2.0
    dz = np.arange(problem.nz, dtype=np.float64) - problem.nz // 2
    offs = dz[:, None] * np.asarray(problem.shear[m], dtype=np.float64)[None, :]
    return mat, np.linalg.inv(mat), centre, offs


def mapped_extent(problem, m):
    """Smallest and largest exit-wave pixel (per axis) that a mapped slice can reach: the
    images of the support's corners widened by one sample (the interpolation's reach)."""
    mat, _, centre, offs = mapped_geometry(problem, m)
    n = problem.probe_n
    corners = np.array([[a, b] for a in (-1.0, float(n)) for b in (-1.0, float(n))]) - n / 2.0
    pts = (corners @ mat.T)[None, :, :] + centre + offs[:, None, :]
    return np.floor(pts.min(axis=(0, 1))).astype(np.int64), np.ceil(pts.max(axis=(0, 1))).astype(np.int64)


def _mapped_taps(problem, m, z, det):
    """For every exit-wave pixel q of the D x D window: the pre-image p = M^-1 (q - centre -
    offset_z) + n/2 in the probe window's coordinates, as the four bilinear taps
    (floor(p) + (dy, dx)) and their weights.  Returns (iy [4][D][D], ix, w)."""
    _, minv, centre, offs = mapped_geometry(problem, m)
    n = problem.probe_n
    qy, qx = np.meshgrid(np.arange(det, dtype=np.float64), np.arange(det, dtype=np.float64), indexing="ij")
    ry, rx = qy - centre - offs[z, 0], qx - centre - offs[z, 1]
    py = minv[0, 0] * ry + minv[0, 1] * rx + n / 2.0
    px = minv[1, 0] * ry + minv[1, 1] * rx + n / 2.0
    y0, x0 = np.floor(py), np.floor(px)
    fy, fx = py - y0, px - x0
    iy = np.stack([y0, y0, y0 + 1, y0 + 1]).astype(np.int64)
    ix = np.stack([x0, x0 + 1, x0, x0 + 1]).astype(np.int64)
    w = np.stack([(1 - fy) * (1 - fx), (1 - fy) * fx, fy * (1 - fx), fy * fx])
    return iy, ix, w


def exit_wave_mapped(o_m, probe_m, py, px, problem, m):
    """R diag(P) S O for one frame with the detector map of peak m: slice z's illuminated
    object, sampled on the probe window's n x n grid (zero off the support and off the
    object grid), is interpolated bilinearly at each exit-wave pixel's pre-image, and the
    slices are summed (the projection along k_f)."""
    nz, ny, nx = o_m.shape
    n = probe_m.shape[-1]
    det = int(problem.det[m])
    psi = np.zeros((det, det), dtype=np.complex128)
    a0, a1 = _support_block(py, n, ny)
    b0, b1 = _support_block(px, n, nx)
    if a1 <= a0 or b1 <= b0:
        return psi
    for z in range(nz):
        ill = np.zeros((n, n), dtype=np.complex128)
        ill[a0:a1, b0:b1] = _probe_slice(probe_m, z)[a0:a1, b0:b1] * o_m[z, py + a0:py + a1, px + b0:px + b1]
        iy, ix, w = _mapped_taps(problem, m, z, det)
        inside = (iy >= 0) & (iy < n) & (ix >= 0) & (ix < n)
        vals = ill[np.clip(iy, 0, n - 1), np.clip(ix, 0, n - 1)]
        psi += np.sum(np.where(inside, w * vals, 0.0), axis=0)
    return psi


def back_project_mapped(g_psi, probe_m, py, px, problem, m, g_o_m):
    """Adjoint of exit_wave_mapped, accumulated into g_o_m in place: every exit-wave
    pixel's gradient goes back to its four taps with the same weights, then
    g_O[z, py + a, px + b] += conj(P_z[a, b]) (sum over those contributions)."""
    nz, ny, nx = g_o_m.shape
    n = probe_m.shape[-1]
    det = g_psi.shape[0]
    a0, a1 = _support_block(py, n, ny)
    b0, b1 = _support_block(px, n, nx)
    if a1 <= a0 or b1 <= b0:
        return
    for z in range(nz):
        iy, ix, w = _mapped_taps(problem, m, z, det)
        inside = (iy >= 0) & (iy < n) & (ix >= 0) & (ix < n)
        acc = np.zeros((n, n), dtype=np.complex128)
        np.add.at(acc, (iy[inside], ix[inside]), (w * g_psi[None, :, :])[inside])
        g_o_m[z, py + a0:py + a1, px + b0:px + b1] += (
            np.conj(_probe_slice(probe_m, z)[a0:a1, b0:b1]) * acc[a0:a1, b0:b1])


class FootprintError(ValueError):
    """The sheared probe support of some slice leaves the detector window."""


def tables(problem):
    """All integer tables of a workload.

    Returns dict with
      scan   [F][2] int: (py, px) per global frame (peaks concatenated, raster order)
      shear  [M][nz][2] int: s_m(z) (with problem.shear_linear: floor of the offset)
      shear_frac [M][nz][2] float or None: fractional offsets (problem.shear_linear)
      y_off  [M+1] int: element offset of peak m's intensities in the ragged y array
      peak_of_frame [F] int, local_index [F] int
      offset [M] int: window offset c_m
    Raises FootprintError when a sheared support leaves its window.
    """
    m_count = problem.n_peaks
    scans, peak_of, local = [], [], []
    shear = np.zeros((m_count, problem.nz, 2), dtype=np.int64)
    linear = bool(getattr(problem, "shear_linear", False))
    frac = np.zeros((m_count, problem.nz, 2)) if linear else None
    y_off = np.zeros(m_count + 1, dtype=np.int64)
    offs = np.zeros(m_count, dtype=np.int64)
    for m in range(m_count):
        det = int(problem.det[m])
        c = window_offset(det, problem.probe_n)
        if c < 0:
            raise FootprintError(f"peak {m}: probe support {problem.probe_n} > window {det}")
        offs[m] = c
        if linear:
            shear[m], frac[m] = shear_table_linear(problem.nz, problem.shear[m])
        else:
            shear[m] = shear_table(problem.nz, problem.shear[m])
        if _lateral_map(problem) is not None:
            qlo, qhi = mapped_extent(problem, m)
            if (qlo < 0).any() or (qhi > det - 1).any():
                raise FootprintError(f"peak {m}: mapped support leaves the {det}x{det} window")
        else:
            lo = shear[m].min(axis=0)
            hi = shear[m].max(axis=0) + (1 if linear else 0)
            if (c + lo < 0).any() or (c + problem.probe_n - 1 + hi > det - 1).any():
                raise FootprintError(f"peak {m}: sheared support leaves the {det}x{det} window")
        pos = scan_positions(problem.scan_n[m], problem.scan_step[m], problem.scan_origin[m])
        scans.append(pos)
        peak_of.append(np.full(len(pos), m, dtype=np.int64))
        local.append(np.arange(len(pos), dtype=np.int64))
        y_off[m + 1] = y_off[m] + len(pos) * det * det
    return {
        "scan": np.concatenate(scans),
        "shear": shear,
        "shear_frac": frac,
        "y_off": y_off,
        "peak_of_frame": np.concatenate(peak_of),
        "local_index": np.concatenate(local),
        "offset": offs,
    }


# ---------------------------------------------------------------------------------
# Forward model, eq. (1)-(3) and eq. (2).
# ---------------------------------------------------------------------------------

def phases(u, g):
    """phi_m = G_m . u for every voxel, u of shape [3][nz][ny][nx]."""
    return g[0] * u[0] + g[1] * u[1] + g[2] * u[2]


def objects(u, chi, alpha, problem):
    """O_m = alpha_m * chi * exp(i G_m . u), complex128 [M][nz][ny][nx] (eq. (3))."""
    u = np.asarray(u, dtype=np.float64)
    chi = np.asarray(chi, dtype=np.float64)
    out = np.empty((problem.n_peaks,) + chi.shape, dtype=np.complex128)
    for m in range(problem.n_peaks):
        out[m] = float(alpha[m]) * chi * np.exp(1j * phases(u, problem.g[m]))
    return out


def _support_block(p0, n, size):
    """Valid probe rows [a0, a1) of a support of n starting at object row p0."""
    a0 = max(0, -p0)
    a1 = min(n, size - p0)
    return a0, max(a0, a1)


def _probe_slice(probe_m, z):
    """The probe of slice z: probe_m is [n][n] (constant along x3) or [nz][n][n] (a 3D
    illumination volume, section 2)."""
    return probe_m[z] if probe_m.ndim == 3 else probe_m


def _taps(frac_m, z):
    """(dy, dx, weight) of slice z: one tap of weight 1 for rounded offsets, four
    bilinear taps for interpolated ones."""
    if frac_m is None:
        return [(0, 0, 1.0)]
    fy, fx = float(frac_m[z, 0]), float(frac_m[z, 1])
    return [(0, 0, (1 - fy) * (1 - fx)), (0, 1, (1 - fy) * fx), (1, 0, fy * (1 - fx)), (1, 1, fy * fx)]


def exit_wave(o_m, probe_m, py, px, shear_m, det, frac_m=None):
    """R diag(P) S O for one frame: the D x D exit wave.

    For every slice z and probe pixel (a, b) with an in-grid object voxel,
      psi[a + c + s_y(z), b + c + s_x(z)] += P_z[a, b] * O[z, py + a, px + b]
    (P_z = P for a probe constant along x3).  With fractional offsets (frac_m), the term
    goes to the four offsets s(z) + (dy, dx), dy, dx in {0, 1}, with the bilinear weights
    of the fractions.
    """
    nz, ny, nx = o_m.shape
    n = probe_m.shape[-1]
    c = window_offset(det, n)
    psi = np.zeros((det, det), dtype=np.complex128)
    a0, a1 = _support_block(py, n, ny)
    b0, b1 = _support_block(px, n, nx)
    if a1 <= a0 or b1 <= b0:
        return psi
    for z in range(nz):
        w = _probe_slice(probe_m, z)[a0:a1, b0:b1] * o_m[z, py + a0:py + a1, px + b0:px + b1]
        for dy, dx, wt in _taps(frac_m, z):
            sy, sx = int(shear_m[z, 0]) + dy, int(shear_m[z, 1]) + dx
            psi[c + sy + a0:c + sy + a1, c + sx + b0:c + sx + b1] += wt * w
    return psi


def back_project(g_psi, probe_m, py, px, shear_m, g_o_m, frac_m=None):
    """Adjoint of exit_wave, accumulated into g_o_m in place:
      g_O[z, py + a, px + b] += conj(P_z[a, b]) * g_psi[a + c + s_y(z), b + c + s_x(z)]
    (with fractional offsets: the bilinearly weighted sum of the four taps).
    """
    nz, ny, nx = g_o_m.shape
    n = probe_m.shape[-1]
    det = g_psi.shape[0]
    c = window_offset(det, n)
    a0, a1 = _support_block(py, n, ny)
    b0, b1 = _support_block(px, n, nx)
    if a1 <= a0 or b1 <= b0:
        return
    for z in range(nz):
        pc = np.conj(_probe_slice(probe_m, z)[a0:a1, b0:b1])
        for dy, dx, wt in _taps(frac_m, z):
            sy, sx = int(shear_m[z, 0]) + dy, int(shear_m[z, 1]) + dx
            g_o_m[z, py + a0:py + a1, px + b0:px + b1] += (
                wt * pc * g_psi[c + sy + a0:c + sy + a1, c + sx + b0:c + sx + b1])


def far_field(psi):
    """F psi: orthonormal 2D DFT, kernel exp(-2 pi i k.x / D), DC at [0, 0]."""
    return np.fft.fft2(psi, norm="ortho")


def far_field_adjoint(g):
    """F^H g (the inverse orthonormal DFT)."""
    return np.fft.ifft2(g, norm="ortho")


def amplitude_residual(psi_ff, y, b=None):
    """Per-frame term of eq. (4) and its gradient with respect to the far field.

    With the model intensity I = |Psi|^2 + b of eq. (2) (b = 0 when None), returns
    (f_frame, R) with f_frame = 1/2 sum (sqrt(I) - sqrt(y))^2 and
    R = (sqrt(I) - sqrt(y)) * Psi / sqrt(I) (0 where I = 0).
    """
    if b is None:
        a = np.abs(psi_ff)
    else:
        a = np.sqrt(np.abs(psi_ff) ** 2 + np.asarray(b, dtype=np.float64))
    r = a - np.sqrt(np.asarray(y, dtype=np.float64))
    f = 0.5 * float(np.sum(r * r))
    safe = np.where(a > 0.0, a, 1.0)
    grad = np.where(a > 0.0, r * psi_ff / safe, 0.0)
    return f, grad


# ---------------------------------------------------------------------------------
# Whole objective and gradient.
# ---------------------------------------------------------------------------------

def _frame_list(problem, frames):
    if frames is None:
        return list(range(problem.n_frames()))
    frames = [int(f) for f in frames]
    if len(set(frames)) != len(frames):
        raise ValueError("duplicate frame ids")
    for f in frames:
        if not 0 <= f < problem.n_frames():
            raise ValueError(f"frame id {f} out of range")
    return frames


def frame_data(y, tab, problem, fid):
    """The D x D intensities of global frame `fid` from the ragged y array."""
    m = int(tab["peak_of_frame"][fid])
    j = int(tab["local_index"][fid])
    det = int(problem.det[m])
    start = int(tab["y_off"][m]) + j * det * det
    return np.asarray(y[start:start + det * det], dtype=np.float64).reshape(det, det)


def _frac(tab, m):
    return None if tab["shear_frac"] is None else tab["shear_frac"][m]


def _exit(o_m, probe_m, py, px, tab, problem, m):
    if _lateral_map(problem) is not None:
        return exit_wave_mapped(o_m, probe_m, py, px, problem, m)
    return exit_wave(o_m, probe_m, py, px, tab["shear"][m], int(problem.det[m]), _frac(tab, m))


def _back(g_psi, probe_m, py, px, tab, problem, m, g_o_m):
    if _lateral_map(problem) is not None:
        back_project_mapped(g_psi, probe_m, py, px, problem, m, g_o_m)
    else:
        back_project(g_psi, probe_m, py, px, tab["shear"][m], g_o_m, _frac(tab, m))


def model_intensity(u, chi, alpha, probe, problem, frames=None, background=None):
    """I_{m,j} of eq. (2) for the listed frames: list of D x D float64 arrays."""
    tab = tables(problem)
    obj = objects(u, chi, alpha, problem)
    probe = np.asarray(probe, dtype=np.complex128)
    out = []
    for fid in _frame_list(problem, frames):
        m = int(tab["peak_of_frame"][fid])
        py, px = (int(v) for v in tab["scan"][fid])
        psi = _exit(obj[m], probe[m], py, px, tab, problem, m)
        inten = np.abs(far_field(psi)) ** 2
        if background is not None:
            inten = inten + frame_data(background, tab, problem, fid)
        out.append(inten)
    return out


def loss(u, chi, alpha, probe, y, problem, frames=None, background=None):
    """f of eq. (4) over the listed frames (all when None).

    Returns (f, per_frame) with per_frame the list of per-frame terms.
    """
    tab = tables(problem)
    obj = objects(u, chi, alpha, problem)
    probe = np.asarray(probe, dtype=np.complex128)
    per = []
    for fid in _frame_list(problem, frames):
        m = int(tab["peak_of_frame"][fid])
        py, px = (int(v) for v in tab["scan"][fid])
        psi = _exit(obj[m], probe[m], py, px, tab, problem, m)
        b = None if background is None else frame_data(background, tab, problem, fid)
        f, _ = amplitude_residual(far_field(psi), frame_data(y, tab, problem, fid), b)
        per.append(f)
    return float(sum(per)), per


def object_gradient(u, chi, alpha, probe, y, problem, frames=None, background=None):
    """f and g_O,m = df/dO_m (complex, [M][nz][ny][nx]) summed over the listed frames."""
    tab = tables(problem)
    obj = objects(u, chi, alpha, problem)
    probe = np.asarray(probe, dtype=np.complex128)
    g_obj = np.zeros_like(obj)
    per = []
    for fid in _frame_list(problem, frames):
        m = int(tab["peak_of_frame"][fid])
        py, px = (int(v) for v in tab["scan"][fid])
        det = int(problem.det[m])
        psi = _exit(obj[m], probe[m], py, px, tab, problem, m)
        b = None if background is None else frame_data(background, tab, problem, fid)
        f, grad_ff = amplitude_residual(far_field(psi), frame_data(y, tab, problem, fid), b)
        per.append(f)
        _back(far_field_adjoint(grad_ff), probe[m], py, px, tab, problem, m, g_obj[m])
    return float(sum(per)), per, g_obj, obj


def loss_grad(u, chi, alpha, probe, y, problem, frames=None, background=None):
    """f and its gradient with respect to u, chi and alpha.

    Chain rule through O_m = alpha_m chi exp(i phi_m), phi_m = G_m . u:
      df/dphi_m   = Im(g_O,m * conj(O_m))
      df/du_c     = sum_m G_m,c * df/dphi_m
      df/dchi     = sum_m Re(conj(g_O,m) * alpha_m * exp(i phi_m))
      df/dalpha_m = sum_voxels Re(conj(g_O,m) * chi * exp(i phi_m))
    Returns dict(loss, frame_loss, grad_u [3][nz][ny][nx], grad_chi, grad_alpha [M]).
    """
    f, per, g_obj, obj = object_gradient(u, chi, alpha, probe, y, problem, frames, background)
    u = np.asarray(u, dtype=np.float64)
    chi = np.asarray(chi, dtype=np.float64)
    grad_u = np.zeros(u.shape)
    grad_chi = np.zeros(chi.shape)
    grad_alpha = np.zeros(problem.n_peaks)
    for m in range(problem.n_peaks):
        e = np.exp(1j * phases(u, problem.g[m]))
        dphi = np.imag(g_obj[m] * np.conj(obj[m]))
        for c in range(3):
            grad_u[c] += problem.g[m][c] * dphi
        grad_chi += np.real(np.conj(g_obj[m]) * float(alpha[m]) * e)
        grad_alpha[m] = float(np.sum(np.real(np.conj(g_obj[m]) * chi * e)))
    return {
        "loss": f,
        "frame_loss": np.asarray(per),
        "grad_u": grad_u,
        "grad_chi": grad_chi,
        "grad_alpha": grad_alpha,
    }


def loss_grad_ztied(u2, chi2, alpha, probe, y, problem, frames=None, background=None):
    """The membrane parameterisation of section 3 (unknowns per lateral pixel, constant
    along x3): u2 [3][1][ny][nx], chi2 [1][ny][nx] broadcast over z; gradients are the
    z-sums of the per-voxel gradients."""
    nz = problem.nz
    u = np.broadcast_to(np.asarray(u2, dtype=np.float64), (3, nz) + tuple(np.shape(u2)[2:]))
    chi = np.broadcast_to(np.asarray(chi2, dtype=np.float64), (nz,) + tuple(np.shape(chi2)[1:]))
    r = loss_grad(u, chi, alpha, probe, y, problem, frames, background)
    r["grad_u"] = r["grad_u"].sum(axis=1, keepdims=True)
    r["grad_chi"] = r["grad_chi"].sum(axis=0, keepdims=True)
    return r


def step(params, grads, eta):
    """Plain gradient step p <- p - eta * g for (u, chi, alpha) with eta = (eta_u,
    eta_chi, eta_alpha)."""
    return tuple(np.asarray(p, dtype=np.float64) - float(e) * np.asarray(g, dtype=np.float64)
                 for p, g, e in zip(params, grads, eta))


# ---------------------------------------------------------------------------------
# The optimiser around the objective (section 3.3, Algorithm 1).
# ---------------------------------------------------------------------------------

def adam_update(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, arXiv:1412.6980, their Algorithm 1) of parameter
    p with gradient g and moments (m, v) at step t >= 1; returns (p', m', v').

      m' = beta1 m + (1 - beta1) g,   v' = beta2 v + (1 - beta2) g^2
      p' = p - lr * (m' / (1 - beta1^t)) / (sqrt(v' / (1 - beta2^t)) + eps)
    """
    p = np.asarray(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def log_param_grad(x, grad_x):
    """Gradient with respect to the log variable x~ of x = exp(x~) (eq. (8)):
    df/dx~ = x * df/dx."""
    return np.asarray(x, dtype=np.float64) * np.asarray(grad_x, dtype=np.float64)


def minibatch(order, n_frames, batch, it):
    """Frames of iteration `it` of Algorithm 1 (section 3.3).

    Each pass over the data starts from a fresh shuffle of the JD = n_frames patterns
    and runs JD/b minibatches (integer division: every minibatch holds b patterns, and
    the JD mod b patterns left at the end of a shuffle wait for a later shuffle).
    `order` holds the shuffles, concatenated (its length a multiple of JD; the passes
    wrap around them).  Iteration it is minibatch t = it mod (JD/b) of pass
    e = it div (JD/b): entries [t b, (t + 1) b) of shuffle e.
    """
    order = np.asarray(order)
    if batch < 1 or batch > n_frames:
        raise ValueError(f"minibatch size {batch} outside [1, {n_frames}]")
    if len(order) == 0 or len(order) % n_frames:
        raise ValueError("order must hold whole shuffles of the frames")
    per_pass = n_frames // batch
    shuffles = len(order) // n_frames
    e, t = divmod(int(it), per_pass)
    perm = order[(e % shuffles) * n_frames:(e % shuffles + 1) * n_frames]
    return [int(f) for f in perm[t * batch:(t + 1) * batch]]


def adam_reconstruct(u, chi_log, alpha_log, probe, y, problem, order, batch, iterations,
                     lr=(0.01, 0.1, 0.1), fixed_alpha=0, beta1=0.9, beta2=0.999, eps=1e-8,
                     unwrap=False):
    """Algorithm 1: the minibatches of `minibatch` (JD/b per shuffle of the frames; the
    shuffles are an input), minibatch gradients summed over the frames (eq. (11)), then
    Adam on u and on the log variables chi~, alpha~ of eq. (8), alpha of peak
    `fixed_alpha` held fixed (-1: none); with unwrap=True every update of u is followed
    by the unwrap projection Pi_U of eq. (10) (the algorithm's last step; without it, the
    concurrent-wrapped variant).  Returns (u, chi_log, alpha_log, losses) with the
    minibatch loss of every iteration (evaluated before that iteration's update)."""
    u = np.array(u, dtype=np.float64)
    cl = np.array(chi_log, dtype=np.float64)
    al = np.array(alpha_log, dtype=np.float64)
    mom = [np.zeros_like(u), np.zeros_like(cl), np.zeros_like(al)]
    sec = [np.zeros_like(u), np.zeros_like(cl), np.zeros_like(al)]
    losses = []
    for it in range(iterations):
        frames = minibatch(order, problem.n_frames(), batch, it)
        chi, alpha = np.exp(cl), np.exp(al)
        r = loss_grad(u, chi, alpha, probe, y, problem, frames)
        losses.append(r["loss"])
        grads = [r["grad_u"], log_param_grad(chi, r["grad_chi"]), log_param_grad(alpha, r["grad_alpha"])]
        t = it + 1
        u, mom[0], sec[0] = adam_update(u, grads[0], mom[0], sec[0], t, lr[0], beta1, beta2, eps)
        if unwrap:
            from oracle.unwrap_oracle import unwrap_projector
            u = unwrap_projector(u.astype(np.float32), problem.g)
        cl, mom[1], sec[1] = adam_update(cl, grads[1], mom[1], sec[1], t, lr[1], beta1, beta2, eps)
        keep = al[fixed_alpha] if fixed_alpha >= 0 else None
        keep_m = (mom[2][fixed_alpha], sec[2][fixed_alpha]) if fixed_alpha >= 0 else None
        al, mom[2], sec[2] = adam_update(al, grads[2], mom[2], sec[2], t, lr[2], beta1, beta2, eps)
        if fixed_alpha >= 0:
            al[fixed_alpha] = keep
            mom[2][fixed_alpha], sec[2][fixed_alpha] = keep_m
    return u, cl, al, losses


def line_search_descent(u, chi, alpha, probe, y, problem, iterations, step0=0.01, c=1e-4,
                        shrink=0.5, grow=2.0, max_backtracks=30, trials=None):
    """Full-batch gradient descent on u (chi, alpha held) with a backtracking (Armijo)
    step-size search: from u, try u - eta g with eta grown by `grow` from the previous
    accepted step (first: step0 over the RMS of g) and shrunk by `shrink` until
    f(u - eta g) <= f(u) - c eta |g|^2.  Returns (u, losses, etas): the loss before each
    iteration and the accepted step sizes; stops early when no step is accepted.  With
    a list `trials`, each iteration appends the (eta, f(u - eta g)) pairs it tried, in
    order."""
    u = np.array(u, dtype=np.float64)
    losses, etas = [], []
    eta = None
    for _ in range(iterations):
        r = loss_grad(u, chi, alpha, probe, y, problem)
        f0, g = r["loss"], r["grad_u"]
        n2 = float(np.sum(g * g))
        losses.append(f0)
        if n2 == 0.0:
            break
        eta = step0 / math.sqrt(n2 / g.size) if eta is None else eta * grow
        tried = []
        if trials is not None:
            trials.append(tried)
        for _ in range(max_backtracks):
            trial = u - eta * g
            f1, _ = loss(trial, chi, alpha, probe, y, problem)
            tried.append((eta, f1))
            if f1 <= f0 - c * eta * n2:
                u = trial
                etas.append(eta)
                break
            eta *= shrink
        else:
            break
    return u, losses, etas
