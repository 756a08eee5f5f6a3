"""Seeded synthetic inputs: geometry, probe and strained-membrane fields.

Random-number order (numpy default_rng(seed)): white noise for the three displacement
components (x, y, z), then white noise for the three components of the perturbation
field delta, then the Poisson draws of the intensities in global frame order.
"""
from dataclasses import dataclass, field
import math

import numpy as np

LATTICE_A_NM = 0.2 * math.sqrt(3.0)   # |G_111| = 2*pi/0.2 nm^-1
STEP_NM = 0.05                        # planar displacement step height


@dataclass
class Problem:
    """Geometry of one multi-peak Bragg ptychography workload (host values).

    g[m]           Bragg vector G_m in rad/nm, lab frame (x1, x2, x3) = (x, y, z)
    shear[m]       (t_y, t_x): lateral exit-beam offset per z-slice, in voxels
    det[m]         detector / window size D_m (square)
    scan_n[m]      raster size (rows, cols); frame j = row * cols + col
    scan_step[m]   raster step (rows, cols) in voxels
    scan_origin[m] top-left of the probe support of frame 0 (may be negative)
    """
    name: str
    nz: int
    ny: int
    nx: int
    probe_n: int
    g: np.ndarray
    shear: np.ndarray
    det: np.ndarray
    scan_n: np.ndarray
    scan_step: np.ndarray
    scan_origin: np.ndarray
    photons: list = field(default_factory=list)
    shear_linear: bool = False   # exit-beam offsets interpolated linearly (not rounded)
    # per-peak map of the probe window's lateral voxel coordinates to exit-wave pixels
    # ([M][2][2]: the detector frame's in-plane rotation and pixel size), or None
    lateral_map: np.ndarray = None

    @property
    def n_peaks(self):
        return int(self.g.shape[0])

    def frames_per_peak(self):
        return [int(self.scan_n[m, 0] * self.scan_n[m, 1]) for m in range(self.n_peaks)]

    def n_frames(self):
        return int(sum(self.frames_per_peak()))


def bragg_vector(hkl, a_nm=LATTICE_A_NM):
    """G_hkl = (2*pi/a) * (h, k, l) in rad/nm (cubic lattice of constant a_nm)."""
    return (2.0 * math.pi / a_nm) * np.asarray(hkl, dtype=np.float64)


def shear_direction(g, tan_theta):
    """Exit-beam lateral offset per slice: tan(theta) along the in-plane direction of G.

    Returns (t_y, t_x) as doubles; zero when G has no in-plane component.
    """
    gx, gy = float(g[0]), float(g[1])
    n = math.sqrt(gx * gx + gy * gy)
    if n == 0.0:
        return np.zeros(2)
    return np.array([tan_theta * (gy / n), tan_theta * (gx / n)], dtype=np.float64)


def scan_origin(n_obj, n_scan, step, probe_n):
    """Centre the raster on the object: (N - ((n - 1) * step + Np)) // 2 (floor)."""
    return (n_obj - ((n_scan - 1) * step + probe_n)) // 2


def make_problem(cfg):
    """Geometry (Bragg vectors, shears, rasters) of workload description `cfg`."""
    m = len(cfg["peaks"])
    g = np.zeros((m, 3))
    shear = np.zeros((m, 2))
    det = np.zeros(m, dtype=np.int64)
    scan_n = np.zeros((m, 2), dtype=np.int64)
    scan_step = np.zeros((m, 2), dtype=np.int64)
    origin = np.zeros((m, 2), dtype=np.int64)
    photons = []
    for k, pk in enumerate(cfg["peaks"]):
        g[k] = bragg_vector(pk["hkl"], cfg.get("lattice_nm", LATTICE_A_NM))
        shear[k] = shear_direction(g[k], pk["tan_theta"])
        det[k] = pk["det"]
        scan_n[k] = pk["scan_n"]
        scan_step[k] = pk["scan_step"]
        origin[k, 0] = scan_origin(cfg["ny"], pk["scan_n"][0], pk["scan_step"][0], cfg["probe_n"])
        origin[k, 1] = scan_origin(cfg["nx"], pk["scan_n"][1], pk["scan_step"][1], cfg["probe_n"])
        photons.append(pk["photons"])
    return Problem(cfg["name"], cfg["nz"], cfg["ny"], cfg["nx"], cfg["probe_n"],
                   g, shear, det, scan_n, scan_step, origin, photons)


def gaussian_probe(n, fwhm):
    """Complex Gaussian probe with a quadratic phase, n x n support.

    Amplitude exp(-4 ln2 r^2 / fwhm^2), phase kappa * r^2 with kappa = pi / (n/2)^2, r
    measured from the support centre ((n-1)/2, (n-1)/2); pixels whose intensity is
    below 2 % of the maximum are set to zero (section 4 thresholds the probe at 2 %).
    """
    c = (n - 1) / 2.0
    yy, xx = np.meshgrid(np.arange(n) - c, np.arange(n) - c, indexing="ij")
    r2 = yy * yy + xx * xx
    kappa = math.pi / (n / 2.0) ** 2
    p = np.exp(-4.0 * math.log(2.0) * r2 / fwhm ** 2) * np.exp(1j * kappa * r2)
    inten = np.abs(p) ** 2
    p[inten < 0.02 * inten.max()] = 0.0
    return p


def _grf(rng, ny, nx, sigma, corr):
    """Periodic Gaussian random field: white N(0,1) smoothed by a Gaussian of std
    `corr` voxels (FFT convolution), rescaled to standard deviation `sigma`."""
    w = rng.standard_normal((ny, nx))
    ky = np.fft.fftfreq(ny)[:, None]
    kx = np.fft.fftfreq(nx)[None, :]
    kern = np.exp(-2.0 * math.pi ** 2 * corr ** 2 * (ky ** 2 + kx ** 2))
    f = np.fft.ifft2(np.fft.fft2(w) * kern).real
    f -= f.mean()
    s = f.std()
    return f * (sigma / s) if s > 0 else f


def _steps(cfg):
    """Planar displacement steps (nm), shape (3, ny, nx)."""
    ny, nx = cfg["ny"], cfg["nx"]
    yy, xx = np.meshgrid(np.arange(ny) - (ny - 1) / 2.0, np.arange(nx) - (nx - 1) / 2.0,
                         indexing="ij")
    out = np.zeros((3, ny, nx))
    if cfg["steps"] == "single":
        a = math.radians(30.0)
        side = (math.cos(a) * xx + math.sin(a) * yy) > 0
        out[0][side] += STEP_NM
    else:
        n = min(nx, ny)
        for comp, (deg, off) in enumerate([(0.0, -n / 4.0), (60.0, 0.0), (120.0, n / 4.0)]):
            a = math.radians(deg)
            side = (math.cos(a) * xx + math.sin(a) * yy) > off
            out[comp][side] += STEP_NM
    return out


def _energy_per_frame(probe, slab, chi):
    # Nominal detected photons of a frame inside the slab: |sum_z chi P|^2 summed over
    # the support = (T chi)^2 sum |P|^2 (Parseval, slices added in phase).
    return (slab * chi) ** 2 * float(np.sum(np.abs(probe) ** 2))


def make_fields(cfg, problem=None):
    """Seeded true fields of workload `cfg`.

    Returns a dict of float32 / complex64 arrays:
      u      [3][nz][ny][nx]  displacement (nm), z-invariant membrane field
      chi    [nz][ny][nx]     amplitude, uniform inside the slab, zero outside
      alpha  [M]              per-peak scale
      probe  [M][Np][Np]      complex64 probe (the same for every peak)
      delta  [3][nz][ny][nx]  independent perturbation field (std 0.01 nm)
    """
    if problem is None:
        problem = make_problem(cfg)
    rng = np.random.default_rng(cfg["seed"])
    nz, ny, nx = cfg["nz"], cfg["ny"], cfg["nx"]
    u2 = np.stack([_grf(rng, ny, nx, cfg["grf_sigma"], cfg["grf_corr"]) for _ in range(3)])
    u2 += _steps(cfg)
    d2 = np.stack([_grf(rng, ny, nx, 0.01, cfg["grf_corr"]) for _ in range(3)])
    u = np.ascontiguousarray(np.broadcast_to(u2[:, None], (3, nz, ny, nx))).astype(np.float32)
    delta = np.ascontiguousarray(np.broadcast_to(d2[:, None], (3, nz, ny, nx))).astype(np.float32)

    probe = gaussian_probe(cfg["probe_n"], cfg["probe_fwhm"])
    m = problem.n_peaks
    slab = cfg["slab"]
    z0 = (nz - slab) // 2
    if cfg["chi_mode"] == "unit":
        amp0 = 1.0
        alpha = np.ones(m)
    else:
        e1 = _energy_per_frame(probe, slab, 1.0)
        scales = [math.sqrt(problem.photons[k] / e1) for k in range(m)]
        amp0 = scales[0]
        alpha = np.array([s / amp0 for s in scales])
    chi = np.zeros((nz, ny, nx), dtype=np.float32)
    chi[z0:z0 + slab] = amp0
    probes = np.broadcast_to(probe.astype(np.complex64), (m,) + probe.shape).copy()
    return {
        "u": u,
        "chi": chi,
        "alpha": alpha.astype(np.float32),
        "probe": probes,
        "delta": delta,
    }


def photon_rng(cfg):
    """The workload's random stream positioned after the field draws, ready for the
    Poisson draws of the intensities (global frame order)."""
    rng = np.random.default_rng(cfg["seed"])
    ny, nx = cfg["ny"], cfg["nx"]
    for _ in range(6):
        rng.standard_normal((ny, nx))
    return rng


def poisson_counts(rng, intensity):
    """Poisson photon counts with mean `intensity` (float32 result)."""
    lam = np.clip(np.asarray(intensity, dtype=np.float64), 0.0, None)
    return rng.poisson(lam).astype(np.float32)


def speckle_counts(rng, det, n_frames, photons):
    """Model-free speckle-like counts for `n_frames` frames of det x det pixels.

    Exponentially distributed speckle under a centred Gaussian envelope (DC at index 0,
    unshifted layout), scaled to `photons` per frame on average, then Poisson.  Used
    where a workload is too large for the CPU forward model: loss and gradient are
    defined for any non-negative data.
    """
    k = np.fft.fftfreq(det) * det
    env = np.exp(-(k[:, None] ** 2 + k[None, :] ** 2) / (2.0 * (det / 10.0) ** 2))
    env *= (photons / det ** 2) / env.mean()
    lam = rng.exponential(1.0, size=(n_frames, det, det)) * env[None]
    return rng.poisson(lam).astype(np.float32)


def crop_problem(problem, peak_rows):
    """A copy of `problem` keeping, for each peak m, the scan rows
    [peak_rows[m][0], peak_rows[m][1]) of its raster (origin shifted accordingly)."""
    out = Problem(problem.name + "_crop", problem.nz, problem.ny, problem.nx,
                  problem.probe_n, problem.g.copy(), problem.shear.copy(),
                  problem.det.copy(), problem.scan_n.copy(), problem.scan_step.copy(),
                  problem.scan_origin.copy(), list(problem.photons))
    for m, (r0, r1) in enumerate(peak_rows):
        out.scan_n[m, 0] = r1 - r0
        out.scan_origin[m, 0] = problem.scan_origin[m, 0] + r0 * problem.scan_step[m, 0]
    return out


def band_problem(problem, row0, row1):
    """One band of scan rows, with the object rows it touches.

    Keeps the raster rows [row0, row1) of every peak (clipped to each raster) and crops
    the object to the rows [lo, hi) that those frames' probe supports reach (clipped to
    the grid), shifting the raster origins by -lo.  Returns (band, lo, hi, frames) with
    `frames` the global frame ids of `problem` that the band's frames are, in the band's
    own frame order (peak-major, raster order), so that band frame k is problem frame
    frames[k].  Geometry only: nothing of the forward model is evaluated.
    """
    rows = []
    lo, hi = problem.ny, 0
    for m in range(problem.n_peaks):
        r0 = max(0, min(int(row0), int(problem.scan_n[m, 0])))
        r1 = max(r0, min(int(row1), int(problem.scan_n[m, 0])))
        rows.append((r0, r1))
        if r1 > r0:
            top = int(problem.scan_origin[m, 0]) + r0 * int(problem.scan_step[m, 0])
            bottom = int(problem.scan_origin[m, 0]) + (r1 - 1) * int(problem.scan_step[m, 0]) + problem.probe_n
            lo, hi = min(lo, max(top, 0)), max(hi, min(bottom, problem.ny))
    if hi <= lo:
        lo, hi = 0, 1
    band = Problem(problem.name + f"_rows{row0}-{row1}", problem.nz, hi - lo, problem.nx, problem.probe_n,
                   problem.g.copy(), problem.shear.copy(), problem.det.copy(), problem.scan_n.copy(),
                   problem.scan_step.copy(), problem.scan_origin.copy(), list(problem.photons),
                   problem.shear_linear, problem.lateral_map)
    frames = []
    base = 0
    for m, (r0, r1) in enumerate(rows):
        cols = int(problem.scan_n[m, 1])
        band.scan_n[m, 0] = r1 - r0
        band.scan_origin[m, 0] = int(problem.scan_origin[m, 0]) + r0 * int(problem.scan_step[m, 0]) - lo
        frames += [base + iy * cols + ix for iy in range(r0, r1) for ix in range(cols)]
        base += int(problem.scan_n[m, 0]) * cols
    return band, lo, hi, frames


def detector_map(pixel_ratio, angle):
    """The 2 x 2 map of one peak's R from the probe window's lateral voxel coordinates
    (y, x) to its exit-wave pixels: a rotation by `angle` (radians, the detector frame's
    in-plane orientation about the exit beam) scaled by `pixel_ratio` = voxel pitch /
    exit-wave pixel pitch (the Nyquist pixel of that peak's detector geometry)."""
    c, s = math.cos(angle), math.sin(angle)
    return pixel_ratio * np.array([[c, -s], [s, c]], dtype=np.float64)


def frame_order(n_frames, seed, epochs):
    """The shuffled frame order of a minibatch reconstruction: one random permutation
    of all frames per epoch (the shuffle of Algorithm 1), concatenated, int32."""
    rng = np.random.default_rng(seed)
    return np.concatenate([rng.permutation(n_frames) for _ in range(epochs)]).astype(np.int32)


def unwrap_field(nz, ny, nx, seed, sigma_nm=0.2, corr=12.0, noise_nm=0.0):
    """Seeded displacement field for the phase-unwrap tests, float32 [3][nz][ny][nx].

    Each component is a smooth periodic Gaussian random field of standard deviation
    `sigma_nm` and correlation length `corr` voxels (z-invariant), plus, per slice, a
    constant offset of 0.05 sigma and white noise of standard deviation `noise_nm`.
    With sigma = 0.2 nm and corr = 12 the phases G . u of the (111) peaks span several
    multiples of 2 pi while neighbouring pixels differ by less than pi."""
    rng = np.random.default_rng(seed)
    base = np.stack([_grf(rng, ny, nx, sigma_nm, corr) for _ in range(3)])
    u = np.repeat(base[:, None], nz, axis=1)
    u += 0.05 * sigma_nm * rng.standard_normal((3, nz, 1, 1))
    if noise_nm > 0:
        u += noise_nm * rng.standard_normal(u.shape)
    return u.astype(np.float32)


def lattice_jump(u, y0, y1, x0, x1, cells=1):
    """Copy of u with `cells` lattice translations a * e_x added on the lateral patch
    [y0, y1) x [x0, x1) of every slice: for every Bragg vector G_hkl = (2 pi / a)(h, k, l)
    the phase changes by 2 pi h cells, a multiple of 2 pi (the periodicity artefact the
    unwrap projector removes)."""
    v = np.array(u, dtype=np.float32, copy=True)
    v[0, ..., y0:y1, x0:x1] += np.float32(cells * LATTICE_A_NM)
    return v


def incident_probe_3d(probe2d, nz, t_in):
    """3D illumination volume [nz][n][n] from a 2D beam profile: the profile is carried
    unchanged along an inclined incident beam, so the support of slice z is the 2D
    profile shifted laterally by round((z - nz // 2) * t_in) pixels (t_in = (t_y, t_x),
    the incident beam's lateral offset per slice).  Pixels shifted out of the n x n
    window are dropped (section 4 builds its 3D probes this way from a measured profile)."""
    p = np.asarray(probe2d)
    n = p.shape[-1]
    out = np.zeros((nz, n, n), dtype=p.dtype)
    for z in range(nz):
        dy = int(np.floor((z - nz // 2) * float(t_in[0]) + 0.5))
        dx = int(np.floor((z - nz // 2) * float(t_in[1]) + 0.5))
        ys, yd = (0, dy) if dy >= 0 else (-dy, 0)
        xs, xd = (0, dx) if dx >= 0 else (-dx, 0)
        h, w = n - abs(dy), n - abs(dx)
        if h > 0 and w > 0:
            out[z, yd:yd + h, xd:xd + w] = p[ys:ys + h, xs:xs + w]
    return out
