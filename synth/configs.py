"""The synthetic strained-membrane workloads (five, and a one-eighth crop of the fifth).

Each workload is a plain dictionary.  Geometry readings (where the paper is silent):

* Bragg vectors G_hkl = (2*pi/a) * (h, k, l) in rad/nm with a = 0.2*sqrt(3) nm, so
  |G_111| = 2*pi/0.2 nm^-1; the phase of the object for peak m is G_m . u (eq. (1)
  and eq. (3) of the paper, with the 2*pi folded into G).
* Exit-beam shear: tan(theta_m) along the in-plane direction of G_m (section 2, the
  operator R of eq. (2) projects along k_f; here as an integer lateral shear per
  z-slice).
* Raster scan origin = (N - ((n - 1) * step + Np)) // 2 per axis (floor), frames in
  row-major raster order.
* Probe support Np = 16 with FWHM 6 for the tiny case and Np = 32 with FWHM 12 for the
  others; slab thickness T = round(0.75 * Nz) centred in z.
"""
import copy

# (h, k, l) and tan(theta) of every Bragg peak used by the workloads, in the order the
# multi-peak workloads list them.
PEAKS = [
    ((1, 1, 1), 0.30),
    ((-1, 1, 1), 0.40),
    ((1, -1, 1), 0.50),
    ((2, 0, 0), 0.60),
    ((0, 2, 0), 0.35),
    ((-1, -1, 1), 0.45),
]

_SEED_BASE = 231214907

# The paper's numerical experiment (section 4, Table 1): a cubic lattice of 0.3905 nm, the
# in-plane peaks [100], [110], [120], [210] at 9 keV (wavelength 0.1377 nm), a 150 x 150
# detector, a 9 x 9 raster at a step of 6 pixels, and mean count rates of 83, 65, 52 and
# 12 photons per detector pixel.  tan(theta) follows from Bragg's law, sin(theta) =
# wavelength / (2 d), d = a / |hkl|.
PAPER_LATTICE_NM = 0.3905
PAPER_WAVELENGTH_NM = 0.1377
PAPER_PEAKS = [(1, 0, 0), (1, 1, 0), (1, 2, 0), (2, 1, 0)]
PAPER_COUNTS = [83.0, 65.0, 52.0, 12.0]


def _paper_tan_theta(hkl):
    import math
    d = PAPER_LATTICE_NM / math.sqrt(sum(h * h for h in hkl))
    s = PAPER_WAVELENGTH_NM / (2.0 * d)
    return s / math.sqrt(1.0 - s * s)


def _scan_step(n_obj, n_scan, probe_n):
    # Evenly spread raster covering the object: step = (N - Np) // (n - 1).
    return (n_obj - probe_n) // (n_scan - 1)


def _peak(k, det, scan_n, scan_step, photons):
    hkl, tan_theta = PEAKS[k]
    return {
        "hkl": hkl,
        "tan_theta": tan_theta,
        "det": det,
        "scan_n": tuple(scan_n),
        "scan_step": tuple(scan_step),
        "photons": photons,
    }


def _c1():
    return {
        "name": "c1_tiny",
        "index": 1,
        "nz": 8, "ny": 32, "nx": 32,
        "voxel_nm": 10.0,
        "probe_n": 16, "probe_fwhm": 6.0,
        "slab": 6,
        "chi_mode": "unit",          # amplitude 1 inside the slab, alpha = 1
        "grf_sigma": 0.02, "grf_corr": 4.0,
        "steps": "single",           # one planar step of 0.05 nm along x
        "noise": False,
        "peaks": [_peak(k, 32, (5, 5), (4, 4), None) for k in range(3)],
    }


def _c2():
    return {
        "name": "c2_forward",
        "index": 2,
        "nz": 16, "ny": 128, "nx": 128,
        "voxel_nm": 10.0,
        "probe_n": 32, "probe_fwhm": 12.0,
        "slab": 12,
        "chi_mode": "photons",
        "grf_sigma": 0.02, "grf_corr": 4.0,
        "steps": "three",
        "noise": True,
        "peaks": [_peak(k, 64, (16, 16), (6, 6), 1e5) for k in range(3)],
    }


def _c3():
    st = _scan_step(256, 32, 32)
    return {
        "name": "c3_grad",
        "index": 3,
        "nz": 24, "ny": 256, "nx": 256,
        "voxel_nm": 10.0,
        "probe_n": 32, "probe_fwhm": 12.0,
        "slab": 18,
        "chi_mode": "photons",
        "grf_sigma": 0.02, "grf_corr": 4.0,
        "steps": "three",
        "noise": True,
        "peaks": [_peak(k, 128, (32, 32), (st, st), 1e5) for k in range(4)],
    }


def _c4():
    scans = [(20, 20), (24, 28), (32, 32), (36, 30), (40, 40), (28, 28)]
    dets = [64, 96, 128, 128, 192, 256]
    peaks = []
    for k in range(6):
        n = scans[k]
        step = (_scan_step(256, n[0], 32), _scan_step(256, n[1], 32))
        photons = 1e4 * 100.0 ** (k / 5.0)
        peaks.append(_peak(k, dets[k], n, step, photons))
    return {
        "name": "c4_batch",
        "index": 4,
        "nz": 32, "ny": 256, "nx": 256,
        "voxel_nm": 10.0,
        "probe_n": 32, "probe_fwhm": 12.0,
        "slab": 24,
        "chi_mode": "photons",
        "grf_sigma": 0.02, "grf_corr": 4.0,
        "steps": "three",
        "noise": True,
        "peaks": peaks,
    }


def _c5():
    return {
        "name": "c5_full",
        "index": 5,
        "nz": 32, "ny": 512, "nx": 512,
        "voxel_nm": 10.0,
        "probe_n": 32, "probe_fwhm": 12.0,
        "slab": 24,
        "chi_mode": "photons",
        "grf_sigma": 0.02, "grf_corr": 4.0,
        "steps": "three",
        "noise": True,
        "peaks": [_peak(k, 256, (64, 64), (8, 8), 1e5) for k in range(3)],
    }


def _c5_crop8():
    # One eighth of c5_full in volume (32 x 256 x 128) and in frames (32 x 16 raster per
    # peak), same peaks, probe, detector and raster step: the CPU-timing stand-in of the
    # full loop.
    cfg = _c5()
    cfg.update({"name": "c5_crop8", "index": 6, "ny": 256, "nx": 128})
    cfg["peaks"] = [_peak(k, 256, (32, 16), (8, 8), 1e5) for k in range(3)]
    return cfg


def _c6():
    # The paper-shaped workload: its detector, peaks, raster and count rates; the
    # probe support (32) and the slab (24 of 32 slices) stay within what the kernels
    # take, where the paper has a 100 x 100 probe and a 100-voxel window in x3.
    peaks = []
    for hkl, counts in zip(PAPER_PEAKS, PAPER_COUNTS):
        peaks.append({"hkl": hkl, "tan_theta": _paper_tan_theta(hkl), "det": 150, "scan_n": (9, 9),
                      "scan_step": (6, 6), "photons": counts * 150 * 150})
    return {
        "name": "c6_paper",
        "index": 7,
        "nz": 32, "ny": 200, "nx": 200,
        "voxel_nm": 1.0,
        "lattice_nm": PAPER_LATTICE_NM,
        "probe_n": 32, "probe_fwhm": 12.0,
        "slab": 24,
        "chi_mode": "photons",
        "grf_sigma": 0.02, "grf_corr": 4.0,
        "steps": "three",
        "noise": True,
        "peaks": peaks,
    }


def _c6_100():
    # The paper-shaped workload with the paper's 100-voxel window along x3 (Table 1) and a
    # film of its 17-voxel thickness (section 4) centred in it.
    cfg = _c6()
    cfg.update({"name": "c6_paper100", "index": 8, "nz": 100, "slab": 17})
    return cfg


_BUILDERS = {
    "c1_tiny": _c1,
    "c2_forward": _c2,
    "c3_grad": _c3,
    "c4_batch": _c4,
    "c5_full": _c5,
    "c5_crop8": _c5_crop8,
    "c6_paper": _c6,
    "c6_paper100": _c6_100,
}
CONFIG_NAMES = tuple(_BUILDERS)


def get_config(name):
    """Return a fresh copy of the workload description `name` (one of CONFIG_NAMES)."""
    if name not in _BUILDERS:
        raise KeyError(f"unknown workload {name!r}; choose from {CONFIG_NAMES}")
    cfg = _BUILDERS[name]()
    cfg["seed"] = _SEED_BASE + cfg["index"]
    return copy.deepcopy(cfg)
