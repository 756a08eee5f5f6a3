"""The objective and gradient of the oracle's steps, evaluated in complex64 / float32.

TEST INFRASTRUCTURE (CPU, numpy only).  Neither the package nor the oracle imports this
module.  It takes the oracle's integer tables and then performs each of the oracle's
steps (eq. (1)/(3) objects, the R diag(P) S projection of eq. (2), the orthonormal DFT,
the eq. (4) residual, the adjoint DFT, back-projection and the chain rule) with every
array held in single precision, so that each operation rounds to FP32 as a GPU
implementation's does (in a different order).  Comparing it with the FP64 oracle
measures how far FP32 arithmetic itself can be from the exact result at a given
evaluation point: the conditioning that any FP32 path inherits.
"""
import numpy as np

from oracle import mpbp_oracle as O

F32, C64 = np.float32, np.complex64


def loss_grad_fp32(u, chi, alpha, probe, y, problem, frames=None):
    tab = O.tables(problem)
    if tab["shear_frac"] is not None:
        raise NotImplementedError("rounded exit-beam offsets only")
    u = np.asarray(u, dtype=F32)
    chi = np.asarray(chi, dtype=F32)
    alpha = np.asarray(alpha, dtype=F32)
    probe = np.asarray(probe, dtype=C64)
    g = np.asarray(problem.g, dtype=F32)
    nz, ny, nx = chi.shape
    n = problem.probe_n
    phi = [g[m, 0] * u[0] + g[m, 1] * u[1] + g[m, 2] * u[2] for m in range(problem.n_peaks)]
    e = [(np.cos(p) + 1j * np.sin(p)).astype(C64) for p in phi]
    obj = [(alpha[m] * chi * e[m]).astype(C64) for m in range(problem.n_peaks)]
    g_obj = [np.zeros((nz, ny, nx), dtype=C64) for _ in range(problem.n_peaks)]
    frames = range(problem.n_frames()) if frames is None else frames
    per = []
    for fid in frames:
        m = int(tab["peak_of_frame"][fid])
        py, px = (int(v) for v in tab["scan"][fid])
        det = int(problem.det[m])
        c = (det - n) // 2
        a0, a1 = max(0, -py), min(n, ny - py)
        b0, b1 = max(0, -px), min(n, nx - px)
        psi = np.zeros((det, det), dtype=C64)
        sh = tab["shear"][m]
        if a1 > a0 and b1 > b0:
            for z in range(nz):
                sy, sx = int(sh[z, 0]), int(sh[z, 1])
                psi[c + sy + a0:c + sy + a1, c + sx + b0:c + sx + b1] += (
                    probe[m, a0:a1, b0:b1] * obj[m][z, py + a0:py + a1, px + b0:px + b1])
        X = np.fft.fft2(psi, norm="ortho")
        assert X.dtype == C64
        start = int(tab["y_off"][m]) + int(tab["local_index"][fid]) * det * det
        yy = np.asarray(y[start:start + det * det], dtype=F32).reshape(det, det)
        a = np.abs(X).astype(F32)
        r = (a - np.sqrt(yy)).astype(F32)
        per.append(0.5 * float(np.sum(r.astype(np.float64) ** 2)))
        R = np.where(a > 0, (r / np.where(a > 0, a, F32(1))).astype(F32) * X, 0).astype(C64)
        gpsi = np.fft.ifft2(R, norm="ortho").astype(C64)
        if a1 > a0 and b1 > b0:
            for z in range(nz):
                sy, sx = int(sh[z, 0]), int(sh[z, 1])
                g_obj[m][z, py + a0:py + a1, px + b0:px + b1] += (
                    np.conj(probe[m, a0:a1, b0:b1]) * gpsi[c + sy + a0:c + sy + a1, c + sx + b0:c + sx + b1])
    grad_u = np.zeros((3, nz, ny, nx), dtype=F32)
    grad_chi = np.zeros((nz, ny, nx), dtype=F32)
    grad_alpha = np.zeros(problem.n_peaks, dtype=np.float64)
    for m in range(problem.n_peaks):
        dphi = np.imag(g_obj[m] * np.conj(obj[m])).astype(F32)
        for k in range(3):
            grad_u[k] += g[m, k] * dphi
        re = np.real(np.conj(g_obj[m]) * e[m]).astype(F32)
        grad_chi += alpha[m] * re
        grad_alpha[m] = float(np.sum((chi * re).astype(np.float64)))
    return {"loss": float(np.sum(per)), "frame_loss": np.asarray(per), "grad_u": grad_u, "grad_chi": grad_chi,
            "grad_alpha": grad_alpha}


def rel_errors(got, ref):
    """Relative 2-norm error per output field (loss: relative error)."""
    out = {"loss": abs(got["loss"] - ref["loss"]) / abs(ref["loss"])}
    for k in ("grad_chi", "grad_alpha"):
        out[k] = float(np.linalg.norm(np.asarray(got[k], np.float64) - ref[k]) / np.linalg.norm(ref[k]))
    for c in range(3):
        out[f"grad_u[{c}]"] = float(np.linalg.norm(np.asarray(got["grad_u"][c], np.float64) - ref["grad_u"][c])
                                    / np.linalg.norm(ref["grad_u"][c]))
    return out
