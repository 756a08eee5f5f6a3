"""The band split of the parallel oracle runs (tests/oracle_pool.py, synth.band_problem)
against the oracle on the whole workload (CPU).

A band keeps some raster rows of every peak and only the object rows their probe
supports reach.  Its model intensities must equal those of the same frames of the whole
workload, and the band results, added up, must give the whole workload's loss and
gradient (eq. (11); pin P12: sums over a partition of the frames).
"""
import numpy as np
import pytest

from oracle import mpbp_oracle as O
from synth import band_problem, get_config, make_fields, make_problem
from tests.oracle_pool import oracle_whole


def test_band_geometry_c5():
    prob = make_problem(get_config("c5_full"))
    band, lo, hi, frames = band_problem(prob, 28, 36)
    # raster origin -12, step 8, probe 32: rows 28..35 reach object rows 212..299
    assert (lo, hi) == (212, 300)
    assert band.n_frames() == len(frames) == 3 * 8 * 64
    assert frames[0] == 28 * 64 and frames[512] == 4096 + 28 * 64 and frames[-1] == 2 * 4096 + 36 * 64 - 1
    assert list(band.scan_origin[:, 0]) == [0, 0, 0]
    edge, lo0, hi0, _ = band_problem(prob, 0, 2)        # windows overhanging the top edge
    assert (lo0, hi0) == (0, 28) and list(edge.scan_origin[:, 0]) == [-12, -12, -12]


def test_band_intensities_equal_whole_workload_c2():
    cfg = get_config("c2_forward")
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    band, lo, hi, frames = band_problem(prob, 5, 8)
    got = O.model_intensity(f["u"][..., lo:hi, :], f["chi"][:, lo:hi], f["alpha"], f["probe"], band)
    ref = O.model_intensity(f["u"], f["chi"], f["alpha"], f["probe"], prob, frames=frames)
    for a, b in zip(got, ref):
        np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12 * b.max())


def test_band_sums_equal_whole_workload_c2():
    name = "c2_forward"
    cfg = get_config(name)
    prob = make_problem(cfg)
    f = make_fields(cfg, prob)
    whole = oracle_whole(name, rows_per_band=3, n_workers=4)
    u = (f["u"] + f["delta"]).astype(np.float32)
    ref = O.loss_grad(u, f["chi"], f["alpha"], f["probe"], whole["y"], prob)
    assert whole["loss"] == pytest.approx(ref["loss"], rel=1e-12)
    np.testing.assert_allclose(whole["frame_loss"], ref["frame_loss"], rtol=1e-12)
    for k in ("grad_u", "grad_chi", "grad_alpha"):
        np.testing.assert_allclose(whole[k], ref[k], rtol=1e-9, atol=1e-10 * np.abs(ref[k]).max())
    # the counts are the seeded Poisson draws of the oracle's own intensities
    fid = 300
    inten = O.model_intensity(f["u"], f["chi"], f["alpha"], f["probe"], prob, frames=[fid])[0]
    draw = np.random.default_rng([cfg["seed"], fid]).poisson(np.clip(inten, 0, None)).astype(np.float32)
    tab = O.tables(prob)
    m, j, d = int(tab["peak_of_frame"][fid]), int(tab["local_index"][fid]), int(prob.det[0])
    s = int(tab["y_off"][m]) + j * d * d
    np.testing.assert_array_equal(whole["y"][s:s + d * d], draw.ravel())
