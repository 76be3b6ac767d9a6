"""Pins of the oracle's image metrics (oracle/metrics.py) and of the finite
beam of the oracle walk, against closed forms and special cases."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import metrics as M
from oracle import walk as owalk


def _blob(n=96, s=20.0, cx=48.0, cy=48.0):
    yy, xx = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5, indexing="ij")
    return np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2 * s * s)) + 0.1 * np.sin(xx / 7.0) ** 2


def test_identical_and_scaled_images():
    a = _blob()
    for b in (a, 3.0 * a):
        m = M.image_metrics(a, b, 48.0, 48.0, 48.0)
        assert m["rmse"] == pytest.approx(0.0, abs=1e-15)
        assert m["r"] == pytest.approx(1.0, abs=1e-14)
        assert m["zone_rmse"] == pytest.approx([0.0, 0.0, 0.0], abs=1e-15)
        assert m["radial_r"] == pytest.approx(1.0, abs=1e-14)


def test_complement_is_perfectly_anticorrelated():
    a = M.normalise(_blob())
    a = (a - a.min()) / (a.max() - a.min())         # spans [0, 1]
    assert M.pearson(a, 1.0 - a) == pytest.approx(-1.0, abs=1e-14)
    assert M.image_metrics(a, 1.0 - a, 48, 48, 48)["r"] == pytest.approx(-1.0, abs=1e-14)


def test_rmse_closed_form():
    n = 50
    a = np.ones((n, n))
    b = np.full((n, n), 0.5)
    b[0, 0] = 1.0                                   # max 1: normalisation leaves b as is
    N = n * n
    assert M.rmse(a, b) == pytest.approx(math.sqrt((N - 1) / N * 0.25), rel=1e-15)


def test_radial_profile_bins_annuli():
    n, c, r_max = 80, 40.0, 40.0
    yy, xx = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5, indexing="ij")
    k = np.floor(np.hypot(xx - c, yy - c))
    img = k + 1.0                                    # constant on every annulus
    prof, cnt = M.radial_profile(img, c, c, r_max)
    assert len(prof) == 40 and np.all(cnt > 0)
    np.testing.assert_allclose(prof, (np.arange(40) + 1.0) / img.max(), rtol=1e-14)
    # Pixels inside radius k approach the disk's area pi k^2 (lattice-point
    # count, error O(k^(2/3))).
    assert cnt.sum() == np.count_nonzero(np.hypot(xx - c, yy - c) < r_max)
    inside = np.cumsum(cnt)
    kk = np.arange(1, 41)
    np.testing.assert_allclose(inside[9:], math.pi * kk[9:] ** 2, rtol=0.03)


def test_zone_edges_and_zone_errors():
    r_max = 60.0
    z = M.zone_of(np.arange(60), r_max)
    assert (z[:10] == 0).all() and (z[10:40] == 1).all() and (z[40:] == 2).all()
    n, c = 120, 60.0
    yy, xx = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5, indexing="ij")
    rho = np.hypot(xx - c, yy - c)
    a = np.ones((n, n))
    b = a.copy()
    b[(rho >= 20) & (rho < 30)] = 0.5                # only the intermediate zone differs
    m = M.image_metrics(a, b, c, c, r_max)
    assert m["zone_rmse"][0] == 0.0 and m["zone_rmse"][2] == 0.0
    assert m["zone_rmse"][1] == pytest.approx(0.5 * math.sqrt(10 / 30), rel=1e-14)


def test_better_fraction():
    a = _blob()
    ref = a
    worse = a + 0.05 * _blob(s=5.0)
    assert M.image_metrics(ref, ref, 48, 48, 48, c=worse)["better"] == pytest.approx(1.0)
    assert M.image_metrics(worse, ref, 48, 48, 48, c=ref)["better"] == pytest.approx(0.0)


def test_finite_beam_enters_uniformly_on_its_disk():
    """No scattering (tau ~ 0) and index-matched walls: photons leave the +z
    face where they entered, so the exits sample the beam disk: none outside
    R, a quarter inside R / 2, mean rho^2 = R^2 / 2, mean cos(phi) = 0."""
    R = 2.0
    w = W.TINY.replace(tau=1e-9, n_outside=1.33, beam_radius_mm=R, n_photons=40000)
    r = owalk.Walk(w).run(records=True)
    assert np.all(r.rec("face") == 5)
    dx, dy = r.rec("px") - 5.0, r.rec("py") - 5.0
    rho2 = dx * dx + dy * dy
    n = w.n_photons
    assert rho2.max() <= R * R * (1 + 1e-12)
    inner = np.mean(rho2 < (R / 2) ** 2)
    assert abs(inner - 0.25) <= 4 * math.sqrt(0.25 * 0.75 / n)
    # rho^2 / R^2 is uniform on [0, 1): mean 1/2, standard deviation 1/sqrt(12).
    assert abs(rho2.mean() / (R * R) - 0.5) <= 4 / math.sqrt(12 * n)
    cosphi = dx / np.sqrt(np.maximum(rho2, 1e-300))
    assert abs(cosphi.mean()) <= 4 * math.sqrt(0.5 / n)
