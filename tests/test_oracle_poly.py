"""Pins of the oracle's polydisperse Mie table (oracle/poly.py) against
closed forms, limits and an independent sampled average.

* Bins: the Gauss-Hermite discretisation must reproduce the lognormal's
  closed-form moments E[d^j] = d_med^j exp(j^2 sigma^2 / 2).
* Limit: a vanishing width gives the single-size table.
* Mixture: the scattering-weighted phase function keeps the normalisation of
  Eq. 10, and its quadrature asymmetry equals the mixture of the per-bin
  series g_k (Eq. 12).
* Sampled average: the quadrature cross-sections and mixture phase function
  agree with plain averages over diameters drawn at random from the
  distribution, within their sampling error (independent of the quadrature;
  a mixture weighted by probability alone, without C_sca, fails it).
"""
import math

import numpy as np
import pytest

from oracle import mie, poly


@pytest.mark.parametrize("sigma", [0.05, 0.3])
def test_lognormal_bins_reproduce_moments(sigma):
    d, p = poly.lognormal_bins(5.0, sigma, 64)
    assert p.sum() == pytest.approx(1.0, abs=1e-14)
    assert np.all(p > 0) and np.all(np.diff(d) > 0)
    for j in range(1, 7):
        exact = 5.0 ** j * math.exp(j * j * sigma * sigma / 2.0)
        assert np.sum(p * d ** j) == pytest.approx(exact, rel=1e-12)
    d1, p1 = poly.lognormal_bins(5.0, sigma, 1)
    assert d1[0] == pytest.approx(5.0, rel=1e-15) and p1[0] == pytest.approx(1.0, rel=1e-15)


def test_narrow_distribution_reduces_to_single_size():
    mono = mie.build_table(5.0, 1.59, 0.0, 1.33, 532.0, 1801, 4096)
    pt = poly.build_poly_table(5.0, 1e-9, 8, 1.59, 0.0, 1.33, 532.0, 1801, 4096)
    np.testing.assert_allclose(pt.P, mono.P, rtol=1e-6)
    np.testing.assert_allclose(pt.v, mono.v, rtol=1e-6, atol=1e-12)
    assert pt.g == pytest.approx(mono.g, rel=1e-8)
    assert pt.sigma_ext_mm2 == pytest.approx(mono.sigma_ext_mm2, rel=1e-8)
    assert pt.sigma_sca_mm2 == pytest.approx(mono.sigma_sca_mm2, rel=1e-8)


@pytest.fixture(scope="module")
def wide():
    # Small spheres (x ~ 7.9 at the median) with a wide distribution, so the
    # weighting matters and the sampled average stays cheap.
    return poly.build_poly_table(1.0, 0.3, 64, 1.59, 0.0, 1.33, 532.0, 1801, 4096)


def test_mixture_normalisation_and_asymmetry(wide):
    th, P = wide.theta, wide.P
    norm = 0.5 * np.trapezoid(P * np.sin(th), th)
    assert norm == pytest.approx(1.0, rel=2e-4)
    g_quad = 0.5 * np.trapezoid(P * np.cos(th) * np.sin(th), th)
    assert g_quad == pytest.approx(wide.g, abs=2e-4)
    # The mixture g lies within the per-bin range and differs from the plain
    # probability average (the weighting by C_sca matters here).
    assert wide.g_k.min() < wide.g < wide.g_k.max()
    assert abs(wide.g - np.sum(wide.probs * wide.g_k)) > 1e-3


def test_mixture_matches_sampled_average(wide):
    rng = np.random.default_rng(11)
    n = 400
    ds = 1.0 * np.exp(0.3 * rng.standard_normal(n))
    m = mie.relative_index(1.59, 0.0, 1.33)
    idx = np.arange(0, 1801, 45)
    th = wide.theta[idx]
    c_ext = np.zeros(n)
    c_sca = np.zeros(n)
    cp = np.zeros((n, len(idx)))
    for i, d in enumerate(ds):
        x = mie.size_parameter(d, 532.0, 1.33)
        a, b = mie.mie_coefficients(x, m)
        qe, qs, _, _ = mie.efficiencies(x, a, b)
        geo = math.pi * (d * 1e-3) ** 2 / 4.0
        c_ext[i], c_sca[i] = qe * geo, qs * geo
        cp[i] = c_sca[i] * mie.phase_function(th, x, a, b, qs)

    def close(q, samples):
        return abs(q - samples.mean()) <= 4.0 * samples.std(ddof=1) / math.sqrt(n)

    assert close(wide.sigma_ext_mm2, c_ext)
    assert close(wide.sigma_sca_mm2, c_sca)
    for j in range(len(idx)):
        assert close(wide.P[idx[j]] * wide.sigma_sca_mm2, cp[:, j]), j
    # The probability-only mixture misses the sampled average at some angle.
    unweighted = np.zeros(len(idx))
    for k in range(len(wide.probs)):
        x = mie.size_parameter(wide.diameters_um[k], 532.0, 1.33)
        a, b = mie.mie_coefficients(x, m)
        unweighted += wide.probs[k] * mie.phase_function(th, x, a, b, wide.q_sca_k[k])
    assert any(not close(unweighted[j] * wide.sigma_sca_mm2, cp[:, j]) for j in range(len(idx)))
