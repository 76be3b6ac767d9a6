"""Pins of the oracle's CDF and inverse-table construction (Sec. 2.6, Sec. 3.1.2).

The same table code is fed phase functions whose inverse CDF is known in
closed form (Henyey-Greenstein, Eq. 11; isotropic), so a mistake in the
quadrature, the search or the interpolation shows as a departure from that
closed form, which must shrink as the angle grid is refined (trapezoid rule,
error ~ dtheta^2).  The Mie table is then checked against the series g.
"""
import math

import numpy as np
import pytest

from oracle import mie


@pytest.mark.parametrize("g", [0.0, 0.5, 0.8668, -0.4])
def test_hg_table_matches_closed_form_inverse(g):
    u = np.arange(4096) / 4095
    errs = []
    for na in (1801, 18001):
        th = mie.angle_grid(na)
        F = mie.cdf_in_theta(th, mie.hg_phase(th, g))
        v = mie.inverse_table(th, F, 4096)
        errs.append(np.abs(v - mie.hg_v(u, g)).max())
    assert errs[0] < 2e-5
    assert errs[1] < errs[0] / 50            # second-order convergence


@pytest.mark.parametrize("g", [0.0, 0.3, 0.8668, -0.5])
def test_hg_inverse_is_the_integral_of_eq11(g):
    # The HG CDF in cos(theta) from -1, by integrating Eq. 11:
    #   G(mu) = (1 - g^2)/(2g) [ (1 + g^2 - 2 g mu)^(-1/2) - 1/(1 + g) ]  (g != 0)
    # and F(theta) = 1 - G(cos theta).  hg_v must invert it.
    u = np.linspace(0.001, 0.999, 999)
    mu = 1.0 - mie.hg_v(u, g)
    if g == 0.0:
        G = (mu + 1.0) / 2.0
    else:
        G = (1 - g * g) / (2 * g) * ((1 + g * g - 2 * g * mu) ** -0.5 - 1.0 / (1 + g))
    np.testing.assert_allclose(1.0 - G, u, atol=1e-12)
    # Mean cosine of HG is g (Eq. 12 for Eq. 11), midpoint rule over u.
    uu = (np.arange(1 << 20) + 0.5) / (1 << 20)
    assert (1.0 - mie.hg_v(uu, g)).mean() == pytest.approx(g, abs=1e-9)


def test_isotropic_table_is_linear_in_cosine():
    th = mie.angle_grid(1801)
    F = mie.cdf_in_theta(th, np.ones_like(th))
    v = mie.inverse_table(th, F, 1024)
    np.testing.assert_allclose(v, 2.0 * np.arange(1024) / 1023, atol=1e-6)


@pytest.mark.parametrize("n_cdf", [4096, 16384])
def test_mie_table_shape_and_mean(n_cdf):
    t = mie.build_table(5.0, 1.59, 0.0, 1.33, 532.0, n_angles=1801, n_cdf=n_cdf)
    assert t.F[0] == 0.0 and t.F[-1] == 1.0
    assert np.all(np.diff(t.F) >= 0)
    assert t.v[0] == 0.0 and t.v[-1] == pytest.approx(2.0, abs=1e-15)
    assert np.all(np.diff(t.v) >= 0)
    # Sampled mean cosine equals the series g up to the table's quadrature error.
    u = (np.arange(1 << 20) + 0.5) / (1 << 20)
    assert 1.0 - mie.sample_table(t.v, u).mean() == pytest.approx(t.g, abs=5e-5)


def test_sampler_index_stays_in_table_at_largest_uniform():
    v = np.linspace(0, 2, 16384)
    u_max = 1.0 - 2.0 ** -24                 # largest uniform the walk can draw
    assert mie.sample_table(v, u_max) == pytest.approx(2.0 * u_max, rel=1e-12)
    assert mie.sample_table(v, 2.0 ** -24) == pytest.approx(2.0 * 2.0 ** -24, rel=1e-9)
