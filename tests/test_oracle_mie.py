"""Pins of the oracle's Mie module against mathematics the paper fixes.

Each test checks the oracle against something other than itself: a 50-digit
evaluation of Eqs. 7-8 with spherical Bessel functions (the paper's own
multi-precision tool, Sec. 3.1.2), the Rayleigh limit, the optical theorem,
energy conservation for a real index, Eq. 10's normalisation against the
series Q_sca, Eq. 12 by quadrature against the series g, and the printed
numbers of Sec. 2.5 / Table 2 as loose bounds.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import mie

# ---------------------------------------------------------------- helpers


def _mp_coefficients(n, x, m, dps=50):
    """a_n, b_n straight from Eqs. 7-8 with psi_n(z) = z j_n(z) and
    xi_n(x) = x h_n^(1)(x), evaluated with mpmath at `dps` digits."""
    with mp.workdps(dps):
        x = mp.mpf(x)
        m = mp.mpc(m.real, m.imag)
        mx = m * x

        def j(k, z):
            return mp.sqrt(mp.pi / (2 * z)) * mp.besselj(k + mp.mpf(1) / 2, z)

        def y(k, z):
            return mp.sqrt(mp.pi / (2 * z)) * mp.bessely(k + mp.mpf(1) / 2, z)

        def psi(z, k):
            return z * j(k, z)

        def dpsi(z, k):              # d/dz [z j_k(z)] = z j_{k-1}(z) - k j_k(z)
            return z * j(k - 1, z) - k * j(k, z)

        def h(k):
            return j(k, x) + mp.mpc(0, 1) * y(k, x)

        xi = x * h(n)
        dxi = x * h(n - 1) - n * h(n)
        a = (m * psi(mx, n) * dpsi(x, n) - psi(x, n) * dpsi(mx, n)) / \
            (m * psi(mx, n) * dxi - xi * dpsi(mx, n))
        b = (psi(mx, n) * dpsi(x, n) - m * psi(x, n) * dpsi(mx, n)) / \
            (psi(mx, n) * dxi - m * xi * dpsi(mx, n))
        return complex(a), complex(b)


# --------------------------------------------------------------- the pins

X_C1 = math.pi * 5.0 * 1.33 / 0.532       # 5 um polystyrene in water at 532 nm


@pytest.mark.parametrize("x", [0.1, 1.0, 10.0, X_C1, 79.0])
@pytest.mark.parametrize("m", [1.59 / 1.33, 1.5 + 0j, 1.2 + 0.01j])
def test_coefficients_match_50_digit_bessel(x, m):
    a, b = mie.mie_coefficients(x, complex(m))
    ref = np.array([_mp_coefficients(n, x, complex(m)) for n in range(1, len(a) + 1)])
    big = np.max(np.abs(ref))
    err = np.max(np.abs(np.stack([a, b], axis=1) - ref))
    assert err <= 1e-12 * big, (x, m, err, big)
    # Every coefficient above 1e-3 of the largest is good to 1e-8 relative.
    sig = np.abs(ref) > 1e-3 * big
    rel = np.abs(np.stack([a, b], axis=1) - ref)[sig] / np.abs(ref)[sig]
    assert rel.max() <= 1e-8


def test_size_parameter_uses_medium_wavelength():
    # Eq. 3 with lambda = lambda0 / n_med: 5 um spheres in water at 532 nm.
    assert mie.size_parameter(5.0, 532.0, 1.33) == pytest.approx(39.26990816987241, rel=1e-15)
    assert mie.relative_index(1.59, 0.0, 1.33) == pytest.approx(1.59 / 1.33)


@pytest.mark.parametrize("m", [1.5 + 0j, 1.33 + 0.05j])
def test_rayleigh_limit(m):
    # x -> 0: Q_sca -> (8/3) x^4 |(m^2-1)/(m^2+2)|^2, Q_abs -> 4 x Im((m^2-1)/(m^2+2)).
    x = 0.01
    a, b = mie.mie_coefficients(x, m)
    q_ext, q_sca, q_abs, g = mie.efficiencies(x, a, b)
    K = (m * m - 1) / (m * m + 2)
    assert q_sca == pytest.approx(8.0 / 3.0 * x**4 * abs(K) ** 2, rel=1e-3)
    if m.imag > 0:
        assert q_abs == pytest.approx(4 * x * K.imag, rel=1e-3)
    assert abs(g) < 1e-3          # Rayleigh scattering is symmetric fore/aft


def test_rayleigh_phase_shape():
    # x -> 0: the normalised phase function tends to (3/4)(1 + cos^2 theta).
    x, m = 0.01, 1.5 + 0j
    a, b = mie.mie_coefficients(x, m)
    _, q_sca, _, _ = mie.efficiencies(x, a, b)
    th = np.linspace(0, math.pi, 37)
    P = mie.phase_function(th, x, a, b, q_sca)
    np.testing.assert_allclose(P, 0.75 * (1 + np.cos(th) ** 2), rtol=2e-4)


@pytest.mark.parametrize("x", [0.5, 5.0, X_C1, 79.0])
@pytest.mark.parametrize("m", [1.59 / 1.33 + 0j, 1.2 + 0.01j])
def test_optical_theorem(x, m):
    # Q_ext = (4 / x^2) Re S(0), with S(0) = S1(0) = S2(0) from Eqs. 5-6.
    a, b = mie.mie_coefficients(x, m)
    q_ext, *_ = mie.efficiencies(x, a, b)
    S1, S2 = mie.amplitudes(np.array([0.0]), a, b)
    assert S1[0] == pytest.approx(S2[0], rel=1e-13)
    assert q_ext == pytest.approx(4.0 / x**2 * S1[0].real, rel=1e-12)


@pytest.mark.parametrize("x", [1.0, X_C1, 79.0])
def test_real_index_conserves_energy(x):
    # For real m no energy is absorbed: Re a_n = |a_n|^2 and Re b_n = |b_n|^2.
    a, b = mie.mie_coefficients(x, 1.59 / 1.33 + 0j)
    np.testing.assert_allclose(a.real, np.abs(a) ** 2, atol=1e-14)
    np.testing.assert_allclose(b.real, np.abs(b) ** 2, atol=1e-14)
    q_ext, q_sca, q_abs, _ = mie.efficiencies(x, a, b)
    assert abs(q_abs) <= 1e-13 * q_ext


@pytest.mark.parametrize("x,m", [(3.0, 1.5 + 0j), (X_C1, 1.59 / 1.33 + 0j), (20.0, 1.33 + 0.01j)])
def test_normalisation_eq10_and_g_eq12_by_quadrature(x, m):
    # (1/x^2) int (|S1|^2 + |S2|^2) sin(theta) dtheta = Q_sca (series), i.e.
    # Eq. 10 holds for the normalised P; and Eq. 12 by quadrature = series g.
    a, b = mie.mie_coefficients(x, m)
    q_ext, q_sca, q_abs, g = mie.efficiencies(x, a, b)
    th = np.linspace(0.0, math.pi, 40001)
    S1, S2 = mie.amplitudes(th, a, b)
    f = (np.abs(S1) ** 2 + np.abs(S2) ** 2) * np.sin(th)
    from scipy.integrate import simpson
    assert simpson(f, x=th) / x**2 == pytest.approx(q_sca, rel=1e-7)
    P = mie.phase_function(th, x, a, b, q_sca)
    assert 0.5 * simpson(P * np.sin(th), x=th) == pytest.approx(1.0, rel=1e-7)   # Eq. 10
    g_quad = 0.5 * simpson(P * np.cos(th) * np.sin(th), x=th)                    # Eq. 12
    assert g_quad == pytest.approx(g, abs=1e-7)


def test_large_sphere_extinction_tends_to_two():
    # Extinction paradox: Q_ext -> 2 as x -> infinity (within the ripple).
    a, b = mie.mie_coefficients(1000.0, 1.2 + 0.001j)
    q_ext, *_ = mie.efficiencies(1000.0, a, b)
    assert abs(q_ext - 2.0) < 0.05


def test_printed_paper_values_loosely():
    """Sec. 2.5 prints Q_ext = 2.25 and sigma_e = 4.42e-5 mm^2; Table 2 prints
    g = 0.8722 for 5 um polystyrene (1.594 - 0.00033i) in water (1.333) at
    532 nm.  They do not reproduce exactly under any size convention, so they
    are loose bounds (20 % on Q_ext, 0.03 on g); Eq. 14's unit conversion is
    checked exactly."""
    lines = open(__file__.replace("test_oracle_mie.py", "golden/paper_mie_values.txt")).read().split("\n")
    vals = dict(l.split("=")[0:2] for l in lines if l and not l.startswith("#"))
    q_paper = float(vals["q_ext"])
    g_paper = float(vals["g"])
    sig_paper = float(vals["sigma_e_mm2"])
    t = mie.build_table(5.0, 1.594, 0.00033, 1.333, 532.0, n_angles=1801, n_cdf=64)
    assert abs(t.q_ext - q_paper) / q_paper < 0.2
    assert abs(t.g - g_paper) < 0.03
    assert t.q_abs > 0                      # the printed index absorbs a little
    # Eq. 14: sigma = Q pi d^2 / 4, micrometres squared to mm^2.
    assert q_paper * math.pi * (5e-3) ** 2 / 4 == pytest.approx(sig_paper, rel=2e-3)


@pytest.mark.parametrize("diameter_um", [532e-3 / (math.pi * 1.33), 5.0, 10.0, 120.0])   # x = 1, 39.27, 78.5, 942
def test_series_truncation_has_converged(diameter_um):
    """The truncation N = round(x + 4 x^(1/3) + 2) drops only negligible terms:
    twenty more terms change Q_ext, Q_sca and g by less than 1e-12 (relative
    for the efficiencies).  Dropping the x^(1/3) term, for instance, changes
    them by 2e-9 at x = 1 and by 0.06 at x = 39.27."""
    x = mie.size_parameter(diameter_um, 532.0, 1.33)
    m = mie.relative_index(1.59, 0.0, 1.33)
    N = mie.n_terms(x)
    q_ext, q_sca, _, g = mie.efficiencies(x, *mie.mie_coefficients(x, m))
    q_ext2, q_sca2, _, g2 = mie.efficiencies(x, *mie.mie_coefficients(x, m, N + 20))
    assert abs(q_ext - q_ext2) <= 1e-12 * q_ext2
    assert abs(q_sca - q_sca2) <= 1e-12 * q_sca2
    assert abs(g - g2) <= 1e-12
