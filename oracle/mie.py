"""Oracle Mie theory and phase-function tables, FP64 numpy.

Test infrastructure only (see the package docstring).  Every function follows
the passage cited in its docstring; the steps are kept in the paper's order and
notation so they can be checked against it by eye.

Readings of the paper taken here (each is listed with its reason in the design
notes of the repository):
  * size parameter uses the wavelength in the medium, x = pi d n_med / lambda0
    (Eq. 3 together with the medium wavenumber under Eq. 9);
  * the particle index enters relative to the medium, m = (n + ik) / n_med,
    with k >= 0 absorbing (Eq. 4, Bohren-Huffman time convention);
  * series truncation N = round(x + 4 x^(1/3) + 2) (Wiscombe's criterion; the
    paper is silent);
  * the phase function is tabulated at n_angles equally spaced angles over
    [0, pi] inclusive, the CDF is the trapezoid rule in theta of P sin(theta),
    and the inverse table holds v = 1 - cos(theta) at u_i = i / (N_cdf - 1)
    by linear interpolation of theta against the CDF (Sec. 2.6, Sec. 3.1.2).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def size_parameter(diameter_um: float, wavelength_nm: float, n_medium: float) -> float:
    """Eq. 3, x = pi d / lambda, with lambda the wavelength inside the medium."""
    lam_medium_um = wavelength_nm * 1e-3 / n_medium
    return math.pi * diameter_um / lam_medium_um


def relative_index(m_re: float, m_im: float, n_medium: float) -> complex:
    """Eq. 4, m = n + ik, taken relative to the host medium."""
    return complex(m_re, m_im) / n_medium


def n_terms(x: float) -> int:
    """Number of series terms (Wiscombe 1980 criterion)."""
    return int(round(x + 4.0 * x ** (1.0 / 3.0) + 2.0))


def mie_coefficients(x: float, m: complex, n_max: int | None = None):
    """a_n, b_n for n = 1..N (Eqs. 7-8), by the Bohren-Huffman recurrence (Sec. 2.5).

    N is n_terms(x) unless n_max is given (used to check that the terms the
    truncation drops are negligible).

    D_n(mx) = psi_n'(mx)/psi_n(mx) by downward recurrence from D = 0 at
    n_start = ceil(max(N, |mx|)) + 16 + ceil(8 |mx|^(1/3)) (the start error
    decays slowly across the turning point n ~ |mx|, whose width grows like
    |mx|^(1/3); a margin of 16 alone leaves errors up to 1e-4 at x ~ 40,
    m = 1.5); psi_n(x) and chi_n(x) by upward
    recurrence from psi_-1 = cos x, psi_0 = sin x, chi_-1 = -sin x,
    chi_0 = cos x; xi_n = psi_n - i chi_n.  Eqs. 7-8 divided through by
    psi_n(mx) give
      a_n = [(D_n/m + n/x) psi_n - psi_{n-1}] / [(D_n/m + n/x) xi_n - xi_{n-1}]
      b_n = [(m D_n + n/x) psi_n - psi_{n-1}] / [(m D_n + n/x) xi_n - xi_{n-1}]
    """
    N = n_terms(x) if n_max is None else int(n_max)
    mx = m * x
    n_start = int(math.ceil(max(N, abs(mx)))) + 16 + int(math.ceil(8.0 * abs(mx) ** (1.0 / 3.0)))
    D = np.zeros(n_start + 1, dtype=np.complex128)
    for n in range(n_start, 0, -1):
        D[n - 1] = n / mx - 1.0 / (D[n] + n / mx)

    psi_prev, psi_cur = math.cos(x), math.sin(x)      # psi_{-1}, psi_0
    chi_prev, chi_cur = -math.sin(x), math.cos(x)     # chi_{-1}, chi_0
    a = np.zeros(N, dtype=np.complex128)
    b = np.zeros(N, dtype=np.complex128)
    for n in range(1, N + 1):
        psi_n = (2 * n - 1) / x * psi_cur - psi_prev
        chi_n = (2 * n - 1) / x * chi_cur - chi_prev
        xi_n = complex(psi_n, -chi_n)
        xi_nm1 = complex(psi_cur, -chi_cur)
        da = D[n] / m + n / x
        db = m * D[n] + n / x
        a[n - 1] = (da * psi_n - psi_cur) / (da * xi_n - xi_nm1)
        b[n - 1] = (db * psi_n - psi_cur) / (db * xi_n - xi_nm1)
        psi_prev, psi_cur = psi_cur, psi_n
        chi_prev, chi_cur = chi_cur, chi_n
    return a, b


def efficiencies(x: float, a: np.ndarray, b: np.ndarray):
    """Q_ext (Eq. 13), Q_sca, Q_abs = Q_ext - Q_sca and the asymmetry g.

    g is Eq. 12 evaluated in closed form over the series (Bohren-Huffman 4.62):
      g Q_sca = (4/x^2) [ sum n(n+2)/(n+1) Re(a_n a*_{n+1} + b_n b*_{n+1})
                          + sum (2n+1)/(n(n+1)) Re(a_n b*_n) ]
    """
    N = len(a)
    n = np.arange(1, N + 1, dtype=np.float64)
    q_ext = 2.0 / x**2 * np.sum((2 * n + 1) * (a + b).real)
    q_sca = 2.0 / x**2 * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2))
    nn = n[:-1]
    t1 = np.sum(nn * (nn + 2) / (nn + 1) * (a[:-1] * np.conj(a[1:]) + b[:-1] * np.conj(b[1:])).real)
    t2 = np.sum((2 * n + 1) / (n * (n + 1)) * (a * np.conj(b)).real)
    g = 4.0 / (x**2 * q_sca) * (t1 + t2)
    return float(q_ext), float(q_sca), float(q_ext - q_sca), float(g)


def angular_functions(mu: np.ndarray, N: int):
    """pi_n(mu), tau_n(mu) for n = 1..N (Eqs. 5-6), by upward recurrence:
    pi_0 = 0, pi_1 = 1, pi_n = (2n-1)/(n-1) mu pi_{n-1} - n/(n-1) pi_{n-2},
    tau_n = n mu pi_n - (n+1) pi_{n-1}.  Returns arrays of shape (N, len(mu))."""
    mu = np.asarray(mu, dtype=np.float64)
    pi = np.zeros((N + 1, mu.size))
    tau = np.zeros((N + 1, mu.size))
    pi[1] = 1.0
    tau[1] = mu
    for n in range(2, N + 1):
        pi[n] = (2 * n - 1) / (n - 1) * mu * pi[n - 1] - n / (n - 1) * pi[n - 2]
        tau[n] = n * mu * pi[n] - (n + 1) * pi[n - 1]
    return pi[1:], tau[1:]


def amplitudes(theta: np.ndarray, a: np.ndarray, b: np.ndarray):
    """S1(theta), S2(theta), Eqs. 5-6."""
    N = len(a)
    pi, tau = angular_functions(np.cos(theta), N)
    n = np.arange(1, N + 1, dtype=np.float64)
    c = ((2 * n + 1) / (n * (n + 1)))[:, None]
    S1 = np.sum(c * (a[:, None] * pi + b[:, None] * tau), axis=0)
    S2 = np.sum(c * (a[:, None] * tau + b[:, None] * pi), axis=0)
    return S1, S2


def phase_function(theta: np.ndarray, x: float, a, b, q_sca: float) -> np.ndarray:
    """Eq. 9 normalised by Eq. 10: (1/4pi) int P dOmega = 1.

    With k the medium wavenumber, (1/k^2) int (|S1|^2+|S2|^2)/2 dOmega is the
    scattering cross-section pi x^2 Q_sca / k^2, so the normalised phase
    function is P = 2 (|S1|^2 + |S2|^2) / (x^2 Q_sca)."""
    S1, S2 = amplitudes(theta, a, b)
    return 2.0 * (np.abs(S1) ** 2 + np.abs(S2) ** 2) / (x**2 * q_sca)


def angle_grid(n_angles: int) -> np.ndarray:
    """n_angles equally spaced scattering angles over [0, pi], ends included."""
    return np.arange(n_angles, dtype=np.float64) * (math.pi / (n_angles - 1))


def cdf_in_theta(theta: np.ndarray, P: np.ndarray) -> np.ndarray:
    """Cumulative distribution of the scattering angle (Sec. 2.6):
    F_j = trapezoid integral of P sin(theta) from 0 to theta_j, scaled so the
    last entry is 1."""
    f = P * np.sin(theta)
    F = np.zeros_like(theta)
    for j in range(1, len(theta)):
        F[j] = F[j - 1] + 0.5 * (theta[j] - theta[j - 1]) * (f[j - 1] + f[j])
    return F / F[-1]


def inverse_table(theta: np.ndarray, F: np.ndarray, n_cdf: int) -> np.ndarray:
    """Inverse CDF sampled at u_i = i/(n_cdf-1) (Sec. 2.6, Sec. 3.1.2).

    For each u the first grid index j with F_j >= u is found by binary search;
    theta(u) interpolates linearly between theta_{j-1} and theta_j; the table
    stores v = 1 - cos(theta(u)), evaluated as 2 sin^2(theta/2), the same
    quantity without the cancellation of 1 - cos at small angles (at
    x ~ 940 the first entries have theta ~ 1e-6, where 1 - cos(theta) in
    FP64 keeps three significant digits)."""
    v = np.zeros(n_cdf)
    for i in range(n_cdf):
        u = i / (n_cdf - 1)
        j = int(np.searchsorted(F, u, side="left"))    # first j with F_j >= u
        if j == 0:
            th = theta[0]
        else:
            th = theta[j - 1] + (u - F[j - 1]) / (F[j] - F[j - 1]) * (theta[j] - theta[j - 1])
        v[i] = 2.0 * math.sin(0.5 * th) ** 2
    return v


def sample_table(v_table: np.ndarray, u) -> np.ndarray:
    """Direct-index lookup of the inverse table at uniform(s) u in (0, 1):
    t = u (N-1), i = floor(t), v = T_i + (t - i)(T_{i+1} - T_i)."""
    u = np.asarray(u, dtype=np.float64)
    N = len(v_table)
    t = u * (N - 1)
    i = np.minimum(np.floor(t).astype(np.int64), N - 2)
    f = t - i
    return v_table[i] + f * (v_table[i + 1] - v_table[i])


def hg_phase(theta: np.ndarray, g: float) -> np.ndarray:
    """Eq. 11 scaled to (1/4pi) int P dOmega = 1 (i.e. 4 pi f)."""
    mu = np.cos(theta)
    return (1 - g * g) / (1 + g * g - 2 * g * mu) ** 1.5


def hg_v(u, g: float):
    """Closed-form inverse of the Henyey-Greenstein CDF in theta (Eq. 11),
    returned as v = 1 - cos(theta); u = 0 is forward, u = 1 backward.
    Inverting F(theta) = u gives, with D = 1 + g - 2 g u and t = (1 - g^2)/D,
      cos(theta) = (1 + g^2 - t^2) / (2g),
    which rearranges without cancellation to v = (1 - g) u (t + 1 - g) / D.
    At g = 0 this is v = 2u (isotropic)."""
    u = np.asarray(u, dtype=np.float64)
    D = 1.0 + g - 2.0 * g * u
    t = (1.0 - g * g) / D
    return (1.0 - g) * u * (t + 1.0 - g) / D


@dataclass
class MieTable:
    x: float
    m: complex
    a: np.ndarray
    b: np.ndarray
    q_ext: float
    q_sca: float
    q_abs: float
    g: float
    sigma_ext_mm2: float
    sigma_sca_mm2: float
    theta: np.ndarray
    P: np.ndarray
    F: np.ndarray
    v: np.ndarray          # FP64 inverse table, v = 1 - cos(theta)


def build_table(diameter_um: float, m_re: float, m_im: float, n_medium: float,
                wavelength_nm: float, n_angles: int = 1801, n_cdf: int = 4096) -> MieTable:
    """Parameter processing (Sec. 3.1.1) and the rigorous Mie module (Sec. 3.1.2):
    x, m -> a_n, b_n -> Q_ext, Q_sca, g -> P on the angle grid -> CDF ->
    inverse table.  Cross-sections sigma = Q pi d^2 / 4 (Eq. 14) in mm^2."""
    x = size_parameter(diameter_um, wavelength_nm, n_medium)
    m = relative_index(m_re, m_im, n_medium)
    a, b = mie_coefficients(x, m)
    q_ext, q_sca, q_abs, g = efficiencies(x, a, b)
    theta = angle_grid(n_angles)
    P = phase_function(theta, x, a, b, q_sca)
    F = cdf_in_theta(theta, P)
    v = inverse_table(theta, F, n_cdf)
    geo_mm2 = math.pi * (diameter_um * 1e-3) ** 2 / 4.0
    return MieTable(x, m, a, b, q_ext, q_sca, q_abs, g, q_ext * geo_mm2,
                    q_sca * geo_mm2, theta, P, F, v)


def table_from_workload(w) -> MieTable:
    p = w.particle
    return build_table(p.diameter_um, p.m_re, p.m_im, p.n_medium, p.wavelength_nm,
                       w.n_angles, w.n_cdf)
