"""Oracle polydisperse Mie table, FP64 numpy.

Test infrastructure only (see the package docstring).

A lognormal size distribution of sphere diameters (median d_med, width
sigma_ln of ln d) replaces the single diameter of the rigorous Mie module
(Sec. 3.1.2).  Readings taken here, none of them fixed by the paper, which
simulates one diameter and discusses size only qualitatively:
  * the distribution is a number distribution, ln d ~ Normal(ln d_med, sigma_ln^2);
  * it is discretised by Gauss-Hermite quadrature in ln d: with nodes t_k and
    weights W_k for the weight function exp(-t^2), the bins are
    d_k = d_med exp(sqrt(2) sigma_ln t_k) with probabilities p_k = W_k / sqrt(pi);
  * the medium's cross-sections are the number averages
    sigma = sum_k p_k Q_k pi d_k^2 / 4 (Eq. 14 per bin), and the phase function
    is the scattering-weighted mixture
    P(theta) = sum_k p_k C_sca,k P_k(theta) / sum_k p_k C_sca,k,
    each P_k normalised as Eq. 10, so P keeps that normalisation;
  * the asymmetry parameter is the same mixture of the per-bin g_k (Eq. 12);
  * the CDF and the inverse table are built from P exactly as for one size.
The Gauss-Hermite nodes and weights come from numpy's library routine; the
tests pin them to the closed-form lognormal moments.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import mie


def lognormal_bins(median_um: float, sigma_ln: float, n_bins: int):
    """Diameters d_k (um) and probabilities p_k of the Gauss-Hermite
    discretisation of ln d ~ Normal(ln median, sigma_ln^2)."""
    t, W = np.polynomial.hermite.hermgauss(n_bins)
    d = median_um * np.exp(math.sqrt(2.0) * sigma_ln * t)
    p = W / math.sqrt(math.pi)
    return d, p


@dataclass
class PolyTable:
    median_um: float
    sigma_ln: float
    diameters_um: np.ndarray
    probs: np.ndarray
    q_ext_k: np.ndarray
    q_sca_k: np.ndarray
    g_k: np.ndarray
    sigma_ext_mm2: float    # number-averaged cross-sections (mm^2)
    sigma_sca_mm2: float
    sigma_abs_mm2: float
    g: float
    x: float                # size parameter of the median diameter
    theta: np.ndarray
    P: np.ndarray
    F: np.ndarray
    v: np.ndarray           # FP64 inverse table, v = 1 - cos(theta)

    @property
    def q_ext(self) -> float:
        """Mean extinction cross-section over the median's geometric cross-section."""
        return self.sigma_ext_mm2 / (math.pi * (self.median_um * 1e-3) ** 2 / 4.0)


def build_poly_table(median_um: float, sigma_ln: float, n_bins: int, m_re: float, m_im: float,
                     n_medium: float, wavelength_nm: float, n_angles: int = 1801,
                     n_cdf: int = 4096) -> PolyTable:
    """Per bin: x_k, a_n, b_n, Q_ext,k, Q_sca,k, g_k and P_k on the angle grid
    (the single-size steps of Sec. 3.1.2); then the mixture, its trapezoid CDF
    and its inverse table."""
    d, p = lognormal_bins(median_um, sigma_ln, n_bins)
    m = mie.relative_index(m_re, m_im, n_medium)
    theta = mie.angle_grid(n_angles)
    q_ext = np.zeros(n_bins)
    q_sca = np.zeros(n_bins)
    g = np.zeros(n_bins)
    c_sca = np.zeros(n_bins)
    mix = np.zeros(n_angles)
    for k in range(n_bins):
        x = mie.size_parameter(d[k], wavelength_nm, n_medium)
        a, b = mie.mie_coefficients(x, m)
        q_ext[k], q_sca[k], _, g[k] = mie.efficiencies(x, a, b)
        geo_mm2 = math.pi * (d[k] * 1e-3) ** 2 / 4.0
        c_sca[k] = q_sca[k] * geo_mm2
        mix += p[k] * c_sca[k] * mie.phase_function(theta, x, a, b, q_sca[k])
    geo = math.pi * (d * 1e-3) ** 2 / 4.0
    sigma_ext = float(np.sum(p * q_ext * geo))
    sigma_sca = float(np.sum(p * c_sca))
    P = mix / sigma_sca
    F = mie.cdf_in_theta(theta, P)
    v = mie.inverse_table(theta, F, n_cdf)
    g_mix = float(np.sum(p * c_sca * g) / sigma_sca)
    x_med = mie.size_parameter(median_um, wavelength_nm, n_medium)
    return PolyTable(median_um, sigma_ln, d, p, q_ext, q_sca, g, sigma_ext, sigma_sca,
                     sigma_ext - sigma_sca, g_mix, x_med, theta, P, F, v)


def poly_table_from_workload(w) -> PolyTable:
    q = w.particle
    return build_poly_table(q.diameter_um, q.sigma_ln, q.n_bins, q.m_re, q.m_im, q.n_medium,
                            q.wavelength_nm, w.n_angles, w.n_cdf)
