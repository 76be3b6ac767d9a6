"""Oracle image metrics, FP64 numpy: the comparison measures of Sec. 5.2.

Test infrastructure only (see the package docstring).

Readings taken here (the paper names the measures but not their formulas):
  * normalisation (Sec. 3.1.4, Sec. 4.4): each image divided by its largest
    pixel, so both lie in [0, 1];
  * RMSE (Table 3): square root of the mean over pixels of the squared
    difference of the normalised images;
  * r (Table 3): Pearson's correlation coefficient over pixels;
  * radial analysis (Table 4): the normalised image averaged over annuli one
    pixel wide around a centre (cx, cy) in pixel units (pixel (row i,
    column j) sits at (j + 0.5, i + 0.5)), out to r_max; annulus k covers
    k <= rho < k + 1;
  * the three zones are named by scattering angle (theta < 30 deg,
    30 <= theta <= 120 deg, theta > 120 deg); an image radius is mapped to an
    angle linearly, theta = 180 deg * rho / r_max at the annulus mid-radius, so
    the zone edges fall at r_max / 6 and 2 r_max / 3;
  * a zone's radial error is the RMSE of the two radial profiles over its
    non-empty annuli; the radial correlation is Pearson's r of the profiles;
  * "better" fraction (Table 4, last column): the share of non-empty annuli
    where one profile is closer to a reference profile than another.
"""
from __future__ import annotations

import math

import numpy as np


def normalise(img: np.ndarray) -> np.ndarray:
    img = np.asarray(img, dtype=np.float64)
    m = img.max()
    return img / m if m > 0 else img * 0.0


def rmse(a: np.ndarray, b: np.ndarray) -> float:
    na, nb = normalise(a), normalise(b)
    return math.sqrt(np.mean((na - nb) ** 2))


def pearson(x: np.ndarray, y: np.ndarray) -> float:
    x = np.asarray(x, dtype=np.float64).ravel()
    y = np.asarray(y, dtype=np.float64).ravel()
    dx, dy = x - x.mean(), y - y.mean()
    den = math.sqrt(np.sum(dx * dx) * np.sum(dy * dy))
    return float(np.sum(dx * dy) / den) if den > 0 else float("nan")   # undefined for a constant input


def radial_profile(img: np.ndarray, cx: float, cy: float, r_max: float):
    """(mean of the normalised image per annulus, pixel count per annulus)."""
    n = normalise(img)
    ny, nx = n.shape
    yy, xx = np.meshgrid(np.arange(ny) + 0.5, np.arange(nx) + 0.5, indexing="ij")
    dx, dy = xx - cx, yy - cy
    rho = np.sqrt(dx * dx + dy * dy)
    n_r = int(math.ceil(r_max))
    keep = rho < r_max
    k = np.floor(rho[keep]).astype(np.int64)
    count = np.bincount(k, minlength=n_r)[:n_r].astype(np.float64)
    total = np.bincount(k, weights=n[keep], minlength=n_r)[:n_r]
    prof = np.where(count > 0, total / np.maximum(count, 1.0), 0.0)
    return prof, count


def zone_of(k: np.ndarray, r_max: float) -> np.ndarray:
    """0 forward (< 30 deg), 1 intermediate, 2 edge (> 120 deg) for annulus k."""
    theta = 180.0 * (np.asarray(k, dtype=np.float64) + 0.5) / r_max
    return np.where(theta < 30.0, 0, np.where(theta <= 120.0, 1, 2))


def image_metrics(a: np.ndarray, b: np.ndarray, cx: float, cy: float, r_max: float, c=None) -> dict:
    """The measures of Tables 3 and 4 between images a and b (b the
    reference); with a third image c, also the share of annuli where a is
    closer to b than c is."""
    pa, cnt = radial_profile(a, cx, cy, r_max)
    pb, _ = radial_profile(b, cx, cy, r_max)
    used = cnt > 0
    zone = zone_of(np.arange(len(pa)), r_max)
    zerr = []
    for z in range(3):
        sel = used & (zone == z)
        zerr.append(math.sqrt(np.mean((pa[sel] - pb[sel]) ** 2)) if sel.any() else 0.0)
    out = dict(rmse=rmse(a, b), r=pearson(a, b), zone_rmse=zerr, radial_r=pearson(pa[used], pb[used]),
               n_annuli=int(len(pa)), profile_a=pa, profile_b=pb, count=cnt)
    if c is not None:
        pc, _ = radial_profile(c, cx, cy, r_max)
        out["better"] = float(np.mean(np.abs(pa[used] - pb[used]) < np.abs(pc[used] - pb[used])))
    return out
