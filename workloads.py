"""Seeded synthetic workloads shared by the oracle, the tests and the benchmark.

This module holds only input descriptions: physical parameters of the cuvette,
the particles, the beam and the detector, photon budgets and seeds.  It holds
none of the method's arithmetic (no Mie series, no sampling, no transport), so
both the oracle and the HIP path can read it without sharing any computation.

The workloads stand in for the paper's experiment (Sec. 4, Sec. 5.2): 5 um
polystyrene spheres in water, 532 nm light, optical depths of a few to ~10,
1e8-scale photon counts per image.  The cuvette is a 10 mm cube rather than the
paper's 30 x 10 x 45 mm cell; every size is a parameter.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

PHASE_MIE = 0
PHASE_HG = 1


@dataclass(frozen=True)
class Particle:
    """Sphere and host medium (Sec. 2.2, Eqs. 3-4; Sec. 2.5)."""
    diameter_um: float = 5.0
    m_re: float = 1.59           # particle index, real part
    m_im: float = 0.0            # particle index, imaginary part (>= 0 absorbs)
    n_medium: float = 1.33       # water
    wavelength_nm: float = 532.0
    sigma_ln: float = 0.0        # lognormal width of ln d (diameter_um is then the median)
    n_bins: int = 1              # Gauss-Hermite bins in ln d (1: a single size)


@dataclass(frozen=True)
class Workload:
    """One forward run of the photon walk (Sec. 3.1.3)."""
    name: str
    particle: Particle = Particle()
    tau: float = 1.0                      # optical depth along the beam (Eq. 1)
    albedo: float = 0.9999                # single-scatter albedo mu_s / mu_ext
    size_mm: tuple = (10.0, 10.0, 10.0)   # cuboid x, y, z
    n_outside: float = 1.0                # index outside the walls (air)
    src_pos_mm: tuple = (5.0, 5.0, 0.0)   # pencil beam at the z = 0 face centre
    src_dir: tuple = (0.0, 0.0, 1.0)
    beam_radius_mm: float = 0.0           # parallel beam of this radius (0: pencil)
    n_angles: int = 1801                  # 0.1 degree phase table
    n_cdf: int = 4096
    phase: int = PHASE_MIE
    side_px: int = 128                    # side image on the +x face (rows y, cols z)
    trans_px: int = 128                   # transmitted image on the +z face (rows y, cols x)
    n_photons: int = 100_000
    seed: int = 1234
    instance: int = 0
    roulette_w: float = 1e-4
    roulette_p: float = 0.1
    max_steps: int = 1 << 20

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# Plain forward, tiny: the parity workload.
TINY = Workload(name="tiny_tau1_1e5", tau=1.0, n_cdf=4096, side_px=128,
                trans_px=128, n_photons=100_000)

# Plain forward at paper scale: tau in {1, 2, 4, 8}, 1e8 photons, 16384-entry
# inverse CDF, 512 x 512 images; tau = 4 is the headline throughput workload.
PAPER_TAUS = (1.0, 2.0, 4.0, 8.0)


def paper_scale(tau: float = 4.0, phase: int = PHASE_MIE,
                n_photons: int = 100_000_000) -> Workload:
    tag = "mie" if phase == PHASE_MIE else "hg"
    return Workload(name=f"paper_tau{tau:g}_{tag}_{n_photons:.0e}", tau=tau,
                    n_cdf=16384, side_px=512, trans_px=512,
                    n_photons=n_photons, phase=phase)


HEADLINE = paper_scale(4.0)

# Differentiation workload: tau = 4, 1e7 photons per evaluation; target image
# at tau = 4.5 with seed 99.
DIFF = paper_scale(4.0, n_photons=10_000_000).replace(name="diff_tau4_1e7")
DIFF_TARGET = DIFF.replace(name="diff_target_tau4.5", tau=4.5, seed=99)


# Polydisperse heavy scattering: lognormal sizes (median 5 um, sigma_ln 0.05,
# 64 Gauss-Hermite bins), tau = 16, 1e9 photons, 1024 x 1024 images in int64
# fixed point; the oracle checks it on its first 1e6 photons.
HEAVY = Workload(name="heavy_poly_tau16_1e9", particle=Particle(sigma_ln=0.05, n_bins=64), tau=16.0,
                 n_cdf=16384, side_px=1024, trans_px=1024, n_photons=1_000_000_000)


# The paper's image comparison (Sec. 5.2): a 2.5 mm wide parallel beam (Sec.
# 4.1, radius 1.25 mm) at the optical depths of Tables 3 and 4, 512 x 512
# images of 1e8 photons per phase function; an independent Mie run (seed
# 4321) stands in for the experimental reference image.
ANALYSIS_ODS = (5.0, 7.5, 8.0, 10.0, 12.5)
ANALYSIS_REF_SEED = 4321


def analysis_workload(tau: float, phase: int = PHASE_MIE, seed: int = 1234,
                      n_photons: int = 100_000_000) -> "Workload":
    tag = "mie" if phase == PHASE_MIE else "hg"
    return Workload(name=f"analysis_od{tau:g}_{tag}_s{seed}", tau=tau, n_cdf=16384, side_px=512,
                    trans_px=512, n_photons=n_photons, phase=phase, seed=seed, beam_radius_mm=1.25)


@dataclass(frozen=True)
class BatchInstance:
    diameter_um: float
    tau: float
    albedo: float
    n_photons: int


def batch_instances(n: int = 256, seed: int = 2507) -> List[BatchInstance]:
    """Batched media: d log-uniform 0.5-10 um, tau ~ U(0.5, 10),
    albedo ~ U(0.95, 1), photons log-uniform 1e5-1e7 (numpy PCG64 seed 2507)."""
    rng = np.random.default_rng(seed)
    d = np.exp(rng.uniform(np.log(0.5), np.log(10.0), n))
    tau = rng.uniform(0.5, 10.0, n)
    alb = rng.uniform(0.95, 1.0, n)
    nph = np.exp(rng.uniform(np.log(1e5), np.log(1e7), n)).astype(np.int64)
    return [BatchInstance(float(a), float(b), float(c), int(e))
            for a, b, c, e in zip(d, tau, alb, nph)]


# Batched media share the cuvette and beam of the parity workload, with
# 4096-entry tables and their own 256 x 256 lateral (and transmitted) images;
# instance i draws Philox counter word 1 = i.
BATCH_BASE = Workload(name="batch", tau=1.0, n_cdf=4096, side_px=256, trans_px=256, n_photons=0)


def batch_workloads(n: int = 256, seed: int = 2507, photon_scale: float = 1.0) -> List[Workload]:
    """One Workload per batched medium (batch_instances), photon counts scaled
    by photon_scale (at least one photon each)."""
    out = []
    for i, b in enumerate(batch_instances(n, seed)):
        part = dataclasses.replace(BATCH_BASE.particle, diameter_um=b.diameter_um)
        out.append(BATCH_BASE.replace(name=f"batch{n}_{i}", particle=part, tau=b.tau, albedo=b.albedo,
                                      n_photons=max(1, int(round(b.n_photons * photon_scale))), instance=i))
    return out


def sample_ids(n_total: int, n_sample: int, seed: int = 7) -> np.ndarray:
    """Sorted distinct photon ids spread over [0, n_total) for sampled parity
    at full size (numpy PCG64)."""
    rng = np.random.default_rng(seed)
    n_sample = min(n_sample, n_total)
    ids = rng.choice(n_total, size=n_sample, replace=False)
    return np.sort(ids.astype(np.uint64))
