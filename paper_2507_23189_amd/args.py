"""Map a workload description (any object with the attributes used below) to
the C-ABI argument structs.  Pure marshalling: no arithmetic of the method."""
from __future__ import annotations

from ._capi import MC_MEDIUM_TAU, MC_PHASE_MIE, BatchItem, Detector, Geometry, Medium, MieSpec, Run, Source


def args_from_workload(w, table=None, *, g=None, flags=0, record_stride=1, block_size=0, grid_blocks=0,
                       n_photons=None, photon_offset=0):
    """Return (spec, medium, source, geometry, detector, run) for workload `w`.
    `table` is a MieTable from mie_table_build (MIE phase); `g` the HG
    asymmetry (defaults to the table's g)."""
    p = w.particle
    spec = MieSpec(n_medium=p.n_medium, m_re=p.m_re, m_im=p.m_im, diameter_um=p.diameter_um,
                   wavelength_nm=p.wavelength_nm, n_angles=w.n_angles, n_cdf=w.n_cdf)
    med = Medium(input=MC_MEDIUM_TAU, tau=w.tau, albedo=w.albedo, phase=w.phase,
                 n_cdf=w.n_cdf if w.phase == MC_PHASE_MIE else 0,
                 inv_cdf=(table.inv_cdf.data_ptr() if (table is not None and w.phase == MC_PHASE_MIE) else None),
                 g=(g if g is not None else (table.g if table is not None else 0.0)),
                 sigma_sca_mm2=(table.sigma_sca_mm2 if table is not None else 0.0) or 0.0,
                 sigma_abs_mm2=(table.sigma_abs_mm2 if table is not None else 0.0) or 0.0)
    src = Source()
    for i in range(3):
        src.pos_mm[i] = w.src_pos_mm[i]
        src.dir[i] = w.src_dir[i]
    src.beam_radius_mm = getattr(w, "beam_radius_mm", 0.0)
    geo = Geometry()
    for i in range(3):
        geo.size_mm[i] = w.size_mm[i]
    geo.n_medium = p.n_medium
    geo.n_outside = w.n_outside
    det = Detector(side_nx=w.side_px, side_ny=w.side_px, trans_nx=w.trans_px, trans_ny=w.trans_px, flags=flags)
    run = Run(n_photons=w.n_photons if n_photons is None else n_photons, photon_offset=photon_offset,
              seed=w.seed, instance=w.instance, max_steps=w.max_steps, roulette_w=w.roulette_w,
              roulette_p=w.roulette_p, record_stride=record_stride, block_size=block_size,
              grid_blocks=grid_blocks)
    return spec, med, src, geo, det, run


def batch_item(w, table) -> BatchItem:
    """BatchItem for workload `w` with its Mie table (from mie_table_build)."""
    return BatchItem(tau=w.tau, albedo=w.albedo, inv_cdf=table.inv_cdf.data_ptr(), n_photons=w.n_photons,
                     instance=w.instance)


def table_for_workload(w, device="cuda"):
    """The Mie table a workload asks for: single size, or the lognormal
    mixture when its particle has more than one size bin."""
    from ._capi import mie_table_build, mie_table_build_poly
    spec = args_from_workload(w)[0]
    if getattr(w.particle, "n_bins", 1) > 1:
        return mie_table_build_poly(spec, w.particle.sigma_ln, w.particle.n_bins, device)
    return mie_table_build(spec, device)
