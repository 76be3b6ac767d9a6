"""MI355X-native Monte Carlo / rigorous-Mie photon walk (arXiv 2507.23189).

The computation lives in libmcmie.so (hand-written HIP for gfx950, C ABI in
include/mcmie.h); this package only marshals arguments to it.  Importing the
package does not load the library; the first call does, and raises if it has
not been built.
"""
from ._capi import (MC_ACCUMULATE, MC_EDEVICE, MC_EINVAL, MC_ENOMEM, MC_EUNSUPPORTED, MC_FIX64, MC_MAX_N_ANGLES, MC_MOMENTS,
                    MC_MOMENTS_PIXEL2, MC_EXIT_LOG, MC_S_SIDE_W2, MC_S_SIDE_W2K, MC_S_SIDE_W2L, MC_S_FACE,
                    MC_S_ABSORBED, MC_S_ROULETTE_NET, MC_S_CAPPED_W, MC_S_EVENTS, MC_S_PHOTONS, MC_S_ROULETTE_KILLS,
                    MC_S_CAPPED, MC_S_REFLECTIONS, MC_S_STEPS,
                    MC_MAX_N_CDF, MC_MAX_TERMS, MC_N_SCALARS, MC_OK, MC_PHASE_HG, MC_PHASE_MIE, MC_RECORD,
                    MC_SIGMA, Detector, Geometry, McError, Medium, MieSpec, MieTable, Run, Source, Tally, lib,
                    mc_grad, mc_philox_blocks, mc_simulate, mc_version, mc_workspace_bytes, mie_table_build,
                    mc_workspace_bytes_log,
                    BatchItem, MC_MAX_BATCH, AUTOTUNE_BLOCKS, AUTOTUNE_CHUNKS, mc_simulate_batch,
                    mc_autotune_batch, mc_workspace_bytes_batch, mc_workspace_bytes_batch_log, MiePoly, MC_MAX_BINS, mie_table_build_poly,
                    mc_lognormal_bins, Radial, MC_METRICS_N, MC_MAX_ANNULI, image_metrics,
                    mie_table_enqueue, MC_MEDIUM_TAU, MC_MEDIUM_MU, MC_MEDIUM_CONCENTRATION,
                    mc_medium_coefficients, mc_simulate_noalloc, MC_NOALLOC_SCRATCH_BYTES)
from .args import args_from_workload, batch_item, table_for_workload
from .autograd import SideImage, side_image, side_l2_loss

__all__ = [n for n in dir() if not n.startswith("_")]
