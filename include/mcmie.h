/*
 * mcmie.h -- C ABI of the MI355X Monte Carlo / rigorous-Mie photon-walk library.
 *
 * The library implements the GPU part of the Monte Carlo - rigorous Mie
 * transport model (arXiv 2507.23189): the Mie table of Sec. 2.2-2.6 and
 * Sec. 3.1.2 and the photon walk of Sec. 3.1.3, as hand-written HIP kernels
 * for gfx950.  Every call is plain C: host structs in, caller-owned device
 * buffers, an int status out.  No exception crosses this boundary.
 *
 * Conventions
 *   Units: lengths in mm, particle diameter in um, wavelength in nm,
 *          coefficients in 1/mm (Table 2, Eq. 14).
 *   Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *          stream).  Work is enqueued on it and the call returns without
 *          waiting unless stated otherwise; the caller keeps every buffer
 *          alive until the stream has drained.
 *   Ownership: the caller allocates every buffer, including the walk's
 *          workspace (size from mc_workspace_bytes).  The library keeps no
 *          pointer after a call returns.  Its only device memory of its own
 *          is a small per-device scratch block for the table build.
 *   Tallies: weights are accumulated in 64-bit fixed point (weight * 2^32,
 *          rounded to nearest), so every sum is exact and independent of the
 *          order in which photons finish: results are bit-identical for any
 *          launch shape, and photon ranges tallied separately add up to the
 *          single run exactly (with MC_FIX64 images).
 *   Errors: functions return MC_OK (0) or a negative MC_E* code; the
 *          message of the last failure on the calling thread is returned by
 *          mc_last_error().  Arguments are validated on the host before any
 *          work is enqueued; on an error nothing is enqueued.
 */
#ifndef MCMIE_H
#define MCMIE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MC_OK 0
#define MC_EINVAL (-1)        /* an argument is out of range or inconsistent */
#define MC_EDEVICE (-2)       /* a HIP runtime call failed */
#define MC_ENOMEM (-3)        /* device scratch could not be allocated */
#define MC_EUNSUPPORTED (-4)  /* a valid request this library does not implement */

#define MC_PHASE_MIE 0        /* polar angle from the inverse-CDF table */
#define MC_PHASE_HG 1         /* polar angle from Henyey-Greenstein (Eq. 11) */

/* Detector flags (mc_detector_t.flags). */
#define MC_ACCUMULATE 1u      /* add into images and scalars instead of zeroing them first */
#define MC_SIGMA 2u           /* also tally squared weights (side_w2, trans_w2) */
#define MC_RECORD 4u          /* write per-photon end records (mc_tally_t.rec_*) */
#define MC_FIX64 8u           /* images (and squared-weight images) are int64 fixed point,
                                 value = weight * 2^32; otherwise they are double */
#define MC_MOMENTS 16u        /* also tally the path moments of the side image used by mc_grad:
                                 per pixel sum(w k) and sum(w L) (side_wk, side_wl, double), and
                                 over all side-image exits sum(w^2), sum(w^2 k), sum(w^2 L)
                                 (scalars MC_S_SIDE_W2, MC_S_SIDE_W2K, MC_S_SIDE_W2L) */
#define MC_MOMENTS_PIXEL2 32u /* with MC_MOMENTS: also per pixel sum(w^2 k) and sum(w^2 L)
                                 (side_w2k, side_w2l), for losses whose second derivative
                                 varies from pixel to pixel */
#define MC_EXIT_LOG 64u       /* gather image exits in a log in the workspace and sum them in a
                                 second pass instead of adding each to the images as it happens;
                                 the results are identical bit for bit.  The log fills the
                                 workspace beyond mc_workspace_bytes (size it with
                                 mc_workspace_bytes_log); exits that find their part of it full
                                 are added directly, so any size is correct.  Not with
                                 MC_RECORD; batched launches size it with
                                 mc_workspace_bytes_batch_log. */

/* Scalar tallies: mc_tally_t.scalars holds MC_N_SCALARS doubles. */
#define MC_S_FACE 0           /* 0..5: weight leaving faces -x, +x, -y, +y, -z, +z */
#define MC_S_ABSORBED 6       /* weight absorbed at interactions (Eq. 16) */
#define MC_S_ROULETTE_NET 7   /* sum of weight changes made by Russian roulette */
#define MC_S_CAPPED_W 8       /* weight of photons stopped by the step cap */
#define MC_S_EVENTS 9         /* scatter events (interactions) */
#define MC_S_PHOTONS 10       /* photons finished */
#define MC_S_ROULETTE_KILLS 11
#define MC_S_CAPPED 12        /* photons stopped by the step cap */
#define MC_S_REFLECTIONS 13   /* Fresnel / total internal reflections at walls */
#define MC_S_STEPS 14         /* random-number blocks drawn (walk steps) */
#define MC_S_RESERVED 15      /* reserved (written as 0) */
#define MC_S_SIDE_W2 16       /* MC_MOMENTS: sum of w^2 over photons leaving through the side image */
#define MC_S_SIDE_W2K 17      /* MC_MOMENTS: sum of w^2 k over the same photons */
#define MC_S_SIDE_W2L 18      /* MC_MOMENTS: sum of w^2 L (mm) over the same photons */
#define MC_S_RESERVED2 19     /* reserved (written as 0) */
#define MC_N_SCALARS 20

/* Per-photon record fields (structure of arrays, rec_rows rows per field). */
#define MC_REC_I_FACE 0       /* exit face 0..5, or -1 */
#define MC_REC_I_CAUSE 1      /* 0 exited, 1 roulette, 2 step cap */
#define MC_REC_I_K 2          /* scatter events */
#define MC_REC_I_STEPS 3      /* walk steps */
#define MC_REC_I_N 4
#define MC_REC_F_POS 0        /* 0..2: end position (on the face for exits) */
#define MC_REC_F_DIR 3        /* 3..5: end direction (refracted outside for exits) */
#define MC_REC_F_W 6          /* end weight (exit weight; 0 after a roulette kill) */
#define MC_REC_F_L 7          /* path length */
#define MC_REC_F_A 8          /* weight absorbed along the path */
#define MC_REC_F_N 9

#define MC_MAX_N_CDF 16384    /* largest inverse table (64 KB, held in LDS) */
#define MC_MAX_N_ANGLES 3001  /* largest phase-function grid */
#define MC_MAX_TERMS 1024     /* largest Mie series length (x up to ~980) */
#define MC_MAX_BINS 64        /* most size bins of a polydisperse table */

/* ------------------------------------------------------------------ Mie */

/* Particle, host medium and table resolution (Sec. 2.2, Eqs. 3-4; Sec. 3.1.2). */
typedef struct {
    double n_medium;       /* real index of the host medium (> 0) */
    double m_re, m_im;     /* particle index m = n + ik (Eq. 4), m_re > 0, m_im >= 0 absorbs */
    double diameter_um;    /* sphere diameter d (> 0) */
    double wavelength_nm;  /* vacuum wavelength (> 0); x = pi d n_medium / wavelength (Eq. 3) */
    int32_t n_angles;      /* phase-table angles over [0, pi], ends included, 3..MC_MAX_N_ANGLES */
    int32_t n_cdf;         /* inverse-table entries, 2..MC_MAX_N_CDF */
} mie_spec_t;

/* Results of mie_table_build.  Scalars are written on the host; the arrays
 * are caller-owned DEVICE buffers (NULL to skip an optional one). */
typedef struct {
    double x;              /* size parameter (Eq. 3) */
    double m_rel_re, m_rel_im;   /* m / n_medium */
    double q_ext, q_sca, q_abs;  /* efficiencies (Eq. 13; Q_abs = Q_ext - Q_sca) */
    double g;              /* asymmetry (Eq. 12) from the series */
    double sigma_ext_mm2, sigma_sca_mm2, sigma_abs_mm2;   /* Q pi d^2 / 4 (Eq. 14) */
    int32_t n_terms;       /* series terms used */
    int32_t n_cdf;         /* entries written to inv_cdf */
    float *inv_cdf;        /* device, n_cdf floats: v_i = 1 - cos(theta(u_i)), u_i = i/(n_cdf-1) (required) */
    double *phase;         /* device, n_angles doubles: P(theta_j), (1/4pi) int P dOmega = 1 (Eqs. 9-10), optional */
    double *cdf;           /* device, n_angles doubles: F(theta_j), trapezoid rule, F = 1 at pi, optional */
    double *coef;          /* device, 4 * coef_capacity doubles: Re a_n, Im a_n, Re b_n, Im b_n per n (Eqs. 7-8), optional */
    int32_t coef_capacity; /* terms coef can hold; must be >= n_terms when coef is set */
    double *result;        /* device, 4 doubles: Q_ext, Q_sca, g, n_terms as computed by the kernel
                              (optional for mie_table_build, required for mie_table_enqueue) */
    double *work;          /* device, n_angles doubles of scratch: P(theta_j) sin(theta_j), passed from the
                              angle-grid kernel to the CDF kernel (optional for mie_table_build, which then
                              uses library scratch; required for mie_table_enqueue) */
} mie_table_t;

/*
 * Build the Mie phase-function table on the device (Sec. 2.2-2.6, Sec. 3.1.2):
 * a_n, b_n by the Bohren-Huffman logarithmic-derivative recurrence (Sec. 2.5),
 * Q_ext/Q_sca/g (Eqs. 12-13), S1/S2 (Eqs. 5-6) and the normalised phase
 * function (Eqs. 9-10) on n_angles angles, its CDF in theta, and the inverse
 * table sampled at n_cdf equally spaced probabilities.  It runs as two FP64
 * kernels on `stream` (one lane per angle, then one lane per inverse-table
 * entry); the call then waits for the stream so the host scalars of `table`
 * are valid on return.  The device buffers of `table` must hold the sizes
 * stated above; without result or work it uses per-device library scratch,
 * held under a lock until the call returns.  Returns MC_EINVAL on a bad spec
 * (also |m| x below 1e-6) or missing buffer, MC_EDEVICE / MC_ENOMEM on
 * runtime failure.
 */
int mie_table_build(const mie_spec_t *spec, mie_table_t *table, void *stream);

/*
 * The same table build, enqueued on `stream` without waiting: the device
 * arrays and table->result are written when the stream reaches the kernels;
 * table->result and table->work are required, and work must not be shared
 * with a build running at the same time.
 * On return the host fields x, m_rel_re, m_rel_im, n_terms and n_cdf are
 * set; the efficiencies, g and cross-sections are NaN (read them from
 * table->result).  For pipelines that need the table only on the device.
 */
int mie_table_enqueue(const mie_spec_t *spec, mie_table_t *table, void *stream);

/*
 * Polydisperse table.  Diameters follow a lognormal number distribution whose
 * median is spec->diameter_um: ln d ~ Normal(ln d_med, sigma_ln^2),
 * discretised by n_bins-point Gauss-Hermite quadrature in ln d (bins
 * d_k = d_med exp(sqrt(2) sigma_ln t_k), probabilities p_k = W_k / sqrt(pi);
 * mc_lognormal_bins returns them).  Each bin runs the single-size series and
 * phase function of mie_table_build (one workgroup per bin and slice of 256
 * angles); the table is built from the scattering-weighted mixture
 *     P(theta) = sum_k p_k C_sca,k P_k(theta) / sum_k p_k C_sca,k
 * (each P_k normalised as Eq. 10, so P is too), with the number-averaged
 * cross-sections sigma = sum_k p_k Q_k pi d_k^2 / 4 (Eq. 14 per bin) and the
 * same mixture of the per-bin asymmetries (Eq. 12).  The table's q_* are
 * those cross-sections over the median's pi d_med^2 / 4, x is the median's
 * size parameter and n_terms the longest bin series; coef must be NULL and
 * table->work is not used (poly->work holds the rows, the bins' scalars and
 * the mixture's angle grid: n_bins * n_angles + 4 n_bins + n_angles doubles).
 * Waits for the stream (like mie_table_build).
 */
typedef struct {
    double sigma_ln;       /* width of ln d, >= 0 (0 with any n_bins gives the single size) */
    int32_t n_bins;        /* Gauss-Hermite bins, 1..MC_MAX_BINS */
    int32_t reserved;      /* set to 0 */
    double *work;          /* DEVICE scratch of at least mie_poly_work_bytes(spec, poly) bytes */
    uint64_t work_bytes;
} mie_poly_t;

uint64_t mie_poly_work_bytes(const mie_spec_t *spec, const mie_poly_t *poly);
int mie_table_build_poly(const mie_spec_t *spec, const mie_poly_t *poly, mie_table_t *table, void *stream);

/* Host: the bins of the lognormal discretisation above (diameters in um,
 * probabilities summing to 1), n_bins entries each. */
int mc_lognormal_bins(double median_um, double sigma_ln, int32_t n_bins, double *diameters_um, double *probs);

/* -------------------------------------------------------------- the walk */

/* How a medium's coefficients are given (mc_medium_t.input). */
#define MC_MEDIUM_TAU 0            /* optical depth along z and albedo (Eq. 1, Eq. 16) */
#define MC_MEDIUM_MU 1             /* scattering and absorption coefficients (Sec. 3.1.1) */
#define MC_MEDIUM_CONCENTRATION 2  /* particle concentration and cross-sections (Eq. 14, Eq. 17) */

/* Medium filling the cuboid.  The walk needs the extinction coefficient
 * mu_ext = mu_sca + mu_abs (free paths, Eq. 15) and the albedo
 * mu_sca / mu_ext (weight update, Eq. 16); `input` says which fields give
 * them:
 *   MC_MEDIUM_TAU            mu_ext = tau / size_z (Eq. 1, the optical depth
 *                            taken along the beam axis) and the albedo given,
 *                            or, with albedo < 0, the particles' own albedo
 *                            Q_sca / Q_ext = sigma_sca / (sigma_sca + sigma_abs);
 *   MC_MEDIUM_MU             mu_sca and mu_abs as given;
 *   MC_MEDIUM_CONCENTRATION  mu_sca = c sigma_sca and
 *                            mu_abs = c sigma_abs + mu_abs_host (Eq. 17 with
 *                            the cross-sections of Eq. 14), c in 1/mm^3.
 * mc_medium_coefficients returns the coefficients the library derives.
 * With mu_ext = 0 no photon interacts (the albedo is then taken as 1). */
typedef struct {
    int32_t input;         /* MC_MEDIUM_TAU, MC_MEDIUM_MU or MC_MEDIUM_CONCENTRATION */
    int32_t phase;         /* MC_PHASE_MIE or MC_PHASE_HG */
    double tau;            /* TAU: optical depth along z, >= 0 */
    double albedo;         /* TAU: mu_sca / mu_ext in [0, 1]; < 0: sigma_sca / (sigma_sca + sigma_abs) */
    double mu_sca, mu_abs; /* MU: coefficients in 1/mm, >= 0 */
    double concentration_per_mm3;   /* CONCENTRATION: particles per mm^3, >= 0 */
    double mu_abs_host;    /* CONCENTRATION: absorption of the host medium in 1/mm, >= 0 */
    int32_t n_cdf;         /* MIE: entries of inv_cdf, 2..MC_MAX_N_CDF */
    int32_t reserved;      /* set to 0 */
    const float *inv_cdf;  /* MIE: device inverse table as written by mie_table_build (values in [0, 2]) */
    double g;              /* HG: asymmetry in (-1, 1) */
    double sigma_sca_mm2;  /* particle cross-sections (Eq. 14, e.g. mie_table_t.sigma_sca_mm2): used by */
    double sigma_abs_mm2;  /* CONCENTRATION, by TAU with albedo < 0 and by mc_grad for the concentration
                              derivative (0 and 0 make that derivative NaN) */
} mc_medium_t;


/* Collimated beam entering the z = 0 face (Sec. 3.1.3: parallel beam, all
 * photons with the same initial direction), a pencil or a disk. */
typedef struct {
    double pos_mm[3];      /* entry point: z must be 0, x and y inside the face */
    double dir[3];         /* incident direction outside the cuboid, dir[2] > 0 (normalised here) */
    double beam_radius_mm; /* 0: pencil beam; > 0: a parallel beam whose photons enter uniformly
                              on the disk of this radius around pos_mm (Sec. 4.1), drawn from each
                              photon's Philox block at the reserved step counter 2^32 - 1 (radius
                              R sqrt(u0), azimuth 2 pi u1, a counter no step reaches); the disk must
                              lie inside the z = 0 face.  A beam whose refracted
                              direction has no x (y) component must not reach the x = size
                              (y = size) edge of the face: MC_EINVAL */
} mc_source_t;

/* Cuboid cuvette (Sec. 4.3) with one refractive-index step at every wall. */
typedef struct {
    double size_mm[3];     /* extent along x, y, z, each > 0 */
    double n_medium;       /* index inside (> 0) */
    double n_outside;      /* index outside (> 0); equal to n_medium means no Fresnel term */
} mc_geometry_t;

/*
 * Host only: the coefficients the walk takes from `medium` in `geometry`
 * (Eq. 1, Eq. 16, Eq. 17): out[0] = mu_sca, out[1] = mu_abs, out[2] = mu_ext
 * (1/mm) and out[3] = albedo, in FP64 (the walk rounds mu_ext and the albedo
 * to FP32).  MC_EINVAL for a medium mc_simulate would reject.
 */
int mc_medium_coefficients(const mc_medium_t *medium, const mc_geometry_t *geometry, double out[4]);

/* Detector images: side view on the +x face (rows y, columns z) and the
 * transmitted image on the +z face (rows y, columns x); pixel index =
 * floor(coord / size * n), clamped to n - 1 (Sec. 4.3, Sec. 5.2), evaluated
 * in FP32 as floor(coord * (n / size)) with n / size rounded once (an exit
 * exactly on a pixel edge may fall on either side of it). */
typedef struct {
    int32_t side_nx, side_ny;     /* columns (z) and rows (y) of the side image, >= 1 */
    int32_t trans_nx, trans_ny;   /* columns (x) and rows (y) of the transmitted image, >= 1 */
    uint32_t flags;               /* MC_ACCUMULATE, MC_SIGMA, MC_RECORD, MC_FIX64, MC_MOMENTS,
                                     MC_MOMENTS_PIXEL2, MC_EXIT_LOG */
} mc_detector_t;

/* Photon budget, random streams, termination and launch shape. */
typedef struct {
    uint64_t n_photons;    /* photons in this call (0 allowed: only zeroing happens);
                              n_photons * max(1, roulette_w / roulette_p) must stay below 2^31
                              so no fixed-point sum can overflow */
    uint64_t photon_offset;/* id of the first photon; ids are offset .. offset + n - 1 */
    uint64_t seed;         /* Philox4x32-10 key (seed_lo, seed_hi) */
    uint32_t instance;     /* Philox counter word 1 (independent medium instances) */
    uint32_t max_steps;    /* step cap per photon, 1..2^24 */
    double roulette_w;     /* Russian roulette below this weight (0 disables) */
    double roulette_p;     /* survival probability in (0, 1]; survivors' weight / p */
    uint64_t record_stride;/* MC_RECORD: photon offset + r * stride goes to row r (>= 1) */
    int32_t block_size;    /* threads per block, multiple of 64 in 64..1024; 0 = library choice */
    int32_t grid_blocks;   /* blocks; 0 = library choice (enough to fill every CU) */
    uint32_t chunk;        /* photons a wave claims at a time, 1..65536; 0 = library choice */
    uint32_t reserved;     /* set to 0 */
    void *walk_events[2];  /* optional hipEvent_t pair (NULL: none): set to the start and the end of
                              the walk kernel, so the caller can time that kernel alone
                              (hipEventElapsedTime); attached to the kernel's dispatch
                              (hipExtLaunchKernel), so they add no barrier between kernels */
    void *sim_events[2];   /* optional hipEvent_t pair (NULL: none): set to the start of the call's
                              first kernel and the end of its last, attached the same way, to time
                              the whole call on the device */
} mc_run_t;

/* Caller-owned DEVICE outputs and workspace. */
typedef struct {
    void *side;            /* side_ny * side_nx double (int64 with MC_FIX64), row-major (required) */
    void *trans;           /* trans_ny * trans_nx double (int64 with MC_FIX64), row-major (required) */
    void *side_w2;         /* MC_SIGMA: squared-weight image, same shape and type */
    void *trans_w2;        /* MC_SIGMA */
    double *scalars;       /* MC_N_SCALARS doubles (required) */
    int32_t *rec_i;        /* MC_RECORD: MC_REC_I_N * rec_rows int32 */
    float *rec_f;          /* MC_RECORD: MC_REC_F_N * rec_rows float */
    uint64_t rec_rows;     /* MC_RECORD: rows available (0: record nothing, buffers may be NULL) */
    void *workspace;       /* device scratch of at least mc_workspace_bytes(detector) bytes, 8-byte
                              aligned (required); its contents on entry do not matter */
    uint64_t workspace_bytes;
    double *side_wk;       /* MC_MOMENTS: side-image shape, sum over detected photons of w k */
    double *side_wl;       /* MC_MOMENTS: side-image shape, sum over detected photons of w L (mm) */
    double *side_w2k;      /* MC_MOMENTS_PIXEL2: side-image shape, sum of w^2 k */
    double *side_w2l;      /* MC_MOMENTS_PIXEL2: side-image shape, sum of w^2 L */
} mc_tally_t;

/*
 * Bytes of device workspace mc_simulate needs for this detector: per-XCD
 * fixed-point copies of the images (and of the squared-weight images with
 * MC_SIGMA) plus scalar accumulators.  0 for a NULL or invalid detector.
 */
uint64_t mc_workspace_bytes(const mc_detector_t *detector);

/*
 * Bytes of workspace for a walk of n_photons photons with MC_EXIT_LOG set in
 * detector->flags: mc_workspace_bytes plus a log in which each block of a
 * full launch (512 blocks) owns a region of the same number of 8-byte entries
 * in each of 64 key ranges, 1.5 times its share of photons in a range plus
 * 256 (about 12 bytes per photon plus 67 MB), and a count per region.  Exits
 * spread over the images normally never find their region full.  0 for a NULL
 * or invalid detector, or one without MC_EXIT_LOG.  The log is scratch: walks
 * run one after another on one stream may share a workspace.
 */
uint64_t mc_workspace_bytes_log(const mc_detector_t *detector, uint64_t n_photons);

/*
 * Run the photon walk of Sec. 3.1.3 for run->n_photons photons: start at the
 * source with the entry Fresnel loss, free paths from Eq. 15, boundary
 * determination with Fresnel reflection / refraction at the walls, polar
 * angle from the inverse CDF (Sec. 2.6) or HG (Eq. 11), uniform azimuth,
 * the weight update of Eq. 16 with Russian roulette, and atomic tallies of
 * exit positions into the detector images (Sec. 3.1.3, last paragraph).
 * Photon i draws one Philox4x32-10 block per step with counter
 * (step, instance, id_lo, id_hi) and key (seed_lo, seed_hi), so a run split
 * into photon ranges with MC_ACCUMULATE equals one run up to tally rounding.
 * Unless MC_ACCUMULATE is set the images, scalars and records are zeroed on
 * `stream` first.  Asynchronous.  Calls that share a tally buffer or a
 * workspace must not overlap in time.
 */
int mc_simulate(const mc_medium_t *medium, const mc_source_t *source, const mc_geometry_t *geometry,
                const mc_detector_t *detector, const mc_run_t *run, const mc_tally_t *tally,
                void *stream);

/*
 * mc_simulate for callers that cannot allocate device memory: code being
 * captured into a HIP graph, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments and results as mc_simulate, except that
 * tally->workspace and tally->workspace_bytes are ignored: the images are
 * tallied in one fixed-point copy (instead of eight per-XCD copies) held in a
 * device array of MC_NOALLOC_SCRATCH_BYTES that the library keeps on every
 * GPU it runs on until the process ends.  The call allocates nothing (no
 * hipMalloc, no hipFree, no allocating library routine); the caller still
 * owns the images, scalars, records and moment buffers.
 * Limits: side + transmitted pixels at most 2^21 (2^20 with MC_SIGMA), and no
 * MC_EXIT_LOG (the log needs a caller workspace): MC_EINVAL otherwise.
 * The array is cleared by the call's own fill kernel on `stream` (no memset),
 * and every call on one GPU shares it: calls that overlap in time on one GPU
 * (other streams, other threads) race and give wrong tallies.  With MC_FIX64
 * the results equal mc_simulate's bit for bit.  Asynchronous.
 */
#define MC_NOALLOC_SCRATCH_BYTES 16777472ull   /* 8 * (32 + 2^21) */
int mc_simulate_noalloc(const mc_medium_t *medium, const mc_source_t *source, const mc_geometry_t *geometry,
                        const mc_detector_t *detector, const mc_run_t *run, const mc_tally_t *tally,
                        void *stream);

/*
 * Batched launch: many media in one persistent kernel.  Every item is a
 * medium in the same cuvette, with the same source, detector and run
 * settings, the Mie phase function (its own device inverse table of n_cdf
 * entries, from mie_table_build) and its own optical depth, albedo, photon
 * count and Philox counter word.  Photon i of an item follows exactly the
 * walk mc_simulate gives it for that medium with run->instance = item.instance
 * and photon id i, so each item's tallies equal a separate mc_simulate of the
 * item (bit for bit with MC_FIX64; up to FP64 summation order otherwise).
 *
 * Work is handed out in units of run->chunk photons of one item (0: library
 * choice), items ordered by decreasing estimated cost (photons x (1 + tau))
 * so the long ones start first; each lane carries its own photon's medium, so
 * waves move from one item to the next without waiting for each other.
 * Outputs are item-major: side is n_items x side_ny x side_nx, trans and the
 * MC_SIGMA images likewise, scalars n_items x MC_N_SCALARS.  run->n_photons,
 * photon_offset, instance and record_stride are ignored.  Supported flags:
 * MC_ACCUMULATE, MC_SIGMA, MC_FIX64, MC_EXIT_LOG (MC_RECORD and MC_MOMENTS
 * give MC_EUNSUPPORTED).  n_items is 1..MC_MAX_BATCH.  Asynchronous.
 */
#define MC_MAX_BATCH 512
typedef struct {
    double tau;            /* optical depth along z (Eq. 1), >= 0 */
    double albedo;         /* mu_sca / mu_ext, in [0, 1] */
    const float *inv_cdf;  /* DEVICE inverse table of v = 1 - cos(theta) in [0, 2], n_cdf floats (Sec. 2.6) */
    uint64_t n_photons;    /* photons of this medium, ids 0 .. n_photons - 1 (0 allowed) */
    uint32_t instance;     /* Philox counter word 1 of its photons */
    uint32_t reserved;     /* set to 0 */
} mc_batch_item_t;

int mc_simulate_batch(const mc_batch_item_t *items, uint32_t n_items, int32_t n_cdf, const mc_source_t *source,
                      const mc_geometry_t *geometry, const mc_detector_t *detector, const mc_run_t *run,
                      const mc_tally_t *tally, void *stream);

/* Workspace bytes mc_simulate_batch needs for n_items media (0 if invalid). */
uint64_t mc_workspace_bytes_batch(const mc_detector_t *detector, uint32_t n_items);

/* The same with MC_EXIT_LOG in detector->flags: mc_workspace_bytes_batch plus
 * an exit log sized for total_photons photons over all items, in regions of
 * key ranges fine enough that each range holds at most 8192 of the batch's
 * keys (0 if invalid or without MC_EXIT_LOG). */
uint64_t mc_workspace_bytes_batch_log(const mc_detector_t *detector, uint32_t n_items, uint64_t total_photons);

/*
 * Launch-shape autotuner for mc_simulate_batch.  Runs the batch with every
 * item's photon count scaled by sample_fraction (in (0, 1], at least one
 * photon for a nonzero count) once for each candidate block size
 * {256, 512, 1024} and chunk {256, 512, 1024, 2048, 4096} (block-major order),
 * timing each candidate's second launch with HIP events on `stream`, and
 * writes the fastest pair to *block_size and *chunk and its time to *best_ms.
 * candidate_ms, if not NULL, receives all 15 times.  The tally buffers are
 * overwritten by the trial runs.  Waits for the stream.
 */
int mc_autotune_batch(const mc_batch_item_t *items, uint32_t n_items, int32_t n_cdf, const mc_source_t *source,
                      const mc_geometry_t *geometry, const mc_detector_t *detector, const mc_run_t *run,
                      const mc_tally_t *tally, double sample_fraction, int32_t *block_size, uint32_t *chunk,
                      double *best_ms, double *candidate_ms, void *stream);

/*
 * Perturbation Monte Carlo adjoint of a loss on the side image.  A detected
 * photon's weight, for a path with k interactions and length L sampled with
 * free paths from Eq. 15 and weighted by Eq. 16, is proportional to
 * mu_sca^k exp(-(mu_sca + mu_abs) L); its score is s = k / mu_sca - L for
 * mu_sca and s = -L for mu_abs, and dI_p = D_p = sum over the photons in pixel
 * p of w s (from the moment images M_k = sum w k, M_L = sum w L).
 *
 * Given g = dLoss/dI (device, side-image shape) and a tally filled by
 * mc_simulate with MC_MOMENTS for the same medium and geometry:
 *     G = sum_p g_p D_p                      (no second derivative)
 *     G = sum_p (g_p D_p - h_p Q_p)          (h_p = d2loss_dside2[p], device, needs MC_MOMENTS_PIXEL2)
 *     G = sum_p g_p D_p - h sum_p Q_p        (h = d2loss_uniform, d2loss_dside2 NULL)
 * with Q_p = sum w^2 s over the photons in pixel p (sum_p Q_p from the
 * MC_S_SIDE_W2K / MC_S_SIDE_W2L scalars).  The first is the exact derivative
 * of the loss of this sample with the paths held fixed; when g is computed
 * from the same sample (g = 2 (I - T) for an L2 loss, h = 2) it is biased by
 * the sample's self-correlation, and the other two remove that bias to first
 * order, estimating the gradient of Loss(E[I]).  Passing both a
 * d2loss_dside2 array and a nonzero d2loss_uniform is MC_EINVAL.
 * Writes on the host out_grad[0] = G for mu_sca, out_grad[1] = G for mu_abs,
 * out_grad[2] = sigma_sca out_grad[0] + sigma_abs out_grad[1], the derivative
 * with respect to the particle concentration c in 1/mm^3 (Eq. 17, with
 * mu_sca = c sigma_sca and mu_abs = mu_abs,medium + c sigma_abs; NaN when both
 * sigmas are 0).  The dot products run on the device in a fixed order
 * (deterministic), with the tally's workspace beyond its scalar words as
 * scratch (it holds mc_simulate's image copies, consumed by then; a walk
 * sharing that workspace must not run concurrently).  The call waits for the
 * stream.  Roulette's dependence on the weight threshold is not
 * differentiated.
 */
int mc_grad(const mc_medium_t *medium, const mc_geometry_t *geometry, const mc_detector_t *detector,
            const mc_tally_t *tally, const double *dloss_dside, const double *d2loss_dside2,
            double d2loss_uniform, double out_grad[3], void *stream);

/*
 * The random numbers the walk draws: for each of n_ids photon ids (device
 * array) and steps step0 .. step0 + n_steps - 1, write the four 32-bit
 * Philox4x32-10 words to out (device, n_ids * n_steps * 4 uint32, photon-major).
 * Exposed so the generator can be checked word for word.  Asynchronous.
 */
int mc_philox_blocks(uint64_t seed, uint32_t instance, const uint64_t *ids, uint64_t n_ids,
                     uint32_t step0, uint32_t n_steps, uint32_t *out, void *stream);

/* ------------------------------------------------------- image measures */

/*
 * Comparison measures of Sec. 5.2 (Tables 3 and 4) between two images a and
 * b (b the reference), and optionally a third c, all DEVICE row-major
 * ny x nx doubles (at most 2^24 pixels).  Each image is divided by its largest
 * pixel first.  out[] (host) receives:
 *   0 RMSE over pixels of the difference of the normalised images (Table 3)
 *   1 Pearson's r over pixels (Table 3; NaN when an image is constant)
 *   2, 3, 4  radial RMSE of the normalised images' annulus profiles in the
 *      forward (theta < 30 deg), intermediate (30..120 deg) and edge
 *      (> 120 deg) zones (Table 4), with theta = 180 deg (k + 0.5) / r_max for
 *      annulus k (k <= rho < k + 1 pixels around (cx, cy), pixel centres at
 *      (column + 0.5, row + 0.5)); empty zones give 0
 *   5 Pearson's r of the two profiles over non-empty annuli (Table 4)
 *   6 annuli ceil(r_max);  7, 8, 9 largest pixel of a, b, c
 *   10 with c: share of non-empty annuli where a's profile is closer to b's
 *      than c's is (Table 4, last column); NaN without c
 *   11 pixels compared
 * profiles, if not NULL, receives 4 x annuli doubles on the device: the
 * profiles of a, b, c and the pixel count of each annulus.  work is DEVICE
 * scratch of mc_metrics_work_bytes bytes.  Sums over pixels use a fixed
 * partition and tree reductions; annulus sums are int64 fixed point, so the
 * results do not depend on scheduling.  Waits for the stream.
 */
#define MC_METRICS_N 12
#define MC_MAX_ANNULI 2048
typedef struct {
    double cx, cy;         /* radial centre in pixel units (column, row), e.g. nx / 2, ny / 2 */
    double r_max;          /* outer radius in pixels, 0 < r_max <= MC_MAX_ANNULI */
} mc_radial_t;

uint64_t mc_metrics_work_bytes(int32_t nx, int32_t ny, const mc_radial_t *radial);
int mc_image_metrics(const double *a, const double *b, const double *c, int32_t nx, int32_t ny,
                     const mc_radial_t *radial, double *profiles, void *work, uint64_t work_bytes,
                     double out[MC_METRICS_N], void *stream);

/* Message of the last failed call on this thread ("" if none). */
const char *mc_last_error(void);

/* Library version, major * 10000 + minor * 100 + patch. */
int mc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MCMIE_H */
