/*
 * Sanitizer driver for the host side of the C ABI (built by
 * tests/test_sanitizers.py from the library's sources compiled for the host
 * only, with AddressSanitizer and UndefinedBehaviorSanitizer; CPU only).  It
 * calls every entry point on arguments the host checks reject, and the
 * host-only helpers on valid ones, so argument validation, workspace sizing
 * and the medium and size-bin derivations run under the sanitizers without
 * any device work.
 */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "mcmie.h"

static int fails = 0;

static void expect(const char *what, int rc, int want)
{
    if (rc != want) {
        printf("%s: got %d, want %d (%s)\n", what, rc, want, mc_last_error());
        ++fails;
    } else if (want != MC_OK && mc_last_error()[0] == '\0') {
        printf("%s: no message\n", what);
        ++fails;
    }
}

int main(void)
{
    static char fake[4096];   /* never dereferenced: every call below fails validation first */
    mc_medium_t med;
    memset(&med, 0, sizeof med);
    med.input = MC_MEDIUM_TAU; med.phase = MC_PHASE_HG; med.tau = 1.0; med.albedo = 0.9; med.g = 0.5;
    mc_source_t src;
    memset(&src, 0, sizeof src);
    src.pos_mm[0] = src.pos_mm[1] = 5.0; src.dir[2] = 1.0;
    mc_geometry_t geo = {{10.0, 10.0, 10.0}, 1.33, 1.0};
    mc_detector_t det = {16, 16, 16, 16, 0};
    mc_run_t run;
    memset(&run, 0, sizeof run);
    run.n_photons = 1000; run.seed = 1234; run.max_steps = 1000; run.roulette_p = 0.1; run.record_stride = 1;
    mc_tally_t tal;
    memset(&tal, 0, sizeof tal);
    tal.side = tal.trans = fake; tal.scalars = (double *)fake; tal.workspace = fake;
    tal.workspace_bytes = mc_workspace_bytes(&det);

    /* Host-only helpers on valid input. */
    double coef[4];
    expect("coefficients", mc_medium_coefficients(&med, &geo, coef), MC_OK);
    if (fabs(coef[2] - 0.1) > 1e-15 || fabs(coef[3] - 0.9) > 1e-15) { printf("coefficients wrong\n"); ++fails; }
    double d[64], p[64];
    expect("lognormal bins", mc_lognormal_bins(5.0, 0.05, 64, d, p), MC_OK);
    double sum = 0.0;
    for (int i = 0; i < 64; ++i) sum += p[i];
    if (fabs(sum - 1.0) > 1e-12) { printf("bin probabilities sum to %.17g\n", sum); ++fails; }
    mie_spec_t spec = {1.33, 1.59, 0.0, 5.0, 532.0, 1801, 16384};
    mie_poly_t poly = {0.05, 64, 0, NULL, 0};
    if (mie_poly_work_bytes(&spec, &poly) == 0) { printf("poly work bytes 0\n"); ++fails; }
    mc_radial_t rad = {256.0, 256.0, 256.0};
    if (mc_metrics_work_bytes(512, 512, &rad) == 0) { printf("metrics work bytes 0\n"); ++fails; }
    mc_detector_t big = {1024, 1024, 1024, 1024, MC_SIGMA | MC_EXIT_LOG};
    if (mc_workspace_bytes_log(&big, 1000000000ull) <= mc_workspace_bytes(&big)) { printf("log bytes\n"); ++fails; }
    if (mc_workspace_bytes_batch(&det, 512) == 0 || mc_workspace_bytes_batch(&det, 513) != 0) {
        printf("batch bytes\n"); ++fails;
    }
    if (mc_workspace_bytes(NULL) != 0 || mc_version() <= 0) { printf("null detector\n"); ++fails; }

    /* Rejections. */
    mc_medium_t m2 = med;
    m2.input = 7;
    expect("medium input", mc_simulate(&m2, &src, &geo, &det, &run, &tal, NULL), MC_EINVAL);
    m2 = med; m2.input = MC_MEDIUM_CONCENTRATION; m2.concentration_per_mm3 = NAN;
    expect("concentration", mc_medium_coefficients(&m2, &geo, coef), MC_EINVAL);
    m2 = med; m2.tau = -1.0;
    expect("tau", mc_simulate(&m2, &src, &geo, &det, &run, &tal, NULL), MC_EINVAL);
    m2 = med; m2.phase = MC_PHASE_MIE; m2.n_cdf = 1;
    expect("n_cdf", mc_simulate(&m2, &src, &geo, &det, &run, &tal, NULL), MC_EINVAL);
    mc_source_t s2 = src;
    s2.pos_mm[2] = 1.0;
    expect("source", mc_simulate(&med, &s2, &geo, &det, &run, &tal, NULL), MC_EINVAL);
    s2 = src; s2.beam_radius_mm = 6.0;
    expect("beam disk", mc_simulate(&med, &s2, &geo, &det, &run, &tal, NULL), MC_EINVAL);
    mc_geometry_t g2 = geo;
    g2.size_mm[1] = 0.0;
    expect("geometry", mc_simulate(&med, &src, &g2, &det, &run, &tal, NULL), MC_EINVAL);
    mc_detector_t d2 = det;
    d2.flags = 1u << 12;
    expect("flags", mc_simulate(&med, &src, &geo, &d2, &run, &tal, NULL), MC_EINVAL);
    d2 = det; d2.flags = MC_EXIT_LOG | MC_RECORD;
    expect("log + record", mc_simulate(&med, &src, &geo, &d2, &run, &tal, NULL), MC_EINVAL);
    mc_tally_t t2 = tal;
    t2.workspace_bytes = 8;
    expect("workspace", mc_simulate(&med, &src, &geo, &det, &run, &t2, NULL), MC_EINVAL);
    mc_run_t r2 = run;
    r2.n_photons = 1ull << 40;
    expect("overflow bound", mc_simulate(&med, &src, &geo, &det, &r2, &tal, NULL), MC_EINVAL);
    r2 = run; r2.block_size = 100;
    expect("block size", mc_simulate(&med, &src, &geo, &det, &r2, &tal, NULL), MC_EINVAL);
    d2 = det; d2.flags = MC_SIGMA; d2.side_nx = d2.side_ny = d2.trans_nx = d2.trans_ny = 1024;
    expect("noalloc size", mc_simulate_noalloc(&med, &src, &geo, &d2, &run, &tal, NULL), MC_EINVAL);
    expect("null", mc_simulate(NULL, &src, &geo, &det, &run, &tal, NULL), MC_EINVAL);
    double grad[3];
    m2 = med; m2.albedo = 0.0;
    expect("grad mu_sca", mc_grad(&m2, &geo, &det, &tal, (const double *)fake, NULL, 0.0, grad, NULL), MC_EINVAL);
    expect("grad moments", mc_grad(&med, &geo, &det, &tal, (const double *)fake, NULL, 0.0, grad, NULL), MC_EINVAL);
    mc_batch_item_t item = {1.0, 1.5, (const float *)fake, 10, 0, 0};
    expect("batch albedo", mc_simulate_batch(&item, 1, 4096, &src, &geo, &det, &run, &tal, NULL), MC_EINVAL);
    expect("batch count", mc_simulate_batch(&item, 0, 4096, &src, &geo, &det, &run, &tal, NULL), MC_EINVAL);
    int32_t bs; uint32_t ch; double best;
    expect("autotune fraction", mc_autotune_batch(&item, 1, 4096, &src, &geo, &det, &run, &tal, 2.0, &bs, &ch,
                                                  &best, NULL, NULL), MC_EINVAL);
    mie_spec_t sp2 = spec;
    sp2.diameter_um = -1.0;
    mie_table_t tab;
    memset(&tab, 0, sizeof tab);
    tab.inv_cdf = (float *)fake;
    expect("mie spec", mie_table_build(&sp2, &tab, NULL), MC_EINVAL);
    sp2 = spec; sp2.n_angles = 2;
    expect("mie angles", mie_table_enqueue(&sp2, &tab, NULL), MC_EINVAL);
    mie_poly_t pl2 = poly;
    pl2.n_bins = 65;
    expect("poly bins", mie_table_build_poly(&spec, &pl2, &tab, NULL), MC_EINVAL);
    expect("lognormal sigma", mc_lognormal_bins(5.0, -1.0, 4, d, p), MC_EINVAL);
    double out[MC_METRICS_N];
    mc_radial_t r0 = {1.0, 1.0, 0.0};
    expect("metrics radius", mc_image_metrics((const double *)fake, (const double *)fake, NULL, 8, 8, &r0, NULL,
                                              fake, sizeof fake, out, NULL), MC_EINVAL);
    expect("philox empty", mc_philox_blocks(1, 0, NULL, 0, 0, 1, NULL, NULL), MC_OK);
    expect("philox null", mc_philox_blocks(1, 0, NULL, 4, 0, 1, NULL, NULL), MC_EINVAL);
    printf(fails ? "FAILED (%d)\n" : "OK\n", fails);
    return fails != 0;
}
