/*
 * Sanitizer driver for the oracle's C walk (built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_sanitizers.py, CPU only).  It
 * compiles the walk into this translation unit and runs it over the paths a
 * test exercises: the inverse table and Henyey-Greenstein, pencil and finite
 * beams, index-matched and refracting walls, heavy roulette, the step cap,
 * records by id list and by range, ragged images, and the standalone
 * probes.  Each run must close its energy bookkeeping (Eq. 16) to 1e-12.
 */
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/walk.c"

static int check_run(const char *name, oracle_params *p, uint64_t n, const uint64_t *ids)
{
    const size_t ns = (size_t)p->side_nx * p->side_ny, nt = (size_t)p->trans_nx * p->trans_ny;
    double *side = calloc(ns, sizeof(double)), *trans = calloc(nt, sizeof(double));
    double *side2 = calloc(ns, sizeof(double)), *trans2 = calloc(nt, sizeof(double));
    double scal[S_COUNT] = {0};
    int32_t *irec = calloc(4 * n, sizeof(int32_t));
    double *frec = calloc(9 * n, sizeof(double));
    int bad = 0;
    if (oracle_simulate(p, ids, 17, n, side, trans, side2, trans2, scal, irec, frec) != 0) {
        printf("%s: rejected\n", name);
        bad = 1;
    } else {
        /* Start weight at normal incidence for the beams used here. */
        const double r = (p->n_out - p->n_med) / (p->n_out + p->n_med);
        const double w0 = 1.0 - r * r;
        double out = scal[S_ABSORBED] + scal[S_CAPPED_W] - scal[S_ROULETTE_NET];
        for (int f = 0; f < 6; ++f) out += scal[S_FACE0 + f];
        const double resid = out / ((double)n * w0) - 1.0;
        double img = 0.0;
        for (size_t i = 0; i < ns; ++i) img += side[i];
        printf("%s: %llu photons, %g events, residual %.3e, side %.6g (face %.6g)\n", name, (unsigned long long)n,
               scal[S_EVENTS], resid, img, scal[S_FACE0 + 1]);
        if (!(fabs(resid) < 1e-12) || !(fabs(img - scal[S_FACE0 + 1]) <= 1e-9 * (1.0 + img))) bad = 1;
        for (uint64_t i = 0; i < n; ++i)
            if (irec[i] < -1 || irec[i] > 5 || irec[n + i] < 0 || irec[n + i] > 2) bad = 1;
    }
    free(side); free(trans); free(side2); free(trans2); free(irec); free(frec);
    return bad;
}

int main(void)
{
    /* An isotropic inverse table (v = 1 - cos(theta) = 2u) of 9 entries. */
    double table[9];
    for (int i = 0; i < 9; ++i) table[i] = 2.0 * i / 8.0;
    oracle_params p;
    memset(&p, 0, sizeof p);
    p.size[0] = 10.0; p.size[1] = 7.0; p.size[2] = 5.0;
    p.n_med = 1.33; p.n_out = 1.0;
    p.mu_t = 0.8; p.albedo = 0.99;
    p.src_pos[0] = 5.0; p.src_pos[1] = 3.5; p.src_pos[2] = 0.0;
    p.src_dir[0] = 0.0; p.src_dir[1] = 0.0; p.src_dir[2] = 1.0;
    p.phase = 0; p.n_table = 9; p.table = table; p.g = 0.0;
    p.seed = 1234; p.instance = 3; p.max_steps = 1u << 20;
    p.roulette_w = 1e-4; p.roulette_p = 0.1;
    p.side_nx = 7; p.side_ny = 5; p.trans_nx = 3; p.trans_ny = 11;
    int bad = 0;
    bad |= check_run("table", &p, 3000, NULL);
    p.phase = 1; p.g = 0.9;
    bad |= check_run("hg", &p, 3000, NULL);
    p.beam_radius = 1.25;
    bad |= check_run("finite beam", &p, 2000, NULL);
    p.beam_radius = 0.0; p.n_out = p.n_med;
    bad |= check_run("matched walls", &p, 2000, NULL);
    p.albedo = 0.5; p.roulette_w = 0.3; p.roulette_p = 0.25;
    bad |= check_run("roulette", &p, 2000, NULL);
    p.max_steps = 3;
    bad |= check_run("step cap", &p, 2000, NULL);
    p.max_steps = 1u << 20; p.mu_t = 0.0;
    bad |= check_run("empty medium", &p, 500, NULL);
    const uint64_t ids[5] = {0, 7, 1ull << 33, 12345678901ull, ~0ull};
    p.mu_t = 2.0; p.albedo = 1.0; p.roulette_w = 0.0;
    bad |= check_run("ids", &p, 5, ids);
    /* Standalone probes. */
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    oracle_philox4x32_10(ctr, key, out);
    double d[3] = {0.0, 0.0, -1.0};
    oracle_rotate(d, 0.5, sqrt(0.75), 0.0, 1.0);
    const double fr = oracle_fresnel(0.3, 1.33, 1.0) + oracle_fresnel(1.0, 1.0, 1.33);
    p.phase = 0;
    const double v = oracle_sample_v(&p, 0.999999);
    printf("probes: philox %08x, rotated |d| %.15f, fresnel %.6f, v %.6f\n", out[0],
           sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]), fr, v);
    if (oracle_params_size() != sizeof(oracle_params)) bad = 1;
    printf(bad ? "FAILED\n" : "OK\n");
    return bad;
}
