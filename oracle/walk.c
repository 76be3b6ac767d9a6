/*
 * Oracle photon walk: plain C, FP64, one photon at a time.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product path.  It shares no code
 * with the HIP library.
 *
 * The walk follows the Monte Carlo module of Sec. 3.1.3 of the paper:
 * photon start (parallel beam at normal incidence), free path from Eq. 15,
 * boundary determination at the cuvette walls, polar angle from the
 * precomputed inverse CDF (Sec. 2.6) or from Henyey-Greenstein (Eq. 11),
 * azimuth uniform on [0, 2 pi) (Sec. 2.6), weight update of Eq. 16 at every
 * interaction, and tallies of exit positions into detector images.
 *
 * Readings where the paper is silent (each is stated with its reason in the
 * design notes of the repository):
 *   - random numbers: one Philox4x32-10 block per step (counter = step,
 *     instance, id_lo, id_hi; key = seed_lo, seed_hi); u0 free path,
 *     u1 polar angle, u2 azimuth, u3 Fresnel choice or roulette;
 *     u = (2 floor(r / 2^9) + 1) / 2^24;
 *   - walls: one n_med -> n_out interface per face, unpolarised Fresnel
 *     reflectance with total internal reflection, chosen stochastically;
 *     the entry loss at the source face is a deterministic weight 1 - R;
 *   - termination: Russian roulette below roulette_w with survival
 *     probability roulette_p (weight divided by roulette_p) instead of the
 *     paper's hard cut at w < 0.001; a step cap counts as "capped";
 *   - absorption: w *= albedo and absorbed += w (1 - albedo) at interactions
 *     only (implicit capture, Eq. 16);
 *   - direction update: orthonormal basis of Duff et al. 2017 ("Building an
 *     Orthonormal Basis, Revisited", JCGT 6(1)) around the current direction;
 *   - detector: exit position on the +x face (side image, rows y, columns z)
 *     and on the +z face (transmitted image, rows y, columns x); pixel =
 *     floor(coord / size * n), clamped to n - 1.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <string.h>

typedef struct {
    double size[3];          /* cuboid extent along x, y, z (mm) */
    double n_med, n_out;     /* refractive index inside / outside the walls */
    double mu_t;             /* extinction coefficient (1/mm), Eq. 1 */
    double albedo;           /* mu_sca / mu_ext */
    double src_pos[3];       /* on the z = 0 face */
    double src_dir[3];       /* incident direction outside, dir_z > 0 */
    int32_t phase;           /* 0: inverse table, 1: Henyey-Greenstein */
    int32_t n_table;
    const double *table;     /* inverse table, v = 1 - cos(theta) */
    double g;                /* HG asymmetry */
    uint64_t seed;
    uint32_t instance;
    uint32_t max_steps;
    double roulette_w, roulette_p;
    int32_t side_nx, side_ny, trans_nx, trans_ny;
    double beam_radius;      /* radius of the parallel beam's disk on the z = 0 face (mm), 0: pencil */
} oracle_params;

enum { S_FACE0 = 0, S_ABSORBED = 6, S_ROULETTE_NET = 7, S_CAPPED_W = 8, S_EVENTS = 9,
       S_PHOTONS = 10, S_ROULETTE_KILLS = 11, S_CAPPED = 12, S_REFLECTIONS = 13,
       S_STEPS = 14, S_COUNT = 16 };
enum { CAUSE_EXIT = 0, CAUSE_ROULETTE = 1, CAUSE_CAPPED = 2 };

/* ---------------- Philox4x32-10 (Salmon et al., SC'11) ---------------- */

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        uint32_t n1 = (uint32_t)p1;
        uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        uint32_t n3 = (uint32_t)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double uniform_of(uint32_t r)
{
    return (double)(2u * (r >> 9) + 1u) / 16777216.0;
}

/* ---------------- physics helpers ---------------- */

/* Unpolarised Fresnel reflectance going from index n1 into n2 at incidence
 * cosine cos_i; 1 beyond the critical angle. */
double oracle_fresnel(double cos_i, double n1, double n2)
{
    if (n1 == n2) return 0.0;
    double sin_i = sqrt(fmax(0.0, 1.0 - cos_i * cos_i));
    double sin_t = n1 / n2 * sin_i;
    if (sin_t >= 1.0) return 1.0;
    double cos_t = sqrt(1.0 - sin_t * sin_t);
    double rs = (n1 * cos_i - n2 * cos_t) / (n1 * cos_i + n2 * cos_t);
    double rp = (n2 * cos_i - n1 * cos_t) / (n2 * cos_i + n1 * cos_t);
    return 0.5 * (rs * rs + rp * rp);
}

/* v = 1 - cos(theta) for the polar draw u (table lookup or HG closed form). */
double oracle_sample_v(const oracle_params *p, double u)
{
    if (p->phase == 1) {
        double g = p->g;
        double D = 1.0 + g - 2.0 * g * u;
        double t = (1.0 - g * g) / D;
        return (1.0 - g) * u * (t + 1.0 - g) / D;
    }
    int N = p->n_table;
    double t = u * (double)(N - 1);
    int i = (int)floor(t);
    if (i > N - 2) i = N - 2;
    double f = t - (double)i;
    return p->table[i] + f * (p->table[i + 1] - p->table[i]);
}

/* New direction at polar angle (cos_t, sin_t) and azimuth (cos_p, sin_p)
 * about the unit direction d, in the basis of Duff et al. 2017; renormalised. */
void oracle_rotate(double d[3], double cos_t, double sin_t, double cos_p, double sin_p)
{
    double sign = copysign(1.0, d[2]);
    double a = -1.0 / (sign + d[2]);
    double b = d[0] * d[1] * a;
    double e1[3] = {1.0 + sign * d[0] * d[0] * a, sign * b, -sign * d[0]};
    double e2[3] = {b, sign + d[1] * d[1] * a, -d[1]};
    double n[3];
    for (int i = 0; i < 3; ++i)
        n[i] = cos_t * d[i] + sin_t * (cos_p * e1[i] + sin_p * e2[i]);
    double len = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    for (int i = 0; i < 3; ++i) d[i] = n[i] / len;
}

static int pixel_index(double coord, double size, int n)
{
    double f = floor(coord / size * (double)n);
    if (f < 0.0) f = 0.0;
    if (f > (double)(n - 1)) f = (double)(n - 1);
    return (int)f;
}

/* ---------------- one photon ---------------- */

typedef struct {
    int face, cause;
    uint32_t k, steps;
    double pos[3], dir[3], w, L, A;
} photon_end;

static photon_end walk_one(const oracle_params *p, uint64_t id, double *scal)
{
    photon_end e;
    const uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};

    /* Start: parallel beam entering the z = 0 face (Sec. 3.1.3); the incident
     * direction refracts into the medium and the beam keeps 1 - R of its
     * weight. */
    double din[3] = {p->src_dir[0], p->src_dir[1], p->src_dir[2]};
    double dl = sqrt(din[0] * din[0] + din[1] * din[1] + din[2] * din[2]);
    for (int i = 0; i < 3; ++i) din[i] /= dl;
    double cos_i = din[2];
    double eta = p->n_out / p->n_med;
    double d[3] = {eta * din[0], eta * din[1], 0.0};
    double tang2 = d[0] * d[0] + d[1] * d[1];
    d[2] = sqrt(fmax(0.0, 1.0 - tang2));
    double w = 1.0 - oracle_fresnel(cos_i, p->n_out, p->n_med);
    double pos[3] = {p->src_pos[0], p->src_pos[1], p->src_pos[2]};
    if (p->beam_radius > 0.0) {
        /* A beam of finite width (Sec. 4.1): the entry point is uniform on the
         * disk of that radius around the source position, drawn from the
         * photon's Philox block at the reserved step counter 2^32 - 1:
         * radius R sqrt(u0), azimuth 2 pi u1. */
        uint32_t ctr[4] = {0xFFFFFFFFu, p->instance, (uint32_t)id, (uint32_t)(id >> 32)};
        uint32_t r[4];
        oracle_philox4x32_10(ctr, key, r);
        const double rho = p->beam_radius * sqrt(uniform_of(r[0]));
        const double phi = 2.0 * M_PI * uniform_of(r[1]);
        pos[0] += rho * cos(phi);
        pos[1] += rho * sin(phi);
    }
    double L = 0.0, A = 0.0;
    uint32_t k = 0, step = 0, refl = 0;
    int face = -1, cause = CAUSE_CAPPED;
    double roulette_net = 0.0;

    for (step = 0; step < p->max_steps; ++step) {
        uint32_t ctr[4] = {step, p->instance, (uint32_t)id, (uint32_t)(id >> 32)};
        uint32_t r[4];
        oracle_philox4x32_10(ctr, key, r);
        double u0 = uniform_of(r[0]), u1 = uniform_of(r[1]);
        double u2 = uniform_of(r[2]), u3 = uniform_of(r[3]);

        /* Eq. 15: free path. */
        double s = -log(u0) / p->mu_t;

        /* Boundary determination: nearest wall along d, ties to the lower axis. */
        double db = INFINITY;
        int axis = -1;
        for (int i = 0; i < 3; ++i) {
            double t;
            if (d[i] > 0.0) t = (p->size[i] - pos[i]) / d[i];
            else if (d[i] < 0.0) t = -pos[i] / d[i];
            else continue;
            if (t < 0.0) t = 0.0;
            if (t < db) { db = t; axis = i; }
        }

        if (s >= db) {
            /* Move to the wall; reflect with probability R, else leave. */
            for (int i = 0; i < 3; ++i) pos[i] += db * d[i];
            pos[axis] = d[axis] > 0.0 ? p->size[axis] : 0.0;
            L += db;
            double ci = fabs(d[axis]);
            double R = oracle_fresnel(ci, p->n_med, p->n_out);
            if (u3 < R) {
                d[axis] = -d[axis];
                ++refl;
                continue;
            }
            face = 2 * axis + (d[axis] > 0.0 ? 1 : 0);
            /* Refracted exit direction (recorded only). */
            double et = p->n_med / p->n_out;
            double o[3] = {et * d[0], et * d[1], et * d[2]};
            double t2 = 0.0;
            for (int i = 0; i < 3; ++i) if (i != axis) t2 += o[i] * o[i];
            o[axis] = copysign(sqrt(fmax(0.0, 1.0 - t2)), d[axis]);
            for (int i = 0; i < 3; ++i) d[i] = o[i];
            cause = CAUSE_EXIT;
            ++step;
            break;
        }

        /* Interaction: move, count the event, absorb (Eq. 16). */
        for (int i = 0; i < 3; ++i) pos[i] += s * d[i];
        L += s;
        ++k;
        A += w * (1.0 - p->albedo);
        w *= p->albedo;

        /* Russian roulette. */
        if (w < p->roulette_w) {
            if (u3 < p->roulette_p) {
                double wn = w / p->roulette_p;
                roulette_net += wn - w;
                w = wn;
            } else {
                roulette_net -= w;
                w = 0.0;
                cause = CAUSE_ROULETTE;
                ++step;
                break;
            }
        }

        /* Scatter: polar angle from the inverse CDF (or HG), azimuth 2 pi u2. */
        double v = oracle_sample_v(p, u1);
        double cos_t = 1.0 - v;
        double sin_t = sqrt(fmax(0.0, v * (2.0 - v)));
        double phi = 2.0 * M_PI * u2;
        oracle_rotate(d, cos_t, sin_t, cos(phi), sin(phi));
    }

    e.face = face; e.cause = cause; e.k = k; e.steps = step;
    for (int i = 0; i < 3; ++i) { e.pos[i] = pos[i]; e.dir[i] = d[i]; }
    e.w = w; e.L = L; e.A = A;

    if (cause == CAUSE_EXIT) scal[S_FACE0 + face] += w;
    if (cause == CAUSE_CAPPED) { scal[S_CAPPED_W] += w; scal[S_CAPPED] += 1.0; }
    if (cause == CAUSE_ROULETTE) scal[S_ROULETTE_KILLS] += 1.0;
    scal[S_ABSORBED] += A;
    scal[S_ROULETTE_NET] += roulette_net;
    scal[S_EVENTS] += (double)k;
    scal[S_PHOTONS] += 1.0;
    scal[S_REFLECTIONS] += (double)refl;
    scal[S_STEPS] += (double)step;
    return e;
}

/*
 * Simulate photons ids[0..n) (or id0 .. id0+n when ids is NULL) in order.
 * Images are rows x cols, row-major, accumulated (+=).  scal has S_COUNT
 * entries, accumulated.  irec (4 x n int32: face, cause, k, steps) and frec
 * (9 x n double: px, py, pz, dx, dy, dz, w, L, A), structure of arrays, are
 * optional.  Returns 0, or -1 on a parameter the walk cannot take.
 */
int oracle_simulate(const oracle_params *p, const uint64_t *ids, uint64_t id0, uint64_t n,
                    double *side, double *trans, double *side_w2, double *trans_w2,
                    double *scal, int32_t *irec, double *frec)
{
    if (p->phase == 0 && (p->n_table < 2 || !p->table)) return -1;
    if (p->src_dir[2] <= 0.0) return -1;
    for (uint64_t r = 0; r < n; ++r) {
        uint64_t id = ids ? ids[r] : id0 + r;
        photon_end e = walk_one(p, id, scal);
        if (e.cause == CAUSE_EXIT && e.face == 1) {
            int row = pixel_index(e.pos[1], p->size[1], p->side_ny);
            int col = pixel_index(e.pos[2], p->size[2], p->side_nx);
            size_t at = (size_t)row * (size_t)p->side_nx + (size_t)col;
            if (side) side[at] += e.w;
            if (side_w2) side_w2[at] += e.w * e.w;
        }
        if (e.cause == CAUSE_EXIT && e.face == 5) {
            int row = pixel_index(e.pos[1], p->size[1], p->trans_ny);
            int col = pixel_index(e.pos[0], p->size[0], p->trans_nx);
            size_t at = (size_t)row * (size_t)p->trans_nx + (size_t)col;
            if (trans) trans[at] += e.w;
            if (trans_w2) trans_w2[at] += e.w * e.w;
        }
        if (irec) {
            irec[0 * n + r] = e.face;
            irec[1 * n + r] = e.cause;
            irec[2 * n + r] = (int32_t)e.k;
            irec[3 * n + r] = (int32_t)e.steps;
        }
        if (frec) {
            for (int i = 0; i < 3; ++i) frec[(0 + i) * n + r] = e.pos[i];
            for (int i = 0; i < 3; ++i) frec[(3 + i) * n + r] = e.dir[i];
            frec[6 * n + r] = e.w;
            frec[7 * n + r] = e.L;
            frec[8 * n + r] = e.A;
        }
    }
    return 0;
}

size_t oracle_params_size(void) { return sizeof(oracle_params); }
