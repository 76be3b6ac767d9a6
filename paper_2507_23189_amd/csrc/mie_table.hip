// Mie phase-function table on the device, FP64 (Sec. 2.2-2.6, Sec. 3.1.2).
//
// Two kernels build one table:
//   mie_phase_kernel, one lane per angle, 256-lane workgroups:
//   1. every workgroup runs the Bohren-Huffman series (Sec. 2.5) for itself:
//      one lane runs the logarithmic derivative D_n(mx) by downward
//      recurrence (in homogeneous form, D_n = P_n / Q_n, so the serial chain
//      holds no division) while a lane of another wave runs psi_n(x) and
//      chi_n(x) upward; then every lane forms a_n and b_n for its n (Eqs. 7-8
//      divided through by psi_n(mx)), and Q_ext (Eq. 13), Q_sca and the
//      asymmetry sums (Eq. 12) are added in a fixed order;
//   2. each lane evaluates S1, S2 (Eqs. 5-6) at its angle with the angular
//      functions pi_n, tau_n by upward recurrence (the per-n divisions done
//      once beforehand), giving the phase function normalised so that
//      (1/4pi) int P dOmega = 1 (Eqs. 9-10); P sin(theta) goes to a device
//      buffer of n_angles doubles;
//   mie_inverse_kernel, one lane per inverse-table entry, 1024-lane groups:
//   3. every workgroup reads the whole P sin(theta) grid into LDS and forms
//      its trapezoid CDF by a block scan;
//   4. each inverse-table entry u_i = i/(N-1) finds the first angle with
//      F >= u_i by binary search and interpolates theta linearly; the table
//      stores v = 1 - cos(theta) = 2 sin^2(theta/2) in FP32.
// The series is short and serial, so repeating it per workgroup costs no
// time, while the angle grid and the inverse table, which took a single
// compute unit's FP64 issue, spread over ~8 and ~16 of them.  Arrays live in
// LDS (coefficients 32 KB, pi_n recurrence coefficients 16 KB, psi and chi
// 16 KB, angle grid 24 KB at the limits; gfx950 gives a workgroup up to
// 160 KB).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "common.hpp"

namespace mcmie {
namespace {

constexpr int kPhaseThreads = 256;    // phase kernels: one angle per lane
constexpr int kInvThreads = 1024;     // CDF and inverse: one entry per lane, 1..3 angles per lane in the scan

struct cplx {
    double re, im;
};
__device__ __forceinline__ cplx operator+(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx operator-(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx operator*(cplx a, cplx b)
{
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cplx operator*(double s, cplx a) { return {s * a.re, s * a.im}; }
__device__ __forceinline__ cplx operator+(cplx a, double s) { return {a.re + s, a.im}; }
// Smith's division: no overflow of |b|^2 for large operands.
__device__ __forceinline__ cplx operator/(cplx a, cplx b)
{
    if (fabs(b.re) >= fabs(b.im)) {
        const double r = b.im / b.re, den = b.re + b.im * r;
        return {(a.re + a.im * r) / den, (a.im - a.re * r) / den};
    }
    const double r = b.re / b.im, den = b.re * r + b.im;
    return {(a.re * r + a.im) / den, (a.im * r - a.re) / den};
}
__device__ __forceinline__ double norm2(cplx a) { return a.re * a.re + a.im * a.im; }

// sin(t) for |t| <= pi/2 from its Taylor series through t^19/19!, in Horner
// form in t^2 (truncation below (pi/2)^21/21! < 3e-16): no range reduction is
// needed on this interval.
__device__ __forceinline__ double sin_half_pi(double t)
{
    const double s = t * t;
    double p = 1.0 / 121645100408832000.0;               // 1/19!
    p = fma(p, s, -1.0 / 355687428096000.0);             // -1/17!
    p = fma(p, s, 1.0 / 1307674368000.0);                // 1/15!
    p = fma(p, s, -1.0 / 6227020800.0);                  // -1/13!
    p = fma(p, s, 1.0 / 39916800.0);                     // 1/11!
    p = fma(p, s, -1.0 / 362880.0);                      // -1/9!
    p = fma(p, s, 1.0 / 5040.0);                         // 1/7!
    p = fma(p, s, -1.0 / 120.0);                         // -1/5!
    p = fma(p, s, 1.0 / 6.0);                            // 1/3! (subtracted below)
    return t - t * s * p;
}
// sin and cos of theta in [0, pi].  sin by reflection onto [0, pi/2];
// cos as 1 - 2 sin^2(theta/2) (or its mirror about pi/2), which keeps full
// accuracy where cos is near +-1 and the angular functions are most sensitive.
__device__ __forceinline__ double sin_0_pi(double th) { return sin_half_pi(th <= 0.5 * M_PI ? th : M_PI - th); }
__device__ __forceinline__ double cos_0_pi(double th)
{
    const bool back = th > 0.5 * M_PI;
    const double h = sin_half_pi(0.5 * (back ? M_PI - th : th));
    const double c = 1.0 - 2.0 * h * h;
    return back ? -c : c;
}

struct MieArgs {
    double x, m_re, m_im;
    int n_terms, n_start, n_angles, n_cdf;
    float *inv_cdf;
    double *phase, *cdf, *coef;
    double *result;          // q_ext, q_sca, g, n_terms
    double *work;            // n_angles: P(theta_j) sin(theta_j), from the phase kernel to the inverse kernel
};

// Step 1 by every lane of a workgroup: the series for size parameter x and relative
// index m.  The two recurrences are serial and run at once on lanes of two
// different waves: D_n(mx) downward from n_start and psi_n(x), chi_n(x)
// upward (into s_psi, s_chi at index n, n = 0..N).  One downward step
//     D_{n-1} = n/(mx) - 1/(D_n + n/(mx))
// is the Moebius map of the matrix [[k, k^2 - 1], [1, k]], k = n/(mx), so it
// runs on D_n = P_n / Q_n as Q' = P + k Q, P' = k Q' - Q: eight FMAs and no
// division on the serial chain (one wave runs it, so its instruction count
// is its time).  One step grows or shrinks max(|P|, |Q|) by at most
// (1 + |k|)^2, with |k| < 2e9 for every size and index this library accepts
// (n_start <= ~1100 where |mx| < n_terms, |mx| >= 1e-6), so rescaling (P, Q)
// by a power of two every 8 steps keeps both far inside the FP64 range; the
// scale is exact and cancels in P / Q.  Its rounding matches that of the
// direct form (checked against a 50-digit evaluation of the recurrence).
// P_n and Q_n go to s_a and s_b (n = 1..N at index n - 1), and each lane
// forms D_n = P_n / Q_n for its n.  Then each lane forms a_n and b_n (in
// place of P_n and Q_n),
// and the sums of Q_ext (Eq. 13), Q_sca and the asymmetry (Eq. 12) are
// added per lane, per wave and over the waves in a fixed order.  On return
// (after a barrier) s_sums holds Q_ext, Q_sca and g for every lane.
__device__ __forceinline__ void mie_series_block(double x, double m_re, double m_im, int N, int n_start, cplx *s_a, cplx *s_b,
                                 double *s_psi, double *s_chi, double *s_red, double *s_sums)
{
    const int tid = threadIdx.x;
    const cplx m = {m_re, m_im};
    if (tid == 0) {
        const cplx mx = x * m;
        const cplx inv_mx = cplx{1.0, 0.0} / mx;
        cplx P = {0.0, 0.0}, Q = {1.0, 0.0};   // D_{n_start} = 0
        auto step = [&](int n) {
            const cplx k = (double)n * inv_mx;
            const cplx Q1 = {fma(k.re, Q.re, fma(-k.im, Q.im, P.re)), fma(k.re, Q.im, fma(k.im, Q.re, P.im))};
            P = {fma(k.re, Q1.re, fma(-k.im, Q1.im, -Q.re)), fma(k.re, Q1.im, fma(k.im, Q1.re, -Q.im))};
            Q = Q1;
            if ((n & 7) == 0) {
                int e;
                (void)frexp(fmax(fmax(fabs(P.re), fabs(P.im)), fmax(fabs(Q.re), fabs(Q.im))), &e);
                P = {ldexp(P.re, -e), ldexp(P.im, -e)};
                Q = {ldexp(Q.re, -e), ldexp(Q.im, -e)};
            }
        };
        int n = n_start;
        for (; n > N; --n) step(n);
        for (; n >= 1; --n) {   // keep D_n = P_n / Q_n for n <= N
            s_a[n - 1] = P;
            s_b[n - 1] = Q;
            step(n);
        }
    } else if (tid == 64) {
        double psi_prev = cos(x), psi = sin(x);        // psi_{-1}, psi_0
        double chi_prev = -sin(x), chi = cos(x);       // chi_{-1}, chi_0
        s_psi[0] = psi;
        s_chi[0] = chi;
        for (int n = 1; n <= N; ++n) {
            const double f = (2.0 * n - 1.0) / x;
            const double psi_n = f * psi - psi_prev;
            const double chi_n = f * chi - chi_prev;
            s_psi[n] = psi_n;
            s_chi[n] = chi_n;
            psi_prev = psi;
            psi = psi_n;
            chi_prev = chi;
            chi = chi_n;
        }
    }
    __syncthreads();
    const cplx inv_m = cplx{1.0, 0.0} / m;
    for (int n = tid + 1; n <= N; n += blockDim.x) {
        const double psi_n = s_psi[n], psi = s_psi[n - 1];
        const cplx xi_n = {psi_n, -s_chi[n]};
        const cplx xi_nm1 = {psi, -s_chi[n - 1]};
        const cplx Dn = s_a[n - 1] / s_b[n - 1];
        const double nx = (double)n / x;
        const cplx da = Dn * inv_m + nx;
        const cplx db = m * Dn + nx;
        s_a[n - 1] = (psi_n * da - cplx{psi, 0.0}) / (da * xi_n - xi_nm1);
        s_b[n - 1] = (psi_n * db - cplx{psi, 0.0}) / (db * xi_n - xi_nm1);
    }
    __syncthreads();
    double sum_ext = 0.0, sum_sca = 0.0, sum_g = 0.0;
    for (int n = tid + 1; n <= N; n += blockDim.x) {
        const cplx an = s_a[n - 1], bn = s_b[n - 1];
        const double w = 2.0 * n + 1.0;
        sum_ext += w * (an.re + bn.re);
        sum_sca += w * (norm2(an) + norm2(bn));
        // asymmetry: (n-1)(n+1)/n Re(a_{n-1} a_n* + b_{n-1} b_n*) + (2n+1)/(n(n+1)) Re(a_n b_n*)
        if (n > 1) {
            const cplx ap = s_a[n - 2], bp = s_b[n - 2];
            const double c = (double)(n - 1) * (n + 1) / n;
            sum_g += c * (ap.re * an.re + ap.im * an.im + bp.re * bn.re + bp.im * bn.im);
        }
        sum_g += w / ((double)n * (n + 1)) * (an.re * bn.re + an.im * bn.im);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        sum_ext += __shfl_xor(sum_ext, off, 64);
        sum_sca += __shfl_xor(sum_sca, off, 64);
        sum_g += __shfl_xor(sum_g, off, 64);
    }
    const int waves = blockDim.x >> 6;
    if ((tid & 63) == 0) {
        s_red[3 * (tid >> 6) + 0] = sum_ext;
        s_red[3 * (tid >> 6) + 1] = sum_sca;
        s_red[3 * (tid >> 6) + 2] = sum_g;
    }
    __syncthreads();
    if (tid == 0) {
        double e = 0.0, q = 0.0, g = 0.0;
        for (int w = 0; w < waves; ++w) {
            e += s_red[3 * w + 0];
            q += s_red[3 * w + 1];
            g += s_red[3 * w + 2];
        }
        const double inv_x2 = 1.0 / (x * x);
        const double q_sca = 2.0 * inv_x2 * q;
        s_sums[0] = 2.0 * inv_x2 * e;
        s_sums[1] = q_sca;
        s_sums[2] = 4.0 * inv_x2 * g / q_sca;
    }
    __syncthreads();
}

// Before step 2: fold the angular weight (2n + 1)/(n(n + 1)) of Eqs. 5-6 into
// a_n and b_n (in place) and tabulate the coefficients (2n - 1)/(n - 1) and
// n/(n - 1) of the pi_n recurrence, so the per-angle loop neither divides nor
// converts n.  Ends with a barrier.
__device__ void prepare_angular(int N, cplx *s_a, cplx *s_b, double2 *s_pi)
{
    for (int n = threadIdx.x + 1; n <= N; n += blockDim.x) {
        const double c = (2.0 * n + 1.0) / ((double)n * (n + 1));
        s_a[n - 1] = c * s_a[n - 1];
        s_b[n - 1] = c * s_b[n - 1];
        s_pi[n - 1] = n > 1 ? double2{(2.0 * n - 1.0) / (double)(n - 1), (double)n / (double)(n - 1)}
                            : double2{0.0, 0.0};
    }
    __syncthreads();
}

// Step 2 at one angle: |S1|^2 + |S2|^2 (Eqs. 5-6) with the angular functions
// upward, pi_n = ((2n - 1) mu pi_{n-1} - n pi_{n-2}) / (n - 1) from pi_0 = 0,
// pi_1 = 1, and tau_n = n mu pi_n - (n + 1) pi_{n-1}, on the coefficients
// prepared above.
__device__ double mie_intensity(double th, int N, const cplx *s_a, const cplx *s_b, const double2 *s_pi)
{
    const double mu = cos_0_pi(th);
    double pi_prev = 0.0, pi_n = 1.0;              // pi_0, pi_1
    // n = 1: tau_1 = mu
    cplx S1 = pi_n * s_a[0] + mu * s_b[0];
    cplx S2 = mu * s_a[0] + pi_n * s_b[0];
    double dn = 1.0;
    for (int n = 2; n <= N; ++n) {
        dn += 1.0;
        const double2 c = s_pi[n - 1];
        const double p = fma(c.x * mu, pi_n, -c.y * pi_prev);
        pi_prev = pi_n;
        pi_n = p;
        const double tau_n = fma(dn * mu, pi_n, -(dn + 1.0) * pi_prev);
        const cplx an = s_a[n - 1], bn = s_b[n - 1];
        S1 = {fma(pi_n, an.re, fma(tau_n, bn.re, S1.re)), fma(pi_n, an.im, fma(tau_n, bn.im, S1.im))};
        S2 = {fma(tau_n, an.re, fma(pi_n, bn.re, S2.re)), fma(tau_n, an.im, fma(pi_n, bn.im, S2.im))};
    }
    return norm2(S1) + norm2(S2);
}

// Step 2 at angle j of the na-point grid: scale x (|S1|^2 + |S2|^2) to
// phase_out[j] and, times sin(theta_j), to ang[j] (each if given).
__device__ void phase_at(int j, int na, int N, double scale, const cplx *s_a, const cplx *s_b, const double2 *s_pi,
                         double *phase_out, double *ang)
{
    const double dth = M_PI / (double)(na - 1);
    const double th = (double)j * dth;
    const double P = scale * mie_intensity(th, N, s_a, s_b, s_pi);
    if (phase_out) phase_out[j] = P;
    if (ang) ang[j] = P * sin_0_pi(th);
}

// Steps 1-2 for one size: workgroup b runs the series, workgroup 0 writes the
// scalar results (and the coefficients if asked), and lane t evaluates angle
// j = 256 b + t into work[j] = P sin(theta_j) (and phase[j] = P if asked).
__global__ __launch_bounds__(kPhaseThreads) void mie_phase_kernel(MieArgs a)
{
    __shared__ cplx s_a[MC_MAX_TERMS];
    __shared__ cplx s_b[MC_MAX_TERMS];
    __shared__ double s_rec[2 * (MC_MAX_TERMS + 1)];   // psi_n, chi_n
    __shared__ double2 s_pi[MC_MAX_TERMS];              // pi_n recurrence coefficients
    __shared__ double s_red[3 * (kPhaseThreads / 64)];
    __shared__ double s_sums[3];                       // Q_ext, Q_sca, g

    const int tid = threadIdx.x;
    const int N = a.n_terms;
    const double x = a.x;
    mie_series_block(x, a.m_re, a.m_im, N, a.n_start, s_a, s_b, s_rec, s_rec + MC_MAX_TERMS + 1, s_red, s_sums);
    if (blockIdx.x == 0) {
        if (tid == 0) {
            a.result[0] = s_sums[0];
            a.result[1] = s_sums[1];
            a.result[2] = s_sums[2];
            a.result[3] = (double)N;
        }
        if (a.coef) {
            for (int n = tid; n < N; n += kPhaseThreads) {
                a.coef[4 * n + 0] = s_a[n].re;
                a.coef[4 * n + 1] = s_a[n].im;
                a.coef[4 * n + 2] = s_b[n].re;
                a.coef[4 * n + 3] = s_b[n].im;
            }
        }
    }
    __syncthreads();
    prepare_angular(N, s_a, s_b, s_pi);
    // Phase function normalised as Eq. 10: P = 2 (|S1|^2 + |S2|^2) / (x^2 Q_sca).
    const int j = blockIdx.x * kPhaseThreads + tid;
    if (j < a.n_angles) phase_at(j, a.n_angles, N, 2.0 / (x * x * s_sums[1]), s_a, s_b, s_pi, a.phase, a.work);
}

__device__ int first_at_least(const double *f, int l, int r, double u)
{
    while (l < r) {
        const int mid = (l + r) >> 1;
        if (f[mid] < u) l = mid + 1;
        else r = mid;
    }
    return l;
}

// Steps 3-4: ang holds P sin(theta) on the na-point grid.  Every workgroup
// reads it into LDS and forms the trapezoid CDF F_j in place (F = 1 at pi):
// each lane adds the increments of its run of at most three angles, a
// shuffle scan within each wave and a scan of the wave totals give every run
// the sum before it, and each run is then accumulated in order and divided
// by the total.  Workgroup 0 writes F to cdf_out (if given).  Then lane i of
// the grid takes inverse-table entry u_i = i / (nc - 1): the first angle with
// F >= u_i by binary search, theta interpolated linearly in F, and
// v = 1 - cos(theta) = 2 sin^2(theta/2) stored in FP32.
__global__ __launch_bounds__(kInvThreads) void mie_inverse_kernel(const double *ang, int na, int nc, float *inv_cdf,
                                                                  double *cdf_out)
{
    __shared__ double s_ang[MC_MAX_N_ANGLES];
    __shared__ double s_wave[kInvThreads / 64];
    __shared__ double s_total;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int j = tid; j < na; j += kInvThreads) s_ang[j] = ang[j];
    __syncthreads();

    const double dth = M_PI / (double)(na - 1);
    const int per = (na + kInvThreads - 1) / kInvThreads;
    const int lo = min(tid * per, na), hi = min(lo + per, na);
    const double f_left = lo >= 1 && lo < na ? s_ang[lo - 1] : 0.0;
    double local = 0.0;
    for (int j = max(lo, 1); j < hi; ++j) {
        const double th_j = (double)j * dth, th_p = (double)(j - 1) * dth;
        local += 0.5 * (th_j - th_p) * (s_ang[j - 1] + s_ang[j]);
    }
    double incl = local;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    double excl = __shfl_up(incl, 1, 64);
    if (lane == 0) excl = 0.0;
    if (lane == 63) s_wave[wave] = incl;
    __syncthreads();
    if (tid == 0) {   // exclusive scan of the wave totals
        double run = 0.0;
        for (int w = 0; w < kInvThreads / 64; ++w) {
            const double v = s_wave[w];
            s_wave[w] = run;
            run += v;
        }
        s_total = run;
    }
    __syncthreads();
    double acc = s_wave[wave] + excl;
    const double total = s_total;
    double prev = f_left;
    for (int j = lo; j < hi; ++j) {
        const double f = s_ang[j];
        if (j >= 1) {
            const double th_j = (double)j * dth, th_p = (double)(j - 1) * dth;
            acc += 0.5 * (th_j - th_p) * (prev + f);
        }
        prev = f;
        s_ang[j] = (j == na - 1) ? 1.0 : acc / total;
    }
    __syncthreads();
    if (cdf_out && blockIdx.x == 0)
        for (int j = tid; j < na; j += kInvThreads) cdf_out[j] = s_ang[j];

    const int i = blockIdx.x * kInvThreads + tid;
    if (i >= nc) return;
    const double u = (double)i / (double)(nc - 1);
    // u <= 1 = F at pi, so only rounding could leave an entry past the grid.
    const int l = min(first_at_least(s_ang, 0, na, u), na - 1);
    double th = 0.0;
    if (l > 0) {
        const double th_j = (double)l * dth, th_p = (double)(l - 1) * dth;
        th = th_p + (u - s_ang[l - 1]) / (s_ang[l] - s_ang[l - 1]) * (th_j - th_p);
    }
    const double sh = sin_half_pi(0.5 * th);
    inv_cdf[i] = (float)(2.0 * sh * sh);
}

// ---- polydisperse: the bins, the mixture, then the same inverse ----------

struct PolyArgs {
    double x[MC_MAX_BINS];         // size parameter of each bin
    double c[MC_MAX_BINS];         // probability x geometric cross-section (mm^2) of each bin
    int n_terms[MC_MAX_BINS], n_start[MC_MAX_BINS];
    double m_re, m_im;
    int n_bins, n_angles, n_cdf;
    double geo_median;             // geometric cross-section of the median diameter (mm^2)
    double *rows;                  // n_bins x n_angles: c_k Q_sca,k P_k(theta_j)
    double *bins;                  // n_bins x 4: Q_ext,k, Q_sca,k, g_k, N_k
    double *ang;                   // n_angles: P(theta_j) sin(theta_j) of the mixture
    double *phase;
    double *result;                // q_ext, q_sca (over geo_median), g, max N
};

// Workgroup (s, k) runs bin k's series (workgroup (0, k) writes its scalars to
// bins) and its lanes evaluate row k at the 256 angles of slice s.
__global__ __launch_bounds__(kPhaseThreads) void mie_bin_kernel(PolyArgs a)
{
    __shared__ cplx s_a[MC_MAX_TERMS];
    __shared__ cplx s_b[MC_MAX_TERMS];
    __shared__ double s_rec[2 * (MC_MAX_TERMS + 1)];   // psi_n, chi_n
    __shared__ double2 s_pi[MC_MAX_TERMS];              // pi_n recurrence coefficients
    __shared__ double s_red[3 * (kPhaseThreads / 64)];
    __shared__ double s_sums[3];
    const int k = blockIdx.y, tid = threadIdx.x;
    const double x = a.x[k];
    const int N = a.n_terms[k];
    mie_series_block(x, a.m_re, a.m_im, N, a.n_start[k], s_a, s_b, s_rec, s_rec + MC_MAX_TERMS + 1, s_red, s_sums);
    if (blockIdx.x == 0 && tid == 0) {
        a.bins[4 * k + 0] = s_sums[0];
        a.bins[4 * k + 1] = s_sums[1];
        a.bins[4 * k + 2] = s_sums[2];
        a.bins[4 * k + 3] = (double)N;
    }
    prepare_angular(N, s_a, s_b, s_pi);
    // c_k Q_sca,k P_k with P_k = 2 (|S1|^2 + |S2|^2) / (x^2 Q_sca,k): the Q_sca,k cancel.
    const int j = blockIdx.x * kPhaseThreads + tid;
    if (j < a.n_angles)
        phase_at(j, a.n_angles, N, a.c[k] * 2.0 / (x * x), s_a, s_b, s_pi, a.rows + (uint64_t)k * a.n_angles,
                 nullptr);
}

// Lane t of workgroup b mixes the rows at angle j = 256 b + t into ang[j]
// (and phase[j]); every workgroup sums the bins' cross-sections itself, in
// bin order, and workgroup 0 writes the scalar results.
__global__ __launch_bounds__(kPhaseThreads) void mie_mix_kernel(PolyArgs a)
{
    __shared__ double s_sca;
    const int tid = threadIdx.x;
    if (tid == 0) {
        // Number-averaged cross-sections and the C_sca-weighted asymmetry, in bin order.
        double ext = 0.0, sca = 0.0, gs = 0.0, nmax = 0.0;
#pragma unroll 8
        for (int k = 0; k < a.n_bins; ++k) {
            const double q_ext = a.bins[4 * k + 0], q_sca = a.bins[4 * k + 1];
            const double g = a.bins[4 * k + 2], n = a.bins[4 * k + 3];
            ext += a.c[k] * q_ext;
            sca += a.c[k] * q_sca;
            gs += a.c[k] * q_sca * g;
            nmax = fmax(nmax, n);
        }
        s_sca = sca;
        if (blockIdx.x == 0) {
            a.result[0] = ext / a.geo_median;
            a.result[1] = sca / a.geo_median;
            a.result[2] = gs / sca;
            a.result[3] = nmax;
        }
    }
    __syncthreads();
    const int na = a.n_angles;
    const int j = blockIdx.x * kPhaseThreads + tid;
    if (j >= na) return;
    const double dth = M_PI / (double)(na - 1);
    // The rows added in bin order, their loads issued eight at a time.
    double mix = 0.0;
    int k = 0;
    for (; k + 8 <= a.n_bins; k += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = a.rows[(uint64_t)(k + u) * na + j];
#pragma unroll
        for (int u = 0; u < 8; ++u) mix += v[u];
    }
    for (; k < a.n_bins; ++k) mix += a.rows[(uint64_t)k * na + j];
    const double P = mix * (1.0 / s_sca);
    if (a.phase) a.phase[j] = P;
    a.ang[j] = P * sin_0_pi((double)j * dth);
}

// Per-device scratch for the scalar results (8 doubles) and the angle grid
// (MC_MAX_N_ANGLES doubles) of synchronous builds whose caller passes none
// (allocated once per device, kept until the process ends).
constexpr size_t kScratchDoubles = 8 + MC_MAX_N_ANGLES;
std::mutex g_scratch_mu;
double *g_scratch[64] = {nullptr};

// Validate the spec and derive x, m and the series length (no device work).
int prepare_table(const mie_spec_t *spec, const mie_table_t *table, MieArgs *args, const char *who)
{
    if (!spec || !table) return fail(MC_EINVAL, "%s: null spec or table", who);
    const mie_spec_t s = *spec;
    if (!(s.n_medium > 0) || !(s.m_re > 0) || !(s.m_im >= 0) || !(s.diameter_um > 0) ||
        !(s.wavelength_nm > 0) || !std::isfinite(s.n_medium * s.m_re * s.m_im * s.diameter_um *
                                                   s.wavelength_nm))
        return fail(MC_EINVAL, "%s: indices, diameter and wavelength must be finite, positive (m_im >= 0)", who);
    if (s.n_angles < 3 || s.n_angles > MC_MAX_N_ANGLES)
        return fail(MC_EINVAL, "%s: n_angles %d outside 3..%d", who, s.n_angles, MC_MAX_N_ANGLES);
    if (s.n_cdf < 2 || s.n_cdf > MC_MAX_N_CDF)
        return fail(MC_EINVAL, "%s: n_cdf %d outside 2..%d", who, s.n_cdf, MC_MAX_N_CDF);
    if (!table->inv_cdf) return fail(MC_EINVAL, "%s: inv_cdf buffer is required", who);

    // Parameter processing (Sec. 3.1.1): x = pi d n_med / lambda0 (Eq. 3 with
    // the wavelength in the medium), m relative to the medium (Eq. 4).
    const double x = M_PI * s.diameter_um * 1e3 * s.n_medium / s.wavelength_nm;
    const double m_re = s.m_re / s.n_medium, m_im = s.m_im / s.n_medium;
    const double mx_abs = x * std::hypot(m_re, m_im);
    if (!(x >= 1e-6)) return fail(MC_EINVAL, "%s: size parameter %g below 1e-6", who, x);
    if (!(mx_abs >= 1e-6)) return fail(MC_EINVAL, "%s: |m| x = %g below 1e-6", who, mx_abs);
    const int n_terms = (int)std::lround(x + 4.0 * std::cbrt(x) + 2.0);   // Wiscombe 1980
    if (n_terms > MC_MAX_TERMS)
        return fail(MC_EINVAL, "%s: %d series terms exceed %d (x = %g)", who, n_terms, MC_MAX_TERMS, x);
    if (table->coef && table->coef_capacity < n_terms)
        return fail(MC_EINVAL, "%s: coef holds %d terms, %d needed", who, table->coef_capacity, n_terms);
    // Downward start: the start error decays slowly across the turning point
    // n ~ |mx|, whose width grows like |mx|^(1/3).
    const int n_start = (int)std::ceil(std::max((double)n_terms, mx_abs)) + 16 +
                        (int)std::ceil(8.0 * std::cbrt(mx_abs));

    *args = MieArgs{x, m_re, m_im, n_terms, n_start, s.n_angles, s.n_cdf,
                    table->inv_cdf, table->phase, table->cdf, table->coef, nullptr, nullptr};
    return MC_OK;
}

// Launch the prepared table kernels on `st`: scalar results to `result`,
// the angle grid through `work` (both device).
int launch_table(MieArgs args, mie_table_t *table, hipStream_t st, double *result, double *work)
{
    args.result = result;
    args.work = work;
    const int g_phase = (args.n_angles + kPhaseThreads - 1) / kPhaseThreads;
    const int g_inv = (args.n_cdf + kInvThreads - 1) / kInvThreads;
    hipLaunchKernelGGL(mie_phase_kernel, dim3(g_phase), dim3(kPhaseThreads), 0, st, args);
    hipLaunchKernelGGL(mie_inverse_kernel, dim3(g_inv), dim3(kInvThreads), 0, st, (const double *)work, args.n_angles,
                       args.n_cdf, args.inv_cdf, args.cdf);
    MC_HIP_CHECK(hipGetLastError());
    table->x = args.x;
    table->m_rel_re = args.m_re;
    table->m_rel_im = args.m_im;
    table->n_terms = args.n_terms;
    table->n_cdf = args.n_cdf;
    return MC_OK;
}

void set_scalars(mie_table_t *table, const mie_spec_t &s, const double res[3])
{
    const double geo_mm2 = M_PI * (s.diameter_um * 1e-3) * (s.diameter_um * 1e-3) / 4.0;   // Eq. 14
    table->q_ext = res[0];
    table->q_sca = res[1];
    table->q_abs = res[0] - res[1];
    table->g = res[2];
    table->sigma_ext_mm2 = res[0] * geo_mm2;
    table->sigma_sca_mm2 = res[1] * geo_mm2;
    table->sigma_abs_mm2 = (res[0] - res[1]) * geo_mm2;
}

// The caller's result buffer and (if `work` is not null) angle-grid buffer,
// or for each one missing the library's per-device scratch (then `lock`
// holds the scratch until the results are back on the host).
int scratch_buffers(const mie_table_t *table, std::unique_lock<std::mutex> &lock, double **result, double **work,
                    const char *who)
{
    *result = table->result;
    if (work) *work = table->work;
    if (*result && (!work || *work)) return MC_OK;
    int dev = 0;
    MC_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(MC_EDEVICE, "device index %d out of range", dev);
    lock.lock();
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipMalloc(&p, kScratchDoubles * sizeof(double)) != hipSuccess)
            return fail(MC_ENOMEM, "%s: scratch allocation failed", who);
        g_scratch[dev] = (double *)p;
    }
    if (!*result) *result = g_scratch[dev];
    if (work && !*work) *work = g_scratch[dev] + 8;
    return MC_OK;
}

// Orthonormal Hermite polynomial h_n(t) for the weight exp(-t^2), by the
// three-term recurrence h_{j+1} = sqrt(2/(j+1)) t h_j - sqrt(j/(j+1)) h_{j-1}
// from h_0 = pi^(-1/4), together with sum_{j<n} h_j(t)^2.
struct HermiteCoef {
    double a[MC_MAX_BINS], b[MC_MAX_BINS];   // sqrt(2 / (j + 1)), sqrt(j / (j + 1))
};

void hermite_orthonormal(const HermiteCoef &c, int n, double t, double *h_n, double *sum_sq)
{
    double h_prev = 0.0, h = std::pow(M_PI, -0.25), s = 0.0;
    for (int j = 0; j < n; ++j) {
        s += h * h;
        const double h_next = c.a[j] * t * h - c.b[j] * h_prev;
        h_prev = h;
        h = h_next;
    }
    *h_n = h;
    *sum_sq = s;
}

// Gauss-Hermite rule for the weight exp(-t^2): the nodes are the n roots of
// h_n, all inside (-sqrt(2n+1), sqrt(2n+1)); each is bracketed by a sign
// change on a grid far finer than the root spacing and bisected to machine
// precision.  The weights are the Christoffel numbers 1 / sum_{j<n} h_j(t)^2.
int gauss_hermite(int n, double *t, double *w)
{
    if (n == 1) {
        t[0] = 0.0;
        w[0] = std::sqrt(M_PI);
        return MC_OK;
    }
    HermiteCoef c;
    for (int j = 0; j < n; ++j) {
        c.a[j] = std::sqrt(2.0 / (j + 1));
        c.b[j] = std::sqrt((double)j / (j + 1));
    }
    // Grid step 2R / (40 n) < 0.04 for n <= 64, well below the smallest
    // spacing of neighbouring roots (about pi / sqrt(2n + 1) > 0.27).
    const double R = std::sqrt(2.0 * n + 1.0) + 1.0;
    const int steps = 40 * n;
    int found = 0;
    double t_prev = -R, h_prev, s;
    hermite_orthonormal(c, n, t_prev, &h_prev, &s);
    for (int i = 1; i <= steps && found < n; ++i) {
        const double ti = -R + 2.0 * R * (double)i / steps;
        double hi;
        hermite_orthonormal(c, n, ti, &hi, &s);
        if ((h_prev < 0.0) != (hi < 0.0) || hi == 0.0) {
            double lo = t_prev, up = ti, h_lo = h_prev;
            for (int it = 0; it < 200 && hi != 0.0; ++it) {
                const double mid = 0.5 * (lo + up);
                if (mid <= lo || mid >= up) break;
                double hm;
                hermite_orthonormal(c, n, mid, &hm, &s);
                if ((hm < 0.0) == (h_lo < 0.0)) {
                    lo = mid;
                    h_lo = hm;
                } else {
                    up = mid;
                }
            }
            const double root = hi == 0.0 ? ti : 0.5 * (lo + up);
            double hr;
            hermite_orthonormal(c, n, root, &hr, &s);
            t[found] = root;
            w[found] = 1.0 / s;
            ++found;
            // Step past an exact zero so it is not found twice.
            hermite_orthonormal(c, n, ti, &hi, &s);
            if (hi == 0.0) hi = -h_prev;
        }
        t_prev = ti;
        h_prev = hi;
    }
    return found == n ? MC_OK : fail(MC_EINVAL, "Gauss-Hermite: found %d of %d nodes", found, n);
}

int lognormal_bins(double median_um, double sigma_ln, int n, double *d, double *p)
{
    if (!(median_um > 0.0) || !std::isfinite(median_um) || !(sigma_ln >= 0.0) || !std::isfinite(sigma_ln))
        return fail(MC_EINVAL, "lognormal bins: median must be > 0 and sigma_ln >= 0, both finite");
    if (n < 1 || n > MC_MAX_BINS) return fail(MC_EINVAL, "lognormal bins: n_bins %d outside 1..%d", n, MC_MAX_BINS);
    double t[MC_MAX_BINS], w[MC_MAX_BINS];
    if (int rc = gauss_hermite(n, t, w)) return rc;
    for (int k = 0; k < n; ++k) {
        d[k] = median_um * std::exp(std::sqrt(2.0) * sigma_ln * t[k]);
        p[k] = w[k] / std::sqrt(M_PI);
    }
    return MC_OK;
}

uint64_t poly_work_words(int n_angles, int n_bins) { return (uint64_t)n_bins * n_angles + 4ull * n_bins + n_angles; }

}  // namespace
}  // namespace mcmie

extern "C" int mc_lognormal_bins(double median_um, double sigma_ln, int32_t n_bins, double *diameters_um,
                                 double *probs)
{
    using namespace mcmie;
    clear_error();
    if (!diameters_um || !probs) return fail(MC_EINVAL, "mc_lognormal_bins: null output");
    return lognormal_bins(median_um, sigma_ln, n_bins, diameters_um, probs);
}

extern "C" uint64_t mie_poly_work_bytes(const mie_spec_t *spec, const mie_poly_t *poly)
{
    if (!spec || !poly || spec->n_angles < 3 || spec->n_angles > MC_MAX_N_ANGLES || poly->n_bins < 1 ||
        poly->n_bins > MC_MAX_BINS)
        return 0;
    return mcmie::poly_work_words(spec->n_angles, poly->n_bins) * 8;
}

extern "C" int mie_table_build_poly(const mie_spec_t *spec, const mie_poly_t *poly, mie_table_t *table, void *stream)
{
    using namespace mcmie;
    clear_error();
    const char *who = "mie_table_build_poly";
    MieArgs med;
    if (int rc = prepare_table(spec, table, &med, who)) return rc;
    if (!poly) return fail(MC_EINVAL, "%s: null poly", who);
    const mie_spec_t s = *spec;
    const mie_poly_t q = *poly;
    if (table->coef) return fail(MC_EINVAL, "%s: coef is not produced for a size distribution (set it to NULL)", who);
    if (!q.work || ((uintptr_t)q.work & 7) || q.work_bytes < poly_work_words(s.n_angles, q.n_bins) * 8)
        return fail(MC_EINVAL, "%s: work needs %llu bytes, 8-byte aligned", who,
                    (unsigned long long)(poly_work_words(s.n_angles, std::max(1, q.n_bins)) * 8));
    double d[MC_MAX_BINS], p[MC_MAX_BINS];
    if (int rc = lognormal_bins(s.diameter_um, q.sigma_ln, q.n_bins, d, p)) return rc;
    PolyArgs a{};
    a.m_re = med.m_re;
    a.m_im = med.m_im;
    a.n_bins = q.n_bins;
    a.n_angles = s.n_angles;
    a.n_cdf = s.n_cdf;
    for (int k = 0; k < q.n_bins; ++k) {
        // Each bin's parameters as prepare_table derives them for one size.
        const double x = M_PI * d[k] * 1e3 * s.n_medium / s.wavelength_nm;
        const double mx_abs = x * std::hypot(med.m_re, med.m_im);
        const int n_terms = (int)std::lround(x + 4.0 * std::cbrt(x) + 2.0);
        if (n_terms > MC_MAX_TERMS)
            return fail(MC_EINVAL, "%s: bin %d needs %d series terms, more than %d", who, k, n_terms, MC_MAX_TERMS);
        a.x[k] = x;
        a.n_terms[k] = n_terms;
        a.n_start[k] = (int)std::ceil(std::max((double)n_terms, mx_abs)) + 16 + (int)std::ceil(8.0 * std::cbrt(mx_abs));
        a.c[k] = p[k] * M_PI * (d[k] * 1e-3) * (d[k] * 1e-3) / 4.0;
    }
    a.geo_median = M_PI * (s.diameter_um * 1e-3) * (s.diameter_um * 1e-3) / 4.0;
    a.rows = q.work;
    a.bins = q.work + (uint64_t)q.n_bins * s.n_angles;
    a.ang = a.bins + 4ull * q.n_bins;
    a.phase = table->phase;
    std::unique_lock<std::mutex> lock(g_scratch_mu, std::defer_lock);
    if (int rc = scratch_buffers(table, lock, &a.result, nullptr, who)) return rc;
    hipStream_t st = (hipStream_t)stream;
    const int slices = (s.n_angles + kPhaseThreads - 1) / kPhaseThreads;
    hipLaunchKernelGGL(mie_bin_kernel, dim3(slices, q.n_bins), dim3(kPhaseThreads), 0, st, a);
    hipLaunchKernelGGL(mie_mix_kernel, dim3(slices), dim3(kPhaseThreads), 0, st, a);
    hipLaunchKernelGGL(mie_inverse_kernel, dim3((s.n_cdf + kInvThreads - 1) / kInvThreads), dim3(kInvThreads), 0, st,
                       (const double *)a.ang, s.n_angles, s.n_cdf, table->inv_cdf, table->cdf);
    MC_HIP_CHECK(hipGetLastError());
    double res[4];
    MC_HIP_CHECK(hipMemcpyAsync(res, a.result, sizeof res, hipMemcpyDeviceToHost, st));
    MC_HIP_CHECK(hipStreamSynchronize(st));
    table->x = med.x;
    table->m_rel_re = med.m_re;
    table->m_rel_im = med.m_im;
    table->n_terms = (int)res[3];
    table->n_cdf = s.n_cdf;
    set_scalars(table, s, res);
    return MC_OK;
}

extern "C" int mie_table_build(const mie_spec_t *spec, mie_table_t *table, void *stream)
{
    using namespace mcmie;
    clear_error();
    hipStream_t st = (hipStream_t)stream;
    MieArgs args;
    if (int rc = prepare_table(spec, table, &args, "mie_table_build")) return rc;
    double *result = nullptr, *work = nullptr;
    std::unique_lock<std::mutex> lock(g_scratch_mu, std::defer_lock);
    if (int rc = scratch_buffers(table, lock, &result, &work, "mie_table_build")) return rc;
    if (int rc = launch_table(args, table, st, result, work)) return rc;
    double res[4];
    MC_HIP_CHECK(hipMemcpyAsync(res, result, sizeof res, hipMemcpyDeviceToHost, st));
    MC_HIP_CHECK(hipStreamSynchronize(st));
    set_scalars(table, *spec, res);
    return MC_OK;
}

extern "C" int mie_table_enqueue(const mie_spec_t *spec, mie_table_t *table, void *stream)
{
    using namespace mcmie;
    clear_error();
    MieArgs args;
    if (int rc = prepare_table(spec, table, &args, "mie_table_enqueue")) return rc;
    if (!table->result) return fail(MC_EINVAL, "mie_table_enqueue: result buffer is required");
    if (!table->work) return fail(MC_EINVAL, "mie_table_enqueue: work buffer (n_angles doubles) is required");
    if (int rc = launch_table(args, table, (hipStream_t)stream, table->result, table->work)) return rc;
    const double nan3[3] = {NAN, NAN, NAN};
    set_scalars(table, *spec, nan3);
    return MC_OK;
}
