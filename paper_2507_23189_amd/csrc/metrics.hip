// Image comparison measures of Sec. 5.2 (Tables 3 and 4) on the device.
//
// Both images are divided by their largest pixel.  Over pixels: RMSE of the
// difference and Pearson's r.  Radially: the normalised images averaged over
// annuli one pixel wide around (cx, cy) out to r_max (annulus k holds
// k <= rho < k + 1, rho from the pixel centre (j + 0.5, i + 0.5), computed
// from rho^2, exact for such centres), zones by theta = 180 deg (k + 0.5) /
// r_max (< 30, 30..120, > 120 deg) with the RMSE of the two profiles in each,
// Pearson's r of the profiles, and, given a third image c, the share of
// annuli where a is closer to b than c is.
//
// Three kernels: block maxima; per-block pixel sums (fixed partition, tree
// reductions) with the annulus sums in int64 fixed point (2^38 per unit, so
// their totals do not depend on the order of the atomics); one workgroup for
// the totals, profiles and measures.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "common.hpp"

namespace mcmie {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxGrid = 256;
constexpr double kRadFix = 274877906944.0;     // 2^38
constexpr int kPix = 7;                        // pixel sums per block: n, x, y, xx, yy, xy, (x - y)^2

struct MetricsArgs {
    const double *a, *b, *c;
    int nx, ny;
    double cx, cy, r_max;
    int n_r;
    uint64_t n_pix, per_block;
    double *blk_max;                 // grid x 3
    double *blk_sum;                 // grid x kPix
    unsigned long long *rad;         // n_r x 4: pixels, a, b, c (fixed point)
    double *out;                     // MC_METRICS_N
    double *profiles;                // optional: 4 x n_r (a, b, c profiles, pixel counts)
};

__device__ double block_max(double v, double *s)
{
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + off]);
        __syncthreads();
    }
    const double r = s[0];
    __syncthreads();
    return r;
}

__device__ double block_sum(double v, double *s)
{
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    const double r = s[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kThreads) void metrics_max(MetricsArgs m)
{
    __shared__ double s[kThreads];
    const uint64_t lo = (uint64_t)blockIdx.x * m.per_block;
    const uint64_t hi = lo + m.per_block < m.n_pix ? lo + m.per_block : m.n_pix;
    double ma = 0.0, mb = 0.0, mc = 0.0;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
        ma = fmax(ma, m.a[i]);
        mb = fmax(mb, m.b[i]);
        if (m.c) mc = fmax(mc, m.c[i]);
    }
    ma = block_max(ma, s);
    mb = block_max(mb, s);
    mc = block_max(mc, s);
    if (threadIdx.x == 0) {
        m.blk_max[3 * blockIdx.x + 0] = ma;
        m.blk_max[3 * blockIdx.x + 1] = mb;
        m.blk_max[3 * blockIdx.x + 2] = mc;
    }
    // Clear the annulus sums for the next kernel.
    for (int i = blockIdx.x * kThreads + threadIdx.x; i < 4 * m.n_r; i += gridDim.x * kThreads) m.rad[i] = 0ull;
}

__global__ __launch_bounds__(kThreads) void metrics_sums(MetricsArgs m)
{
    extern __shared__ __attribute__((aligned(16))) unsigned long long s_rad[];   // 4 x n_r
    __shared__ double s[kThreads];
    __shared__ double s_inv[3];
    if (threadIdx.x == 0) {
        double ma = 0.0, mb = 0.0, mc = 0.0;
        for (int g = 0; g < (int)gridDim.x; ++g) {
            ma = fmax(ma, m.blk_max[3 * g + 0]);
            mb = fmax(mb, m.blk_max[3 * g + 1]);
            mc = fmax(mc, m.blk_max[3 * g + 2]);
        }
        s_inv[0] = ma > 0.0 ? 1.0 / ma : 0.0;
        s_inv[1] = mb > 0.0 ? 1.0 / mb : 0.0;
        s_inv[2] = mc > 0.0 ? 1.0 / mc : 0.0;
        if (blockIdx.x == 0) {
            m.out[7] = ma;
            m.out[8] = mb;
            m.out[9] = mc;
        }
    }
    for (int i = threadIdx.x; i < 4 * m.n_r; i += kThreads) s_rad[i] = 0ull;
    __syncthreads();
    const double ia = s_inv[0], ib = s_inv[1], ic = s_inv[2];
    const uint64_t lo = (uint64_t)blockIdx.x * m.per_block;
    const uint64_t hi = lo + m.per_block < m.n_pix ? lo + m.per_block : m.n_pix;
    double acc[kPix] = {0, 0, 0, 0, 0, 0, 0};
    const double r2max = m.r_max * m.r_max;
    for (uint64_t i = lo + threadIdx.x; i < hi; i += kThreads) {
        // Normalised by the largest pixel (a zero image stays zero).
        const double x = m.a[i] * ia, y = m.b[i] * ib;
        acc[0] += 1.0;
        acc[1] += x;
        acc[2] += y;
        acc[3] += x * x;
        acc[4] += y * y;
        acc[5] += x * y;
        acc[6] += (x - y) * (x - y);
        const int row = (int)(i / (uint64_t)m.nx), col = (int)(i % (uint64_t)m.nx);
        const double dx = (col + 0.5) - m.cx, dy = (row + 0.5) - m.cy;
        const double r2 = dx * dx + dy * dy;
        if (r2 < r2max) {
            const int k = min((int)floor(sqrt(r2)), m.n_r - 1);
            atomicAdd(&s_rad[4 * k + 0], 1ull);
            atomicAdd(&s_rad[4 * k + 1], (unsigned long long)llrint(x * kRadFix));
            atomicAdd(&s_rad[4 * k + 2], (unsigned long long)llrint(y * kRadFix));
            if (m.c) atomicAdd(&s_rad[4 * k + 3], (unsigned long long)llrint(m.c[i] * ic * kRadFix));
        }
    }
    for (int j = 0; j < kPix; ++j) {
        const double t = block_sum(acc[j], s);
        if (threadIdx.x == 0) m.blk_sum[kPix * blockIdx.x + j] = t;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 4 * m.n_r; i += kThreads)
        if (s_rad[i]) atomicAdd(&m.rad[i], s_rad[i]);
}

__global__ __launch_bounds__(kThreads) void metrics_final(MetricsArgs m, int grid)
{
    if (threadIdx.x != 0) return;
    double t[kPix] = {0, 0, 0, 0, 0, 0, 0};
    for (int g = 0; g < grid; ++g)
        for (int j = 0; j < kPix; ++j) t[j] += m.blk_sum[kPix * g + j];
    const double n = t[0];
    m.out[0] = n > 0.0 ? sqrt(t[6] / n) : NAN;
    const double cov = t[5] - t[1] * t[2] / n, vx = t[3] - t[1] * t[1] / n, vy = t[4] - t[2] * t[2] / n;
    const double den = sqrt(vx * vy);
    m.out[1] = den > 0.0 ? cov / den : NAN;
    // Radial profiles and the measures over non-empty annuli.
    double zs[3] = {0, 0, 0}, zn[3] = {0, 0, 0};
    double used = 0.0, sa = 0.0, sb = 0.0, better = 0.0;
    for (int k = 0; k < m.n_r; ++k) {
        const double cnt = (double)m.rad[4 * k + 0];
        const double pa = cnt > 0 ? (double)m.rad[4 * k + 1] / kRadFix / cnt : 0.0;
        const double pb = cnt > 0 ? (double)m.rad[4 * k + 2] / kRadFix / cnt : 0.0;
        const double pc = cnt > 0 ? (double)m.rad[4 * k + 3] / kRadFix / cnt : 0.0;
        if (m.profiles) {
            m.profiles[k] = pa;
            m.profiles[m.n_r + k] = pb;
            m.profiles[2 * m.n_r + k] = pc;
            m.profiles[3 * m.n_r + k] = cnt;
        }
        if (cnt > 0) {
            const double theta = 180.0 * (k + 0.5) / m.r_max;
            const int z = theta < 30.0 ? 0 : (theta <= 120.0 ? 1 : 2);
            zs[z] += (pa - pb) * (pa - pb);
            zn[z] += 1.0;
            used += 1.0;
            sa += pa;
            sb += pb;
            if (m.c && fabs(pa - pb) < fabs(pc - pb)) better += 1.0;
        }
    }
    for (int z = 0; z < 3; ++z) m.out[2 + z] = zn[z] > 0 ? sqrt(zs[z] / zn[z]) : 0.0;
    const double ma = used > 0 ? sa / used : 0.0, mb = used > 0 ? sb / used : 0.0;
    double cab = 0.0, caa = 0.0, cbb = 0.0;
    for (int k = 0; k < m.n_r; ++k) {
        const double cnt = (double)m.rad[4 * k + 0];
        if (cnt <= 0) continue;
        const double pa = (double)m.rad[4 * k + 1] / kRadFix / cnt - ma;
        const double pb = (double)m.rad[4 * k + 2] / kRadFix / cnt - mb;
        cab += pa * pb;
        caa += pa * pa;
        cbb += pb * pb;
    }
    const double rden = sqrt(caa * cbb);
    m.out[5] = rden > 0.0 ? cab / rden : NAN;
    m.out[6] = (double)m.n_r;
    m.out[10] = m.c ? (used > 0 ? better / used : NAN) : NAN;
    m.out[11] = n;
}

uint64_t grid_for(uint64_t n_pix)
{
    uint64_t g = (n_pix + kThreads * 16 - 1) / (kThreads * 16);
    return g < 1 ? 1 : (g > kMaxGrid ? kMaxGrid : g);
}

uint64_t metrics_work_words(uint64_t n_pix, int n_r)
{
    const uint64_t g = grid_for(n_pix);
    return g * 3 + g * kPix + 4ull * n_r + MC_METRICS_N;
}

int annuli(const mc_radial_t &r) { return (int)std::ceil(r.r_max); }

}  // namespace
}  // namespace mcmie

extern "C" uint64_t mc_metrics_work_bytes(int32_t nx, int32_t ny, const mc_radial_t *radial)
{
    using namespace mcmie;
    if (nx < 1 || ny < 1 || !radial || !(radial->r_max > 0.0) || annuli(*radial) > MC_MAX_ANNULI) return 0;
    return metrics_work_words((uint64_t)nx * ny, annuli(*radial)) * 8;
}

extern "C" int mc_image_metrics(const double *a, const double *b, const double *c, int32_t nx, int32_t ny,
                                const mc_radial_t *radial, double *profiles, void *work, uint64_t work_bytes,
                                double out[MC_METRICS_N], void *stream)
{
    using namespace mcmie;
    clear_error();
    if (!a || !b || !radial || !work || !out) return fail(MC_EINVAL, "mc_image_metrics: null argument");
    if (nx < 1 || ny < 1 || (uint64_t)nx * ny > (1ull << 24))
        return fail(MC_EINVAL, "mc_image_metrics: image of %d x %d outside 1 .. 2^24 pixels", nx, ny);
    const mc_radial_t r = *radial;
    if (!std::isfinite(r.cx) || !std::isfinite(r.cy) || !(r.r_max > 0.0) || !std::isfinite(r.r_max) ||
        annuli(r) > MC_MAX_ANNULI)
        return fail(MC_EINVAL, "mc_image_metrics: need a finite centre and 0 < r_max <= %d", MC_MAX_ANNULI);
    const uint64_t n_pix = (uint64_t)nx * ny;
    const int n_r = annuli(r);
    if (((uintptr_t)work & 7) || work_bytes < metrics_work_words(n_pix, n_r) * 8)
        return fail(MC_EINVAL, "mc_image_metrics: work needs %llu bytes, 8-byte aligned",
                    (unsigned long long)(metrics_work_words(n_pix, n_r) * 8));
    const uint64_t g = grid_for(n_pix);
    MetricsArgs m{};
    m.a = a; m.b = b; m.c = c;
    m.nx = nx; m.ny = ny;
    m.cx = r.cx; m.cy = r.cy; m.r_max = r.r_max;
    m.n_r = n_r;
    m.n_pix = n_pix;
    m.per_block = (n_pix + g - 1) / g;
    double *w = (double *)work;
    m.blk_max = w;
    m.blk_sum = w + 3 * g;
    m.rad = (unsigned long long *)(w + 3 * g + kPix * g);
    m.out = w + 3 * g + kPix * g + 4ull * n_r;
    m.profiles = profiles;
    hipStream_t st = (hipStream_t)stream;
    const size_t lds = (size_t)4 * n_r * sizeof(unsigned long long);
    MC_HIP_CHECK(hipFuncSetAttribute((const void *)metrics_sums, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(metrics_max, dim3((unsigned)g), dim3(kThreads), 0, st, m);
    hipLaunchKernelGGL(metrics_sums, dim3((unsigned)g), dim3(kThreads), lds, st, m);
    hipLaunchKernelGGL(metrics_final, dim3(1), dim3(kThreads), 0, st, m, (int)g);
    MC_HIP_CHECK(hipGetLastError());
    MC_HIP_CHECK(hipMemcpyAsync(out, m.out, MC_METRICS_N * sizeof(double), hipMemcpyDeviceToHost, st));
    MC_HIP_CHECK(hipStreamSynchronize(st));
    return MC_OK;
}
