// The photon walk of Sec. 3.1.3 on gfx950.
//
// Each lane carries one photon at a time in registers (position, direction,
// weight, path length, scatter count, step) and runs the walk one step per
// loop trip.  When a lane's photon ends it takes the next photon id from its
// wave's current id range; a wave claims ranges of `chunk` ids from a global
// counter with one atomic, so lanes stay busy until the budget is spent and
// the work counter sees one atomic per chunk rather than per photon.
//
// One step: a Philox4x32-10 block (counter = step, instance, id_lo, id_hi;
// key = seed) gives four uniforms u0..u3; the free path s = -ln(u0)/mu_ext
// (Eq. 15) is compared with the distance to the nearest wall.  Reaching the
// wall first, the photon moves there and is reflected with the unpolarised
// Fresnel reflectance (u3) or leaves and is tallied.  Otherwise it interacts:
// the weight update of Eq. 16 (implicit capture), Russian roulette (u3), and
// a new direction at the polar angle read from the LDS-resident inverse CDF
// (u1, direct index and linear interpolation of v = 1 - cos(theta)) or from
// Henyey-Greenstein (Eq. 11), with azimuth 2 pi u2, built in the orthonormal
// basis of Duff et al. 2017 around the old direction.
//
// The kernel is bound by VALU issue.  On gfx950 a wave64 FP32 add, multiply
// or fma whose operands are all vector registers issues in 2 cycles, while
// compares, selects, min/max, conversions, shifts, 32-bit products and any
// FP32 operation with a scalar-register operand take 4 and transcendentals
// 8.  The step is written for that: its FP32 constants sit in vector
// registers, the wall distances need neither compares nor selects, and
// guards the arithmetic already ensures are left out.
//
// Transport runs in FP32.  Weights are tallied in 64-bit fixed point
// (weight * 2^32, rounded to nearest): integer sums do not depend on the order
// in which photons finish, so results are bit-identical for any launch shape
// and for either tally path.  Exits through the imaged faces are first queued
// per wave in LDS and handled 64 at a time by the whole wave, so the pixel
// arithmetic runs with full lanes instead of on the few lanes that exit in
// any one step.  A flush then either
//   * appends them to the exit log (MC_EXIT_LOG): each block owns a region
//     of every key range and appends at the position an LDS counter of the
//     block hands out (one LDS add and one store per exit); a second kernel
//     (log_bin) sums each range in an LDS histogram and writes the sums into
//     image copies with plain loads and stores; or
//   * adds them into a per-block LDS tally cache (direct-mapped pixel ids
//     claimed with an LDS compare-and-swap) whose sums go to the images once
//     per block, with a global atomic into one of eight per-XCD copies of the
//     images for the pixels that miss the cache.
// On gfx950 every global image atomic is performed at the memory side, so the
// log, which needs none, is the faster path.  Unscattered photons all leave
// through one pixel with one weight and are only counted.  A finalize pass
// sums the copies in integer arithmetic and converts to the caller's images.
// Scalar tallies use LDS atomics and lane accumulators, flushed once per
// block; reflections are not counted but derived from the step, event and
// exit counts when finalizing.  The kernel is specialised at compile time on the phase function,
// the squared-weight tally, per-photon records, path moments, batching and
// the exit log.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cmath>
#include <cstdint>
#include <algorithm>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "philox.hpp"

// Device scratch of mc_simulate_noalloc: the scalar words and one fixed-point
// copy of the images (and squared-weight images), for callers that cannot
// allocate a workspace.  Every GPU the library runs on holds its own copy
// until the process ends.
constexpr unsigned long long kNoAllocWords = 32 + (1ull << 21);
static __device__ __align__(256) unsigned long long scratch[kNoAllocWords];

namespace mcmie {
namespace {

// One medium of a batched launch, in the order its work units are handed out.
struct BatchInst {
    float neg_ln2_over_mu, albedo, absorb, pad;   // as WalkArgs, for this medium
    const float *inv_cdf;     // device inverse table of this medium (n_cdf entries)
    uint64_t n_photons;
    uint64_t unit_begin;      // first work unit of this medium
    uint32_t counter;         // Philox counter word 1 of its photons
    uint32_t slot;            // index of its images and scalars in the caller's arrays
};

struct WalkArgs {
    float size[3];
    float neg_ln2_over_mu;    // s = log2(u0) * neg_ln2_over_mu  (= -ln(u0) / mu_ext)
    float albedo, absorb;     // albedo and 1 - albedo
    float n21, n12sq;         // n_out / n_med and (n_med / n_out)^2
    float n12;                // n_med / n_out (exit refraction, records only)
    int matched;              // n_out == n_med: no Fresnel term
    float pos0[3], dir0[3], w0;
    float beam_radius;        // > 0: entry points uniform on the disk of this radius around pos0
    float roulette_w, roulette_p, inv_roulette_p;
    int phase, n_cdf;
    const float *inv_cdf;
    float hg_a, hg_b, hg_c, hg_d;   // 1 + g, 2g, 1 - g^2, 1 - g
    uint32_t key0, key1, instance, max_steps;
    uint64_t n_photons, photon_offset;
    uint32_t chunk;
    uint32_t refill_min;      // free lanes that trigger end-of-photon work and refill (1..64)
    uint32_t flags;
    int cache_bits;           // log2 of the tally-cache slots (0: no cache)
    uint32_t n_side;          // pixels of the side image (cache key offset of the transmitted image)
    int side_nx, side_ny, trans_nx, trans_ny;
    // Pixels per mm: side rows (y), side columns (z), transmitted rows (y),
    // transmitted columns (x).
    float pix_scale[4];
    unsigned long long *ws_scal;   // workspace: 16 fixed-point scalar sums, work counter at MC_S_RESERVED
    unsigned long long *ws_img;    // workspace: kCopies x n_pix fixed-point weight sums
    unsigned long long *ws_img2;   // workspace (MC_SIGMA): kCopies x n_pix squared-weight sums
    uint64_t n_pix;
    uint32_t copy_mask;       // image copy of a wave: XCC_ID & copy_mask (kCopies - 1, or 0 for one copy)
    int32_t *rec_i;
    float *rec_f;
    double *side_wk, *side_wl;     // MC_MOMENTS: per side pixel, sum w k and sum w L
    double *side_w2k, *side_w2l;   // MC_MOMENTS_PIXEL2: per side pixel, sum w^2 k and sum w^2 L
    uint64_t rec_rows, record_stride;
    // Exit log (kOptLog): block b's entries of key range r occupy
    // log[(r * gridDim.x + b) * log_cap ...], their number (at most log_cap)
    // is log_count[r * gridDim.x + b], written when the block ends.
    unsigned long long *log;
    uint32_t *log_count;
    uint32_t log_cap, log_bits;      // log_bits: scrambled group index width, >= log_rbits
    uint32_t log_rbits;              // key ranges: 2^log_rbits
    // Batched launch: media in schedule order, work units over all of them.
    const BatchInst *insts;
    uint32_t n_inst;          // media (slots) in the launch
    uint32_t n_pix_inst;      // side + transmitted pixels of one medium (key stride)
    uint64_t n_units;
};

constexpr int kCopies = 8;                 // per-XCD image copies in the workspace (at most)
constexpr uint64_t kLogBinBlocks = 512;    // log_bin blocks that fill the chip (two per CU)
constexpr double kFix = 4294967296.0;      // fixed-point scale 2^32 per unit weight

// w * 2^32 rounded to nearest, ties to even, for 0 <= w < 2^32.  The integer
// part of w and its fraction are exact in FP32, and the fraction times 2^32
// is an exact FP32 value below 2^32, so two FP32 conversions give the same
// integer as llrint((double)w * 2^32) with no FP64 arithmetic (an even
// multiple of 2^32 does not change the tie-breaking parity).  No fused
// multiply-add may absorb w's own rounding: a squared weight passed as w * w
// is the rounded FP32 product.
__device__ __forceinline__ unsigned long long fix(float w)
{
#pragma clang fp contract(off)
    const float hi = truncf(w);
    const float lo = rintf((w - hi) * 4294967296.f);
    return ((unsigned long long)(uint32_t)hi << 32) + (unsigned long long)(uint32_t)lo;
}

// The same for 0 <= w < 1 (every weight of the walk unless roulette is set
// to raise weights above 1): the integer part is 0 and w * 2^32 < 2^32.
__device__ __forceinline__ unsigned long long fix_below_one(float w)
{
    return (unsigned long long)(uint32_t)rintf(w * 4294967296.f);
}

// Pixel = floor(coord / size * n), clamped to the image (IEEE division, so a
// coordinate on a pixel edge lands where the FP64 definition puts it).  Used
// for the beam's unscattered exit pixel, where every such photon lands on
// the same point.
__device__ __forceinline__ int pixel(float coord, float size, int n)
{
    const int i = (int)floorf(coord / size * (float)n);
    return min(max(i, 0), n - 1);
}

// The same with one product by pixels per mm in place of the division, for
// the exits of scattered photons: only at a coordinate exactly on a pixel
// edge may the product round to the other side of it.
__device__ __forceinline__ int pixel_scaled(float coord, float per_mm, int n)
{
    const int i = (int)floorf(coord * per_mm);
    return min(max(i, 0), n - 1);
}

// Distances to the walls ahead along d, per axis.  With r = 1/d, the walls
// at L and at 0 lie (L - p) r and -p r ahead; for p inside the box one of the
// two is negative, so the larger is the wall the photon moves towards.  It is
// clamped at 0, so a position that rounding left a hair outside the box is
// taken back at once.  An axis with d = 0 gives r = inf and so t = inf: it is
// never hit (short of a position exactly on one of its walls, where 0 x inf
// makes the far term NaN, the maximum drops it and t is 0; the host keeps the
// source off that case).  No compare or select: three full-rate operations
// and one three-way maximum per axis.
__device__ __forceinline__ void wall_distances(float px, float py, float pz, float dx, float dy, float dz,
                                               float Lx, float Ly, float Lz, float &tx, float &ty, float &tz)
{
    const float rx = __builtin_amdgcn_rcpf(dx), ry = __builtin_amdgcn_rcpf(dy), rz = __builtin_amdgcn_rcpf(dz);
    tx = fmaxf(fmaxf((Lx - px) * rx, -px * rx), 0.f);
    ty = fmaxf(fmaxf((Ly - py) * ry, -py * ry), 0.f);
    tz = fmaxf(fmaxf((Lz - pz) * rz, -pz * rz), 0.f);
}

// The axis of the nearest wall, db = min(tx, ty, tz) (ties go to the lower
// axis).  The walk takes it only for the steps that reach a wall.
__device__ __forceinline__ int wall_axis(float db, float tx, float ty)
{
    return db == tx ? 0 : (db == ty ? 1 : 2);
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}


constexpr int kQueue = 64;                 // queued image exits per wave
constexpr uint32_t kEmpty = 0xFFFFFFFFu;   // free tally-cache slot

constexpr int kOptSigma = 1, kOptRecord = 2, kOptMoments = 4, kOptBatch = 8, kOptLog = 16;
// Exit log: image exits appended as (key << 32 | weight bits).  Keys fall
// into 2^rbits ranges; every block of the launch owns a region of log_cap
// entries in each range's part of the log and appends to it at the position a
// counter in its LDS hands out (no global atomic).  The waves of a block thus
// fill the same few lines of each range together, which stay in the L2 until
// they are whole.  Keys go to ranges by groups of eight (one 64-byte line of a
// tally copy): the group g is scrambled by p = g * kLogHashMul mod 2^bits (an
// odd multiplier, so a bijection), its top rbits bits pick the range and the
// rest, with the key's place in its group, index the key within the range.
// Bright spots of an image thus spread evenly over the ranges.  rbits grows
// with the images so that a range holds at most 2^kLogHistBits keys where the
// LDS allows (one binning block per range and copy).
constexpr uint32_t kLogMinRangeBits = 6;
constexpr uint32_t kLogHistBits = 13;      // keys per binning block: 2^13 (64 KB of int64 sums)
constexpr uint32_t kLogHashMul = 0x9E3779B1u;
__device__ __forceinline__ uint32_t log_scramble(uint32_t key, uint32_t bits)
{
    return ((key >> 3) * kLogHashMul) & ((1u << bits) - 1u);
}
__device__ __forceinline__ uint32_t log_bucket(uint32_t key, uint32_t bits, uint32_t rbits)
{
    return log_scramble(key, bits) >> (bits - rbits);
}
__device__ __forceinline__ uint32_t log_index(uint32_t key, uint32_t bits, uint32_t rbits)
{
    return ((log_scramble(key, bits) & ((1u << (bits - rbits)) - 1u)) << 3) | (key & 7u);
}
constexpr int kBatchScal = 16;             // LDS scalar words per medium in a batched launch
constexpr uint64_t kWsScalarWords = 32;    // workspace scalar words per medium
static_assert(kNoAllocWords == kWsScalarWords + (1ull << 21) && kNoAllocWords * 8 == MC_NOALLOC_SCRATCH_BYTES,
              "scratch holds the scalar words and 2^21 image words");
constexpr int kLdsBallistic = 15;          // LDS scalar word (per medium) counting first-step exits
constexpr int kWsBallistic = 19;           // workspace word (per medium) of that count
constexpr int kWsBeamKey = 20;             // workspace word (first medium): beam exit key + 1, or 0
constexpr int kWsLogFallback = 21;         // workspace word: exits added directly because the log was full

// Waves per SIMD a walk kernel is built for: eight (64 vector registers
// each), or six (80 each) with path moments, whose tallies would otherwise
// leave no registers for the step's constants (measured: six waves with the
// constants beat eight without by 7 %, while the plain walk loses 3 % at six).
template <int OPT>
constexpr int walk_waves_per_simd() { return (OPT & 4) ? 6 : 8; }

template <int PHASE, int OPT>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(walk_waves_per_simd<OPT>())))
void walk_kernel(WalkArgs a)
{
    constexpr bool SIGMA = OPT & kOptSigma, RECORD = OPT & kOptRecord, MOMENTS = OPT & kOptMoments;
    constexpr bool BATCH = OPT & kOptBatch, LOG = OPT & kOptLog;
    constexpr bool GLOBAL_TABLE = BATCH;   // batched: each medium's inverse table stays in global memory
    // LDS layout: inverse table (n_cdf floats, padded to 4; batched launches
    // read each medium's table from global memory instead), scalar words
    // (MC_N_SCALARS, or kBatchScal per medium), tally cache (slots words of
    // weight, [SIGMA] slots words of squared weight, slots uint32 keys),
    // per-wave exit queues (3 x kQueue floats, a fourth for the medium's slot),
    // with the exit log then the block's 2^log_rbits append counters.
    // (The kernel declares no static LDS: the dynamic array starts at offset 0,
    // and its 16-byte alignment keeps the 64-bit words below aligned.)
    extern __shared__ __attribute__((aligned(16))) float s_table[];
    constexpr int kQueueArrays = BATCH ? 4 : 3;
    unsigned long long *s_scal = (unsigned long long *)(s_table + (GLOBAL_TABLE ? 0 : ((a.n_cdf + 3) & ~3)));
    const int n_scal = BATCH ? (int)a.n_inst * kBatchScal : MC_N_SCALARS;
    const int slots = a.cache_bits ? 1 << a.cache_bits : 0;
    unsigned long long *s_cw = s_scal + n_scal;
    unsigned long long *s_cw2 = s_cw + (SIGMA ? slots : 0);
    uint32_t *s_key = (uint32_t *)(s_cw2 + slots);
    float *s_queue = (float *)(s_key + slots);
    // Exit log: entries the block has appended to each key range.
    uint32_t *s_lcnt = (uint32_t *)(s_queue + (blockDim.x >> 6) * (kQueueArrays * kQueue));
    if (LOG)
        for (int i = threadIdx.x; i < (1 << a.log_rbits); i += blockDim.x) s_lcnt[i] = 0u;

    if (PHASE == MC_PHASE_MIE && !GLOBAL_TABLE)
        for (int i = threadIdx.x; i < a.n_cdf; i += blockDim.x) s_table[i] = a.inv_cdf[i];
    for (int i = threadIdx.x; i < n_scal; i += blockDim.x) s_scal[i] = 0ull;
    for (int i = threadIdx.x; i < slots; i += blockDim.x) {
        s_cw[i] = 0ull;
        if (SIGMA) s_cw2[i] = 0ull;
        s_key[i] = kEmpty;
    }
    // Unscattered photons that leave on their first step all take the same
    // path from the source to the same pixel with the same weight w0, so the
    // walk only counts them (per medium) and the finalize pass adds count x w0
    // to that pixel.  The pixel (its key within a medium's key range) and face
    // are found here, by every thread, with the walk's own arithmetic; face -1
    // when the beam leaves through a face without an image (or through the
    // side image while its path moments are tallied).
    int beam_face = -2;   // -2: no face (it matches no photon's face, which is -1 or up)
    {
        float tx, ty, tz;
        wall_distances(a.pos0[0], a.pos0[1], a.pos0[2], a.dir0[0], a.dir0[1], a.dir0[2], a.size[0], a.size[1],
                       a.size[2], tx, ty, tz);
        const float db = fminf(fminf(tx, ty), tz);
        const int ax = wall_axis(db, tx, ty);
        const float bx = fmaf(db, a.dir0[0], a.pos0[0]), by = fmaf(db, a.dir0[1], a.pos0[1]);
        const float bz = fmaf(db, a.dir0[2], a.pos0[2]);
        const float da = ax == 0 ? a.dir0[0] : (ax == 1 ? a.dir0[1] : a.dir0[2]);
        int face = -2;
        uint32_t key = 0;
        if (da > 0.f && (ax == 0 || ax == 2) && !(MOMENTS && ax == 0) && !(a.beam_radius > 0.f)) {
            face = 2 * ax + 1;
            key = ax == 0 ? (uint32_t)(pixel(by, a.size[1], a.side_ny) * a.side_nx + pixel(bz, a.size[2], a.side_nx))
                          : a.n_side + (uint32_t)(pixel(by, a.size[1], a.trans_ny) * a.trans_nx +
                                                  pixel(bx, a.size[0], a.trans_nx));
            if (blockIdx.x == 0 && threadIdx.x == 0) a.ws_scal[kWsBeamKey] = (unsigned long long)key + 1ull;
        }
        beam_face = face;
    }
    // Every wave reads the whole table and adds into the scalars, cache and
    // log cursors set up above by the block's threads together.
    __syncthreads();

    const int lane = __lane_id();
    const uint32_t xcc = __builtin_amdgcn_s_getreg((3 << 11) | 20) & a.copy_mask;   // hwreg(HW_REG_XCC_ID, 0, 4)
    unsigned long long *my_img = a.ws_img + (uint64_t)xcc * a.n_pix;
    unsigned long long *my_img2 = SIGMA ? a.ws_img2 + (uint64_t)xcc * a.n_pix : nullptr;
    float *q_y = s_queue + (threadIdx.x >> 6) * (kQueueArrays * kQueue);
    float *q_b = q_y + kQueue;
    float *q_w = q_b + kQueue;                 // weight bits, bit 31 set for the side image
    float *q_s = q_w + kQueue;                 // batched: the medium's slot (uint32 bits)
    uint32_t q_n = 0;                          // wave-uniform queue fill

    // Tally the first n queued exits, one per lane: pixel key, then the LDS
    // cache (claim or hit, up to four linear probes) or, when every probed
    // slot holds another pixel, a global atomic.  With the exit log the exits
    // are appended to the log instead; a global atomic is then the fallback
    // for a range whose region of the log is full.
    auto flush = [&](uint32_t n) {
        __builtin_amdgcn_wave_barrier();
        const bool act = (uint32_t)lane < n;
        uint32_t key = 0;
        float wf = 0.f;
        unsigned long long wq = 0ull, wq2 = 0ull;
        if (act) {
            const float y = q_y[lane], b = q_b[lane];
            const uint32_t wb = __float_as_uint(q_w[lane]);
            const bool side = wb >> 31;
            wf = __uint_as_float(wb & 0x7FFFFFFFu);
            const uint32_t key_base = BATCH ? __float_as_uint(q_s[lane]) * a.n_pix_inst : 0u;
            const float per_row = side ? a.pix_scale[0] : a.pix_scale[2];
            const float per_col = side ? a.pix_scale[1] : a.pix_scale[3];
            const int n_row = side ? a.side_ny : a.trans_ny, n_col = side ? a.side_nx : a.trans_nx;
            key = key_base + (side ? 0u : a.n_side) +
                  (uint32_t)(pixel_scaled(y, per_row, n_row) * n_col + pixel_scaled(b, per_col, n_col));
        }
        if (act && !LOG) {
            wq = fix(wf);
            wq2 = SIGMA ? fix(wf * wf) : 0ull;
        }
        if (LOG) {
            // Append to the block's region of the key's range at the position
            // the block's LDS counter hands out; past the region's end, the
            // exit is added directly.
            const uint32_t bucket = log_bucket(key, a.log_bits, a.log_rbits);
            bool direct = false;
            if (act) {
                const uint32_t e = atomicAdd(&s_lcnt[bucket], 1u);
                if (e < a.log_cap)
                    a.log[(uint64_t)(bucket * gridDim.x + blockIdx.x) * a.log_cap + e] =
                        ((unsigned long long)key << 32) | __float_as_uint(wf);
                else
                    direct = true;
            }
            if (direct) {
                atomicAdd(my_img + key, fix(wf));
                if (SIGMA) atomicAdd(my_img2 + key, fix(wf * wf));
            }
            const uint64_t took = __ballot(direct);
            if (took && lane == 0) atomicAdd(a.ws_scal + kWsLogFallback, (unsigned long long)__popcll(took));
        } else if (act) {
            bool cached = false;
            if (slots) {
                uint32_t slot = (key * 2654435761u) >> (32 - a.cache_bits);
                for (int probe = 0; probe < 4 && !cached; ++probe) {
                    const uint32_t old = atomicCAS(&s_key[slot], kEmpty, key);
                    if (old == kEmpty || old == key) {
                        atomicAdd(&s_cw[slot], wq);
                        if (SIGMA) atomicAdd(&s_cw2[slot], wq2);
                        cached = true;
                    }
                    slot = (slot + 1) & (uint32_t)(slots - 1);
                }
            }
            if (!cached) {
                atomicAdd(my_img + key, wq);
                if (SIGMA) atomicAdd(my_img2 + key, wq2);
            }
        }
        __builtin_amdgcn_wave_barrier();
    };

    unsigned long long *work = a.ws_scal + MC_S_RESERVED;
    const float tab_scale = (float)(a.n_cdf - 1);

    // Wave-uniform id range: next id and ids left in the claimed chunk.
    uint64_t q_next = 0;
    uint32_t q_rem = 0;
    bool exhausted = false;

    // Lane state.
    bool alive = false;
    uint64_t id = 0;
    float px = 0.f, py = 0.f, pz = 0.f, dx = 0.f, dy = 0.f, dz = 1.f;
    float w = 0.f, L = 0.f, A = 0.f;
    uint32_t k = 0, step = 0;
    // Lane accumulators.
    unsigned long long acc_abs = 0ull;
    uint32_t acc_events = 0, acc_steps = 0, acc_photons = 0, acc_ball = 0;
    double acc_w2 = 0.0, acc_w2k = 0.0, acc_w2l = 0.0;   // MOMENTS: image-wide second moments
    // The medium of the lane's photon (batched launches change it per photon;
    // otherwise these stay the launch's values).
    uint32_t l_slot = kEmpty, q_p = 0;
    float l_mu = a.neg_ln2_over_mu, l_alb = a.albedo, l_abs = a.absorb;
    // FP32 operations with a scalar-register operand issue at half the rate
    // of those whose operands are all vector registers; the constants of the
    // step therefore live in vector registers (the empty asm hides that they
    // are wave-uniform; batched media keep theirs per lane anyway).
    float v_lx = a.size[0], v_ly = a.size[1], v_lz = a.size[2], v_n21 = a.n21, v_n12sq = a.n12sq;
    asm volatile("" : "+v"(l_mu), "+v"(l_alb), "+v"(l_abs));
    asm volatile("" : "+v"(v_lx), "+v"(v_ly), "+v"(v_lz), "+v"(v_n21), "+v"(v_n12sq));
    // A new photon's starting state, likewise in vector registers (a refill
    // then copies at full rate instead of from scalar registers, and seven
    // scalar registers fewer need spilling); not for batched media, whose
    // kernels have no registers to spare and whose photons start the same.
    constexpr bool INIT_V = !BATCH;
    float i_px = a.pos0[0], i_py = a.pos0[1], i_pz = a.pos0[2], i_dx = a.dir0[0], i_dy = a.dir0[1];
    float i_dz = a.dir0[2], i_w = a.w0;
    if (INIT_V)
        asm volatile("" : "+v"(i_px), "+v"(i_py), "+v"(i_pz), "+v"(i_dx), "+v"(i_dy), "+v"(i_dz), "+v"(i_w));
    // The roulette threshold, compared at every interaction, likewise: in a
    // scalar register it was spilled and reloaded (four v_readlane) each time.
    float v_rw = a.roulette_w;
    if (INIT_V) asm volatile("" : "+v"(v_rw));
    // 1 where the walls have a Fresnel term, 0 where the indices match.
    float v_fresnel = a.matched ? 0.f : 1.f;
    if (INIT_V) asm volatile("" : "+v"(v_fresnel));
    const float *l_tab = a.inv_cdf;
    uint32_t l_ctr = a.instance;
    // Batched: move the lane accumulators into the LDS scalars of its medium.
    auto flush_lane = [&]() {
        unsigned long long *sc = s_scal + l_slot * kBatchScal;
        atomicAdd(&sc[MC_S_ABSORBED], acc_abs);
        atomicAdd(&sc[MC_S_EVENTS], (unsigned long long)acc_events);
        atomicAdd(&sc[MC_S_STEPS], (unsigned long long)acc_steps);
        atomicAdd(&sc[MC_S_PHOTONS], (unsigned long long)acc_photons);
        if (acc_ball) atomicAdd(&sc[kLdsBallistic], (unsigned long long)acc_ball);
        acc_abs = 0ull;
        acc_events = acc_steps = acc_photons = acc_ball = 0;
    };

    // A lane whose photon has ended keeps its state until the end-of-photon
    // work (tallies, records, the exit queue) and the refill run for several
    // lanes at once: when at least refill_min lanes are free (refill_min <= 64,
    // so also when none is still walking).  Few lanes finish in any one step,
    // so doing that work every step would run it with most lanes masked off.
    // An ended photon's face is its exit face (0..5) exactly when it left
    // through a wall (cause 0); roulette kills and the step cap leave it -1.
    // A photon that leaves on its first step met a wall before any
    // interaction, so leaving through the beam's own exit face at step 1
    // makes it an unscattered first-step exit.
    bool pending = false;
    int cause = 0, face = -1, axis = 0;

    for (;;) {
        // Free lanes (wave-uniform counts); refill_min <= 64, so a wave whose
        // lanes are all free always runs the end-of-photon work.
        const uint64_t need = __ballot(!alive);
        const uint32_t n_need = (uint32_t)__popcll(need);
        uint32_t n_alive = 64u - n_need;
        if (n_need >= a.refill_min) {
            // ---- end-of-photon work of the waiting lanes ----------------------
            if (pending) {
                const uint32_t scal_at = BATCH ? l_slot * kBatchScal : 0u;
                // Faces +x and +z are totalled from their images when finalizing.
                const bool below_one = __ballot(w >= 1.f || A >= 1.f) == 0;   // wave-uniform
                if (face >= 0 && (face | 4) != 5)
                    atomicAdd(&s_scal[scal_at + MC_S_FACE + face], below_one ? fix_below_one(w) : fix(w));
                if (MOMENTS && cause == 0 && face == 1) {
                    // Path moments of the side image (perturbation Monte Carlo):
                    // first order per pixel, second order summed over the image
                    // in lane registers (per pixel as well when asked for).
                    const uint32_t key = (uint32_t)(pixel_scaled(py, a.pix_scale[0], a.side_ny) * a.side_nx +
                                                    pixel_scaled(pz, a.pix_scale[1], a.side_nx));
                    const double wd = (double)w, wk = wd * (double)k, wl = wd * (double)L;
                    atomicAdd(a.side_wk + key, wk);
                    atomicAdd(a.side_wl + key, wl);
                    acc_w2 += wd * wd;
                    acc_w2k += wd * wk;
                    acc_w2l += wd * wl;
                    if (a.side_w2k) {
                        atomicAdd(a.side_w2k + key, wd * wk);
                        atomicAdd(a.side_w2l + key, wd * wl);
                    }
                }
                acc_abs += below_one ? fix_below_one(A) : fix(A);
                acc_events += k;
                acc_steps += step;
                ++acc_photons;
                if (RECORD) {
                    const uint64_t rel = id - a.photon_offset;
                    if (rel % a.record_stride == 0 && rel / a.record_stride < a.rec_rows) {
                        const uint64_t row = rel / a.record_stride, n = a.rec_rows;
                        float ox = dx, oy = dy, oz = dz;
                        if (cause == 0 && !a.matched) {
                            // Refracted direction outside the wall (Snell).
                            ox *= a.n12; oy *= a.n12; oz *= a.n12;
                            const float t2 = (axis == 0 ? oy * oy + oz * oz
                                                        : (axis == 1 ? ox * ox + oz * oz : ox * ox + oy * oy));
                            const float on = copysignf(sqrtf(fmaxf(1.f - t2, 0.f)),
                                                       axis == 0 ? dx : (axis == 1 ? dy : dz));
                            if (axis == 0) ox = on; else if (axis == 1) oy = on; else oz = on;
                        }
                        a.rec_i[MC_REC_I_FACE * n + row] = face;
                        a.rec_i[MC_REC_I_CAUSE * n + row] = cause;
                        a.rec_i[MC_REC_I_K * n + row] = (int32_t)k;
                        a.rec_i[MC_REC_I_STEPS * n + row] = (int32_t)step;
                        a.rec_f[(MC_REC_F_POS + 0) * n + row] = px;
                        a.rec_f[(MC_REC_F_POS + 1) * n + row] = py;
                        a.rec_f[(MC_REC_F_POS + 2) * n + row] = pz;
                        a.rec_f[(MC_REC_F_DIR + 0) * n + row] = ox;
                        a.rec_f[(MC_REC_F_DIR + 1) * n + row] = oy;
                        a.rec_f[(MC_REC_F_DIR + 2) * n + row] = oz;
                        a.rec_f[MC_REC_F_W * n + row] = w;
                        a.rec_f[MC_REC_F_L * n + row] = L;
                        a.rec_f[MC_REC_F_A * n + row] = A;
                    }
                }
            }
            // ---- queue exits through the imaged faces (+x side, +z transmitted) ----
            const bool ballistic = pending && step == 1 && face == beam_face;
            acc_ball += ballistic ? 1u : 0u;
            const bool to_img = pending && (face | 4) == 5 && !ballistic;
            const uint64_t m = __ballot(to_img);
            if (m) {
                const uint32_t n_push = __popcll(m);
                if (q_n + n_push > (uint32_t)kQueue) {
                    flush(q_n);
                    q_n = 0;
                }
                if (to_img) {
                    const uint32_t at = q_n + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    q_y[at] = py;
                    q_b[at] = face == 1 ? pz : px;
                    q_w[at] = __uint_as_float(__float_as_uint(w) | (face == 1 ? 0x80000000u : 0u));
                    if (BATCH) q_s[at] = __uint_as_float(l_slot);
                }
                q_n += n_push;
            }

            pending = false;

            // Lane counters stay below 2^31: steps bound the others, and a
            // photon adds at most max_steps <= 2^24.  Past 2^31 they move into
            // the 64-bit LDS words (batched: of the lane's medium).
            if (__ballot(acc_steps >= 0x80000000u)) {
                if (BATCH) {
                    if (acc_steps >= 0x80000000u) flush_lane();
                } else {
                    atomicAdd(&s_scal[MC_S_EVENTS], (unsigned long long)acc_events);
                    atomicAdd(&s_scal[MC_S_STEPS], (unsigned long long)acc_steps);
                    atomicAdd(&s_scal[MC_S_PHOTONS], (unsigned long long)acc_photons);
                    atomicAdd(&s_scal[kLdsBallistic], (unsigned long long)acc_ball);
                    acc_events = acc_steps = acc_photons = acc_ball = 0;
                }
            }

            // ---- refill free lanes ---------------------------------------------
            if (q_rem == 0 && !exhausted) {
                // Single medium: claim the next `chunk` photon ids.  Batched:
                // claim the next work unit, `chunk` photons of one medium.
                unsigned long long base = 0;
                if (lane == 0) base = atomicAdd(work, BATCH ? 1ull : (unsigned long long)a.chunk);
                const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)base);
                const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(base >> 32));
                const uint64_t b = ((uint64_t)hi << 32) | lo;
                if (BATCH) {
                    if (b >= a.n_units) {
                        exhausted = true;
                    } else {
                        // The unit's medium: the last one whose first unit is <= b
                        // (media without photons own no units and are never found).
                        uint32_t l = 0, h = a.n_inst;
                        while (h - l > 1) {
                            const uint32_t mid = (l + h) >> 1;
                            if (a.insts[mid].unit_begin <= b) l = mid; else h = mid;
                        }
                        q_p = l;
                        q_next = (b - a.insts[l].unit_begin) * a.chunk;
                        q_rem = (uint32_t)min((uint64_t)a.chunk, a.insts[l].n_photons - q_next);
                    }
                } else if (b >= a.n_photons) {
                    exhausted = true;
                } else {
                    q_next = b;
                    q_rem = (uint32_t)min((uint64_t)a.chunk, a.n_photons - b);
                }
            }
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(need >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
            if (!alive && rank < q_rem) {
                id = (BATCH ? 0ull : a.photon_offset) + q_next + rank;
                if (BATCH) {
                    const BatchInst &bi = a.insts[q_p];
                    if (bi.slot != l_slot) {
                        if (l_slot != kEmpty) flush_lane();
                        l_slot = bi.slot;
                        l_mu = bi.neg_ln2_over_mu;
                        l_alb = bi.albedo;
                        l_abs = bi.absorb;
                        l_tab = bi.inv_cdf;
                        l_ctr = bi.counter;
                    }
                }
                alive = true;
                px = INIT_V ? i_px : a.pos0[0];
                py = INIT_V ? i_py : a.pos0[1];
                pz = INIT_V ? i_pz : a.pos0[2];
                if (a.beam_radius > 0.f) {
                    // Finite beam: entry point uniform on the disk, from the
                    // photon's Philox block at the reserved step counter.
                    uint32_t k0 = a.key0, k1 = a.key1;
                    const Block4 rb = philox4x32_10(0xFFFFFFFFu, l_ctr, (uint32_t)id, (uint32_t)(id >> 32), k0, k1);
                    const float rho = a.beam_radius * __builtin_amdgcn_sqrtf(uniform01(rb.r0));
                    const float u1 = uniform01(rb.r1);
                    px = fmaf(rho, __builtin_amdgcn_cosf(u1), px);    // cos(2 pi u1)
                    py = fmaf(rho, __builtin_amdgcn_sinf(u1), py);    // sin(2 pi u1)
                }
                dx = INIT_V ? i_dx : a.dir0[0];
                dy = INIT_V ? i_dy : a.dir0[1];
                dz = INIT_V ? i_dz : a.dir0[2];
                w = INIT_V ? i_w : a.w0;
                L = 0.f; A = 0.f; k = 0; step = 0;
            }
            const uint32_t took = min(n_need, q_rem);
            q_next += took;
            q_rem -= took;
            n_alive += took;
        }
        if (n_alive == 0) break;

        bool ended = false;
        const uint32_t scal_at = BATCH ? l_slot * kBatchScal : 0u;   // the medium's LDS scalars
        if (alive) {
            cause = 0;
            face = -1;
            // ---- one step ---------------------------------------------------
            // The round keys derive from the seed inside the loop (scalar adds)
            // rather than living in 20 scalar registers across it.
            uint32_t k0 = a.key0, k1 = a.key1;
            asm volatile("" : "+s"(k0), "+s"(k1));
            const Block4 r = philox4x32_10(step, l_ctr, (uint32_t)id, (uint32_t)(id >> 32), k0, k1);
            const float u0 = uniform01(r.r0), u1 = uniform01(r.r1);
            const float u2 = uniform01(r.r2), u3 = uniform01(r.r3);
            const float s = __builtin_amdgcn_logf(u0) * l_mu;     // Eq. 15
            ++step;

            // Nearest wall along the direction.
            float tx, ty, tz;
            wall_distances(px, py, pz, dx, dy, dz, v_lx, v_ly, v_lz, tx, ty, tz);
            const float db = fminf(fminf(tx, ty), tz);

            const bool hit = s >= db;
            const float t = fminf(s, db);
            px = fmaf(t, dx, px); py = fmaf(t, dy, py); pz = fmaf(t, dz, pz);
            L += t;
            if (hit) {
                // Boundary: clamp into the box (a move that overshot the wall
                // by rounding lands on it), then reflect (u3 < R) or leave.
                // Written as selects so the wave runs it without branches.
                axis = wall_axis(db, tx, ty);
                const bool on_x = axis == 0, on_y = axis == 1, on_z = axis == 2;
                const float da = on_x ? dx : (on_y ? dy : dz);
                const bool pos_side = da > 0.f;
                px = __builtin_amdgcn_fmed3f(px, 0.f, v_lx);
                py = __builtin_amdgcn_fmed3f(py, 0.f, v_ly);
                pz = __builtin_amdgcn_fmed3f(pz, 0.f, v_lz);
                // Index-matched walls reflect nothing: R is scaled by 0 there
                // (v_fresnel) rather than skipped on a flag the wave would
                // have to reload from a spilled scalar register every step.
                const float ci = fabsf(da);
                const float st2 = v_n12sq * fmaf(-ci, ci, 1.f);
                // 1 - st2 > 0 wherever R uses ct; under TIR the select drops it.
                const float ct = __builtin_amdgcn_sqrtf(1.f - st2);
                const float ds = fmaf(v_n21, ct, ci), dp = fmaf(v_n21, ci, ct);   // both > 0 (ci > 0)
                const float r = __builtin_amdgcn_rcpf(ds * dp);
                const float rs = fmaf(-v_n21, ct, ci) * dp * r;
                const float rp = fmaf(v_n21, ci, -ct) * ds * r;
                const float R = v_fresnel * (st2 >= 1.f ? 1.f : 0.5f * fmaf(rs, rs, rp * rp));
                const bool refl = u3 < R;
                dx = refl && on_x ? -dx : dx;
                dy = refl && on_y ? -dy : dy;
                dz = refl && on_z ? -dz : dz;
                ended = !refl;
                face = refl ? -1 : 2 * axis + (pos_side ? 1 : 0);
            } else {
                // Interaction: count, absorb (Eq. 16), roulette, scatter.
                ++k;
                A = fmaf(w, l_abs, A);
                w *= l_alb;
                if (w < v_rw) {
                    if (u3 < a.roulette_p) {
                        const float wn = w * a.inv_roulette_p;
                        atomicAdd(&s_scal[scal_at + MC_S_ROULETTE_NET], fix(wn) - fix(w));
                        w = wn;
                    } else {
                        atomicAdd(&s_scal[scal_at + MC_S_ROULETTE_NET], 0ull - fix(w));
                        atomicAdd(&s_scal[scal_at + MC_S_ROULETTE_KILLS], 1ull);
                        w = 0.f;
                        ended = true;
                        cause = 1;
                    }
                }
                if (!ended) {
                    float v;
                    if (PHASE == MC_PHASE_MIE) {
                        // u1 <= 1 - 2^-24, so u1 (n - 1) rounds below n - 1 (exact when
                        // n - 1 is a power of two, else more than half an ulp short of
                        // it): i <= n - 2 and entry i + 1 exists.
                        const float tt = u1 * tab_scale;
                        const int i = (int)tt;
                        // The fraction from the unrounded product u1 (n - 1).
                        const float f = fmaf(u1, tab_scale, -(float)i);
                        const float t0 = GLOBAL_TABLE ? l_tab[i] : s_table[i];
                        const float t1 = GLOBAL_TABLE ? l_tab[i + 1] : s_table[i + 1];
                        v = fmaf(f, t1 - t0, t0);
                    } else {
                        const float D = fmaf(-a.hg_b, u1, a.hg_a);
                        const float rD = __builtin_amdgcn_rcpf(D);
                        v = a.hg_d * u1 * fmaf(a.hg_c, rD, a.hg_d) * rD;
                    }
                    const float ct = 1.f - v;
                    // A table value lies in [0, 2], and so does a rounded point between
                    // two of them: v (2 - v) >= 0.  The HG formula can overshoot 2.
                    const float st = __builtin_amdgcn_sqrtf(PHASE == MC_PHASE_MIE ? v * (2.f - v)
                                                                                  : fmaxf(v * (2.f - v), 0.f));
                    const float cp = __builtin_amdgcn_cosf(u2);        // cos(2 pi u2)
                    const float sp = __builtin_amdgcn_sinf(u2);        // sin(2 pi u2)
                    // Orthonormal basis around d (Duff et al. 2017).
                    const float sg = copysignf(1.f, dz);
                    const float ia = -__builtin_amdgcn_rcpf(sg + dz);
                    const float b = dx * dy * ia;
                    const float e1x = fmaf(sg * dx * dx, ia, 1.f), e1y = sg * b, e1z = -sg * dx;
                    const float e2x = b, e2y = fmaf(dy * dy, ia, sg), e2z = -dy;
                    const float qx = fmaf(cp, e1x, sp * e2x), qy = fmaf(cp, e1y, sp * e2y),
                                qz = fmaf(cp, e1z, sp * e2z);
                    const float nx = fmaf(ct, dx, st * qx), ny = fmaf(ct, dy, st * qy), nz = fmaf(ct, dz, st * qz);
                    // |n|^2 is 1 up to rounding, so one Newton step of 1/sqrt from 1
                    // (1.5 - |n|^2 / 2) renormalises to within 1e-13.
                    const float inv = fmaf(-0.5f, fmaf(nx, nx, fmaf(ny, ny, nz * nz)), 1.5f);
                    dx = nx * inv; dy = ny * inv; dz = nz * inv;
                }
            }
            if (!ended && step >= a.max_steps) {
                ended = true;
                cause = 2;
                atomicAdd(&s_scal[scal_at + MC_S_CAPPED_W], fix(w));
                atomicAdd(&s_scal[scal_at + MC_S_CAPPED], 1ull);
            }
            if (ended) {
                pending = true;
                alive = false;
            }
        }
    }
    flush(q_n);

    // ---- block-level flush of the scalar tallies and the cache ---------------
    if (BATCH) {
        if (l_slot != kEmpty) flush_lane();
        __syncthreads();
        for (int i = threadIdx.x; i < n_scal; i += blockDim.x) {
            const int j = i % kBatchScal;
            const unsigned long long v = s_scal[i];
            if (v != 0ull && (j < MC_S_RESERVED || j == kLdsBallistic))
                atomicAdd(&a.ws_scal[(uint64_t)(i / kBatchScal) * kWsScalarWords +
                                     (j == kLdsBallistic ? kWsBallistic : j)], v);
        }
    } else {
        const unsigned long long wabs = wave_sum(acc_abs);
        // Lane counters are below 2^32; their wave sums are taken in 64 bits.
        const unsigned long long wev = wave_sum((unsigned long long)acc_events);
        const unsigned long long wst = wave_sum((unsigned long long)acc_steps);
        const unsigned long long wph = wave_sum((unsigned long long)acc_photons);
        const unsigned long long wbl = wave_sum((unsigned long long)acc_ball);
        if (lane == 0) {
            if (wbl) atomicAdd(&s_scal[kLdsBallistic], wbl);
            atomicAdd(&s_scal[MC_S_ABSORBED], wabs);
            atomicAdd(&s_scal[MC_S_EVENTS], wev);
            atomicAdd(&s_scal[MC_S_STEPS], wst);
            atomicAdd(&s_scal[MC_S_PHOTONS], wph);
        }
        if (MOMENTS) {
            const double m0 = wave_sum(acc_w2), m1 = wave_sum(acc_w2k), m2 = wave_sum(acc_w2l);
            if (lane == 0) {
                double *s_m2 = (double *)(s_scal + MC_S_SIDE_W2);
                atomicAdd(s_m2 + 0, m0);
                atomicAdd(s_m2 + 1, m1);
                atomicAdd(s_m2 + 2, m2);
            }
        }
        __syncthreads();
        if (threadIdx.x < MC_S_RESERVED) {
            const unsigned long long v = s_scal[threadIdx.x];
            if (v != 0ull) atomicAdd(&a.ws_scal[threadIdx.x], v);
        } else if (threadIdx.x == kLdsBallistic) {
            const unsigned long long v = s_scal[kLdsBallistic];
            if (v != 0ull) atomicAdd(&a.ws_scal[kWsBallistic], v);
        } else if (MOMENTS && threadIdx.x >= MC_S_SIDE_W2 && threadIdx.x <= MC_S_SIDE_W2L) {
            const double v = __longlong_as_double((long long)s_scal[threadIdx.x]);
            if (v != 0.0) atomicAdd((double *)&a.ws_scal[threadIdx.x], v);
        }
    }
    for (int i = threadIdx.x; i < slots; i += blockDim.x) {
        const uint32_t key = s_key[i];
        if (key == kEmpty) continue;
        atomicAdd(my_img + key, s_cw[i]);
        if (SIGMA) atomicAdd(my_img2 + key, s_cw2[i]);
    }
    // The block's entries in each range of the exit log (all its waves have
    // appended: the barrier above).
    if (LOG)
        for (int i = threadIdx.x; i < (1 << a.log_rbits); i += blockDim.x)
            a.log_count[i * gridDim.x + blockIdx.x] = min(s_lcnt[i], a.log_cap);
}

// Zero the workspace words [0, n_ws) and [ws2, ws2 + n_ws2), and the outputs
// unless accumulating.  (Fill kernels,
// not memset, so the sequence stays valid under stream capture.)
__global__ void init_kernel(unsigned long long *ws, size_t n_ws, unsigned long long *ws2, size_t n_ws2,
                            unsigned long long *side, unsigned long long *trans,
                            unsigned long long *side_w2, unsigned long long *trans_w2, size_t n_side, size_t n_trans,
                            double *scalars, size_t n_scalars, int32_t *rec_i, float *rec_f, size_t n_rec,
                            double *side_wk,
                            double *side_wl, double *side_w2k, double *side_w2l, int zero_all)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (size_t i = t0; i < n_ws; i += stride) ws[i] = 0ull;
    for (size_t i = t0; i < n_ws2; i += stride) ws2[i] = 0ull;
    if (!zero_all) return;
    for (size_t i = t0; i < n_side; i += stride) {
        side[i] = 0ull;                 // +0.0 and int64 0 share the bit pattern
        if (side_w2) side_w2[i] = 0ull;
        if (side_wk) {
            side_wk[i] = 0.0;
            side_wl[i] = 0.0;
        }
        if (side_w2k) {
            side_w2k[i] = 0.0;
            side_w2l[i] = 0.0;
        }
    }
    for (size_t i = t0; i < n_trans; i += stride) {
        trans[i] = 0ull;
        if (trans_w2) trans_w2[i] = 0ull;
    }
    for (size_t i = t0; i < n_scalars; i += stride) scalars[i] = 0.0;
    for (size_t i = t0; i < (size_t)MC_REC_I_N * n_rec; i += stride) rec_i[i] = (i / n_rec == MC_REC_I_FACE) ? -1 : 0;
    for (size_t i = t0; i < (size_t)MC_REC_F_N * n_rec; i += stride) rec_f[i] = 0.f;
}

// Sum the exit log into the image copies.  Block (range b, part p, copy s)
// takes the regions of range b that every n_copies-th of the walk's blocks,
// from block s, wrote (log_count entries each), adds the fixed-point weights (and
// squared weights) of the entries whose index within the range lies in part
// p into an LDS histogram of 2^kLogHistBits sums, then writes the sums into
// copy s.  Copy 0 also holds the walk's fallback atomics (exits that found
// their region full), so it was cleared and takes the non-zero sums as
// adds; the other copies were not cleared and take every key's sum as a
// store (the blocks of copy s cover each of its keys exactly once).  No
// other writer touches those keys now, so plain loads and stores do.  The
// sums are of the same fix() values the walk would have added, so the
// images equal those of the atomic path bit for bit.
template <bool SIGMA>
__global__ __launch_bounds__(1024) void log_bin(const unsigned long long *log, const uint32_t *count, uint32_t cap,
                                                uint32_t walk_blocks, unsigned long long *copies,
                                                unsigned long long *copies2, uint32_t n_copies, uint64_t n_total,
                                                uint32_t parts, uint32_t bits, uint32_t rbits, uint32_t inv_mul)
{
    extern __shared__ __attribute__((aligned(16))) unsigned long long s_hist[];
    constexpr uint32_t H = 1u << kLogHistBits;
    unsigned long long *s_hist2 = s_hist + H;
    const uint32_t s = blockIdx.x % n_copies, rest = blockIdx.x / n_copies;
    const uint32_t part = rest % parts, b = rest / parts;
    for (uint32_t i = threadIdx.x; i < H; i += blockDim.x) {
        s_hist[i] = 0ull;
        if (SIGMA) s_hist2[i] = 0ull;
    }
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u, waves = blockDim.x >> 6;
    constexpr uint32_t U = 4;   // entries in flight per lane
    // Copy s takes the walk's blocks s, s + n_copies, s + 2 n_copies, ...:
    // the walk's blocks log very unequal numbers of exits (work is claimed
    // per wave, and the older workgroup on a compute unit wins most issue
    // cycles: at the headline the first 256 of 512 blocks log four times as
    // many as the rest), so contiguous shares would load some copies 1.6
    // times the mean.  Each wave takes every waves-th of them and reads its
    // entries U x 64 at a time.
    for (uint32_t g = s + n_copies * (threadIdx.x >> 6); g < walk_blocks; g += n_copies * waves) {
        const uint64_t region = (uint64_t)b * walk_blocks + g;
        const uint32_t n = count[region];
        const unsigned long long *ent = log + region * cap;
        for (uint32_t base = 0; base < n; base += U * 64) {
            unsigned long long e[U];
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                const uint32_t i = base + u * 64 + lane;
                e[u] = i < n ? ent[i] : 0ull;
            }
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                if (base + u * 64 + lane >= n) continue;
                const uint32_t h = log_index((uint32_t)(e[u] >> 32), bits, rbits);
                if ((h >> kLogHistBits) != part) continue;
                const float wf = __uint_as_float((uint32_t)e[u]);
                atomicAdd(&s_hist[h & (H - 1)], fix(wf));
                if (SIGMA) atomicAdd(&s_hist2[h & (H - 1)], fix(wf * wf));
            }
        }
    }
    __syncthreads();
    unsigned long long *dst = copies + (uint64_t)s * n_total;
    unsigned long long *dst2 = SIGMA ? copies2 + (uint64_t)s * n_total : nullptr;
    const uint32_t per_range = 1u << (bits - rbits + 3);
    for (uint32_t i = threadIdx.x; i < H; i += blockDim.x) {
        const uint32_t h = part * H + i;
        if (h >= per_range) break;
        // Undo the scramble: p = range bits | group bits, g = p / kLogHashMul mod 2^bits.
        const uint32_t p = (b << (bits - rbits)) | (h >> 3);
        const uint64_t key = ((uint64_t)((p * inv_mul) & ((1u << bits) - 1u)) << 3) | (h & 7u);
        if (key >= n_total) continue;
        const unsigned long long v = s_hist[i];
        const unsigned long long v2 = SIGMA ? s_hist2[i] : 0ull;
        if (s != 0) {
            dst[key] = v;
            if (SIGMA) dst2[key] = v2;
        } else {
            if (v) dst[key] += v;
            if (SIGMA && v2) dst2[key] += v2;
        }
    }
}

// Sum the n_copies fixed-point copies of every pixel (integer adds, so the
// order is immaterial) and add them to the caller's images, as int64 (FIX) or
// converted to double.  Weight sums of the +x and +z images also give those
// faces' totals.
// One medium per blockIdx.y: its pixels are keys [y * n_pix, (y + 1) * n_pix)
// of copies that hold n_total keys each; its images start at y * n_side and
// y * (n_pix - n_side) in the outputs and its face totals are at
// face_side / face_trans + y * face_stride.
//
// Unscattered first-step exits were only counted (workspace word kWsBallistic
// of each medium); the beam pixel (word kWsBeamKey) gets count x ball_w.
template <bool FIX>
__global__ __launch_bounds__(256) void finalize_images(const unsigned long long *copies, int n_copies, uint64_t n_total,
                                                       uint64_t n_pix, uint32_t n_side, void *side, void *trans,
                                                       unsigned long long *face_side, unsigned long long *face_trans,
                                                       uint64_t face_stride, const unsigned long long *ws_scal,
                                                       unsigned long long ball_w)
{
    const uint64_t inst = blockIdx.y;
    const uint64_t key0 = inst * n_pix;
    side = FIX ? (void *)((long long *)side + inst * n_side) : (void *)((double *)side + inst * n_side);
    trans = FIX ? (void *)((long long *)trans + inst * (n_pix - n_side))
                : (void *)((double *)trans + inst * (n_pix - n_side));
    if (face_side) {
        face_side += inst * face_stride;
        face_trans += inst * face_stride;
    }
    unsigned long long sum_side = 0ull, sum_trans = 0ull;
    const unsigned long long beam_key = ws_scal[kWsBeamKey];
    const unsigned long long beam_v = ws_scal[inst * kWsScalarWords + kWsBallistic] * ball_w;
    // Each thread takes kFinPix pixels a grid-stride apart per pass and issues
    // the loads of all their copies and outputs before using any.
    constexpr int kFinPix = 4;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i0 < n_pix; i0 += kFinPix * stride) {
        unsigned long long part[kFinPix][kCopies];
        long long prev[kFinPix];
#pragma unroll
        for (int u = 0; u < kFinPix; ++u) {
            const uint64_t i = i0 + u * stride;
            const bool in = i < n_pix, is_side = i < n_side;
            const uint64_t j = is_side ? i : i - n_side;
            long long *out = (long long *)(is_side ? side : trans);
#pragma unroll
            for (int c = 0; c < kCopies; ++c)
                part[u][c] = in && c < n_copies ? copies[(uint64_t)c * n_total + key0 + i] : 0ull;
            prev[u] = in ? out[j] : 0ll;   // the output's bits (int64, or a double's)
        }
#pragma unroll
        for (int u = 0; u < kFinPix; ++u) {
            const uint64_t i = i0 + u * stride;
            if (i >= n_pix) break;
            unsigned long long v = 0ull;
#pragma unroll
            for (int c = 0; c < kCopies; ++c) v += part[u][c];
            if (beam_key == i + 1) v += beam_v;
            const bool is_side = i < n_side;
            const uint64_t j = is_side ? i : i - n_side;
            if (FIX) ((long long *)(is_side ? side : trans))[j] = prev[u] + (long long)v;
            else ((double *)(is_side ? side : trans))[j] =
                __longlong_as_double(prev[u]) + (double)(long long)v * (1.0 / kFix);
            if (is_side) sum_side += v; else sum_trans += v;
        }
    }
    if (face_side) {
        // One atomic per block and face: same-address global atomics serialise.
        __shared__ unsigned long long s_part[2][4];
        sum_side = wave_sum(sum_side);
        sum_trans = wave_sum(sum_trans);
        const int wave = threadIdx.x >> 6;
        if (__lane_id() == 0) {
            s_part[0][wave] = sum_side;
            s_part[1][wave] = sum_trans;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned long long a0 = s_part[0][0] + s_part[0][1] + s_part[0][2] + s_part[0][3];
            const unsigned long long a1 = s_part[1][0] + s_part[1][1] + s_part[1][2] + s_part[1][3];
            if (a0) atomicAdd(face_side, a0);
            if (a1) atomicAdd(face_trans, a1);
        }
    }
}

// Fixed-point scalar sums to the caller's doubles (weights scaled back by
// 2^-32, counts as they are); the second-order side moments are FP64 sums.
// One medium per block.
__global__ void finalize_scalars(const unsigned long long *ws_scal, double *scalars)
{
    ws_scal += (uint64_t)blockIdx.x * kWsScalarWords;
    scalars += (uint64_t)blockIdx.x * MC_N_SCALARS;
    const int t = threadIdx.x;
    if (t < MC_S_RESERVED) {
        const bool weight = t <= MC_S_CAPPED_W;
        long long v = (long long)ws_scal[t];
        // Reflections are not counted by the walk: every step interacts or
        // reaches a wall, and a wall step reflects unless the photon leaves,
        // which every photon not killed by roulette or capped does once.
        if (t == MC_S_REFLECTIONS)
            v = (long long)(ws_scal[MC_S_STEPS] - ws_scal[MC_S_EVENTS] -
                            (ws_scal[MC_S_PHOTONS] - ws_scal[MC_S_ROULETTE_KILLS] - ws_scal[MC_S_CAPPED]));
        scalars[t] += weight ? (double)v * (1.0 / kFix) : (double)v;
    } else if (t >= MC_S_SIDE_W2 && t <= MC_S_SIDE_W2L) {
        scalars[t] += __longlong_as_double((long long)ws_scal[t]);
    }
}

__global__ void philox_blocks_kernel(uint32_t k0, uint32_t k1, uint32_t instance, const uint64_t *ids,
                                     uint64_t n_ids, uint32_t step0, uint32_t n_steps, uint32_t *out)
{
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_ids * (uint64_t)n_steps) return;
    const uint64_t i = t / n_steps;
    const uint32_t st = step0 + (uint32_t)(t % n_steps);
    const uint64_t id = ids[i];
    const Block4 r = philox4x32_10(st, instance, (uint32_t)id, (uint32_t)(id >> 32), k0, k1);
    out[4 * t + 0] = r.r0;
    out[4 * t + 1] = r.r1;
    out[4 * t + 2] = r.r2;
    out[4 * t + 3] = r.r3;
}

// sum_p g_p M_k[p], sum_p g_p M_L[p] and, with per-pixel h, sum_p h_p M2_k[p]
// and sum_p h_p M2_L[p], in two passes with a fixed order (deterministic):
// block b of grad_partial sums pixels b x 1024 + t + j x (gridDim x 1024) per
// lane t, then over the block by a fixed tree, into part[4 b .. 4 b + 3];
// grad_final adds the blocks' partials in block order.  With a uniform h
// instead, h times the image-wide second moments.
__global__ __launch_bounds__(1024) void grad_partial(const double *g, const double *h, const double *wk,
                                                     const double *wl, const double *w2k, const double *w2l,
                                                     uint64_t n, double *part)
{
    __shared__ double s_red[4][1024];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        acc[0] = fma(g[i], wk[i], acc[0]);
        acc[1] = fma(g[i], wl[i], acc[1]);
        if (h) {
            acc[2] = fma(h[i], w2k[i], acc[2]);
            acc[3] = fma(h[i], w2l[i], acc[3]);
        }
    }
    for (int c = 0; c < 4; ++c) s_red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int c = 0; c < 4; ++c) s_red[c][threadIdx.x] += s_red[c][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x < 4) part[4 * (uint64_t)blockIdx.x + threadIdx.x] = s_red[threadIdx.x][0];
}

__global__ void grad_final(const double *part, uint32_t n_blocks, bool per_pixel_h, double h_uniform,
                           const double *scalars, double *out)
{
    if (threadIdx.x >= 4) return;
    double v = 0.0;
    for (uint32_t b = 0; b < n_blocks; ++b) v += part[4 * (uint64_t)b + threadIdx.x];
    if (!per_pixel_h && threadIdx.x >= 2)
        v = h_uniform != 0.0 ? h_uniform * scalars[threadIdx.x == 2 ? MC_S_SIDE_W2K : MC_S_SIDE_W2L] : 0.0;
    out[threadIdx.x] = v;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// Workspace layout: per medium kWsScalarWords uint64 scalar words (0..14
// fixed-point scalar sums, 15 the photon work counter (first medium), 16..18
// FP64 second-order side moments, 24..27 mc_grad's dot products), then
// kCopies fixed-point copies of the images of every medium (and of the
// squared-weight images with MC_SIGMA); a batched launch appends its schedule
// (one BatchInst per medium).
uint64_t workspace_words(const mc_detector_t &d, uint64_t n_inst = 1, uint64_t copies = kCopies)
{
    const uint64_t n_pix = (uint64_t)d.side_nx * d.side_ny + (uint64_t)d.trans_nx * d.trans_ny;
    return kWsScalarWords * n_inst + copies * n_pix * n_inst * ((d.flags & MC_SIGMA) ? 2 : 1);
}

// The exit log (MC_EXIT_LOG) follows the workspace words (and a batched
// launch's schedule): the counts of 2^rbits x blocks regions (uint32, padded
// to 8 bytes), then the regions of cap entries each, with cap the largest
// the caller's workspace holds.  The key width and range bits follow from
// the number of keys: a range of at most 2^kLogHistBits keys where the LDS
// takes 2^rbits counters (up to 2^8 beside a Mie table, 2^12 otherwise).
constexpr uint64_t kLogSizingBlocks = 256 * 2;   // resident blocks of a full MI355X launch
struct LogShape {
    uint32_t bits, rbits;
};
LogShape log_shape(uint64_t n_keys, bool table_in_lds)
{
    const uint64_t groups = (n_keys + 7) / 8;
    uint32_t bits = 1;
    while ((1ull << bits) < groups) ++bits;
    const uint32_t max_r = table_in_lds ? 8u : 12u;
    const uint32_t want = bits > kLogHistBits - 3 ? bits - (kLogHistBits - 3) : 0u;
    const uint32_t rbits = std::min(max_r, std::max(kLogMinRangeBits, want));
    return {std::max(bits, rbits), rbits};
}
// Region capacities are whole granules of entries: 256 (2 KiB of region
// stride) from 1024 entries up, else 64.  The binning pass streams thousands
// of regions at once, one per wave, and its read rate depends on their
// stride: at 512 blocks x 64 regions of 2100 entries, every capacity of a
// multiple of 256 entries from 2304 to 8192 read at 5.5-5.9 TB/s, while some
// other capacities lost up to a quarter of that (4640 or 4641 entries:
// 4.6 TB/s; 8128: 4.3 TB/s).
uint64_t log_cap_granule(uint64_t cap) { return cap >= 1024 ? 256 : 64; }
uint32_t log_cap_for(uint64_t extra_bytes, uint64_t regions)
{
    const uint64_t count_bytes = (regions * 4 + 7) / 8 * 8;
    if (regions == 0 || extra_bytes < count_bytes) return 0;
    uint64_t cap = (extra_bytes - count_bytes) / (regions * 8);
    // Entry positions are 32-bit.
    cap = std::min<uint64_t>(cap, 0x7FFFFF00ull);
    if (cap >= 64) cap -= cap % log_cap_granule(cap);
    return (uint32_t)cap;
}
// Log bytes for n_photons over `regions` regions: each photon leaves through an
// image at most once; spread evenly over the ranges and the blocks of a full
// launch, a region gets about n / regions entries, and holds half as many again
// (for uneven spread and unequal shares of photons) plus 64, rounded up to a
// whole granule (so that log_cap_for gives back exactly this capacity).
uint64_t log_bytes_for(uint64_t n_photons, uint64_t regions)
{
    uint64_t cap = std::min<uint64_t>((n_photons + n_photons / 2 + regions - 1) / regions + 64, 0x7FFFFF00ull);
    const uint64_t gr = log_cap_granule(cap);
    cap = (cap + gr - 1) / gr * gr;
    return (regions * 4 + 7) / 8 * 8 + regions * cap * 8;
}

uint64_t batch_workspace_words(const mc_detector_t &d, uint64_t n_items)
{
    return workspace_words(d, n_items) + (n_items * sizeof(BatchInst) + 7) / 8;
}

bool dims_ok(const mc_detector_t &d) { return d.side_nx >= 1 && d.side_ny >= 1 && d.trans_nx >= 1 && d.trans_ny >= 1; }

// Checks of the cuboid and its walls (Sec. 3.1.1: parameter validity).
int check_geometry(const char *fn, const mc_geometry_t &geo)
{
    for (int i = 0; i < 3; ++i)
        if (!finite_pos(geo.size_mm[i])) return fail(MC_EINVAL, "%s: size_mm[%d] must be > 0", fn, i);
    if (!finite_pos(geo.n_medium) || !finite_pos(geo.n_outside))
        return fail(MC_EINVAL, "%s: refractive indices must be > 0", fn);
    return MC_OK;
}

// Component i of the beam direction inside the medium (refracted at the
// z = 0 face, Snell), as the walk gets it: FP32, a zero always +0.
float entry_dir(const mc_source_t &src, const mc_geometry_t &geo, int i)
{
    const double dl = std::sqrt(src.dir[0] * src.dir[0] + src.dir[1] * src.dir[1] + src.dir[2] * src.dir[2]);
    const double eta = geo.n_outside / geo.n_medium;
    double d[3] = {eta * (src.dir[0] / dl), eta * (src.dir[1] / dl), 0.0};
    d[2] = std::sqrt(std::max(0.0, 1.0 - d[0] * d[0] - d[1] * d[1]));
    const float f = (float)d[i];
    return f == 0.f ? 0.f : f;   // -0 (or an underflow to it) becomes +0
}

// Checks of the source, detector, tally buffers and run settings shared by
// single and batched walks.
int check_setup(const char *fn, const mc_source_t &src, const mc_geometry_t &geo, const mc_detector_t &det,
                const mc_run_t &rn, const mc_tally_t &t)
{
    if (!(src.pos_mm[2] == 0.0) || !(src.pos_mm[0] >= 0.0 && src.pos_mm[0] <= geo.size_mm[0]) ||
        !(src.pos_mm[1] >= 0.0 && src.pos_mm[1] <= geo.size_mm[1]))
        return fail(MC_EINVAL, "%s: the source must lie on the z = 0 face", fn);
    const double dl = std::sqrt(src.dir[0] * src.dir[0] + src.dir[1] * src.dir[1] + src.dir[2] * src.dir[2]);
    if (!(dl > 0.0) || !std::isfinite(dl) || !(src.dir[2] > 0.0))
        return fail(MC_EINVAL, "%s: the source direction must point into the cuboid (dir[2] > 0)", fn);
    const double R = src.beam_radius_mm;
    if (!(R >= 0.0) || !std::isfinite(R))
        return fail(MC_EINVAL, "%s: beam_radius_mm must be finite and >= 0", fn);
    if (R > 0.0 && (src.pos_mm[0] - R < 0.0 || src.pos_mm[0] + R > geo.size_mm[0] || src.pos_mm[1] - R < 0.0 ||
                    src.pos_mm[1] + R > geo.size_mm[1]))
        return fail(MC_EINVAL, "%s: the beam disk must lie inside the z = 0 face", fn);
    // A photon exactly on a side wall with no direction component across it
    // would meet that wall at distance 0 (the walk's wall distance has no
    // zero-component test): keep the entry points off the far side walls
    // when the refracted beam runs parallel to them.
    for (int i = 0; i < 2; ++i)
        if (entry_dir(src, geo, i) == 0.f && (float)src.pos_mm[i] + (float)R >= (float)geo.size_mm[i])
            return fail(MC_EINVAL, "%s: the beam must not run along the face %s = %g", fn, i ? "y" : "x",
                        geo.size_mm[i]);
    if (!dims_ok(det)) return fail(MC_EINVAL, "%s: image dimensions must be >= 1", fn);
    if (!t.side || !t.trans || !t.scalars) return fail(MC_EINVAL, "%s: side, trans and scalars are required", fn);
    if ((det.flags & MC_SIGMA) && (!t.side_w2 || !t.trans_w2))
        return fail(MC_EINVAL, "%s: MC_SIGMA needs side_w2 and trans_w2", fn);
    if (rn.max_steps < 1 || rn.max_steps > (1u << 24))
        return fail(MC_EINVAL, "%s: max_steps must be in 1..2^24", fn);
    if (!(rn.roulette_w >= 0.0) || !(rn.roulette_p > 0.0 && rn.roulette_p <= 1.0))
        return fail(MC_EINVAL, "%s: roulette_w >= 0 and roulette_p in (0, 1] required", fn);
    if (rn.block_size != 0 && (rn.block_size < 64 || rn.block_size > 1024 || rn.block_size % 64))
        return fail(MC_EINVAL, "%s: block_size must be a multiple of 64 in 64..1024", fn);
    if (rn.grid_blocks < 0) return fail(MC_EINVAL, "%s: grid_blocks must be >= 0", fn);
    if (rn.chunk > 65536) return fail(MC_EINVAL, "%s: chunk must be at most 65536", fn);
    return MC_OK;
}

// Fixed-point sums stay below 2^63: every weight is at most
// max(1, roulette_w / roulette_p), so n_photons times that (squared for
// MC_SIGMA) must stay below 2^31.
int check_overflow(const char *fn, uint64_t n_photons, const mc_detector_t &det, const mc_run_t &rn)
{
    const double wmax = std::max(1.0, rn.roulette_w / rn.roulette_p);
    const double bound = (double)n_photons * ((det.flags & MC_SIGMA) ? wmax * wmax : wmax);
    if (!(bound < 2147483648.0))
        return fail(MC_EINVAL, "%s: %llu photons with weights up to %g could overflow the fixed-point tallies; "
                    "split the run into photon ranges", fn, (unsigned long long)n_photons, wmax);
    return MC_OK;
}

// Launch-independent kernel arguments: the cuboid and its walls, the entry
// beam (refracted at the z = 0 face, keeping 1 - R of its weight), roulette,
// the Philox key and the detector.
void fill_common(WalkArgs &a, const mc_source_t &src, const mc_geometry_t &geo, const mc_detector_t &det,
                 const mc_run_t &rn)
{
    for (int i = 0; i < 3; ++i) a.size[i] = (float)geo.size_mm[i];
    a.matched = geo.n_outside == geo.n_medium;
    a.n21 = (float)(geo.n_outside / geo.n_medium);
    a.n12 = (float)(geo.n_medium / geo.n_outside);
    a.n12sq = (float)((geo.n_medium / geo.n_outside) * (geo.n_medium / geo.n_outside));
    const double dl = std::sqrt(src.dir[0] * src.dir[0] + src.dir[1] * src.dir[1] + src.dir[2] * src.dir[2]);
    double din[3] = {src.dir[0] / dl, src.dir[1] / dl, src.dir[2] / dl};
    double R0 = 0.0;
    if (!a.matched) {
        const double n1 = geo.n_outside, n2 = geo.n_medium, ci = din[2];
        const double si = std::sqrt(std::max(0.0, 1.0 - ci * ci)), st = n1 / n2 * si;
        if (st >= 1.0) {
            R0 = 1.0;
        } else {
            const double ct = std::sqrt(1.0 - st * st);
            const double rs = (n1 * ci - n2 * ct) / (n1 * ci + n2 * ct);
            const double rp = (n2 * ci - n1 * ct) / (n2 * ci + n1 * ct);
            R0 = 0.5 * (rs * rs + rp * rp);
        }
    }
    for (int i = 0; i < 3; ++i) {
        a.pos0[i] = (float)src.pos_mm[i];
        a.dir0[i] = entry_dir(src, geo, i);
    }
    a.w0 = (float)(1.0 - R0);
    a.beam_radius = (float)src.beam_radius_mm;
    a.roulette_w = (float)rn.roulette_w;
    a.roulette_p = (float)rn.roulette_p;
    a.inv_roulette_p = (float)(1.0 / rn.roulette_p);
    a.key0 = (uint32_t)rn.seed;
    a.key1 = (uint32_t)(rn.seed >> 32);
    a.max_steps = rn.max_steps;
    a.flags = det.flags;
    a.side_nx = det.side_nx; a.side_ny = det.side_ny;
    a.trans_nx = det.trans_nx; a.trans_ny = det.trans_ny;
    a.pix_scale[0] = (float)(det.side_ny / geo.size_mm[1]);
    a.pix_scale[1] = (float)(det.side_nx / geo.size_mm[2]);
    a.pix_scale[2] = (float)(det.trans_ny / geo.size_mm[1]);
    a.pix_scale[3] = (float)(det.trans_nx / geo.size_mm[0]);
    a.copy_mask = kCopies - 1;
    a.n_side = (uint32_t)((uint64_t)det.side_nx * det.side_ny);
    a.n_pix_inst = (uint32_t)((uint64_t)det.side_nx * det.side_ny + (uint64_t)det.trans_nx * det.trans_ny);
}

// Per-medium coefficients (Eq. 1 and Eq. 16): s = log2(u0) * neg_ln2_over_mu.
void fill_medium(float &neg_ln2_over_mu, float &albedo, float &absorb, double mu_t, double alb)
{
    neg_ln2_over_mu = mu_t > 0.0 ? (float)(-M_LN2 / mu_t) : -__builtin_huge_valf();
    albedo = (float)alb;
    absorb = (float)(1.0 - alb);
}

// A medium's coefficients in 1/mm from the form the caller gave them in.
struct MediumCoef {
    double mu_sca, mu_abs, mu_ext, albedo;
};

bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }

// Eq. 1 (optical depth along the beam axis), Eq. 16 (albedo) or Eq. 17
// (concentration times the cross-sections of Eq. 14), validated.  The optical
// depth form keeps mu_ext = tau / size_z and the given albedo exactly, the
// others form mu_ext as the sum and the albedo as the quotient.
int medium_coefficients(const char *fn, const mc_medium_t &m, double size_z, MediumCoef &c)
{
    const bool sig_ok = finite_nonneg(m.sigma_sca_mm2) && finite_nonneg(m.sigma_abs_mm2);
    if (m.input == MC_MEDIUM_TAU) {
        if (!finite_nonneg(m.tau)) return fail(MC_EINVAL, "%s: tau must be finite and >= 0", fn);
        double alb = m.albedo;
        if (alb < 0.0) {
            if (!sig_ok || !(m.sigma_sca_mm2 + m.sigma_abs_mm2 > 0.0))
                return fail(MC_EINVAL, "%s: albedo < 0 takes sigma_sca / (sigma_sca + sigma_abs), which needs "
                                       "cross-sections >= 0 with a positive sum", fn);
            alb = m.sigma_sca_mm2 / (m.sigma_sca_mm2 + m.sigma_abs_mm2);
        } else if (!(alb <= 1.0)) {
            return fail(MC_EINVAL, "%s: albedo must be in [0, 1] (or < 0 to derive it)", fn);
        }
        c.mu_ext = m.tau / size_z;
        c.albedo = alb;
        c.mu_sca = alb * c.mu_ext;
        c.mu_abs = (1.0 - alb) * c.mu_ext;
        return MC_OK;
    }
    if (m.input == MC_MEDIUM_MU) {
        if (!finite_nonneg(m.mu_sca) || !finite_nonneg(m.mu_abs))
            return fail(MC_EINVAL, "%s: mu_sca and mu_abs must be finite and >= 0", fn);
        c.mu_sca = m.mu_sca;
        c.mu_abs = m.mu_abs;
    } else if (m.input == MC_MEDIUM_CONCENTRATION) {
        if (!finite_nonneg(m.concentration_per_mm3) || !sig_ok || !finite_nonneg(m.mu_abs_host))
            return fail(MC_EINVAL, "%s: concentration, cross-sections and mu_abs_host must be finite and >= 0", fn);
        c.mu_sca = m.concentration_per_mm3 * m.sigma_sca_mm2;
        c.mu_abs = m.concentration_per_mm3 * m.sigma_abs_mm2 + m.mu_abs_host;
        if (!std::isfinite(c.mu_sca) || !std::isfinite(c.mu_abs))
            return fail(MC_EINVAL, "%s: the coefficients overflow", fn);
    } else {
        return fail(MC_EINVAL, "%s: unknown medium input %d", fn, m.input);
    }
    c.mu_ext = c.mu_sca + c.mu_abs;
    if (!std::isfinite(c.mu_ext)) return fail(MC_EINVAL, "%s: the coefficients overflow", fn);
    c.albedo = c.mu_ext > 0.0 ? c.mu_sca / c.mu_ext : 1.0;
    return MC_OK;
}

// A batched launch's schedule is written into the workspace by small kernels
// whose arguments carry up to kInstPerCopy media each (no host buffer has to
// outlive the call).
constexpr int kInstPerCopy = 32;
constexpr uint32_t kRefillMin = 12;        // free lanes of a wave that trigger end-of-photon work (batched)

// The same for a single medium of optical depth tau along the beam axis,
// from a sweep of thresholds 4..60 at tau = 0.25..16 (1e8 photons, 512 x 512,
// exit log): 12 is within 2 % of the best from tau = 1.5 to 12.5 and 8 at 16;
// media up to tau = 1 end most photons within two steps, and there refilling
// only when 52 lanes are free (nearly the whole wave at once) ran 19 % faster
// at tau = 1 than 12 and no slower below it.
uint32_t refill_min_for(double tau)
{
    if (!(tau >= 0.0)) return kRefillMin;
    if (tau <= 1.05) return 52;
    return tau < 14.0 ? 12 : 8;
}

// Photon ids a wave claims at once (single medium, when the caller leaves
// it to the library): 16 claims per wave, at most 1024.  Every claim is one
// device-scope atomic on one word, which takes about 78 million per second
// (at 256 ids per claim the tau = 4 walk took 5.0 ms instead of 2.75); where
// photons end within a few steps that rate binds, so below tau = 3 a claim
// takes 2048 ids (up to tau = 1.05) or 3072, but no fewer than four claims
// per wave.  mc_simulate at 1e8 photons, 512 x 512: tau = 0.5 1.84 -> 1.21
// ms, tau = 1 1.91 -> 1.58, tau = 2 2.04 -> 1.88; tau = 4 and 8 ran alike
// from 384 to 1536 ids.
uint64_t chunk_for(uint64_t total_photons, uint64_t waves_total, double tau)
{
    uint64_t chunk = std::min<uint64_t>(1024, total_photons / std::max<uint64_t>(1, waves_total * 16));
    if (tau >= 0.0 && tau < 3.0)
        chunk = std::max(chunk, std::min<uint64_t>(tau <= 1.05 ? 2048 : 3072,
                                                   total_photons / std::max<uint64_t>(1, waves_total * 4)));
    return std::max<uint64_t>(64, (chunk + 63) / 64 * 64);
}

struct InstChunk {
    BatchInst v[kInstPerCopy];
    uint32_t n, first;
};

__global__ void set_schedule(BatchInst *dst, InstChunk c)
{
    if (threadIdx.x < c.n) dst[c.first + threadIdx.x] = c.v[threadIdx.x];
}

// Enqueue init, walk and finalize for n_inst media (a single medium, or a
// batch whose schedule `sched` is given) on `st`.
int launch_walk(WalkArgs &a, const mc_detector_t &det, const mc_run_t &rn, const mc_tally_t &t, int phase,
                uint32_t n_inst, uint64_t total_photons, const std::vector<BatchInst> *sched, hipStream_t st)
{
    const bool batch = sched != nullptr;
    int cus = 0;
    if (int rc = device_cu_count(&cus)) return rc;
    const uint64_t n_pix = a.n_pix_inst, n_side = a.n_side, n_trans = n_pix - n_side;
    const uint64_t n_total = n_pix * n_inst;
    unsigned long long *ws = (unsigned long long *)t.workspace;
    const uint64_t max_copies = (uint64_t)a.copy_mask + 1;
    a.ws_scal = ws;
    a.ws_img = ws + kWsScalarWords * n_inst;
    a.n_pix = n_total;
    a.n_inst = n_inst;

    // A batched launch keeps its schedule after the workspace words; the exit
    // log follows: its counts, then the regions.  A workspace without room for
    // the counts takes the atomic path (the same sums).
    const uint64_t sched_words = batch ? (n_inst * sizeof(BatchInst) + 7) / 8 : 0;
    const LogShape shape = log_shape(n_total, !batch && phase == MC_PHASE_MIE);
    // Keys of a range have indices below 2^(bits - rbits + 3); log_bin takes
    // them in parts of 2^kLogHistBits.
    const uint64_t per_range = 1ull << (shape.bits - shape.rbits + 3);
    const uint32_t parts = (uint32_t)((per_range + (1u << kLogHistBits) - 1) >> kLogHistBits);
    // With the exit log the image copies take log_bin's sums (and the rare
    // fallback atomics): as many copies as give it kLogBinBlocks blocks, so
    // that fine key ranges (large images, batches) leave fewer copies to clear
    // and to sum.  Without it, one per XCD for the image atomics.  The
    // workspace layout keeps room for all of them either way (the schedule and
    // the log start at the same place); the copies in use come first.
    auto copies_for = [&](bool log) -> uint64_t {
        if (!log) return max_copies;
        const uint64_t bin_blocks = ((uint64_t)1 << shape.rbits) * parts;
        uint64_t c = 1;
        while (c < max_copies && bin_blocks * c < kLogBinBlocks) c <<= 1;
        return c;
    };

    // ---- launch shape: 1024-lane blocks (768 with path moments), two per CU, each with
    // the table (single medium), the scalar words, the per-wave exit queues and
    // as large a tally cache as fits in half the CU's 160 KB LDS (with the exit
    // log: the block's append counters and no cache) ----
    // Path-moment kernels are built for six waves per SIMD: 768-lane blocks,
    // two per CU.
    const int block = rn.block_size ? rn.block_size : ((det.flags & MC_MOMENTS) ? 768 : 1024);
    const size_t table_bytes = batch ? 0 : (size_t)((a.n_cdf + 3) & ~3) * sizeof(float);
    const size_t scal_bytes = (batch ? (size_t)n_inst * kBatchScal : MC_N_SCALARS) * sizeof(double);
    const size_t queue_arrays = batch ? 4 : 3;
    const size_t slot_bytes = sizeof(uint32_t) + sizeof(double) * ((det.flags & MC_SIGMA) ? 2 : 1);
    const size_t lds_half_cu = 80 * 1024;
    size_t lds = 0;
    int grid = 0;
    auto launch_shape = [&](bool log) {
        const size_t lds_fixed = table_bytes + scal_bytes + (size_t)(block / 64) * queue_arrays * kQueue * sizeof(float) +
                                 (log ? ((size_t)4 << shape.rbits) : 0);
        a.cache_bits = 0;
        for (int b = 10; b >= 4 && !log; --b)
            if (lds_fixed + (slot_bytes << b) <= lds_half_cu) { a.cache_bits = b; break; }
        lds = lds_fixed + (a.cache_bits ? (slot_bytes << a.cache_bits) : 0);
        const int blocks_per_cu = std::max(1, std::min((int)(160 * 1024 / lds), 32 / (block / 64)));
        grid = rn.grid_blocks > 0 ? rn.grid_blocks : cus * blocks_per_cu;
    };
    const uint64_t ws_words = workspace_words(det, n_inst, max_copies);
    bool use_log = (det.flags & MC_EXIT_LOG) != 0;
    launch_shape(use_log);
    if (use_log && t.workspace_bytes / 8 < ws_words + sched_words + (((uint64_t)grid << shape.rbits) * 4 + 7) / 8) {
        use_log = false;
        launch_shape(false);
    }
    const uint64_t copies = copies_for(use_log);
    // With the exit log the walk's only image atomics are its fallback ones
    // (an exit whose region is full): all of them go to copy 0.
    a.copy_mask = use_log ? 0u : (uint32_t)(copies - 1);
    a.ws_img2 = (det.flags & MC_SIGMA) ? a.ws_img + copies * n_total : nullptr;
    if (lds > 160 * 1024) return fail(MC_EINVAL, "mc_simulate: %zu bytes of LDS per block do not fit a CU", lds);
    const uint64_t waves_total = (uint64_t)grid * (block / 64);
    // The optical depth along the beam axis (negative for a batch).
    const double tau_z = !batch && a.neg_ln2_over_mu < 0.f && std::isfinite(a.neg_ln2_over_mu)
                             ? -M_LN2 / (double)a.neg_ln2_over_mu * a.size[2]
                             : -1.0;
    uint64_t chunk = rn.chunk;
    if (chunk == 0) chunk = chunk_for(total_photons, waves_total, batch ? -1.0 : tau_z);
    a.chunk = (uint32_t)chunk;
    // Refill threshold from the optical depth; batched launches take the
    // fixed one (12 ran 1 % faster there than 16, and 8 and 24 slower).
    a.refill_min = batch ? kRefillMin : refill_min_for(tau_z >= 0.0 ? tau_z : 0.0);

    // ---- exit log: a region of log_cap entries per block and key range in
    // what the caller gave beyond the workspace words (the walk writes every
    // count, so nothing needs clearing) ----
    // What init clears: the scalar words and every image copy, except when
    // log_bin will run (the exit log and some photons): then only copy 0 (and
    // copy 0 of the squared weights), since log_bin stores into the others.
    const bool bin_stores = use_log && total_photons > 0;
    const uint64_t clear_words = bin_stores ? kWsScalarWords * n_inst + n_total : workspace_words(det, n_inst, copies);
    unsigned long long *clear2 = bin_stores && (det.flags & MC_SIGMA) ? a.ws_img2 : nullptr;
    const uint64_t clear2_words = clear2 ? n_total : 0;
    if (use_log) {
        const uint64_t regions = ((uint64_t)1 << shape.rbits) * grid;
        const uint64_t log_at = ws_words + sched_words;
        a.log_cap = t.workspace_bytes > log_at * 8 ? log_cap_for(t.workspace_bytes - log_at * 8, regions) : 0;
        a.log_count = (uint32_t *)(ws + log_at);
        a.log = ws + log_at + (regions * 4 + 7) / 8;
        a.log_bits = shape.bits;
        a.log_rbits = shape.rbits;
    }

    const int zero_all = (det.flags & MC_ACCUMULATE) ? 0 : 1;
    const bool sig = (det.flags & MC_SIGMA) != 0, rec = (det.flags & MC_RECORD) != 0;
    // The caller's timing events ride on the dispatches themselves
    // (hipExtLaunchKernel): a separate event record would put a barrier, and
    // several microseconds of idle device, between two kernels.
    hipExtLaunchKernelGGL(init_kernel, dim3(1024), dim3(256), 0, st, (hipEvent_t)rn.sim_events[0], nullptr, 0u, ws,
                          (size_t)clear_words, clear2,
                       (size_t)clear2_words, (unsigned long long *)t.side, (unsigned long long *)t.trans,
                       sig ? (unsigned long long *)t.side_w2 : nullptr, sig ? (unsigned long long *)t.trans_w2 : nullptr,
                       (size_t)(n_side * n_inst), (size_t)(n_trans * n_inst), t.scalars,
                       (size_t)MC_N_SCALARS * n_inst, a.rec_i, a.rec_f, (size_t)a.rec_rows, a.side_wk, a.side_wl,
                       a.side_w2k, a.side_w2l, zero_all);
    MC_HIP_CHECK(hipGetLastError());

    using Kern = void (*)(WalkArgs);
    Kern kern = nullptr;
    uint64_t units = 0;
    if (batch) {
        // The schedule: unit ranges in schedule order, copied after the scalars
        // and images of the workspace (after init has cleared it).
        BatchInst *dst = (BatchInst *)(ws + ws_words);
        std::vector<BatchInst> s = *sched;
        for (auto &b : s) {
            b.unit_begin = units;
            units += (b.n_photons + chunk - 1) / chunk;
        }
        for (uint32_t i = 0; i < n_inst; i += kInstPerCopy) {
            InstChunk c{};
            c.first = i;
            c.n = std::min<uint32_t>(kInstPerCopy, n_inst - i);
            for (uint32_t j = 0; j < c.n; ++j) c.v[j] = s[i + j];
            hipLaunchKernelGGL(set_schedule, dim3(1), dim3(kInstPerCopy), 0, st, dst, c);
        }
        MC_HIP_CHECK(hipGetLastError());
        a.insts = dst;
        a.n_units = units;
        static const Kern batch_kernels[4] = {
            walk_kernel<MC_PHASE_MIE, kOptBatch>, walk_kernel<MC_PHASE_MIE, kOptBatch | kOptSigma>,
            walk_kernel<MC_PHASE_MIE, kOptBatch | kOptLog>, walk_kernel<MC_PHASE_MIE, kOptBatch | kOptLog | kOptSigma>};
        kern = batch_kernels[(sig ? 1 : 0) + (use_log ? 2 : 0)];
    } else {
        const int opt = (sig ? kOptSigma : 0) | (rec ? kOptRecord : 0) | ((det.flags & MC_MOMENTS) ? kOptMoments : 0);
        static const Kern mie_kernels[8] = {walk_kernel<MC_PHASE_MIE, 0>, walk_kernel<MC_PHASE_MIE, 1>,
                                            walk_kernel<MC_PHASE_MIE, 2>, walk_kernel<MC_PHASE_MIE, 3>,
                                            walk_kernel<MC_PHASE_MIE, 4>, walk_kernel<MC_PHASE_MIE, 5>,
                                            walk_kernel<MC_PHASE_MIE, 6>, walk_kernel<MC_PHASE_MIE, 7>};
        static const Kern hg_kernels[8] = {walk_kernel<MC_PHASE_HG, 0>, walk_kernel<MC_PHASE_HG, 1>,
                                           walk_kernel<MC_PHASE_HG, 2>, walk_kernel<MC_PHASE_HG, 3>,
                                           walk_kernel<MC_PHASE_HG, 4>, walk_kernel<MC_PHASE_HG, 5>,
                                           walk_kernel<MC_PHASE_HG, 6>, walk_kernel<MC_PHASE_HG, 7>};
        kern = phase == MC_PHASE_MIE ? mie_kernels[opt] : hg_kernels[opt];
        if (use_log) {
            // Exit log with optional squared weights and path moments (index
            // sigma + 2 x moments); records take the atomic path.
            static const Kern log_kernels[8] = {
                walk_kernel<MC_PHASE_MIE, kOptLog>, walk_kernel<MC_PHASE_MIE, kOptLog | kOptSigma>,
                walk_kernel<MC_PHASE_MIE, kOptLog | kOptMoments>,
                walk_kernel<MC_PHASE_MIE, kOptLog | kOptMoments | kOptSigma>,
                walk_kernel<MC_PHASE_HG, kOptLog>, walk_kernel<MC_PHASE_HG, kOptLog | kOptSigma>,
                walk_kernel<MC_PHASE_HG, kOptLog | kOptMoments>,
                walk_kernel<MC_PHASE_HG, kOptLog | kOptMoments | kOptSigma>};
            kern = log_kernels[(phase == MC_PHASE_MIE ? 0 : 4) + (sig ? 1 : 0) +
                               ((det.flags & MC_MOMENTS) ? 2 : 0)];
        }
        units = total_photons;
    }
    if (units > 0) {
        MC_HIP_CHECK(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipExtLaunchKernelGGL(kern, dim3(grid), dim3(block), (uint32_t)lds, st, (hipEvent_t)rn.walk_events[0],
                              (hipEvent_t)rn.walk_events[1], 0u, a);
        MC_HIP_CHECK(hipGetLastError());
    } else {
        // No walk: the events mark the (empty) place where it would run.
        if (rn.walk_events[0]) MC_HIP_CHECK(hipEventRecord((hipEvent_t)rn.walk_events[0], st));
        if (rn.walk_events[1]) MC_HIP_CHECK(hipEventRecord((hipEvent_t)rn.walk_events[1], st));
    }
    if (use_log && units > 0) {
        uint32_t inv = kLogHashMul;   // inverse of the odd multiplier mod 2^32 (Newton: x <- x (2 - m x))
        for (int i = 0; i < 5; ++i) inv *= 2u - kLogHashMul * inv;
        const size_t hist = ((size_t)8 << kLogHistBits) * (sig ? 2 : 1);
        auto bin = sig ? log_bin<true> : log_bin<false>;
        MC_HIP_CHECK(hipFuncSetAttribute((const void *)bin, hipFuncAttributeMaxDynamicSharedMemorySize, (int)hist));
        hipLaunchKernelGGL(bin, dim3((1u << a.log_rbits) * parts * (uint32_t)copies), dim3(1024), hist, st,
                           (const unsigned long long *)a.log, (const uint32_t *)a.log_count, a.log_cap,
                           (uint32_t)grid, a.ws_img, a.ws_img2, (uint32_t)copies, n_total, parts, a.log_bits,
                           a.log_rbits, inv);
        MC_HIP_CHECK(hipGetLastError());
    }
    // ---- finalize: per-XCD copies to the caller's images, scalars to doubles ----
    const bool fix64 = (det.flags & MC_FIX64) != 0;
    const unsigned fin_x = (unsigned)std::max<uint64_t>(1, std::min<uint64_t>(batch ? 64 : 512, (n_pix + 255) / 256));
    auto fin = fix64 ? finalize_images<true> : finalize_images<false>;
    // The fixed-point weight (and squared weight, an FP32 product as in the
    // walk) of an unscattered first-step exit, as the walk's fix() rounds it.
    const float w0sq = a.w0 * a.w0;
    const unsigned long long ball_w = (unsigned long long)std::llrint((double)a.w0 * kFix);
    const unsigned long long ball_w2 = (unsigned long long)std::llrint((double)w0sq * kFix);
    hipLaunchKernelGGL(fin, dim3(fin_x, n_inst), dim3(256), 0, st, a.ws_img, (int)copies, n_total, n_pix,
                       (uint32_t)n_side, t.side, t.trans, ws + MC_S_FACE + 1, ws + MC_S_FACE + 5, kWsScalarWords,
                       (const unsigned long long *)ws, ball_w);
    if (sig)
        hipLaunchKernelGGL(fin, dim3(fin_x, n_inst), dim3(256), 0, st, a.ws_img2, (int)copies, n_total, n_pix,
                           (uint32_t)n_side, t.side_w2, t.trans_w2, (unsigned long long *)nullptr,
                           (unsigned long long *)nullptr, kWsScalarWords, (const unsigned long long *)ws, ball_w2);
    hipExtLaunchKernelGGL(finalize_scalars, dim3(n_inst), dim3(64), 0, st, nullptr, (hipEvent_t)rn.sim_events[1], 0u,
                          (const unsigned long long *)ws, t.scalars);
    MC_HIP_CHECK(hipGetLastError());
    return MC_OK;
}

// Checks and schedule of a batched launch (items in decreasing estimated
// cost, photons x (1 + tau), so the longest start first).
int prepare_batch(const char *fn, const mc_batch_item_t *items, uint32_t n_items, int32_t n_cdf,
                  const mc_source_t *source, const mc_geometry_t *geometry, const mc_detector_t *detector,
                  const mc_run_t *run, const mc_tally_t *tally, double photon_scale, WalkArgs &a,
                  std::vector<BatchInst> &sched, uint64_t &total)
{
    if (!items || !source || !geometry || !detector || !run || !tally) return fail(MC_EINVAL, "%s: null argument", fn);
    if (n_items < 1 || n_items > MC_MAX_BATCH) return fail(MC_EINVAL, "%s: n_items must be in 1..%d", fn, MC_MAX_BATCH);
    if (n_cdf < 2 || n_cdf > MC_MAX_N_CDF) return fail(MC_EINVAL, "%s: n_cdf %d outside 2..%d", fn, n_cdf, MC_MAX_N_CDF);
    const mc_geometry_t &geo = *geometry;
    const mc_detector_t &det = *detector;
    const mc_run_t &rn = *run;
    const mc_tally_t &t = *tally;
    if (int rc = check_geometry(fn, geo)) return rc;
    if (int rc = check_setup(fn, *source, geo, det, rn, t)) return rc;
    if (det.flags & (MC_RECORD | MC_MOMENTS | MC_MOMENTS_PIXEL2))
        return fail(MC_EUNSUPPORTED, "%s: MC_RECORD and MC_MOMENTS are not available for batched launches", fn);
    if (det.flags & ~(MC_ACCUMULATE | MC_SIGMA | MC_FIX64 | MC_EXIT_LOG))
        return fail(MC_EINVAL, "%s: unknown detector flags 0x%x", fn, det.flags);
    const uint64_t n_pix = (uint64_t)det.side_nx * det.side_ny + (uint64_t)det.trans_nx * det.trans_ny;
    if (n_pix * n_items >= 0xFFFFFFFFull)
        return fail(MC_EINVAL, "%s: images exceed 2^32 - 2 pixels over all items", fn);
    if (!t.workspace || ((uintptr_t)t.workspace & 7) || t.workspace_bytes < batch_workspace_words(det, n_items) * 8)
        return fail(MC_EINVAL, "%s: workspace needs %llu bytes, 8-byte aligned", fn,
                    (unsigned long long)(batch_workspace_words(det, n_items) * 8));
    sched.clear();
    total = 0;
    std::vector<double> cost;
    for (uint32_t i = 0; i < n_items; ++i) {
        const mc_batch_item_t &it = items[i];
        if (!(it.tau >= 0.0) || !std::isfinite(it.tau)) return fail(MC_EINVAL, "%s: item %u: tau must be >= 0", fn, i);
        if (!(it.albedo >= 0.0 && it.albedo <= 1.0))
            return fail(MC_EINVAL, "%s: item %u: albedo must be in [0, 1]", fn, i);
        if (!it.inv_cdf) return fail(MC_EINVAL, "%s: item %u: inv_cdf is required", fn, i);
        uint64_t n = it.n_photons;
        if (photon_scale < 1.0 && n > 0) n = std::max<uint64_t>(1, (uint64_t)std::llround((double)n * photon_scale));
        if (int rc = check_overflow(fn, n, det, rn)) return rc;
        BatchInst b{};
        fill_medium(b.neg_ln2_over_mu, b.albedo, b.absorb, it.tau / geo.size_mm[2], it.albedo);
        b.inv_cdf = it.inv_cdf;
        b.n_photons = n;
        b.counter = it.instance;
        b.slot = i;
        sched.push_back(b);
        cost.push_back((double)n * (1.0 + it.tau));
        total += n;
    }
    std::vector<uint32_t> order(n_items);
    for (uint32_t i = 0; i < n_items; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) { return cost[x] > cost[y]; });
    std::vector<BatchInst> sorted;
    for (uint32_t i : order) sorted.push_back(sched[i]);
    sched.swap(sorted);

    a = WalkArgs{};
    fill_common(a, *source, geo, det, rn);
    a.phase = MC_PHASE_MIE;
    a.n_cdf = n_cdf;
    a.inv_cdf = nullptr;
    a.instance = 0;
    a.n_photons = 0;
    a.photon_offset = 0;
    a.record_stride = 1;
    return MC_OK;
}

}  // namespace
}  // namespace mcmie

namespace mcmie {
namespace {

// The walk of mc_simulate.  With `scratch_ws` set, the caller's workspace is
// ignored: the images are tallied in one fixed-point copy held in that device
// array (noalloc callers) instead of in per-XCD copies in the workspace.
int simulate(const char *fn, const mc_medium_t *medium, const mc_source_t *source, const mc_geometry_t *geometry,
             const mc_detector_t *detector, const mc_run_t *run, const mc_tally_t *tally, void *scratch_ws,
             void *stream)
{
    clear_error();
    if (!medium || !source || !geometry || !detector || !run || !tally)
        return fail(MC_EINVAL, "%s: null argument", fn);
    const mc_medium_t m = *medium;
    const mc_geometry_t geo = *geometry;
    const mc_detector_t det = *detector;
    const mc_run_t rn = *run;
    mc_tally_t t = *tally;

    // ---- parameter checks (Sec. 3.1.1) ----
    if (int rc = check_geometry(fn, geo)) return rc;
    MediumCoef coef{};
    if (int rc = medium_coefficients(fn, m, geo.size_mm[2], coef)) return rc;
    if (m.phase == MC_PHASE_MIE) {
        if (m.n_cdf < 2 || m.n_cdf > MC_MAX_N_CDF)
            return fail(MC_EINVAL, "%s: n_cdf %d outside 2..%d", fn, m.n_cdf, MC_MAX_N_CDF);
        if (!m.inv_cdf) return fail(MC_EINVAL, "%s: inv_cdf is required for MC_PHASE_MIE", fn);
    } else if (m.phase == MC_PHASE_HG) {
        if (!(m.g > -1.0 && m.g < 1.0)) return fail(MC_EINVAL, "%s: HG g must be in (-1, 1)", fn);
    } else {
        return fail(MC_EINVAL, "%s: unknown phase %d", fn, m.phase);
    }
    if (scratch_ws) {
        // The library's array stands in for the workspace (checked by check_setup).
        t.workspace = scratch_ws;
        t.workspace_bytes = kNoAllocWords * 8;
    }
    if (int rc = check_setup(fn, *source, geo, det, rn, t)) return rc;
    if ((det.flags & MC_RECORD) && (rn.record_stride < 1 || (t.rec_rows > 0 && (!t.rec_i || !t.rec_f))))
        return fail(MC_EINVAL, "%s: MC_RECORD needs record_stride >= 1 and, for rec_rows > 0, rec_i and rec_f", fn);
    if (rn.photon_offset > UINT64_MAX - rn.n_photons) return fail(MC_EINVAL, "%s: photon ids overflow", fn);
    if (det.flags & ~(MC_ACCUMULATE | MC_SIGMA | MC_RECORD | MC_FIX64 | MC_MOMENTS | MC_MOMENTS_PIXEL2 | MC_EXIT_LOG))
        return fail(MC_EINVAL, "%s: unknown detector flags 0x%x", fn, det.flags);
    if ((det.flags & MC_EXIT_LOG) && (det.flags & MC_RECORD))
        return fail(MC_EINVAL, "%s: MC_EXIT_LOG does not combine with MC_RECORD", fn);
    if ((det.flags & MC_MOMENTS) && (!t.side_wk || !t.side_wl))
        return fail(MC_EINVAL, "%s: MC_MOMENTS needs side_wk and side_wl", fn);
    if ((det.flags & MC_MOMENTS_PIXEL2) && (!(det.flags & MC_MOMENTS) || !t.side_w2k || !t.side_w2l))
        return fail(MC_EINVAL, "%s: MC_MOMENTS_PIXEL2 needs MC_MOMENTS, side_w2k and side_w2l", fn);
    const uint64_t copies = scratch_ws ? 1 : kCopies;
    if (!t.workspace || ((uintptr_t)t.workspace & 7) || t.workspace_bytes < workspace_words(det, 1, copies) * 8) {
        if (scratch_ws)
            return fail(MC_EINVAL, "%s: the images need %llu bytes of scratch, more than the library's %llu "
                        "(at most 2^21 pixels over both images, 2^20 with MC_SIGMA)", fn,
                        (unsigned long long)(workspace_words(det, 1, copies) * 8),
                        (unsigned long long)(kNoAllocWords * 8));
        return fail(MC_EINVAL, "%s: workspace needs %llu bytes, 8-byte aligned", fn,
                    (unsigned long long)(workspace_words(det) * 8));
    }
    if (int rc = check_overflow(fn, rn.n_photons, det, rn)) return rc;
    const uint64_t n_pix = (uint64_t)det.side_nx * det.side_ny + (uint64_t)det.trans_nx * det.trans_ny;
    if (n_pix >= 0xFFFFFFFFull) return fail(MC_EINVAL, "%s: images exceed 2^32 - 2 pixels in total", fn);

    WalkArgs a{};
    fill_common(a, *source, geo, det, rn);
    fill_medium(a.neg_ln2_over_mu, a.albedo, a.absorb, coef.mu_ext, coef.albedo);
    a.copy_mask = (uint32_t)(copies - 1);
    a.phase = m.phase;
    a.n_cdf = m.phase == MC_PHASE_MIE ? m.n_cdf : 0;
    a.inv_cdf = m.inv_cdf;
    a.hg_a = (float)(1.0 + m.g);
    a.hg_b = (float)(2.0 * m.g);
    a.hg_c = (float)(1.0 - m.g * m.g);
    a.hg_d = (float)(1.0 - m.g);
    a.instance = rn.instance;
    a.n_photons = rn.n_photons;
    a.photon_offset = rn.photon_offset;
    a.rec_i = t.rec_i; a.rec_f = t.rec_f;
    a.side_wk = (det.flags & MC_MOMENTS) ? t.side_wk : nullptr;
    a.side_wl = (det.flags & MC_MOMENTS) ? t.side_wl : nullptr;
    a.side_w2k = (det.flags & MC_MOMENTS_PIXEL2) ? t.side_w2k : nullptr;
    a.side_w2l = (det.flags & MC_MOMENTS_PIXEL2) ? t.side_w2l : nullptr;
    a.rec_rows = (det.flags & MC_RECORD) ? t.rec_rows : 0;
    a.record_stride = rn.record_stride >= 1 ? rn.record_stride : 1;
    return launch_walk(a, det, rn, t, m.phase, 1, rn.n_photons, nullptr, (hipStream_t)stream);
}

// Address of this device's copy of `scratch`, looked up once per device
// with the device current (the array's name is a host-side stand-in).
std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {nullptr};

int device_scratch(const char *fn, void **out)
{
    int dev = 0;
    MC_HIP_CHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(MC_EDEVICE, "%s: device index %d out of range", fn, dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(MC_EDEVICE, "%s: hipGetSymbolAddress(scratch) failed: %s", fn, hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MC_OK;
}

}  // namespace
}  // namespace mcmie

extern "C" int mc_simulate(const mc_medium_t *medium, const mc_source_t *source, const mc_geometry_t *geometry,
                           const mc_detector_t *detector, const mc_run_t *run, const mc_tally_t *tally,
                           void *stream)
{
    return mcmie::simulate("mc_simulate", medium, source, geometry, detector, run, tally, nullptr, stream);
}

extern "C" int mc_simulate_noalloc(const mc_medium_t *medium, const mc_source_t *source,
                                   const mc_geometry_t *geometry, const mc_detector_t *detector, const mc_run_t *run,
                                   const mc_tally_t *tally, void *stream)
{
    using namespace mcmie;
    const char *fn = "mc_simulate_noalloc";
    clear_error();
    if (!detector || !tally) return fail(MC_EINVAL, "%s: null argument", fn);
    if (detector->flags & MC_EXIT_LOG)
        return fail(MC_EINVAL, "%s: MC_EXIT_LOG needs a caller workspace (use mc_simulate)", fn);
    if (!dims_ok(*detector)) return fail(MC_EINVAL, "%s: image dimensions must be >= 1", fn);
    if (workspace_words(*detector, 1, 1) > kNoAllocWords)
        return fail(MC_EINVAL, "%s: the images need %llu bytes of scratch, more than the library's %llu "
                    "(at most 2^21 pixels over both images, 2^20 with MC_SIGMA)", fn,
                    (unsigned long long)(workspace_words(*detector, 1, 1) * 8),
                    (unsigned long long)(kNoAllocWords * 8));
    void *ws = nullptr;
    if (int rc = device_scratch(fn, &ws)) return rc;
    return simulate(fn, medium, source, geometry, detector, run, tally, ws, stream);
}

extern "C" int mc_medium_coefficients(const mc_medium_t *medium, const mc_geometry_t *geometry, double out[4])
{
    using namespace mcmie;
    clear_error();
    if (!medium || !geometry || !out) return fail(MC_EINVAL, "mc_medium_coefficients: null argument");
    if (int rc = check_geometry("mc_medium_coefficients", *geometry)) return rc;
    MediumCoef c{};
    if (int rc = medium_coefficients("mc_medium_coefficients", *medium, geometry->size_mm[2], c)) return rc;
    out[0] = c.mu_sca;
    out[1] = c.mu_abs;
    out[2] = c.mu_ext;
    out[3] = c.albedo;
    return MC_OK;
}

extern "C" uint64_t mc_workspace_bytes(const mc_detector_t *detector)
{
    if (!detector || !mcmie::dims_ok(*detector)) return 0;
    return mcmie::workspace_words(*detector) * 8;
}

extern "C" uint64_t mc_workspace_bytes_log(const mc_detector_t *detector, uint64_t n_photons)
{
    if (!detector || !mcmie::dims_ok(*detector) || !(detector->flags & MC_EXIT_LOG)) return 0;
    using namespace mcmie;
    const mc_detector_t &d = *detector;
    const uint64_t n_keys = (uint64_t)d.side_nx * d.side_ny + (uint64_t)d.trans_nx * d.trans_ny;
    // The table-in-LDS shape: at most as many ranges as the HG walk takes.
    const uint64_t regions = ((uint64_t)1 << log_shape(n_keys, true).rbits) * kLogSizingBlocks;
    return workspace_words(d) * 8 + log_bytes_for(n_photons, regions);
}

extern "C" uint64_t mc_workspace_bytes_batch(const mc_detector_t *detector, uint32_t n_items)
{
    if (!detector || !mcmie::dims_ok(*detector) || n_items < 1 || n_items > MC_MAX_BATCH) return 0;
    return mcmie::batch_workspace_words(*detector, n_items) * 8;
}

extern "C" uint64_t mc_workspace_bytes_batch_log(const mc_detector_t *detector, uint32_t n_items,
                                                 uint64_t total_photons)
{
    using namespace mcmie;
    if (!detector || !dims_ok(*detector) || !(detector->flags & MC_EXIT_LOG) || n_items < 1 ||
        n_items > MC_MAX_BATCH)
        return 0;
    const mc_detector_t &d = *detector;
    const uint64_t n_keys = ((uint64_t)d.side_nx * d.side_ny + (uint64_t)d.trans_nx * d.trans_ny) * n_items;
    const uint64_t regions = ((uint64_t)1 << log_shape(n_keys, false).rbits) * kLogSizingBlocks;
    return batch_workspace_words(d, n_items) * 8 + log_bytes_for(total_photons, regions);
}

extern "C" int mc_simulate_batch(const mc_batch_item_t *items, uint32_t n_items, int32_t n_cdf,
                                 const mc_source_t *source, const mc_geometry_t *geometry,
                                 const mc_detector_t *detector, const mc_run_t *run, const mc_tally_t *tally,
                                 void *stream)
{
    using namespace mcmie;
    clear_error();
    WalkArgs a{};
    std::vector<BatchInst> sched;
    uint64_t total = 0;
    if (int rc = prepare_batch("mc_simulate_batch", items, n_items, n_cdf, source, geometry, detector, run, tally,
                               1.0, a, sched, total))
        return rc;
    return launch_walk(a, *detector, *run, *tally, MC_PHASE_MIE, n_items, total, &sched, (hipStream_t)stream);
}

extern "C" int mc_autotune_batch(const mc_batch_item_t *items, uint32_t n_items, int32_t n_cdf,
                                 const mc_source_t *source, const mc_geometry_t *geometry,
                                 const mc_detector_t *detector, const mc_run_t *run, const mc_tally_t *tally,
                                 double sample_fraction, int32_t *block_size, uint32_t *chunk, double *best_ms,
                                 double *candidate_ms, void *stream)
{
    using namespace mcmie;
    clear_error();
    if (!block_size || !chunk || !best_ms) return fail(MC_EINVAL, "mc_autotune_batch: null output");
    if (!(sample_fraction > 0.0 && sample_fraction <= 1.0))
        return fail(MC_EINVAL, "mc_autotune_batch: sample_fraction must be in (0, 1]");
    WalkArgs a0{};
    std::vector<BatchInst> sched;
    uint64_t total = 0;
    if (int rc = prepare_batch("mc_autotune_batch", items, n_items, n_cdf, source, geometry, detector, run, tally,
                               sample_fraction, a0, sched, total))
        return rc;
    static const int32_t blocks[3] = {256, 512, 1024};
    static const uint32_t chunks[5] = {256, 512, 1024, 2048, 4096};
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    MC_HIP_CHECK(hipEventCreate(&e0));
    MC_HIP_CHECK(hipEventCreate(&e1));
    double best = INFINITY;
    int32_t bb = 0;
    uint32_t bc = 0;
    int rc = MC_OK;
    for (int i = 0; i < 3 && rc == MC_OK; ++i) {
        for (int j = 0; j < 5 && rc == MC_OK; ++j) {
            mc_run_t rn = *run;
            rn.block_size = blocks[i];
            rn.chunk = chunks[j];
            rn.grid_blocks = 0;
            float ms = 0.f;
            for (int rep = 0; rep < 2 && rc == MC_OK; ++rep) {
                WalkArgs a = a0;
                if (rep == 1 && hipEventRecord(e0, st) != hipSuccess) rc = fail(MC_EDEVICE, "hipEventRecord failed");
                if (rc == MC_OK) rc = launch_walk(a, *detector, rn, *tally, MC_PHASE_MIE, n_items, total, &sched, st);
                if (rc == MC_OK && rep == 1) {
                    if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                        rc = fail(MC_EDEVICE, "mc_autotune_batch: event timing failed");
                }
            }
            if (rc != MC_OK) break;
            if (candidate_ms) candidate_ms[i * 5 + j] = ms;
            if (ms < best) {
                best = ms;
                bb = blocks[i];
                bc = chunks[j];
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != MC_OK) return rc;
    *block_size = bb;
    *chunk = bc;
    *best_ms = best;
    return MC_OK;
}

extern "C" int mc_grad(const mc_medium_t *medium, const mc_geometry_t *geometry, const mc_detector_t *detector,
                       const mc_tally_t *tally, const double *dloss_dside, const double *d2loss_dside2,
                       double d2loss_uniform, double out_grad[3], void *stream)
{
    using namespace mcmie;
    clear_error();
    if (!medium || !geometry || !detector || !tally || !dloss_dside || !out_grad)
        return fail(MC_EINVAL, "mc_grad: null argument");
    const mc_medium_t m = *medium;
    const mc_geometry_t geo = *geometry;
    const mc_detector_t det = *detector;
    const mc_tally_t t = *tally;
    if (!finite_pos(geo.size_mm[2])) return fail(MC_EINVAL, "mc_grad: size_mm[2] must be > 0");
    MediumCoef coef{};
    if (int rc = medium_coefficients("mc_grad", m, geo.size_mm[2], coef)) return rc;
    if (!(coef.mu_sca > 0.0)) return fail(MC_EINVAL, "mc_grad: needs mu_sca > 0");
    if (det.side_nx < 1 || det.side_ny < 1) return fail(MC_EINVAL, "mc_grad: side image dimensions must be >= 1");
    if (!t.side_wk || !t.side_wl || !t.scalars)
        return fail(MC_EINVAL, "mc_grad: the tally has no moment images (MC_MOMENTS)");
    if (d2loss_dside2 && (!t.side_w2k || !t.side_w2l))
        return fail(MC_EINVAL, "mc_grad: a per-pixel second derivative needs the MC_MOMENTS_PIXEL2 images");
    if (!std::isfinite(d2loss_uniform))
        return fail(MC_EINVAL, "mc_grad: d2loss_uniform must be finite");
    if (d2loss_dside2 && d2loss_uniform != 0.0)
        return fail(MC_EINVAL, "mc_grad: give either d2loss_dside2 or d2loss_uniform, not both");
    if (!t.workspace || ((uintptr_t)t.workspace & 7) || t.workspace_bytes < (kWsScalarWords + 4) * 8)
        return fail(MC_EINVAL, "mc_grad: workspace of at least %llu bytes required",
                    (unsigned long long)((kWsScalarWords + 4) * 8));
    const double mu_s = coef.mu_sca;
    hipStream_t st = (hipStream_t)stream;
    double *dots = (double *)t.workspace + 24;    // scalar words 24..27
    const uint64_t n = (uint64_t)det.side_nx * det.side_ny;
    // The blocks' partials go after the scalar words, where mc_simulate keeps
    // its image copies (consumed by then): one block per 8192 pixels, at most
    // 256, and no more than the workspace holds.
    double *part = (double *)t.workspace + kWsScalarWords;
    const uint64_t room = t.workspace_bytes / 8 - kWsScalarWords;
    const uint32_t n_blocks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>({256, (n + 8191) / 8192, room / 4}));
    hipLaunchKernelGGL(grad_partial, dim3(n_blocks), dim3(1024), 0, st, dloss_dside, d2loss_dside2,
                       (const double *)t.side_wk, (const double *)t.side_wl, (const double *)t.side_w2k,
                       (const double *)t.side_w2l, n, part);
    hipLaunchKernelGGL(grad_final, dim3(1), dim3(64), 0, st, (const double *)part, n_blocks,
                       d2loss_dside2 != nullptr, d2loss_uniform, (const double *)t.scalars, dots);
    MC_HIP_CHECK(hipGetLastError());
    double d[4];
    MC_HIP_CHECK(hipMemcpyAsync(d, dots, sizeof d, hipMemcpyDeviceToHost, st));
    MC_HIP_CHECK(hipStreamSynchronize(st));
    // D = M_k / mu_s - M_L (mu_sca), -M_L (mu_abs); Q likewise from the w^2 moments.
    const double gq_s = d[2] / mu_s - d[3], gq_a = -d[3];
    out_grad[0] = (d[0] / mu_s - d[1]) - gq_s;
    out_grad[1] = -d[1] - gq_a;
    const bool have_sigma = m.sigma_sca_mm2 != 0.0 || m.sigma_abs_mm2 != 0.0;
    out_grad[2] = have_sigma ? m.sigma_sca_mm2 * out_grad[0] + m.sigma_abs_mm2 * out_grad[1] : NAN;
    return MC_OK;
}

extern "C" int mc_philox_blocks(uint64_t seed, uint32_t instance, const uint64_t *ids, uint64_t n_ids,
                                uint32_t step0, uint32_t n_steps, uint32_t *out, void *stream)
{
    using namespace mcmie;
    clear_error();
    if (n_ids == 0 || n_steps == 0) return MC_OK;
    if (!ids || !out) return fail(MC_EINVAL, "mc_philox_blocks: null buffer");
    if ((uint64_t)step0 + n_steps > (1ull << 32)) return fail(MC_EINVAL, "mc_philox_blocks: step range overflows");
    const uint64_t total = n_ids * (uint64_t)n_steps;
    if (total / n_steps != n_ids || total > (1ull << 40)) return fail(MC_EINVAL, "mc_philox_blocks: too many blocks");
    const uint64_t grid = (total + 255) / 256;
    hipLaunchKernelGGL(philox_blocks_kernel, dim3((uint32_t)grid), dim3(256), 0, (hipStream_t)stream,
                       (uint32_t)seed, (uint32_t)(seed >> 32), instance, ids, n_ids, step0, n_steps, out);
    MC_HIP_CHECK(hipGetLastError());
    return MC_OK;
}
