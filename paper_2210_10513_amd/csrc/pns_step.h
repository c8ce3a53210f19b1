// Step kernel of the Partial Neighbor Search sampler for gfx950 (MI355X).
// Included by one translation unit per matrix element type.
//
// One workgroup runs one chain.  The chain's N bits are spread over the
// workgroup in groups of four consecutive bits per lane:
//     field f = (g * BLOCK + tid) * 4 + v,   g < G, v < 4,
// so group g covers the contiguous bit range [g*BLOCK*4, (g+1)*BLOCK*4) and a
// row of the coefficient matrix is read with one 8- or 16-byte load per lane
// and group, fully coalesced.  Fields, bits and the diagonal stay in
// registers for the whole launch; only the row of the flipped bit is read
// from memory each step.
//
// Per step (loop body of Alg 2 / Alg 3 / Alg 6):
//   subset  : all bits (RF), systematic window (Unbiased-sys), random n-subset
//             (Basic every step, Unbiased-rand per block) drawn in LDS;
//   weights : w_j = min(1, exp(-beta dE_j)), dE_j = (1-2x_j)(Q_jj + s h_j);
//             for integer Q, dE is an integer and exp(-beta dE) is read from
//             two LDS tables, exp(-beta*64a) * exp(-beta*b) for dE = 64a + b;
//   reduce  : sums of four consecutive bits -> wave inclusive scans (DPP) ->
//             one LDS exchange -> every wave scans the 256-bit segment sums
//             the same way, so the rounding of every prefix is fixed by the
//             bit order alone, whatever the tile shape;
//   p, M    : p = S / n, M = 1 + floor(log U1 / log1p(-p)) in FP64;
//   budget  : Unbiased: stay with M = L when M > L, else L -= M (Alg 6);
//   select  : inverse CDF (appendix "How to Sample Proportionally") over the
//             subset in increasing bit order, resolved segment -> lane -> bit,
//             published through LDS;
//   update  : flip, E += dE_c, h_j +-= A[c][j] from one coalesced row read,
//             overlapped with the next step's random numbers.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "pns_internal.h"

namespace pns {
namespace step {

constexpr uint32_t kStreamStep = 0u;
constexpr uint32_t kStreamSubset = 0x40000000u;
constexpr int kModeRF = 0, kModeBasic = 1, kModeSys = 2, kModeRand = 3;
// Optimization RF / PNS (Alg 9, 10): the jump chain at beta / T with no
// multiplicity; a fresh random subset each step when n < N (as in Alg 3).
constexpr int kModeOpt = 4;

// Kernel flavours: how the subset of a step is formed.
constexpr int FLAV_ALL = 0;     // every bit (RF, and Basic with n = N)
constexpr int FLAV_WINDOW = 1;  // systematic window (Unbiased-sys, Unbiased-rand with n = N)
constexpr int FLAV_DRAWN = 2;   // random n-subset drawn in LDS (Basic, Unbiased-rand)
constexpr int FLAV_WINDOW_C = 3; // systematic window touching at most one 4-bit group in any
                                 // wave (checked on the host): one scan per wave, four weights
                                 // per lane, diagonal read from LDS
constexpr int FLAV_WINDOW_C2 = 4; // the same with at most two 4-bit groups in any wave (windows
                                  // that span two groups or wrap from the last group to bit 0):
                                  // two scans in the waves that hold both, eight weights per lane

// Weight tables for integer energy differences: dE = 64 a + b, b < 64, a < 1024.
constexpr int kTabLo = 64;
constexpr int kTabHi = 1024;
constexpr int64_t kTabMax = (int64_t)kTabLo * kTabHi;

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// multiplications whose halves are mixed with the other counter words and the
// key; the key advances by the two Weyl increments between rounds.
struct Words {
    uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ Words philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t key)
{
    uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// Step uniforms: U1 in (0, 1] from words 0, 1 (kept as log U1) and U2 in
// [0, 1) from words 2, 3, each from the top 53 bits of 64.
struct StepUniforms {
    double logU1;
    double U2;
};

// Uniforms of 64 consecutive steps kb .. kb+63, one step per lane: lane j
// holds step kb + j.  A step then reads its pair with two lane reads, so the
// counter-based draws and the logarithm cost one pass per 64 steps.
__device__ __forceinline__ void batch_uniforms(uint32_t cid, int64_t kb, uint64_t seed, int lane, bool want_log,
                                               double* logU1, double* U2)
{
    const int64_t k = kb + lane;
    const Words o = philox(cid, (uint32_t)k, (uint32_t)((uint64_t)k >> 32), kStreamStep, seed);
    const double u1 = (double)(((((uint64_t)o.w0 << 32) | o.w1) >> 11) + 1u) * 0x1p-53;
    *U2 = (double)((((uint64_t)o.w2 << 32) | o.w3) >> 11) * 0x1p-53;
    *logU1 = want_log ? log(u1) : 0.0;
}

// ---- wave64 primitives (DPP) ----
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWMASK, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWMASK, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Inclusive prefix sum over the 64 lanes: within rows of 16 by shifts of 1, 2,
// 4, 8, then the row totals by the broadcasts of lanes 15 and 31.  The order
// of additions for lane l depends only on l.
__device__ __forceinline__ double wave_scan(double v)
{
    v += dpp_f64<0x111, 0xF>(v);  // row_shr:1
    v += dpp_f64<0x112, 0xF>(v);  // row_shr:2
    v += dpp_f64<0x114, 0xF>(v);  // row_shr:4
    v += dpp_f64<0x118, 0xF>(v);  // row_shr:8
    v += dpp_f64<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_f64<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// The same inclusive prefix sum restricted to lanes 0 .. NS-1 (the other
// lanes' values are not used): the shifts and broadcasts that cannot reach
// those lanes from below are skipped, which leaves their sums unchanged.
template <int NS>
__device__ __forceinline__ double small_scan(double v)
{
    v += dpp_f64<0x111, 0xF>(v);
    if constexpr (NS > 2) v += dpp_f64<0x112, 0xF>(v);
    if constexpr (NS > 4) v += dpp_f64<0x114, 0xF>(v);
    if constexpr (NS > 8) v += dpp_f64<0x118, 0xF>(v);
    if constexpr (NS > 16) v += dpp_f64<0x142, 0xA>(v);
    if constexpr (NS > 32) v += dpp_f64<0x143, 0xC>(v);
    return v;
}

__device__ __forceinline__ double read_lane(double v, int lane)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = fmax(v, __shfl_xor(v, d, 64));
    return v;
}

__device__ __forceinline__ uint32_t wave_or(uint32_t v)
{
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v |= (uint32_t)__shfl_xor((int)v, d, 64);
    return v;
}

__device__ __forceinline__ int nth_set_bit(uint64_t m, int r)
{
    for (int i = 0; i < r; ++i) m &= m - 1;
    return __builtin_ctzll(m);
}

// ---- four consecutive elements ----
template <typename T>
struct Four {
    T v[4];
};

// Raw loads of four consecutive coefficients and their widening, split so
// that the wait for the load can sit at the first use of the values.
__device__ __forceinline__ uint2 load_raw4(const int16_t* p) { return *reinterpret_cast<const uint2*>(p); }
__device__ __forceinline__ int4 load_raw4(const int32_t* p) { return *reinterpret_cast<const int4*>(p); }
__device__ __forceinline__ float4 load_raw4(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ __forceinline__ Four<int32_t> widen4(uint2 r)
{
    Four<int32_t> o;
    o.v[0] = (int32_t)(int16_t)(r.x & 0xFFFFu);
    o.v[1] = (int32_t)(int16_t)(r.x >> 16);
    o.v[2] = (int32_t)(int16_t)(r.y & 0xFFFFu);
    o.v[3] = (int32_t)(int16_t)(r.y >> 16);
    return o;
}
__device__ __forceinline__ Four<int32_t> widen4(int4 r) { return {{r.x, r.y, r.z, r.w}}; }
__device__ __forceinline__ Four<float> widen4(float4 r) { return {{r.x, r.y, r.z, r.w}}; }

template <typename T>
__device__ __forceinline__ Four<T> load4(const T* p)
{
    Four<T> o;
#pragma unroll
    for (int v = 0; v < 4; ++v) o.v[v] = p[v];
    return o;
}
template <>
__device__ __forceinline__ Four<int32_t> load4(const int32_t* p)
{
    const int4 r = *reinterpret_cast<const int4*>(p);
    return {{r.x, r.y, r.z, r.w}};
}
template <>
__device__ __forceinline__ Four<float> load4(const float* p)
{
    const float4 r = *reinterpret_cast<const float4*>(p);
    return {{r.x, r.y, r.z, r.w}};
}
template <typename T>
__device__ __forceinline__ void store4(T* p, const T* v)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) p[i] = v[i];
}
template <>
__device__ __forceinline__ void store4(int32_t* p, const int32_t* v)
{
    *reinterpret_cast<int4*>(p) = make_int4(v[0], v[1], v[2], v[3]);
}

template <typename QT>
struct Wide {
    using T = int32_t;
};
template <>
struct Wide<float> {
    using T = float;
};

// Energy difference of flipping a bit with value xbit: integer or FP64.
// (int32 fields: |Q_jj| + s |h_j| < 2^31 is checked on creation.)
template <typename HT>
__device__ __forceinline__ HT delta_int(int32_t d, HT h, int s, uint32_t xbit)
{
    const HT e = (HT)d + (s == 2 ? (HT)(h + h) : h);
    return xbit ? -e : e;
}
__device__ __forceinline__ double delta_f64(float d, double h, int s, uint32_t xbit)
{
    const double e = (double)d + (double)s * h;
    return xbit ? -e : e;
}

// q = log U1 / log1p(-p) for 0 < p < 1: M = 1 + floor(q) (Thm 3 (2): the
// failures before the first success of a Bernoulli(p) sequence), and a
// budgeted record stays when q >= L (Alg 6).  The FP64 log1p and division
// are about 1400 cycles of one lane, so a cheap estimate decides first:
// log1p(-p) from its series (p <= 2^-6, relative error < 1.3e-8) or from the
// float logarithm of 1 - p (relative error < 5e-6 there), divided in FP64.
// When the interval q_est (1 -+ d) -- d = 1e-7 after the series, 1e-4 after
// the float logarithm, at least 7 times the estimate's error -- holds neither
// L nor an integer, the estimate has the same floor and the same order
// against L as the exact quotient and is returned; otherwise the exact
// quotient is.  L < 0: no budget.
__device__ __noinline__ double exact_quotient(double logU1, double p) { return logU1 / log1p(-p); }

__device__ __forceinline__ double geometric_quotient(double logU1, double p, double L)
{
    double l1p = 0.0, d = 1e-7;
    bool est = true;
    if (p <= 0x1p-6) {
        l1p = -p * (1.0 + p * (0.5 + p * (1.0 / 3.0 + p * 0.25)));
    } else {
        const double x = 1.0 - p;
        est = x >= 0x1p-100;
        l1p = est ? (double)logf((float)x) : -1.0;
        d = 1e-4;
    }
    if (est) {
        const double qe = logU1 / l1p;
        const double lo = qe * (1.0 - d), hi = qe * (1.0 + d);
        if (qe < 0x1p52 && floor(lo) == floor(hi) && !(lo < L && hi >= L)) return qe;
    }
    // (out of line: the logarithm's constants would otherwise be kept in
    // registers across the step loop)
    return exact_quotient(logU1, p);
}

// Mean multiplicity of a record given its state, subset and remaining budget
// L (Thm 3 (2): M = 1 + G, G ~ Geometric(p) counting failures, cut at L when
// the record is budgeted): E[min(1 + G, L)] = (1 - (1 - p)^L) / p, and 1 / p
// with no budget.  These are the Rao-Blackwell weights of the ratio estimator
// of Thm 3 (5).  p <= 0 (every weight underflowed) gives L, or +inf unbudgeted.
__device__ __noinline__ double expected_multiplicity(double p, int64_t L, bool budgeted)
{
    if (p >= 1.0) return 1.0;
    if (p <= 0.0) return budgeted ? (double)L : INFINITY;
    if (!budgeted) return 1.0 / p;
    return -expm1((double)L * log1p(-p)) / p;
}

// Uniformly random n-subset of {0..N-1}: the first n distinct values of the
// i.i.d. candidate stream, candidate s drawn from Philox stream
// 0x40000000 | (s/2) of step `k` (words 0,1 for even s, 2,3 for odd s) and
// mapped to floor(u64 * N / 2^64).  Positions are processed BLOCK at a time;
// own[f] keeps the first position where f appeared (LDS atomicMin), so f is in
// the subset iff own[f] <= pos_n, the position of the n-th first occurrence.
template <int BLOCK, int G>
__device__ uint32_t draw_subset(uint32_t* own, uint64_t* masks, int tid, int64_t pitch, int32_t N, int32_t n,
                                uint64_t seed, uint32_t cid, int64_t k)
{
    constexpr int W = BLOCK / 64;
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t fb = ((int64_t)g * BLOCK + tid) * 4;
        if (fb < pitch) {
#pragma unroll
            for (int v = 0; v < 4; ++v) own[fb + v] = 0xFFFFFFFFu;
        }
    }
    __syncthreads();
    uint32_t base = 0;
    int32_t have = 0;
    for (;;) {
        const uint32_t pos = base + (uint32_t)tid;
        const Words o = philox(cid, (uint32_t)k, (uint32_t)((uint64_t)k >> 32), kStreamSubset | (pos >> 1), seed);
        const uint32_t hi = (pos & 1u) ? o.w2 : o.w0;
        const uint32_t lo = (pos & 1u) ? o.w3 : o.w1;
        const uint64_t u = ((uint64_t)hi << 32) | (uint64_t)lo;
        const uint32_t cand = (uint32_t)__umul64hi(u, (uint64_t)(uint32_t)N);
        atomicMin(&own[cand], pos);
        __syncthreads();
        const bool first = own[cand] == pos;
        const uint64_t bal = __ballot(first);
        if (lane == 0) masks[wave] = bal;
        __syncthreads();
        const int32_t need = n - have;
        int32_t tot = 0;
        uint32_t pos_n = 0xFFFFFFFFu;
        for (int w = 0; w < W; ++w) {
            const uint64_t m = masks[w];
            const int c = __popcll(m);
            if (pos_n == 0xFFFFFFFFu && tot + c >= need) pos_n = base + (uint32_t)(w * 64 + nth_set_bit(m, need - tot - 1));
            tot += c;
        }
        __syncthreads();  // masks are rewritten by the next round or draw
        if (pos_n != 0xFFFFFFFFu) return pos_n;
        have += tot;
        base += BLOCK;
        // n < N distinct values appear within ~N ln N draws; this bound is
        // never reached by a correct stream and only keeps the loop finite.
        if (base >= (1u << 24)) return 0xFFFFFFFEu;
    }
}

// Words of the leader lane's LDS state.
constexpr int kLsE = 0, kLsL = 1, kLsLastA = 2, kLsLastM = 3, kLsLastE = 4, kLsSteps = 5, kLsFlips = 6,
              kLsStays = 7, kLsSat = 8, kLsBad = 9, kLsSumM = 10, kLsBest = 11, kLeadWords = 12;

// Occupancy asked of the compiler (waves per SIMD): compact-window kernels
// of 512 lanes target two co-resident chains per compute unit (128 VGPRs);
// compact and two-group windows on 256 x 8 tiles three chains of four waves
// (168 VGPRs), on 256 x 16 tiles (64 fields per lane) two; the flavours that
// weigh every group of a lane (all bits, general window, drawn subset) keep
// two waves on the wide tiles (they are not what those tiles are for); other
// 1024-lane kernels keep the register budget of one chain per unit.
template <int BLOCK, int G, int FLAV>
constexpr int min_waves_per_eu()
{
    constexpr bool win = FLAV == FLAV_WINDOW_C || FLAV == FLAV_WINDOW_C2;
    if (BLOCK == 256 && G >= 8) return (win && G == 8) ? 3 : 2;
    return ((win && BLOCK == 512) || (G == 1 && BLOCK <= 512)) ? 4 : 1;
}

template <typename QT, typename HT, int BLOCK, int G, int FLAV, bool INSTR>
__global__ __attribute__((amdgpu_flat_work_group_size(1, BLOCK), amdgpu_waves_per_eu(min_waves_per_eu<BLOCK, G, FLAV>())))
void step_kernel(const StepArgs a)
{
    using QW = typename Wide<QT>::T;
    constexpr bool kInt = !std::is_floating_point<HT>::value;
    constexpr int F = 4 * G;
    constexpr int W = BLOCK / 64;
    constexpr int NSEG = G * W;
    static_assert(NSEG <= 64, "segment scan needs at most 64 segments");
    static_assert(F <= 64, "bit masks are at most 64 bits");
    // per-lane bit masks (state, membership, existing bits): one bit per field
    using MT = std::conditional_t<(F > 32), uint64_t, uint32_t>;

    // dynamic LDS: [random-subset table, pitch entries (FLAV_DRAWN only)][diagonal, pitch entries]
    extern __shared__ uint32_t own[];
    __shared__ double seg_sum[NSEG];
    __shared__ double mx_part[W];
    __shared__ uint64_t masks[W];
    __shared__ int64_t sel[2];
    __shared__ int32_t stay_flag;
    __shared__ uint32_t hist_idx;
    __shared__ double tab_lo[kInt ? 2 * kTabLo : 1];
    __shared__ double tab_hi[kInt ? kTabHi : 1];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int chain = a.chain_list ? a.chain_list[blockIdx.x] : a.chain_first + (int)blockIdx.x;
    // The leader wave keeps the chain's scalars (energy, budget, records) and
    // does the per-step FP64 work; it rotates with the workgroup so that the
    // leaders of co-resident chains fall on different SIMDs.
    const int leader = (int)(blockIdx.x % (unsigned)W);
    const bool lead = wave == leader;
    const int lead_tid = leader * 64;
    // Uninstrumented window and drawn-subset kernels split the per-step record
    // between the leader lane (budget, multiplicity) and lane 0 of the next
    // wave (energy, action, counters), so that the two halves run on
    // different SIMDs after the choice; the leader's half is what the next
    // budget decision waits for.
    constexpr bool kSplitRec = !INSTR && FLAV != FLAV_ALL;
    const int rec_tid = W > 1 ? ((leader + 1) % W) * 64 : lead_tid + 1;
    const Problem P = a.problems[a.chain_problem[chain]];
    const int32_t N = P.N;
    const int64_t pitch = P.pitch;
    // Register budget: with four or more bits per lane beyond one group
    // (G >= 2) the diagonal lives in LDS and only four-bit weight sums are
    // kept (the chosen lane recomputes its weights); one group keeps both in
    // registers.  The compact and two-group windows read the diagonal from LDS.
    constexpr bool kLdsDiag = FLAV == FLAV_WINDOW_C || FLAV == FLAV_WINDOW_C2 || G >= 2;
    // The row of the flip is loaded before the record bookkeeping, which then
    // runs while the loads are in flight: with one field group per lane (the
    // registers allow it) and in the kernels whose record is split over two
    // lanes (each half is short); the other wide tiles keep the shorter live
    // ranges of loading after the record.
    constexpr bool kEarly = (G == 1 && FLAV != FLAV_WINDOW_C) || kSplitRec;
    constexpr bool kKeepW = FLAV == FLAV_WINDOW_C || G == 1;
    QW* const dsh = reinterpret_cast<QW*>(own + (FLAV == FLAV_DRAWN ? pitch : 0));
    const int mode = a.mode;
    const bool unbiased = mode == kModeSys || mode == kModeRand;
    // RF / Basic advancing by exactly a.orig_time original samples: the
    // budget rule of Alg 6 used as a stopping time (the record covering the
    // end is cut to the remaining time and the chain stops there)
    const bool timed = a.orig_time > 0;
    constexpr bool kWin = FLAV == FLAV_WINDOW || FLAV == FLAV_WINDOW_C || FLAV == FLAV_WINDOW_C2;
    constexpr bool kCompact = FLAV == FLAV_WINDOW_C;
    constexpr bool kTwo = FLAV == FLAV_WINDOW_C2;
    static_assert(!kTwo || G >= 2, "the two-group window needs two groups");
    const int32_t n = FLAV == FLAV_ALL ? N : P.n;
    const int s = P.s;
    const int64_t off = a.foff[chain];
    const double beta = a.beta[chain] * a.inv_temp;  // inv_temp = 1 except in kModeOpt
    const uint32_t cid = a.chain_id[chain];
    const uint64_t seed = a.seed;

    if constexpr (kInt) {
        // tab_lo[kTabLo .. 2 kTabLo) = 0 are the weights of bits outside the subset
        for (int i = tid; i < 2 * kTabLo + kTabHi; i += BLOCK) {
            if (i < kTabLo) tab_lo[i] = exp(-beta * (double)i);
            else if (i < 2 * kTabLo) tab_lo[i] = 0.0;
            else tab_hi[i - 2 * kTabLo] = exp(-beta * (double)(kTabLo * (i - 2 * kTabLo)));
        }
    }

    // ---- chain state into registers ----
    HT h[F];
    QW dg[kLdsDiag ? 1 : F];
    MT xb = 0;
    HT* hbase = reinterpret_cast<HT*>(a.h) + off;
    const QW* dbase = reinterpret_cast<const QW*>(P.diag);
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t fb = ((int64_t)g * BLOCK + tid) * 4;
        if (fb < pitch) {
            const Four<HT> hv = load4(hbase + fb);
            const Four<QW> dv = load4(dbase + fb);
            const uint32_t xw = *reinterpret_cast<const uint32_t*>(a.x + off + fb);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                h[g * 4 + v] = hv.v[v];
                if constexpr (kLdsDiag) dsh[fb + v] = dv.v[v];
                else dg[g * 4 + v] = dv.v[v];
                xb |= (MT)((xw >> (8 * v)) & 1u) << (g * 4 + v);
            }
        } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                h[g * 4 + v] = (HT)0;
                if constexpr (!kLdsDiag) dg[g * 4 + v] = (QW)0;
            }
        }
    }
    // bits of this lane that exist (f < N)
    MT valid = 0;
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int v = 0; v < 4; ++v) valid |= (MT)((g * BLOCK + tid) * 4 + v < N) << (g * 4 + v);

    // this lane's bits as bytes at dst[f] (the layout of x)
    auto store_bits = [&](uint8_t* dst) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const int64_t fb = ((int64_t)g * BLOCK + tid) * 4;
            if (fb < pitch) {
                uint32_t xw = 0;
#pragma unroll
                for (int v = 0; v < 4; ++v) xw |= (uint32_t)((xb >> (g * 4 + v)) & 1u) << (8 * v);
                *reinterpret_cast<uint32_t*>(dst + fb) = xw;
            }
        }
    };
    int64_t k = a.step[chain];
    const int64_t kend = k + a.steps;
    // Scalars only the leader lane uses (energy, budget, last record,
    // counters) live in LDS, not in every lane's registers.
    __shared__ int64_t lead_st[kLeadWords];
    __shared__ int best_flag;  // the state after the last flip is a new X_max
    if (tid == lead_tid) {
        lead_st[kLsE] = a.E[chain];
        if constexpr (INSTR) {
            if (a.xbest != nullptr) lead_st[kLsBest] = a.Ebest[chain];
        }
        lead_st[kLsL] = timed ? a.orig_time : a.L[chain];
        lead_st[kLsLastA] = a.last_action[chain];
        lead_st[kLsLastM] = a.last_M[chain];
        lead_st[kLsLastE] = a.last_E[chain];
        for (int q = kLsSteps; q <= kLsSumM; ++q) lead_st[q] = 0;
        best_flag = 0;
    }
    int64_t sub = a.sub[chain];
    int32_t snap_n = 0;
    if constexpr (INSTR) snap_n = a.snap_every > 0 ? a.snap_count[chain] : 0;
    uint32_t pos_n = 0;
    int32_t last_row = 0;  // the row loaded by the previous step
    const bool full = n >= N;
    int64_t sys_start = kWin ? (int64_t)(((sub % P.num_sets) * (int64_t)n) % N) : 0;

    if constexpr (FLAV == FLAV_DRAWN) {
        if (mode == kModeRand) {
            if (k == 0) {
                pos_n = draw_subset<BLOCK, G>(own, masks, tid, pitch, N, n, seed, cid, k);
            } else {
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const int64_t fb = ((int64_t)g * BLOCK + tid) * 4;
                    if (fb < pitch) {
                        const uint32_t mw = *reinterpret_cast<const uint32_t*>(a.rmem + off + fb);
#pragma unroll
                        for (int v = 0; v < 4; ++v) own[fb + v] = ((mw >> (8 * v)) & 1u) ? 0u : 0xFFFFFFFFu;
                    }
                }
                pos_n = 0;
            }
        }
    }
    __syncthreads();  // tables and subset table ready

    double ubLog = 0.0, ubU2 = 0.0;
    int64_t ub_base = k;
    batch_uniforms(cid, ub_base, seed, lane, lead, &ubLog, &ubU2);
    // p = S / n: for a power-of-two n the product by 1/n is the same number
    const bool n_pow2 = (n & (n - 1)) == 0;
    const double inv_n = 1.0 / (double)n;

    // Membership of this lane's bits in the current subset.  It changes only
    // when the subset does (a new window or draw), so it is kept across steps.
    auto compute_mem = [&]() -> MT {
        MT m = valid;
        if constexpr (kWin) {
            if (!full) {
                // bit f is in the window iff (f - start) mod N < n
                // (built by shifts from the top bit down: no per-bit mask
                // constants, which would sit in registers for the whole loop)
                m = 0;
                const int32_t d0 = tid * 4 - (int32_t)sys_start;
#pragma unroll
                for (int i = F - 1; i >= 0; --i) {
                    int32_t d = d0 + (i >> 2) * (BLOCK * 4) + (i & 3);
                    d += d < 0 ? N : 0;
                    m = (m << 1) | (MT)(d < n);
                }
                m &= valid;
            }
        } else if constexpr (FLAV == FLAV_DRAWN) {
            m = 0;
#pragma unroll
            for (int i = 0; i < F; ++i) {
                const int32_t f = ((i >> 2) * BLOCK + tid) * 4 + (i & 3);
                if ((valid >> i) & 1u) m |= (MT)(own[f] <= pos_n) << i;
            }
        }
        return m;
    };
    const bool draw_each_step = mode == kModeBasic || mode == kModeOpt;
    MT mem = (FLAV == FLAV_DRAWN && draw_each_step) ? (MT)0 : compute_mem();
    // one group per lane, 32-bit integer fields: the table reads of the
    // weights by byte offset (below), with the offset of the zero slots of
    // tab_lo for each bit outside the subset kept with the membership
    constexpr bool kByteTab = kInt && sizeof(HT) == 4 && G == 1 && !kCompact && !kTwo;
    uint32_t zo[kByteTab ? 4 : 1] = {};
    auto set_zo = [&]() {
        if constexpr (kByteTab) {
#pragma unroll
            for (int v = 0; v < 4; ++v) zo[v] = ((mem >> v) & 1u) ? 0u : (uint32_t)(8 * kTabLo);
        }
    };
    set_zo();

    // RF / Basic sampling without per-step outputs: M steers nothing, so the
    // multiplicities of up to 64 steps are computed together by the leader
    // wave, lane j for step ub_base + j (the step uniforms are laid out the
    // same way); lane j of pbuf keeps that step's escape probability p.
    const bool lazy_m = !INSTR && !unbiased && !timed && mode != kModeOpt;
    double pbuf = 0.0;
    auto flush_m = [&](int cnt) {  // leader wave only
        const double pj = pbuf;
        double qj;
        if (pj >= 1.0) qj = 0.0;
        else if (pj <= 0.0) qj = INFINITY;
        else qj = ubLog / log1p(-pj);
        const bool act = lane < cnt;
        const bool satj = act && !(qj < 0x1p63);
        const int64_t mj = satj ? INT64_MAX : (act ? (int64_t)floor(qj) + 1 : 0);
        double tot = act ? (double)mj : 0.0;
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) tot += __shfl_xor(tot, d, 64);
        const uint64_t nsat = __ballot(satj);
        const int lo = __shfl((int)(uint32_t)mj, cnt - 1, 64), hi = __shfl((int)(mj >> 32), cnt - 1, 64);
        if (tid == lead_tid) {
            lead_st[kLsSumM] = __double_as_longlong(__longlong_as_double(lead_st[kLsSumM]) + tot);
            lead_st[kLsSat] += __builtin_popcountll(nsat);
            lead_st[kLsLastM] = (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
        }
    };

    for (; k < kend; ++k) {
        __builtin_amdgcn_s_setprio(0);
        if (k - ub_base >= 64) {
            if (lazy_m && lead) flush_m(64);
            ub_base = k;
            batch_uniforms(cid, ub_base, seed, lane, lead, &ubLog, &ubU2);
        }
        const int uj = (int)(k - ub_base);
        StepUniforms U;
        U.U2 = read_lane(ubU2, uj);
        U.logU1 = lead ? read_lane(ubLog, uj) : 0.0;
        if constexpr (FLAV == FLAV_DRAWN) {
            if (draw_each_step) {
                // the draw is barrier-gated too (its rounds meet in LDS)
                __builtin_amdgcn_s_setprio(1);
                pos_n = draw_subset<BLOCK, G>(own, masks, tid, pitch, N, n, seed, cid, k);
                mem = compute_mem();
                set_zo();
                __builtin_amdgcn_s_setprio(0);
            }
        }

        // acceptance weights of the subset, summed four bits at a time
        // the diagonal entry of the lane's bit i (i a compile-time index
        // unless the diagonal is in LDS); 0 past the pitch
        auto diag_of = [&](int i) -> QW {
            if constexpr (kLdsDiag) {
                const int64_t f = ((int64_t)(i >> 2) * BLOCK + tid) * 4 + (i & 3);
                return f < pitch ? dsh[f] : (QW)0;
            } else {
                return dg[i % F];
            }
        };
        auto member_weight = [&](int i, double shift) -> double {
            const QW di = diag_of(i);
            if constexpr (kInt) {
                const HT e = delta_int(di, h[i], s, (xb >> i) & 1u);
                if (shift == 0.0) {
                    const HT ep = e > 0 ? e : 0;
                    if (ep < (HT)kTabMax) return tab_hi[(uint32_t)(ep >> 6)] * tab_lo[(uint32_t)ep & 63u];
                    return exp(-beta * (double)e);
                }
                double l = -beta * (double)e;
                l = l < 0.0 ? l : 0.0;
                return exp(l - shift);
            } else {
                double l = -beta * delta_f64(di, h[i], s, (xb >> i) & 1u);
                l = l < 0.0 ? l : 0.0;
                return shift == 0.0 ? exp(l) : exp(l - shift);
            }
        };
        double w[kKeepW || kTwo ? 4 : 1];  // weights of the lane's four bits (compact: in group gw; two-group: ga)
        double w2[kTwo ? 4 : 1];            // two-group window: the four bits in group gb
        double ls[kCompact || kTwo ? 1 : G];
        // Compact window: a wave's subset bits lie in one 4-bit group (gw) and
        // each lane's in its four bits of that group.
        double lsum = 0.0;
        int gw = 0;
        auto compact_weights = [&](double shift) {
            constexpr MT k1 = (MT)0x1111111111111111ull;
            const MT gmask = (mem & k1) | ((mem >> 1) & k1) | ((mem >> 2) & k1) | ((mem >> 3) & k1);
            const int gs = gmask ? (__builtin_ctzll((uint64_t)gmask) >> 2) : 0;
            const uint32_t mg = (uint32_t)(mem >> (4 * gs)) & 0xFu;
            const uint64_t bm = __ballot(mg != 0);
            gw = bm ? __builtin_amdgcn_readlane(gs, (int)__builtin_ctzll(bm)) : 0;
            double w4[4] = {0.0, 0.0, 0.0, 0.0};
            if (bm) {
                HT h4[4];
#pragma unroll
                for (int v = 0; v < 4; ++v) h4[v] = h[v];
#pragma unroll
                for (int g = 1; g < G; ++g) {
                    if (gw == g) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) h4[v] = h[g * 4 + v];
                    }
                }
                const int32_t fb = (gw * BLOCK + tid) * 4;
                const Four<QW> d4 = load4(dsh + (fb < pitch ? fb : 0));
                const uint32_t x4 = (uint32_t)(xb >> (4 * gw)) & 0xFu;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    double wv;
                    if constexpr (kInt) {
                        const HT e = delta_int(d4.v[v], h4[v], s, (x4 >> v) & 1u);
                        if (shift == 0.0) {
                            const HT ep = e > 0 ? e : 0;
                            wv = ep < (HT)kTabMax ? tab_hi[(uint32_t)(ep >> 6)] * tab_lo[(uint32_t)ep & 63u]
                                                  : exp(-beta * (double)e);
                        } else {
                            double l = -beta * (double)e;
                            l = l < 0.0 ? l : 0.0;
                            wv = exp(l - shift);
                        }
                    } else {
                        double l = -beta * delta_f64(d4.v[v], h4[v], s, (x4 >> v) & 1u);
                        l = l < 0.0 ? l : 0.0;
                        wv = shift == 0.0 ? exp(l) : exp(l - shift);
                    }
                    w4[v] = ((mg >> v) & 1u) ? wv : 0.0;
                }
            }
            lsum = ((w4[0] + w4[1]) + w4[2]) + w4[3];
#pragma unroll
            for (int v = 0; v < 4; ++v) w[v] = w4[v];
        };
        // Two-group window: a wave's subset bits lie in groups ga <= gb (the
        // lowest and highest it holds), so each lane weighs at most its four
        // bits of ga and its four bits of gb.
        double lsum2 = 0.0;
        int ga = 0, gb = 0;
        auto group_weights = [&](int gsel, double shift, double* w4) {
            const uint32_t mg = (uint32_t)(mem >> (4 * gsel)) & 0xFu;
            HT h4[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) h4[v] = h[v];
#pragma unroll
            for (int g = 1; g < G; ++g) {
                if (gsel == g) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) h4[v] = h[g * 4 + v];
                }
            }
            const int32_t fb = (gsel * BLOCK + tid) * 4;
            const Four<QW> d4 = load4(dsh + (fb < pitch ? fb : 0));
            const uint32_t x4 = (uint32_t)(xb >> (4 * gsel)) & 0xFu;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double wv;
                if constexpr (kInt) {
                    const HT e = delta_int(d4.v[v], h4[v], s, (x4 >> v) & 1u);
                    if (shift == 0.0) {
                        const HT ep = e > 0 ? e : 0;
                        wv = ep < (HT)kTabMax ? tab_hi[(uint32_t)(ep >> 6)] * tab_lo[(uint32_t)ep & 63u]
                                              : exp(-beta * (double)e);
                    } else {
                        double l = -beta * (double)e;
                        l = l < 0.0 ? l : 0.0;
                        wv = exp(l - shift);
                    }
                } else {
                    double l = -beta * delta_f64(d4.v[v], h4[v], s, (x4 >> v) & 1u);
                    l = l < 0.0 ? l : 0.0;
                    wv = shift == 0.0 ? exp(l) : exp(l - shift);
                }
                w4[v] = ((mg >> v) & 1u) ? wv : 0.0;
            }
        };
        auto two_group_weights = [&](double shift) {
            uint32_t wg = 0;
#pragma unroll
            for (int g = 0; g < G; ++g) wg |= __ballot(((mem >> (4 * g)) & 0xFu) != 0) ? (1u << g) : 0u;
            ga = wg ? __builtin_ctz(wg) : 0;
            gb = wg ? 31 - __builtin_clz(wg) : 0;
            double wa[4] = {0.0, 0.0, 0.0, 0.0}, wb[4] = {0.0, 0.0, 0.0, 0.0};
            if (wg) group_weights(ga, shift, wa);
            if (gb != ga) group_weights(gb, shift, wb);
            lsum = ((wa[0] + wa[1]) + wa[2]) + wa[3];
            lsum2 = ((wb[0] + wb[1]) + wb[2]) + wb[3];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                w[v] = wa[v];
                w2[v] = wb[v];
            }
        };
        if constexpr (kCompact) {
            compact_weights(0.0);
        } else if constexpr (kTwo) {
            two_group_weights(0.0);
        } else if constexpr (kInt) {
            // exp(-beta * max(e, 0)) = tab_hi[e >> 6] * tab_lo[e & 63]; exp(-0) = 1
            // covers e <= 0, and a bit outside the subset reads the zero slot.
#pragma unroll
            for (int g = 0; g < G; ++g) {
                Four<QW> d4;
                if constexpr (kLdsDiag) {
                    const int64_t fb = ((int64_t)g * BLOCK + tid) * 4;
                    d4 = fb < pitch ? load4(dsh + fb) : Four<QW>{};
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v) d4.v[v] = dg[(g * 4 + v) % F];
                }
                double w4[4];
                HT emax = 0;
                HT ep4[kByteTab ? 4 : 1];
                if constexpr (kByteTab) {
                    // The tables are read by byte offset and the eight reads
                    // go out together (one LDS round trip); wider tiles and
                    // 64-bit fields keep the per-bit form below, which holds
                    // fewer registers.  tab_hi[ep >> 6] sits at
                    // (ep >> 3) & ~7 (an ep past the table wraps inside it and
                    // its weight is recomputed by exp below), tab_lo[ep & 63]
                    // at 8 (ep & 63), moved into the zero slots for a bit
                    // outside the subset.
                    const char* thb = reinterpret_cast<const char*>(tab_hi);
                    const char* tlb = reinterpret_cast<const char*>(tab_lo);
                    uint32_t ho[4], lo[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        // dE with the sign of the bit as (t ^ m) - m, m = 0 or -1
                        const HT m = -(HT)((xb >> v) & 1u);
                        const HT t = (HT)d4.v[v] + (s == 2 ? (HT)(h[v] + h[v]) : h[v]);
                        const HT e = (t ^ m) - m;
                        const HT ep = e > 0 ? e : 0;
                        ep4[v] = ep;
                        emax = emax > ep ? emax : ep;
                        const uint32_t u = (uint32_t)ep;
                        ho[v] = (u >> 3) & (uint32_t)(8 * (kTabHi - 1));
                        lo[v] = ((u << 3) & (uint32_t)(8 * (kTabLo - 1))) | zo[v];
                    }
                    double th[4], tl[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        th[v] = *reinterpret_cast<const double*>(thb + ho[v]);
                        tl[v] = *reinterpret_cast<const double*>(tlb + lo[v]);
                    }
                    __builtin_amdgcn_sched_group_barrier(0x0100, 8, 0);
#pragma unroll
                    for (int v = 0; v < 4; ++v) w4[v] = th[v] * tl[v];
                } else {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = g * 4 + v;
                        const HT e = delta_int(d4.v[v], h[i], s, (xb >> i) & 1u);
                        const HT ep = e > 0 ? e : 0;
                        emax = emax > ep ? emax : ep;
                        const uint32_t hi =
                            (uint32_t)(ep >> 6) < (uint32_t)kTabHi ? (uint32_t)(ep >> 6) : (uint32_t)(kTabHi - 1);
                        const uint32_t lo = ((mem >> i) & 1u) ? (uint32_t)ep & 63u : (uint32_t)kTabLo;
                        w4[v] = tab_hi[hi] * tab_lo[lo];
                    }
                }
                if (__ballot(emax >= (HT)kTabMax)) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = g * 4 + v;
                        // (e = ep when e reaches the tables' end)
                        HT e;
                        if constexpr (kByteTab) e = ep4[v];
                        else e = delta_int(d4.v[v], h[i], s, (xb >> i) & 1u);
                        if (((mem >> i) & 1u) && e >= (HT)kTabMax) w4[v] = exp(-beta * (double)e);
                    }
                }
                ls[g] = ((w4[0] + w4[1]) + w4[2]) + w4[3];
                if constexpr (kKeepW) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) w[v] = w4[v];
                }
            }
        } else {
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const uint32_t mg = (uint32_t)(mem >> (4 * g)) & 0xFu;
                double w4[4] = {0.0, 0.0, 0.0, 0.0};
                if (__ballot(mg != 0)) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) w4[v] = ((mg >> v) & 1u) ? member_weight(g * 4 + v, 0.0) : 0.0;
                }
                ls[g] = ((w4[0] + w4[1]) + w4[2]) + w4[3];
                if constexpr (kKeepW) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) w[v] = w4[v];
                }
            }
        }
        double inc[kCompact || kTwo ? 1 : G];
        double inc2 = 0.0;
        auto scan_and_publish = [&]() {
            if constexpr (kCompact) {
                inc[0] = wave_scan(lsum);
                if (lane == 63) {
#pragma unroll
                    for (int g = 0; g < G; ++g) seg_sum[g * W + wave] = g == gw ? inc[0] : 0.0;
                }
            } else if constexpr (kTwo) {
                inc[0] = wave_scan(lsum);
                inc2 = gb != ga ? wave_scan(lsum2) : 0.0;  // ga, gb are wave-uniform
                if (lane == 63) {
#pragma unroll
                    for (int g = 0; g < G; ++g) seg_sum[g * W + wave] = g == ga ? inc[0] : (g == gb ? inc2 : 0.0);
                }
            } else {
#pragma unroll
                for (int g = 0; g < G; ++g) inc[g] = wave_scan(ls[g]);
                if (lane == 63) {
#pragma unroll
                    for (int g = 0; g < G; ++g) seg_sum[g * W + wave] = inc[g];
                }
            }
        };
        // From the wave scans to the issue of the row load every wave of the
        // chain waits at a barrier for the slowest one, so these phases take
        // issue priority over the weights and field updates of the other
        // chains on the SIMD.
        __builtin_amdgcn_s_setprio(1);
        scan_and_publish();
        __syncthreads();
        if constexpr (INSTR) {
            // X_max of Alg 9/10: the state reached by the previous step's flip
            if (a.xbest != nullptr && best_flag) store_bits(a.xbest + off);
        }
        double sv = lane < NSEG ? seg_sum[lane] : 0.0;
        double sinc = small_scan<NSEG>(sv);
        double S = read_lane(sinc, NSEG - 1);
        double mx = 0.0;
        bool scaled = false;
        if (S < 0x1p-1000) {
            // Every weight underflowed: rescale by the largest log-weight.
            double lm = -INFINITY;
#pragma unroll
            for (int i = 0; i < F; ++i) {
                if ((mem >> i) & 1u) {
                    const QW di = diag_of(i);
                    double l;
                    if constexpr (kInt) l = -beta * (double)delta_int(di, h[i], s, (xb >> i) & 1u);
                    else l = -beta * delta_f64(di, h[i], s, (xb >> i) & 1u);
                    l = l < 0.0 ? l : 0.0;
                    lm = fmax(lm, l);
                }
            }
            lm = wave_max(lm);
            if (lane == 0) mx_part[wave] = lm;
            __syncthreads();
            mx = -INFINITY;
            for (int ww = 0; ww < W; ++ww) mx = fmax(mx, mx_part[ww]);
            scaled = true;
            if constexpr (kCompact) {
                compact_weights(mx);
            } else if constexpr (kTwo) {
                two_group_weights(mx);
            } else {
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    double w4[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = g * 4 + v;
                        w4[v] = ((mem >> i) & 1u) ? member_weight(i, mx) : 0.0;
                    }
                    ls[g] = ((w4[0] + w4[1]) + w4[2]) + w4[3];
                    if constexpr (kKeepW) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) w[v] = w4[v];
                    }
                }
            }
            scan_and_publish();
            __syncthreads();
            sv = lane < NSEG ? seg_sum[lane] : 0.0;
            sinc = small_scan<NSEG>(sv);
            S = read_lane(sinc, NSEG - 1);
        }

        if (lazy_m && lead) {
            const double Ss = scaled ? exp(mx) * S : S;
            const double pv = n_pow2 ? Ss * inv_n : Ss / (double)n;
            pbuf = lane == uj ? pv : pbuf;
        }

        // Escape probability and multiplicity M = 1 + G, G ~ Geometric(p)
        // counting failures; uniform FP64 work done by wave 0 only.
        double p = 0.0, q = 0.0;
        int64_t m = 0;
        bool sat = false;
        // (Lq: the budget the quotient is compared with, or -1 without one)
        auto multiplicity = [&](double Lq) {
            const double Ss = scaled ? exp(mx) * S : S;
            p = n_pow2 ? Ss * inv_n : Ss / (double)n;
            if (p >= 1.0) q = 0.0;
            else if (p <= 0.0) q = INFINITY;
            else if constexpr (FLAV == FLAV_ALL) q = U.logU1 / log1p(-p);  // budgets only in timed runs
            else q = geometric_quotient(U.logU1, p, Lq);
            if (!(q < 0x1p63)) {
                m = INT64_MAX;
                sat = true;
            } else {
                m = (int64_t)floor(q) + 1;
                sat = false;
            }
        };
        // Budgeted runs: the leader takes the budget decision of Alg 6 while
        // the winner wave resolves the (speculative) choice; both meet at the
        // barrier.  Otherwise M does not steer the chain and is computed with
        // the record, off the path to the next step.
        if ((unbiased || timed) && tid == lead_tid) {
            const double Lb = (double)lead_st[kLsL];
            multiplicity(Lb);
            stay_flag = q >= Lb ? 1 : 0;
        }
        uint32_t rec_idx = 0;
        bool snap = false;
        if constexpr (INSTR) {
            // state index of the record for the histograms (N <= 24: lanes 0..5 of
            // wave 0), handed to the leader through LDS
            if (a.hist_w != nullptr) {
                if (wave == 0) {
                    rec_idx = wave_or(tid < 8 ? ((uint32_t)(xb & 0xFu) << (4 * tid)) : 0u);
                    if (tid == 0) hist_idx = rec_idx;
                }
            }
            snap = a.snap_every > 0 && ((k + 1) % a.snap_every) == 0;
            if (snap) {
                const int32_t slot = snap_n % a.snap_cap;
                uint8_t* sx = a.snap_x + ((int64_t)chain * a.snap_cap + slot) * a.snap_pitch;
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const int64_t fb = ((int64_t)g * BLOCK + tid) * 4;
                    if (fb < a.snap_pitch) {
                        uint32_t wv = 0;
#pragma unroll
                        for (int v = 0; v < 4; ++v) wv |= (uint32_t)((xb >> (g * 4 + v)) & 1u) << (8 * v);
                        *reinterpret_cast<uint32_t*>(sx + fb) = wv;
                    }
                }
            }
        }

        // Proportional choice (appendix "How to Sample Proportionally"): first
        // bit whose running sum exceeds U2 * S, resolved segment -> lane -> bit.
        {
            const double t = U.U2 * S;
            const bool pos_seg = lane < NSEG && sv > 0.0;
            const uint64_t bseg = __ballot(pos_seg && sinc > t);
            const uint64_t bpos = __ballot(pos_seg);
            int jstar = bseg ? __builtin_ctzll(bseg) : (bpos ? 63 - __builtin_clzll(bpos) : 0);
            jstar = jstar < NSEG ? jstar : NSEG - 1;
            const int gstar = jstar / W, wstar = jstar % W;
            if (wave == wstar) {
                const double base = jstar > 0 ? read_lane(sinc, jstar - 1) : 0.0;  // jstar is wave-uniform
                double my_inc = 0.0, my_ls = 0.0;
                if constexpr (kCompact) {
                    my_inc = inc[0];
                    my_ls = lsum;
                } else if constexpr (kTwo) {
                    const bool second = gstar == gb && gb != ga;
                    my_inc = second ? inc2 : inc[0];
                    my_ls = second ? lsum2 : lsum;
                } else {
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        if (g == gstar) {
                            my_inc = inc[g];
                            my_ls = ls[g];
                        }
                    }
                }
                const double Gl = base + my_inc;
                const uint64_t bl = __ballot(my_ls > 0.0 && Gl > t);
                const uint64_t blp = __ballot(my_ls > 0.0);
                const int lstar = bl ? __builtin_ctzll(bl) : (blp ? 63 - __builtin_clzll(blp) : 0);
                const double prev_l = read_lane(my_inc, lstar > 0 ? lstar - 1 : 0);  // lstar is wave-uniform
                if (lane == lstar) {
                    double run = lstar > 0 ? base + prev_l : base;
                    int vstar = -1, vlast = -1;
                    // the chosen lane's four weights in group gstar: kept, or
                    // recomputed (the same values as summed above)
                    double wsel[4];
                    if constexpr (kTwo) {
                        const bool second = gstar == gb && gb != ga;
#pragma unroll
                        for (int v = 0; v < 4; ++v) wsel[v] = second ? w2[v] : w[v];
                    } else if constexpr (kKeepW) {
#pragma unroll
                        for (int v = 0; v < 4; ++v) wsel[v] = w[v];
                    } else {
                        const uint32_t mg = (uint32_t)(mem >> (4 * gstar)) & 0xFu;
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            wsel[v] = ((mg >> v) & 1u) ? member_weight(gstar * 4 + v, scaled ? mx : 0.0) : 0.0;
                    }
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const double wv = wsel[v];
                        if (wv > 0.0) {
                            vlast = v;
                            run += wv;
                            if (vstar < 0 && run > t) vstar = v;
                        }
                    }
                    if (vstar < 0) vstar = vlast;
                    // No positive weight in the chosen lane cannot happen when S > 0;
                    // keep the address in range and report it.
                    int64_t bad = 0;
                    if (vstar < 0) {
                        vstar = 0;
                        bad = 1;
                    }
                    const int i = gstar * 4 + vstar;
                    HT hc = (HT)0;
                    QW dc = (QW)0;
#pragma unroll
                    for (int ii = 0; ii < F; ++ii) {
                        if (ii == i) {
                            hc = h[ii];
                            if constexpr (!kLdsDiag) dc = dg[ii];
                        }
                    }
                    if constexpr (kLdsDiag) dc = diag_of(i);
                    int64_t dEc;
                    if constexpr (kInt) dEc = (int64_t)delta_int(dc, hc, s, (xb >> i) & 1u);
                    else dEc = __double_as_longlong(delta_f64(dc, hc, s, (xb >> i) & 1u));
                    int64_t c = ((int64_t)gstar * BLOCK + tid) * 4 + vstar;
                    if (c >= N) {
                        c = 0;
                        bad = 1;
                    }
                    sel[0] = c | ((int64_t)((xb >> i) & 1u) << 40) | (bad << 41);
                    sel[1] = dEc;
                }
            }
        }
        __syncthreads();
        const bool stay = (unbiased || timed) && stay_flag != 0;

        // row c of the flip: in the early-load kernels it is loaded before the
        // record bookkeeping below, which then runs while the loads are in
        // flight, and the fields are updated after it
        decltype(load_raw4(static_cast<const QT*>(nullptr))) raw[G];
        bool xc = false;
        auto update_fields = [&]() {
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const auto r = widen4(raw[g]);
                if (((int64_t)g * BLOCK + tid) * 4 < pitch) {
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        if (xc) h[g * 4 + v] -= (HT)r.v[v];
                        else h[g * 4 + v] += (HT)r.v[v];
                    }
                }
            }
        };
        const int64_t sv0 = sel[0];
        const int32_t csel = (int32_t)(sv0 & 0xFFFFFFFFll);  // in [0, N) on every step
        // Row csel: every lane loads (lanes past the pitch read the row's start
        // and drop it), so no branch forces an early wait.  The early-load
        // kernels load whether or not the chain stays (a stay drops it), so
        // that the loaded registers are not joined from two branches; a stay
        // reads the row loaded last, which the caches still hold, instead of
        // the speculative choice's (in Unbiased PNS at low acceptance most
        // steps are stays).
        const int32_t rsel = (kEarly && stay) ? last_row : csel;
        last_row = rsel;
        const QT* row = reinterpret_cast<const QT*>(P.A) + (int64_t)rsel * pitch;
        if constexpr (kEarly) {
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int64_t fb = ((int64_t)g * BLOCK + tid) * 4;
                raw[g] = load_raw4(row + (fb < pitch ? fb : 0));
            }
        }
        // (the leader wave takes a higher one through the record when it
        // writes all of it: the next step's first barrier waits for it)
        __builtin_amdgcn_s_setprio(0);
        if constexpr (!kSplitRec) {
            if (lead) __builtin_amdgcn_s_setprio(2);
        }
        if (stay) {
            // Alg 6: not enough remaining original samples; stay L times and
            // switch to the next partial neighbor set (a timed run just ends).
            if (!timed) {
                ++sub;
                if constexpr (FLAV == FLAV_DRAWN) {
                    pos_n = draw_subset<BLOCK, G>(own, masks, tid, pitch, N, n, seed, cid, k + 1);
                } else if constexpr (kWin) {
                    sys_start = (int64_t)(((sub % P.num_sets) * (int64_t)n) % N);
                }
                mem = compute_mem();
                set_zo();
            }
        } else {
            const int32_t c = csel;
            xc = (sv0 >> 40) & 1;
            if constexpr (!kEarly) {
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const int64_t fb = ((int64_t)g * BLOCK + tid) * 4;
                    raw[g] = load_raw4(row + (fb < pitch ? fb : 0));
                }
            }
            const int cl = (c >> 2) % BLOCK;
            const int cg = (c >> 2) / BLOCK;
            if (tid == cl) xb ^= (MT)1 << (cg * 4 + (c & 3));
            if constexpr (!kEarly) update_fields();
        }
        if constexpr (INSTR) {
            if (snap) ++snap_n;
        }

        // record k = (state before the step, M)
        if constexpr (kSplitRec) {
            if (tid == lead_tid) {
                int64_t M;
                if (stay) {
                    M = lead_st[kLsL];
                    lead_st[kLsL] = timed ? 0 : P.L0;
                } else {
                    if (mode == kModeOpt) {
                        m = 1;  // no multiplicity: each jump counts once
                        sat = false;
                    }
                    if (unbiased || timed) lead_st[kLsL] -= m;
                    lead_st[kLsSat] += sat ? 1 : 0;
                    M = m;
                }
                if (!lazy_m) lead_st[kLsSumM] = __double_as_longlong(__longlong_as_double(lead_st[kLsSumM]) + (double)M);
                if (!lazy_m) lead_st[kLsLastM] = M;
            }
            if (tid == rec_tid) {
                const int64_t Erec = lead_st[kLsE];
                int32_t action = -1;
                if (stay) {
                    lead_st[kLsStays] += 1;
                } else {
                    const int64_t dEc = sel[1];
                    lead_st[kLsBad] += (sv0 >> 41) & 1;
                    if constexpr (kInt) lead_st[kLsE] = Erec + dEc;
                    else lead_st[kLsE] = __double_as_longlong(__longlong_as_double(Erec) + __longlong_as_double(dEc));
                    lead_st[kLsFlips] += 1;
                    action = (int32_t)(sv0 & 0xFFFFFFFFll);
                }
                lead_st[kLsSteps] += 1;
                lead_st[kLsLastA] = action;
                lead_st[kLsLastE] = Erec;
            }
        } else if (tid == lead_tid) {
            const int64_t Erec = lead_st[kLsE];
            const int64_t Lrec = lead_st[kLsL];  // budget at the start of the record
            int32_t action;
            int64_t M;
            if (stay) {
                M = lead_st[kLsL];
                action = -1;
                lead_st[kLsL] = timed ? 0 : P.L0;
                lead_st[kLsStays] += 1;
                if constexpr (INSTR) best_flag = 0;
            } else {
                const int64_t sv0 = sel[0];
                const int64_t dEc = sel[1];
                if (!unbiased && !timed && !lazy_m) multiplicity(-1.0);
                if (mode == kModeOpt) {
                    m = 1;  // no multiplicity: each jump counts once
                    sat = false;
                }
                if (unbiased || timed) lead_st[kLsL] -= m;
                lead_st[kLsSat] += sat ? 1 : 0;
                lead_st[kLsBad] += (sv0 >> 41) & 1;
                if constexpr (kInt) lead_st[kLsE] = Erec + dEc;
                else lead_st[kLsE] = __double_as_longlong(__longlong_as_double(Erec) + __longlong_as_double(dEc));
                lead_st[kLsFlips] += 1;
                M = m;
                action = (int32_t)(sv0 & 0xFFFFFFFFll);
                if constexpr (INSTR) {
                    if (a.xbest != nullptr) {
                        const int64_t En = lead_st[kLsE], Eb = lead_st[kLsBest];
                        const bool better = kInt ? En < Eb : __longlong_as_double(En) < __longlong_as_double(Eb);
                        if (better) lead_st[kLsBest] = En;
                        best_flag = better ? 1 : 0;
                    }
                }
            }
            lead_st[kLsSteps] += 1;
            if (!lazy_m) lead_st[kLsSumM] = __double_as_longlong(__longlong_as_double(lead_st[kLsSumM]) + (double)M);
            lead_st[kLsLastA] = action;
            if (!lazy_m) lead_st[kLsLastM] = M;
            lead_st[kLsLastE] = Erec;
            if constexpr (INSTR) {
                // Rao-Blackwell weight of the record: E[M | state, subset, budget]
                double wrb = 1.0;
                if (mode != kModeOpt && (snap || a.log_cap > 0 || a.hist_w != nullptr))
                    wrb = expected_multiplicity(p, Lrec, unbiased || timed);
                if (a.hist_w != nullptr) rec_idx = hist_idx;
                if (a.log_cap > 0) {
                    const int64_t slot = (int64_t)chain * a.log_cap + (k % a.log_cap);
                    a.log_action[slot] = action;
                    a.log_M[slot] = M;
                    a.log_E[slot] = Erec;
                    a.log_p[slot] = p;
                    a.log_w[slot] = wrb;
                }
                if (a.hist_w != nullptr) {
                    atomicAdd(&a.hist_w[rec_idx], (unsigned long long)M);
                    atomicAdd(&a.hist_v[rec_idx], 1ull);
                    atomicAdd(&a.hist_rb[rec_idx], wrb);
                }
                if (snap) {
                    const int32_t slot = (snap_n - 1) % a.snap_cap;
                    a.snap_M[(int64_t)chain * a.snap_cap + slot] = M;
                    a.snap_E[(int64_t)chain * a.snap_cap + slot] = Erec;
                    a.snap_w[(int64_t)chain * a.snap_cap + slot] = wrb;
                }
            }
        }
        if constexpr (kEarly) {
            if (!stay) update_fields();
        }
        if (timed && stay) {
            ++k;  // the cut record was the run's last
            break;
        }
    }
    if (lazy_m && lead && k > ub_base) flush_m((int)(k - ub_base));
    if constexpr (kSplitRec) __syncthreads();  // the record lane's words, for the write-out below

    if constexpr (INSTR) {
        __syncthreads();
        if (a.xbest != nullptr && best_flag) store_bits(a.xbest + off);
        if (a.xbest != nullptr && tid == lead_tid) a.Ebest[chain] = lead_st[kLsBest];
    }

    // ---- chain state back to memory ----
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t fb = ((int64_t)g * BLOCK + tid) * 4;
        if (fb < pitch) {
            HT hv[4];
            uint32_t xw = 0, mw = 0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                hv[v] = h[g * 4 + v];
                xw |= (uint32_t)((xb >> (g * 4 + v)) & 1u) << (8 * v);
                if constexpr (FLAV == FLAV_DRAWN) mw |= (uint32_t)(own[fb + v] <= pos_n) << (8 * v);
            }
            store4(hbase + fb, hv);
            *reinterpret_cast<uint32_t*>(a.x + off + fb) = xw;
            if constexpr (FLAV == FLAV_DRAWN) {
                if (mode == kModeRand) *reinterpret_cast<uint32_t*>(a.rmem + off + fb) = mw;
            }
        }
    }
    if (tid == lead_tid) {
        a.step[chain] = k;
        a.E[chain] = lead_st[kLsE];
        a.L[chain] = lead_st[kLsL];
        a.sub[chain] = sub;
        a.last_action[chain] = (int32_t)lead_st[kLsLastA];
        a.last_M[chain] = lead_st[kLsLastM];
        a.last_E[chain] = lead_st[kLsLastE];
        if constexpr (INSTR) {
            if (a.snap_every > 0) a.snap_count[chain] = snap_n;
        }
        int64_t* cn = a.counters + (int64_t)chain * 6;
        cn[0] += lead_st[kLsSteps];
        cn[1] += lead_st[kLsFlips];
        cn[2] += lead_st[kLsStays];
        cn[3] += lead_st[kLsSat];
        cn[4] = __double_as_longlong(__longlong_as_double(cn[4]) + __longlong_as_double(lead_st[kLsSumM]));
        cn[5] += lead_st[kLsBad];
    }
}

template <typename QT, typename HT, int BLOCK, int G, int FLAV, bool INSTR>
hipError_t launch_one(int32_t grid, size_t dyn, hipStream_t st, const StepArgs& a)
{
    hipLaunchKernelGGL((step_kernel<QT, HT, BLOCK, G, FLAV, INSTR>), dim3(grid), dim3(BLOCK), dyn, st, a);
    return hipGetLastError();
}

// Tile shapes (workgroup size, 4-bit groups per lane) compiled for every type.
#define PNS_TILE_LIST(X, QT, HT) \
    X(QT, HT, 64, 1)             \
    X(QT, HT, 64, 2)             \
    X(QT, HT, 64, 4)             \
    X(QT, HT, 128, 1)            \
    X(QT, HT, 128, 2)            \
    X(QT, HT, 128, 4)            \
    X(QT, HT, 256, 1)            \
    X(QT, HT, 256, 2)            \
    X(QT, HT, 256, 4)            \
    X(QT, HT, 256, 8)            \
    X(QT, HT, 512, 2)            \
    X(QT, HT, 512, 4)            \
    X(QT, HT, 1024, 2)           \
    X(QT, HT, 1024, 4)

// 64 fields per lane: compiled for 32-bit fields only (int16 and int32
// coefficients); N up to 16384 in four waves, two chains per compute unit.
#define PNS_TILE_LIST_WIDE(X, QT, HT) X(QT, HT, 256, 16)

// One tile of the dispatch: `probe` only asks whether the tile exists.
#define PNS_DISPATCH_TILE(QT, HT, B, GG)                                                                     \
    if (block == B && groups == GG) {                                                                       \
        if (probe) return hipSuccess;                                                                       \
        if (flav == FLAV_ALL)                                                                               \
            return instr ? launch_one<QT, HT, B, GG, FLAV_ALL, true>(grid, dyn, st, a)                      \
                         : launch_one<QT, HT, B, GG, FLAV_ALL, false>(grid, dyn, st, a);                    \
        if (flav == FLAV_WINDOW)                                                                            \
            return instr ? launch_one<QT, HT, B, GG, FLAV_WINDOW, true>(grid, dyn, st, a)                   \
                         : launch_one<QT, HT, B, GG, FLAV_WINDOW, false>(grid, dyn, st, a);                 \
        if (flav == FLAV_DRAWN)                                                                             \
            return instr ? launch_one<QT, HT, B, GG, FLAV_DRAWN, true>(grid, dyn, st, a)                    \
                         : launch_one<QT, HT, B, GG, FLAV_DRAWN, false>(grid, dyn, st, a);                  \
        if (flav == FLAV_WINDOW_C)                                                                          \
            return instr ? launch_one<QT, HT, B, GG, FLAV_WINDOW_C, true>(grid, dyn, st, a)                 \
                         : launch_one<QT, HT, B, GG, FLAV_WINDOW_C, false>(grid, dyn, st, a);               \
        if (flav == FLAV_WINDOW_C2) {                                                                       \
            if constexpr (GG >= 2)                                                                          \
                return instr ? launch_one<QT, HT, B, GG, FLAV_WINDOW_C2, true>(grid, dyn, st, a)            \
                             : launch_one<QT, HT, B, GG, FLAV_WINDOW_C2, false>(grid, dyn, st, a);          \
        }                                                                                                   \
        return hipErrorInvalidConfiguration;                                                                \
    }

}  // namespace step
}  // namespace pns
