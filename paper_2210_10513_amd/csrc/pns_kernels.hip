// HIP kernels of the Partial Neighbor Search sampler for gfx950 (MI355X).
//
// One workgroup runs one chain.  The chain's N bits are spread over the
// workgroup in groups of four consecutive bits per lane:
//     field f = (g * BLOCK + tid) * 4 + v,   g < G, v < 4,
// so group g covers the contiguous bit range [g*BLOCK*4, (g+1)*BLOCK*4) and a
// row of the coefficient matrix is read with one 8- or 16-byte load per lane
// and group, fully coalesced.  Local fields, bits and the diagonal stay in
// registers for the whole launch (persistent form); only the row of the
// flipped bit comes from memory each step.
//
// Per step (loop body of Alg 2 / Alg 3 / Alg 6):
//   subset  : all bits (RF), systematic window (Unbiased-sys), random n-subset
//             (Basic every step, Unbiased-rand per block) drawn in LDS;
//   weights : dE_j = (1-2x_j)(Q_jj + s h_j), w_j = exp(min(0, -beta dE_j));
//   reduce  : per-lane sums -> wave inclusive scans -> one LDS exchange ->
//             every wave scans the (group, wave) segment sums identically;
//   p, M    : p = S / n, M = 1 + floor(log U1 / log1p(-p)) in FP64;
//   budget  : Unbiased: stay with M = L when M > L, else L -= M (Alg 6);
//   select  : inverse CDF (App. C) over the subset in increasing bit order,
//             resolved segment -> lane -> bit, published through LDS;
//   update  : flip, E += dE_c, h_j += +-A[c][j] from one coalesced row read.
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "pns_internal.h"

namespace pns {
namespace {

constexpr uint32_t kStreamStep = 0u;
constexpr uint32_t kStreamInit = 0x20000000u;
constexpr uint32_t kStreamSubset = 0x40000000u;
constexpr int kModeRF = 0, kModeBasic = 1, kModeSys = 2, kModeRand = 3;

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

__device__ __forceinline__ double wave_scan_incl(double v, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
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

// ---- four consecutive matrix / state elements ----
template <typename T>
struct Four {
    T v[4];
};

__device__ __forceinline__ Four<int32_t> load_row4(const int16_t* p)
{
    const uint2 r = *reinterpret_cast<const uint2*>(p);
    Four<int32_t> o;
    o.v[0] = (int32_t)(int16_t)(r.x & 0xFFFFu);
    o.v[1] = (int32_t)(int16_t)(r.x >> 16);
    o.v[2] = (int32_t)(int16_t)(r.y & 0xFFFFu);
    o.v[3] = (int32_t)(int16_t)(r.y >> 16);
    return o;
}
__device__ __forceinline__ Four<int32_t> load_row4(const int32_t* p)
{
    const int4 r = *reinterpret_cast<const int4*>(p);
    return {{r.x, r.y, r.z, r.w}};
}
__device__ __forceinline__ Four<float> load_row4(const float* p)
{
    const float4 r = *reinterpret_cast<const float4*>(p);
    return {{r.x, r.y, r.z, r.w}};
}

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

// Matrix element type -> widened type used in arithmetic.
template <typename QT>
struct Wide {
    using T = int32_t;
};
template <>
struct Wide<float> {
    using T = float;
};

// Energy difference of flipping a bit whose value is xbit.
template <typename HT>
__device__ __forceinline__ double delta_e(int32_t d, HT h, int s, uint32_t xbit, int64_t* dEi)
{
    int64_t e = (int64_t)d + (int64_t)s * (int64_t)h;
    if (xbit) e = -e;
    *dEi = e;
    return (double)e;
}
__device__ __forceinline__ double delta_e(float d, double h, int s, uint32_t xbit, int64_t* dEi)
{
    double e = (double)d + (double)s * h;
    if (xbit) e = -e;
    *dEi = __double_as_longlong(e);
    return e;
}

template <typename HT>
__device__ __forceinline__ void add_energy(int64_t* Ebits, int64_t dE)
{
    *Ebits += dE;
}
template <>
__device__ __forceinline__ void add_energy<double>(int64_t* Ebits, int64_t dE)
{
    *Ebits = __double_as_longlong(__longlong_as_double(*Ebits) + __longlong_as_double(dE));
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

template <typename QT, typename HT, int BLOCK, int G>
__global__ __launch_bounds__(BLOCK) void step_kernel(const StepArgs a)
{
    using QW = typename Wide<QT>::T;
    constexpr int F = 4 * G;
    constexpr int W = BLOCK / 64;
    constexpr int NSEG = G * W;
    static_assert(NSEG <= 64, "segment scan needs at most 64 segments");
    static_assert(F <= 32, "bit mask is 32 bits");

    extern __shared__ uint32_t own[];  // random-subset table, pitch entries
    __shared__ double seg_sum[NSEG];
    __shared__ double mx_part[W];
    __shared__ uint64_t masks[W];
    __shared__ int64_t sel[2];

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int chain = a.chain_list ? a.chain_list[blockIdx.x] : a.chain_first + (int)blockIdx.x;
    const Problem P = a.problems[a.chain_problem[chain]];
    const int32_t N = P.N;
    const int64_t pitch = P.pitch;
    const int mode = a.mode;
    const bool unbiased = mode == kModeSys || mode == kModeRand;
    const int32_t n = mode == kModeRF ? N : P.n;
    const bool full = n >= N;
    const int s = P.s;
    const int64_t off = a.foff[chain];
    const double beta = a.beta[chain];
    const uint32_t cid = a.chain_id[chain];
    const uint64_t seed = a.seed;

    // ---- load the chain state into registers ----
    HT h[F];
    QW dg[F];
    uint32_t xb = 0;
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
                dg[g * 4 + v] = dv.v[v];
                xb |= ((xw >> (8 * v)) & 1u) << (g * 4 + v);
            }
        } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                h[g * 4 + v] = (HT)0;
                dg[g * 4 + v] = (QW)0;
            }
        }
    }
    int64_t k = a.step[chain];
    const int64_t kend = k + a.steps;
    int64_t Ebits = a.E[chain];
    int64_t L = a.L[chain];
    int64_t sub = a.sub[chain];
    int32_t last_action = a.last_action[chain];
    int64_t last_M = a.last_M[chain];
    int64_t last_E = a.last_E[chain];
    int64_t c_steps = 0, c_flips = 0, c_stays = 0, c_sat = 0, c_bad = 0;
    double c_sumM = 0.0;
    int32_t snap_n = a.snap_every > 0 ? a.snap_count[chain] : 0;
    uint32_t pos_n = 0;
    int64_t sys_start = unbiased && mode == kModeSys ? (int64_t)(((sub % P.num_sets) * (int64_t)n) % N) : 0;

    if (mode == kModeRand && !full) {
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
            __syncthreads();
        }
    }

    for (; k < kend; ++k) {
        if (mode == kModeBasic && !full) pos_n = draw_subset<BLOCK, G>(own, masks, tid, pitch, N, n, seed, cid, k);

        // membership of this lane's fields in the step's subset
        uint32_t mem = 0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t f = ((int64_t)g * BLOCK + tid) * 4 + v;
                bool in = f < N;
                if (in && !full) {
                    if (mode == kModeSys) {
                        int64_t d = f - sys_start;
                        if (d < 0) d += N;
                        in = d < n;
                    } else if (mode == kModeBasic || mode == kModeRand) {
                        in = own[f] <= pos_n;
                    }
                }
                mem |= (uint32_t)in << (g * 4 + v);
            }
        }

        // the step's two uniforms
        const Words o = philox(cid, (uint32_t)k, (uint32_t)((uint64_t)k >> 32), kStreamStep, seed);
        const double U1 = (double)(((((uint64_t)o.w0 << 32) | o.w1) >> 11) + 1u) * 0x1p-53;
        const double U2 = (double)((((uint64_t)o.w2 << 32) | o.w3) >> 11) * 0x1p-53;

        // acceptance weights of the subset
        double w[F];
        double ls[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            ls[g] = 0.0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = g * 4 + v;
                double wi = 0.0;
                if ((mem >> i) & 1u) {
                    int64_t dEi;
                    const double dE = delta_e(dg[i], h[i], s, (xb >> i) & 1u, &dEi);
                    double l = -beta * dE;
                    l = l < 0.0 ? l : 0.0;
                    wi = exp(l);
                }
                w[i] = wi;
                ls[g] += wi;
            }
        }
        double inc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) inc[g] = wave_scan_incl(ls[g], lane);
        if (lane == 63) {
#pragma unroll
            for (int g = 0; g < G; ++g) seg_sum[g * W + wave] = inc[g];
        }
        __syncthreads();
        double sv = lane < NSEG ? seg_sum[lane] : 0.0;
        double sinc = wave_scan_incl(sv, lane);
        double S = __shfl(sinc, NSEG - 1, 64);
        double p;
        if (S < 0x1p-1000) {
            // Every weight underflowed: rescale by the largest log-weight.
            double lm = -INFINITY;
#pragma unroll
            for (int i = 0; i < F; ++i) {
                if ((mem >> i) & 1u) {
                    int64_t dEi;
                    const double dE = delta_e(dg[i], h[i], s, (xb >> i) & 1u, &dEi);
                    double l = -beta * dE;
                    l = l < 0.0 ? l : 0.0;
                    lm = fmax(lm, l);
                }
            }
            lm = wave_max(lm);
            if (lane == 0) mx_part[wave] = lm;
            __syncthreads();
            double mx = -INFINITY;
            for (int ww = 0; ww < W; ++ww) mx = fmax(mx, mx_part[ww]);
#pragma unroll
            for (int g = 0; g < G; ++g) {
                ls[g] = 0.0;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = g * 4 + v;
                    double wi = 0.0;
                    if ((mem >> i) & 1u) {
                        int64_t dEi;
                        const double dE = delta_e(dg[i], h[i], s, (xb >> i) & 1u, &dEi);
                        double l = -beta * dE;
                        l = l < 0.0 ? l : 0.0;
                        wi = exp(l - mx);
                    }
                    w[i] = wi;
                    ls[g] += wi;
                }
            }
#pragma unroll
            for (int g = 0; g < G; ++g) inc[g] = wave_scan_incl(ls[g], lane);
            if (lane == 63) {
#pragma unroll
                for (int g = 0; g < G; ++g) seg_sum[g * W + wave] = inc[g];
            }
            __syncthreads();
            sv = lane < NSEG ? seg_sum[lane] : 0.0;
            sinc = wave_scan_incl(sv, lane);
            S = __shfl(sinc, NSEG - 1, 64);
            p = exp(mx) * S / (double)n;
        } else {
            p = S / (double)n;
        }

        // multiplicity M = 1 + G, G ~ Geometric(p) counting failures
        double q;
        if (p >= 1.0) q = 0.0;
        else if (p <= 0.0) q = INFINITY;
        else q = log(U1) / log1p(-p);
        int64_t m;
        bool sat = false;
        if (!(q < 0x1p63)) {
            m = INT64_MAX;
            sat = true;
        } else {
            m = (int64_t)floor(q) + 1;
        }

        const int64_t Erec = Ebits;
        int32_t action;
        int64_t M;
        // state index of the record for the histograms (N <= 24: lanes 0..5 of wave 0)
        uint32_t rec_idx = 0;
        if (a.hist_w != nullptr && wave == 0) rec_idx = wave_or(tid < 8 ? ((xb & 0xFu) << (4 * tid)) : 0u);
        // snapshot of the record's state
        const bool snap = a.snap_every > 0 && ((k + 1) % a.snap_every) == 0;
        if (snap) {
            const int32_t slot = snap_n % a.snap_cap;
            uint8_t* sx = a.snap_x + ((int64_t)chain * a.snap_cap + slot) * a.snap_pitch;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int64_t fb = ((int64_t)g * BLOCK + tid) * 4;
                if (fb < a.snap_pitch) {
                    uint32_t wv = 0;
#pragma unroll
                    for (int v = 0; v < 4; ++v) wv |= ((xb >> (g * 4 + v)) & 1u) << (8 * v);
                    *reinterpret_cast<uint32_t*>(sx + fb) = wv;
                }
            }
        }

        if (unbiased && q >= (double)L) {
            // Alg 6: not enough remaining original samples; stay L times and
            // switch to the next partial neighbor set.
            M = L;
            action = -1;
            L = P.L0;
            ++sub;
            ++c_stays;
            if (mode == kModeSys) {
                sys_start = (int64_t)(((sub % P.num_sets) * (int64_t)n) % N);
                __syncthreads();  // seg_sum is rewritten next step
            } else if (!full) {
                pos_n = draw_subset<BLOCK, G>(own, masks, tid, pitch, N, n, seed, cid, k + 1);
            } else {
                __syncthreads();
            }
        } else {
            M = m;
            if (unbiased) L -= m;
            c_sat += sat ? 1 : 0;
            const double t = U2 * S;
            const bool pos_seg = lane < NSEG && sv > 0.0;
            const uint64_t bseg = __ballot(pos_seg && sinc > t);
            const uint64_t bpos = __ballot(pos_seg);
            int jstar = bseg ? __builtin_ctzll(bseg) : (bpos ? 63 - __builtin_clzll(bpos) : 0);
            jstar = jstar < NSEG ? jstar : NSEG - 1;
            const double prev_seg = __shfl(sinc, jstar > 0 ? jstar - 1 : 0, 64);
            const double base = jstar > 0 ? prev_seg : 0.0;
            const int gstar = jstar / W, wstar = jstar % W;
            if (wave == wstar) {
                double my_inc = 0.0, my_ls = 0.0;
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    if (g == gstar) {
                        my_inc = inc[g];
                        my_ls = ls[g];
                    }
                }
                const double Gl = base + my_inc;
                const uint64_t bl = __ballot(my_ls > 0.0 && Gl > t);
                const uint64_t blp = __ballot(my_ls > 0.0);
                const int lstar = bl ? __builtin_ctzll(bl) : (blp ? 63 - __builtin_clzll(blp) : 0);
                const double prev_l = __shfl(my_inc, lstar > 0 ? lstar - 1 : 0, 64);
                if (lane == lstar) {
                    double run = lstar > 0 ? base + prev_l : base;
                    int vstar = -1, vlast = -1;
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        if (g == gstar) {
#pragma unroll
                            for (int v = 0; v < 4; ++v) {
                                const double wv = w[g * 4 + v];
                                if (wv > 0.0) {
                                    vlast = v;
                                    run += wv;
                                    if (vstar < 0 && run > t) vstar = v;
                                }
                            }
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
                    int64_t dEc = 0;
#pragma unroll
                    for (int ii = 0; ii < F; ++ii) {
                        if (ii == i) delta_e(dg[ii], h[ii], s, (xb >> ii) & 1u, &dEc);
                    }
                    int64_t c = ((int64_t)gstar * BLOCK + tid) * 4 + vstar;
                    if (c >= N) {
                        c = 0;
                        bad = 1;
                    }
                    sel[0] = c | ((int64_t)((xb >> i) & 1u) << 40) | (bad << 41);
                    sel[1] = dEc;
                }
            }
            __syncthreads();
            const int64_t sv0 = sel[0];
            const int64_t dEc = sel[1];
            const int32_t c = (int32_t)(sv0 & 0xFFFFFFFFll);
            const bool xc = (sv0 >> 40) & 1;
            c_bad += (sv0 >> 41) & 1;
            action = c;
            add_energy<HT>(&Ebits, dEc);
            // owner flips the bit
            const int cl = (c >> 2) % BLOCK;
            const int cg = (c >> 2) / BLOCK;
            if (tid == cl) xb ^= 1u << (cg * 4 + (c & 3));
            // field update from row c
            const QT* row = reinterpret_cast<const QT*>(P.A) + (int64_t)c * pitch;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const int64_t fb = ((int64_t)g * BLOCK + tid) * 4;
                if (fb < pitch) {
                    const auto r = load_row4(row + fb);
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        if (xc) h[g * 4 + v] -= (HT)r.v[v];
                        else h[g * 4 + v] += (HT)r.v[v];
                    }
                }
            }
            ++c_flips;
        }

        // record k = (state before the step, M)
        if (snap) ++snap_n;
        ++c_steps;
        c_sumM += (double)M;
        last_action = action;
        last_M = M;
        last_E = Erec;
        if (tid == 0) {
            if (a.log_cap > 0) {
                const int64_t slot = (int64_t)chain * a.log_cap + (k % a.log_cap);
                a.log_action[slot] = action;
                a.log_M[slot] = M;
                a.log_E[slot] = Erec;
                a.log_p[slot] = p;
            }
            if (a.hist_w != nullptr) {
                atomicAdd(&a.hist_w[rec_idx], (unsigned long long)M);
                atomicAdd(&a.hist_v[rec_idx], 1ull);
            }
            if (snap) {
                const int32_t slot = snap_n % a.snap_cap;
                a.snap_M[(int64_t)chain * a.snap_cap + slot] = M;
                a.snap_E[(int64_t)chain * a.snap_cap + slot] = Erec;
            }
        }
    }

    // ---- store the chain state ----
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t fb = ((int64_t)g * BLOCK + tid) * 4;
        if (fb < pitch) {
            HT hv[4];
            uint32_t xw = 0, mw = 0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                hv[v] = h[g * 4 + v];
                xw |= ((xb >> (g * 4 + v)) & 1u) << (8 * v);
                if (mode == kModeRand && !full) mw |= (uint32_t)(own[fb + v] <= pos_n) << (8 * v);
            }
            store4(hbase + fb, hv);
            *reinterpret_cast<uint32_t*>(a.x + off + fb) = xw;
            if (mode == kModeRand && !full) *reinterpret_cast<uint32_t*>(a.rmem + off + fb) = mw;
        }
    }
    if (tid == 0) {
        a.step[chain] = kend;
        a.E[chain] = Ebits;
        a.L[chain] = L;
        a.sub[chain] = sub;
        a.last_action[chain] = last_action;
        a.last_M[chain] = last_M;
        a.last_E[chain] = last_E;
        if (a.snap_every > 0) a.snap_count[chain] = snap_n;
        int64_t* cn = a.counters + (int64_t)chain * 6;
        cn[0] += c_steps;
        cn[1] += c_flips;
        cn[2] += c_stays;
        cn[3] += c_sat;
        cn[4] = __double_as_longlong(__longlong_as_double(cn[4]) + c_sumM);
        cn[5] += c_bad;
    }
}

// ---------------------------------------------------------------------------
// a0: initial bits, fields and energies.
// ---------------------------------------------------------------------------

// Bernoulli(1/2) bits: bit j of chain c from stream 0x20000000 | (j/128),
// word (j/32) mod 4, bit j mod 32, step 0.
__global__ void init_random_bits_kernel(InitArgs a)
{
    const int chain = blockIdx.y;
    const Problem P = a.problems[a.chain_problem[chain]];
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= P.pitch) return;
    uint8_t bit = 0;
    if (j < P.N) {
        const Words o = philox(a.chain_id[chain], 0u, 0u, kStreamInit | (uint32_t)(j >> 7), a.seed);
        const uint32_t wsel[4] = {o.w0, o.w1, o.w2, o.w3};
        bit = (uint8_t)((wsel[(j >> 5) & 3] >> (j & 31)) & 1u);
    }
    a.x[a.foff[chain] + j] = bit;
}

// h[c][f] = sum_j x[c][j] A[j][f] for a tile of 16 chains of one problem and
// 256 fields; each row segment of A read is reused by the 16 chains.
template <typename QT, typename HT>
__global__ __launch_bounds__(256) void init_fields_kernel(InitArgs a, int32_t cbeg, int32_t cend)
{
    constexpr int CT = 16;
    __shared__ uint8_t xs[CT][256];
    const int tid = threadIdx.x;
    const int c0 = cbeg + blockIdx.y * CT;
    const Problem P = a.problems[a.chain_problem[c0]];
    const int64_t f = (int64_t)blockIdx.x * 256 + tid;
    HT acc[CT];
#pragma unroll
    for (int i = 0; i < CT; ++i) acc[i] = (HT)0;
    const QT* A = reinterpret_cast<const QT*>(P.A);
    for (int64_t j0 = 0; j0 < P.N; j0 += 256) {
        __syncthreads();
        for (int i = 0; i < CT; ++i) {
            const int c = c0 + i;
            const int64_t j = j0 + tid;
            xs[i][tid] = (c < cend && j < P.N) ? a.x[a.foff[c] + j] : (uint8_t)0;
        }
        __syncthreads();
        if (f < P.pitch) {
            const int64_t jn = P.N - j0 < 256 ? P.N - j0 : 256;
            for (int64_t jj = 0; jj < jn; ++jj) {
                const HT v = (HT)A[(j0 + jj) * P.pitch + f];
#pragma unroll
                for (int i = 0; i < CT; ++i)
                    if (xs[i][jj]) acc[i] += v;
            }
        }
    }
    if (f < P.pitch) {
#pragma unroll
        for (int i = 0; i < CT; ++i) {
            const int c = c0 + i;
            if (c < cend) reinterpret_cast<HT*>(a.h)[a.foff[c] + f] = acc[i];
        }
    }
}

// E = sum_f x_f (Q_ff + (s/2) h_f), one workgroup of 256 per chain.
template <typename QT, typename HT>
__global__ __launch_bounds__(256) void init_energy_kernel(InitArgs a)
{
    using QW = typename Wide<QT>::T;
    const int chain = blockIdx.x;
    const Problem P = a.problems[a.chain_problem[chain]];
    const HT* h = reinterpret_cast<const HT*>(a.h) + a.foff[chain];
    const QW* d = reinterpret_cast<const QW*>(P.diag);
    const uint8_t* x = a.x + a.foff[chain];
    __shared__ double sd[256];
    __shared__ long long si[256];
    double accd = 0.0;
    long long acci = 0;
    for (int64_t f = threadIdx.x; f < P.N; f += 256) {
        if (!x[f]) continue;
        if constexpr (std::is_floating_point<HT>::value) {
            accd += (double)d[f] + 0.5 * (double)P.s * (double)h[f];
        } else {
            acci += 2 * (long long)d[f] + (long long)P.s * (long long)h[f];
        }
    }
    sd[threadIdx.x] = accd;
    si[threadIdx.x] = acci;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            sd[threadIdx.x] += sd[threadIdx.x + st];
            si[threadIdx.x] += si[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int64_t e;
        if constexpr (std::is_floating_point<HT>::value) e = __double_as_longlong(sd[0]);
        else e = si[0] / 2;
        a.E[chain] = e;
        a.last_E[chain] = e;
    }
}

__global__ void fill64_kernel(int64_t* p, int64_t count, int64_t value)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

template <typename QT, typename HT, int BLOCK, int G>
hipError_t launch_one(int32_t grid, size_t dyn, hipStream_t st, const StepArgs& a)
{
    hipLaunchKernelGGL((step_kernel<QT, HT, BLOCK, G>), dim3(grid), dim3(BLOCK), dyn, st, a);
    return hipGetLastError();
}

#define PNS_TILES(X, QT, HT) \
    X(QT, HT, 64, 1)         \
    X(QT, HT, 64, 4)         \
    X(QT, HT, 128, 4)        \
    X(QT, HT, 256, 1)        \
    X(QT, HT, 256, 2)        \
    X(QT, HT, 256, 4)        \
    X(QT, HT, 512, 2)        \
    X(QT, HT, 512, 4)        \
    X(QT, HT, 1024, 4)

#define PNS_TYPES(X)                 \
    PNS_TILES(X, int16_t, int32_t)   \
    PNS_TILES(X, int32_t, int32_t)   \
    PNS_TILES(X, int32_t, int64_t)   \
    PNS_TILES(X, float, double)

template <typename T>
struct TypeId;
template <>
struct TypeId<int16_t> {
    static constexpr int q = Q_I16;
};
template <>
struct TypeId<int32_t> {
    static constexpr int q = Q_I32;
    static constexpr int h = H_I32;
};
template <>
struct TypeId<int64_t> {
    static constexpr int h = H_I64;
};
template <>
struct TypeId<float> {
    static constexpr int q = Q_F32;
};
template <>
struct TypeId<double> {
    static constexpr int h = H_F64;
};

}  // namespace

hipError_t launch_steps(int32_t qtype, int32_t htype, int32_t block, int32_t groups, int32_t grid, size_t dyn_lds,
                        hipStream_t stream, const StepArgs& args)
{
#define PNS_DISPATCH(QT, HT, B, G)                                                                      \
    if (qtype == TypeId<QT>::q && htype == TypeId<HT>::h && block == B && groups == G)                   \
        return launch_one<QT, HT, B, G>(grid, dyn_lds, stream, args);
    PNS_TYPES(PNS_DISPATCH)
#undef PNS_DISPATCH
    return hipErrorInvalidConfiguration;
}

bool have_tile(int32_t qtype, int32_t htype, int32_t block, int32_t groups)
{
#define PNS_HAVE(QT, HT, B, G) \
    if (qtype == TypeId<QT>::q && htype == TypeId<HT>::h && block == B && groups == G) return true;
    PNS_TYPES(PNS_HAVE)
#undef PNS_HAVE
    return false;
}

template <typename QT, typename HT>
static hipError_t init_typed(int32_t max_pitch, hipStream_t st, const InitArgs& a, const int32_t* host_chain_problem)
{
    if (a.init == 1) {
        hipLaunchKernelGGL(init_random_bits_kernel, dim3((max_pitch + 255) / 256, a.num_chains), dim3(256), 0, st, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // fields: one launch per run of consecutive chains of the same problem
    int32_t c = 0;
    while (c < a.num_chains) {
        int32_t e = c + 1;
        while (e < a.num_chains && host_chain_problem[e] == host_chain_problem[c]) ++e;
        for (int32_t t = c; t < e; t += 16 * 65535) {
            const int32_t tend = t + 16 * 65535 < e ? t + 16 * 65535 : e;
            hipLaunchKernelGGL((init_fields_kernel<QT, HT>), dim3((max_pitch + 255) / 256, (tend - t + 15) / 16),
                               dim3(256), 0, st, a, t, tend);
            hipError_t er = hipGetLastError();
            if (er != hipSuccess) return er;
        }
        c = e;
    }
    hipLaunchKernelGGL((init_energy_kernel<QT, HT>), dim3(a.num_chains), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_init_with_map(int32_t qtype, int32_t htype, int32_t max_pitch, hipStream_t stream,
                                const InitArgs& args, const int32_t* host_chain_problem)
{
    if (qtype == Q_I16 && htype == H_I32) return init_typed<int16_t, int32_t>(max_pitch, stream, args, host_chain_problem);
    if (qtype == Q_I32 && htype == H_I32) return init_typed<int32_t, int32_t>(max_pitch, stream, args, host_chain_problem);
    if (qtype == Q_I32 && htype == H_I64) return init_typed<int32_t, int64_t>(max_pitch, stream, args, host_chain_problem);
    if (qtype == Q_F32 && htype == H_F64) return init_typed<float, double>(max_pitch, stream, args, host_chain_problem);
    return hipErrorInvalidConfiguration;
}

hipError_t launch_fill64(void* p, int64_t count, int64_t value, hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill64_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream,
                       reinterpret_cast<int64_t*>(p), count, value);
    return hipGetLastError();
}

}  // namespace pns
