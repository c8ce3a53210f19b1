// Kernels of the differentiation path.
//
// * Multiplicity-weighted second moments G = X^T diag(m) X of jump-chain
//   records (x_k, m_k): the estimate of E_pi[x x^T] (times sum_k m_k) whose
//   product with -beta is grad_Q log Z.  Dense contraction over the records
//   on the bf16 matrix cores (v_mfma_f32_16x16x32_bf16) with FP32
//   accumulation: x is 0/1 (exact in bf16) and each m_k is split into up to
//   three bf16 pieces that sum to it (exact for m_k < 2^24), so every product
//   is exact and an FP32 partial sum is exact while it stays below 2^24; the
//   records are cut into chunks short enough for that, and chunk results are
//   added into FP64.
// * log Z = log sum_x exp(-beta x^T Q x) by enumeration of all 2^N states
//   (N <= 32) in Gray-code order with an incremental energy, FP64
//   log-sum-exp.
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "pns_internal.h"

namespace pns {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Round-to-nearest-even of a float to bf16 (bit pattern).
__device__ __forceinline__ uint16_t bf16_bits(float f)
{
    const uint32_t u = __float_as_uint(f);
    const uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(r >> 16);
}

__device__ __forceinline__ float bf16_value(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Pieces of each weight (m = p0 + p1 + p2, each a bf16) and the exact sum
// and maximum of the weights.  Pieces are stored [3][kpad], zero past K.
// Grid-stride loop; one atomic per workgroup for the sum and the maximum.
__global__ __launch_bounds__(256) void moments_prep_kernel(const int64_t* m, int64_t K, int64_t kpad, uint16_t* pieces,
                                                           unsigned long long* sum_m, unsigned long long* max_m)
{
    __shared__ unsigned long long red[2][4];
    const int64_t n = kpad > K ? kpad : K;
    unsigned long long sv = 0, mv = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        int64_t mk = 0;
        if (k < K) mk = m[k] > 0 ? m[k] : 0;
        if (k < kpad) {
            // m < 2^24 is exact in float; the pieces then sum to it exactly
            float r = (float)mk;
            uint16_t b[3];
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                b[s] = bf16_bits(r);
                r = r - bf16_value(b[s]);
            }
#pragma unroll
            for (int s = 0; s < 3; ++s) pieces[s * kpad + k] = b[s];
        }
        sv += (unsigned long long)mk;
        mv = mv > (unsigned long long)mk ? mv : (unsigned long long)mk;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        sv += __shfl_xor(sv, d, 64);
        const unsigned long long o = __shfl_xor(mv, d, 64);
        mv = mv > o ? mv : o;
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = sv;
        red[1][threadIdx.x >> 6] = mv;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long ts = 0, tm = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            ts += red[0][w];
            tm = tm > red[1][w] ? tm : red[1][w];
        }
        atomicAdd(sum_m, ts);
        atomicMax(max_m, tm);
    }
}

// Real (FP64) weights, e.g. the expected multiplicities 1 / p of Thm 3 (5).
// First the largest |w_k| (finite ones; bit patterns of non-negative doubles
// order like the numbers), so that the weights can be scaled by a power of
// two into [-2, 2] before they are rounded to FP32 (relative 2^-24) and split
// exactly into three bf16 pieces; G is scaled back at the end.  Non-finite
// weights count as 0 in G and in the sum.
__global__ __launch_bounds__(256) void moments_absmax_kernel(const double* w, int64_t K, unsigned long long* maxbits)
{
    __shared__ unsigned long long red[4];
    unsigned long long b = 0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < K; k += (int64_t)gridDim.x * blockDim.x) {
        const double v = isfinite(w[k]) ? fabs(w[k]) : 0.0;
        const unsigned long long vb = (unsigned long long)__double_as_longlong(v);
        b = b > vb ? b : vb;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        const unsigned long long o = __shfl_xor(b, d, 64);
        b = b > o ? b : o;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = b;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t = t > red[i] ? t : red[i];
        atomicMax(maxbits, t);
    }
}

__device__ __forceinline__ int weight_exponent(const unsigned long long* maxbits)
{
    const double mx = __longlong_as_double((long long)*maxbits);
    return mx > 0.0 ? ilogb(mx) : 0;
}

__global__ __launch_bounds__(256) void moments_prep_f64_kernel(const double* w, int64_t K, int64_t kpad,
                                                               uint16_t* pieces, double* sum_w,
                                                               const unsigned long long* maxbits)
{
    __shared__ double red[4];
    const int64_t n = kpad > K ? kpad : K;
    const int e = weight_exponent(maxbits);
    double sv = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        double wk = 0.0;
        if (k < K && isfinite(w[k])) wk = w[k];
        if (k < kpad) {
            float r = (float)ldexp(wk, -e);
            uint16_t b[3];
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                b[s] = bf16_bits(r);
                r = r - bf16_value(b[s]);
            }
#pragma unroll
            for (int s = 0; s < 3; ++s) pieces[s * kpad + k] = b[s];
        }
        sv += wk;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) sv += __shfl_xor(sv, d, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sv;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
        atomicAdd(sum_w, t);
    }
}

// G *= 2^e, the scale the weights were divided by.
__global__ void moments_unscale_kernel(double* G, int64_t n, const unsigned long long* maxbits)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) G[i] = ldexp(G[i], weight_exponent(maxbits));
}

constexpr int kTile = 64;  // output tile (rows and columns) per wave

// Upper-triangle tile t (row-major over ti <= tj) -> (ti, tj).
__device__ __forceinline__ void upper_tile(int t, int nt, int* ti, int* tj)
{
    int r = 0, rem = t;
    while (rem >= nt - r) {
        rem -= nt - r;
        ++r;
    }
    *ti = r;
    *tj = r + rem;
}

// Records packed column by column: word (w, i) holds bit r = X[32 w + r][i]
// (zero past K), so the eight records a lane feeds to one MFMA step are one
// byte of one word.  One thread per (column, word).
__global__ void pack_bits_kernel(const uint8_t* __restrict__ X, int64_t ldx, int64_t K, int32_t N, int32_t npad,
                                 int64_t words, uint32_t* __restrict__ Xb)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t w = t / npad;
    const int32_t i = (int32_t)(t % npad);
    if (w >= words) return;
    uint32_t v = 0;
    if (i < N) {
        const int64_t k0 = w * 32;
        const int rmax = K - k0 < 32 ? (int)(K - k0) : 32;
        for (int r = 0; r < rmax; ++r) v |= (uint32_t)(X[(k0 + r) * ldx + i] != 0) << r;
    }
    Xb[w * npad + i] = v;
}

// The same packing four columns per thread: one 32-bit load per record
// (rows 4-byte aligned: ldx % 4 == 0 and X aligned), npad % 4 == 0.
__global__ void pack_bits4_kernel(const uint8_t* __restrict__ X, int64_t ldx, int64_t K, int32_t N, int32_t npad,
                                  int64_t words, uint32_t* __restrict__ Xb)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t q = npad / 4;
    const int64_t w = t / q;
    const int32_t i0 = (int32_t)(t % q) * 4;
    if (w >= words) return;
    uint32_t v0 = 0, v1 = 0, v2 = 0, v3 = 0;
    if (i0 < N) {
        const int64_t k0 = w * 32;
        const int rmax = K - k0 < 32 ? (int)(K - k0) : 32;
        // columns at or past N (inside the row's pitch, or past it when
        // N = ldx) are masked below; a load never starts past the row
        const bool full = i0 + 4 <= ldx;
        for (int r = 0; r < rmax; ++r) {
            const uint8_t* row = X + (k0 + r) * ldx;
            uint32_t b;
            if (full) {
                b = *reinterpret_cast<const uint32_t*>(row + i0);
            } else {
                b = 0;
                for (int c = 0; c < 4 && i0 + c < ldx; ++c) b |= (uint32_t)row[i0 + c] << (8 * c);
            }
            v0 |= (uint32_t)((b & 0xFFu) != 0) << r;
            v1 |= (uint32_t)((b & 0xFF00u) != 0) << r;
            v2 |= (uint32_t)((b & 0xFF0000u) != 0) << r;
            v3 |= (uint32_t)((b & 0xFF000000u) != 0) << r;
        }
        if (i0 + 1 >= N) v1 = 0;
        if (i0 + 2 >= N) v2 = 0;
        if (i0 + 3 >= N) v3 = 0;
    }
    uint4 out = make_uint4(v0, v1, v2, v3);
    *reinterpret_cast<uint4*>(Xb + w * npad + i0) = out;
}

// 0xFFFF per set bit of a 2-bit field, in the matching half word.
__device__ __forceinline__ uint32_t half_mask(uint32_t two_bits)
{
    return ((two_bits & 1u) ? 0x0000FFFFu : 0u) | ((two_bits & 2u) ? 0xFFFF0000u : 0u);
}

// One wave computes one 64 x 64 tile (ti, tj) of G over the records
// [32 w0, 32 w1) as 4 x 4 MFMA tiles of 16 x 16 (v_mfma_f32_16x16x32_bf16).
// Lane l supplies row (A) or column (B) l % 16 of each 16-block and the eight
// records 8 (l / 16) .. + 7 of the 32-record step (the same assignment for A
// and B, so their order inside the step does not matter); lane l receives C
// rows 4 (l / 16) + e, column l % 16.  A = diag(piece_s(m)) x, B = x.
// FP32 accumulation stays exact while flush * max(m) < 2^24: past that many
// records the accumulators are added into G with FP64 atomics; the final
// accumulators go to this wave's slot of `part` (FP32, exact integers).
__global__ __launch_bounds__(256) void moments_kernel(const uint32_t* __restrict__ Xb, int32_t npad, int64_t words,
                                                      int32_t N, const uint16_t* __restrict__ pieces, int64_t kpad,
                                                      int64_t chunk_words, int32_t tiles,
                                                      const unsigned long long* __restrict__ max_m,
                                                      float* __restrict__ part, double* __restrict__ G)
{
    const int lane = threadIdx.x & 63;
    const int64_t gw = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t chunks = (words + chunk_words - 1) / chunk_words;
    if (gw >= (int64_t)tiles * chunks) return;
    const int t = (int)(gw % tiles);
    const int64_t c = gw / tiles;
    const int nt = (N + kTile - 1) / kTile;
    int ti, tj;
    upper_tile(t, nt, &ti, &tj);
    const int i0 = ti * kTile, j0 = tj * kTile;
    const int64_t w0 = c * chunk_words;
    const int64_t w1 = w0 + chunk_words < words ? w0 + chunk_words : words;
    const unsigned long long mm = *max_m;
    int64_t flush_words = w1 - w0;
    if (mm > 0) {
        const double lim = (double)(1 << 24) / ((double)mm * 1.01) / 32.0;
        if (lim < (double)flush_words) flush_words = lim < 2.0 ? 2 : (int64_t)lim;
    }
    const int l16 = lane & 15, lg = lane >> 4;

    f32x4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};

    auto flush_atomic = [&]() {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const int j = j0 + b * 16 + l16;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int i = i0 + a * 16 + lg * 4 + e;
                    const double v = (double)acc[a][b][e];
                    if (i < N && j < N && v != 0.0) {
                        atomicAdd(&G[(int64_t)i * N + j], v);
                        if (ti != tj) atomicAdd(&G[(int64_t)j * N + i], v);
                    }
                }
                acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};
            }
    };

    const int sh = lg * 8;
    int64_t since = 0;
    for (int64_t w = w0; w < w1; ++w) {
        const uint32_t* row = Xb + w * npad;
        uint32_t ba[4], bb[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) ba[a] = (row[i0 + a * 16 + l16] >> sh) & 0xFFu;
#pragma unroll
        for (int b = 0; b < 4; ++b) bb[b] = (row[j0 + b * 16 + l16] >> sh) & 0xFFu;
        // weights of this lane's eight records, as four pairs per piece
        const int64_t kb = w * 32 + sh;
        uint4 wp[3];
        bool use[3];
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            wp[s] = *reinterpret_cast<const uint4*>(pieces + s * kpad + kb);
            const uint32_t any = (wp[s].x | wp[s].y | wp[s].z | wp[s].w) & 0x7FFF7FFFu;
            use[s] = s == 0 || __ballot(any != 0) != 0;
        }
        bf16x8 bop[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            uint4 v;
            v.x = half_mask(bb[b]) & 0x3F803F80u;
            v.y = half_mask(bb[b] >> 2) & 0x3F803F80u;
            v.z = half_mask(bb[b] >> 4) & 0x3F803F80u;
            v.w = half_mask(bb[b] >> 6) & 0x3F803F80u;
            bop[b] = __builtin_bit_cast(bf16x8, v);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const uint32_t m0 = half_mask(ba[a]), m1 = half_mask(ba[a] >> 2), m2 = half_mask(ba[a] >> 4),
                           m3 = half_mask(ba[a] >> 6);
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                if (!use[s]) continue;
                uint4 v;
                v.x = m0 & wp[s].x;
                v.y = m1 & wp[s].y;
                v.z = m2 & wp[s].z;
                v.w = m3 & wp[s].w;
                const bf16x8 aop = __builtin_bit_cast(bf16x8, v);
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, bop[b], acc[a][b], 0, 0, 0);
            }
        }
        if (++since >= flush_words && w + 1 < w1) {
            flush_atomic();
            since = 0;
        }
    }
    // this wave's partial tile: part[c][t][64][64]
    float* dst = part + (c * tiles + t) * (int64_t)(kTile * kTile);
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int e = 0; e < 4; ++e) dst[(a * 16 + lg * 4 + e) * kTile + b * 16 + l16] = acc[a][b][e];
}

// G[i][j] += sum over chunks of the partial tiles (FP64, in chunk order).
// One thread per element of an upper-triangle tile (reads coalesced along the
// tile row); an off-diagonal tile's element also gives G[j][i].
__global__ void moments_reduce_kernel(const float* __restrict__ part, int64_t chunks, int32_t tiles, int32_t N,
                                      double* __restrict__ G)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)tiles * (kTile * kTile)) return;
    const int t = (int)(e / (kTile * kTile));
    const int off = (int)(e % (kTile * kTile));
    const int nt = (N + kTile - 1) / kTile;
    int ti, tj;
    upper_tile(t, nt, &ti, &tj);
    const int i = ti * kTile + off / kTile, j = tj * kTile + off % kTile;
    if (i >= N || j >= N) return;
    double s = 0.0;
    for (int64_t c = 0; c < chunks; ++c) s += (double)part[c * tiles * (int64_t)(kTile * kTile) + e];
    G[(int64_t)i * N + j] += s;
    if (ti != tj) G[(int64_t)j * N + i] += s;
}

// sum of the weights as FP64 into a device word.
__global__ void moments_sum_kernel(const unsigned long long* sum_m, double* out) { *out = (double)*sum_m; }

// ---- log Z by enumeration ----

template <typename T>
struct Acc {
    using type = int64_t;
};
template <>
struct Acc<float> {
    using type = double;
};

// Thread t enumerates the 2^lowbits states whose high bits are t, the low
// bits in Gray-code order (one flip per state, energy updated by dE).
// Writes the thread's (max, sum) of exp(-beta E - max) pairs, block-reduced.
template <typename QT>
__global__ __launch_bounds__(256) void logz_kernel(const QT* __restrict__ Q, int32_t N, int32_t layout, double beta,
                                                   int32_t lowbits, int64_t nthreads, double* out_max, double* out_sum)
{
    using AT = typename Acc<QT>::type;
    __shared__ AT W[32][32];
    __shared__ AT dq[32];
    __shared__ double smax[256], ssum[256];
    const int tid = threadIdx.x;
    for (int e = tid; e < N * N; e += blockDim.x) {
        const int i = e / N, j = e % N;
        AT v;
        if (i == j) {
            v = (AT)Q[i * N + i];
            dq[i] = v;
            v = (AT)0;
        } else if (layout == 0) {
            v = (AT)Q[i * N + j] + (AT)Q[j * N + i];
        } else {
            v = i < j ? (AT)Q[i * N + j] : (AT)Q[j * N + i];
        }
        W[i][j] = v;
    }
    __syncthreads();
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + tid;
    double mx = -INFINITY, sm = 0.0;
    if (t < nthreads) {
        const uint64_t hi = (uint64_t)t << lowbits;
        uint32_t x = 0;  // low bits
        AT h[32];        // h_j = sum_{i != j} W_ij x_i over the whole state
        AT E = 0;
        for (int j = 0; j < N; ++j) {
            AT acc = 0;
            for (int i = 0; i < N; ++i)
                if (i != j && ((hi >> i) & 1u)) acc += W[i][j];
            h[j] = acc;
        }
        for (int i = lowbits; i < N; ++i)
            if ((hi >> i) & 1u) E += dq[i];
        // E = sum_i d_i x_i + sum_{i<j} W_ij x_i x_j for the high bits alone
        for (int i = lowbits; i < N; ++i) {
            if (!((hi >> i) & 1u)) continue;
            for (int j = i + 1; j < N; ++j)
                if ((hi >> j) & 1u) E += W[i][j];
        }
        const uint64_t count = (uint64_t)1 << lowbits;
        for (uint64_t g = 0; g < count; ++g) {
            if (g > 0) {
                const int c = __builtin_ctzll(g);
                const bool on = (x >> c) & 1u;
                const AT dE = on ? -(dq[c] + h[c]) : (dq[c] + h[c]);
                E += dE;
                x ^= 1u << c;
                for (int j = 0; j < N; ++j)
                    if (j != c) h[j] += on ? -W[c][j] : W[c][j];
            }
            const double v = -beta * (double)E;
            if (v > mx) {
                sm = sm * exp(mx - v) + 1.0;
                mx = v;
            } else {
                sm += exp(v - mx);
            }
        }
    }
    smax[tid] = mx;
    ssum[tid] = sm;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) {
            const double m1 = smax[tid], m2 = smax[tid + st];
            const double s1 = ssum[tid], s2 = ssum[tid + st];
            const double m = fmax(m1, m2);
            smax[tid] = m;
            ssum[tid] = (m1 == -INFINITY ? 0.0 : s1 * exp(m1 - m)) + (m2 == -INFINITY ? 0.0 : s2 * exp(m2 - m));
        }
        __syncthreads();
    }
    if (tid == 0) {
        out_max[blockIdx.x] = smax[0];
        out_sum[blockIdx.x] = ssum[0];
    }
}

// Final log-sum-exp of the per-block pairs, one workgroup.
__global__ __launch_bounds__(256) void logz_finish_kernel(const double* pm, const double* ps, int32_t n, double* out)
{
    __shared__ double smax[256], ssum[256];
    const int tid = threadIdx.x;
    double mx = -INFINITY, sm = 0.0;
    for (int i = tid; i < n; i += 256) {
        const double m = fmax(mx, pm[i]);
        sm = (mx == -INFINITY ? 0.0 : sm * exp(mx - m)) + (pm[i] == -INFINITY ? 0.0 : ps[i] * exp(pm[i] - m));
        mx = m;
    }
    smax[tid] = mx;
    ssum[tid] = sm;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (tid < st) {
            const double m1 = smax[tid], m2 = smax[tid + st];
            const double m = fmax(m1, m2);
            ssum[tid] = (m1 == -INFINITY ? 0.0 : ssum[tid] * exp(m1 - m)) +
                        (m2 == -INFINITY ? 0.0 : ssum[tid + st] * exp(m2 - m));
            smax[tid] = m;
        }
        __syncthreads();
    }
    if (tid == 0) out[0] = smax[0] + log(ssum[0]);
}

}  // namespace

hipError_t launch_moments_prep(const int64_t* m, int64_t K, int64_t kpad, uint16_t* pieces, unsigned long long* sum_m,
                               unsigned long long* max_m, hipStream_t st)
{
    const int64_t n = kpad > K ? kpad : K;
    const int64_t blocks = std::min<int64_t>(256, std::max<int64_t>(1, (n + 255) / 256));
    hipLaunchKernelGGL(moments_prep_kernel, dim3((unsigned)blocks), dim3(256), 0, st, m, K, kpad, pieces, sum_m, max_m);
    return hipGetLastError();
}

hipError_t launch_moments_prep_f64(const double* w, int64_t K, int64_t kpad, uint16_t* pieces, double* sum_w,
                                   unsigned long long* maxbits, hipStream_t st)
{
    const int64_t n = kpad > K ? kpad : K;
    const int64_t blocks = std::min<int64_t>(256, std::max<int64_t>(1, (n + 255) / 256));
    if (K > 0) hipLaunchKernelGGL(moments_absmax_kernel, dim3((unsigned)blocks), dim3(256), 0, st, w, K, maxbits);
    hipLaunchKernelGGL(moments_prep_f64_kernel, dim3((unsigned)blocks), dim3(256), 0, st, w, K, kpad, pieces, sum_w,
                       maxbits);
    return hipGetLastError();
}

// G <- G * (-beta / sum): the weighted second moments to the gradient of
// log Z, the weight sum read on the device.
__global__ void moments_to_grad_kernel(double* G, int64_t n, double beta, const double* sum)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double f = -beta / *sum;
    G[i] = G[i] * f;
}

hipError_t launch_moments_to_grad(double* G, int64_t n, double beta, const double* sum, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(moments_to_grad_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, G, n, beta, sum);
    return hipGetLastError();
}

hipError_t launch_moments_unscale(double* G, int64_t n, const unsigned long long* maxbits, hipStream_t st)
{
    hipLaunchKernelGGL(moments_unscale_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, G, n, maxbits);
    return hipGetLastError();
}

hipError_t launch_pack_bits(const uint8_t* X, int64_t ldx, int64_t K, int32_t N, int32_t npad, int64_t words,
                            uint32_t* Xb, hipStream_t st)
{
    if (ldx % 4 == 0 && (reinterpret_cast<uintptr_t>(X) & 3u) == 0 && npad % 4 == 0) {
        const int64_t n = words * (npad / 4);
        hipLaunchKernelGGL(pack_bits4_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, X, ldx, K, N, npad,
                           words, Xb);
    } else {
        const int64_t n = words * npad;
        hipLaunchKernelGGL(pack_bits_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, X, ldx, K, N, npad,
                           words, Xb);
    }
    return hipGetLastError();
}

hipError_t launch_moments(const uint32_t* Xb, int32_t npad, int64_t words, int32_t N, const uint16_t* pieces,
                          int64_t kpad, int64_t chunk_words, const unsigned long long* max_m, float* part, double* G,
                          hipStream_t st)
{
    const int nt = (N + kTile - 1) / kTile;
    const int32_t tiles = nt * (nt + 1) / 2;
    const int64_t chunks = (words + chunk_words - 1) / chunk_words;
    const int64_t waves = (int64_t)tiles * chunks;
    hipLaunchKernelGGL(moments_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, st, Xb, npad, words, N, pieces,
                       kpad, chunk_words, tiles, max_m, part, G);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)tiles * kTile * kTile;
    hipLaunchKernelGGL(moments_reduce_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part, chunks, tiles,
                       N, G);
    return hipGetLastError();
}

hipError_t launch_moments_sum(const unsigned long long* sum_m, double* out, hipStream_t st)
{
    hipLaunchKernelGGL(moments_sum_kernel, dim3(1), dim3(1), 0, st, sum_m, out);
    return hipGetLastError();
}

hipError_t launch_logz(int32_t qtype, const void* Q, int32_t N, int32_t layout, double beta, double* part_max,
                       double* part_sum, int32_t blocks, int32_t lowbits, int64_t nthreads, double* out, hipStream_t st)
{
    if (qtype == Q_I16)
        hipLaunchKernelGGL(logz_kernel<int16_t>, dim3(blocks), dim3(256), 0, st, reinterpret_cast<const int16_t*>(Q), N,
                           layout, beta, lowbits, nthreads, part_max, part_sum);
    else if (qtype == Q_I32)
        hipLaunchKernelGGL(logz_kernel<int32_t>, dim3(blocks), dim3(256), 0, st, reinterpret_cast<const int32_t*>(Q), N,
                           layout, beta, lowbits, nthreads, part_max, part_sum);
    else
        hipLaunchKernelGGL(logz_kernel<float>, dim3(blocks), dim3(256), 0, st, reinterpret_cast<const float*>(Q), N,
                           layout, beta, lowbits, nthreads, part_max, part_sum);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(logz_finish_kernel, dim3(1), dim3(256), 0, st, part_max, part_sum, blocks, out);
    return hipGetLastError();
}

}  // namespace pns

// ---- moments into a static workspace (pns_moments_noalloc) ----

#include <mutex>

#include "pns.h"

namespace {

// Workspace of pns_moments_noalloc on each GPU: weight pieces, counters,
// packed records and partial tiles of one call.  A device global holds no
// valid address on the host: host code uses the per-device address from
// hipGetSymbolAddress, never this name.
constexpr size_t kScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Address of `scratch` on the current device, looked up on the first call
// on that device.
int scratch_address(void** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return pns::set_error(PNS_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return pns::set_error(PNS_EDEVICE, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return pns::set_error(PNS_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return PNS_OK;
}

bool on_device(const void* p)
{
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice;
}

}  // namespace

extern "C" int pns_moments_noalloc(const uint8_t* X, int64_t ldx, const int64_t* m, int64_t K, int32_t N, double* G,
                                   double* sum_m, void* stream)
{
    using namespace pns;
    if (!X || !m || !G) return set_error(PNS_EINVAL, "NULL argument");
    if (N < 1 || N > 32768) return set_error(PNS_EINVAL, "N must be in [1, 32768]");
    if (K < 0) return set_error(PNS_EINVAL, "K must be >= 0");
    if (ldx < N) return set_error(PNS_EINVAL, "ldx must be >= N");
    if (!on_device(X) || !on_device(m) || !on_device(G) || (sum_m && !on_device(sum_m)))
        return set_error(PNS_EINVAL, "X, m, G and sum_m must be device memory (nothing is staged here)");
    // the sizes of pns_moments' workspace
    const int64_t kpad = std::max<int64_t>(64, (K + 63) / 64 * 64);
    const int32_t npad = (N + 63) / 64 * 64;
    const int64_t words = std::max<int64_t>(1, (K + 31) / 32);
    const int64_t nt = npad / 64;
    const int64_t tiles = nt * (nt + 1) / 2;
    const size_t fixed = align256((size_t)3 * kpad * 2) + 256 + align256((size_t)words * npad * 4);
    const size_t tile_bytes = (size_t)tiles * 64 * 64 * 4;
    if (fixed + tile_bytes > kScratchBytes)
        return set_error(PNS_EINVAL,
                         "K = %lld records of N = %d need %zu bytes of workspace; the static workspace holds %zu "
                         "(use pns_moments)",
                         (long long)K, N, fixed + tile_bytes, kScratchBytes);
    // about 2048 waves, as pns_moments, with no more chunks than fit
    int64_t chunk_words = std::max<int64_t>(32, (words * tiles + 2047) / 2048);
    const int64_t max_chunks = (int64_t)((kScratchBytes - fixed) / tile_bytes);
    if ((words + chunk_words - 1) / chunk_words > max_chunks) chunk_words = (words + max_chunks - 1) / max_chunks;
    void* base = nullptr;
    int rc = scratch_address(&base);
    if (rc) return rc;
    unsigned char* b = static_cast<unsigned char*>(base);
    uint16_t* pieces = reinterpret_cast<uint16_t*>(b);
    b += align256((size_t)3 * kpad * 2);
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(b);
    b += 256;
    uint32_t* Xb = reinterpret_cast<uint32_t*>(b);
    b += align256((size_t)words * npad * 4);
    float* part = reinterpret_cast<float*>(b);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    // every buffer is written before it is read, except the counters and G:
    // cleared here (the workspace keeps the previous call's contents)
    hipError_t e = launch_fill64(G, (int64_t)N * N, 0, st);
    if (e == hipSuccess) e = launch_fill64(cnt, 3, 0, st);
    if (e == hipSuccess) e = launch_moments_prep(m, K, kpad, pieces, cnt, cnt + 1, st);
    if (e == hipSuccess) e = launch_pack_bits(X, ldx, K, N, npad, words, Xb, st);
    if (e == hipSuccess) e = launch_moments(Xb, npad, words, N, pieces, kpad, chunk_words, cnt + 1, part, G, st);
    if (e == hipSuccess && sum_m) e = launch_moments_sum(cnt, sum_m, st);
    if (e != hipSuccess) return set_error(PNS_EDEVICE, "moments kernels: %s", hipGetErrorString(e));
    return PNS_OK;
}

