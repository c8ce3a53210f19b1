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
__global__ void moments_prep_kernel(const int64_t* m, int64_t K, int64_t kpad, uint16_t* pieces,
                                    unsigned long long* sum_m, unsigned long long* max_m)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
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
    // wave reductions, then one atomic per wave
    unsigned long long sv = (unsigned long long)mk, mv = (unsigned long long)mk;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
        sv += __shfl_xor(sv, d, 64);
        const unsigned long long o = __shfl_xor(mv, d, 64);
        mv = mv > o ? mv : o;
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(sum_m, sv);
        atomicMax(max_m, mv);
    }
}

constexpr int kTile = 64;   // output tile (rows and columns) per workgroup
constexpr int kKT = 64;     // records staged per LDS round (two MFMA k-steps)
constexpr int kPadT = 8;    // bytes of padding per transposed LDS row

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

// One workgroup (4 waves) computes the 64 x 64 tile (ti, tj) of G over the
// records [k0, k0 + chunk); wave w owns the 32 x 32 quarter (w >> 1, w & 1)
// as 2 x 2 MFMA tiles of 16 x 16.
//
// MFMA operands (v_mfma_f32_16x16x32_bf16): lane l supplies row (A) or
// column (B) l % 16 and eight values of the contraction index; A and B use
// the same assignment of (lane / 16, element) to records, so the record order
// inside the 32-wide step does not matter.  Lane l receives C rows
// 4 * (l / 16) + e, column l % 16.
template <int P>
__global__ __launch_bounds__(256) void moments_kernel(const uint8_t* __restrict__ X, int64_t ldx, int64_t K, int32_t N,
                                                      const uint16_t* __restrict__ pieces, int64_t kpad, int64_t chunk,
                                                      double* __restrict__ G)
{
    __shared__ __attribute__((aligned(16))) uint8_t xi[kTile][kKT + kPadT];
    __shared__ __attribute__((aligned(16))) uint8_t xj[kTile][kKT + kPadT];
    __shared__ __attribute__((aligned(16))) uint16_t pw[P][kKT];

    const int nt = (N + kTile - 1) / kTile;
    int ti, tj;
    upper_tile((int)blockIdx.x, nt, &ti, &tj);
    const int i0 = ti * kTile, j0 = tj * kTile;
    const int64_t kbeg = (int64_t)blockIdx.y * chunk;
    const int64_t kend = kbeg + chunk < K ? kbeg + chunk : K;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    const int l16 = lane & 15, lg = lane >> 4;

    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = (f32x4){0.f, 0.f, 0.f, 0.f};

    for (int64_t k0 = kbeg; k0 < kend; k0 += kKT) {
        __syncthreads();
        // stage records [k0, k0 + 64) of the two column ranges, transposed:
        // thread t loads column t % 64 of rows t / 64 + 4e (coalesced rows)
        {
            const int c = tid & 63;
            const int rbase = tid >> 6;
#pragma unroll 4
            for (int e = 0; e < kKT / 4; ++e) {
                const int r = rbase + 4 * e;
                const int64_t k = k0 + r;
                uint8_t bi = 0, bj = 0;
                if (k < kend) {
                    const uint8_t* row = X + k * ldx;
                    if (i0 + c < N) bi = row[i0 + c] != 0;
                    if (j0 + c < N) bj = row[j0 + c] != 0;
                }
                xi[c][r] = bi;
                xj[c][r] = bj;
            }
            if (tid < kKT) {
                const int64_t k = k0 + tid;
#pragma unroll
                for (int s = 0; s < P; ++s) pw[s][tid] = k < kend ? pieces[s * kpad + k] : (uint16_t)0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kKT; ks += 32) {
            const int kk = ks + lg * 8;  // this lane's eight records in the step
            // B operands: x of the wave's two 16-column blocks
            bf16x8 bop[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const uint8_t* src = &xj[wc + b * 16 + l16][kk];
                const uint2 raw = *reinterpret_cast<const uint2*>(src);
                uint16_t v[8];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    v[e] = (uint16_t)(((raw.x >> (8 * e)) & 1u) * 0x3F80u);
                    v[4 + e] = (uint16_t)(((raw.y >> (8 * e)) & 1u) * 0x3F80u);
                }
                bop[b] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(v));
            }
#pragma unroll
            for (int s = 0; s < P; ++s) {
                uint16_t wv[8];
#pragma unroll
                for (int e = 0; e < 8; ++e) wv[e] = pw[s][kk + e];
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const uint8_t* src = &xi[wr + a * 16 + l16][kk];
                    const uint2 raw = *reinterpret_cast<const uint2*>(src);
                    uint16_t v[8];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        v[e] = ((raw.x >> (8 * e)) & 1u) ? wv[e] : (uint16_t)0;
                        v[4 + e] = ((raw.y >> (8 * e)) & 1u) ? wv[4 + e] : (uint16_t)0;
                    }
                    const bf16x8 aop = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(v));
#pragma unroll
                    for (int b = 0; b < 2; ++b)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, bop[b], acc[a][b], 0, 0, 0);
                }
            }
        }
    }

    // chunk result into FP64 G; an off-diagonal tile also feeds its mirror
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int j = j0 + wc + b * 16 + l16;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int i = i0 + wr + a * 16 + lg * 4 + e;
                const double v = (double)acc[a][b][e];
                if (i < N && j < N && v != 0.0) {
                    atomicAdd(&G[(int64_t)i * N + j], v);
                    if (ti != tj) atomicAdd(&G[(int64_t)j * N + i], v);
                }
            }
        }
    }
}

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
    hipLaunchKernelGGL(moments_prep_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, m, K, kpad, pieces,
                       sum_m, max_m);
    return hipGetLastError();
}

hipError_t launch_moments(int32_t pieces_used, const uint8_t* X, int64_t ldx, int64_t K, int32_t N,
                          const uint16_t* pieces, int64_t kpad, int64_t chunk, double* G, hipStream_t st)
{
    const int nt = (N + kTile - 1) / kTile;
    const unsigned tiles = (unsigned)(nt * (nt + 1) / 2);
    const unsigned chunks = (unsigned)((K + chunk - 1) / chunk);
    const dim3 grid(tiles, chunks);
    if (pieces_used == 1) hipLaunchKernelGGL(moments_kernel<1>, grid, dim3(256), 0, st, X, ldx, K, N, pieces, kpad, chunk, G);
    else if (pieces_used == 2) hipLaunchKernelGGL(moments_kernel<2>, grid, dim3(256), 0, st, X, ldx, K, N, pieces, kpad, chunk, G);
    else hipLaunchKernelGGL(moments_kernel<3>, grid, dim3(256), 0, st, X, ldx, K, N, pieces, kpad, chunk, G);
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
