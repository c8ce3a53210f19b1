// Initial-state kernels (bits, fields, energies), the fill kernel and the
// dispatch of the step kernels (pns_step.h, one translation unit per type).
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "pns_internal.h"

namespace pns {
namespace {

constexpr uint32_t kStreamStep = 0u;
constexpr uint32_t kStreamInit = 0x20000000u;
constexpr uint32_t kStreamSubset = 0x40000000u;
constexpr uint32_t kStreamSwap = 0x60000000u;
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

// Fields of many chains as one matrix product, H = X A (X the chains' 0/1
// states, [chains][N]; A the off-diagonal coefficients, symmetric), on the
// matrix cores.  A workgroup of four waves computes 64 chains x 64 fields,
// each wave 16 chains x four 16 x 16 tiles.  A is symmetric, so the operand
// column of field f over k is row f of A, read contiguously.  Bits past N
// (pitch padding of x) are masked out.

typedef int i32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x4_t __attribute__((ext_vector_type(4)));

// 16 int8 (0/1) states x[row][k .. k+15] as the int8 operand, bytes at or
// past N cleared; also their sum.
__device__ __forceinline__ i32x4_t x_bytes16(const uint8_t* xrow, int64_t k, int64_t N, int32_t* sum)
{
    uint4 v = make_uint4(0u, 0u, 0u, 0u);
    if (xrow != nullptr) v = *reinterpret_cast<const uint4*>(xrow + k);
    uint32_t w[4] = {v.x, v.y, v.z, v.w};
    int32_t s = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            if (k + 4 * q + b >= N) w[q] &= ~(0xFFu << (8 * b));
        }
        w[q] &= 0x01010101u;  // states are 0/1 bytes
        s += __builtin_popcount(w[q]);
    }
    *sum += s;
    return (i32x4_t){(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
}

// Integer coefficients on the int8 matrix cores (exact int32 sums): an entry
// is split into bytes, the top one signed and the others offset by -128 into
// int8, v = sum_p 256^p b_p + 128 (1 + 256 + ...), so
// H = sum_p 256^p (X B_p) + 128 (1 + 256 + ...) rowsum(X).
template <typename QT, typename HT>
__global__ __launch_bounds__(256) void init_fields_i8_kernel(InitArgs a, int32_t cbeg, int32_t cend)
{
    constexpr int NP = (int)sizeof(QT);  // byte pieces of an entry: 2 (int16) or 4 (int32)
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, kg = lane >> 4;
    const Problem P = a.problems[a.chain_problem[cbeg]];
    const int32_t cw = cbeg + (int32_t)blockIdx.y * 64 + wave * 16;  // this wave's first chain
    const int64_t f0 = (int64_t)blockIdx.x * 64;
    const int32_t crow = cw + r16;  // chain of this lane's operand row
    const uint8_t* xrow = crow < cend ? a.x + a.foff[crow] : nullptr;
    const QT* A = reinterpret_cast<const QT*>(P.A);
    i32x4_t acc[NP][4];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[p][t] = (i32x4_t){0, 0, 0, 0};
    int32_t xsum = 0;
    for (int64_t k0 = 0; k0 < P.pitch; k0 += 64) {
        const int64_t k = k0 + 16 * kg;  // this lane's 16 values of the 64-deep step
        const i32x4_t xop = x_bytes16(xrow, k, P.N, &xsum);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            // A has N rows: the fields past N (pitch padding) read zeros
            const int64_t fr = f0 + 16 * t + r16;
            const bool rok = fr < P.N;
            const QT* src = A + (rok ? fr : 0) * P.pitch + k;
            uint32_t bw[NP][4];
            if constexpr (NP == 2) {
                uint4 u[2] = {make_uint4(0u, 0u, 0u, 0u), make_uint4(0u, 0u, 0u, 0u)};
                if (rok) {
                    u[0] = *reinterpret_cast<const uint4*>(src);
                    u[1] = *reinterpret_cast<const uint4*>(src + 8);
                }
                const uint32_t wd[8] = {u[0].x, u[0].y, u[0].z, u[0].w, u[1].x, u[1].y, u[1].z, u[1].w};
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    // entries 4q .. 4q+3: two 16-bit entries per word
                    const uint32_t e0 = wd[2 * q] & 0xFFFFu, e1 = wd[2 * q] >> 16;
                    const uint32_t e2 = wd[2 * q + 1] & 0xFFFFu, e3 = wd[2 * q + 1] >> 16;
                    bw[1][q] = (e0 >> 8) | ((e1 >> 8) << 8) | ((e2 >> 8) << 16) | ((e3 >> 8) << 24);
                    bw[0][q] = ((e0 & 0xFFu) | ((e1 & 0xFFu) << 8) | ((e2 & 0xFFu) << 16) | ((e3 & 0xFFu) << 24)) ^
                               0x80808080u;
                }
            } else {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint4 u = rok ? *reinterpret_cast<const uint4*>(src + 4 * q) : make_uint4(0u, 0u, 0u, 0u);
                    const uint32_t e[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
                    for (int p = 0; p < 4; ++p) {
                        uint32_t w = 0;
#pragma unroll
                        for (int b = 0; b < 4; ++b) w |= ((e[b] >> (8 * p)) & 0xFFu) << (8 * b);
                        bw[p][q] = p == 3 ? w : (w ^ 0x80808080u);
                    }
                }
            }
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                const i32x4_t bop = {(int)bw[p][0], (int)bw[p][1], (int)bw[p][2], (int)bw[p][3]};
                acc[p][t] = __builtin_amdgcn_mfma_i32_16x16x64_i8(xop, bop, acc[p][t], 0, 0, 0);
            }
        }
    }
    // the states' sums of the 16 operand rows (four lanes hold each row)
    xsum += __shfl_xor(xsum, 16, 64);
    xsum += __shfl_xor(xsum, 32, 64);
    constexpr int64_t kOff = NP == 2 ? 128 : 128 * (1 + 256 + 65536);  // offsets of the low bytes
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int row = kg * 4 + e;  // output rows of this lane: chain cw + row, field f0 + 16t + r16
        const int64_t rs = __shfl(xsum, row, 64);
        const int32_t c = cw + row;
        if (c >= cend) continue;
        HT* hc = reinterpret_cast<HT*>(a.h) + a.foff[c];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            int64_t v = kOff * rs;
            int64_t scale = 1;
#pragma unroll
            for (int p = 0; p < NP; ++p) {
                v += scale * (int64_t)acc[p][t][e];
                scale *= 256;
            }
            hc[f0 + 16 * t + r16] = (HT)v;
        }
    }
}

// Float coefficients on the FP64 matrix cores: x and A as FP64 (both exact),
// FP64 accumulation, the precision of the FP64 fields.  Each lane takes four
// consecutive k of its row (k0 + 4 kg + m); MFMA m of a 16-deep step sums over
// the four lane groups.
template <typename QT, typename HT>
__global__ __launch_bounds__(256) void init_fields_f64_kernel(InitArgs a, int32_t cbeg, int32_t cend)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int r16 = lane & 15, kg = lane >> 4;
    const Problem P = a.problems[a.chain_problem[cbeg]];
    const int32_t cw = cbeg + (int32_t)blockIdx.y * 64 + wave * 16;
    const int64_t f0 = (int64_t)blockIdx.x * 64;
    const int32_t crow = cw + r16;
    const uint8_t* xrow = crow < cend ? a.x + a.foff[crow] : nullptr;
    const float* A = reinterpret_cast<const float*>(P.A);
    f64x4_t acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = (f64x4_t){0.0, 0.0, 0.0, 0.0};
    for (int64_t k0 = 0; k0 < P.pitch; k0 += 16) {
        const int64_t k = k0 + 4 * kg;
        uint32_t xw = xrow != nullptr ? *reinterpret_cast<const uint32_t*>(xrow + k) : 0u;
        double xd[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) xd[m] = (k + m < P.N && ((xw >> (8 * m)) & 1u)) ? 1.0 : 0.0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int64_t fr = f0 + 16 * t + r16;  // A has N rows: fields past N read zeros
            const float4 av = fr < P.N ? *reinterpret_cast<const float4*>(A + fr * P.pitch + k)
                                       : make_float4(0.f, 0.f, 0.f, 0.f);
            const float am[4] = {av.x, av.y, av.z, av.w};
#pragma unroll
            for (int m = 0; m < 4; ++m)
                acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(xd[m], (double)am[m], acc[t], 0, 0, 0);
        }
    }
    // output register e of a lane holds row kg + 4 e (rows interleaved across
    // the lane groups in the FP64 product), column r16
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int32_t c = cw + kg + 4 * e;
        if (c >= cend) continue;
        HT* hc = reinterpret_cast<HT*>(a.h) + a.foff[c];
#pragma unroll
        for (int t = 0; t < 4; ++t) hc[f0 + 16 * t + r16] = (HT)acc[t][e];
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
        if (a.last_E != nullptr) a.last_E[chain] = e;
    }
}

// Row i of a new coefficient matrix: A (zero diagonal, pitch-padded) and
// the diagonal; flags[0] |= asymmetry (SYMMETRIC layout), flags[1] |= a
// non-finite entry, flags[2] = max over rows of sum_j |A_ij|, flags[3] =
// max |Q_ii| (both as FP64 bits; non-negative doubles order like integers).
template <typename QT>
__global__ __launch_bounds__(256) void prepare_row_kernel(const QT* __restrict__ Q, int32_t N, int32_t layout,
                                                          int64_t pitch, QT* __restrict__ A,
                                                          typename Wide<QT>::T* __restrict__ diag,
                                                          unsigned long long* flags)
{
    const int i = blockIdx.x;
    __shared__ double ssum[256];
    double rs = 0.0;
    unsigned long long asym = 0, nonfin = 0;
    for (int64_t j = threadIdx.x; j < pitch; j += blockDim.x) {
        QT v = (QT)0;
        if (j < N) {
            const QT q = Q[(int64_t)i * N + j];
            if constexpr (std::is_floating_point<QT>::value) nonfin |= !isfinite(q);
            if (j == i) {
                diag[i] = (typename Wide<QT>::T)q;
                const double dq = fabs((double)q);
                atomicMax(&flags[3], (unsigned long long)__double_as_longlong(dq));
            } else if (layout == 0) {
                v = q;
                asym |= !(q == Q[j * N + i]);
            } else {
                v = i < j ? q : Q[j * N + i];
            }
        }
        A[(int64_t)i * pitch + j] = v;
        rs += fabs((double)v);
    }
    if (threadIdx.x == 0 && i == 0) {
        // padding entries of the diagonal
        for (int64_t j = N; j < pitch; ++j) diag[j] = (typename Wide<QT>::T)0;
    }
    if (asym) atomicOr(&flags[0], 1ull);
    if (nonfin) atomicOr(&flags[1], 1ull);
    ssum[threadIdx.x] = rs;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) ssum[threadIdx.x] += ssum[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(&flags[2], (unsigned long long)__double_as_longlong(ssum[0]));
}

// Parallel tempering: one thread per pair of adjacent ladder positions
// (pos, pos + 1), pos = round mod 2, round mod 2 + 2, ...  The chains exchange
// inverse temperatures with probability min{1, exp[(b_a - b_b)(E_a - E_b)]};
// U in (0, 1] from Philox (group, round, stream 0x60000000 | pos).
__global__ void pt_swap_kernel(const int64_t* E, int32_t is_float, double* beta, int32_t* ladder, int32_t groups,
                               int32_t T, uint64_t seed, uint64_t round, int32_t* accepted)
{
    const int32_t first = (int32_t)(round & 1u);
    const int32_t pairs = (T - 1 - first + 1) / 2;
    if (pairs <= 0) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t g = (int32_t)(t / pairs);
    if (g >= groups) return;
    const int32_t pos = first + 2 * (int32_t)(t % pairs);
    int32_t* lad = ladder + (int64_t)g * T;
    const int64_t ca = (int64_t)g * T + lad[pos];
    const int64_t cb = (int64_t)g * T + lad[pos + 1];
    const double dE = is_float ? __longlong_as_double(E[ca]) - __longlong_as_double(E[cb]) : (double)(E[ca] - E[cb]);
    const double ex = (beta[ca] - beta[cb]) * dE;
    const Words o = philox((uint32_t)g, (uint32_t)round, (uint32_t)(round >> 32), kStreamSwap | (uint32_t)pos, seed);
    const double u = (double)(((((uint64_t)o.w0 << 32) | o.w1) >> 11) + 1u) * 0x1p-53;
    const bool take = ex >= 0.0 || log(u) < ex;
    if (accepted) accepted[(int64_t)g * T + pos] = take ? 1 : 0;
    if (take) {
        const double tb = beta[ca];
        beta[ca] = beta[cb];
        beta[cb] = tb;
        const int32_t tl = lad[pos];
        lad[pos] = lad[pos + 1];
        lad[pos + 1] = tl;
    }
}

__global__ void fill64_kernel(int64_t* p, int64_t count, int64_t value)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

}  // namespace

hipError_t launch_steps(int32_t qtype, int32_t htype, int32_t flav, bool instr, int32_t block, int32_t groups,
                        int32_t grid, size_t dyn_lds, hipStream_t stream, const StepArgs& args)
{
    if (flav == 5) {
        if (qtype == Q_I16 && htype == H_I32) return launch_waves_i16(instr, block, groups, grid, stream, args, false);
        if (qtype == Q_I32 && htype == H_I32) return launch_waves_i32(instr, block, groups, grid, stream, args, false);
        return hipErrorInvalidConfiguration;
    }
    if (qtype == Q_I16 && htype == H_I32) return launch_steps_i16(flav, instr, block, groups, grid, dyn_lds, stream, args, false);
    if (qtype == Q_I32 && htype == H_I32) return launch_steps_i32(flav, instr, block, groups, grid, dyn_lds, stream, args, false);
    if (qtype == Q_I32 && htype == H_I64) return launch_steps_i64(flav, instr, block, groups, grid, dyn_lds, stream, args, false);
    if (qtype == Q_F32 && htype == H_F64) return launch_steps_f32(flav, instr, block, groups, grid, dyn_lds, stream, args, false);
    return hipErrorInvalidConfiguration;
}

bool have_tile(int32_t qtype, int32_t htype, int32_t block, int32_t groups)
{
    StepArgs none{};
    hipError_t e = hipErrorInvalidConfiguration;
    if (qtype == Q_I16 && htype == H_I32) e = launch_steps_i16(0, false, block, groups, 0, 0, nullptr, none, true);
    if (qtype == Q_I32 && htype == H_I32) e = launch_steps_i32(0, false, block, groups, 0, 0, nullptr, none, true);
    if (qtype == Q_I32 && htype == H_I64) e = launch_steps_i64(0, false, block, groups, 0, 0, nullptr, none, true);
    if (qtype == Q_F32 && htype == H_F64) e = launch_steps_f32(0, false, block, groups, 0, 0, nullptr, none, true);
    return e == hipSuccess;
}

bool have_wave_tile(int32_t qtype, int32_t htype, int32_t block, int32_t groups)
{
    StepArgs none{};
    hipError_t e = hipErrorInvalidConfiguration;
    if (qtype == Q_I16 && htype == H_I32) e = launch_waves_i16(false, block, groups, 0, nullptr, none, true);
    if (qtype == Q_I32 && htype == H_I32) e = launch_waves_i32(false, block, groups, 0, nullptr, none, true);
    return e == hipSuccess;
}

template <typename QT, typename HT>
static hipError_t init_typed(int32_t max_pitch, hipStream_t st, const InitArgs& a, const int32_t* host_chain_problem,
                             const int64_t* host_pitch)
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
        for (int32_t t = c; t < e; t += 64 * 65535) {
            const int32_t tend = t + 64 * 65535 < e ? t + 64 * 65535 : e;
            // every chain of [t, tend) belongs to one problem: its pitch tiles the fields
            const dim3 grid((unsigned)(host_pitch[host_chain_problem[c]] / 64), (unsigned)((tend - t + 63) / 64));
            if constexpr (std::is_floating_point<QT>::value)
                hipLaunchKernelGGL((init_fields_f64_kernel<QT, HT>), grid, dim3(256), 0, st, a, t, tend);
            else
                hipLaunchKernelGGL((init_fields_i8_kernel<QT, HT>), grid, dim3(256), 0, st, a, t, tend);
            hipError_t er = hipGetLastError();
            if (er != hipSuccess) return er;
        }
        c = e;
    }
    hipLaunchKernelGGL((init_energy_kernel<QT, HT>), dim3(a.num_chains), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_init_with_map(int32_t qtype, int32_t htype, int32_t max_pitch, hipStream_t stream,
                                const InitArgs& args, const int32_t* host_chain_problem, const int64_t* host_pitch)
{
    if (qtype == Q_I16 && htype == H_I32)
        return init_typed<int16_t, int32_t>(max_pitch, stream, args, host_chain_problem, host_pitch);
    if (qtype == Q_I32 && htype == H_I32)
        return init_typed<int32_t, int32_t>(max_pitch, stream, args, host_chain_problem, host_pitch);
    if (qtype == Q_I32 && htype == H_I64)
        return init_typed<int32_t, int64_t>(max_pitch, stream, args, host_chain_problem, host_pitch);
    if (qtype == Q_F32 && htype == H_F64)
        return init_typed<float, double>(max_pitch, stream, args, host_chain_problem, host_pitch);
    return hipErrorInvalidConfiguration;
}

hipError_t launch_prepare_rows(int32_t qtype, const void* Q, int32_t N, int32_t layout, int64_t pitch, void* A,
                               void* diag, unsigned long long* flags, hipStream_t st)
{
    if (qtype == Q_I16)
        hipLaunchKernelGGL(prepare_row_kernel<int16_t>, dim3(N), dim3(256), 0, st, reinterpret_cast<const int16_t*>(Q), N,
                           layout, pitch, reinterpret_cast<int16_t*>(A), reinterpret_cast<int32_t*>(diag), flags);
    else if (qtype == Q_I32)
        hipLaunchKernelGGL(prepare_row_kernel<int32_t>, dim3(N), dim3(256), 0, st, reinterpret_cast<const int32_t*>(Q), N,
                           layout, pitch, reinterpret_cast<int32_t*>(A), reinterpret_cast<int32_t*>(diag), flags);
    else
        hipLaunchKernelGGL(prepare_row_kernel<float>, dim3(N), dim3(256), 0, st, reinterpret_cast<const float*>(Q), N,
                           layout, pitch, reinterpret_cast<float*>(A), reinterpret_cast<float*>(diag), flags);
    return hipGetLastError();
}

hipError_t launch_pt_swap(const int64_t* E, int32_t is_float, double* beta, int32_t* ladder, int32_t groups, int32_t T,
                          uint64_t seed, uint64_t round, int32_t* accepted, hipStream_t st)
{
    const int64_t pairs = (int64_t)groups * ((T - (int32_t)(round & 1u)) / 2);
    if (pairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(pt_swap_kernel, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, st, E, is_float, beta, ladder,
                       groups, T, seed, round, accepted);
    return hipGetLastError();
}

// One wave that waits `ticks` of the constant-rate wall clock and exits: a
// bounded delay on a stream.
__global__ void hold_kernel(uint64_t ticks)
{
    const uint64_t t0 = wall_clock64();
    while (wall_clock64() - t0 < ticks) __builtin_amdgcn_s_sleep(8);
}

hipError_t launch_hold(uint64_t ticks, hipStream_t st)
{
    hipLaunchKernelGGL(hold_kernel, dim3(1), dim3(64), 0, st, ticks);
    return hipGetLastError();
}

hipError_t launch_fill64(void* p, int64_t count, int64_t value, hipStream_t stream)
{
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(fill64_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream,
                       reinterpret_cast<int64_t*>(p), count, value);
    return hipGetLastError();
}

}  // namespace pns
