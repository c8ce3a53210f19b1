// Unbiased PNS for continuous states (Alg 7) on the donut target of Sec 7:
// log pi(x) = -(|x|^2 - mu0)^2 / (2 sigma^2) on R^D, symmetric normal
// increments as the proposal, so every acceptance ratio is pi(y) / pi(x).
//
// Partial neighbor set i of a chain: P offset vectors delta_j with i.i.d.
// N(0, 1) coordinates, each used with both signs (the pairs keep the set
// reversible); neighbour j of x is x + delta_j for j < P and x - delta_{j-P}
// for P <= j < 2P.  The set is drawn anew when a block of L0 original
// samples runs out (the "else" branch of Alg 7).  The proposal restricted to
// the set is uniform over its 2P points, so p = (1/2P) sum_j min(1, pi(y_j) /
// pi(x)) and the next state is chosen proportionally to min(1, pi(y_j) /
// pi(x)).
//
// Layout: a group of 8 lanes per chain, 8 chains per wave, 32 per 256-thread
// workgroup.  Lane r of a group holds the signed offsets of neighbours
// j = r m .. r m + m - 1 (m = ceil(2P / 8) <= 8) in registers and evaluates
// their weights one after the other; a segmented DPP scan over the group gives
// S, p and the inverse-CDF choice (appendix "How to Sample Proportionally":
// the first neighbour whose running sum exceeds U2 S).  The per-record scalar work (the multiplicity, the
// budget, the expected multiplicity) is then shared by 8 chains per wave
// instruction instead of being repeated by a whole wave for one chain.  The
// state, its log-density, the budget and the estimator sums stay in registers
// for the whole launch.  Normal offsets: Box-Muller on two uniforms of one
// Philox block, counter (chain, set index low, set index high, 0x80000000 |
// j << 8 | t) for coordinates 2t, 2t + 1.  Step uniforms: those of the
// discrete samplers (counter (chain, step low, step high, 0)), drawn 8 steps at
// a time (lane r of a group holds step k + r).
//
// Floating-point contraction is off in this file so that the density and the
// estimator sums round like their plain definitions.
#pragma clang fp contract(off)

#include "pns_step.h"

namespace pns {
namespace cont {

using step::dpp_f64;
using step::philox;
using step::Words;

constexpr uint32_t kStreamOffsets = 0x80000000u;
constexpr int kGroup = 8;                  // lanes per chain
constexpr int kChainsPerBlock = 256 / kGroup;

// Coordinates of offset pair `pj` of set `set`: Box-Muller, z0 = sqrt(-2 log
// u1) cos(2 pi u2) for coordinate 2t and z1 = sqrt(-2 log u1) sin(2 pi u2) for
// 2t + 1, u1 in (0, 1] from words 0, 1 and u2 in [0, 1) from words 2, 3.
// Not inlined: the transcendental code stays out of the step loop's registers.
template <int D>
struct Offset {
    double v[D];
};

template <int D>
__device__ __noinline__ Offset<D> draw_offset(uint64_t seed, uint32_t cid, int64_t set, int pj)
{
    Offset<D> o{};
#pragma unroll
    for (int t = 0; 2 * t < D; ++t) {
        const Words w =
            philox(cid, (uint32_t)set, (uint32_t)((uint64_t)set >> 32), kStreamOffsets | ((uint32_t)pj << 8) | t, seed);
        const double u1 = (double)(((((uint64_t)w.w0 << 32) | w.w1) >> 11) + 1u) * 0x1p-53;
        const double u2 = (double)((((uint64_t)w.w2 << 32) | w.w3) >> 11) * 0x1p-53;
        const double r = sqrt(-2.0 * log(u1));
        const double ang = 6.283185307179586 * u2;  // 2 pi, rounded to double
        o.v[2 * t] = r * cos(ang);
        if (2 * t + 1 < D) o.v[2 * t + 1] = r * sin(ang);
    }
    return o;
}

// The multiplicity quotient q = log U1 / log(1 - p) (M = 1 + floor(q)) and
// the expected multiplicity E[min(1 + G, L)] = (1 - (1 - p)^L) / p of a
// budgeted record.  Not inlined: keeps the FP64 library code out of the step
// loop's registers.
struct Geo {
    double q, wrb;
};

__device__ __noinline__ Geo geometric(double p, double logU1, int64_t L)
{
    if (p >= 1.0) return {0.0, 1.0};
    if (p <= 0.0) return {INFINITY, (double)L};
    const double lg = log1p(-p);
    return {logU1 / lg, -expm1((double)L * lg) / p};
}

// Uniforms of step k of chain cid: log U1 (U1 in (0, 1], words 0, 1) and U2
// in [0, 1) (words 2, 3), returned as (q, wrb) = (log U1, U2).
__device__ __noinline__ Geo step_uniforms(uint32_t cid, int64_t k, uint64_t seed)
{
    const Words o = philox(cid, (uint32_t)k, (uint32_t)((uint64_t)k >> 32), 0u, seed);
    const double u1 = (double)(((((uint64_t)o.w0 << 32) | o.w1) >> 11) + 1u) * 0x1p-53;
    return {log(u1), (double)((((uint64_t)o.w2 << 32) | o.w3) >> 11) * 0x1p-53};
}

template <int D>
__device__ __forceinline__ double pick(const double* v, int i)
{
    double r = v[0];
#pragma unroll
    for (int t = 1; t < D; ++t)
        if (i == t) r = v[t];
    return r;
}

// log pi(x) = -(|x|^2 - mu0)^2 c with c = 1 / (2 sigma^2) rounded once (on the
// host).
template <int D>
__device__ __forceinline__ double log_density(const double* x, double mu0, double c)
{
    double r2 = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) r2 += x[i] * x[i];
    const double tt = r2 - mu0;
    return -(tt * tt) * c;
}

// Inclusive prefix sum within each group of 8 lanes (rows of 16 hold two
// groups; row_shr by 1, 2, 4 with the lanes below the shift masked off).
__device__ __forceinline__ double group_scan(double v, int r)
{
    double t = dpp_f64<0x111, 0xF>(v);
    if (r >= 1) v += t;
    t = dpp_f64<0x112, 0xF>(v);
    if (r >= 2) v += t;
    t = dpp_f64<0x114, 0xF>(v);
    if (r >= 4) v += t;
    return v;
}

// exp(l) for l <= 0 (the weights min(1, pi(y)/pi(x))): Cody-Waite reduction
// l = k ln 2 + r with |r| <= ln 2 / 2 (ln 2 split in two so that k ln2_hi is
// exact), exp(r) by its Taylor series to degree 13 (truncation below 2^-57
// relative) in Horner form, scaled by 2^k with ldexp (gradual underflow; 0
// below the smallest subnormal).  Within 2 ulp of the correctly rounded
// value.  The constants are wave-uniform values passed in scalar registers,
// read once before the step loop.
struct ExpConsts {
    double c[14];  // 1 / j!
    double log2e, ln2_hi, ln2_lo;
};

__device__ __forceinline__ ExpConsts exp_consts()
{
    ExpConsts e;
    double f = 1.0;
#pragma unroll
    for (int j = 0; j < 14; ++j) {
        if (j > 0) f = f / (double)j;
        e.c[j] = f;
    }
    e.log2e = 0x1.71547652b82fep+0;
    e.ln2_hi = 0x1.62e42fee00000p-1;
    e.ln2_lo = 0x1.a39ef35793c76p-33;
#pragma unroll
    for (int j = 0; j < 14; ++j) asm volatile("" : "+s"(e.c[j]));
    asm volatile("" : "+s"(e.log2e), "+s"(e.ln2_hi), "+s"(e.ln2_lo));
    return e;
}

__device__ __forceinline__ double exp_nonpos(double l, const ExpConsts& e)
{
    l = fmax(l, -746.0);
    const double k = rint(l * e.log2e);
    const double r = fma(-k, e.ln2_lo, fma(-k, e.ln2_hi, l));
    double p = e.c[13];
#pragma unroll
    for (int j = 12; j >= 0; --j) p = fma(p, r, e.c[j]);
    return ldexp(p, (int)k);
}

// MP: neighbours per lane the kernel is built for (m <= MP; the launcher
// picks the smallest of 2, 4, 7, 8 that holds m), so that the weights of a
// lane are straight-line code without branches and their exponentials
// interleave.
template <int D, int MP>
__global__ __launch_bounds__(256) void cont_kernel(const ContArgs a)
{
    const int lane = threadIdx.x & 63;
    const int r = lane & (kGroup - 1);            // lane within the chain's group
    const int gbase = lane & ~(kGroup - 1);       // first lane of the group
    const int32_t chain = (int32_t)blockIdx.x * kChainsPerBlock + (int32_t)(threadIdx.x / kGroup);
    // groups past the last chain run along on chain 0's data and write nothing,
    // so that every lane takes part in the wave-wide exchanges
    const bool live = chain < a.num_chains;
    const int32_t ch = live ? chain : 0;
    const int P = a.pairs, n = 2 * a.pairs;
    const int m = (n + kGroup - 1) / kGroup;      // neighbours per lane
    const uint32_t cid = a.chain_id[ch];
    constexpr int NS = 4 * D + 1;                 // estimator sums per weighting
    constexpr int NA = (2 * NS + kGroup - 1) / kGroup;  // sums per lane

    double x[D], s[MP][D], w[MP];
#pragma unroll
    for (int i = 0; i < D; ++i) x[i] = a.x[(int64_t)ch * D + i];
    double lpx = a.lpx[ch];
    int64_t L = a.L[ch], set = a.set[ch];
    const int64_t k0 = a.step[ch];
    int64_t flips = 0, stays = 0;

    auto load_set = [&]() {
#pragma unroll
        for (int t = 0; t < MP; ++t) {
            const int j = r * m + t;
            if (t < m && j < n) {
                const int pj = j < P ? j : j - P;
                const Offset<D> dl = draw_offset<D>(a.seed, cid, set, pj);
#pragma unroll
                for (int i = 0; i < D; ++i) s[t][i] = j < P ? dl.v[i] : -dl.v[i];
            } else {
#pragma unroll
                for (int i = 0; i < D; ++i) s[t][i] = 0.0;
            }
        }
    };
    load_set();

    // lane r keeps estimator sums r, r + 8, ...: weighting idx / NS (M, then
    // the expected multiplicity), component idx % NS (sum w, then w x_i,
    // w x_i^2, w x_i^4, w 1(x_i > 0))
    double acc[NA];
    int akind[NA], agrp[NA], aci[NA];
#pragma unroll
    for (int u = 0; u < NA; ++u) {
        const int idx = r + kGroup * u;
        akind[u] = idx < 2 * NS ? idx / NS : -1;
        const int comp = idx % NS;
        agrp[u] = comp == 0 ? -1 : (comp - 1) / D;
        aci[u] = comp == 0 ? 0 : (comp - 1) % D;
        acc[u] = akind[u] >= 0 ? a.sums[(int64_t)ch * 2 * NS + idx] : 0.0;
    }

    const ExpConsts ek = exp_consts();
    double logU1b = 0.0, U2b = 0.0;
    for (int64_t it = 0; it < a.steps; ++it) {
        const int64_t k = k0 + it;
        const int bl = (int)(it & (kGroup - 1));
        if (bl == 0) {
            const Geo u = step_uniforms(cid, k + r, a.seed);
            logU1b = u.q;
            U2b = u.wrb;
        }
        // weights of this lane's neighbours, min(1, pi(y)/pi(x)) = exp(min(l, 0))
        // (exp(0) = 1 exactly), summed in neighbour order
        double ls = 0.0;
#pragma unroll
        for (int t = 0; t < MP; ++t) {
            double y[D];
#pragma unroll
            for (int i = 0; i < D; ++i) y[i] = x[i] + s[t][i];
            const double l = fmin(log_density<D>(y, a.mu0, a.c) - lpx, 0.0);
            const bool on = t < m && r * m + t < n;
            w[t] = on ? exp_nonpos(l, ek) : 0.0;
            ls += w[t];
        }
        const double incl = group_scan(ls, r);
        const double S = __shfl(incl, gbase + kGroup - 1, 64);
        const double p = S / (double)n;
        const double logU1 = __shfl(logU1b, gbase + bl, 64), U2 = __shfl(U2b, gbase + bl, 64);
        const Geo g = geometric(p, logU1, L);
        const bool stay = g.q >= (double)L;
        const int64_t M = stay ? L : (int64_t)floor(g.q) + 1;

        // the record (J_k, M_k): estimator sums over the state before the move
#pragma unroll
        for (int u = 0; u < NA; ++u) {
            if (akind[u] < 0) continue;
            const double wt = akind[u] == 0 ? (double)M : g.wrb;
            if (agrp[u] < 0) {
                acc[u] += wt;
            } else {
                const double v = pick<D>(x, aci[u]), v2 = v * v;
                if (agrp[u] == 0) acc[u] += wt * v;
                else if (agrp[u] == 1) acc[u] += wt * v2;
                else if (agrp[u] == 2) acc[u] += wt * (v2 * v2);
                else acc[u] += v > 0.0 ? wt : 0.0;
            }
        }
        const int64_t slot = (int64_t)ch * a.log_cap + (a.log_cap > 0 ? k % a.log_cap : 0);
        if (a.log_cap > 0 && live && r == 0) {
            a.log_M[slot] = M;
            a.log_lp[slot] = lpx;
            a.log_p[slot] = p;
            a.log_w[slot] = g.wrb;
        }
        int32_t action;
        if (stay) {
            // Alg 7 "else": stay for the remaining L samples, next set
            action = -1;
            L = a.L0;
            ++set;
            ++stays;
            load_set();
        } else {
            L -= M;
            // first neighbour whose running sum exceeds U2 * S (weights > 0);
            // rounding fallback: the last positive one
            const double t2 = U2 * S;
            double run = incl - ls;
            int found = -1, lastpos = -1;
#pragma unroll
            for (int t = 0; t < MP; ++t) {
                if (w[t] > 0.0) lastpos = t;
                run += w[t];
                if (found < 0 && run > t2 && w[t] > 0.0) found = t;
            }
            const uint32_t hit = (uint32_t)(__ballot(found >= 0) >> gbase) & 0xFFu;
            int src, tsel;
            if (hit != 0) {
                src = __builtin_ctz(hit);
                tsel = __shfl(found, gbase + src, 64);
            } else {
                const uint32_t pos = (uint32_t)(__ballot(lastpos >= 0) >> gbase) & 0xFFu;
                src = 31 - __builtin_clz(pos);
                tsel = __shfl(lastpos, gbase + src, 64);
            }
            // the chosen offset, from lane src of the group
#pragma unroll
            for (int i = 0; i < D; ++i) {
                double v = s[0][i];
#pragma unroll
                for (int t = 1; t < MP; ++t)
                    if (tsel == t) v = s[t][i];
                x[i] = x[i] + __shfl(v, gbase + src, 64);
            }
            lpx = log_density<D>(x, a.mu0, a.c);
            action = src * m + tsel;
            ++flips;
        }
        if (a.log_cap > 0 && live && r == 0) a.log_action[slot] = action;
    }

    // chain state back to memory
    if (!live) return;
    if (r < D) a.x[(int64_t)chain * D + r] = pick<D>(x, r);
#pragma unroll
    for (int u = 0; u < NA; ++u)
        if (akind[u] >= 0) a.sums[(int64_t)chain * 2 * NS + r + kGroup * u] = acc[u];
    if (r == 0) {
        a.lpx[chain] = lpx;
        a.L[chain] = L;
        a.set[chain] = set;
        a.step[chain] = k0 + a.steps;
        a.counters[(int64_t)chain * 2 + 0] += flips;
        a.counters[(int64_t)chain * 2 + 1] += stays;
    }
}

// log pi of each chain's state (on creation and after the state is set).
template <int D>
__global__ void cont_init_kernel(const ContArgs a)
{
    const int32_t c = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (c >= a.num_chains) return;
    double x[D];
#pragma unroll
    for (int i = 0; i < D; ++i) x[i] = a.x[(int64_t)c * D + i];
    a.lpx[c] = log_density<D>(x, a.mu0, a.c);
}

}  // namespace cont

hipError_t launch_cont(const ContArgs& a, bool init, hipStream_t st)
{
    if (a.num_chains <= 0) return hipSuccess;
    const dim3 grid_run((unsigned)((a.num_chains + cont::kChainsPerBlock - 1) / cont::kChainsPerBlock));
    const dim3 grid_init((unsigned)((a.num_chains + 255) / 256));
    const int m = (2 * a.pairs + cont::kGroup - 1) / cont::kGroup;
#define PNS_CONT_CASE(DD)                                                                                \
    case DD:                                                                                             \
        if (init) hipLaunchKernelGGL(cont::cont_init_kernel<DD>, grid_init, dim3(256), 0, st, a);        \
        else if (m <= 2) hipLaunchKernelGGL((cont::cont_kernel<DD, 2>), grid_run, dim3(256), 0, st, a);  \
        else if (m <= 4) hipLaunchKernelGGL((cont::cont_kernel<DD, 4>), grid_run, dim3(256), 0, st, a);  \
        else if (m <= 7) hipLaunchKernelGGL((cont::cont_kernel<DD, 7>), grid_run, dim3(256), 0, st, a);  \
        else hipLaunchKernelGGL((cont::cont_kernel<DD, 8>), grid_run, dim3(256), 0, st, a);              \
        break;
    switch (a.dim) {
        PNS_CONT_CASE(1)
        PNS_CONT_CASE(2)
        PNS_CONT_CASE(3)
        PNS_CONT_CASE(4)
        PNS_CONT_CASE(5)
        PNS_CONT_CASE(6)
        PNS_CONT_CASE(7)
        default:
            return hipErrorInvalidValue;
    }
#undef PNS_CONT_CASE
    return hipGetLastError();
}

}  // namespace pns
