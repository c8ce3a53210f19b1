// Unbiased PNS for continuous states (Alg 7) on the donut target of Sec 6:
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
// Layout: one wave per chain (four chains per 256-thread block); lane j keeps
// neighbour j's signed offset in registers and evaluates its weight; a wave
// prefix sum gives p and the inverse-CDF choice (App. C); the state, its
// log-density, the budget and the estimator sums stay in registers for the
// whole launch.  Normal offsets: Box-Muller on two uniforms of one Philox
// block, counter (chain, set index low, set index high, 0x80000000 | j << 8 |
// t) for coordinates 2t, 2t + 1.  Step uniforms: those of the discrete
// samplers (stream 0, counter (chain, step low, step high, 0)).
//
// Floating-point contraction is off in this file so that the density and the
// estimator sums round like their plain definitions.
#pragma clang fp contract(off)

#include "pns_step.h"

namespace pns {
namespace cont {

using step::batch_uniforms;
using step::philox;
using step::read_lane;
using step::wave_scan;
using step::Words;

constexpr uint32_t kStreamOffsets = 0x80000000u;

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

template <int D>
__device__ __forceinline__ double pick(const double* v, int i)
{
    double r = v[0];
#pragma unroll
    for (int t = 1; t < D; ++t)
        if (i == t) r = v[t];
    return r;
}

template <int D>
__global__ __launch_bounds__(256) void cont_kernel(const ContArgs a)
{
    const int lane = threadIdx.x & 63;
    const int32_t chain = (int32_t)blockIdx.x * 4 + (int32_t)(threadIdx.x >> 6);
    if (chain >= a.num_chains) return;  // wave-uniform
    const int P = a.pairs, n = 2 * a.pairs;
    const bool active = lane < n;
    const int pj = lane < P ? lane : lane - P;
    const double sgn = lane < P ? 1.0 : -1.0;
    const uint32_t cid = a.chain_id[chain];
    constexpr int NS = 4 * D + 1;  // estimator sums per weighting

    double x[D], s[D];
#pragma unroll
    for (int i = 0; i < D; ++i) x[i] = a.x[(int64_t)chain * D + i];
    double lpx = a.lpx[chain];
    int64_t L = a.L[chain], set = a.set[chain];
    const int64_t k0 = a.step[chain];
    int64_t flips = 0, stays = 0;

    auto load_set = [&]() {
        const Offset<D> dl = draw_offset<D>(a.seed, cid, set, pj);
#pragma unroll
        for (int i = 0; i < D; ++i) s[i] = active ? sgn * dl.v[i] : 0.0;
    };
    load_set();

    // lane t < 2 NS keeps estimator sum t: weighting t / NS (M, then the
    // expected multiplicity), component t % NS (sum w, then w x_i, w x_i^2,
    // w x_i^4, w 1(x_i > 0))
    const bool has_acc = lane < 2 * NS;
    const int kind = lane < NS ? 0 : 1;
    const int comp = lane - kind * NS;
    const int grp = comp == 0 ? -1 : (comp - 1) / D;
    const int ci = comp == 0 ? 0 : (comp - 1) % D;
    double acc = has_acc ? a.sums[(int64_t)chain * 2 * NS + lane] : 0.0;

    double logU1b = 0.0, U2b = 0.0;
    for (int64_t it = 0; it < a.steps; ++it) {
        const int64_t k = k0 + it;
        const int bl = (int)(it & 63);
        if (bl == 0) batch_uniforms(cid, k, a.seed, lane, true, &logU1b, &U2b);
        // weight of this lane's neighbour
        double y[D], r2 = 0.0;
#pragma unroll
        for (int i = 0; i < D; ++i) {
            y[i] = x[i] + s[i];
            r2 += y[i] * y[i];
        }
        const double tt = r2 - a.mu0;
        const double lpy = -(tt * tt) / a.den;
        const double l = lpy - lpx;
        const double w = active ? (l < 0.0 ? exp(l) : 1.0) : 0.0;
        const double incl = wave_scan(w);
        const double S = read_lane(incl, 63);
        const double p = S / (double)n;
        const double logU1 = read_lane(logU1b, bl), U2 = read_lane(U2b, bl);
        const Geo g = geometric(p, logU1, L);
        const double q = g.q, wrb = g.wrb;
        const bool stay = q >= (double)L;
        const int64_t M = stay ? L : (int64_t)floor(q) + 1;

        // the record (J_k, M_k): estimator sums over the state before the move
        if (has_acc) {
            const double wt = kind == 0 ? (double)M : wrb;
            if (grp < 0) {
                acc += wt;
            } else {
                const double v = pick<D>(x, ci), v2 = v * v;
                if (grp == 0) acc += wt * v;
                else if (grp == 1) acc += wt * v2;
                else if (grp == 2) acc += wt * (v2 * v2);
                else acc += v > 0.0 ? wt : 0.0;
            }
        }
        int32_t action;
        if (a.log_cap > 0 && lane == 0) {
            const int64_t slot = (int64_t)chain * a.log_cap + (k % a.log_cap);
            a.log_M[slot] = M;
            a.log_lp[slot] = lpx;
            a.log_p[slot] = p;
            a.log_w[slot] = wrb;
        }
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
            const uint64_t hit = __ballot(active && incl > t2 && w > 0.0);
            int sel;
            if (hit != 0) {
                sel = __builtin_ctzll(hit);
            } else {
                const uint64_t pos = __ballot(w > 0.0);
                sel = 63 - __builtin_clzll(pos);
            }
#pragma unroll
            for (int i = 0; i < D; ++i) x[i] = x[i] + __shfl(s[i], sel, 64);
            lpx = __shfl(lpy, sel, 64);
            action = sel;
            ++flips;
        }
        if (a.log_cap > 0 && lane == 0) a.log_action[(int64_t)chain * a.log_cap + (k % a.log_cap)] = action;
    }

    // chain state back to memory
    if (lane < D) a.x[(int64_t)chain * D + lane] = pick<D>(x, lane);
    if (has_acc) a.sums[(int64_t)chain * 2 * NS + lane] = acc;
    if (lane == 0) {
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
    double r2 = 0.0;
#pragma unroll
    for (int i = 0; i < D; ++i) {
        const double v = a.x[(int64_t)c * D + i];
        r2 += v * v;
    }
    const double tt = r2 - a.mu0;
    a.lpx[c] = -(tt * tt) / a.den;
}

}  // namespace cont

hipError_t launch_cont(const ContArgs& a, bool init, hipStream_t st)
{
    if (a.num_chains <= 0) return hipSuccess;
    const dim3 grid_run((unsigned)((a.num_chains + 3) / 4)), grid_init((unsigned)((a.num_chains + 255) / 256));
#define PNS_CONT_CASE(DD)                                                                              \
    case DD:                                                                                           \
        if (init) hipLaunchKernelGGL(cont::cont_init_kernel<DD>, grid_init, dim3(256), 0, st, a);      \
        else hipLaunchKernelGGL(cont::cont_kernel<DD>, grid_run, dim3(256), 0, st, a);                 \
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
