// Window kernel of one or two waves per chain: Unbiased PNS (Alg 6) with the
// systematic partial neighbor sets on integer coefficient matrices.
// Included by the integer step translation units after pns_step.h.
//
// The chain's N bits are laid out as in the step kernel, f = (g*BLOCK+tid)*4+v,
// so the bits of one wave in one group form a 256-bit segment and segment
// g*W + w covers bits [256 (g W + w), +256).  What differs is where the work
// goes:
//   * the lanes keep u_j = Q_jj + s h_j instead of h_j, so that
//     dE_j = (1 - 2 x_j) u_j needs no diagonal, and a flip of c adds
//     s (1 - 2 x_c) A[c][j] to u_j (A has a zero diagonal, so u_c is
//     unchanged); the fields are converted back on exit;
//   * a step weighs only the groups whose segments the window meets (a
//     uniform mask kept per window), sums and scans them as the step kernel
//     does (four-bit sums, DPP wave scan per segment, one scan over the
//     segment totals in bit order);
//   * the energy differences of those groups are staged in LDS (one slot per
//     group the window meets, at most kSlots per wave), so that the choice,
//     which is resolved only when the chain moves, and the rare paths (a
//     weight past the tables, a window whose weights all underflow) read them
//     by slot instead of indexing registers;
//   * with one wave there is no barrier at all; with two, one exchange of
//     the segment totals (every step) and one of the choice (moves only).
// Chain scalars (energy, budget, window, counters) are wave-uniform values.
#pragma once

#include <utility>

#include "pns_step.h"

namespace pns {
namespace wave {

using step::kTabHi;
using step::kTabLo;
using step::kTabMax;

// Flavour code of this kernel in the launch classes.
constexpr int FLAV_WAVE = 5;
// Groups of one wave that one window may meet (checked on the host for every
// systematic set).
constexpr int kSlots = 4;
// Energy difference slot value of a bit outside the window.
constexpr int32_t kOut = INT32_MIN;

// Waves per SIMD asked of the compiler: the fields take F = 4 G registers.
template <int W, int G>
constexpr int waves_per_eu()
{
    return G <= 8 ? 4 : (G <= 16 ? 3 : 2);
}

// Two 16-bit integers of one register (operands of the 16-bit dot product).
typedef int16_t v2i16 __attribute__((ext_vector_type(2)));

// Bit i of a lane's packed state words (i a compile-time index).
template <int NW>
__device__ __forceinline__ uint32_t get_bit(const uint32_t (&xw)[NW], int i)
{
    return (xw[i >> 5] >> (i & 31)) & 1u;
}

// body(integral_constant<i>) for every i of the sequence, in order.
template <int... I, typename Fn>
__device__ __forceinline__ void for_each_index(std::integer_sequence<int, I...>, Fn&& body)
{
    (body(std::integral_constant<int, I>{}), ...);
}

// The lane's index in its wave, formed where it is used: a per-lane value
// kept across the step loop takes a register or is spilled and reloaded.
__device__ __forceinline__ int lane_here()
{
    uint32_t m = ~0u;
    asm volatile("" : "+s"(m));
    return (int)__builtin_amdgcn_mbcnt_hi(m, __builtin_amdgcn_mbcnt_lo(m, 0u));
}

// A wave-uniform 64-bit value read from lane 0 into scalar registers (a
// value formed from vector results would otherwise stay in a vector
// register pair across the step loop).
__device__ __forceinline__ int64_t uniform64(int64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double uniform_f64(double v)
{
    return __longlong_as_double(uniform64(__double_as_longlong(v)));
}

// Mask of the 256-bit segments [lo, hi] (0 <= lo <= hi <= 63).
__device__ __forceinline__ uint64_t seg_range(int lo, int hi)
{
    return (~0ull >> (63 - hi)) & (~0ull << lo);
}

// Step uniforms of steps kb .. kb + 63 (lane j: step kb + j), out of line:
// called once per 64 steps, and its logarithm's constants would otherwise be
// kept in registers across the step loop.
struct Uniforms64 {
    double logU1, U2;
};
__device__ __noinline__ Uniforms64 uniforms64(uint32_t cid, int64_t kb, uint64_t seed, int lane)
{
    Uniforms64 r;
    step::batch_uniforms(cid, kb, seed, lane, true, &r.logU1, &r.U2);
    return r;
}

// exp(-beta e) (shift = 0), else exp(min(-beta e, 0) - shift): the weights
// past the tables and those of a rescaled window (out of line, rare).
__device__ __noinline__ double exp_weight(double beta, int32_t e, double shift)
{
    if (shift == 0.0) return exp(-beta * (double)e);
    double l = -beta * (double)e;
    l = l < 0.0 ? l : 0.0;
    return exp(l - shift);
}

__device__ __noinline__ double exp_of(double x) { return exp(x); }

template <typename QT, int W, int G, bool INSTR>
__global__ __attribute__((amdgpu_flat_work_group_size(64 * W, 64 * W), amdgpu_waves_per_eu(waves_per_eu<W, G>())))
void wave_kernel(const StepArgs a)
{
    // A weight is the rounded product of its two table entries, summed as
    // such (no fused multiply-add into the sums), as in the step kernel.
#pragma clang fp contract(off)
    constexpr int BLOCK = 64 * W;
    constexpr int F = 4 * G;
    constexpr int NSEG = G * W;
    constexpr int NW = (F + 31) / 32;  // 32-bit state words (the last one partly used)
    static_assert(NSEG <= 64, "segment scan needs at most 64 segments");
    using step::read_lane;
    using step::small_scan;
    using step::wave_scan;

    // tab_lo[64 .. 128) = 0: the weight of a bit outside the window
    __shared__ double tab_lo[2 * kTabLo];
    __shared__ double tab_hi[kTabHi];
    // per-step exchanges, two buffers (even and odd steps): a wave may write
    // the next step's while another wave still reads this step's
    __shared__ double seg_sum[2][NSEG];
    __shared__ int32_t slow_part[2][W];
    __shared__ double mx_part[W];
    __shared__ int64_t xchg[2];
    // energy differences of the window's groups, per wave and slot (kOut
    // outside the window), and the inclusive scans of their four-bit sums
    __shared__ int4 eslot[W][kSlots][64];
    __shared__ double islot[W][kSlots][64];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = W > 1 ? __builtin_amdgcn_readfirstlane(tid >> 6) : 0;
    const int chain = a.chain_list ? a.chain_list[blockIdx.x] : a.chain_first + (int)blockIdx.x;
    const Problem P = a.problems[a.chain_problem[chain]];
    const int32_t N = P.N;
    const int64_t pitch = P.pitch;
    const int32_t n = P.n;
    const int s = P.s;
    const int64_t off = a.foff[chain];
    const double beta = a.beta[chain];
    const uint32_t cid = a.chain_id[chain];
    const uint64_t seed = a.seed;

    // Issue priority by chain size: a launch class ends with its slowest
    // chain, and with several classes on the device at once the chains of the
    // largest problems (the most waves and fields per chain, the fewest
    // chains per class) set the end of the step.
    __builtin_amdgcn_s_setprio(W >= 4 ? 3 : (W == 2 ? 2 : (G >= 16 ? 1 : 0)));

    for (int i = tid; i < 2 * kTabLo + kTabHi; i += BLOCK) {
        if (i < kTabLo) tab_lo[i] = exp(-beta * (double)i);
        else if (i < 2 * kTabLo) tab_lo[i] = 0.0;
        else tab_hi[i - 2 * kTabLo] = exp(-beta * (double)(kTabLo * (i - 2 * kTabLo)));
    }

    // ---- chain state: u = diag + s h and the bits, in registers ----
    int32_t u[F];
    uint32_t xw[NW];
#pragma unroll
    for (int i = 0; i < NW; ++i) xw[i] = 0u;
    int32_t* hbase = reinterpret_cast<int32_t*>(a.h) + off;
    const int32_t* dbase = reinterpret_cast<const int32_t*>(P.diag);
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t fb = ((int64_t)g * BLOCK + tid) * 4;
        if (fb < pitch) {
            const int4 hv = *reinterpret_cast<const int4*>(hbase + fb);
            const int4 dv = *reinterpret_cast<const int4*>(dbase + fb);
            const uint32_t xb4 = *reinterpret_cast<const uint32_t*>(a.x + off + fb);
            u[g * 4 + 0] = dv.x + s * hv.x;
            u[g * 4 + 1] = dv.y + s * hv.y;
            u[g * 4 + 2] = dv.z + s * hv.z;
            u[g * 4 + 3] = dv.w + s * hv.w;
#pragma unroll
            for (int v = 0; v < 4; ++v) xw[(g * 4 + v) >> 5] |= ((xb4 >> (8 * v)) & 1u) << ((g * 4 + v) & 31);
        } else {
#pragma unroll
            for (int v = 0; v < 4; ++v) u[g * 4 + v] = 0;
        }
    }

    // ---- chain scalars (wave-uniform) ----
    // (read into scalar registers: the arrays are written back at the end,
    // so the compiler loads them as vector values)
    int64_t k = uniform64(a.step[chain]);
    const int64_t kend = k + a.steps;
    int64_t E = uniform64(a.E[chain]);
    int64_t L = uniform64(a.L[chain]);
    int64_t sub = uniform64(a.sub[chain]);
    int32_t last_a = __builtin_amdgcn_readfirstlane(a.last_action[chain]);
    int64_t last_M = uniform64(a.last_M[chain]);
    int64_t last_E = uniform64(a.last_E[chain]);
    int64_t c_steps = 0, c_flips = 0, c_stays = 0, c_sat = 0, c_bad = 0;
    // running sum of M as the bits of a double in scalar registers (a
    // uniform double would otherwise take a vector register pair)
    int64_t c_sumM = 0;
    int32_t snap_n = 0;
    if constexpr (INSTR) snap_n = a.snap_every > 0 ? a.snap_count[chain] : 0;
    // window start (i n) mod N of set i = sub mod (number of sets); advanced
    // by n mod N per stay, which walks the same sets in the same order
    int32_t s0 = (int32_t)(((sub % P.num_sets) * (int64_t)n) % N);
    // p = S / n: for n = 2^j the product S 2^-j (exact scaling, the same
    // rounding as the division), formed from an integer exponent
    const bool n_pow2 = (n & (n - 1)) == 0;
    const int neg_log2n = -__builtin_ctz((unsigned)n);

    // The window: the 256-bit segments the cyclic window [st, st + n) meets
    // and the groups of this wave among them.  Bit f of the lane is in the
    // window iff f < N and (f - st) mod N < n.  With d = f - st =
    // wbase + (4 BLOCK g + v) that is 0 <= d < min(n, N - st) (the part up to
    // the end of the bits) or d < n - N (the part wrapped to the start); both
    // bounds are values of the window rather than of the bit, so that no
    // per-bit constant is kept live across the steps.
    uint64_t smask = 0, gmask = 0;
    int32_t wbase = 0;
    uint32_t wlo = 0;
    const int32_t wneg = n - N;
    auto set_window = [&](int32_t st) {
        wbase = (wave * 64 + lane_here()) * 4 - st;
        wlo = (uint32_t)__builtin_amdgcn_readfirstlane(n < N - st ? n : N - st);
        const int32_t e0 = st + n < N ? st + n : N;
        uint64_t m = seg_range(st >> 8, (e0 - 1) >> 8);
        if (st + n > N) m |= seg_range(0, (st + n - N - 1) >> 8);
        smask = m;
        if constexpr (W == 1) {
            gmask = m;
        } else {
            uint64_t gm = 0;
#pragma unroll
            for (int g = 0; g < G; ++g) gm |= ((m >> (g * W + wave)) & 1ull) << g;
            gmask = gm;
        }
    };
    set_window(s0);

    __syncthreads();  // tables ready

    int64_t ub_base = k;
    Uniforms64 ub = uniforms64(cid, ub_base, seed, lane);

    // weight of a bit from its slot value: tables below 64 x 1024, else the
    // exponential; shift != 0 (rescaled window): exp(min(-beta e, 0) - shift)
    auto weight_of = [&](int32_t e, double shift) -> double {
        const bool in = e != kOut;
        if (shift != 0.0) return in ? exp_weight(beta, e, shift) : 0.0;
        const uint32_t ep = e > 0 ? (uint32_t)e : 0u;
        if (in && ep >= (uint32_t)kTabMax) return exp_weight(beta, e, 0.0);
        const uint32_t hi = ep >> 6 < (uint32_t)kTabHi ? ep >> 6 : (uint32_t)(kTabHi - 1);
        return tab_hi[hi] * tab_lo[in ? (ep & 63u) : (uint32_t)kTabLo];
    };
    auto slot_sum = [&](const int4 ev, double shift, double (&w4)[4]) -> double {
        w4[0] = weight_of(ev.x, shift);
        w4[1] = weight_of(ev.y, shift);
        w4[2] = weight_of(ev.z, shift);
        w4[3] = weight_of(ev.w, shift);
        return ((w4[0] + w4[1]) + w4[2]) + w4[3];
    };
    // segment totals of the window (lane j: segment j) after this wave's
    // totals were written to seg_sum
    auto read_totals = [&]() -> double {
        if constexpr (W > 1) __syncthreads();
        // (one wave: its own LDS accesses complete in order)
        return lane < NSEG && ((smask >> lane) & 1ull) ? seg_sum[k & 1][lane] : 0.0;
    };
    // the window's sums again from the slots (rare paths)
    auto slot_totals = [&](double shift) -> double {
        if constexpr (W > 1) __syncthreads();  // every wave has read this step's totals
        uint64_t gm = gmask;
        int r = 0;
        while (gm && r < kSlots) {
            const int g = __builtin_ctzll(gm);
            gm &= gm - 1;
            double w4[4];
            const double ls = slot_sum(eslot[wave][r][lane], shift, w4);
            const double inc = wave_scan(ls);
            islot[wave][r][lane] = inc;
            if (lane == 63) seg_sum[k & 1][g * W + wave] = inc;
            ++r;
        }
        return read_totals();
    };

    for (; k < kend; ++k) {
        if (k - ub_base >= 64) {
            ub_base = k;
            // the key as a value of this iteration: the Philox round keys are
            // then formed here, once per 64 steps, instead of being kept live
            // in registers across the whole loop
            uint32_t key_lo = (uint32_t)seed, key_hi = (uint32_t)(seed >> 32);
            asm volatile("" : "+s"(key_lo), "+s"(key_hi));
            ub = uniforms64(cid, ub_base, ((uint64_t)key_hi << 32) | key_lo, lane);
        }
        const int uj = (int)(k - ub_base);
        const double U2 = read_lane(ub.U2, uj);
        const double logU1 = read_lane(ub.logU1, uj);

        // ---- S: window weights from the tables, four-bit sums, segment
        // scans; the energy differences go to the slots ----
        bool big = false;  // a window bit of this lane past the tables
        // one wave: the sum of the window's segment totals in segment order
        // (used when there are at most two, where it is what the segment
        // scan gives)
        double S2 = 0.0;
        {
            int r = 0;
            auto weigh = [&](auto gc) {
                constexpr int g = decltype(gc)::value;
                {
                    int32_t es[4];
                    double w4[4];
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int i = g * 4 + v;
                        const int32_t d = wbase + (g * BLOCK * 4 + v);
                        const bool in = (uint32_t)d < wlo || d < wneg;
                        // dE = (1 - 2 x) u: the bit as a sign mask (0 or -1)
                        const int32_t sm = __builtin_amdgcn_sbfe((int32_t)xw[i >> 5], i & 31, 1);
                        const int32_t e = (u[i] ^ sm) - sm;
                        es[v] = in ? e : kOut;
                        big |= in && e >= (int32_t)kTabMax;
                        // table index of max(dE, 0), clamped below kTabMax (a
                        // window weight past the tables is recomputed: big)
                        const uint32_t ep = (uint32_t)max(0, min(e, (int32_t)kTabMax - 1));
                        w4[v] = tab_hi[ep >> 6] * tab_lo[in ? (ep & 63u) : (uint32_t)kTabLo];
                    }
                    const double ls = ((w4[0] + w4[1]) + w4[2]) + w4[3];
                    const double inc = wave_scan(ls);
                    // (r < kSlots for every window the host lets run here)
                    if (r < kSlots) {
                        eslot[wave][r][lane] = make_int4(es[0], es[1], es[2], es[3]);
                        islot[wave][r][lane] = inc;
                    }
                    if (lane == 63) seg_sum[k & 1][g * W + wave] = inc;
                    if constexpr (W == 1) S2 = S2 + read_lane(inc, 63);
                    ++r;
                }
            };
            // the groups the window meets, tested four at a time
            for_each_index(std::make_integer_sequence<int, (G + 3) / 4>{}, [&](auto qc) {
                constexpr int q = decltype(qc)::value;
                if ((gmask >> (4 * q)) & 0xFull) {
                    for_each_index(std::make_integer_sequence<int, 4>{}, [&](auto vc) {
                        constexpr int g = 4 * q + decltype(vc)::value;
                        if constexpr (g < G) {
                            if ((gmask >> g) & 1ull) weigh(std::integral_constant<int, g>{});
                        }
                    });
                }
            });
        }
        bool slow = __ballot(big) != 0;
        if constexpr (W > 1) {
            if (lane == 0) slow_part[k & 1][wave] = slow ? 1 : 0;
        }
        // one wave and at most two segments: S from the pass, and the
        // segment scan only when the chain moves
        const bool fast_S = W == 1 && __builtin_popcountll(smask) <= 2;
        double sv = fast_S ? 0.0 : read_totals();
        if constexpr (W > 1) {
            int any = 0;
#pragma unroll
            for (int ww = 0; ww < W; ++ww) any |= slow_part[k & 1][ww];
            slow = any != 0;
        }
        double sinc = 0.0, S = S2;
        bool scanned = false;
        // a weight past the tables: the window's sums with the exponential
        if (slow) sv = slot_totals(0.0);
        if (slow || !fast_S) {
            sinc = small_scan<NSEG>(sv);
            S = read_lane(sinc, NSEG - 1);
            scanned = true;
        }
        double mx = 0.0;
        bool scaled = false;
        if (S < 0x1p-1000) {
            // every weight underflowed: rescale by the largest log-weight
            double lm = -INFINITY;
            const int nslots = min(__builtin_popcountll(gmask), kSlots);
            for (int r = 0; r < nslots; ++r) {
                const int4 ev = eslot[wave][r][lane];
                const int32_t e4[4] = {ev.x, ev.y, ev.z, ev.w};
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    double l = -beta * (double)e4[v];
                    l = l < 0.0 ? l : 0.0;
                    if (e4[v] != kOut) lm = fmax(lm, l);
                }
            }
            lm = step::wave_max(lm);
            if constexpr (W > 1) {
                if (lane == 0) mx_part[wave] = lm;
                __syncthreads();
                lm = -INFINITY;
                for (int ww = 0; ww < W; ++ww) lm = fmax(lm, mx_part[ww]);
            }
            mx = lm;
            scaled = true;
            sv = slot_totals(mx);
            sinc = small_scan<NSEG>(sv);
            S = read_lane(sinc, NSEG - 1);
            scanned = true;
        }

        // ---- p, M and the budget decision of Alg 6 (uniform) ----
        const double Ss = scaled ? exp_of(mx) * S : S;
        // (uniform: the branches on p below are then scalar branches)
        const double p = uniform_f64(n_pow2 ? ldexp(Ss, neg_log2n) : Ss / (double)n);
        double q;
        if (p >= 1.0) q = 0.0;
        else if (p <= 0.0) q = INFINITY;
        else q = step::geometric_quotient(logU1, p, (double)L);
        const bool stay = __builtin_amdgcn_readfirstlane((int)(q >= (double)L)) != 0;

        const int64_t Erec = E;
        const int64_t Lrec = L;
        bool snap = false;
        if constexpr (INSTR) {
            snap = a.snap_every > 0 && ((k + 1) % a.snap_every) == 0;
            if (snap) {
                const int32_t slot = snap_n % a.snap_cap;
                uint8_t* sx = a.snap_x + ((int64_t)chain * a.snap_cap + slot) * a.snap_pitch;
                int tid_s = tid;  // (opaque: no per-group address kept across the loop)
                asm volatile("" : "+v"(tid_s));
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const int64_t fb = ((int64_t)g * BLOCK + tid_s) * 4;
                    if (fb < a.snap_pitch) {
                        uint32_t wv = 0;
#pragma unroll
                        for (int v = 0; v < 4; ++v) wv |= get_bit(xw, g * 4 + v) << (8 * v);
                        *reinterpret_cast<uint32_t*>(sx + fb) = wv;
                    }
                }
                ++snap_n;
            }
        }

        int32_t action = -1;
        int64_t M;
        // the row of a move and, for 16-bit coefficients, the multiplier of
        // its update, which runs after the two paths join (defined on both,
        // so that the fields are not copied to other registers and back)
        decltype(step::load_raw4(static_cast<const QT*>(nullptr))) raw[G];
        [[maybe_unused]] int32_t mult = 0;
        if (stay) {
            // stay L times and move to the next systematic set
            M = L;
            L = uniform64(P.L0);
            ++sub;
            s0 += n;
            s0 -= s0 >= N ? N : 0;
            set_window(s0);
            ++c_stays;
            // (the fields stay where the move path updates them in place)
#pragma unroll
            for (int i = 0; i < F; ++i) asm volatile("" : "+v"(u[i]));
            if constexpr (sizeof(QT) == 2) {
                // (no row: the registers as they are, unused on this path)
#pragma unroll
                for (int g = 0; g < G; ++g) asm volatile("" : "=v"(raw[g].x), "=v"(raw[g].y));
            }
        } else {
            // ---- proportional choice (appendix "How to Sample
            // Proportionally"): first bit of the window, in bit order, whose
            // running sum exceeds U2 S; segment -> lane -> bit ----
            if (!scanned) {
                sv = read_totals();
                sinc = small_scan<NSEG>(sv);
            }
            const double t = U2 * S;
            const bool pos_seg = lane < NSEG && sv > 0.0;
            const uint64_t bseg = __ballot(pos_seg && sinc > t);
            const uint64_t bpos = __ballot(pos_seg);
            int jstar = bseg ? __builtin_ctzll(bseg) : (bpos ? 63 - __builtin_clzll(bpos) : 0);
            jstar = jstar < NSEG ? jstar : NSEG - 1;
            const int gstar = jstar / W, wstar = jstar % W;
            int64_t selc = 0, seld = 0;
            if (wave == wstar) {
                const double base = jstar > 0 ? read_lane(sinc, jstar - 1) : 0.0;
                const int rstar = min(__builtin_popcountll(gmask & ((1ull << gstar) - 1ull)), kSlots - 1);
                const int4 ev = eslot[wave][rstar][lane];
                double w4[4];
                double my_ls;
                if (!slow && !scaled) {
                    // every window weight from the tables: the pass's
                    // branch-free lookups (the same products)
                    const int32_t e4[4] = {ev.x, ev.y, ev.z, ev.w};
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const uint32_t ep = (uint32_t)max(0, min(e4[v], (int32_t)kTabMax - 1));
                        w4[v] = tab_hi[ep >> 6] * tab_lo[e4[v] != kOut ? (ep & 63u) : (uint32_t)kTabLo];
                    }
                    my_ls = ((w4[0] + w4[1]) + w4[2]) + w4[3];
                } else {
                    my_ls = slot_sum(ev, scaled ? mx : 0.0, w4);
                }
                // (the scan of these sums, kept when the totals were formed)
                const double my_inc = islot[wave][rstar][lane];
                const double Gl = base + my_inc;
                const uint64_t bl = __ballot(my_ls > 0.0 && Gl > t);
                const uint64_t blp = __ballot(my_ls > 0.0);
                const int lstar = bl ? __builtin_ctzll(bl) : (blp ? 63 - __builtin_clzll(blp) : 0);
                const double prev_l = read_lane(my_inc, lstar > 0 ? lstar - 1 : 0);
                double run = lstar > 0 ? base + prev_l : base;
                int vstar = -1, vlast = -1;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    if (w4[v] > 0.0) {
                        vlast = v;
                        run += w4[v];
                        if (vstar < 0 && run > t) vstar = v;
                    }
                }
                if (vstar < 0) vstar = vlast;
                // no positive weight in the chosen lane cannot happen when
                // S > 0; keep the address in range and report it
                int64_t bad = 0;
                if (vstar < 0) {
                    vstar = 0;
                    bad = 1;
                }
                const int32_t ec = vstar == 0 ? ev.x : (vstar == 1 ? ev.y : (vstar == 2 ? ev.z : ev.w));
                int64_t c = ((int64_t)gstar * BLOCK + wave * 64 + lane_here()) * 4 + vstar;
                if (c >= N) {
                    c = 0;
                    bad = 1;
                }
                const int ib = gstar * 4 + vstar;
                uint32_t xword = xw[0];
#pragma unroll
                for (int i = 1; i < NW; ++i) xword = (ib >> 5) == i ? xw[i] : xword;
                const uint32_t xbit = (xword >> (ib & 31)) & 1u;
                const int64_t packed = c | ((int64_t)xbit << 40) | (bad << 41);
                const int lo = __builtin_amdgcn_readlane((int)(uint32_t)packed, lstar);
                const int hi = __builtin_amdgcn_readlane((int)(packed >> 32), lstar);
                selc = (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
                seld = __builtin_amdgcn_readlane(ec, lstar);
                if constexpr (W > 1) {
                    if (lane == 0) {
                        xchg[0] = selc;
                        xchg[1] = seld;
                    }
                }
            }
            if constexpr (W > 1) {
                // (the next write of xchg follows the next step's segment
                // barrier, which every wave passes after these reads)
                __syncthreads();
                selc = uniform64(xchg[0]);
                seld = uniform64(xchg[1]);
            }
            const int32_t c = (int32_t)(selc & 0xFFFFFFFFll);
            const bool xc = (selc >> 40) & 1;
            c_bad = uniform64(c_bad + ((selc >> 41) & 1));
            // ---- move: flip c, E += dE_c, u_j += s (1 - 2 x_c) A[c][j] ----
            // (lanes past the pitch read on into the next rows or the
            // matrix's tail padding and drop what they read)
            const QT* row = reinterpret_cast<const QT*>(P.A) + (int64_t)c * pitch + (wave * 64 + lane_here()) * 4;
#pragma unroll
            for (int g = 0; g < G; ++g) raw[g] = step::load_raw4(row + g * BLOCK * 4);
            const int cl = (c >> 2) % BLOCK;
            const int ci = ((c >> 2) / BLOCK) * 4 + (c & 3);
            if (wave * 64 + lane_here() == cl) {
#pragma unroll
                for (int i = 0; i < NW; ++i)
                    if ((ci >> 5) == i) xw[i] ^= 1u << (ci & 31);
            }
            E = uniform64(E + seld);
            // M = 1 + floor(q) (formed on this path only: a stay takes M = L)
            const bool sat = __builtin_amdgcn_readfirstlane((int)!(q < 0x1p63)) != 0;
            const int64_t m = uniform64(sat ? INT64_MAX : (int64_t)floor(q) + 1);
            L = uniform64(L - m);
            c_sat = uniform64(c_sat + (sat ? 1 : 0));
            M = m;
            action = c;
            ++c_flips;
            if constexpr (sizeof(QT) == 2) {
                mult = __builtin_amdgcn_readfirstlane(xc ? -s : s);
            } else {
                const int sh = s - 1;
                if (xc) {
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        const auto r = step::widen4(raw[g]);
#pragma unroll
                        for (int v = 0; v < 4; ++v) u[g * 4 + v] -= r.v[v] << sh;
                    }
                } else {
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        const auto r = step::widen4(raw[g]);
#pragma unroll
                        for (int v = 0; v < 4; ++v) u[g * 4 + v] += r.v[v] << sh;
                    }
                }
            }
        }
        if constexpr (sizeof(QT) == 2) {
            if (!stay) {
                // 16-bit coefficients times +-1 or +-2: one two-term 16-bit
                // dot product per field, accumulated in place (the pair of
                // coefficients against (mult, 0) or (0, mult))
                const v2i16 mlo = {(int16_t)mult, 0}, mhi = {0, (int16_t)mult};
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    const v2i16 p0 = __builtin_bit_cast(v2i16, raw[g].x);
                    const v2i16 p1 = __builtin_bit_cast(v2i16, raw[g].y);
                    u[g * 4 + 0] = __builtin_amdgcn_sdot2(p0, mlo, u[g * 4 + 0], false);
                    u[g * 4 + 1] = __builtin_amdgcn_sdot2(p0, mhi, u[g * 4 + 1], false);
                    u[g * 4 + 2] = __builtin_amdgcn_sdot2(p1, mlo, u[g * 4 + 2], false);
                    u[g * 4 + 3] = __builtin_amdgcn_sdot2(p1, mhi, u[g * 4 + 3], false);
                }
            }
        }
        ++c_steps;
        c_sumM = uniform64(__double_as_longlong(__longlong_as_double(c_sumM) + (double)M));
        last_a = action;
        last_M = M;
        last_E = Erec;
        if constexpr (INSTR) {
            double wrb = 1.0;
            if (snap || a.log_cap > 0) wrb = step::expected_multiplicity(p, Lrec, true);
            if (tid == 0) {
                if (a.log_cap > 0) {
                    const int64_t slot = (int64_t)chain * a.log_cap + (k % a.log_cap);
                    a.log_action[slot] = action;
                    a.log_M[slot] = M;
                    a.log_E[slot] = Erec;
                    a.log_p[slot] = p;
                    a.log_w[slot] = wrb;
                }
                if (snap) {
                    const int32_t slot = (snap_n - 1) % a.snap_cap;
                    a.snap_M[(int64_t)chain * a.snap_cap + slot] = M;
                    a.snap_E[(int64_t)chain * a.snap_cap + slot] = Erec;
                    a.snap_w[(int64_t)chain * a.snap_cap + slot] = wrb;
                }
            }
        }
    }

    // ---- chain state back to memory: h = (u - diag) / s ----
    // (the lane index, pitch and bases made opaque here, so that the
    // per-group addresses and bounds of the loads above are not kept live
    // across the step loop for these stores)
    int tid_e = tid;
    int64_t pitch_e = pitch;
    int32_t* hbase_e = hbase;
    const int32_t* dbase_e = dbase;
    uint8_t* xbase_e = a.x + off;
    asm volatile("" : "+v"(tid_e), "+s"(pitch_e), "+s"(hbase_e), "+s"(dbase_e), "+s"(xbase_e));
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const int64_t fb = ((int64_t)g * BLOCK + tid_e) * 4;
        if (fb < pitch_e) {
            const int4 dv = *reinterpret_cast<const int4*>(dbase_e + fb);
            const int32_t dd[4] = {dv.x, dv.y, dv.z, dv.w};
            int32_t hv[4];
            uint32_t xb4 = 0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int32_t t = u[g * 4 + v] - dd[v];
                hv[v] = s == 2 ? (t >> 1) : t;
                xb4 |= get_bit(xw, g * 4 + v) << (8 * v);
            }
            *reinterpret_cast<int4*>(hbase_e + fb) = make_int4(hv[0], hv[1], hv[2], hv[3]);
            *reinterpret_cast<uint32_t*>(xbase_e + fb) = xb4;
        }
    }
    if (tid == 0) {
        a.step[chain] = k;
        a.E[chain] = E;
        a.L[chain] = L;
        a.sub[chain] = sub;
        a.last_action[chain] = last_a;
        a.last_M[chain] = last_M;
        a.last_E[chain] = last_E;
        if constexpr (INSTR) {
            if (a.snap_every > 0) a.snap_count[chain] = snap_n;
        }
        int64_t* cn = a.counters + (int64_t)chain * 6;
        cn[0] += c_steps;
        cn[1] += c_flips;
        cn[2] += c_stays;
        cn[3] += c_sat;
        cn[4] = __double_as_longlong(__longlong_as_double(cn[4]) + __longlong_as_double(c_sumM));
        cn[5] += c_bad;
    }
}

template <typename QT, int W, int G, bool INSTR>
hipError_t launch_one(int32_t grid, hipStream_t st, const StepArgs& a)
{
    hipLaunchKernelGGL((wave_kernel<QT, W, G, INSTR>), dim3(grid), dim3(64 * W), 0, st, a);
    return hipGetLastError();
}

// Tiles of the window kernel (workgroup size, 4-bit groups per lane): one
// wave from 512 up to 6144 bits, two up to 12288, four up to 16384 (at most
// 96 fields per lane: more do not fit the registers of two waves per SIMD).
#define PNS_WAVE_TILE_LIST(X, QT) \
    X(QT, 64, 2)                  \
    X(QT, 64, 4)                  \
    X(QT, 64, 8)                  \
    X(QT, 64, 16)                 \
    X(QT, 64, 24)                 \
    X(QT, 128, 16)                \
    X(QT, 128, 24)                \
    X(QT, 256, 16)

#define PNS_WAVE_DISPATCH_TILE(QT, B, GG)                                                              \
    if (block == B && groups == GG) {                                                                  \
        if (probe) return hipSuccess;                                                                  \
        return instr ? wave::launch_one<QT, B / 64, GG, true>(grid, st, a)                             \
                     : wave::launch_one<QT, B / 64, GG, false>(grid, st, a);                           \
    }

}  // namespace wave
}  // namespace pns
