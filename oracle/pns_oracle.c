/*
 * Reference oracle for Partial Neighbor Search sampling on QUBO targets.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load this file's library.  The product
 * path (the HIP library and its Python binding) never links, imports or calls
 * it, and this file shares no code, header, table or constant generator with
 * the product path.
 *
 * A deliberately plain, slow, single-threaded implementation in FP64 / int64
 * of what the paper computes:
 *   - Rejection-Free for the discrete case (Alg 2, Sec 1.2, eqs. (1)-(2));
 *   - Basic Partial Neighbor Search (Alg 3, Sec 2), with the proposal of a
 *     step restricted to a fresh random subset and normalised on it;
 *   - Unbiased Partial Neighbor Search (Alg 6, Sec 3.2), with L0-original-
 *     sample blocks per partial neighbor set, systematic or random sets
 *     (Sec 5);
 *   - on the QUBO target of Sec 4 with single-bit-flip neighbours and a
 *     uniform proposal 1/N (so the proposal cancels in every ratio);
 *   - Unbiased PNS for continuous states (Alg 7) on the donut target of
 *     Sec 7 (orc_cont_run, at the end of this file);
 *   - proportional choice by the inverse-CDF rule of the appendix "How to
 *     Sample Proportionally" (first index whose running sum exceeds U times
 *     the total).
 * Conventions (each one a reading of the paper where it is silent):
 *   - target pi_beta(x) proportional to exp(-beta * x^T Q x); the paper's
 *     pi(x) = exp{x^T Q x} is beta = 1 with Q replaced by -Q;
 *   - Q is given either symmetric (full matrix) or upper triangular
 *     (only entries i <= j are read), as Sec 4 allows both;
 *   - a subset is scanned in increasing bit index;
 *   - multiplicity M = 1 + G with G counting failures (M = 1 when p = 1,
 *     as in Example 1 of Sec 2.1);
 *   - in Basic PNS p is the average of the subset's acceptance
 *     probabilities (proposal normalised on the subset, Sec 2);
 *   - random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11),
 *     written here from its published definition.
 * Energies, local fields and multiplicities are exact (int64) for integer Q;
 * everything else is IEEE double.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MODE_RF 0
#define ORC_MODE_BASIC 1
#define ORC_MODE_UNBIASED_SYS 2
#define ORC_MODE_UNBIASED_RAND 3
/* Optimization Rejection-Free (Alg 9, n = N) and Optimization PNS (Alg 10,
 * a fresh uniformly random n-subset every step, the subset rule of Alg 3):
 * the jump chain with acceptance min{1, [pi(y)/pi(x)]^(1/T)} at a constant
 * temperature T, no multiplicity, and the best state X_max kept. */
#define ORC_MODE_OPT 4

#define ORC_LAYOUT_SYMMETRIC 0
#define ORC_LAYOUT_UPPER 1

#define ORC_STAY (-1)

/* ------------------------------------------------------------------------- */
/* Philox4x32-10, from the description in Salmon et al., SC'11, Sec 3.3:      */
/* each round multiplies counter words 0 and 2 by two fixed odd constants,    */
/* swaps/xors the high and low halves with the other two words and the key,  */
/* and the key is bumped by two Weyl constants between rounds.                */
/* ------------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Counter layout: (chain id, step low word, step high word, stream word). */
static void draw4(uint64_t seed, uint32_t chain, uint64_t step, uint32_t stream, uint32_t out[4])
{
    uint32_t ctr[4] = {chain, (uint32_t)step, (uint32_t)(step >> 32), stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* 53 random bits from two words: ((hi << 32) | lo) >> 11. */
static uint64_t bits53(uint32_t hi, uint32_t lo)
{
    return (((uint64_t)hi << 32) | (uint64_t)lo) >> 11;
}

/* Uniform on (0, 1] from words 0 and 1; uniform on [0, 1) from words 2, 3. */
void orc_uniforms(uint64_t seed, uint32_t chain, uint64_t step, double* u_open_closed, double* u_closed_open)
{
    uint32_t w[4];
    draw4(seed, chain, step, 0u, w);
    *u_open_closed = (double)(bits53(w[0], w[1]) + 1u) * 0x1p-53;
    *u_closed_open = (double)bits53(w[2], w[3]) * 0x1p-53;
}

/* Uniformly random n-subset of {0..N-1} (Sec 2 "random subset", Sec 5 random
 * partial neighbor sets): take a stream of i.i.d. uniform indices and keep the
 * first n distinct values.  Candidate s uses stream word 0x40000000 | (s/2),
 * words (0,1) for even s and (2,3) for odd s, mapped to an index as
 * floor(u64 * N / 2^64).  n == N takes every index without drawing. */
void orc_random_subset(uint64_t seed, uint32_t chain, uint64_t step, int32_t N, int32_t n, uint8_t* member)
{
    memset(member, 0, (size_t)N);
    if (n >= N) {
        memset(member, 1, (size_t)N);
        return;
    }
    int32_t distinct = 0;
    for (uint32_t s = 0; distinct < n; ++s) {
        uint32_t w[4];
        draw4(seed, chain, step, 0x40000000u | (s >> 1), w);
        uint32_t hi = (s & 1u) ? w[2] : w[0];
        uint32_t lo = (s & 1u) ? w[3] : w[1];
        uint64_t u = ((uint64_t)hi << 32) | (uint64_t)lo;
        int32_t cand = (int32_t)(((unsigned __int128)u * (unsigned __int128)(uint64_t)N) >> 64);
        if (!member[cand]) {
            member[cand] = 1;
            ++distinct;
        }
    }
}

/* Systematic partial neighbor set i (Sec 4 halves; Sec 5 wrap-around sets
 * for n not dividing N): bits (i*n + t) mod N for t = 0..n-1. */
void orc_sys_subset(int32_t N, int32_t n, int64_t i, uint8_t* member)
{
    memset(member, 0, (size_t)N);
    int64_t start = (int64_t)(((__int128)i * n) % N);
    for (int32_t t = 0; t < n; ++t) member[(start + t) % N] = 1;
}

static int64_t gcd64(int64_t a, int64_t b)
{
    while (b) {
        int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

/* Number of distinct systematic sets: N / gcd(N, n). */
int64_t orc_sys_count(int32_t N, int32_t n)
{
    return (int64_t)N / gcd64(N, n);
}

/* Bernoulli(1/2) initial bit j of a chain: stream 0x20000000 | (j / 128),
 * word (j / 32) mod 4, bit j mod 32, step 0. */
void orc_random_state(uint64_t seed, uint32_t chain, int32_t N, uint8_t* x)
{
    for (int32_t j = 0; j < N; ++j) {
        uint32_t w[4];
        draw4(seed, chain, 0, 0x20000000u | ((uint32_t)j >> 7), w);
        x[j] = (uint8_t)((w[((uint32_t)j >> 5) & 3u] >> ((uint32_t)j & 31u)) & 1u);
    }
}

/* ------------------------------------------------------------------------- */
/* QUBO energy and local fields (Sec 4, pi(x) = exp{x^T Q x}).                */
/* ------------------------------------------------------------------------- */

/* Coefficient c(i, j) of x_i x_j in x^T Q x for i != j, counting both orders:
 * symmetric Q -> Q_ij + Q_ji = 2 Q_ij; upper triangular Q -> Q_min,max. */
static int64_t pair_coef_i(const int64_t* Q, int32_t N, int32_t layout, int32_t i, int32_t j)
{
    if (layout == ORC_LAYOUT_SYMMETRIC) return Q[(size_t)i * N + j] + Q[(size_t)j * N + i];
    return i < j ? Q[(size_t)i * N + j] : Q[(size_t)j * N + i];
}

static double pair_coef_f(const double* Q, int32_t N, int32_t layout, int32_t i, int32_t j)
{
    if (layout == ORC_LAYOUT_SYMMETRIC) return 2.0 * Q[(size_t)i * N + j];
    return i < j ? Q[(size_t)i * N + j] : Q[(size_t)j * N + i];
}

/* x^T Q x written out as a double sum over the entries the layout defines. */
int64_t orc_energy_i(const int64_t* Q, int32_t N, int32_t layout, const uint8_t* x)
{
    int64_t e = 0;
    for (int32_t i = 0; i < N; ++i) {
        if (!x[i]) continue;
        for (int32_t j = 0; j < N; ++j) {
            if (!x[j]) continue;
            if (layout == ORC_LAYOUT_UPPER && j < i) continue;
            e += Q[(size_t)i * N + j];
        }
    }
    return e;
}

double orc_energy_f(const double* Q, int32_t N, int32_t layout, const uint8_t* x)
{
    double e = 0.0;
    for (int32_t i = 0; i < N; ++i) {
        if (!x[i]) continue;
        for (int32_t j = 0; j < N; ++j) {
            if (!x[j]) continue;
            if (layout == ORC_LAYOUT_UPPER && j < i) continue;
            e += Q[(size_t)i * N + j];
        }
    }
    return e;
}

/* ------------------------------------------------------------------------- */
/* Chain simulation.                                                         */
/* ------------------------------------------------------------------------- */

typedef struct {
    /* problem */
    int32_t N;
    int32_t is_int;           /* 1: Qi (int64) is used, 0: Qf (double) */
    int32_t layout;           /* ORC_LAYOUT_* */
    const int64_t* Qi;        /* N*N row-major */
    const double* Qf;         /* N*N row-major */
    /* method */
    int32_t mode;             /* ORC_MODE_* */
    int32_t n;                /* subset size (ignored for RF) */
    int64_t L0;               /* block length in original samples (Unbiased) */
    uint64_t seed;
    /* chains */
    int32_t num_chains;
    const uint32_t* chain_ids;  /* [num_chains] counter word 0 of each chain */
    const double* betas;        /* [num_chains] */
    const uint8_t* x0;          /* [num_chains][N] */
    int64_t K;                  /* steps (records) per chain */
    int64_t step0;              /* index of the first step (for resumed runs) */
    /* per-step outputs [num_chains][K], each may be NULL */
    int32_t* log_action;        /* flipped bit, or ORC_STAY */
    int64_t* log_M;             /* multiplicity of the record */
    int64_t* log_Ei;            /* energy of the record's state (integer Q) */
    double* log_Ef;             /* energy of the record's state (double) */
    double* log_p;              /* escape probability p */
    double* log_q;              /* log(U1) / log1p(-p) (+inf when p == 0) */
    double* log_tmargin;        /* distance of U2*S to the chosen interval's ends, / S */
    /* final state outputs, each may be NULL */
    uint8_t* x_final;           /* [num_chains][N] */
    int64_t* hi_final;          /* [num_chains][N] local fields (integer Q) */
    double* hf_final;           /* [num_chains][N] local fields (double Q) */
    int64_t* Ei_final;          /* [num_chains] */
    double* Ef_final;           /* [num_chains] */
    int64_t* L_final;           /* [num_chains] remaining budget */
    int64_t* sub_final;         /* [num_chains] systematic set index */
    /* multiplicity-weighted and visit histograms over 2^N states, N <= 24 */
    uint64_t* hist_w;
    uint64_t* hist_v;
    int64_t hist_from;          /* first step index counted */
    /* counters [num_chains], each may be NULL */
    int64_t* n_flips;
    int64_t* n_stays;
    int64_t* n_saturated;
    /* ORC_MODE_OPT: temperature T > 0 and the best state X_max of each chain
     * (outputs may be NULL) */
    double temperature;
    uint8_t* x_best;            /* [num_chains][N] */
    int64_t* Ei_best;           /* [num_chains] */
    double* Ef_best;            /* [num_chains] */
    /* RF / Basic: advance each chain by exactly orig_time original samples
     * (0 = off): the records run until the multiplicities reach orig_time,
     * the last one cut to the remaining time (the budget rule of Alg 6 used
     * as a stopping time); n_records receives each chain's record count.
     * step0s, if not NULL, gives each chain's first step index. */
    int64_t orig_time;
    int64_t* n_records;         /* [num_chains] */
    const int64_t* step0s;      /* [num_chains] */
    /* Rao-Blackwell weights (Thm 3 (2), (5)): the expected multiplicity of
     * each record given its state, subset and budget, per step
     * ([num_chains][K]) and summed per state ([2^N], N <= 24, from
     * hist_from on); each may be NULL */
    double* log_w;
    double* hist_rb;
    /* Replay: follow another implementation's records (rp_action, rp_M
     * [num_chains][K], or NULL for a plain run).  Every step still derives
     * the oracle's own decision from its own state and draws (logged in
     * log_action / log_M), classifies the given record against it into
     * rp_class [num_chains][K] (see orc_replay_class), and then continues
     * from the given record's decision, so that every later record, the
     * energies, p and the final state are derived along the given
     * trajectory.  rp_tol is the relative tolerance on p between the two
     * implementations that sets the width of the decision windows. */
    const int32_t* rp_action;
    const int64_t* rp_M;
    int32_t* rp_class;
    double rp_tol;
} orc_run_args;

/* Expected multiplicity of a record (Thm 3 (2)): M = 1 + G with G a
 * geometric number of failures of success probability p, so
 * P(M >= m) = (1 - p)^(m - 1), and for a record cut at a remaining budget L
 * (Alg 6) the recorded value is min(M, L).  Its mean is the sum over m >= 1
 * of P(min(M, L) >= m), added term by term up to m = L (L < 0: no budget;
 * the infinite series then sums to 1 / p).  Terms below 2^-60 of the running
 * sum are dropped. */
double orc_expected_multiplicity(double p, int64_t L)
{
    if (p >= 1.0) return 1.0;
    if (p <= 0.0) return L < 0 ? INFINITY : (double)L;
    if (L < 0) return 1.0 / p;
    double sum = 0.0, term = 1.0;
    for (int64_t m = 1; m <= L; ++m) {
        sum += term;
        term *= 1.0 - p;
        if (term < sum * 0x1p-60) break;
    }
    return sum;
}

/* Local field of bit j: the part of dE_j that depends on the other bits,
 * h_j = sum_{i != j} c(i, j) x_i / s where s = 2 for symmetric Q (so that
 * dE_j = (1 - 2 x_j)(Q_jj + 2 h_j) as in the symmetric form) and s = 1 for
 * upper-triangular Q (dE_j = (1 - 2 x_j)(Q_jj + h_j)). */
static void fields_init(const orc_run_args* a, const uint8_t* x, int64_t* hi, double* hf)
{
    int32_t N = a->N;
    for (int32_t j = 0; j < N; ++j) {
        if (a->is_int) {
            int64_t acc = 0;
            for (int32_t i = 0; i < N; ++i) {
                if (i == j || !x[i]) continue;
                acc += a->layout == ORC_LAYOUT_SYMMETRIC ? a->Qi[(size_t)j * N + i]
                                                         : pair_coef_i(a->Qi, N, a->layout, i, j);
            }
            hi[j] = acc;
        } else {
            double acc = 0.0;
            for (int32_t i = 0; i < N; ++i) {
                if (i == j || !x[i]) continue;
                acc += a->layout == ORC_LAYOUT_SYMMETRIC ? a->Qf[(size_t)j * N + i]
                                                         : pair_coef_f(a->Qf, N, a->layout, i, j);
            }
            hf[j] = acc;
        }
    }
}

/* Change of the field of bit j when bit c flips by delta = +-1. */
static int64_t field_step_i(const orc_run_args* a, int32_t j, int32_t c)
{
    if (a->layout == ORC_LAYOUT_SYMMETRIC) return a->Qi[(size_t)j * a->N + c];
    return pair_coef_i(a->Qi, a->N, a->layout, j, c);
}

static double field_step_f(const orc_run_args* a, int32_t j, int32_t c)
{
    if (a->layout == ORC_LAYOUT_SYMMETRIC) return a->Qf[(size_t)j * a->N + c];
    return pair_coef_f(a->Qf, a->N, a->layout, j, c);
}

/* Energy difference E(x with bit j flipped) - E(x). */
static int64_t delta_i(const orc_run_args* a, const uint8_t* x, const int64_t* hi, int32_t j)
{
    int64_t d = a->Qi[(size_t)j * a->N + j];
    int64_t s = a->layout == ORC_LAYOUT_SYMMETRIC ? 2 : 1;
    return (x[j] ? -1 : 1) * (d + s * hi[j]);
}

static double delta_f(const orc_run_args* a, const uint8_t* x, const double* hf, int32_t j)
{
    double d = a->Qf[(size_t)j * a->N + j];
    double s = a->layout == ORC_LAYOUT_SYMMETRIC ? 2.0 : 1.0;
    return (x[j] ? -1.0 : 1.0) * (d + s * hf[j]);
}

static uint64_t sat_add(uint64_t a, uint64_t b)
{
    uint64_t r = a + b;
    return r < a ? UINT64_MAX : r;
}

/* Proportional choice (the paper's appendix "How to Sample Proportionally",
 * first method): the first candidate, in scan order, whose running sum of
 * weights exceeds t = U2 * S; if rounding leaves none, the last candidate of
 * positive weight.  Candidates are the j < n with use[j] != 0 (use == NULL:
 * all).  *tmargin receives the distance of t to the ends of the chosen
 * interval over S (0 for the fallback). */
static int32_t choose_proportional(const uint8_t* use, const double* w, int32_t n, double t, double S,
                                   double* tmargin)
{
    double run = 0.0, prev = 0.0;
    int32_t last_pos = -1;
    for (int32_t j = 0; j < n; ++j) {
        if (use && !use[j]) continue;
        if (w[j] > 0.0) last_pos = j;
        prev = run;
        run += w[j];
        if (run > t && w[j] > 0.0) {
            const double lo = t - prev, hi = run - t;
            *tmargin = (lo < hi ? lo : hi) / S;
            return j;
        }
    }
    *tmargin = 0.0;
    return last_pos;
}

/* Replay classes (rp_class): how a given record relates to the oracle's own
 * decision at the same state and draws. */
#define ORC_RP_SAME 0         /* same action and multiplicity                 */
#define ORC_RP_BUDGET 1       /* stay vs move differs, q within the window of L */
#define ORC_RP_MULT 2         /* multiplicity differs, q within the window of
                                 the interval [M - 1, M) the given M needs    */
#define ORC_RP_CHOICE 3       /* chosen neighbour differs, U2 S within the
                                 window of a running-sum end of the given one  */
#define ORC_RP_MISMATCH (-1)  /* differs off every decision window            */
#define ORC_RP_INVALID (-2)   /* the given action is impossible here           */

/* Half-width of the band around a boundary b of q = log U1 / log1p(-p) in
 * which two computations of p that agree to a relative `tol` may fall on
 * different sides: dq / q = kappa(p) dp / p with
 * kappa(p) = p / ((1 - p) |log1p(-p)|), plus 8 ulp of each side's
 * rounding. */
static double q_window(double p, double q, double tol)
{
    double kappa = 1.0;
    if (p > 0.0 && p < 1.0) kappa = p / ((1.0 - p) * fabs(log1p(-p)));
    return (kappa * tol + 8.0 * 0x1p-52) * fabs(q);
}

/* Is t = U2 S within the window of the interval of candidate g, i.e. could
 * a running sum computed in another order, agreeing to tol * S, choose g?
 * Running sums and t each move by at most tol * S (plus 8 ulp of S). */
static int choice_in_window(const uint8_t* use, const double* w, int32_t g, double t, double S, double tol)
{
    double before = 0.0;
    for (int32_t j = 0; j < g; ++j)
        if (!use || use[j]) before += w[j];
    const double win = (2.0 * tol + 8.0 * 0x1p-52) * S;
    return t >= before - win && t < before + w[g] + win;
}

/* Classify the given record (g_action, g_M) against the oracle's own
 * decision (own_stay, own_c, own_m) of a step with escape probability p,
 * quotient q, remaining budget L (budgeted: Unbiased PNS or an exact-time
 * run), candidates use[0..n) with weights w, their sum S and t = U2 S. */
static int32_t orc_replay_class(int budgeted, int own_stay, int32_t own_c, int64_t own_m, int32_t g_action,
                                int64_t g_M, int64_t L, double p, double q, double tol, const uint8_t* use,
                                const double* w, int32_t n, double t, double S)
{
    const int32_t own_action = own_stay ? ORC_STAY : own_c;
    const int64_t own_M = own_stay ? L : own_m;
    if (g_action == own_action && g_M == own_M) return ORC_RP_SAME;
    if (g_action == ORC_STAY) {
        if (!budgeted) return ORC_RP_INVALID;
    } else if (g_action < 0 || g_action >= n || (use && !use[g_action]) || !(w[g_action] > 0.0)) {
        return ORC_RP_INVALID;
    }
    const int g_stay = g_action == ORC_STAY;
    if (g_stay != own_stay) {
        /* at the budget boundary q = L both sides record M = L */
        if (g_M != L || !(fabs(q - (double)L) <= q_window(p, q, tol))) return ORC_RP_MISMATCH;
        if (!g_stay && g_action != own_c && !choice_in_window(use, w, g_action, t, S, tol)) return ORC_RP_MISMATCH;
        return ORC_RP_BUDGET;
    }
    if (g_stay) return ORC_RP_MISMATCH; /* both stay, so both must record L */
    int32_t cls = ORC_RP_SAME;
    if (g_M != own_m) {
        /* the given M = 1 + floor(q') needs q' in [M - 1, M): q must lie
         * within the window of that interval (for q near 2^53 and beyond the
         * window spans several integers) */
        if (g_M < 1) return ORC_RP_MISMATCH;
        const double lo = (double)(g_M - 1), hi = (double)g_M;
        const double dist = q < lo ? lo - q : (q >= hi ? q - hi : 0.0);
        if (!(dist <= q_window(p, q, tol))) return ORC_RP_MISMATCH;
        cls = ORC_RP_MULT;
    }
    if (g_action != own_c) {
        if (!choice_in_window(use, w, g_action, t, S, tol)) return ORC_RP_MISMATCH;
        cls = ORC_RP_CHOICE;
    }
    return cls;
}

int orc_run(const orc_run_args* a)
{
    const int32_t N = a->N;
    if (N <= 0) return -1;
    if (a->mode != ORC_MODE_RF && (a->n < 1 || a->n > N)) return -2;
    if (a->mode == ORC_MODE_OPT && !(a->temperature > 0.0)) return -4;
    if (a->orig_time < 0 || (a->orig_time > 0 && a->mode != ORC_MODE_RF && a->mode != ORC_MODE_BASIC)) return -5;
    const int timed = a->orig_time > 0;
    const int32_t n = a->mode == ORC_MODE_RF ? N : a->n;
    const int64_t I = orc_sys_count(N, n);

    uint8_t* x = (uint8_t*)malloc((size_t)N);
    uint8_t* xbest = (uint8_t*)malloc((size_t)N);
    uint8_t* member = (uint8_t*)malloc((size_t)N);
    int64_t* hi = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    double* hf = (double*)malloc(sizeof(double) * (size_t)N);
    int64_t* dEi = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    double* dEf = (double*)malloc(sizeof(double) * (size_t)N);
    double* lw = (double*)malloc(sizeof(double) * (size_t)N);
    double* w = (double*)malloc(sizeof(double) * (size_t)N);
    if (!x || !xbest || !member || !hi || !hf || !dEi || !dEf || !lw || !w) {
        free(x); free(xbest); free(member); free(hi); free(hf); free(dEi); free(dEf); free(lw); free(w);
        return -3;
    }

    for (int32_t ch = 0; ch < a->num_chains; ++ch) {
        const uint32_t cid = a->chain_ids[ch];
        /* Alg 9/10 weigh by [pi(y)/pi(x)]^(1/T): the target at beta / T */
        const double beta = a->mode == ORC_MODE_OPT ? a->betas[ch] / a->temperature : a->betas[ch];
        memcpy(x, a->x0 + (size_t)ch * N, (size_t)N);
        fields_init(a, x, hi, hf);
        int64_t Ei = a->is_int ? orc_energy_i(a->Qi, N, a->layout, x) : 0;
        double Ef = a->is_int ? (double)Ei : orc_energy_f(a->Qf, N, a->layout, x);
        int64_t L = timed ? a->orig_time : a->L0;
        const int64_t step0 = a->step0s ? a->step0s[ch] : a->step0;
        int64_t nrec = 0;
        int64_t sub = 0;
        int64_t flips = 0, stays = 0, saturated = 0;
        /* X_max = J_0 */
        memcpy(xbest, x, (size_t)N);
        int64_t Ei_best = Ei;
        double Ef_best = Ef;

        /* Alg 6: the first partial neighbor set is N_0 (systematic) or a
         * fresh random set drawn for the step where the block starts. */
        if (a->mode == ORC_MODE_UNBIASED_SYS) orc_sys_subset(N, n, sub, member);
        if (a->mode == ORC_MODE_UNBIASED_RAND) orc_random_subset(a->seed, cid, (uint64_t)step0, N, n, member);
        if (a->mode == ORC_MODE_RF || (a->mode == ORC_MODE_OPT && n == N)) memset(member, 1, (size_t)N);

        for (int64_t kk = 0; kk < a->K; ++kk) {
            const int64_t k = step0 + kk;
            const size_t rec = (size_t)ch * (size_t)a->K + (size_t)kk;

            /* Alg 3: a fresh partial neighbor set every step. */
            if (a->mode == ORC_MODE_BASIC || (a->mode == ORC_MODE_OPT && n < N))
                orc_random_subset(a->seed, cid, (uint64_t)k, N, n, member);

            /* Acceptance probabilities min{1, pi(y)/pi(x)} of the subset's
             * neighbours (the uniform proposal cancels), kept as logs. */
            for (int32_t j = 0; j < N; ++j) {
                if (!member[j]) continue;
                double dE;
                if (a->is_int) {
                    dEi[j] = delta_i(a, x, hi, j);
                    dE = (double)dEi[j];
                } else {
                    dEf[j] = delta_f(a, x, hf, j);
                    dE = dEf[j];
                }
                double l = -beta * dE;
                lw[j] = l < 0.0 ? l : 0.0;
            }
            /* Sum in subset order.  If every term underflows, rescale by the
             * largest term so the proportional choice stays defined; the
             * escape probability then carries the scale back. */
            double S = 0.0;
            for (int32_t j = 0; j < N; ++j) {
                if (!member[j]) continue;
                w[j] = exp(lw[j]);
                S += w[j];
            }
            double p;
            if (S < 0x1p-1000) {
                double mx = -INFINITY;
                for (int32_t j = 0; j < N; ++j)
                    if (member[j] && lw[j] > mx) mx = lw[j];
                S = 0.0;
                for (int32_t j = 0; j < N; ++j) {
                    if (!member[j]) continue;
                    w[j] = exp(lw[j] - mx);
                    S += w[j];
                }
                p = exp(mx) * S / (double)n;
            } else {
                p = S / (double)n;
            }

            /* Multiplicity 1 + G, G ~ Geometric(p) counting failures:
             * G = floor(log U1 / log(1 - p)) with U1 uniform on (0, 1]. */
            double U1, U2;
            orc_uniforms(a->seed, cid, (uint64_t)k, &U1, &U2);
            double q;
            if (p >= 1.0) q = 0.0;
            else if (p <= 0.0) q = INFINITY;
            else q = log(U1) / log1p(-p);
            int64_t m;
            int sat = 0;
            if (a->mode == ORC_MODE_OPT) {
                m = 1; /* no multiplicity: each jump counts once */
            } else if (!(q < 0x1p63)) {
                m = INT64_MAX;
                sat = 1;
            } else {
                m = (int64_t)floor(q) + 1;
            }

            const int unbiased = a->mode == ORC_MODE_UNBIASED_SYS || a->mode == ORC_MODE_UNBIASED_RAND;
            /* Rao-Blackwell weight: the budget L at the start of the record
             * cuts M for Unbiased PNS and exact-time runs */
            const double wrb = a->mode == ORC_MODE_OPT ? 1.0
                                                       : orc_expected_multiplicity(p, (unbiased || timed) ? L : -1);
            /* The record's state is the state before this step. */
            const int64_t Ei_rec = Ei;
            const double Ef_rec = Ef;
            /* Alg 6 "else" branch (and the end of an exact-time run): not
             * enough original samples left in the budget, stay with M = L. */
            const int own_stay = (unbiased || timed) && q >= (double)L;
            /* Proportional choice over the subset in bit order. */
            const double t = U2 * S;
            double tmargin = 0.0;
            const int32_t own_c = choose_proportional(member, w, N, t, S, &tmargin);
            if (own_stay) tmargin = 0.0;
            int32_t action = own_stay ? ORC_STAY : own_c;
            int64_t M = own_stay ? L : m;
            if (a->log_action) a->log_action[rec] = action;
            if (a->log_M) a->log_M[rec] = M;
            if (a->rp_action) {
                const int32_t cls = orc_replay_class(unbiased || timed, own_stay, own_c, m, a->rp_action[rec],
                                                     a->rp_M[rec], L, p, q, a->rp_tol, member, w, N, t, S);
                if (a->rp_class) a->rp_class[rec] = cls;
                if (cls != ORC_RP_INVALID) {
                    action = a->rp_action[rec];
                    M = a->rp_M[rec];
                    sat = M == INT64_MAX;
                }
            }
            if (action == ORC_STAY && timed) {
                /* the original chain is still at J when the requested time
                 * runs out: record the remaining time and stop */
                L = 0;
                ++stays;
            } else if (action == ORC_STAY) {
                /* stay L times and move to the next set */
                L = a->L0;
                ++sub;
                if (a->mode == ORC_MODE_UNBIASED_SYS) orc_sys_subset(N, n, sub % I, member);
                else orc_random_subset(a->seed, cid, (uint64_t)(k + 1), N, n, member);
                ++stays;
            } else {
                if (unbiased || timed) L -= M;
                saturated += sat;
                const int32_t c = action;
                /* Move: flip bit c and update energy and every other field. */
                if (a->is_int) {
                    int64_t delta = x[c] ? -1 : 1;
                    Ei += dEi[c];
                    for (int32_t j = 0; j < N; ++j)
                        if (j != c) hi[j] += delta * field_step_i(a, j, c);
                } else {
                    double delta = x[c] ? -1.0 : 1.0;
                    Ef += dEf[c];
                    for (int32_t j = 0; j < N; ++j)
                        if (j != c) hf[j] += delta * field_step_f(a, j, c);
                }
                x[c] ^= 1u;
                ++flips;
                /* Alg 9/10: keep the state of largest pi seen so far */
                if (a->mode == ORC_MODE_OPT && (a->is_int ? Ei < Ei_best : Ef < Ef_best)) {
                    memcpy(xbest, x, (size_t)N);
                    Ei_best = Ei;
                    Ef_best = Ef;
                }
            }

            /* Record k is (J_k-before, M_k) with its energy. */
            if (a->log_Ei) a->log_Ei[rec] = a->is_int ? Ei_rec : 0;
            if (a->log_Ef) a->log_Ef[rec] = a->is_int ? (double)Ei_rec : Ef_rec;
            if (a->log_p) a->log_p[rec] = p;
            if (a->log_q) a->log_q[rec] = q;
            if (a->log_tmargin) a->log_tmargin[rec] = tmargin;
            if (a->log_w) a->log_w[rec] = wrb;
            if ((a->hist_w || a->hist_v || a->hist_rb) && N <= 24 && k >= a->hist_from) {
                uint32_t idx = 0;
                for (int32_t j = 0; j < N; ++j) {
                    uint8_t bit = x[j];
                    if (j == action) bit ^= 1u; /* the record's state is before the flip */
                    idx |= (uint32_t)bit << j;
                }
                if (a->hist_w) a->hist_w[idx] = sat_add(a->hist_w[idx], (uint64_t)M);
                if (a->hist_v) a->hist_v[idx] += 1u;
                if (a->hist_rb) a->hist_rb[idx] += wrb;
            }
            ++nrec;
            if (timed && action == ORC_STAY) break;
        }
        if (a->n_records) a->n_records[ch] = nrec;

        if (a->x_final) memcpy(a->x_final + (size_t)ch * N, x, (size_t)N);
        if (a->hi_final && a->is_int) memcpy(a->hi_final + (size_t)ch * N, hi, sizeof(int64_t) * (size_t)N);
        if (a->hf_final && !a->is_int) memcpy(a->hf_final + (size_t)ch * N, hf, sizeof(double) * (size_t)N);
        if (a->Ei_final) a->Ei_final[ch] = Ei;
        if (a->Ef_final) a->Ef_final[ch] = Ef;
        if (a->L_final) a->L_final[ch] = L;
        if (a->sub_final) a->sub_final[ch] = sub;
        if (a->n_flips) a->n_flips[ch] = flips;
        if (a->n_stays) a->n_stays[ch] = stays;
        if (a->n_saturated) a->n_saturated[ch] = saturated;
        if (a->x_best) memcpy(a->x_best + (size_t)ch * N, xbest, (size_t)N);
        if (a->Ei_best) a->Ei_best[ch] = Ei_best;
        if (a->Ef_best) a->Ef_best[ch] = Ef_best;
    }

    free(x); free(xbest); free(member); free(hi); free(hf); free(dEi); free(dEf); free(lw); free(w);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Parallel tempering (replica exchange between temperatures).               */
/* ------------------------------------------------------------------------- */

/* One swap round over `groups` groups of T chains (chains g*T .. g*T+T-1).
 * ladder[g*T + t] is the chain of group g (0..T-1) holding the t-th
 * temperature of the group's ladder.  Round r tries the pairs of positions
 * (t, t+1) with t = r mod 2, r mod 2 + 2, ...: chains a (position t) and b
 * (position t+1) exchange their inverse temperatures with probability
 * min{1, exp[(beta_a - beta_b)(E_a - E_b)]}, the Metropolis ratio of
 * pi_{beta_a}(x_b) pi_{beta_b}(x_a) / (pi_{beta_a}(x_a) pi_{beta_b}(x_b)).
 * The uniform U in (0, 1] of a pair comes from Philox4x32-10 with key seed
 * and counter (g, r low, r high, 0x60000000 | t), words 0 and 1 as for U1;
 * the swap is accepted iff the exponent is >= 0 or log U < exponent.
 * Energies are int64 (is_int) or double; accepted[g*T + t] = 1 if taken. */
int orc_pt_round(int32_t groups, int32_t T, int32_t is_int, const int64_t* Ei, const double* Ef, double* betas,
                 int32_t* ladder, uint64_t seed, uint64_t round, int32_t* accepted)
{
    if (groups < 0 || T < 1) return -1;
    for (int32_t g = 0; g < groups; ++g) {
        for (int32_t t = (int32_t)(round & 1u); t + 1 < T; t += 2) {
            const int64_t ca = (int64_t)g * T + ladder[(int64_t)g * T + t];
            const int64_t cb = (int64_t)g * T + ladder[(int64_t)g * T + t + 1];
            const double dE = is_int ? (double)(Ei[ca] - Ei[cb]) : Ef[ca] - Ef[cb];
            const double ex = (betas[ca] - betas[cb]) * dE;
            uint32_t ctr[4] = {(uint32_t)g, (uint32_t)round, (uint32_t)(round >> 32), 0x60000000u | (uint32_t)t};
            uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
            uint32_t o[4];
            orc_philox4x32_10(ctr, key, o);
            const double u = (double)(((((uint64_t)o[0] << 32) | o[1]) >> 11) + 1u) * 0x1p-53;
            const int take = ex >= 0.0 || log(u) < ex;
            if (accepted) accepted[(int64_t)g * T + t] = take;
            if (take) {
                const double tb = betas[ca];
                betas[ca] = betas[cb];
                betas[cb] = tb;
                const int32_t tl = ladder[(int64_t)g * T + t];
                ladder[(int64_t)g * T + t] = ladder[(int64_t)g * T + t + 1];
                ladder[(int64_t)g * T + t + 1] = tl;
            }
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Exact quantities by enumeration (test pins, N <= 24).                      */
/* ------------------------------------------------------------------------- */

/* Energy x^T Q x of every state x = sum_j x_j 2^j. */
int orc_enumerate_energies_i(const int64_t* Q, int32_t N, int32_t layout, int64_t* E)
{
    if (N <= 0 || N > 24) return -1;
    uint8_t x[24];
    for (uint32_t s = 0; s < (1u << N); ++s) {
        for (int32_t j = 0; j < N; ++j) x[j] = (uint8_t)((s >> j) & 1u);
        E[s] = orc_energy_i(Q, N, layout, x);
    }
    return 0;
}

int orc_enumerate_energies_f(const double* Q, int32_t N, int32_t layout, double* E)
{
    if (N <= 0 || N > 24) return -1;
    uint8_t x[24];
    for (uint32_t s = 0; s < (1u << N); ++s) {
        for (int32_t j = 0; j < N; ++j) x[j] = (uint8_t)((s >> j) & 1u);
        E[s] = orc_energy_f(Q, N, layout, x);
    }
    return 0;
}

/* Exact one-step quantities of Basic PNS (Alg 3) on a regular neighbour graph
 * with D neighbours per state and a uniformly random n-subset of them each
 * step, p = average over the subset:
 *   T[s*D + j] = P(next = nbr[s][j]) = E_S[ 1{j in S} w_j / sum_{i in S} w_i ]
 *   EM[s]      = E[M | s]            = E_S[ n / sum_{i in S} w_i ]
 * with w_j = min(1, pi(nbr)/pi(s)) given as logpi.  Enumerates all C(D, n)
 * subsets (small D only). */
int orc_basic_onestep(int64_t num_states, int32_t D, const int64_t* nbr, const double* logpi,
                      int32_t n, double* T, double* EM)
{
    if (D <= 0 || D > 30 || n < 1 || n > D) return -1;
    int32_t idx[32];
    double wv[32];
    double nsub = 0.0;
    /* count subsets */
    {
        double c = 1.0;
        for (int32_t r = 0; r < n; ++r) c = c * (double)(D - r) / (double)(r + 1);
        nsub = floor(c + 0.5);
    }
    for (int64_t s = 0; s < num_states; ++s) {
        for (int32_t j = 0; j < D; ++j) {
            double l = logpi[nbr[s * D + j]] - logpi[s];
            wv[j] = l < 0.0 ? exp(l) : 1.0;
            T[s * D + j] = 0.0;
        }
        double em = 0.0;
        for (int32_t r = 0; r < n; ++r) idx[r] = r;
        for (;;) {
            double sw = 0.0;
            for (int32_t r = 0; r < n; ++r) sw += wv[idx[r]];
            for (int32_t r = 0; r < n; ++r) T[s * D + idx[r]] += wv[idx[r]] / sw / nsub;
            em += (double)n / sw / nsub;
            /* next combination in lexicographic order */
            int32_t r = n - 1;
            while (r >= 0 && idx[r] == D - n + r) --r;
            if (r < 0) break;
            ++idx[r];
            for (int32_t t = r + 1; t < n; ++t) idx[t] = idx[t - 1] + 1;
        }
        EM[s] = em;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Continuous Unbiased PNS (Alg 7) on the donut target of Sec 7.             */
/* ------------------------------------------------------------------------- */
/*
 * Target on R^d: log pi(x) = -(|x|^2 - mu0)^2 / (2 sigma^2) + const (the
 * density of Sec 7 written for any dimension d; d = 2 in the paper).
 * Proposal: standard normal increments, symmetric, so every acceptance ratio
 * is pi(y) / pi(x).  Partial neighbor set i of a chain: P offset vectors
 * delta_1..delta_P with i.i.d. N(0, 1) coordinates, each used with both signs
 * (the pairs of Sec 7 keep the set reversible); the neighbours of x are
 * x + delta_j (j = 0..P-1) then x - delta_j (j = P..2P-1), in that order,
 * and the set is drawn anew after each block of L0 original samples.
 * Reading: the proposal restricted to the finite set is uniform over its 2P
 * points (the offsets are already draws of the proposal density), so
 * p = (1 / 2P) sum_j min(1, pi(y_j) / pi(x)) and the next state is chosen
 * proportionally to min(1, pi(y_j) / pi(x)), as in Alg 6.
 * Normal draws: Box-Muller (Box and Muller, 1958) on two uniforms from one
 * Philox block with counter (chain, set index low, set index high,
 * 0x80000000 | pair << 8 | t): u1 in (0, 1] from words 0, 1 and u2 in [0, 1)
 * from words 2, 3, z0 = sqrt(-2 log u1) cos(2 pi u2) for coordinate 2t and
 * z1 = sqrt(-2 log u1) sin(2 pi u2) for coordinate 2t + 1.
 * The two uniforms of step k are those of the discrete samplers.
 */
#define ORC_CONT_MAX_DIM 7
#define ORC_CONT_MAX_PAIRS 32

typedef struct {
    int32_t dim;                /* 1 .. 7 */
    double mu0, sigma;          /* donut radius^2 and width */
    int32_t pairs;              /* P: 2P neighbours per set, 1 .. 32 */
    int64_t L0;
    uint64_t seed;
    int32_t num_chains;
    const uint32_t* chain_ids;  /* [num_chains] */
    const double* x0;           /* [num_chains][dim] */
    int64_t K;                  /* records per chain */
    /* per-step outputs [num_chains][K], each may be NULL */
    int32_t* log_action;        /* neighbour index 0 .. 2P-1, or ORC_STAY */
    int64_t* log_M;
    double* log_lp;             /* log pi of the record's state (without the constant) */
    double* log_p;
    double* log_q;
    double* log_tmargin;
    double* log_w;              /* expected multiplicity (Rao-Blackwell weight) */
    double* log_x;              /* [num_chains][K][dim] the record's state */
    /* final outputs, each may be NULL */
    double* x_final;            /* [num_chains][dim] */
    int64_t* L_final;
    int64_t* set_final;         /* index of the current partial neighbor set */
    int64_t* n_flips;           /* jumps */
    int64_t* n_stays;
    /* estimator sums [num_chains][2][4 dim + 1]: for weights M (row 0) and
     * the expected multiplicities (row 1): sum w, then sum w x_i, sum w x_i^2,
     * sum w x_i^4 and sum w 1(x_i > 0) for i = 0..dim-1 (each may be NULL) */
    double* sums;
    /* Replay of given records, as for the discrete chains (orc_run_args):
     * rp_action, rp_M [num_chains][K] or NULL, classes into rp_class. */
    const int32_t* rp_action;
    const int64_t* rp_M;
    int32_t* rp_class;
    double rp_tol;
} orc_cont_args;

/* log pi(x) = -(|x|^2 - mu0)^2 / (2 sigma^2), the donut density of Sec 7
 * (without its normalising constant). */
static double cont_logpi(const orc_cont_args* a, const double* x)
{
    double r2 = 0.0;
    for (int32_t i = 0; i < a->dim; ++i) r2 += x[i] * x[i];
    const double t = r2 - a->mu0;
    return -(t * t) / (2.0 * a->sigma * a->sigma);
}

/* Offsets of set `set` of a chain: delta[j][i] for pair j, coordinate i. */
void orc_cont_offsets(uint64_t seed, uint32_t chain, uint64_t set, int32_t pairs, int32_t dim, double* delta)
{
    for (int32_t j = 0; j < pairs; ++j) {
        for (int32_t t = 0; 2 * t < dim; ++t) {
            uint32_t w[4];
            draw4(seed, chain, set, 0x80000000u | ((uint32_t)j << 8) | (uint32_t)t, w);
            const double u1 = (double)(bits53(w[0], w[1]) + 1u) * 0x1p-53;
            const double u2 = (double)bits53(w[2], w[3]) * 0x1p-53;
            const double r = sqrt(-2.0 * log(u1));
            const double ang = 6.283185307179586 * u2; /* 2 pi, rounded to double */
            delta[j * dim + 2 * t] = r * cos(ang);
            if (2 * t + 1 < dim) delta[j * dim + 2 * t + 1] = r * sin(ang);
        }
    }
}

int orc_cont_run(const orc_cont_args* a)
{
    const int32_t d = a->dim, P = a->pairs, n = 2 * a->pairs;
    if (d < 1 || d > ORC_CONT_MAX_DIM) return -1;
    if (P < 1 || P > ORC_CONT_MAX_PAIRS) return -2;
    if (a->L0 < 1) return -3;
    if (!(a->sigma > 0.0)) return -4;
    const int32_t nsum = 4 * d + 1;
    for (int32_t ch = 0; ch < a->num_chains; ++ch) {
        const uint32_t cid = a->chain_ids[ch];
        double x[ORC_CONT_MAX_DIM], delta[ORC_CONT_MAX_PAIRS * ORC_CONT_MAX_DIM];
        double lpy[2 * ORC_CONT_MAX_PAIRS], w[2 * ORC_CONT_MAX_PAIRS];
        double acc[2][4 * ORC_CONT_MAX_DIM + 1];
        memset(acc, 0, sizeof(acc));
        memcpy(x, a->x0 + (size_t)ch * d, sizeof(double) * (size_t)d);
        int64_t L = a->L0, set = 0, flips = 0, stays = 0;
        orc_cont_offsets(a->seed, cid, (uint64_t)set, P, d, delta);
        double lpx = cont_logpi(a, x);
        for (int64_t k = 0; k < a->K; ++k) {
            const size_t rec = (size_t)ch * (size_t)a->K + (size_t)k;
            /* weights of the 2P neighbours, summed in neighbour order */
            double S = 0.0;
            for (int32_t j = 0; j < n; ++j) {
                double y[ORC_CONT_MAX_DIM];
                const double sgn = j < P ? 1.0 : -1.0;
                for (int32_t i = 0; i < d; ++i) y[i] = x[i] + sgn * delta[(j % P) * d + i];
                lpy[j] = cont_logpi(a, y);
                const double l = lpy[j] - lpx;
                w[j] = l < 0.0 ? exp(l) : 1.0;
                S += w[j];
            }
            const double p = S / (double)n;
            double U1, U2;
            orc_uniforms(a->seed, cid, (uint64_t)k, &U1, &U2);
            double q;
            if (p >= 1.0) q = 0.0;
            else if (p <= 0.0) q = INFINITY;
            else q = log(U1) / log1p(-p);
            const double wrb = orc_expected_multiplicity(p, L);
            /* the record's state, before the move */
            double xr[ORC_CONT_MAX_DIM];
            memcpy(xr, x, sizeof(double) * (size_t)d);
            const double lpr = lpx;
            /* not enough original samples left: stay L times, new set */
            const int own_stay = q >= (double)L;
            const int64_t own_m = !(q < 0x1p63) ? INT64_MAX : (int64_t)floor(q) + 1;
            const double t = U2 * S;
            double tmargin = 0.0;
            const int32_t own_c = choose_proportional(NULL, w, n, t, S, &tmargin);
            if (own_stay) tmargin = 0.0;
            int32_t action = own_stay ? ORC_STAY : own_c;
            int64_t M = own_stay ? L : own_m;
            if (a->log_action) a->log_action[rec] = action;
            if (a->log_M) a->log_M[rec] = M;
            if (a->rp_action) {
                const int32_t cls = orc_replay_class(1, own_stay, own_c, own_m, a->rp_action[rec], a->rp_M[rec], L,
                                                     p, q, a->rp_tol, NULL, w, n, t, S);
                if (a->rp_class) a->rp_class[rec] = cls;
                if (cls != ORC_RP_INVALID) {
                    action = a->rp_action[rec];
                    M = a->rp_M[rec];
                }
            }
            if (action == ORC_STAY) {
                L = a->L0;
                ++set;
                ++stays;
                orc_cont_offsets(a->seed, cid, (uint64_t)set, P, d, delta);
            } else {
                L -= M;
                const int32_t c = action;
                const double sgn = c < P ? 1.0 : -1.0;
                for (int32_t i = 0; i < d; ++i) x[i] = x[i] + sgn * delta[(c % P) * d + i];
                lpx = lpy[c];
                ++flips;
            }
            /* estimator sums over the record (J_k, M_k) */
            const double wt[2] = {(double)M, wrb};
            for (int32_t r = 0; r < 2; ++r) {
                acc[r][0] += wt[r];
                for (int32_t i = 0; i < d; ++i) {
                    const double v = xr[i], v2 = v * v;
                    acc[r][1 + i] += wt[r] * v;
                    acc[r][1 + d + i] += wt[r] * v2;
                    acc[r][1 + 2 * d + i] += wt[r] * (v2 * v2);
                    acc[r][1 + 3 * d + i] += v > 0.0 ? wt[r] : 0.0;
                }
            }
            if (a->log_lp) a->log_lp[rec] = lpr;
            if (a->log_p) a->log_p[rec] = p;
            if (a->log_q) a->log_q[rec] = q;
            if (a->log_tmargin) a->log_tmargin[rec] = tmargin;
            if (a->log_w) a->log_w[rec] = wrb;
            if (a->log_x) memcpy(a->log_x + rec * (size_t)d, xr, sizeof(double) * (size_t)d);
        }
        if (a->x_final) memcpy(a->x_final + (size_t)ch * d, x, sizeof(double) * (size_t)d);
        if (a->L_final) a->L_final[ch] = L;
        if (a->set_final) a->set_final[ch] = set;
        if (a->n_flips) a->n_flips[ch] = flips;
        if (a->n_stays) a->n_stays[ch] = stays;
        if (a->sums)
            for (int32_t r = 0; r < 2; ++r)
                memcpy(a->sums + ((size_t)ch * 2 + r) * nsum, acc[r], sizeof(double) * (size_t)nsum);
    }
    return 0;
}
