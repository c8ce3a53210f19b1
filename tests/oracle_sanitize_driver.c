/* Host-only driver that exercises every entry point of the C oracle, so that
 * the oracle can be built and run under AddressSanitizer and
 * UndefinedBehaviorSanitizer (gcc, CPU only).  Each call fills every output
 * it accepts; the driver checks return codes and the invariants that need no
 * second implementation (each chain's flips and stays add up to its records,
 * subsets have n members, a replay of a run's own records classifies every
 * one of them as the same), then prints an FNV-1a checksum of all outputs,
 * so that a plain and a sanitized build can be compared byte for byte.
 *
 * Inputs come from a small linear congruential generator local to this file:
 * they are test inputs only and carry none of the method's arithmetic.
 *
 * Build: gcc -std=c11 -I<oracle dir> oracle_sanitize_driver.c -lm */
#include "pns_oracle.c"

#include <stdio.h>

static uint64_t g_lcg = 0x9e3779b97f4a7c15ull;
static uint32_t lcg32(void)
{
    g_lcg = g_lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)(g_lcg >> 32);
}
static int32_t lcg_range(int32_t lo, int32_t hi) { return lo + (int32_t)(lcg32() % (uint32_t)(hi - lo + 1)); }

static uint64_t g_sum = 0xcbf29ce484222325ull;
static void mix(const void* p, size_t bytes)
{
    const unsigned char* c = (const unsigned char*)p;
    for (size_t i = 0; i < bytes; ++i) {
        g_sum ^= c[i];
        g_sum *= 0x100000001b3ull;
    }
}

static int g_fail = 0;
#define CHECK(cond)                                                                   \
    do {                                                                              \
        if (!(cond)) {                                                                \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond);        \
            g_fail = 1;                                                               \
        }                                                                             \
    } while (0)

static void* xcalloc(size_t count, size_t size)
{
    void* p = calloc(count ? count : 1, size);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

/* Random streams, subsets and states. */
static void check_streams(void)
{
    const uint32_t ctr[4] = {0u, 1u, 2u, 3u}, key[2] = {0xdeadbeefu, 0x12345678u};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    mix(out, sizeof out);
    for (uint64_t step = 0; step < 64; ++step) {
        double u1, u2;
        orc_uniforms(7, 3, step, &u1, &u2);
        CHECK(u1 > 0.0 && u1 <= 1.0 && u2 >= 0.0 && u2 < 1.0);
        mix(&u1, sizeof u1);
        mix(&u2, sizeof u2);
    }
    const int32_t sizes[][2] = {{1, 1}, {5, 3}, {7, 7}, {64, 64}, {100, 7}, {257, 64}, {1000, 128}};
    for (size_t s = 0; s < sizeof sizes / sizeof sizes[0]; ++s) {
        const int32_t N = sizes[s][0], n = sizes[s][1];
        uint8_t* m = (uint8_t*)xcalloc((size_t)N, 1);
        for (uint64_t step = 0; step < 8; ++step) {
            orc_random_subset(11, 2, step, N, n, m);
            int32_t c = 0;
            for (int32_t j = 0; j < N; ++j) c += m[j];
            CHECK(c == n);
            mix(m, (size_t)N);
        }
        /* the systematic sets cover every index n / gcd(N, n) times per sweep */
        const int64_t I = orc_sys_count(N, n);
        int32_t* cover = (int32_t*)xcalloc((size_t)N, sizeof(int32_t));
        for (int64_t i = 0; i < I; ++i) {
            orc_sys_subset(N, n, i, m);
            for (int32_t j = 0; j < N; ++j) cover[j] += m[j];
            mix(m, (size_t)N);
        }
        for (int32_t j = 0; j < N; ++j) CHECK(cover[j] == n / gcd64(N, n));
        orc_random_state(5, 9, N, m);
        mix(m, (size_t)N);
        free(cover);
        free(m);
    }
}

/* Every mode, integer and double Q, both layouts, all outputs on, then a
 * replay of the run's own records. */
static void check_runs(void)
{
    const int32_t modes[] = {ORC_MODE_RF, ORC_MODE_BASIC, ORC_MODE_UNBIASED_SYS, ORC_MODE_UNBIASED_RAND,
                             ORC_MODE_OPT};
    const int32_t Ns[] = {1, 2, 13, 20, 70};
    for (size_t mi = 0; mi < sizeof modes / sizeof modes[0]; ++mi)
        for (size_t ni = 0; ni < sizeof Ns / sizeof Ns[0]; ++ni)
            for (int32_t is_int = 0; is_int < 2; ++is_int)
                for (int32_t layout = 0; layout < 2; ++layout) {
                    const int32_t mode = modes[mi], N = Ns[ni], C = 3;
                    const int64_t K = 60;
                    const int32_t n = N < 4 ? N : N / 3 + 1;
                    int64_t* Qi = (int64_t*)xcalloc((size_t)N * N, sizeof(int64_t));
                    double* Qf = (double*)xcalloc((size_t)N * N, sizeof(double));
                    for (int32_t i = 0; i < N; ++i)
                        for (int32_t j = 0; j < N; ++j) {
                            if (layout == ORC_LAYOUT_UPPER && j < i) continue;
                            const int32_t v = lcg_range(-20, 20);
                            Qi[(size_t)i * N + j] = v;
                            Qf[(size_t)i * N + j] = v * 0.37;
                            if (layout == ORC_LAYOUT_SYMMETRIC) {
                                Qi[(size_t)j * N + i] = v;
                                Qf[(size_t)j * N + i] = v * 0.37;
                            }
                        }
                    uint32_t ids[3] = {0u, 5u, 77u};
                    double betas[3] = {0.05, 0.2, 1.0};
                    uint8_t* x0 = (uint8_t*)xcalloc((size_t)C * N, 1);
                    for (int32_t c = 0; c < C; ++c) orc_random_state(3, ids[c], N, x0 + (size_t)c * N);
                    const size_t CK = (size_t)C * (size_t)K;
                    const int hist = N <= 24;
                    const size_t H = hist ? (size_t)1 << N : 0;
                    int32_t* act = (int32_t*)xcalloc(CK, sizeof(int32_t));
                    int64_t* M = (int64_t*)xcalloc(CK, sizeof(int64_t));
                    int64_t* Ei = (int64_t*)xcalloc(CK, sizeof(int64_t));
                    double* Ef = (double*)xcalloc(CK, sizeof(double));
                    double* p = (double*)xcalloc(CK, sizeof(double));
                    double* q = (double*)xcalloc(CK, sizeof(double));
                    double* tm = (double*)xcalloc(CK, sizeof(double));
                    double* lw = (double*)xcalloc(CK, sizeof(double));
                    int32_t* cls = (int32_t*)xcalloc(CK, sizeof(int32_t));
                    uint8_t* xf = (uint8_t*)xcalloc((size_t)C * N, 1);
                    uint8_t* xb = (uint8_t*)xcalloc((size_t)C * N, 1);
                    int64_t* hi = (int64_t*)xcalloc((size_t)C * N, sizeof(int64_t));
                    double* hf = (double*)xcalloc((size_t)C * N, sizeof(double));
                    int64_t c64[7][3];
                    double cf[2][3];
                    memset(c64, 0, sizeof c64);
                    memset(cf, 0, sizeof cf);
                    uint64_t* hw = hist ? (uint64_t*)xcalloc(H, sizeof(uint64_t)) : NULL;
                    uint64_t* hv = hist ? (uint64_t*)xcalloc(H, sizeof(uint64_t)) : NULL;
                    double* hrb = hist ? (double*)xcalloc(H, sizeof(double)) : NULL;
                    orc_run_args a;
                    memset(&a, 0, sizeof a);
                    a.N = N;
                    a.is_int = is_int;
                    a.layout = layout;
                    a.Qi = Qi;
                    a.Qf = Qf;
                    a.mode = mode;
                    a.n = n;
                    a.L0 = 30;
                    a.seed = 0x1234u + (uint64_t)mi;
                    a.num_chains = C;
                    a.chain_ids = ids;
                    a.betas = betas;
                    a.x0 = x0;
                    a.K = K;
                    a.step0 = 4;
                    a.log_action = act;
                    a.log_M = M;
                    a.log_Ei = Ei;
                    a.log_Ef = Ef;
                    a.log_p = p;
                    a.log_q = q;
                    a.log_tmargin = tm;
                    a.x_final = xf;
                    a.hi_final = hi;
                    a.hf_final = hf;
                    a.Ei_final = c64[0];
                    a.Ef_final = cf[0];
                    a.L_final = c64[1];
                    a.sub_final = c64[2];
                    a.hist_w = hw;
                    a.hist_v = hv;
                    a.hist_rb = hrb;
                    a.hist_from = 5;
                    a.n_flips = c64[3];
                    a.n_stays = c64[4];
                    a.n_saturated = c64[5];
                    a.temperature = 0.5;
                    a.x_best = xb;
                    a.Ei_best = c64[6];
                    a.Ef_best = cf[1];
                    a.log_w = lw;
                    CHECK(orc_run(&a) == 0);
                    for (int32_t c = 0; c < C; ++c) CHECK(c64[3][c] + c64[4][c] == K);
                    mix(act, CK * sizeof(int32_t));
                    mix(M, CK * sizeof(int64_t));
                    mix(is_int ? (const void*)Ei : (const void*)Ef, CK * 8);
                    mix(p, CK * sizeof(double));
                    mix(lw, CK * sizeof(double));
                    mix(xf, (size_t)C * N);
                    mix(xb, (size_t)C * N);
                    mix(is_int ? (const void*)hi : (const void*)hf, (size_t)C * N * 8);
                    mix(c64, sizeof c64);
                    if (hist) {
                        mix(hw, H * sizeof(uint64_t));
                        mix(hv, H * sizeof(uint64_t));
                    }
                    /* replay of its own records: every record is the same */
                    int32_t* act2 = (int32_t*)xcalloc(CK, sizeof(int32_t));
                    int64_t* M2 = (int64_t*)xcalloc(CK, sizeof(int64_t));
                    memcpy(act2, act, CK * sizeof(int32_t));
                    memcpy(M2, M, CK * sizeof(int64_t));
                    a.rp_action = act2;
                    a.rp_M = M2;
                    a.rp_class = cls;
                    a.rp_tol = 1e-9;
                    a.hist_w = a.hist_v = NULL;
                    a.hist_rb = NULL;
                    CHECK(orc_run(&a) == 0);
                    for (size_t r = 0; r < CK; ++r) CHECK(cls[r] == ORC_RP_SAME);
                    free(act2);
                    free(M2);
                    /* RF and Basic on a fixed budget of original time */
                    if (mode == ORC_MODE_RF || mode == ORC_MODE_BASIC) {
                        int64_t nrec[3], s0[3] = {0, 9, 100};
                        a.rp_action = NULL;
                        a.rp_M = NULL;
                        a.rp_class = NULL;
                        a.orig_time = 200;
                        a.n_records = nrec;
                        a.step0s = s0;
                        CHECK(orc_run(&a) == 0);
                        for (int32_t c = 0; c < C; ++c) {
                            CHECK(nrec[c] >= 1 && nrec[c] <= K);
                            int64_t t = 0;
                            for (int64_t k = 0; k < nrec[c]; ++k) t += M[(size_t)c * K + (size_t)k];
                            CHECK(nrec[c] == K || t == 200);
                        }
                        mix(nrec, sizeof nrec);
                        mix(M, CK * sizeof(int64_t));
                    }
                    free(Qi); free(Qf); free(x0); free(act); free(M); free(Ei); free(Ef); free(p); free(q);
                    free(tm); free(lw); free(cls); free(xf); free(xb); free(hi); free(hf);
                    free(hw); free(hv); free(hrb);
                }
}

/* Rejected arguments return an error and touch no output. */
static void check_errors(void)
{
    orc_run_args a;
    memset(&a, 0, sizeof a);
    CHECK(orc_run(&a) < 0); /* N = 0 */
    a.N = 4;
    a.mode = ORC_MODE_UNBIASED_SYS;
    a.n = 5;
    CHECK(orc_run(&a) < 0); /* n > N */
    a.n = 2;
    a.mode = ORC_MODE_OPT;
    a.temperature = 0.0;
    CHECK(orc_run(&a) < 0);
    a.mode = ORC_MODE_UNBIASED_SYS;
    a.orig_time = 10;
    CHECK(orc_run(&a) < 0);
    int64_t E[1];
    CHECK(orc_enumerate_energies_i(NULL, 25, 0, E) < 0);
    CHECK(orc_enumerate_energies_f(NULL, 0, 0, NULL) < 0);
    CHECK(orc_basic_onestep(1, 31, NULL, NULL, 1, NULL, NULL) < 0);
    CHECK(orc_pt_round(1, 0, 1, NULL, NULL, NULL, NULL, 0, 0, NULL) < 0);
    orc_cont_args c;
    memset(&c, 0, sizeof c);
    CHECK(orc_cont_run(&c) < 0); /* dim = 0 */
    c.dim = 2;
    c.pairs = 33;
    CHECK(orc_cont_run(&c) < 0);
    c.pairs = 2;
    CHECK(orc_cont_run(&c) < 0); /* L0 = 0 */
    c.L0 = 5;
    CHECK(orc_cont_run(&c) < 0); /* sigma = 0 */
}

/* Tempering rounds, enumeration and the exact one-step quantities. */
static void check_exact(void)
{
    const int32_t groups = 2, T = 5;
    int64_t Ei[10];
    double Ef[10], betas[10];
    int32_t ladder[10], acc[10];
    for (int32_t i = 0; i < groups * T; ++i) {
        Ei[i] = lcg_range(-50, 50);
        Ef[i] = Ei[i] * 0.5;
        betas[i] = 0.1 * (i % T + 1);
        ladder[i] = i % T;
    }
    for (uint64_t r = 0; r < 6; ++r) {
        CHECK(orc_pt_round(groups, T, (int32_t)(r & 1u), Ei, Ef, betas, ladder, 99, r, acc) == 0);
        mix(ladder, sizeof ladder);
        mix(betas, sizeof betas);
    }
    const int32_t N = 10;
    int64_t Qi[100];
    double Qf[100];
    for (int32_t i = 0; i < N * N; ++i) {
        Qi[i] = lcg_range(-9, 9);
        Qf[i] = Qi[i] * 0.25;
    }
    int64_t* E = (int64_t*)xcalloc((size_t)1 << N, sizeof(int64_t));
    double* F = (double*)xcalloc((size_t)1 << N, sizeof(double));
    for (int32_t layout = 0; layout < 2; ++layout) {
        CHECK(orc_enumerate_energies_i(Qi, N, layout, E) == 0);
        CHECK(orc_enumerate_energies_f(Qf, N, layout, F) == 0);
        mix(E, sizeof(int64_t) << N);
        mix(F, sizeof(double) << N);
    }
    /* hypercube of dimension 5: single-bit-flip neighbours */
    const int32_t D = 5;
    const int64_t S = (int64_t)1 << D;
    int64_t nbr[32 * 5];
    double logpi[32], Tm[32 * 5], EM[32];
    for (int64_t s = 0; s < S; ++s) {
        logpi[s] = 0.3 * (double)lcg_range(-10, 10);
        for (int32_t j = 0; j < D; ++j) nbr[s * D + j] = s ^ ((int64_t)1 << j);
    }
    for (int32_t n = 1; n <= D; ++n) {
        CHECK(orc_basic_onestep(S, D, nbr, logpi, n, Tm, EM) == 0);
        for (int64_t s = 0; s < S; ++s) {
            double row = 0.0;
            for (int32_t j = 0; j < D; ++j) row += Tm[s * D + j];
            CHECK(fabs(row - 1.0) < 1e-12);
            CHECK(EM[s] >= 1.0 - 1e-12); /* n over a sum of n weights at most 1 */
        }
        mix(Tm, sizeof Tm);
        mix(EM, sizeof EM);
    }
    for (int64_t L = 1; L < 40; L += 7) {
        const double w = orc_expected_multiplicity(0.3, L);
        CHECK(w >= 1.0 && w <= (double)L);
        mix(&w, sizeof w);
    }
    free(E);
    free(F);
}

/* The continuous chain of every dimension, with all outputs, then a replay
 * of its own records. */
static void check_cont(void)
{
    const int32_t pairs_list[] = {1, 3, 25, 32};
    for (int32_t d = 1; d <= ORC_CONT_MAX_DIM; ++d)
        for (size_t pi = 0; pi < sizeof pairs_list / sizeof pairs_list[0]; ++pi) {
            const int32_t P = pairs_list[pi], C = 2;
            const int64_t K = 40;
            const size_t CK = (size_t)C * (size_t)K;
            uint32_t ids[2] = {1u, 4u};
            double x0[2 * ORC_CONT_MAX_DIM];
            for (int32_t i = 0; i < 2 * d; ++i) x0[i] = 0.1 * lcg_range(-10, 10);
            int32_t* act = (int32_t*)xcalloc(CK, sizeof(int32_t));
            int64_t* M = (int64_t*)xcalloc(CK, sizeof(int64_t));
            double* lp = (double*)xcalloc(CK, sizeof(double));
            double* p = (double*)xcalloc(CK, sizeof(double));
            double* q = (double*)xcalloc(CK, sizeof(double));
            double* tm = (double*)xcalloc(CK, sizeof(double));
            double* w = (double*)xcalloc(CK, sizeof(double));
            double* lx = (double*)xcalloc(CK * (size_t)d, sizeof(double));
            int32_t* cls = (int32_t*)xcalloc(CK, sizeof(int32_t));
            double xf[2 * ORC_CONT_MAX_DIM];
            double sums[2 * 2 * (4 * ORC_CONT_MAX_DIM + 1)];
            int64_t Lf[2], setf[2], fl[2], st[2];
            orc_cont_args a;
            memset(&a, 0, sizeof a);
            a.dim = d;
            a.mu0 = 4.0;
            a.sigma = 0.5;
            a.pairs = P;
            a.L0 = 25;
            a.seed = 31u + (uint64_t)d;
            a.num_chains = C;
            a.chain_ids = ids;
            a.x0 = x0;
            a.K = K;
            a.log_action = act;
            a.log_M = M;
            a.log_lp = lp;
            a.log_p = p;
            a.log_q = q;
            a.log_tmargin = tm;
            a.log_w = w;
            a.log_x = lx;
            a.x_final = xf;
            a.L_final = Lf;
            a.set_final = setf;
            a.n_flips = fl;
            a.n_stays = st;
            a.sums = sums;
            CHECK(orc_cont_run(&a) == 0);
            for (int32_t c = 0; c < C; ++c) CHECK(fl[c] + st[c] == K);
            mix(act, CK * sizeof(int32_t));
            mix(M, CK * sizeof(int64_t));
            mix(lp, CK * sizeof(double));
            mix(w, CK * sizeof(double));
            mix(lx, CK * (size_t)d * sizeof(double));
            mix(xf, (size_t)C * (size_t)d * sizeof(double));
            mix(sums, (size_t)C * 2 * (size_t)(4 * d + 1) * sizeof(double));
            a.rp_action = act;
            a.rp_M = M;
            a.rp_class = cls;
            a.rp_tol = 1e-9;
            a.log_action = NULL;
            a.log_M = NULL;
            CHECK(orc_cont_run(&a) == 0);
            for (size_t r = 0; r < CK; ++r) CHECK(cls[r] == ORC_RP_SAME);
            double delta[ORC_CONT_MAX_PAIRS * ORC_CONT_MAX_DIM];
            orc_cont_offsets(5, 2, 3, P, d, delta);
            mix(delta, (size_t)P * (size_t)d * sizeof(double));
            free(act); free(M); free(lp); free(p); free(q); free(tm); free(w); free(lx); free(cls);
        }
}

int main(void)
{
    check_streams();
    check_runs();
    check_errors();
    check_exact();
    check_cont();
    printf("checksum %016llx\n", (unsigned long long)g_sum);
    if (g_fail) {
        fprintf(stderr, "driver checks failed\n");
        return 1;
    }
    return 0;
}
