/*
 * pns.h - C ABI of the MI355X (gfx950) Partial Neighbor Search sampler.
 *
 * The library samples many independent chains on QUBO targets
 *     pi_beta(x) proportional to exp(-beta * x^T Q x),  x in {0,1}^N
 * with the single-bit-flip neighbourhood and uniform proposal of the paper's
 * QUBO application (Sec 4), by one of
 *   PNS_MODE_RF             Rejection-Free, discrete case (Alg 2, Sec 1.2):
 *                           every step considers all N neighbours;
 *   PNS_MODE_BASIC          Basic Partial Neighbor Search (Alg 3, Sec 2): a
 *                           fresh uniformly random subset of n neighbours
 *                           every step, p = average over the subset;
 *   PNS_MODE_UNBIASED_SYS   Unbiased PNS (Alg 6, Sec 3.2) with the systematic
 *                           partial neighbor sets of Secs 4-5: set i holds
 *                           bits (i*n + t) mod N, t < n; N/gcd(N,n) sets;
 *   PNS_MODE_UNBIASED_RAND  Unbiased PNS with a fresh uniformly random set
 *                           after each block of L0 original samples (Sec 5).
 * A step (one pass of the loop of Alg 2/3/6) emits one jump-chain record
 * (J, M): the state before the step and its multiplicity M = 1 + G,
 * G ~ Geometric(p) counting failures (Sec 1.2, eq. (2)).  In the Unbiased
 * modes a step whose multiplicity exceeds the remaining budget L emits
 * (J, M = L), keeps the state and switches to the next set (Alg 6).
 * The next state is chosen with probability proportional to
 * min(1, exp(-beta dE_i)) by the inverse-CDF rule of the appendix "How to
 * Sample Proportionally" over the subset in increasing bit order.  Randomness: Philox4x32-10 keyed by the 64-bit
 * seed, counter (chain id, step low, step high, stream); the draws of a step
 * depend only on (seed, chain id, step), so results are identical whatever
 * the launch form, workgroup size or chunking.
 *
 * Conventions shared by every entry point:
 *   - Every function returns PNS_OK (0) or a PNS_E* code; the message of the
 *     last failure on the calling thread is returned by pns_last_error().
 *     No C++ exception crosses the ABI.
 *   - A context is not thread-safe: calls on one context must not overlap.
 *     Work is queued on the context's stream; pns_run is asynchronous and
 *     every pns_read* call synchronises the stream before returning.
 *   - Pointers named "host or device" may point to host memory or to memory
 *     allocated on the context's GPU (hipMalloc, torch tensors); the library
 *     detects which.  Caller-owned buffers stay owned by the caller.
 *   - Arrays indexed [chain][bit] are dense row-major with row length N.
 */
#ifndef PNS_H
#define PNS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define PNS_OK 0
#define PNS_EINVAL 1       /* an argument is out of range or inconsistent   */
#define PNS_ENOMEM 2       /* device or host allocation failed              */
#define PNS_EDEVICE 3      /* a HIP runtime call or kernel launch failed    */
#define PNS_EUNSUPPORTED 4 /* valid request this build does not implement   */

/* ---- methods (Alg 2, Alg 3, Alg 6) ---- */
#define PNS_MODE_RF 0
#define PNS_MODE_BASIC 1
#define PNS_MODE_UNBIASED_SYS 2
#define PNS_MODE_UNBIASED_RAND 3

/* ---- Q element types ---- */
#define PNS_I16 0 /* int16 entries: exact int32 fields, int64 energies     */
#define PNS_I32 1 /* int32 entries: exact int32 or int64 fields            */
#define PNS_F32 2 /* float entries: fields and energies accumulated in FP64 */

/* ---- Q layouts (Sec 4: "usually symmetric or upper triangular") ---- */
#define PNS_SYMMETRIC 0 /* full N x N matrix with Q = Q^T (checked)        */
#define PNS_UPPER 1     /* entries i <= j define x^T Q x; i > j ignored    */

/* ---- initial states J_0 ---- */
#define PNS_INIT_ZERO 0   /* x = 0                                          */
#define PNS_INIT_RANDOM 1 /* Bernoulli(1/2) bits from Philox stream 2^29    */
#define PNS_INIT_GIVEN 2  /* opts->x0                                       */

/* ---- launch forms ---- */
#define PNS_LAUNCH_PLAIN 0      /* one kernel launch per step; chain state
                                   round-trips through HBM every step     */
#define PNS_LAUNCH_PERSISTENT 1 /* one launch runs `chunk` steps with the
                                   chain state held in registers and LDS  */
#define PNS_LAUNCH_GRAPH 2      /* the persistent chunk launches captured
                                   once in a HIP graph and replayed       */

/* Record action of a stay (Unbiased block end). */
#define PNS_STAY (-1)

typedef struct pns_ctx pns_ctx;

typedef struct pns_opts {
    int32_t dtype;          /* PNS_I16 / PNS_I32 / PNS_F32 (default I32)          */
    int32_t layout;         /* PNS_SYMMETRIC / PNS_UPPER (default SYMMETRIC)      */
    int32_t num_chains;     /* independent chains (default 1)                     */
    const double* betas;    /* host [num_chains] inverse temperatures (temperature
                               replicas), or NULL: every chain uses `beta`        */
    int64_t L0;             /* Unbiased block length in original samples
                               (default 100, the value of Secs 4-5)               */
    uint64_t seed;          /* Philox key                                         */
    uint32_t chain_id_base; /* chain c uses counter word chain_id_base + c        */
    int32_t init;           /* PNS_INIT_* (default ZERO)                          */
    const uint8_t* x0;      /* host or device [num_chains][N] for INIT_GIVEN      */
    int32_t launch;         /* PNS_LAUNCH_* (default PERSISTENT)                  */
    int32_t chunk;          /* steps per launch in PERSISTENT / GRAPH; 0 = all
                               steps of a pns_run in one launch                   */
    int32_t block;          /* threads per workgroup (one workgroup per chain);
                               0 = chosen from the tuned table.  Step-kernel
                               tiles (block x groups): 64x1, 64x2, 64x4, 128x1,
                               128x2, 128x4, 256x1, 256x2, 256x4, 256x8, 512x2,
                               512x4, 1024x2, 1024x4, and 256x16 for 32-bit fields
                               (I16, I32 with int32 fields).  Window-kernel tiles
                               (PNS_MODE_UNBIASED_SYS on I16 / I32 with int32
                               fields, flavour 5 of pns_problem_info): 64x2,
                               64x4, 64x8, 64x16, 64x24, 128x16, 128x24 and
                               256x16, which then run the window kernel (64x2
                               and 64x4 no longer run the step kernel there).  4 * block * groups
                               must reach N; another shape, or a window-kernel
                               tile for another mode or type, is PNS_EINVAL       */
    int32_t groups;         /* 4-field groups per lane; 0 = chosen with `block`   */
    void* stream;           /* hipStream_t to queue work on; NULL = a stream the
                               context creates and owns                           */
    int64_t log_capacity;   /* per-chain per-step record log, ring of this many
                               steps (0 = off); read with pns_read_log           */
    int32_t hist;           /* 1: accumulate, pooled over chains, the multiplicity-
                               weighted and the visit histograms over all 2^N
                               states (N <= 24); read with pns_read_hist          */
    int32_t snapshot_every; /* > 0: every this many steps store the record (state
                               bits, M, E) of each chain; read with
                               pns_read_snapshots (0 = off)                       */
    int32_t snapshot_capacity; /* snapshots kept per chain (ring)               */
    int32_t autotune;       /* 1: choose the tile (and a subset size given as 0)
                               from timed trials on the device (pns_autotune);
                               results are cached per process                    */
    int32_t reserved[7];    /* must be zero                                       */
} pns_opts;

/* One problem of a batched context (pns_create_batch). */
typedef struct pns_problem {
    const void* Q;          /* N x N row-major, element type opts->dtype, host or
                               device; copied on creation                        */
    int32_t N;
    int32_t layout;         /* PNS_SYMMETRIC / PNS_UPPER                         */
    int32_t subset_size;    /* n in [1, N]; 0 = chosen by the autotuner (subset
                               modes) ; ignored by RF                            */
    int32_t num_chains;     /* chains of this problem (>= 1)                     */
    int64_t L0;             /* 0 = opts->L0                                      */
    const double* betas;    /* host [num_chains] inverse temperatures, or NULL  */
    double beta;            /* used when betas is NULL                           */
} pns_problem;

/* Tile and subset size of one problem as the library runs it. */
typedef struct pns_problem_info {
    int32_t N;
    int32_t subset_size;
    int32_t block;          /* workgroup size (threads)                          */
    int32_t groups;         /* 4-bit groups per lane                             */
    int32_t chain_begin;    /* first chain of the problem                        */
    int32_t num_chains;
    int32_t flavour;        /* 0 all bits, 1 window, 2 drawn subset, 3 compact
                               window (one 4-bit group per wave), 4 two-group
                               window (at most two groups per wave), 5 window
                               kernel (one to four waves per chain; systematic
                               sets of integer Q; its records equal those of
                               flavours 1, 3 and 4 bit for bit)                 */
    int32_t reserved;
} pns_problem_info;

/* Result of pns_autotune. */
typedef struct pns_tune {
    int32_t block;
    int32_t groups;
    int32_t subset_size;
    int32_t trials;         /* timed configurations                              */
    double records_per_s;   /* records (steps x chains) per second of the choice */
    double flips_per_s;
} pns_tune;

/* Per-chain counters since creation. */
typedef struct pns_chain_stats {
    int64_t steps;      /* records emitted (jump sample size K)                 */
    int64_t flips;      /* moves                                                */
    int64_t stays;      /* Unbiased block-end stays                             */
    int64_t saturated;  /* records whose multiplicity saturated at 2^63-1 (p
                           underflowed to 0)                                     */
    double sum_M;       /* original sample size sum of M (effective MH steps)    */
    int64_t anomalies;  /* selections that found no positive weight in the
                           chosen interval (rounding safeguard; expected 0)     */
} pns_chain_stats;

/* Fill *opts with the defaults documented above. */
void pns_opts_default(pns_opts* opts);

/*
 * Create a sampler for Q (N x N, row-major, element type opts->dtype, host or
 * device), copied into device memory (the caller keeps Q).  beta >= 0 is
 * used for every chain unless opts->betas is given.  subset_size is n in
 * [1, N] for BASIC and the UNBIASED modes and is ignored by RF (n = N).
 * The initial fields h = Q_offdiag x0 and energies x0^T Q x0 are computed on
 * the GPU (one matrix product per problem on the matrix cores, see
 * pns_refresh).  On success *out owns all device memory of the sampler until
 * pns_destroy.
 * Errors: PNS_EINVAL (N <= 0, n outside [1, N], beta < 0 or not finite,
 *         unknown dtype/layout/mode/launch, SYMMETRIC Q not symmetric, a field
 *         bound overflowing 62 bits, hist with N > 24), PNS_ENOMEM,
 *         PNS_EDEVICE, PNS_EUNSUPPORTED (N above 16384, the capacity of the
 *         largest tile; checked before Q is read).
 */
int pns_create(pns_ctx** out, const void* Q, int32_t N, double beta, int32_t subset_size, int32_t mode,
               const pns_opts* opts);

/*
 * Create one context over several problems of the same element type and
 * method (QUBOs of uneven N, each with its own chains and temperatures):
 * chain c of problem p is numbered problems[0..p-1].num_chains + c.  Problems
 * are grouped by workgroup tile and kernel flavour; each group (launch class)
 * runs in its own kernel launch, the launches concurrent on side streams (in
 * the graph form as parallel graph nodes): one stream per class, up to the
 * process's hardware queues (GPU_MAX_HW_QUEUES, read when HIP starts; at most
 * 16), classes packed longest first when there are more.  The streams start
 * largest workgroups first, and in launches of 4096 steps or more those of
 * one-wave classes 200 us after the others (a one-wave delay kernel on the
 * context's stream), so that workgroups of several waves find whole compute
 * units.
 * Per-chain arrays of bits or fields (pns_read, pns_read_current,
 * pns_read_snapshots) are concatenated, chain c occupying the N of its
 * problem; pns_chain_offsets gives the offsets.  Histograms are not
 * available for batches.  Problems with subset_size 0 (or opts->autotune)
 * are tuned with pns_autotune on creation.
 * Errors: as pns_create, PNS_EINVAL for num_problems < 1 or a bad problem.
 */
int pns_create_batch(pns_ctx** out, int32_t num_problems, const pns_problem* problems, int32_t mode,
                     const pns_opts* opts);

/*
 * Choose the workgroup tile and, when subset_size is 0 in a subset mode, the
 * subset size for one problem by timed trials on the device: every compiled
 * tile whose capacity 4 * block * groups lies between N and twice N rounded
 * up to 256 (tiles of 32 or more fields per lane only where a window kernel
 * runs the problem; where a window-kernel tile holds the problem, only the
 * smallest such tile), with every subset size 16, 32, ... up to N/2, is run
 * for trial_steps steps (after a warmup; the faster of two timed runs) from
 * x = 0 with max(3072, opts->num_chains) chains, at most 4096 (the
 * problem's betas repeated), so that the device is loaded as in a real run;
 * the largest subset size whose rate is within 10% of the best trial is
 * chosen, on its fastest tile (Sec 5: on parallel hardware, take the largest
 * affordable partial neighbor set).  Results are cached per process by (N,
 * dtype, layout, mode, n, chains, trial_steps).  Synchronises the device.
 * Errors: as pns_create.
 */
int pns_autotune(const void* Q, int32_t N, double beta, int32_t subset_size, int32_t mode, const pns_opts* opts,
                 int32_t trial_steps, pns_tune* out);

/* Offsets [num_chains + 1] of each chain's bits in concatenated per-chain
 * arrays (c * N for a single-problem context).  Host memory. */
int pns_chain_offsets(const pns_ctx* ctx, int64_t* offsets);

/* Number of problems of the context (1 unless created by pns_create_batch). */
int pns_num_problems(const pns_ctx* ctx);

/* Tile, subset size and chain range of problem p. */
int pns_problem_info_get(const pns_ctx* ctx, int32_t p, pns_problem_info* info);

/*
 * Advance every chain by `steps` steps (records), queued on the context's
 * stream; returns before the GPU finishes.  steps >= 0.
 * Errors: PNS_EINVAL (steps < 0), PNS_EDEVICE (launch failure).
 */
int pns_run(pns_ctx* ctx, int64_t steps);

/*
 * Last completed record of every chain (the paper's (J_{k-1}, M_{k-1})):
 * states [num_chains][N] (uint8 0/1), multiplicities [num_chains] and
 * energies x^T Q x of those states [num_chains] (FP64; exact for integer Q
 * while |E| < 2^53).  Any pointer may be NULL; each is host or device.
 * Before the first step the record is (J_0, 0, E(J_0)).  Synchronises.
 */
int pns_read(pns_ctx* ctx, uint8_t* states, int64_t* multiplicities, double* energies);

/*
 * Current state J_k (the state after the last step) of every chain:
 * states [num_chains][N], energies [num_chains], fields [num_chains][N] of the
 * context's field type (int32 for I16 and bounded I32, int64 for other I32,
 * double for F32; query with pns_field_type), remaining budgets L
 * [num_chains], systematic set indices [num_chains] and step counters
 * [num_chains].  Any pointer may be NULL; each is host or device.
 * The field of bit j is h_j = sum_{i != j} Q_ji x_i for SYMMETRIC Q and
 * sum_{i != j} Q_min(i,j),max(i,j) x_i for UPPER Q, so that
 * dE_j = (1 - 2 x_j)(Q_jj + s h_j), s = 2 (SYMMETRIC) or 1 (UPPER).
 * Synchronises.
 */
int pns_read_current(pns_ctx* ctx, uint8_t* states, double* energies, void* fields, int64_t* L, int64_t* set_index,
                     int64_t* step);

/* Field element type of pns_read_current: 0 = int32, 1 = int64, 2 = double. */
int pns_field_type(const pns_ctx* ctx);

/*
 * Per-step log ring [num_chains][log_capacity]: step k of a chain is at slot
 * k mod log_capacity.  actions: flipped bit or PNS_STAY; multiplicities M;
 * energies of the record's state (FP64); p = escape probability of the step
 * (subset average of min(1, pi(y)/pi(x))).  Any pointer may be NULL; each is
 * host or device.  Errors: PNS_EINVAL if the log is off.  Synchronises.
 */
int pns_read_log(pns_ctx* ctx, int32_t* actions, int64_t* multiplicities, double* energies, double* p);

/* Histograms [2^N] (uint64, pooled over chains): sum of M and number of
 * records per state x = sum_j x_j 2^j.  Host or device.  Synchronises. */
int pns_read_hist(pns_ctx* ctx, uint64_t* hist_weighted, uint64_t* hist_visits);

/* Zero both histograms (e.g. after burn-in), queued on the stream. */
int pns_hist_clear(pns_ctx* ctx);

/*
 * Snapshots [num_chains][count]: states [num_chains][count][N] (uint8),
 * multiplicities and energies of the records taken every snapshot_every
 * steps; *count receives the number stored per chain (at most
 * snapshot_capacity).  Synchronises.
 */
int pns_read_snapshots(pns_ctx* ctx, uint8_t* states, int64_t* multiplicities, double* energies, int32_t* count);

/* Per-chain counters [num_chains] into host memory.  Synchronises. */
int pns_stats(pns_ctx* ctx, pns_chain_stats* stats);

/* Wait for all queued work of the context. */
int pns_sync(pns_ctx* ctx);

/* Release every resource of the context (NULL is accepted). */
int pns_destroy(pns_ctx* ctx);

/* Workgroup size and 4-field groups per lane the context runs with. */
int pns_tile(const pns_ctx* ctx, int32_t* block, int32_t* groups);

/* Message of the last failure on the calling thread ("" if none). */
const char* pns_last_error(void);

/* Library version, e.g. "0.1.0". */
const char* pns_version(void);

/*
 * Replace the coefficient matrix of problem `problem` (same N, element type
 * and layout as on creation; host or device, copied).  The chains keep their
 * states, budgets and random-number positions; their local fields and
 * energies are recomputed for the new matrix, so the next step samples the
 * new target (a warm start, as a fitting loop needs).  The matrix is
 * prepared and checked on the device in a staging buffer and swapped in
 * only if valid.  Synchronises the context's stream.
 * Errors: PNS_EINVAL (NULL Q, problem out of range, asymmetric SYMMETRIC Q,
 * non-finite entries, int64 energy overflow), PNS_EUNSUPPORTED (integer Q
 * whose fields no longer fit the context's 32-bit fields), PNS_ENOMEM,
 * PNS_EDEVICE.
 */
int pns_set_q(pns_ctx* ctx, int32_t problem, const void* Q);

/* Forget every stored snapshot (weights and counts to zero), queued on the
 * context's stream.  Errors: PNS_EINVAL (NULL ctx, snapshots off). */
int pns_snapshots_clear(pns_ctx* ctx);

/*
 * Optimization Rejection-Free (Alg 9) / Optimization PNS (Alg 10) as burn-in
 * (Sec 8): advance every chain by `steps` jumps of the jump chain whose
 * acceptance is min{1, [pi(y)/pi(x)]^(1/T)} (the target at beta / T) with no
 * multiplicity, keeping per chain the state of largest pi seen, X_max
 * (initially the chain's state at the first call).  Problems whose subset
 * size n is below N draw a fresh uniformly random n-subset every step (the
 * subset rule of Alg 3: Basic PNS is Optimization PNS plus multiplicities,
 * Sec 2); RF contexts and n = N consider every neighbour.  A cooling
 * schedule T(k) is a sequence of calls with non-increasing T.  Draws come from
 * the chains' counters like pns_run (step k uses the same Philox numbers), and
 * the per-step log, histograms and snapshots record these jumps with M = 1.
 * Budgets and set indices of Unbiased chains are left as they are; pns_run
 * afterwards samples from the chains' current states (Sec 8.2), or from X_max
 * after pns_adopt_best (Sec 8.1).  Queued on the context's stream.
 * Errors: PNS_EINVAL (steps < 0, T not finite and > 0), PNS_ENOMEM,
 * PNS_EDEVICE.
 */
int pns_optimize(pns_ctx* ctx, int64_t steps, double temperature);

/* X_max of every chain (bits [C][N] concatenated as pns_read, energies [C]),
 * host or device buffers, either may be NULL.  Synchronises.
 * Errors: PNS_EINVAL (no pns_optimize yet). */
int pns_read_best(pns_ctx* ctx, uint8_t* states, double* energies);

/* Move every chain to its X_max: fields and energies recomputed, Unbiased
 * budgets restarted at L0, last records reset.  Synchronises.
 * Errors: PNS_EINVAL (no pns_optimize yet), PNS_EDEVICE. */
int pns_adopt_best(pns_ctx* ctx);

/*
 * Advance every chain of a Rejection-Free or Basic PNS context by exactly
 * `original_steps` original samples (the time of the underlying Metropolis
 * chain, Sec 1.2): records are made until their multiplicities reach
 * original_steps, the record covering the end is cut to the remaining time
 * (M = remaining, action PNS_STAY) and the chain stops on it without moving.
 * This is the budget rule of Alg 6 used as a stopping time; by the
 * memorylessness of the geometric holding time the next run continues the
 * original chain exactly.  At a fixed original time the state follows the
 * original chain's law (pi at stationarity), not the jump chain's alpha pi;
 * parallel tempering (pns_pt_swap) compares chains at such times.  Chains
 * end on different record counts (pns_read_current's step).  Queued on the
 * context's stream.
 * Errors: PNS_EINVAL (not an RF / Basic context, original_steps < 0),
 * PNS_EDEVICE.
 */
int pns_run_original(pns_ctx* ctx, int64_t original_steps);

/*
 * One parallel-tempering swap round over groups of `temps` consecutive chains
 * (chains g*temps .. g*temps+temps-1 hold one copy of each temperature of a
 * ladder; Sec 5 combines replicas at different temperatures with PNS).  On
 * the first call (or a new `temps`) each group's ladder is its chains ordered
 * by their current beta.  Round r tries the adjacent ladder positions
 * (t, t+1), t = r mod 2, r mod 2 + 2, ...: the two chains exchange their
 * inverse temperatures with probability min{1, exp[(b_a - b_b)(E_a - E_b)]}
 * (E the chains' current energies; U in (0, 1] from Philox with the
 * context's seed, counter (group, r low, r high, 0x60000000 | t), accepted
 * iff the exponent is >= 0 or log U is below it).  States stay with their
 * chains; betas (pns_read_betas) and the ladder (pns_read_ladder) move.
 * accepted [num_chains] int32 (host or device, or NULL) receives 1 at the
 * position t of each accepted pair and 0 elsewhere.  Queued on the
 * context's stream (synchronises for a host `accepted` and on the first
 * call).  Errors: PNS_EINVAL (temps < 2 or not dividing the chains, a group
 * across two problems, round < 0), PNS_EDEVICE.
 */
int pns_pt_swap(pns_ctx* ctx, int32_t temps, int64_t round, int32_t* accepted);

/* Current inverse temperature of every chain [num_chains], host or device. */
int pns_read_betas(pns_ctx* ctx, double* betas);

/* Tempering ladder [num_chains]: entry g*temps + t is the chain of group g
 * (0..temps-1) at temperature position t.  Errors: PNS_EINVAL (no swap yet). */
int pns_read_ladder(pns_ctx* ctx, int32_t* ladder);

/*
 * Recompute every chain's local fields h = offdiag(Q) x and energy x^T Q x
 * from its current state, overwriting the incrementally maintained values:
 * H = X A for all chains of a problem as one matrix product on the matrix
 * cores (integer Q on the int8 cores, split into bytes, exact; float Q on the
 * FP64 cores), the computation that also gives the initial fields on
 * creation.  Integer fields are exact either way; float32 Q fields are
 * accumulated in FP64 each flip, so their drift over 1e5 flips stays near
 * FP64 rounding, and a refresh resets it.  States, step counters and the
 * last record are unchanged.  Asynchronous on the context's stream.
 * Errors: PNS_EINVAL (NULL ctx), PNS_EDEVICE.
 */
int pns_refresh(pns_ctx* ctx);

/* ---- kernel timing per launch class ----
 *
 * The chains of a context are grouped into launch classes (same tile and
 * kernel flavour); a batch's classes run concurrently on their own streams.
 * With profiling on, every pns_run records a HIP event before the first and
 * after the last launch of each class on that class's stream and adds their
 * elapsed time.  Events inside a replayed graph cannot be timed, so a
 * context of the graph form queues the same launches directly while
 * profiling is on.  Profiling waits at the start of each pns_run for the
 * previous run's events (one host synchronisation per run). */
typedef struct pns_class_profile {
    int32_t block, groups;  /* tile of the class                               */
    int32_t flavour;        /* as pns_problem_info.flavour                     */
    int32_t chains;         /* chains of the class                             */
    int32_t N_min, N_max;   /* smallest and largest problem of the class       */
    int64_t launches;       /* kernel launches timed                           */
    double kernel_ms;       /* summed event time of the class's launches       */
    int64_t flips;          /* flips of the class's chains while profiling     */
    int64_t records;        /* records (steps) of the class's chains           */
    double row_bytes;       /* algorithmic bytes: one row of the flipped bit's
                               problem per flip, N * sizeof(Q element)         */
} pns_class_profile;

/* enable = 1 starts (and resets) per-class timing and counting, 0 stops it.
 * Synchronises the context's stream.  Errors: PNS_EINVAL (NULL ctx),
 * PNS_EDEVICE. */
int pns_profile(pns_ctx* ctx, int32_t enable);

/* *count = number of launch classes; with out != NULL (capacity entries)
 * fills one pns_class_profile per class, in class order.  Synchronises.
 * Errors: PNS_EINVAL (NULL ctx or count, capacity too small, profiling never
 * started), PNS_EDEVICE. */
int pns_profile_read(pns_ctx* ctx, pns_class_profile* out, int32_t capacity, int32_t* count);

/* Launch class of every chain: cls [num_chains] (host). */
int pns_class_of_chain(const pns_ctx* ctx, int32_t* cls);

/* ---- checkpoints (resume) ----
 *
 * Every draw of a step is keyed by (seed, chain id, step), so a chain
 * continues exactly where it stopped once its state and step counter are
 * restored: K steps, pns_save, pns_load into a new context, K more steps give
 * the records, states and counters of 2K steps in one run.
 *
 * pns_save writes the state of every chain into buf (host or device, caller
 * owned, `capacity` bytes): current bits x, local fields h, energy E,
 * remaining budget L and partial-neighbor-set index of Alg 6, step counter,
 * last record, counters, inverse temperatures (tempering permutes them), the
 * chain ids, and where present the random sets of UNBIASED_RAND, the
 * tempering ladder and the best states of pns_optimize; then a checksum.
 * *size receives the byte count; with buf == NULL only *size is set.
 * Logs, histograms and snapshots are outputs, not state, and are not saved;
 * Q is not saved either (the caller recreates the context from it).
 * Synchronises the context's stream.  Errors: PNS_EINVAL (NULL ctx or size,
 * capacity below the size), PNS_EDEVICE.
 */
int pns_save(pns_ctx* ctx, void* buf, int64_t capacity, int64_t* size);

/* Restore a checkpoint of pns_save into ctx (buf host or device, `size`
 * bytes).  ctx must have been created like the saved context: same mode,
 * element and field type, seed, chain ids, and the same problems in the same
 * order (N, layout, subset size, L0, chains; pass explicit subset sizes when
 * the autotuner could choose differently).  The tile and launch form may
 * differ.  Errors: PNS_EINVAL (not a checkpoint, wrong size or checksum, a
 * context that differs in any of the above; nothing is changed then),
 * PNS_ENOMEM, PNS_EDEVICE. */
int pns_load(pns_ctx* ctx, const void* buf, int64_t size);

/* ---- differentiation path ----
 *
 * The target pi_beta(x) = exp(-beta x^T Q x) / Z(Q, beta) gives
 * d log Z / d Q_ij = -beta E_pi[x_i x_j] for every entry of Q (Sec 4 target;
 * the derivative of the log of a sum of exponentials), and the jump chain
 * estimates E_pi[f] by sum_k M_k f(J_k) / sum_k M_k (Sec 1.2, multiplicity
 * list).  These entry points compute the multiplicity-weighted moment matrix
 * of records and, for small N, log Z itself.
 */

/*
 * G = X^T diag(m) X = sum_k m_k x_k x_k^T over K records.
 *   X      [K][ldx] bytes, record k in row k, bit i in byte i (nonzero = 1),
 *          ldx >= N; host or device.
 *   m      [K] int64 weights (multiplicities; negative values count as 0),
 *          host or device.
 *   G      [N][N] FP64 output, overwritten, host or device.
 *   sum_m  receives sum_k m_k (exact below 2^53) as one FP64, host or
 *          device, or NULL.
 *   stream hipStream_t to queue on (NULL: the default stream).  With X, m,
 *          G and sum_m all in device memory the call only queues work;
 *          any host buffer makes it synchronise the stream before it
 *          returns.
 * Computed on the bf16 matrix cores with FP32 accumulation: x is exact in
 * bf16 and each m_k is split into up to three bf16 pieces (exact for
 * m_k < 2^24), so every product is an exact integer.  The FP32
 * accumulators are added into G (FP64) every F records with
 * F * max(m) < 2^24 (F >= 64), so G is exact whenever m_k <= 2^18 for
 * every k; beyond that each partial sum carries a relative error below
 * 64 * 2^-24 and, for m_k >= 2^24, the weight itself is rounded to 24
 * bits.
 * Errors: PNS_EINVAL (NULL X, m or G, N outside [1, 32768], K < 0,
 * ldx < N), PNS_ENOMEM, PNS_EDEVICE.
 */
int pns_moments(const uint8_t* X, int64_t ldx, const int64_t* m, int64_t K, int32_t N, double* G, double* sum_m,
                void* stream);

/*
 * pns_moments over the snapshot buffer of the chains of one problem of a
 * context (every stored snapshot of every chain of the problem: the state J
 * and multiplicity M of the record at each snapshot step; slots not yet
 * written weigh 0).  G is [N][N] FP64 and sum_m one FP64, each host or
 * device (or sum_m NULL).  Queued on the context's stream; synchronises it
 * only when G or sum_m is in host memory.
 * Errors: PNS_EINVAL (NULL ctx or G, snapshots off, problem out of range),
 * PNS_ENOMEM, PNS_EDEVICE.
 */
int pns_snapshot_moments(pns_ctx* ctx, int32_t problem, double* G, double* sum_m);

/*
 * G = X^T diag(w) X = sum_k w_k x_k x_k^T with real (FP64) weights, e.g. the
 * expected multiplicities of pns_read_rb_weights (the Rao-Blackwellised
 * ratio estimator of Thm 3 (5)).  Arguments as pns_moments, with
 *   w      [K] FP64 weights of any sign, host or device; non-finite weights
 *          count as 0 in G and in the sum.
 *   sum_w  receives sum_k w_k (FP64 atomics: exact up to FP64 rounding in
 *          an unspecified order), host or device, or NULL.
 * The weights are scaled by the power of two 2^-e, e = ilogb(max_k |w_k|),
 * rounded to FP32 (relative error <= 2^-24) and split exactly into three bf16
 * pieces; the matrix cores then form exact products, which each wave sums in
 * FP32 over R records before the FP64 reduction, R = 32 max(32,
 * ceil(ceil(K / 32) T / 2048)) with T = t (t + 1) / 2, t = ceil(N / 64).
 * Hence |G_ij - exact| <= (3 R + 2) 2^-24 sum_k |w_k| x_ki x_kj (a worst-case
 * bound; typical errors are near sqrt(R) 2^-24) for weights within 2^100 of
 * the largest; smaller ones fall below the bf16 normal range and may lose
 * their low pieces.
 * Errors: as pns_moments.
 */
int pns_moments_f64(const uint8_t* X, int64_t ldx, const double* w, int64_t K, int32_t N, double* G, double* sum_w,
                    void* stream);

/*
 * pns_moments without any allocation, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving or training
 * loops, harnesses that forbid hipMalloc.  Same arguments, kernels and
 * results as pns_moments, except:
 *   - X, m, G and sum_m (or NULL) must be device memory (PNS_EINVAL
 *     otherwise): nothing is staged, and the call only queues work on
 *     `stream`;
 *   - the workspace (weight pieces, packed records, partial tiles) is a
 *     static 32 MiB array on each GPU, held until the process ends; a call
 *     whose workspace would exceed it is refused with PNS_EINVAL (about
 *     K * N / 8 bytes of packed records plus 16 KiB per 64 x 64 tile of the
 *     upper triangle; K = 131072 records of N = 512 fit);
 *   - every call on a GPU uses that GPU's one workspace: calls that overlap
 *     on one GPU (other streams, other threads) race and must be ordered by
 *     the caller.  The workspace keeps the last call's contents; each call
 *     clears what it accumulates into.
 * The device is the calling thread's current device (the stream's device).
 * Errors: PNS_EINVAL (as pns_moments, host buffers, workspace too small),
 * PNS_EDEVICE.
 */
int pns_moments_noalloc(const uint8_t* X, int64_t ldx, const int64_t* m, int64_t K, int32_t N, double* G,
                        double* sum_m, void* stream);

/*
 * Rao-Blackwell weights (Thm 3 (2), (5)): the expected multiplicity of a
 * record given its state J_k, its subset and, for a budgeted record
 * (Unbiased PNS, Alg 6, and runs of exact original time), the remaining
 * budget L at the start of the record: with p the escape probability of the
 * step and M = 1 + G, G ~ Geometric(p) counting failures,
 *     w = E[min(M, L)] = (1 - (1 - p)^L) / p,   and w = 1 / p unbudgeted,
 * (w = 1 for p >= 1; p <= 0, where every weight underflowed, gives L, or
 * +inf unbudgeted; w = 1 in optimization runs, where M = 1).
 * sum_k w_k h(J_k) / sum_k w_k estimates pi(h) like the multiplicity-weighted
 * average, with the sampling noise of M removed.
 *   log_w   [num_chains][log_capacity] weights of the per-step log ring
 *           (slots as pns_read_log); PNS_EINVAL if the log is off.
 *   snap_w  [num_chains][snapshot_capacity] weights of the snapshots (slots
 *           as pns_read_snapshots, unwritten slots 0); PNS_EINVAL if
 *           snapshots are off.
 *   hist_rb [2^N] sum of the weights of the records per state (pooled over
 *           chains, cleared by pns_hist_clear); PNS_EINVAL if histograms
 *           are off.
 * Any pointer may be NULL; each is host or device.  Synchronises.
 */
int pns_read_rb_weights(pns_ctx* ctx, double* log_w, double* snap_w, double* hist_rb);

/*
 * pns_snapshot_moments with the snapshots' expected multiplicities
 * (pns_read_rb_weights) as weights, through pns_moments_f64 (same error
 * bound); *sum_w receives their sum.  Queued on the context's stream;
 * synchronises it only when G or sum_w is in host memory.
 * Errors: as pns_snapshot_moments.
 */
int pns_snapshot_moments_rb(pns_ctx* ctx, int32_t problem, double* G, double* sum_w);

/*
 * Gradient of log Z(Q, beta) = log sum_x exp(-beta x^T Q x) from the
 * snapshots of one problem: d log Z / d Q_ij = -beta E_pi[x_i x_j], with
 * E_pi estimated by the weighted average of the snapshot states (the ratio
 * estimator of Thm 3 (5), h = x_i x_j), i.e.
 *     grad = -beta * G / sum_w,  G = pns_snapshot_moments (rb = 0: weights
 *     M) or pns_snapshot_moments_rb (rb != 0: expected multiplicities).
 *   grad   [N][N] FP64, device memory: receives the gradient (the full
 *          matrix; only Q_ij + Q_ji is identifiable, as x_i^2 = x_i).
 *   sum_w  one FP64, device memory: receives sum_w (a zero sum gives
 *          non-finite entries).
 * Queued on the context's stream; no host wait.
 * Errors: PNS_EINVAL (NULL or host buffers, beta not finite, as
 * pns_snapshot_moments), PNS_EDEVICE.
 */
int pns_logz_grad(pns_ctx* ctx, int32_t problem, double beta, int32_t rb, double* grad, double* sum_w);

/*
 * log Z(Q, beta) = log sum_x exp(-beta x^T Q x) by enumeration of all 2^N
 * states on the device (Gray-code order, incremental energies: exact int64
 * for integer Q, FP64 for float Q; FP64 log-sum-exp).  Q [N][N] of `dtype`
 * in `layout`, host or device; *out is host or device.  Synchronises
 * `stream` (NULL: the default stream).
 * Errors: PNS_EINVAL (N outside [1, 32], bad dtype or layout, beta < 0 or
 * not finite), PNS_ENOMEM, PNS_EDEVICE.
 */
int pns_log_partition(const void* Q, int32_t N, int32_t dtype, int32_t layout, double beta, double* out,
                      void* stream);

/* ---- continuous states: Unbiased PNS for the continuous case (Alg 7) ----
 *
 * Target on R^dim (the donut of Sec 7, written for any dimension):
 *     log pi(x) = -(|x|^2 - mu0)^2 / (2 sigma^2) + const.
 * Proposal: increments with i.i.d. N(0, 1) coordinates (Sec 7), symmetric,
 * so every acceptance ratio is pi(y) / pi(x).  A partial neighbor set is
 * `pairs` offsets delta_1..delta_P drawn from the proposal, each used with
 * both signs (Sec 7: 25 pairs, 50 neighbours; the pairs make the set
 * reversible); neighbour j of x is x + delta_j (j < P) and x - delta_{j-P}
 * (P <= j < 2P).  As in Alg 6, with M = 1 + Geometric(p) and
 * p = (1 / 2P) sum_j min(1, pi(y_j) / pi(x)):  M <= L jumps to a neighbour
 * chosen proportionally to min(1, pi(y_j) / pi(x)), L -= M;  otherwise the
 * chain stays (record M = L), L = L0 and a new set is drawn (Alg 7).
 * Reading: the proposal restricted to the finite set is uniform over its
 * 2P points.
 * Random numbers: Philox4x32-10 keyed by the seed; step k of a chain uses
 * counter (chain id, k low, k high, 0) (U1 = (top 53 bits of words 0,1 + 1)
 * 2^-53 for M, U2 = top 53 bits of words 2,3 2^-53 for the choice); the
 * offsets of set s use counter (chain id, s low, s high, 0x80000000 |
 * j << 8 | t) and Box-Muller (coordinates 2t, 2t + 1 of pair j).
 * One wave of 64 lanes per chain on the device (2P <= 64).
 */
typedef struct pns_cont pns_cont;

typedef struct pns_cont_opts {
    int32_t dim;            /* 1 .. 7 (Sec 7: 2)                                */
    int32_t pairs;          /* P, 1 .. 32: 2P neighbours per set (Sec 7: 25)    */
    double mu0;             /* squared radius of the donut (Sec 7: 9)           */
    double sigma;           /* width (Sec 7: 0.1), > 0                          */
    int64_t L0;             /* original samples per set, 1 .. 2^53 (Sec 7: 1000) */
    uint64_t seed;
    int32_t num_chains;     /* >= 1                                             */
    uint32_t chain_id_base; /* chain c uses counter word chain_id_base + c      */
    const double* x0;       /* [num_chains][dim] initial states, host or device;
                               NULL: the origin.  Copied on create.              */
    int64_t log_capacity;   /* per-step log ring per chain (0 = off)            */
    void* stream;           /* hipStream_t (NULL: the context creates its own)  */
    int32_t reserved[8];    /* must be zero                                       */
} pns_cont_opts;

/* Sec 7 defaults: dim 2, 25 pairs, mu0 9, sigma 0.1, L0 1000, one chain. */
void pns_cont_opts_default(pns_cont_opts* opts);

/*
 * Create a continuous sampler; the chains start at x0 with L = L0, set 0,
 * step 0.  Errors: PNS_EINVAL (dim, pairs, sigma, mu0, L0, num_chains,
 * log_capacity out of range, non-finite x0, nonzero reserved fields),
 * PNS_ENOMEM, PNS_EDEVICE.  Synchronises.
 */
int pns_cont_create(pns_cont** ctx, const pns_cont_opts* opts);

/* Queue `steps` records per chain (launches of at most 8192 records). */
int pns_cont_run(pns_cont* ctx, int64_t steps);

/*
 * Chain state: states [num_chains][dim], log pi of each state (without the
 * constant), remaining budgets L, set indices and record counters
 * [num_chains].  Any pointer may be NULL; each is host or device.
 * Synchronises.
 */
int pns_cont_read(pns_cont* ctx, double* states, double* log_density, int64_t* L, int64_t* set_index,
                  int64_t* step);

/*
 * Per-step log ring [num_chains][log_capacity] (record k at slot k mod
 * log_capacity): neighbour index 0 .. 2P-1 or PNS_STAY, multiplicity M,
 * log pi of the record's state, p, and the expected multiplicity
 * (1 - (1 - p)^L) / p of the record (the Rao-Blackwell weight of
 * pns_read_rb_weights).  Any pointer may be NULL; each is host or device.
 * Errors: PNS_EINVAL if the log is off.  Synchronises.
 */
int pns_cont_read_log(pns_cont* ctx, int32_t* actions, int64_t* multiplicities, double* log_density, double* p,
                      double* weights);

/*
 * Estimator sums per chain [num_chains][2][4 dim + 1] (FP64), accumulated
 * over every record since creation or the last pns_cont_clear_sums, with
 * weights M (row 0) and the expected multiplicities (row 1): sum w, then
 * sum w x_i, sum w x_i^2, sum w x_i^4 and sum w 1(x_i > 0) for
 * i = 0 .. dim-1.  Their ratios are the estimators of Sec 7 (E[x_i],
 * E[x_i^2], E[x_i^4], P(x_i > 0)).  Host or device.  Synchronises.
 */
int pns_cont_read_sums(pns_cont* ctx, double* sums);

/* Zero the estimator sums (e.g. after burn-in), queued on the stream. */
int pns_cont_clear_sums(pns_cont* ctx);

/* Jumps and stays per chain [num_chains], host or device.  Synchronises. */
int pns_cont_stats(pns_cont* ctx, int64_t* jumps, int64_t* stays);

/* Wait for the queued work of the context. */
int pns_cont_sync(pns_cont* ctx);

/* Release the context (NULL is accepted). */
int pns_cont_destroy(pns_cont* ctx);

#ifdef __cplusplus
}
#endif

#endif /* PNS_H */
