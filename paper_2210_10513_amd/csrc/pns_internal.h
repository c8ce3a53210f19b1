// Internal interface between the C-ABI runtime (pns_runtime.cpp) and the
// HIP kernels (pns_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pns {

enum QType : int32_t { Q_I16 = 0, Q_I32 = 1, Q_F32 = 2 };
enum HType : int32_t { H_I32 = 0, H_I64 = 1, H_F64 = 2 };

// One QUBO problem as the kernels see it.  A holds the off-diagonal part of
// the coefficient matrix with a zero diagonal, row-major with `pitch`
// elements per row (pitch is a multiple of 64, padding entries are zero);
// diag holds Q_jj widened to int32 (integer Q) or float (F32 Q).  A bit flip
// of c changes the field of j by +-A[c][j] and dE_j = (1-2x_j)(diag_j + s h_j).
struct Problem {
    const void* A;
    const void* diag;
    int64_t pitch;
    int64_t num_sets;  // systematic sets N / gcd(N, n)
    int64_t L0;
    int32_t N;
    int32_t n;
    int32_t s;         // 2 for symmetric input, 1 for upper-triangular input
    int32_t qtype;     // QType
};

// Everything a step kernel launch needs.  Chain c of the context stores its
// state at field offset foff[c] (fields x, h, rand-set membership) and at
// index c in the per-chain arrays.
struct StepArgs {
    const Problem* problems;
    const int32_t* chain_problem;   // [C]
    const int64_t* foff;            // [C]
    const int32_t* chain_list;      // chains of this launch (NULL: chain_first + blockIdx.x)
    int32_t chain_first;
    int32_t mode;
    int64_t steps;                  // steps per chain in this launch
    uint64_t seed;
    const double* beta;             // [C]
    const uint32_t* chain_id;       // [C]
    // chain state
    uint8_t* x;                     // [fields]
    void* h;                        // [fields] of the field type
    uint8_t* rmem;                  // [fields] random-set membership (UNBIASED_RAND)
    int64_t* E;                     // [C] energy bits (int64 or double)
    int64_t* L;                     // [C]
    int64_t* sub;                   // [C]
    int64_t* step;                  // [C]
    int32_t* last_action;           // [C]
    int64_t* last_M;                // [C]
    int64_t* last_E;                // [C] energy bits of the last record
    // counters [C][6]: steps, flips, stays, saturated, sum_M (double bits),
    // anomalies (selection found no positive weight; must stay 0)
    int64_t* counters;
    // optional outputs
    int32_t* log_action;            // [C][log_cap]
    int64_t* log_M;
    int64_t* log_E;                 // energy bits
    double* log_p;
    double* log_w;                  // expected multiplicity of the record (Rao-Blackwell weight)
    int64_t log_cap;
    unsigned long long* hist_w;     // [2^N]
    unsigned long long* hist_v;
    double* hist_rb;                // [2^N] sum of expected multiplicities
    int32_t snap_every;
    int32_t snap_cap;
    uint8_t* snap_x;                // [C][snap_cap][snap_pitch]
    int64_t* snap_M;                // [C][snap_cap]
    int64_t* snap_E;                // [C][snap_cap]
    double* snap_w;                 // [C][snap_cap] expected multiplicity of the record
    int32_t* snap_count;            // [C]
    int64_t snap_pitch;
    // optimization runs (mode 4, instrumented kernels only)
    double inv_temp;                // 1 / T (1 for sampling)
    int64_t orig_time;              // > 0: advance by this many original samples (RF, Basic)
    uint8_t* xbest;                 // [fields] best state X_max, or NULL
    int64_t* Ebest;                 // [C] its energy bits
};

struct InitArgs {
    const Problem* problems;
    const int32_t* chain_problem;
    const int64_t* foff;
    int32_t num_chains;
    int32_t init;                   // 0 zero, 1 random, 2 given (x already in place)
    uint64_t seed;
    const uint32_t* chain_id;
    uint8_t* x;
    void* h;
    int64_t* E;
    int64_t* last_E;
};

// Step kernel launch for one (block, groups) tile shape, field type and Q
// type.  flav: 0 every bit, 1 systematic window, 2 random subset drawn in
// LDS; instr: per-step log / histograms / snapshots compiled in.  Returns
// hipSuccess or the launch error; with probe = true only reports whether
// the tile exists.  dyn_lds is the dynamic LDS byte count (random subsets).
hipError_t launch_steps(int32_t qtype, int32_t htype, int32_t flav, bool instr, int32_t block, int32_t groups,
                        int32_t grid, size_t dyn_lds, hipStream_t stream, const StepArgs& args);
hipError_t launch_steps_i16(int flav, bool instr, int block, int groups, int grid, size_t dyn, hipStream_t st,
                            const StepArgs& a, bool probe);
hipError_t launch_steps_i32(int flav, bool instr, int block, int groups, int grid, size_t dyn, hipStream_t st,
                            const StepArgs& a, bool probe);
hipError_t launch_steps_i64(int flav, bool instr, int block, int groups, int grid, size_t dyn, hipStream_t st,
                            const StepArgs& a, bool probe);
hipError_t launch_steps_f32(int flav, bool instr, int block, int groups, int grid, size_t dyn, hipStream_t st,
                            const StepArgs& a, bool probe);

// Window kernels of one, two or four waves per chain (flavour 5: Unbiased
// PNS with systematic sets, integer coefficients with int32 fields).
hipError_t launch_waves_i16(bool instr, int block, int groups, int grid, hipStream_t st, const StepArgs& a,
                            bool probe);
hipError_t launch_waves_i32(bool instr, int block, int groups, int grid, hipStream_t st, const StepArgs& a,
                            bool probe);

// True if a step kernel exists for this tile shape and types.
bool have_tile(int32_t qtype, int32_t htype, int32_t block, int32_t groups);
// True if a window kernel (flavour 5) exists for this tile shape and types.
bool have_wave_tile(int32_t qtype, int32_t htype, int32_t block, int32_t groups);

// Bytes of readable padding after the last row of a coefficient matrix: the
// window kernels load whole tiles of a row (up to 16384 elements of 4 bytes
// from its start) and drop what lies past the pitch.
constexpr size_t kRowTailBytes = 16384 * 4;

// Initial bits (random policy), fields h = A x (matrix-core products over
// the chains of each problem) and energies of every chain.
// host_chain_problem mirrors args.chain_problem on the host, host_pitch the
// problems' pitches (indexed by problem).  last_E may be NULL (left as is).
hipError_t launch_init_with_map(int32_t qtype, int32_t htype, int32_t max_pitch, hipStream_t stream,
                                const InitArgs& args, const int32_t* host_chain_problem, const int64_t* host_pitch);

// A, diag of a coefficient matrix on the device (one workgroup per row) and
// the checks of its entries: flags [4] (asymmetry, non-finite, max row sum
// of |A| and max |diag| as FP64 bits), accumulated with atomics.
hipError_t launch_prepare_rows(int32_t qtype, const void* Q, int32_t N, int32_t layout, int64_t pitch, void* A,
                               void* diag, unsigned long long* flags, hipStream_t st);

// One parallel-tempering swap round over groups of T consecutive chains
// (ladder [groups][T]: the chain of the group at each temperature position;
// E as int64 or FP64 bits; accepted [C] or NULL).
hipError_t launch_pt_swap(const int64_t* E, int32_t is_float, double* beta, int32_t* ladder, int32_t groups, int32_t T,
                          uint64_t seed, uint64_t round, int32_t* accepted, hipStream_t st);

// G <- G * (-beta / *sum) on the device (G [n], sum one FP64 in device memory).
hipError_t launch_moments_to_grad(double* G, int64_t n, double beta, const double* sum, hipStream_t st);

// A single wave that waits `ticks` of the device's wall clock on `st` and
// exits (a bounded delay between two groups of launches).
hipError_t launch_hold(uint64_t ticks, hipStream_t st);

// Fill `count` 64-bit words with a value (graph-safe alternative to memset).
hipError_t launch_fill64(void* p, int64_t count, int64_t value, hipStream_t stream);

// Record the message of a failed call for pns_last_error() on this thread
// and return `code` (printf-style message).
int set_error(int code, const char* fmt, ...);

}  // namespace pns

namespace pns {

// Differentiation path (pns_moments.hip).
// Weight pieces (3 x kpad bf16), exact sum and max of the weights.
hipError_t launch_moments_prep(const int64_t* m, int64_t K, int64_t kpad, uint16_t* pieces, unsigned long long* sum_m,
                               unsigned long long* max_m, hipStream_t st);
// Records X [K][ldx] bytes -> column-packed bits Xb [words][npad] u32,
// words = ceil(K / 32), npad = N rounded up to 64.
hipError_t launch_pack_bits(const uint8_t* X, int64_t ldx, int64_t K, int32_t N, int32_t npad, int64_t words,
                            uint32_t* Xb, hipStream_t st);
// G += X^T diag(m) X from packed records: one wave per (64 x 64 tile of the
// upper triangle, chunk of chunk_words words), partial tiles in `part`
// [chunks][tiles][64][64] FP32, then an FP64 reduction into G.
hipError_t launch_moments(const uint32_t* Xb, int32_t npad, int64_t words, int32_t N, const uint16_t* pieces,
                          int64_t kpad, int64_t chunk_words, const unsigned long long* max_m, float* part, double* G,
                          hipStream_t st);
// ---- continuous Unbiased PNS (Alg 7, donut target) ----
struct ContArgs {
    int32_t dim;                    // 1 .. 7
    int32_t pairs;                  // P: 2P neighbours per set, 1 .. 32
    double mu0;                     // donut: log pi = -(|x|^2 - mu0)^2 c
    double c;                       // 1 / (2 sigma^2), rounded once
    int64_t L0;
    uint64_t seed;
    int32_t num_chains;
    const uint32_t* chain_id;       // [C]
    double* x;                      // [C][dim]
    double* lpx;                    // [C] log pi of the state
    int64_t* L;                     // [C] remaining budget
    int64_t* set;                   // [C] index of the current partial neighbor set
    int64_t* step;                  // [C] records so far
    int64_t* counters;              // [C][2] jumps, stays
    double* sums;                   // [C][2][4 dim + 1] estimator sums (M, expected multiplicity)
    int64_t steps;                  // records per chain in this launch
    int64_t log_cap;                // per-step log ring (0: off)
    int32_t* log_action;
    int64_t* log_M;
    double* log_lp;
    double* log_p;
    double* log_w;
};
// init = true: lpx from x; else `steps` records per chain.
hipError_t launch_cont(const ContArgs& a, bool init, hipStream_t st);

// Weight pieces of FP64 weights: *maxbits (zeroed by the caller) receives the
// largest finite |w| (as bits), the weights are scaled by 2^-ilogb(max),
// rounded to FP32 and split exactly into three bf16; *sum_w (zeroed) receives
// their unscaled FP64 sum.  Non-finite weights count as 0.
hipError_t launch_moments_prep_f64(const double* w, int64_t K, int64_t kpad, uint16_t* pieces, double* sum_w,
                                   unsigned long long* maxbits, hipStream_t st);
// G[0..n) *= 2^ilogb(max): undoes the weight scaling of launch_moments_prep_f64.
hipError_t launch_moments_unscale(double* G, int64_t n, const unsigned long long* maxbits, hipStream_t st);
// *out = (double)*sum_m on the device.
hipError_t launch_moments_sum(const unsigned long long* sum_m, double* out, hipStream_t st);
// log Z by enumeration: `blocks` x 256 threads, thread t covers the states
// with high bits t and all 2^lowbits low bits; part_* hold `blocks` pairs.
hipError_t launch_logz(int32_t qtype, const void* Q, int32_t N, int32_t layout, double beta, double* part_max,
                       double* part_sum, int32_t blocks, int32_t lowbits, int64_t nthreads, double* out, hipStream_t st);

}  // namespace pns
