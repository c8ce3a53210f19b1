// C-ABI runtime of the Partial Neighbor Search sampler (see include/pns.h).
//
// Owns the device memory of a sampler context, prepares each coefficient
// matrix (zero-diagonal off-diagonal part A with a padded pitch, diagonal
// split off, symmetry and field-bound checks), chooses workgroup tiles (fixed
// table or timed trials), groups the chains of uneven-N problems into launch
// classes that run concurrently, queues the step kernels in the plain,
// persistent or HIP-graph form, and copies results to host or device buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "pns.h"
#include "pns_internal.h"

using namespace pns;

namespace {

thread_local std::string g_error;

int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what)
{
    return fail(PNS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

int pns::set_error(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

namespace {

#define HIP_TRY(call, what)                              \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

bool is_device_ptr(const void* p)
{
    if (p == nullptr) return false;
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice;
}

// Copy `bytes` from host memory to a caller buffer that is host or device.
int copy_out(void* dst, const void* src, size_t bytes)
{
    if (dst == nullptr || bytes == 0) return PNS_OK;
    if (is_device_ptr(dst)) {
        HIP_TRY(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice), "copy to device buffer");
    } else {
        std::memcpy(dst, src, bytes);
    }
    return PNS_OK;
}

// Copy `bytes` from a caller buffer (host or device) into host memory.
int copy_in(void* dst, const void* src, size_t bytes)
{
    if (bytes == 0) return PNS_OK;
    if (is_device_ptr(src)) {
        HIP_TRY(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost), "copy from device buffer");
    } else {
        std::memcpy(dst, src, bytes);
    }
    return PNS_OK;
}

template <typename T>
int dev_alloc(T** p, size_t count)
{
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(PNS_ENOMEM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T), hipGetErrorString(e));
    }
    return PNS_OK;
}

template <typename T>
int d2h(std::vector<T>& v, const void* src, size_t count)
{
    v.resize(count);
    if (count == 0) return PNS_OK;
    HIP_TRY(hipMemcpy(v.data(), src, count * sizeof(T), hipMemcpyDeviceToHost), "download");
    return PNS_OK;
}

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

int64_t gcd64(int64_t a, int64_t b)
{
    while (b) {
        int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

size_t qsize(int32_t qtype) { return qtype == Q_I16 ? 2 : 4; }

struct Tile {
    int32_t block, groups;
};

// Fixed tile table: smallest capacity (block * 4 * groups) covering N.
// Largest problem a tile holds (256 x 16: 64 fields per lane).
constexpr int32_t kMaxN = 16384;

Tile default_tile(int32_t N)
{
    if (N <= 256) return {64, 1};
    if (N <= 512) return {128, 1};
    if (N <= 1024) return {256, 1};
    if (N <= 2048) return {256, 2};
    if (N <= 4096) return {512, 2};
    if (N <= 8192) return {512, 4};
    return {1024, 4};
}

// Tiles of 32 or more fields per lane: the step kernel's four-wave tiles
// (three (256 x 8) or two (256 x 16) chains per compute unit where the table's
// tiles hold two or one) for the subsets whose weights touch at most two 4-bit
// groups per wave (compact and two-group windows), and the window kernel's
// tiles; the other flavours weigh every group of a lane and spill there.
bool wide_tile(Tile t) { return t.groups >= 8; }

// Every tile a kernel is compiled for: the step kernels' and (64 x 8 .. 24,
// 128 x 16 and 24, 256 x 16) the window kernels'.
// (Which exist for which types: have_tile and have_wave_tile tell.)
const Tile kTiles[] = {{64, 1},   {64, 2},  {64, 4},  {64, 8},   {64, 16},  {64, 24}, {128, 1},  {128, 2},
                       {128, 4},  {128, 16}, {128, 24}, {256, 1}, {256, 2},  {256, 4}, {256, 8},  {256, 16},
                       {512, 2},  {512, 4},  {1024, 2}, {1024, 4}};

// True if no window of n cyclically consecutive bits holds bits of two
// different 4-bit groups within one wave: the lanes of wave w in group g hold
// the contiguous range [(g*block + 64w)*4, +256) of bits.
bool window_compact_ok(int32_t N, int32_t n, int32_t block, int32_t groups)
{
    if (groups == 1) return true;
    if (n >= N) return false;
    for (int32_t w = 0; w < block / 64; ++w) {
        for (int32_t ga = 0; ga < groups; ++ga) {
            const int64_t a0 = ((int64_t)ga * block + 64 * w) * 4;
            if (a0 >= N) continue;
            const int64_t a1 = std::min<int64_t>(a0 + 255, N - 1);
            for (int32_t gb = 0; gb < groups; ++gb) {
                if (gb == ga) continue;
                const int64_t b0 = ((int64_t)gb * block + 64 * w) * 4;
                if (b0 >= N) continue;
                // shortest forward distance from a bit of range a to a bit of range b
                if (((b0 - a1) % N + N) % N < n) return false;
            }
        }
    }
    return true;
}

// True if every window the run uses -- the systematic sets S_i = {(i n + t)
// mod N : t < n}, i < N / gcd(N, n), or all bits when n >= N -- holds bits of
// at most two different 4-bit groups within any one wave.
bool window_two_groups_ok(int32_t N, int32_t n, int32_t block, int32_t groups)
{
    if (groups <= 2) return true;
    const int64_t sets = n >= N ? 1 : N / gcd64(N, n);
    for (int64_t i = 0; i < sets; ++i) {
        const int64_t s0 = n >= N ? 0 : (i * n) % N;
        for (int32_t w = 0; w < block / 64; ++w) {
            int hit = 0;
            for (int32_t g = 0; g < groups; ++g) {
                const int64_t a0 = ((int64_t)g * block + 64 * w) * 4;
                if (a0 >= N) continue;
                const int64_t a1 = std::min<int64_t>(a0 + 255, N - 1);
                // the window [s0, s0 + n) (cyclic) meets [a0, a1]
                const bool meets = n >= N || ((a0 - s0) % N + N) % N < n || ((s0 - a0) % N + N) % N <= a1 - a0;
                hit += meets ? 1 : 0;
            }
            if (hit > 2) return false;
        }
    }
    return true;
}

// True if every systematic set of the run, S_i = {(i n + t) mod N : t < n},
// meets at most four of any one wave's groups: the window kernel stages the
// energy differences of that many groups per wave.
bool window_slots_ok(int32_t N, int32_t n, int32_t block, int32_t groups)
{
    if (n >= N || N > 16384) return false;
    const int32_t W = block / 64;
    const int64_t sets = N / gcd64(N, n);
    auto range = [](int64_t lo, int64_t hi) { return (~0ull >> (63 - hi)) & (~0ull << lo); };
    for (int64_t i = 0; i < sets; ++i) {
        const int64_t st = (i * n) % N;
        const int64_t e0 = std::min<int64_t>(st + n, N);
        uint64_t m = range(st >> 8, (e0 - 1) >> 8);
        if (st + n > N) m |= range(0, (st + n - N - 1) >> 8);
        for (int32_t w = 0; w < W; ++w) {
            int hit = 0;
            for (int32_t g = 0; g < groups && g * W + w < 64; ++g) hit += (m >> (g * W + w)) & 1ull ? 1 : 0;
            if (hit > 4) return false;
        }
    }
    return true;
}

// How the step kernel forms the subset: 0 every bit, 1 systematic window,
// 2 random subset drawn in LDS, 3 compact systematic window, 4 two-group
// systematic window.
int32_t flavour_of(int32_t mode, int32_t N, int32_t n, int32_t block, int32_t groups)
{
    if (mode == PNS_MODE_RF) return 0;
    if (mode == PNS_MODE_BASIC) return n < N ? 2 : 0;
    if (mode == PNS_MODE_UNBIASED_SYS || n >= N) {
        if (window_compact_ok(N, n, block, groups)) return 3;
        return groups >= 2 && window_two_groups_ok(N, n, block, groups) ? 4 : 1;
    }
    return 2;
}

bool have_tile_any(int32_t qtype, int32_t htype, Tile t) { return have_tile(qtype, htype, t.block, t.groups); }

// Kernel flavour of a problem on tile t, or -1 if no kernel runs it there:
// the window kernel (5) where it exists and the run is Unbiased PNS with
// systematic sets whose windows fit its slots, else the step kernel's.
int32_t flavour_for(int32_t mode, int32_t N, int32_t n, Tile t, int32_t qtype, int32_t htype)
{
    if (mode == PNS_MODE_UNBIASED_SYS && have_wave_tile(qtype, htype, t.block, t.groups) &&
        window_slots_ok(N, n, t.block, t.groups))
        return 5;
    if (!have_tile(qtype, htype, t.block, t.groups)) return -1;
    return flavour_of(mode, N, n, t.block, t.groups);
}

// Default tile of a problem: above 4096 bits the wide tile of four waves when
// the problem's windows run a compact or two-group kernel on it (and a kernel
// exists for the field type), else the fixed table's.
Tile default_tile_for(int32_t mode, int32_t N, int32_t n, int32_t qtype, int32_t htype)
{
    const Tile t = default_tile(N);
    if (N > 4096) {
        const Tile w = N <= 8192 ? Tile{256, 8} : Tile{256, 16};
        const int32_t fl = flavour_for(mode, N, n, w, qtype, htype);
        if (fl == 3 || fl == 4 || fl == 5) return w;
    }
    return t;
}

// A problem's matrix as the kernels read it, prepared on the host.
struct Prepared {
    std::vector<uint8_t> A, D;  // A: N x pitch, zero diagonal; D: diagonal [pitch]
    double field_bound = 0.0;   // max_i sum_j |A_ij|
    double diag_bound = 0.0;    // max_i |Q_ii|
};

// Build the zero-diagonal off-diagonal matrix A (pitch-padded) and the
// diagonal from the caller's Q, check symmetry (SYMMETRIC) and finiteness,
// and bound the fields.  Rows are split over host threads and walked in
// 64 x 64 tiles so that the transposed reads stay in cache.
template <typename QT>
int prepare_matrix(const QT* Q, int32_t N, int32_t layout, int64_t pitch, Prepared* out)
{
    using DW = typename std::conditional<std::is_same<QT, float>::value, float, int32_t>::type;
    constexpr bool kFloat = std::is_same<QT, float>::value;
    out->A.assign((size_t)N * pitch * sizeof(QT), 0);
    out->D.assign((size_t)pitch * sizeof(DW), 0);
    QT* A = reinterpret_cast<QT*>(out->A.data());
    DW* d = reinterpret_cast<DW*>(out->D.data());
    constexpr int32_t T = 64;
    const int32_t nblk = (N + T - 1) / T;
    const int nthreads = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::string> errs((size_t)nthreads);
    std::vector<double> fbs((size_t)nthreads, 0.0), dbs((size_t)nthreads, 0.0);
    auto work = [&](int t) {
        std::vector<double> rowsum(T);
        for (int32_t bi = t; bi < nblk; bi += nthreads) {
            const int32_t i0 = bi * T, i1 = std::min(N, i0 + T);
            std::fill(rowsum.begin(), rowsum.end(), 0.0);
            for (int32_t bj = 0; bj < nblk; ++bj) {
                const int32_t j0 = bj * T, j1 = std::min(N, j0 + T);
                for (int32_t i = i0; i < i1; ++i) {
                    for (int32_t j = j0; j < j1; ++j) {
                        if (i == j) {
                            const QT q = Q[(size_t)i * N + i];
                            if (kFloat && !std::isfinite((double)q)) {
                                char b[96];
                                snprintf(b, sizeof(b), "Q has a non-finite entry at (%d, %d)", i, i);
                                if (errs[t].empty()) errs[t] = b;
                            }
                            d[i] = (DW)q;
                            dbs[t] = std::max(dbs[t], std::fabs((double)q));
                            continue;
                        }
                        QT v;
                        if (layout == PNS_SYMMETRIC) {
                            v = Q[(size_t)i * N + j];
                            if (!(v == Q[(size_t)j * N + i]) && errs[t].empty()) {
                                char b[96];
                                snprintf(b, sizeof(b), "SYMMETRIC Q is not symmetric at (%d, %d)", i, j);
                                errs[t] = b;
                            }
                        } else {
                            v = i < j ? Q[(size_t)i * N + j] : Q[(size_t)j * N + i];
                        }
                        if (kFloat && !std::isfinite((double)v) && errs[t].empty()) {
                            char b[96];
                            snprintf(b, sizeof(b), "Q has a non-finite entry at (%d, %d)", i, j);
                            errs[t] = b;
                        }
                        A[(size_t)i * pitch + j] = v;
                        rowsum[i - i0] += std::fabs((double)v);
                    }
                }
            }
            for (int32_t i = i0; i < i1; ++i) fbs[t] = std::max(fbs[t], rowsum[i - i0]);
        }
    };
    if (nthreads == 1 || (int64_t)N * N < (1 << 20)) {
        for (int t = 0; t < nthreads; ++t) work(t);  // small matrices: no threads
    } else {
        std::vector<std::thread> pool;
        for (int t = 0; t < nthreads; ++t) pool.emplace_back(work, t);
        for (auto& th : pool) th.join();
    }
    for (int t = 0; t < nthreads; ++t)
        if (!errs[t].empty()) return fail(PNS_EINVAL, "%s", errs[t].c_str());
    out->field_bound = *std::max_element(fbs.begin(), fbs.end());
    out->diag_bound = *std::max_element(dbs.begin(), dbs.end());
    return PNS_OK;
}

// Copy a problem's Q in (host or device) and prepare it.
int prepare_problem(const void* Q, int32_t N, int32_t layout, int32_t qtype, Prepared* out)
{
    const int64_t pitch = round_up(N, 64);
    std::vector<uint8_t> qhost((size_t)N * N * qsize(qtype));
    int rc = copy_in(qhost.data(), Q, qhost.size());
    if (rc) return rc;
    if (qtype == Q_I16) return prepare_matrix(reinterpret_cast<const int16_t*>(qhost.data()), N, layout, pitch, out);
    if (qtype == Q_I32) return prepare_matrix(reinterpret_cast<const int32_t*>(qhost.data()), N, layout, pitch, out);
    return prepare_matrix(reinterpret_cast<const float*>(qhost.data()), N, layout, pitch, out);
}

int check_opts(const pns_opts* o)
{
    for (int i = 0; i < 7; ++i)
        if (o->reserved[i] != 0) return fail(PNS_EINVAL, "opts.reserved must be zero");
    if (o->dtype < PNS_I16 || o->dtype > PNS_F32) return fail(PNS_EINVAL, "unknown dtype %d", o->dtype);
    if (o->layout != PNS_SYMMETRIC && o->layout != PNS_UPPER) return fail(PNS_EINVAL, "unknown layout %d", o->layout);
    if (o->num_chains < 1) return fail(PNS_EINVAL, "num_chains must be >= 1");
    if (o->L0 < 0) return fail(PNS_EINVAL, "L0 must be >= 0");
    if (o->init < PNS_INIT_ZERO || o->init > PNS_INIT_GIVEN) return fail(PNS_EINVAL, "unknown init %d", o->init);
    if (o->init == PNS_INIT_GIVEN && o->x0 == nullptr) return fail(PNS_EINVAL, "INIT_GIVEN needs x0");
    if (o->launch < PNS_LAUNCH_PLAIN || o->launch > PNS_LAUNCH_GRAPH) return fail(PNS_EINVAL, "unknown launch %d", o->launch);
    if (o->chunk < 0) return fail(PNS_EINVAL, "chunk must be >= 0");
    if (o->log_capacity < 0) return fail(PNS_EINVAL, "log_capacity must be >= 0");
    if (o->snapshot_every < 0 || (o->snapshot_every > 0 && o->snapshot_capacity < 1))
        return fail(PNS_EINVAL, "snapshots need snapshot_every >= 0 and snapshot_capacity >= 1");
    return PNS_OK;
}

// One problem as the caller describes it, plus what the library derives.
struct ProblemSpec {
    const void* Q = nullptr;
    int32_t N = 0, layout = 0, n = 0, chains = 0;
    int64_t L0 = 100;
    std::vector<double> betas;
    Tile tile{0, 0};  // 0: default table
};

struct ProblemRun {
    int32_t N, n, layout, s, flav;
    int64_t pitch, L0, num_sets;
    int32_t chain_begin, chains;
    Tile tile;
    void* A = nullptr;
    void* diag = nullptr;
    void* A2 = nullptr;     // staging copies for pns_set_q (allocated on first use)
    void* diag2 = nullptr;
};

// Chains that share a tile shape and kernel flavour: one step-kernel launch.
struct LaunchClass {
    Tile tile;
    int32_t flav;
    size_t dyn;
    std::vector<int32_t> chains;
    int32_t* d_list = nullptr;
    double cost = 0.0;  // estimated time of one step of every chain of the class
};

// Side streams of a context with several launch classes.  HIP spreads a
// process's streams over its hardware queues (GPU_MAX_HW_QUEUES, 4 by
// default) and kernels on one queue run one after another, so classes are
// packed onto one stream per hardware queue (at most 16).
int max_side_streams()
{
    const char* e = std::getenv("GPU_MAX_HW_QUEUES");
    const int q = e ? std::atoi(e) : 4;
    return std::max(1, std::min(16, q > 0 ? q : 4));
}

struct SideStream {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    std::vector<int32_t> classes;  // launched in this order
};

}  // namespace

struct pns_ctx {
    int32_t mode = 0, qtype = 0, htype = 0;
    int32_t num_chains = 0;
    int32_t launch = PNS_LAUNCH_PERSISTENT;
    int32_t chunk = 0;
    uint64_t seed = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipEvent_t fork = nullptr;
    hipEvent_t fork_small = nullptr;  // release of the one-wave classes after a short hold
    uint64_t hold_ticks = 20000;      // 200 us of the device's wall clock (100 MHz unless it says otherwise)
    std::vector<SideStream> sides;
    std::vector<ProblemRun> probs;
    std::vector<int32_t> h_chain_problem;
    std::vector<int64_t> h_foff;
    std::vector<int64_t> h_offsets;  // concatenated per-chain bit arrays, [C+1]
    int64_t fields = 0, max_pitch = 0;
    std::vector<LaunchClass> classes;
    // device memory
    Problem* problems = nullptr;
    int32_t* chain_problem = nullptr;
    int64_t* foff = nullptr;
    double* beta = nullptr;
    uint32_t* chain_id = nullptr;
    uint8_t* x = nullptr;
    void* h = nullptr;
    uint8_t* rmem = nullptr;
    int64_t* E = nullptr;
    int64_t* L = nullptr;
    int64_t* sub = nullptr;
    int64_t* step = nullptr;
    int32_t* last_action = nullptr;
    int64_t* last_M = nullptr;
    int64_t* last_E = nullptr;
    int64_t* counters = nullptr;
    int64_t log_cap = 0;
    int32_t* log_action = nullptr;
    int64_t* log_M = nullptr;
    int64_t* log_E = nullptr;
    double* log_p = nullptr;
    double* log_w = nullptr;
    unsigned long long* hist_w = nullptr;
    unsigned long long* hist_v = nullptr;
    double* hist_rb = nullptr;
    int32_t snap_every = 0, snap_cap = 0;
    uint8_t* snap_x = nullptr;
    int64_t* snap_M = nullptr;
    int64_t* snap_E = nullptr;
    double* snap_w = nullptr;
    int32_t* snap_count = nullptr;
    // optimization runs: best states and their launch classes (built on first use)
    uint8_t* xbest = nullptr;
    int64_t* Ebest = nullptr;
    bool best_valid = false;
    std::vector<LaunchClass> opt_classes;
    // parallel tempering: groups of pt_T consecutive chains, ladder [C]
    int32_t pt_T = 0;
    int32_t* pt_ladder = nullptr;
    int32_t* pt_accepted = nullptr;
    // graph cache
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int64_t graph_steps = -1;
    // kernel timing per launch class (pns_profile): a start and a stop event
    // per class bracket its launches of one pns_run on the class's stream
    bool prof_on = false;
    bool prof_active = false;               // inside pns_run: its launches are timed
    bool prof_pending = false;
    std::vector<hipEvent_t> prof_ev;       // [2 * classes]
    std::vector<double> prof_ms;           // [classes] summed kernel time
    std::vector<int64_t> prof_launches;    // [classes]
    std::vector<int64_t> prof_runs_now;    // [classes] launches queued in the pending run
    std::vector<int64_t> prof_base;        // counters [C][6] when profiling started

    bool instrumented() const { return log_cap > 0 || hist_w != nullptr || snap_every > 0; }

    // pitch of every problem, indexed by problem (for the field kernels)
    std::vector<int64_t> pitches() const
    {
        std::vector<int64_t> v(probs.size());
        for (size_t p = 0; p < probs.size(); ++p) v[p] = probs[p].pitch;
        return v;
    }

    StepArgs args(int64_t steps) const
    {
        StepArgs a{};
        a.problems = problems;
        a.chain_problem = chain_problem;
        a.foff = foff;
        a.chain_list = nullptr;
        a.chain_first = 0;
        a.mode = mode;
        a.steps = steps;
        a.seed = seed;
        a.beta = beta;
        a.chain_id = chain_id;
        a.x = x;
        a.h = h;
        a.rmem = rmem;
        a.E = E;
        a.L = L;
        a.sub = sub;
        a.step = step;
        a.last_action = last_action;
        a.last_M = last_M;
        a.last_E = last_E;
        a.counters = counters;
        a.log_action = log_action;
        a.log_M = log_M;
        a.log_E = log_E;
        a.log_p = log_p;
        a.log_w = log_w;
        a.log_cap = log_cap;
        a.hist_w = hist_w;
        a.hist_v = hist_v;
        a.hist_rb = hist_rb;
        a.snap_every = snap_every;
        a.snap_cap = snap_cap;
        a.snap_x = snap_x;
        a.snap_M = snap_M;
        a.snap_E = snap_E;
        a.snap_w = snap_w;
        a.snap_count = snap_count;
        a.snap_pitch = max_pitch;
        a.inv_temp = 1.0;
        a.xbest = nullptr;
        a.Ebest = nullptr;
        a.orig_time = 0;
        return a;
    }

    // Index of k in `classes`, or -1 (optimization classes are not profiled).
    int class_index(const LaunchClass& k) const
    {
        if (classes.empty() || &k < &classes.front() || &k > &classes.back()) return -1;
        return (int)(&k - &classes.front());
    }

    hipError_t prof_record(int ki, int which, hipStream_t st) { return hipEventRecord(prof_ev[2 * ki + which], st); }

    // Add the kernel time of the pending run (waits for it).
    int prof_collect()
    {
        if (!prof_pending) return PNS_OK;
        for (size_t ki = 0; ki < classes.size(); ++ki) {
            if (prof_runs_now[ki] == 0) continue;
            HIP_TRY(hipEventSynchronize(prof_ev[2 * ki + 1]), "profile event wait");
            float ms = 0.0f;
            HIP_TRY(hipEventElapsedTime(&ms, prof_ev[2 * ki], prof_ev[2 * ki + 1]), "profile event time");
            prof_ms[ki] += ms;
            prof_launches[ki] += prof_runs_now[ki];
            prof_runs_now[ki] = 0;
        }
        prof_pending = false;
        return PNS_OK;
    }

    int launch_class(const LaunchClass& k, int64_t steps, hipStream_t st, int64_t orig_time = 0, bool first = true,
                     bool last = true)
    {
        // host-side check that the launch matches what the kernels assume
        for (int32_t c : {k.chains.front(), k.chains.back()}) {
            const ProblemRun& P = probs[h_chain_problem[c]];
            if ((int64_t)k.tile.block * 4 * k.tile.groups < P.N)
                return fail(PNS_EINVAL, "tile %dx%d does not cover N=%d", k.tile.block, k.tile.groups, P.N);
        }
        StepArgs a = args(steps);
        a.orig_time = orig_time;
        if (classes.size() > 1 || (int32_t)k.chains.size() != num_chains) a.chain_list = k.d_list;
        const int ki = prof_on && prof_active ? class_index(k) : -1;
        if (ki >= 0 && first) HIP_TRY(prof_record(ki, 0, st), "profile start event");
        hipError_t e = launch_steps(qtype, htype, k.flav, instrumented(), k.tile.block, k.tile.groups,
                                    (int32_t)k.chains.size(), k.dyn, st, a);
        if (e != hipSuccess) return hip_fail(e, "step kernel launch");
        if (ki >= 0) {
            ++prof_runs_now[ki];
            if (last) HIP_TRY(prof_record(ki, 1, st), "profile stop event");
        }
        return PNS_OK;
    }

    // One chunk of `steps` steps for every chain: one launch per class; with
    // several classes they run on their own streams between a fork and a join.
    int launch_chunk(int64_t steps, int64_t orig_time = 0, bool first = true, bool last = true)
    {
        if (classes.size() == 1) return launch_class(classes[0], steps, stream, orig_time, first, last);
        HIP_TRY(hipEventRecord(fork, stream), "fork record");
        // The side streams are ordered largest workgroups first; in launches
        // long enough for the order to matter (4096 steps and more, tens of
        // milliseconds) the streams of one-wave classes start 200 us later,
        // so that the workgroups of several waves find whole compute units
        // before the one-wave workgroups fill them (all queues released at
        // once would race).
        const bool stagger = steps >= 4096;
        bool held = false;
        for (auto& sd : sides) {
            const bool small = classes[sd.classes.front()].tile.block <= 64;
            if (stagger && small && !held && &sd != &sides.front()) {
                HIP_TRY(launch_hold(hold_ticks, stream), "hold");
                HIP_TRY(hipEventRecord(fork_small, stream), "fork record");
                held = true;
            }
            HIP_TRY(hipStreamWaitEvent(sd.stream, held ? fork_small : fork, 0), "fork wait");
            for (int32_t ki : sd.classes) {
                int rc = launch_class(classes[ki], steps, sd.stream, orig_time, first, last);
                if (rc) return rc;
            }
            HIP_TRY(hipEventRecord(sd.done, sd.stream), "join record");
        }
        // (the joins after every launch: the hold above sits on this stream)
        for (auto& sd : sides) HIP_TRY(hipStreamWaitEvent(stream, sd.done, 0), "join wait");
        return PNS_OK;
    }

    void free_all()
    {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (hipEvent_t ev : prof_ev)
            if (ev) (void)hipEventDestroy(ev);
        void* ptrs[] = {problems, chain_problem, foff, beta, chain_id, x, h, rmem, E, L, sub, step, last_action, last_M,
                        last_E, counters, log_action, log_M, log_E, log_p, log_w, hist_w, hist_v, hist_rb,
                        snap_x, snap_M, snap_E, snap_w, snap_count};
        for (void* p : ptrs)
            if (p) (void)hipFree(p);
        for (auto& P : probs) {
            void* ps[] = {P.A, P.diag, P.A2, P.diag2};
            for (void* q : ps)
                if (q) (void)hipFree(q);
        }
        for (auto& k : classes)
            if (k.d_list) (void)hipFree(k.d_list);
        for (auto& k : opt_classes)
            if (k.d_list) (void)hipFree(k.d_list);
        if (xbest) (void)hipFree(xbest);
        if (pt_ladder) (void)hipFree(pt_ladder);
        if (pt_accepted) (void)hipFree(pt_accepted);
        if (Ebest) (void)hipFree(Ebest);
        for (auto& sd : sides) {
            if (sd.stream) (void)hipStreamDestroy(sd.stream);
            if (sd.done) (void)hipEventDestroy(sd.done);
        }
        if (fork) (void)hipEventDestroy(fork);
        if (fork_small) (void)hipEventDestroy(fork_small);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

namespace {

std::vector<double> energies_to_double(const pns_ctx* ctx, const std::vector<int64_t>& bits)
{
    std::vector<double> out(bits.size());
    for (size_t i = 0; i < bits.size(); ++i) {
        if (ctx->qtype == Q_F32) {
            double d;
            std::memcpy(&d, &bits[i], 8);
            out[i] = d;
        } else {
            out[i] = (double)bits[i];
        }
    }
    return out;
}

// Per-chain padded rows -> concatenated rows of each chain's own N.
template <typename T>
std::vector<T> compact_rows(const pns_ctx* ctx, const std::vector<T>& padded, int64_t row_pitch, int64_t rows_per_chain)
{
    std::vector<T> out((size_t)ctx->h_offsets.back() * rows_per_chain);
    for (int32_t c = 0; c < ctx->num_chains; ++c) {
        const int32_t N = ctx->probs[ctx->h_chain_problem[c]].N;
        for (int64_t r = 0; r < rows_per_chain; ++r)
            std::memcpy(&out[(size_t)(ctx->h_offsets[c] * rows_per_chain + r * N)],
                        &padded[(size_t)((int64_t)c * rows_per_chain + r) * row_pitch], N * sizeof(T));
    }
    return out;
}

// Everything a context needs, for one or several problems.
// `preps`, if not empty, holds each problem's prepared matrix (as
// prepare_problem makes it); otherwise the matrices are prepared here.
int create_impl(pns_ctx** out, std::vector<ProblemSpec>& specs, int32_t mode, const pns_opts& o,
                const std::vector<const Prepared*>& preps = {})
{
    *out = nullptr;
    if (mode < PNS_MODE_RF || mode > PNS_MODE_UNBIASED_RAND) return fail(PNS_EINVAL, "unknown mode %d", mode);
    if (specs.empty()) return fail(PNS_EINVAL, "no problems");
    const int32_t qtype = o.dtype;
    const bool batch = specs.size() > 1;
    int64_t total_chains = 0;
    for (size_t p = 0; p < specs.size(); ++p) {
        ProblemSpec& S = specs[p];
        if (!S.Q) return fail(PNS_EINVAL, "Q of problem %zu is NULL", p);
        if (S.N <= 0) return fail(PNS_EINVAL, "N must be positive");
        if (S.layout != PNS_SYMMETRIC && S.layout != PNS_UPPER) return fail(PNS_EINVAL, "unknown layout %d", S.layout);
        if (mode == PNS_MODE_RF) S.n = S.N;
        if (S.n < 1 || S.n > S.N) return fail(PNS_EINVAL, "subset size %d outside [1, %d]", S.n, S.N);
        if (S.chains < 1) return fail(PNS_EINVAL, "num_chains must be >= 1");
        if (S.L0 < 0) return fail(PNS_EINVAL, "L0 must be >= 0");
        if ((int32_t)S.betas.size() != S.chains) return fail(PNS_EINVAL, "betas size mismatch");
        for (double b : S.betas)
            if (!(b >= 0.0) || !std::isfinite(b)) return fail(PNS_EINVAL, "beta must be finite and >= 0");
        if (S.N > kMaxN) return fail(PNS_EUNSUPPORTED, "N=%d exceeds the largest tile (%d)", S.N, kMaxN);
        if (S.tile.block != 0 && (int64_t)S.tile.block * 4 * S.tile.groups < S.N)
            return fail(PNS_EINVAL, "tile %dx%d cannot hold N=%d", S.tile.block, S.tile.groups, S.N);
        total_chains += S.chains;
    }
    if (total_chains > (1 << 30)) return fail(PNS_EINVAL, "too many chains");
    if (o.hist && (batch || specs[0].N > 24)) return fail(PNS_EINVAL, "histograms need one problem with N <= 24");

    // matrices: host preparation, field-type choice
    std::vector<Prepared> own(preps.empty() ? specs.size() : 0);
    std::vector<const Prepared*> pp(preps);
    if (pp.empty()) {
        for (size_t p = 0; p < specs.size(); ++p) {
            int rc = prepare_problem(specs[p].Q, specs[p].N, specs[p].layout, qtype, &own[p]);
            if (rc) return rc;
            pp.push_back(&own[p]);
        }
    }
    if (pp.size() != specs.size()) return fail(PNS_EINVAL, "prepared matrices do not match the problems");
    double ebound_max = 0.0, fbound_max = 0.0;
    for (size_t p = 0; p < specs.size(); ++p) {
        const ProblemSpec& S = specs[p];
        const int32_t s = S.layout == PNS_SYMMETRIC ? 2 : 1;
        const double eb = pp[p]->diag_bound + s * pp[p]->field_bound;
        if (qtype != Q_F32 && eb * (double)S.N > 9.0e18) return fail(PNS_EINVAL, "energy bound of Q overflows int64");
        ebound_max = std::max(ebound_max, eb);
        fbound_max = std::max(fbound_max, pp[p]->field_bound);
    }
    int32_t htype;
    if (qtype == Q_F32) htype = H_F64;
    else if (qtype == Q_I16) htype = H_I32;
    else htype = (fbound_max < 2147483647.0 && ebound_max < 2147483647.0) ? H_I32 : H_I64;
    for (auto& S : specs)
        if (S.tile.block == 0) S.tile = default_tile_for(mode, S.N, S.n, qtype, htype);
    for (const auto& S : specs) {
        const int32_t fl = flavour_for(mode, S.N, S.n, S.tile, qtype, htype);
        if (fl < 0) return fail(PNS_EINVAL, "no kernel for tile %dx%d", S.tile.block, S.tile.groups);
        if (fl == 5 && o.hist) return fail(PNS_EINVAL, "histograms need a step-kernel tile (N <= 24)");
    }

    pns_ctx* ctx = new pns_ctx();
    auto fail_free = [&](int r) {
        ctx->free_all();
        delete ctx;
        return r;
    };
    ctx->mode = mode;
    ctx->qtype = qtype;
    ctx->htype = htype;
    ctx->num_chains = (int32_t)total_chains;
    ctx->launch = o.launch;
    ctx->chunk = o.chunk;
    ctx->seed = o.seed;
    if (o.stream) {
        ctx->stream = reinterpret_cast<hipStream_t>(o.stream);
    } else {
        hipError_t e = hipStreamCreate(&ctx->stream);
        if (e != hipSuccess) return fail_free(hip_fail(e, "hipStreamCreate"));
        ctx->own_stream = true;
    }

    // problems, chain tables, launch classes
    const int64_t C = total_chains;
    ctx->h_chain_problem.resize(C);
    ctx->h_foff.resize(C);
    ctx->h_offsets.assign(C + 1, 0);
    std::vector<double> betas((size_t)C);
    std::vector<Problem> dev_probs(specs.size());
    int32_t c0 = 0;
    int64_t f0 = 0;
    std::map<std::pair<std::pair<int32_t, int32_t>, int32_t>, size_t> class_of;
    // Kernel flavour of each problem.  The two-group window kernel also runs
    // compact windows (a window in one group of a wave is a two-group window
    // with both groups equal), so on a tile where both occur the compact
    // problems join the two-group class: fewer launch classes to run
    // concurrently.
    std::vector<int32_t> flav(specs.size());
    std::map<std::pair<int32_t, int32_t>, int32_t> tile_has4;
    for (size_t p = 0; p < specs.size(); ++p) {
        const ProblemSpec& S = specs[p];
        flav[p] = flavour_for(mode, S.N, S.n, S.tile, qtype, htype);
        if (flav[p] == 4) tile_has4[{S.tile.block, S.tile.groups}] = 1;
    }
    for (size_t p = 0; p < specs.size(); ++p)
        if (flav[p] == 3 && specs[p].tile.groups >= 2 && tile_has4.count({specs[p].tile.block, specs[p].tile.groups}))
            flav[p] = 4;
    for (size_t p = 0; p < specs.size(); ++p) {
        const ProblemSpec& S = specs[p];
        ProblemRun R{};
        R.N = S.N;
        R.n = S.n;
        R.layout = S.layout;
        R.s = S.layout == PNS_SYMMETRIC ? 2 : 1;
        R.pitch = round_up(S.N, 64);
        R.L0 = S.L0;
        R.num_sets = S.N / gcd64(S.N, S.n);
        R.chain_begin = c0;
        R.chains = S.chains;
        R.tile = S.tile;
        R.flav = flav[p];
        ctx->probs.push_back(R);
        ProblemRun& RR = ctx->probs.back();
        int r = dev_alloc(reinterpret_cast<uint8_t**>(&RR.A), pp[p]->A.size() + kRowTailBytes);
        if (!r) r = dev_alloc(reinterpret_cast<uint8_t**>(&RR.diag), pp[p]->D.size());
        if (r) return fail_free(r);
        hipError_t e = hipMemcpy(RR.A, pp[p]->A.data(), pp[p]->A.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(static_cast<uint8_t*>(RR.A) + pp[p]->A.size(), 0, kRowTailBytes);
        if (e == hipSuccess) e = hipMemcpy(RR.diag, pp[p]->D.data(), pp[p]->D.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail_free(hip_fail(e, "upload"));
        if (p < own.size()) {
            own[p].A.clear();
            own[p].A.shrink_to_fit();
        }
        Problem& D = dev_probs[p];
        D.A = RR.A;
        D.diag = RR.diag;
        D.pitch = RR.pitch;
        D.num_sets = RR.num_sets;
        D.L0 = RR.L0;
        D.N = RR.N;
        D.n = RR.n;
        D.s = RR.s;
        D.qtype = qtype;
        ctx->max_pitch = std::max(ctx->max_pitch, RR.pitch);
        const auto key = std::make_pair(std::make_pair(RR.tile.block, RR.tile.groups), RR.flav);
        if (!class_of.count(key)) {
            class_of[key] = ctx->classes.size();
            LaunchClass k;
            k.tile = RR.tile;
            k.flav = RR.flav;
            k.dyn = 0;
            ctx->classes.push_back(k);
        }
        LaunchClass& K = ctx->classes[class_of[key]];
        // dynamic LDS: the diagonal, after the random-subset table for drawn
        // subsets (the window kernel keeps neither)
        K.dyn = std::max(K.dyn, RR.flav == 5 ? (size_t)0 : (size_t)RR.pitch * 4 * (RR.flav == 2 ? 2 : 1));
        for (int32_t c = 0; c < S.chains; ++c) {
            ctx->h_chain_problem[c0 + c] = (int32_t)p;
            ctx->h_foff[c0 + c] = f0 + (int64_t)c * RR.pitch;
            ctx->h_offsets[c0 + c + 1] = ctx->h_offsets[c0 + c] + S.N;
            betas[c0 + c] = S.betas[c];
            K.chains.push_back(c0 + c);
        }
        // a step costs about the lane work of the tile: block * groups
        K.cost += (double)S.chains * RR.tile.block * RR.tile.groups;
        f0 += (int64_t)S.chains * RR.pitch;
        c0 += S.chains;
    }
    ctx->fields = f0;
    // longest problems first within a class: the last workgroups to start are short ones
    for (auto& k : ctx->classes)
        std::stable_sort(k.chains.begin(), k.chains.end(), [&](int32_t a, int32_t b) {
            return ctx->probs[ctx->h_chain_problem[a]].N > ctx->probs[ctx->h_chain_problem[b]].N;
        });

    const size_t hbytes = htype == H_I32 ? 4 : 8;
    const size_t fields = (size_t)ctx->fields;
    const bool any_drawn = mode == PNS_MODE_UNBIASED_RAND;
#define ALLOC(ptr, type, count)                                    \
    do {                                                           \
        int r_ = dev_alloc(reinterpret_cast<type**>(&ptr), count); \
        if (r_) return fail_free(r_);                              \
    } while (0)
    ALLOC(ctx->problems, Problem, specs.size());
    ALLOC(ctx->chain_problem, int32_t, C);
    ALLOC(ctx->foff, int64_t, C);
    ALLOC(ctx->beta, double, C);
    ALLOC(ctx->chain_id, uint32_t, C);
    ALLOC(ctx->x, uint8_t, fields);
    ALLOC(ctx->h, uint8_t, fields * hbytes);
    ALLOC(ctx->E, int64_t, C);
    ALLOC(ctx->L, int64_t, C);
    ALLOC(ctx->sub, int64_t, C);
    ALLOC(ctx->step, int64_t, C);
    ALLOC(ctx->last_action, int32_t, C);
    ALLOC(ctx->last_M, int64_t, C);
    ALLOC(ctx->last_E, int64_t, C);
    ALLOC(ctx->counters, int64_t, C * 6);
    if (any_drawn) ALLOC(ctx->rmem, uint8_t, fields);
    if (o.log_capacity > 0) {
        ctx->log_cap = o.log_capacity;
        ALLOC(ctx->log_action, int32_t, (size_t)C * o.log_capacity);
        ALLOC(ctx->log_M, int64_t, (size_t)C * o.log_capacity);
        ALLOC(ctx->log_E, int64_t, (size_t)C * o.log_capacity);
        ALLOC(ctx->log_p, double, (size_t)C * o.log_capacity);
        ALLOC(ctx->log_w, double, (size_t)C * o.log_capacity);
    }
    if (o.hist) {
        ALLOC(ctx->hist_w, unsigned long long, (size_t)1 << specs[0].N);
        ALLOC(ctx->hist_v, unsigned long long, (size_t)1 << specs[0].N);
        ALLOC(ctx->hist_rb, double, (size_t)1 << specs[0].N);
    }
    if (o.snapshot_every > 0) {
        ctx->snap_every = o.snapshot_every;
        ctx->snap_cap = o.snapshot_capacity;
        ALLOC(ctx->snap_x, uint8_t, (size_t)C * o.snapshot_capacity * ctx->max_pitch);
        ALLOC(ctx->snap_M, int64_t, (size_t)C * o.snapshot_capacity);
        ALLOC(ctx->snap_E, int64_t, (size_t)C * o.snapshot_capacity);
        ALLOC(ctx->snap_w, double, (size_t)C * o.snapshot_capacity);
        ALLOC(ctx->snap_count, int32_t, (C + 1) / 2 * 2);  // whole 64-bit words (cleared as such)
    }
    for (auto& k : ctx->classes) ALLOC(k.d_list, int32_t, k.chains.size());
#undef ALLOC

    std::vector<uint32_t> cidv((size_t)C);
    for (int64_t c = 0; c < C; ++c) cidv[c] = o.chain_id_base + (uint32_t)c;
    std::vector<int64_t> Lv((size_t)C), zeros64((size_t)C * 6, 0);
    for (int64_t c = 0; c < C; ++c) Lv[c] = ctx->probs[ctx->h_chain_problem[c]].L0;
    std::vector<int32_t> la((size_t)C, PNS_STAY);
#define H2D(dst, src, bytes)                                               \
    do {                                                                   \
        hipError_t e_ = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice); \
        if (e_ != hipSuccess) return fail_free(hip_fail(e_, "upload"));    \
    } while (0)
    H2D(ctx->problems, dev_probs.data(), dev_probs.size() * sizeof(Problem));
    H2D(ctx->chain_problem, ctx->h_chain_problem.data(), C * sizeof(int32_t));
    H2D(ctx->foff, ctx->h_foff.data(), C * sizeof(int64_t));
    H2D(ctx->beta, betas.data(), C * sizeof(double));
    H2D(ctx->chain_id, cidv.data(), C * sizeof(uint32_t));
    H2D(ctx->L, Lv.data(), C * sizeof(int64_t));
    H2D(ctx->sub, zeros64.data(), C * sizeof(int64_t));
    H2D(ctx->step, zeros64.data(), C * sizeof(int64_t));
    H2D(ctx->last_action, la.data(), C * sizeof(int32_t));
    H2D(ctx->last_M, zeros64.data(), C * sizeof(int64_t));
    H2D(ctx->counters, zeros64.data(), C * 6 * sizeof(int64_t));
    if (ctx->snap_count) H2D(ctx->snap_count, zeros64.data(), C * sizeof(int32_t));
    for (auto& k : ctx->classes) H2D(k.d_list, k.chains.data(), k.chains.size() * sizeof(int32_t));
    hipError_t e;
    if (ctx->hist_w) {
        e = hipMemset(ctx->hist_w, 0, sizeof(unsigned long long) << specs[0].N);
        if (e == hipSuccess) e = hipMemset(ctx->hist_v, 0, sizeof(unsigned long long) << specs[0].N);
        if (e == hipSuccess) e = hipMemset(ctx->hist_rb, 0, sizeof(double) << specs[0].N);
        if (e != hipSuccess) return fail_free(hip_fail(e, "hipMemset"));
    }
    if (ctx->rmem && (e = hipMemset(ctx->rmem, 0, fields)) != hipSuccess) return fail_free(hip_fail(e, "hipMemset"));
    if (ctx->snap_x) {
        // slots not yet written read as x = 0 with weight 0
        e = hipMemset(ctx->snap_x, 0, (size_t)C * ctx->snap_cap * ctx->max_pitch);
        if (e == hipSuccess) e = hipMemset(ctx->snap_M, 0, (size_t)C * ctx->snap_cap * 8);
        if (e == hipSuccess) e = hipMemset(ctx->snap_E, 0, (size_t)C * ctx->snap_cap * 8);
        if (e == hipSuccess) e = hipMemset(ctx->snap_w, 0, (size_t)C * ctx->snap_cap * 8);
        if (e != hipSuccess) return fail_free(hip_fail(e, "hipMemset"));
    }
    if (ctx->classes.size() > 1) {
        if ((e = hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&ctx->fork_small, hipEventDisableTiming)) != hipSuccess)
            return fail_free(hip_fail(e, "hipEventCreate"));
        {
            int dev = 0, khz = 0;
            if (hipGetDevice(&dev) == hipSuccess &&
                hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
                ctx->hold_ticks = (uint64_t)khz / 5;  // kHz x 0.2 ms
        }
        // longest-processing-time-first packing of the classes onto the side streams
        std::vector<int32_t> order(ctx->classes.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = (int32_t)i;
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t a, int32_t b) { return ctx->classes[a].cost > ctx->classes[b].cost; });
        ctx->sides.resize(std::min<size_t>((size_t)max_side_streams(), ctx->classes.size()));
        std::vector<double> load(ctx->sides.size(), 0.0);
        for (int32_t ki : order) {
            const size_t sdi = (size_t)(std::min_element(load.begin(), load.end()) - load.begin());
            ctx->sides[sdi].classes.push_back(ki);
            load[sdi] += ctx->classes[ki].cost;
        }
        // Launch order of the side streams: the largest workgroups first
        // (waves per workgroup, then fields per lane).  Every workgroup keeps
        // its chain for the whole launch, and a workgroup of several waves
        // needs room on one compute unit at once; started after smaller ones
        // it finds the compute units fragmented and waits for them.
        auto footprint = [&](const SideStream& sd) {
            const Tile t = ctx->classes[sd.classes.front()].tile;
            return std::make_pair(t.block, t.groups);
        };
        std::stable_sort(ctx->sides.begin(), ctx->sides.end(),
                         [&](const SideStream& a, const SideStream& b) { return footprint(a) > footprint(b); });
        for (auto& sd : ctx->sides) {
            if ((e = hipStreamCreateWithFlags(&sd.stream, hipStreamNonBlocking)) != hipSuccess)
                return fail_free(hip_fail(e, "hipStreamCreate"));
            if ((e = hipEventCreateWithFlags(&sd.done, hipEventDisableTiming)) != hipSuccess)
                return fail_free(hip_fail(e, "hipEventCreate"));
        }
    }

    // initial state
    if (o.init == PNS_INIT_GIVEN) {
        std::vector<uint8_t> x0((size_t)ctx->h_offsets.back()), xp(fields, 0);
        int rc = copy_in(x0.data(), o.x0, x0.size());
        if (rc) return fail_free(rc);
        for (int64_t c = 0; c < C; ++c) {
            const int32_t N = ctx->probs[ctx->h_chain_problem[c]].N;
            for (int32_t j = 0; j < N; ++j) xp[ctx->h_foff[c] + j] = x0[ctx->h_offsets[c] + j] ? 1 : 0;
        }
        H2D(ctx->x, xp.data(), fields);
    }
#undef H2D
    if (o.init == PNS_INIT_ZERO) {
        if ((e = hipMemset(ctx->x, 0, fields)) != hipSuccess) return fail_free(hip_fail(e, "hipMemset"));
        if ((e = hipMemset(ctx->h, 0, fields * hbytes)) != hipSuccess) return fail_free(hip_fail(e, "hipMemset"));
        if ((e = hipMemset(ctx->E, 0, C * 8)) != hipSuccess) return fail_free(hip_fail(e, "hipMemset"));
        if ((e = hipMemset(ctx->last_E, 0, C * 8)) != hipSuccess) return fail_free(hip_fail(e, "hipMemset"));
    } else {
        InitArgs ia{};
        ia.problems = ctx->problems;
        ia.chain_problem = ctx->chain_problem;
        ia.foff = ctx->foff;
        ia.num_chains = (int32_t)C;
        ia.init = o.init == PNS_INIT_RANDOM ? 1 : 2;
        ia.seed = o.seed;
        ia.chain_id = ctx->chain_id;
        ia.x = ctx->x;
        ia.h = ctx->h;
        ia.E = ctx->E;
        ia.last_E = ctx->last_E;
        e = launch_init_with_map(qtype, htype, (int32_t)ctx->max_pitch, ctx->stream, ia, ctx->h_chain_problem.data(),
                                 ctx->pitches().data());
        if (e != hipSuccess) return fail_free(hip_fail(e, "init kernels"));
    }
    if ((e = hipDeviceSynchronize()) != hipSuccess) return fail_free(hip_fail(e, "create synchronize"));
    *out = ctx;
    return PNS_OK;
}

// ---- autotuner ----

constexpr int32_t kTrialSteps = 256;  // timed steps per trial on creation

std::mutex g_tune_mu;
std::map<std::string, pns_tune> g_tune_cache;

// Chains back to x = 0 at step 0 (the state of a fresh INIT_ZERO context).
int reset_zero_state(pns_ctx* ctx)
{
    const int64_t C = ctx->num_chains;
    const size_t hb = ctx->htype == H_I32 ? 4 : 8;
    std::vector<int64_t> Lv((size_t)C);
    for (int64_t c = 0; c < C; ++c) Lv[c] = ctx->probs[ctx->h_chain_problem[c]].L0;
    std::vector<int32_t> la((size_t)C, PNS_STAY);
    HIP_TRY(hipMemset(ctx->x, 0, (size_t)ctx->fields), "reset");
    HIP_TRY(hipMemset(ctx->h, 0, (size_t)ctx->fields * hb), "reset");
    if (ctx->rmem) HIP_TRY(hipMemset(ctx->rmem, 0, (size_t)ctx->fields), "reset");
    int64_t* zero_arrs[] = {ctx->E, ctx->last_E, ctx->last_M, ctx->sub, ctx->step};
    for (int64_t* p : zero_arrs) HIP_TRY(hipMemset(p, 0, C * 8), "reset");
    HIP_TRY(hipMemset(ctx->counters, 0, C * 6 * 8), "reset");
    HIP_TRY(hipMemcpy(ctx->L, Lv.data(), C * 8, hipMemcpyHostToDevice), "reset");
    HIP_TRY(hipMemcpy(ctx->last_action, la.data(), C * 4, hipMemcpyHostToDevice), "reset");
    return PNS_OK;
}

// Give the single problem of `ctx` another tile and subset size, and reset
// its chains, as if the context had been created with them.
int reconfigure(pns_ctx* ctx, Tile t, int32_t n)
{
    ProblemRun& R = ctx->probs[0];
    R.tile = t;
    R.n = n;
    R.num_sets = R.N / gcd64(R.N, n);
    R.flav = flavour_for(ctx->mode, R.N, n, t, ctx->qtype, ctx->htype);
    Problem D{};
    D.A = R.A;
    D.diag = R.diag;
    D.pitch = R.pitch;
    D.num_sets = R.num_sets;
    D.L0 = R.L0;
    D.N = R.N;
    D.n = R.n;
    D.s = R.s;
    D.qtype = ctx->qtype;
    HIP_TRY(hipMemcpy(ctx->problems, &D, sizeof(Problem), hipMemcpyHostToDevice), "reconfigure");
    LaunchClass& K = ctx->classes[0];
    K.tile = t;
    K.flav = R.flav;
    K.dyn = R.flav == 5 ? 0 : (size_t)R.pitch * 4 * (R.flav == 2 ? 2 : 1);
    return reset_zero_state(ctx);
}

// Records per second (and flips per second) of the context's current
// configuration, from the faster of two timed runs on the device after a
// warmup (one run alone moves the choices of the autotuner by run-to-run
// noise).
int time_config(pns_ctx* ctx, int32_t steps, double* rate, double* frate)
{
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    const int warm = std::max(8, steps / 4);
    int rc = PNS_OK;
    if (e == hipSuccess) rc = ctx->launch_chunk(warm);
    float ms = 0.0f;
    for (int rep = 0; rep < 2 && e == hipSuccess && !rc; ++rep) {
        e = hipEventRecord(a, ctx->stream);
        if (e == hipSuccess) rc = ctx->launch_chunk(steps);
        if (e == hipSuccess && !rc) e = hipEventRecord(b, ctx->stream);
        if (e == hipSuccess && !rc) e = hipEventSynchronize(b);
        float m = 0.0f;
        if (e == hipSuccess && !rc) e = hipEventElapsedTime(&m, a, b);
        if (e == hipSuccess && !rc) ms = rep == 0 ? m : std::min(ms, m);
    }
    std::vector<int64_t> cnt;
    if (e == hipSuccess && !rc) rc = d2h(cnt, ctx->counters, (size_t)ctx->num_chains * 6);
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (rc) return rc;
    if (e != hipSuccess) return hip_fail(e, "autotune timing");
    int64_t flips = 0;
    for (int64_t c = 0; c < ctx->num_chains; ++c) flips += cnt[c * 6 + 1];
    const double sec = std::max(1e-9, (double)ms * 1e-3);
    *rate = (double)ctx->num_chains * steps / sec;
    *frate = (double)flips * steps / (double)(2 * steps + warm) / sec;
    return PNS_OK;
}

int autotune_impl(const ProblemSpec& base, int32_t mode, const pns_opts& o, int32_t trial_steps, pns_tune* out,
                  const Prepared* prep = nullptr)
{
    if (trial_steps <= 0) trial_steps = 64;
    char key[256];
    snprintf(key, sizeof(key), "N%d_q%d_l%d_m%d_n%d_c%d_s%d", base.N, o.dtype, base.layout, mode, base.n, base.chains,
             trial_steps);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            *out = it->second;
            return PNS_OK;
        }
    }
    // Trials run at least 3072 chains (the problem's betas repeated) so that
    // the device is loaded as in a real run -- a few chains alone on an idle
    // device measure step latency, not throughput -- and so that tiles of
    // one to four chains per compute unit all run several full rounds.
    ProblemSpec spec = base;
    spec.chains = std::min<int32_t>(4096, std::max<int32_t>(base.chains, 3072));
    spec.betas.assign(spec.chains, 1.0);
    for (int32_t c = 0; c < spec.chains; ++c)
        spec.betas[c] = base.betas.empty() ? 1.0 : base.betas[c % base.betas.size()];
    const bool tune_n = mode != PNS_MODE_RF && base.n == 0;
    // subset sizes tried: powers of two 16 .. N/2 (or the one given; RF: N)
    std::vector<int32_t> ns;
    if (mode == PNS_MODE_RF) ns.push_back(base.N);
    else if (!tune_n) ns.push_back(base.n);
    else
        for (int32_t n = 16; n <= base.N / 2; n *= 2) ns.push_back(n);
    if (ns.empty()) ns.push_back(std::max(1, base.N / 2));
    spec.n = ns.front();
    spec.tile = default_tile(base.N);
    if ((int64_t)spec.tile.block * 4 * spec.tile.groups < base.N)
        return fail(PNS_EUNSUPPORTED, "no tile holds N=%d", base.N);
    pns_opts t = o;
    t.log_capacity = 0;
    t.hist = 0;
    t.snapshot_every = 0;
    t.launch = PNS_LAUNCH_PERSISTENT;
    t.chunk = 0;
    t.stream = nullptr;
    t.init = PNS_INIT_ZERO;
    t.x0 = nullptr;
    std::vector<ProblemSpec> one{spec};
    pns_ctx* ctx = nullptr;
    std::vector<const Prepared*> preps;
    if (prep) preps.push_back(prep);
    int rc = create_impl(&ctx, one, mode, t, preps);
    if (rc) return rc;
    // Every (tile, subset size): tiles that hold N in at most twice its
    // rounded size, wide tiles only where the subset runs a window kernel.
    struct Trial {
        Tile tile;
        int32_t n;
        double rate, frate;
    };
    std::vector<Trial> res;
    int trials = 0;
    // Where a window kernel tile holds the problem, only the smallest such
    // tile is tried (over the subset sizes): the window kernel ran faster than
    // the step kernel's tiles at every size measured, and its cost per step
    // past the weighing (the move's row and field update) and its registers
    // and LDS per chain grow with the tile, which in a batch limits how many
    // chains are resident; a batch also forms one launch class per tile.
    auto holds = [&](const Tile& tl) {
        const int64_t cap = (int64_t)tl.block * 4 * tl.groups;
        return cap >= base.N && cap <= 2 * round_up(base.N, 256);
    };
    int64_t window_cap = 0;
    for (const Tile& tl : kTiles)
        for (int32_t n : ns)
            if (holds(tl) && flavour_for(mode, base.N, n, tl, ctx->qtype, ctx->htype) == 5) {
                const int64_t cap = (int64_t)tl.block * 4 * tl.groups;
                if (window_cap == 0 || cap < window_cap) window_cap = cap;
            }
    for (const Tile& tl : kTiles) {
        if (!holds(tl)) continue;
        if (window_cap && (int64_t)tl.block * 4 * tl.groups != window_cap) continue;
        for (int32_t n : ns) {
            const int32_t fl = flavour_for(mode, base.N, n, tl, ctx->qtype, ctx->htype);
            if (fl < 0 || (wide_tile(tl) && fl != 3 && fl != 4 && fl != 5)) continue;
            if (window_cap && fl != 5) continue;
            double r = 0.0, fr = 0.0;
            rc = reconfigure(ctx, tl, n);
            if (!rc) rc = time_config(ctx, trial_steps, &r, &fr);
            if (rc) break;
            ++trials;
            res.push_back({tl, n, r, fr});
        }
        if (rc) break;
    }
    pns_tune best{};
    best.records_per_s = -1.0;
    if (!rc && !res.empty()) {
        // the largest subset (Sec 5: the largest partial neighbor set the
        // hardware affords) whose step rate is within 10% of the best trial,
        // on its fastest tile
        double top = 0.0;
        for (const Trial& r : res) top = std::max(top, r.rate);
        for (const Trial& r : res) {
            if (r.rate < 0.9 * top) continue;
            if (best.records_per_s < 0.0 || r.n > best.subset_size ||
                (r.n == best.subset_size && r.rate > best.records_per_s)) {
                best.block = r.tile.block;
                best.groups = r.tile.groups;
                best.subset_size = r.n;
                best.records_per_s = r.rate;
                best.flips_per_s = r.frate;
            }
        }
    }
    ctx->free_all();
    delete ctx;
    if (rc) return rc;
    if (best.records_per_s < 0.0) return fail(PNS_EUNSUPPORTED, "no tile holds N=%d", base.N);
    best.trials = trials;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune_cache[key] = best;
    }
    *out = best;
    return PNS_OK;
}

}  // namespace

extern "C" {

void pns_opts_default(pns_opts* o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->dtype = PNS_I32;
    o->layout = PNS_SYMMETRIC;
    o->num_chains = 1;
    o->L0 = 100;
    o->launch = PNS_LAUNCH_PERSISTENT;
}

const char* pns_last_error(void) { return g_error.c_str(); }

const char* pns_version(void) { return "0.2.0"; }

int pns_create(pns_ctx** out, const void* Q, int32_t N, double beta, int32_t subset_size, int32_t mode,
               const pns_opts* opts)
{
    g_error.clear();
    if (!out) return fail(PNS_EINVAL, "out is NULL");
    *out = nullptr;
    pns_opts o;
    if (opts) o = *opts;
    else pns_opts_default(&o);
    int rc = check_opts(&o);
    if (rc) return rc;
    if (!Q) return fail(PNS_EINVAL, "Q is NULL");
    if (N <= 0) return fail(PNS_EINVAL, "N must be positive");
    // (before the matrix is read: the autotuner prepares it first)
    if (N > kMaxN) return fail(PNS_EUNSUPPORTED, "N=%d exceeds the largest tile (%d)", N, kMaxN);
    if (mode < PNS_MODE_RF || mode > PNS_MODE_UNBIASED_RAND) return fail(PNS_EINVAL, "unknown mode %d", mode);
    if (o.hist && N > 24) return fail(PNS_EINVAL, "histograms need N <= 24");
    const bool tune_n = o.autotune && mode != PNS_MODE_RF && subset_size == 0;
    const int32_t n = mode == PNS_MODE_RF ? N : subset_size;
    if (!tune_n && (n < 1 || n > N)) return fail(PNS_EINVAL, "subset size %d outside [1, %d]", subset_size, N);
    ProblemSpec S;
    S.Q = Q;
    S.N = N;
    S.layout = o.layout;
    S.n = n;
    S.chains = o.num_chains;
    S.L0 = o.L0;
    S.betas.assign((size_t)o.num_chains, beta);
    if (o.betas)
        for (int32_t c = 0; c < o.num_chains; ++c) S.betas[c] = o.betas[c];
    for (double b : S.betas)
        if (!(b >= 0.0) || !std::isfinite(b)) return fail(PNS_EINVAL, "beta must be finite and >= 0");
    if (o.block > 0 || o.groups > 0) {
        const Tile def = default_tile(N);
        S.tile.block = o.block > 0 ? o.block : def.block;
        S.tile.groups = o.groups > 0 ? o.groups
                                     : std::max<int32_t>(1, (int32_t)((N + S.tile.block * 4 - 1) / (S.tile.block * 4)));
    } else if (o.autotune) {
        Prepared prep;
        rc = prepare_problem(Q, N, o.layout, o.dtype, &prep);
        if (rc) return rc;
        pns_tune t{};
        ProblemSpec T = S;
        T.n = tune_n ? 0 : n;
        rc = autotune_impl(T, mode, o, kTrialSteps, &t, &prep);
        if (rc) return rc;
        S.tile = {t.block, t.groups};
        if (tune_n) S.n = t.subset_size;
        std::vector<ProblemSpec> specs{S};
        return create_impl(out, specs, mode, o, {&prep});
    }
    std::vector<ProblemSpec> specs{S};
    return create_impl(out, specs, mode, o);
}

int pns_create_batch(pns_ctx** out, int32_t num_problems, const pns_problem* problems, int32_t mode,
                     const pns_opts* opts)
{
    g_error.clear();
    if (!out) return fail(PNS_EINVAL, "out is NULL");
    *out = nullptr;
    if (num_problems < 1 || !problems) return fail(PNS_EINVAL, "num_problems must be >= 1");
    pns_opts o;
    if (opts) o = *opts;
    else pns_opts_default(&o);
    int rc = check_opts(&o);
    if (rc) return rc;
    if (mode < PNS_MODE_RF || mode > PNS_MODE_UNBIASED_RAND) return fail(PNS_EINVAL, "unknown mode %d", mode);
    std::vector<ProblemSpec> specs((size_t)num_problems);
    std::vector<bool> tune((size_t)num_problems, false), tune_n((size_t)num_problems, false);
    for (int32_t p = 0; p < num_problems; ++p) {
        const pns_problem& q = problems[p];
        ProblemSpec& S = specs[p];
        if (!q.Q) return fail(PNS_EINVAL, "problem %d: Q is NULL", p);
        if (q.N <= 0) return fail(PNS_EINVAL, "problem %d: N must be positive", p);
        if (q.N > kMaxN)
            return fail(PNS_EUNSUPPORTED, "problem %d: N=%d exceeds the largest tile (%d)", p, q.N, kMaxN);
        if (q.layout != PNS_SYMMETRIC && q.layout != PNS_UPPER)
            return fail(PNS_EINVAL, "problem %d: unknown layout %d", p, q.layout);
        if (q.num_chains < 1) return fail(PNS_EINVAL, "problem %d: num_chains must be >= 1", p);
        if (q.L0 < 0) return fail(PNS_EINVAL, "problem %d: L0 must be >= 0", p);
        tune_n[p] = mode != PNS_MODE_RF && q.subset_size == 0;
        if (mode != PNS_MODE_RF && !tune_n[p] && (q.subset_size < 1 || q.subset_size > q.N))
            return fail(PNS_EINVAL, "problem %d: subset size %d outside [1, %d]", p, q.subset_size, q.N);
        S.Q = q.Q;
        S.N = q.N;
        S.layout = q.layout;
        S.n = mode == PNS_MODE_RF ? q.N : q.subset_size;
        S.chains = q.num_chains;
        S.L0 = q.L0 > 0 ? q.L0 : o.L0;
        S.betas.assign((size_t)S.chains, q.beta);
        if (q.betas)
            for (int32_t c = 0; c < S.chains; ++c) S.betas[c] = q.betas[c];
        for (double b : S.betas)
            if (!(b >= 0.0) || !std::isfinite(b)) return fail(PNS_EINVAL, "problem %d: beta must be finite and >= 0", p);
        tune[p] = o.autotune || tune_n[p];
        if (!tune[p] && o.block > 0 && (int64_t)o.block * 4 * std::max(1, o.groups) >= q.N)
            S.tile = {o.block, std::max(1, o.groups)};
    }
    // every matrix is prepared once, for the trials and the context
    std::vector<Prepared> preps((size_t)num_problems);
    std::vector<const Prepared*> pp;
    for (int32_t p = 0; p < num_problems; ++p) {
        rc = prepare_problem(specs[p].Q, specs[p].N, specs[p].layout, o.dtype, &preps[p]);
        if (rc) return rc;
        pp.push_back(&preps[p]);
    }
    for (int32_t p = 0; p < num_problems; ++p) {
        if (!tune[p]) continue;
        pns_opts t = o;
        t.layout = specs[p].layout;
        t.num_chains = specs[p].chains;
        pns_tune r{};
        ProblemSpec T = specs[p];
        T.n = tune_n[p] ? 0 : specs[p].n;
        rc = autotune_impl(T, mode, t, kTrialSteps, &r, &preps[p]);
        if (rc) return rc;
        specs[p].tile = {r.block, r.groups};
        if (tune_n[p]) specs[p].n = r.subset_size;
    }
    return create_impl(out, specs, mode, o, pp);
}

int pns_autotune(const void* Q, int32_t N, double beta, int32_t subset_size, int32_t mode, const pns_opts* opts,
                 int32_t trial_steps, pns_tune* out)
{
    g_error.clear();
    if (!out || !Q) return fail(PNS_EINVAL, "NULL argument");
    pns_opts o;
    if (opts) o = *opts;
    else pns_opts_default(&o);
    int rc = check_opts(&o);
    if (rc) return rc;
    if (N <= 0) return fail(PNS_EINVAL, "N must be positive");
    if (N > kMaxN) return fail(PNS_EUNSUPPORTED, "N=%d exceeds the largest tile (%d)", N, kMaxN);
    if (mode < PNS_MODE_RF || mode > PNS_MODE_UNBIASED_RAND) return fail(PNS_EINVAL, "unknown mode %d", mode);
    if (subset_size < 0 || subset_size > N) return fail(PNS_EINVAL, "subset size %d outside [0, %d]", subset_size, N);
    ProblemSpec S;
    S.Q = Q;
    S.N = N;
    S.layout = o.layout;
    S.n = mode == PNS_MODE_RF ? N : subset_size;
    S.chains = o.num_chains;
    S.L0 = o.L0;
    S.betas.assign((size_t)o.num_chains, beta);
    if (o.betas)
        for (int32_t c = 0; c < o.num_chains; ++c) S.betas[c] = o.betas[c];
    return autotune_impl(S, mode, o, trial_steps, out);
}

}  // extern "C"

namespace {

int run_impl(pns_ctx* ctx, int64_t steps);

}  // namespace

extern "C" {

int pns_run(pns_ctx* ctx, int64_t steps)
{
    g_error.clear();
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    if (steps < 0) return fail(PNS_EINVAL, "steps must be >= 0");
    if (steps == 0) return PNS_OK;
    if (ctx->prof_on) {
        int rc = ctx->prof_collect();
        if (rc) return rc;
        ctx->prof_pending = true;
    }
    ctx->prof_active = ctx->prof_on;
    const int rc = run_impl(ctx, steps);
    ctx->prof_active = false;
    return rc;
}

}  // extern "C"

namespace {

int run_impl(pns_ctx* ctx, int64_t steps)
{
    if (ctx->launch == PNS_LAUNCH_PLAIN) {
        for (int64_t s = 0; s < steps; ++s) {
            int rc = ctx->launch_chunk(1, 0, s == 0, s == steps - 1);
            if (rc) return rc;
        }
        return PNS_OK;
    }
    const int64_t chunk = ctx->chunk > 0 ? std::min<int64_t>(ctx->chunk, steps) : steps;
    // with profiling on, the graph form queues its launches directly: events
    // on the class streams cannot be timed inside a replayed graph here
    if (ctx->launch == PNS_LAUNCH_PERSISTENT || (ctx->launch == PNS_LAUNCH_GRAPH && ctx->prof_on)) {
        for (int64_t done = 0; done < steps; done += chunk) {
            int rc = ctx->launch_chunk(std::min(chunk, steps - done), 0, done == 0, done + chunk >= steps);
            if (rc) return rc;
        }
        return PNS_OK;
    }
    // graph form: capture the chunk launches of a run of `steps` once and replay
    if (ctx->graph_steps != steps) {
        if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
        if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
        ctx->graph_exec = nullptr;
        ctx->graph = nullptr;
        ctx->graph_steps = -1;
        HIP_TRY(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal), "begin capture");
        int rc = PNS_OK;
        for (int64_t done = 0; done < steps && rc == PNS_OK; done += chunk)
            rc = ctx->launch_chunk(std::min(chunk, steps - done), 0, done == 0, done + chunk >= steps);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(ctx->stream, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "end capture");
        ctx->graph = g;
        HIP_TRY(hipGraphInstantiate(&ctx->graph_exec, g, nullptr, nullptr, 0), "graph instantiate");
        ctx->graph_steps = steps;
    }
    HIP_TRY(hipGraphLaunch(ctx->graph_exec, ctx->stream), "graph launch");
    return PNS_OK;
}

}  // namespace

extern "C" {

int pns_profile(pns_ctx* ctx, int32_t enable)
{
    g_error.clear();
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    int rc = pns_sync(ctx);
    if (rc) return rc;
    const size_t K = ctx->classes.size();
    if (ctx->prof_ev.empty()) {
        ctx->prof_ev.assign(2 * K, nullptr);
        for (auto& ev : ctx->prof_ev) HIP_TRY(hipEventCreate(&ev), "profile event create");
    }
    ctx->prof_on = enable != 0;
    ctx->prof_pending = false;
    ctx->prof_ms.assign(K, 0.0);
    ctx->prof_launches.assign(K, 0);
    ctx->prof_runs_now.assign(K, 0);
    if ((rc = d2h(ctx->prof_base, ctx->counters, (size_t)ctx->num_chains * 6))) return rc;
    return PNS_OK;
}

int pns_profile_read(pns_ctx* ctx, pns_class_profile* out, int32_t capacity, int32_t* count)
{
    g_error.clear();
    if (!ctx || !count) return fail(PNS_EINVAL, "NULL argument");
    const int32_t K = (int32_t)ctx->classes.size();
    *count = K;
    if (!out) return PNS_OK;
    if (capacity < K) return fail(PNS_EINVAL, "%d launch classes, capacity %d", K, capacity);
    if (ctx->prof_base.empty()) return fail(PNS_EINVAL, "profiling was never started (pns_profile)");
    int rc = pns_sync(ctx);
    if (rc) return rc;
    if ((rc = ctx->prof_collect())) return rc;
    std::vector<int64_t> cnt;
    if ((rc = d2h(cnt, ctx->counters, (size_t)ctx->num_chains * 6))) return rc;
    for (int32_t ki = 0; ki < K; ++ki) {
        const LaunchClass& k = ctx->classes[ki];
        pns_class_profile p{};
        p.block = k.tile.block;
        p.groups = k.tile.groups;
        p.flavour = k.flav;
        p.chains = (int32_t)k.chains.size();
        p.N_min = INT32_MAX;
        p.N_max = 0;
        for (int32_t c : k.chains) {
            const ProblemRun& P = ctx->probs[ctx->h_chain_problem[c]];
            p.N_min = std::min(p.N_min, P.N);
            p.N_max = std::max(p.N_max, P.N);
            const int64_t fl = cnt[(size_t)c * 6 + 1] - ctx->prof_base[(size_t)c * 6 + 1];
            p.flips += fl;
            p.records += cnt[(size_t)c * 6 + 0] - ctx->prof_base[(size_t)c * 6 + 0];
            p.row_bytes += (double)fl * (double)P.N * (double)qsize(ctx->qtype);
        }
        p.launches = ctx->prof_launches[ki];
        p.kernel_ms = ctx->prof_ms[ki];
        out[ki] = p;
    }
    return PNS_OK;
}

int pns_class_of_chain(const pns_ctx* ctx, int32_t* cls)
{
    g_error.clear();
    if (!ctx || !cls) return fail(PNS_EINVAL, "NULL argument");
    for (size_t ki = 0; ki < ctx->classes.size(); ++ki)
        for (int32_t c : ctx->classes[ki].chains) cls[c] = (int32_t)ki;
    return PNS_OK;
}

int pns_sync(pns_ctx* ctx)
{
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(ctx->stream), "stream synchronize");
    HIP_TRY(hipGetLastError(), "queued work");
    return PNS_OK;
}

int pns_read(pns_ctx* ctx, uint8_t* states, int64_t* multiplicities, double* energies)
{
    g_error.clear();
    int rc = pns_sync(ctx);
    if (rc) return rc;
    const int64_t C = ctx->num_chains;
    if (states) {
        std::vector<uint8_t> xp;
        std::vector<int32_t> la;
        if ((rc = d2h(xp, ctx->x, (size_t)ctx->fields))) return rc;
        if ((rc = d2h(la, ctx->last_action, C))) return rc;
        std::vector<uint8_t> xs((size_t)ctx->h_offsets.back());
        for (int64_t c = 0; c < C; ++c) {
            const int32_t N = ctx->probs[ctx->h_chain_problem[c]].N;
            std::memcpy(&xs[ctx->h_offsets[c]], &xp[ctx->h_foff[c]], N);
            if (la[c] >= 0) xs[ctx->h_offsets[c] + la[c]] ^= 1u;  // the record's state is before the last move
        }
        if ((rc = copy_out(states, xs.data(), xs.size()))) return rc;
    }
    if (multiplicities) {
        std::vector<int64_t> m;
        if ((rc = d2h(m, ctx->last_M, C))) return rc;
        if ((rc = copy_out(multiplicities, m.data(), C * 8))) return rc;
    }
    if (energies) {
        std::vector<int64_t> eb;
        if ((rc = d2h(eb, ctx->last_E, C))) return rc;
        std::vector<double> e = energies_to_double(ctx, eb);
        if ((rc = copy_out(energies, e.data(), C * 8))) return rc;
    }
    return PNS_OK;
}

int pns_field_type(const pns_ctx* ctx) { return ctx ? ctx->htype : -1; }

int pns_tile(const pns_ctx* ctx, int32_t* block, int32_t* groups)
{
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    if (block) *block = ctx->probs[0].tile.block;
    if (groups) *groups = ctx->probs[0].tile.groups;
    return PNS_OK;
}

int pns_num_problems(const pns_ctx* ctx) { return ctx ? (int)ctx->probs.size() : 0; }

int pns_problem_info_get(const pns_ctx* ctx, int32_t p, pns_problem_info* info)
{
    if (!ctx || !info) return fail(PNS_EINVAL, "NULL argument");
    if (p < 0 || p >= (int32_t)ctx->probs.size()) return fail(PNS_EINVAL, "problem %d out of range", p);
    const ProblemRun& R = ctx->probs[p];
    info->N = R.N;
    info->subset_size = R.n;
    info->block = R.tile.block;
    info->groups = R.tile.groups;
    info->chain_begin = R.chain_begin;
    info->num_chains = R.chains;
    info->flavour = R.flav;
    info->reserved = 0;
    return PNS_OK;
}

int pns_chain_offsets(const pns_ctx* ctx, int64_t* offsets)
{
    if (!ctx || !offsets) return fail(PNS_EINVAL, "NULL argument");
    std::memcpy(offsets, ctx->h_offsets.data(), ctx->h_offsets.size() * sizeof(int64_t));
    return PNS_OK;
}

int pns_read_current(pns_ctx* ctx, uint8_t* states, double* energies, void* fields, int64_t* L, int64_t* set_index,
                     int64_t* step)
{
    g_error.clear();
    int rc = pns_sync(ctx);
    if (rc) return rc;
    const int64_t C = ctx->num_chains;
    if (states) {
        std::vector<uint8_t> xp;
        if ((rc = d2h(xp, ctx->x, (size_t)ctx->fields))) return rc;
        std::vector<uint8_t> xs((size_t)ctx->h_offsets.back());
        for (int64_t c = 0; c < C; ++c)
            std::memcpy(&xs[ctx->h_offsets[c]], &xp[ctx->h_foff[c]], ctx->probs[ctx->h_chain_problem[c]].N);
        if ((rc = copy_out(states, xs.data(), xs.size()))) return rc;
    }
    if (energies) {
        std::vector<int64_t> eb;
        if ((rc = d2h(eb, ctx->E, C))) return rc;
        std::vector<double> e = energies_to_double(ctx, eb);
        if ((rc = copy_out(energies, e.data(), C * 8))) return rc;
    }
    if (fields) {
        const size_t hb = ctx->htype == H_I32 ? 4 : 8;
        std::vector<uint8_t> hp, hs((size_t)ctx->h_offsets.back() * hb);
        if ((rc = d2h(hp, ctx->h, (size_t)ctx->fields * hb))) return rc;
        for (int64_t c = 0; c < C; ++c)
            std::memcpy(&hs[ctx->h_offsets[c] * hb], &hp[ctx->h_foff[c] * hb], ctx->probs[ctx->h_chain_problem[c]].N * hb);
        if ((rc = copy_out(fields, hs.data(), hs.size()))) return rc;
    }
    const std::pair<int64_t*, int64_t*> arrs[] = {{L, ctx->L}, {set_index, ctx->sub}, {step, ctx->step}};
    for (const auto& pr : arrs) {
        if (!pr.first) continue;
        std::vector<int64_t> v;
        if ((rc = d2h(v, pr.second, C))) return rc;
        if ((rc = copy_out(pr.first, v.data(), C * 8))) return rc;
    }
    return PNS_OK;
}

int pns_read_log(pns_ctx* ctx, int32_t* actions, int64_t* multiplicities, double* energies, double* p)
{
    g_error.clear();
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    if (ctx->log_cap == 0) return fail(PNS_EINVAL, "the per-step log is off (log_capacity = 0)");
    int rc = pns_sync(ctx);
    if (rc) return rc;
    const size_t cnt = (size_t)ctx->num_chains * ctx->log_cap;
    if (actions) {
        std::vector<int32_t> v;
        if ((rc = d2h(v, ctx->log_action, cnt)) || (rc = copy_out(actions, v.data(), cnt * 4))) return rc;
    }
    if (multiplicities) {
        std::vector<int64_t> v;
        if ((rc = d2h(v, ctx->log_M, cnt)) || (rc = copy_out(multiplicities, v.data(), cnt * 8))) return rc;
    }
    if (energies) {
        std::vector<int64_t> v;
        if ((rc = d2h(v, ctx->log_E, cnt))) return rc;
        std::vector<double> e = energies_to_double(ctx, v);
        if ((rc = copy_out(energies, e.data(), cnt * 8))) return rc;
    }
    if (p) {
        std::vector<double> v;
        if ((rc = d2h(v, ctx->log_p, cnt)) || (rc = copy_out(p, v.data(), cnt * 8))) return rc;
    }
    return PNS_OK;
}

int pns_read_hist(pns_ctx* ctx, uint64_t* hist_weighted, uint64_t* hist_visits)
{
    g_error.clear();
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    if (!ctx->hist_w) return fail(PNS_EINVAL, "histograms are off (opts.hist = 0)");
    int rc = pns_sync(ctx);
    if (rc) return rc;
    const size_t cnt = (size_t)1 << ctx->probs[0].N;
    if (hist_weighted) {
        std::vector<uint64_t> v;
        if ((rc = d2h(v, ctx->hist_w, cnt)) || (rc = copy_out(hist_weighted, v.data(), cnt * 8))) return rc;
    }
    if (hist_visits) {
        std::vector<uint64_t> v;
        if ((rc = d2h(v, ctx->hist_v, cnt)) || (rc = copy_out(hist_visits, v.data(), cnt * 8))) return rc;
    }
    return PNS_OK;
}

int pns_hist_clear(pns_ctx* ctx)
{
    g_error.clear();
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    if (!ctx->hist_w) return fail(PNS_EINVAL, "histograms are off (opts.hist = 0)");
    const int64_t cnt = (int64_t)1 << ctx->probs[0].N;
    hipError_t e = launch_fill64(ctx->hist_w, cnt, 0, ctx->stream);
    if (e == hipSuccess) e = launch_fill64(ctx->hist_v, cnt, 0, ctx->stream);
    if (e == hipSuccess) e = launch_fill64(ctx->hist_rb, cnt, 0, ctx->stream);  // +0.0 is all-zero bits
    if (e != hipSuccess) return hip_fail(e, "histogram clear");
    return PNS_OK;
}

int pns_read_snapshots(pns_ctx* ctx, uint8_t* states, int64_t* multiplicities, double* energies, int32_t* count)
{
    g_error.clear();
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    if (!ctx->snap_x) return fail(PNS_EINVAL, "snapshots are off (snapshot_every = 0)");
    int rc = pns_sync(ctx);
    if (rc) return rc;
    const int64_t C = ctx->num_chains, S = ctx->snap_cap;
    std::vector<int32_t> cnt;
    if ((rc = d2h(cnt, ctx->snap_count, C))) return rc;
    int32_t stored = (int32_t)S;
    for (int32_t v : cnt) stored = std::min<int32_t>(stored, v);
    if (count) *count = stored;
    if (states) {
        std::vector<uint8_t> xp;
        if ((rc = d2h(xp, ctx->snap_x, (size_t)C * S * ctx->max_pitch))) return rc;
        std::vector<uint8_t> xs = compact_rows(ctx, xp, ctx->max_pitch, S);
        if ((rc = copy_out(states, xs.data(), xs.size()))) return rc;
    }
    if (multiplicities) {
        std::vector<int64_t> v;
        if ((rc = d2h(v, ctx->snap_M, (size_t)C * S)) || (rc = copy_out(multiplicities, v.data(), C * S * 8))) return rc;
    }
    if (energies) {
        std::vector<int64_t> v;
        if ((rc = d2h(v, ctx->snap_E, (size_t)C * S))) return rc;
        std::vector<double> e = energies_to_double(ctx, v);
        if ((rc = copy_out(energies, e.data(), C * S * 8))) return rc;
    }
    return PNS_OK;
}

int pns_stats(pns_ctx* ctx, pns_chain_stats* stats)
{
    g_error.clear();
    if (!ctx || !stats) return fail(PNS_EINVAL, "NULL argument");
    int rc = pns_sync(ctx);
    if (rc) return rc;
    std::vector<int64_t> v;
    if ((rc = d2h(v, ctx->counters, (size_t)ctx->num_chains * 6))) return rc;
    for (int64_t c = 0; c < ctx->num_chains; ++c) {
        stats[c].steps = v[c * 6 + 0];
        stats[c].flips = v[c * 6 + 1];
        stats[c].stays = v[c * 6 + 2];
        stats[c].saturated = v[c * 6 + 3];
        std::memcpy(&stats[c].sum_M, &v[c * 6 + 4], 8);
        stats[c].anomalies = v[c * 6 + 5];
    }
    return PNS_OK;
}

int pns_destroy(pns_ctx* ctx)
{
    if (!ctx) return PNS_OK;
    (void)hipStreamSynchronize(ctx->stream);
    ctx->free_all();
    delete ctx;
    return PNS_OK;
}

}  // extern "C"

// ---- differentiation path ----

namespace {

// G (N x N, FP64, overwritten) = X^T diag(w) X, queued on `st` without a
// host synchronisation; device pointers.  The weights are integers m (exact
// path) or, when m is NULL, FP64 weights wf.  The sum of the weights goes to
// *sum_host (synchronising) and/or *sum_dev (queued), either may be NULL.
// Workspace comes from the stream-ordered allocator and is released in
// stream order.
int moments_device(const uint8_t* X, int64_t ldx, const int64_t* m, const double* wf, int64_t K, int32_t N, double* G,
                   hipStream_t st, double* sum_host, double* sum_dev)
{
    const int64_t kpad = std::max<int64_t>(64, round_up(K, 64));
    const int32_t npad = (int32_t)round_up(N, 64);
    const int64_t words = std::max<int64_t>(1, (K + 31) / 32);
    const int nt = npad / 64;
    const int64_t tiles = (int64_t)nt * (nt + 1) / 2;
    // words per wave: at least 32 (1024 records), about 2048 waves in all
    const int64_t chunk_words = std::max<int64_t>(32, (words * tiles + 2047) / 2048);
    const int64_t chunks = (words + chunk_words - 1) / chunk_words;
    uint16_t* pieces = nullptr;
    unsigned long long* cnt = nullptr;
    uint32_t* Xb = nullptr;
    float* part = nullptr;
    auto release = [&]() {
        if (pieces) (void)hipFreeAsync(pieces, st);
        if (cnt) (void)hipFreeAsync(cnt, st);
        if (Xb) (void)hipFreeAsync(Xb, st);
        if (part) (void)hipFreeAsync(part, st);
    };
    hipError_t e = hipMallocAsync(reinterpret_cast<void**>(&pieces), (size_t)3 * kpad * sizeof(uint16_t), st);
    // cnt: [0] sum of the weights (uint64, or FP64 bits), [1] largest integer
    // weight (0 on the FP64 path: no flushes), [2] largest |FP64 weight| bits
    if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&cnt), 3 * sizeof(unsigned long long), st);
    if (e == hipSuccess) e = hipMallocAsync(reinterpret_cast<void**>(&Xb), (size_t)words * npad * sizeof(uint32_t), st);
    if (e == hipSuccess)
        e = hipMallocAsync(reinterpret_cast<void**>(&part), (size_t)chunks * tiles * 64 * 64 * sizeof(float), st);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        release();
        return fail(PNS_ENOMEM, "workspace allocation failed: %s", hipGetErrorString(e));
    }
    e = launch_fill64(G, (int64_t)N * N, 0, st);
    if (e == hipSuccess) e = launch_fill64(cnt, 3, 0, st);
    if (e == hipSuccess) {
        if (m) e = launch_moments_prep(m, K, kpad, pieces, cnt, cnt + 1, st);
        else e = launch_moments_prep_f64(wf, K, kpad, pieces, reinterpret_cast<double*>(cnt), cnt + 2, st);
    }
    if (e == hipSuccess) e = launch_pack_bits(X, ldx, K, N, npad, words, Xb, st);
    if (e == hipSuccess) e = launch_moments(Xb, npad, words, N, pieces, kpad, chunk_words, cnt + 1, part, G, st);
    if (e == hipSuccess && !m) e = launch_moments_unscale(G, (int64_t)N * N, cnt + 2, st);
    if (e == hipSuccess && sum_dev) {
        if (m) e = launch_moments_sum(cnt, sum_dev, st);
        else e = hipMemcpyAsync(sum_dev, cnt, sizeof(double), hipMemcpyDeviceToDevice, st);
    }
    unsigned long long hs = 0;
    if (e == hipSuccess && sum_host) {
        e = hipMemcpyAsync(&hs, cnt, sizeof(hs), hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
    }
    release();
    if (e != hipSuccess) return hip_fail(e, "moments kernels");
    if (sum_host) {
        if (m) *sum_host = (double)hs;
        else std::memcpy(sum_host, &hs, sizeof(double));
    }
    return PNS_OK;
}

// pns_moments / pns_moments_f64: host or device inputs; exactly one of m, wf.
int moments_entry(const uint8_t* X, int64_t ldx, const int64_t* m, const double* wf, int64_t K, int32_t N, double* G,
                  double* sum_w, void* stream)
{
    g_error.clear();
    if (!X || (!m && !wf) || !G) return fail(PNS_EINVAL, "NULL argument");
    if (N < 1 || N > 32768) return fail(PNS_EINVAL, "N must be in [1, 32768]");
    if (K < 0) return fail(PNS_EINVAL, "K must be >= 0");
    if (ldx < N) return fail(PNS_EINVAL, "ldx must be >= N");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const void* wv = m ? static_cast<const void*>(m) : static_cast<const void*>(wf);
    const bool xd = is_device_ptr(X), md = is_device_ptr(wv), gd = is_device_ptr(G);
    uint8_t* dX = nullptr;
    int64_t* dm = nullptr;  // 8-byte weights of either type
    double* dG = nullptr;
    auto done = [&](int r) {
        if (!xd && dX) (void)hipFree(dX);
        if (!md && dm) (void)hipFree(dm);
        if (!gd && dG) (void)hipFree(dG);
        return r;
    };
    int rc = PNS_OK;
    if (xd) dX = const_cast<uint8_t*>(X);
    else if (!(rc = dev_alloc(&dX, (size_t)K * ldx)) && K > 0)
        if (hipMemcpy(dX, X, (size_t)K * ldx, hipMemcpyHostToDevice) != hipSuccess) rc = fail(PNS_EDEVICE, "upload X");
    if (rc) return done(rc);
    if (md) dm = static_cast<int64_t*>(const_cast<void*>(wv));
    else if (!(rc = dev_alloc(&dm, (size_t)K)) && K > 0)
        if (hipMemcpy(dm, wv, (size_t)K * 8, hipMemcpyHostToDevice) != hipSuccess) rc = fail(PNS_EDEVICE, "upload weights");
    if (rc) return done(rc);
    if (gd) dG = G;
    else if ((rc = dev_alloc(&dG, (size_t)N * N))) return done(rc);
    const bool sd = sum_w && is_device_ptr(sum_w);
    rc = moments_device(dX, ldx, m ? dm : nullptr, m ? nullptr : reinterpret_cast<const double*>(dm), K, N, dG, st,
                        sum_w && !sd ? sum_w : nullptr, sd ? sum_w : nullptr);
    if (rc) return done(rc);
    if (!gd) {
        hipError_t e = hipMemcpyAsync(G, dG, (size_t)N * N * 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return done(hip_fail(e, "download G"));
    }
    if (!xd || !md) {
        // host inputs were staged in temporary device buffers
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) return done(hip_fail(e, "moments"));
    }
    return done(PNS_OK);
}

// Snapshot moments of one problem with multiplicities (rb = false) or
// expected multiplicities (rb = true) as weights.
int snapshot_moments(pns_ctx* ctx, int32_t problem, bool rb, double* G, double* sum_w)
{
    g_error.clear();
    if (!ctx || !G) return fail(PNS_EINVAL, "NULL argument");
    if (!ctx->snap_x) return fail(PNS_EINVAL, "snapshots are off (snapshot_every = 0)");
    if (problem < 0 || problem >= (int32_t)ctx->probs.size()) return fail(PNS_EINVAL, "problem %d out of range", problem);
    const ProblemRun& R = ctx->probs[problem];
    const int64_t row0 = (int64_t)R.chain_begin * ctx->snap_cap;
    const int64_t K = (int64_t)R.chains * ctx->snap_cap;
    const bool gd = is_device_ptr(G);
    double* dG = G;
    int rc = PNS_OK;
    if (!gd && (rc = dev_alloc(&dG, (size_t)R.N * R.N))) return rc;
    const bool sd = sum_w && is_device_ptr(sum_w);
    rc = moments_device(ctx->snap_x + row0 * ctx->max_pitch, ctx->max_pitch, rb ? nullptr : ctx->snap_M + row0,
                        rb ? ctx->snap_w + row0 : nullptr, K, R.N, dG, ctx->stream, sum_w && !sd ? sum_w : nullptr,
                        sd ? sum_w : nullptr);
    if (!rc && !gd) {
        hipError_t e = hipMemcpyAsync(G, dG, (size_t)R.N * R.N * 8, hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) rc = hip_fail(e, "download G");
    }
    if (!gd) (void)hipFree(dG);
    return rc;
}

}  // namespace

extern "C" {

int pns_moments(const uint8_t* X, int64_t ldx, const int64_t* m, int64_t K, int32_t N, double* G, double* sum_m,
                void* stream)
{
    if (!m) {
        g_error.clear();
        return fail(PNS_EINVAL, "NULL argument");
    }
    return moments_entry(X, ldx, m, nullptr, K, N, G, sum_m, stream);
}

int pns_moments_f64(const uint8_t* X, int64_t ldx, const double* w, int64_t K, int32_t N, double* G, double* sum_w,
                    void* stream)
{
    if (!w) {
        g_error.clear();
        return fail(PNS_EINVAL, "NULL argument");
    }
    return moments_entry(X, ldx, nullptr, w, K, N, G, sum_w, stream);
}

int pns_snapshot_moments(pns_ctx* ctx, int32_t problem, double* G, double* sum_m)
{
    return snapshot_moments(ctx, problem, false, G, sum_m);
}

int pns_snapshot_moments_rb(pns_ctx* ctx, int32_t problem, double* G, double* sum_w)
{
    return snapshot_moments(ctx, problem, true, G, sum_w);
}

int pns_logz_grad(pns_ctx* ctx, int32_t problem, double beta, int32_t rb, double* grad, double* sum_w)
{
    g_error.clear();
    if (!ctx || !grad || !sum_w) return fail(PNS_EINVAL, "NULL argument");
    if (!is_device_ptr(grad) || !is_device_ptr(sum_w)) return fail(PNS_EINVAL, "grad and sum_w must be device memory");
    if (!std::isfinite(beta)) return fail(PNS_EINVAL, "beta must be finite");
    int rc = snapshot_moments(ctx, problem, rb != 0, grad, sum_w);
    if (rc) return rc;
    const int64_t N = ctx->probs[problem].N;
    HIP_TRY(launch_moments_to_grad(grad, N * N, beta, sum_w, ctx->stream), "gradient");
    return PNS_OK;
}

int pns_read_rb_weights(pns_ctx* ctx, double* log_w, double* snap_w, double* hist_rb)
{
    g_error.clear();
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    if (log_w && ctx->log_cap == 0) return fail(PNS_EINVAL, "the per-step log is off (log_capacity = 0)");
    if (snap_w && !ctx->snap_x) return fail(PNS_EINVAL, "snapshots are off (snapshot_every = 0)");
    if (hist_rb && !ctx->hist_w) return fail(PNS_EINVAL, "histograms are off (opts.hist = 0)");
    int rc = pns_sync(ctx);
    if (rc) return rc;
    const int64_t C = ctx->num_chains;
    auto out = [&](double* dst, const double* src, size_t cnt) {
        std::vector<double> v;
        int r = d2h(v, src, cnt);
        return r ? r : copy_out(dst, v.data(), cnt * 8);
    };
    if (log_w && (rc = out(log_w, ctx->log_w, (size_t)C * ctx->log_cap))) return rc;
    if (snap_w && (rc = out(snap_w, ctx->snap_w, (size_t)C * ctx->snap_cap))) return rc;
    if (hist_rb && (rc = out(hist_rb, ctx->hist_rb, (size_t)1 << ctx->probs[0].N))) return rc;
    return PNS_OK;
}

int pns_log_partition(const void* Q, int32_t N, int32_t dtype, int32_t layout, double beta, double* out, void* stream)
{
    g_error.clear();
    if (!Q || !out) return fail(PNS_EINVAL, "NULL argument");
    if (N < 1 || N > 32) return fail(PNS_EINVAL, "enumeration needs 1 <= N <= 32");
    if (dtype < PNS_I16 || dtype > PNS_F32) return fail(PNS_EINVAL, "unknown dtype %d", dtype);
    if (layout != PNS_SYMMETRIC && layout != PNS_UPPER) return fail(PNS_EINVAL, "unknown layout %d", layout);
    if (!(beta >= 0.0) || !std::isfinite(beta)) return fail(PNS_EINVAL, "beta must be finite and >= 0");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const size_t qbytes = (size_t)N * N * qsize(dtype);
    // the kernels read Q from device memory: copy a host matrix in
    std::vector<uint8_t> qh(qbytes);
    int rc = copy_in(qh.data(), Q, qbytes);
    if (rc) return rc;
    const int32_t lowbits = std::max(std::min(N, 6), N - 14);
    const int64_t nthreads = (int64_t)1 << (N - lowbits);
    const int32_t blocks = (int32_t)((nthreads + 255) / 256);
    uint8_t* dq = nullptr;
    double* part = nullptr;
    double* dout = nullptr;
    auto done = [&](int r) {
        if (dq) (void)hipFree(dq);
        if (part) (void)hipFree(part);
        if (dout) (void)hipFree(dout);
        return r;
    };
    if ((rc = dev_alloc(&dq, qbytes)) || (rc = dev_alloc(&part, (size_t)2 * blocks)) || (rc = dev_alloc(&dout, 1)))
        return done(rc);
    hipError_t e = hipMemcpyAsync(dq, qh.data(), qbytes, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = launch_logz(dtype, dq, N, layout, beta, part, part + blocks, blocks, lowbits, nthreads, dout, st);
    double v = 0.0;
    if (e == hipSuccess) e = hipMemcpyAsync(&v, dout, 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return done(hip_fail(e, "log partition"));
    if (is_device_ptr(out)) {
        if ((e = hipMemcpy(out, &v, 8, hipMemcpyHostToDevice)) != hipSuccess) return done(hip_fail(e, "copy out"));
    } else {
        *out = v;
    }
    return done(PNS_OK);
}

}  // extern "C"

extern "C" {

int pns_set_q(pns_ctx* ctx, int32_t problem, const void* Q)
{
    g_error.clear();
    if (!ctx || !Q) return fail(PNS_EINVAL, "NULL argument");
    if (problem < 0 || problem >= (int32_t)ctx->probs.size()) return fail(PNS_EINVAL, "problem %d out of range", problem);
    ProblemRun& R = ctx->probs[problem];
    hipStream_t st = ctx->stream;
    const size_t qb = qsize(ctx->qtype);
    const size_t qbytes = (size_t)R.N * R.N * qb;
    const size_t abytes = (size_t)R.N * R.pitch * qb;
    const size_t dbytes = (size_t)R.pitch * 4;
    int rc = PNS_OK;
    if (!R.A2) {
        // (with the tail padding the window kernels read past the last row)
        if ((rc = dev_alloc(reinterpret_cast<uint8_t**>(&R.A2), abytes + kRowTailBytes))) return rc;
        HIP_TRY(hipMemset(static_cast<uint8_t*>(R.A2) + abytes, 0, kRowTailBytes), "zero the row tail");
    }
    if (!R.diag2 && (rc = dev_alloc(reinterpret_cast<uint8_t**>(&R.diag2), dbytes))) return rc;
    const void* dq = Q;
    void* tmp = nullptr;
    unsigned long long* flags = nullptr;
    auto done = [&](int r) {
        if (tmp) (void)hipFree(tmp);
        if (flags) (void)hipFree(flags);
        return r;
    };
    if (!is_device_ptr(Q)) {
        if ((rc = dev_alloc(reinterpret_cast<uint8_t**>(&tmp), qbytes))) return done(rc);
        HIP_TRY(hipMemcpyAsync(tmp, Q, qbytes, hipMemcpyHostToDevice, st), "upload Q");
        dq = tmp;
    }
    if ((rc = dev_alloc(&flags, 4))) return done(rc);
    hipError_t e = launch_fill64(flags, 4, 0, st);
    if (e == hipSuccess) e = launch_prepare_rows(ctx->qtype, dq, R.N, R.layout, R.pitch, R.A2, R.diag2, flags, st);
    unsigned long long hf[4] = {0, 0, 0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return done(hip_fail(e, "prepare Q"));
    if (hf[0]) return done(fail(PNS_EINVAL, "SYMMETRIC Q is not symmetric"));
    if (hf[1]) return done(fail(PNS_EINVAL, "Q has a non-finite entry"));
    double fb, db;
    std::memcpy(&fb, &hf[2], 8);
    std::memcpy(&db, &hf[3], 8);
    const double eb = db + R.s * fb;
    if (ctx->qtype != Q_F32) {
        if (eb * (double)R.N > 9.0e18) return done(fail(PNS_EINVAL, "energy bound of Q overflows int64"));
        if (ctx->htype == H_I32 && !(fb < 2147483647.0 && eb < 2147483647.0))
            return done(fail(PNS_EUNSUPPORTED, "the new Q needs 64-bit fields; this context has 32-bit fields"));
    }
    std::swap(R.A, R.A2);
    std::swap(R.diag, R.diag2);
    Problem D{};
    D.A = R.A;
    D.diag = R.diag;
    D.pitch = R.pitch;
    D.num_sets = R.num_sets;
    D.L0 = R.L0;
    D.N = R.N;
    D.n = R.n;
    D.s = R.s;
    D.qtype = ctx->qtype;
    // the struct copy is staged through host memory the call keeps alive
    // until the synchronisation below
    HIP_TRY(hipMemcpyAsync(ctx->problems + problem, &D, sizeof(Problem), hipMemcpyHostToDevice, st), "upload problem");
    // fields and energies of the problem's chains from their current states
    InitArgs ia{};
    const int32_t c0 = R.chain_begin;
    ia.problems = ctx->problems;
    ia.chain_problem = ctx->chain_problem + c0;
    ia.foff = ctx->foff + c0;
    ia.num_chains = R.chains;
    ia.init = 2;
    ia.seed = ctx->seed;
    ia.chain_id = ctx->chain_id + c0;
    ia.x = ctx->x;
    ia.h = ctx->h;
    ia.E = ctx->E + c0;
    ia.last_E = ctx->last_E + c0;
    e = launch_init_with_map(ctx->qtype, ctx->htype, (int32_t)R.pitch, st, ia, ctx->h_chain_problem.data() + c0,
                             ctx->pitches().data());
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return done(hip_fail(e, "recompute fields"));
    return done(PNS_OK);
}

int pns_snapshots_clear(pns_ctx* ctx)
{
    g_error.clear();
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    if (!ctx->snap_x) return fail(PNS_EINVAL, "snapshots are off (snapshot_every = 0)");
    const int64_t C = ctx->num_chains;
    hipError_t e = launch_fill64(ctx->snap_M, C * ctx->snap_cap, 0, ctx->stream);
    if (e == hipSuccess) e = launch_fill64(ctx->snap_w, C * ctx->snap_cap, 0, ctx->stream);
    // counts are int32: clear them as 64-bit words, rounded up (the buffer
    // holds whole 64-bit words)
    if (e == hipSuccess) e = launch_fill64(ctx->snap_count, (C + 1) / 2, 0, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "clear snapshots");
    return PNS_OK;
}

}  // extern "C"

extern "C" {

int pns_optimize(pns_ctx* ctx, int64_t steps, double temperature)
{
    g_error.clear();
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    if (steps < 0) return fail(PNS_EINVAL, "steps must be >= 0");
    if (!(temperature > 0.0) || !std::isfinite(temperature)) return fail(PNS_EINVAL, "temperature must be finite and > 0");
    if (steps == 0) return PNS_OK;
    const int64_t C = ctx->num_chains;
    hipStream_t st = ctx->stream;
    if (!ctx->xbest) {
        int rc = dev_alloc(&ctx->xbest, (size_t)ctx->fields);
        if (!rc) rc = dev_alloc(&ctx->Ebest, (size_t)C);
        if (rc) return rc;
    }
    if (!ctx->best_valid) {
        // X_max = J_0: the current states
        HIP_TRY(hipMemcpyAsync(ctx->xbest, ctx->x, (size_t)ctx->fields, hipMemcpyDeviceToDevice, st), "best init");
        HIP_TRY(hipMemcpyAsync(ctx->Ebest, ctx->E, (size_t)C * 8, hipMemcpyDeviceToDevice, st), "best init");
        ctx->best_valid = true;
    }
    if (ctx->opt_classes.empty()) {
        // every chain of a problem with n < N draws a fresh subset each step
        // (flavour 2), the others consider all bits (flavour 0)
        std::map<std::pair<std::pair<int32_t, int32_t>, int32_t>, size_t> class_of;
        for (size_t p = 0; p < ctx->probs.size(); ++p) {
            const ProblemRun& R = ctx->probs[p];
            const int32_t flav = (ctx->mode != PNS_MODE_RF && R.n < R.N) ? 2 : 0;
            const auto key = std::make_pair(std::make_pair(R.tile.block, R.tile.groups), flav);
            if (!class_of.count(key)) {
                class_of[key] = ctx->opt_classes.size();
                LaunchClass k;
                // (a window-kernel tile runs the optimization on the table's)
                k.tile = have_tile(ctx->qtype, ctx->htype, R.tile.block, R.tile.groups) ? R.tile : default_tile(R.N);
                k.flav = flav;
                k.dyn = 0;
                ctx->opt_classes.push_back(k);
            }
            LaunchClass& K = ctx->opt_classes[class_of[key]];
            K.dyn = std::max(K.dyn, (size_t)R.pitch * 4 * (flav == 2 ? 2 : 1));
            for (int32_t c = 0; c < R.chains; ++c) K.chains.push_back(R.chain_begin + c);
        }
        for (auto& k : ctx->opt_classes) {
            int rc = dev_alloc(&k.d_list, k.chains.size());
            if (rc) return rc;
            HIP_TRY(hipMemcpy(k.d_list, k.chains.data(), k.chains.size() * sizeof(int32_t), hipMemcpyHostToDevice),
                    "upload chain list");
        }
    }
    const int64_t chunk = ctx->chunk > 0 ? std::min<int64_t>(ctx->chunk, steps) : steps;
    for (int64_t done = 0; done < steps; done += chunk) {
        for (auto& k : ctx->opt_classes) {
            StepArgs a = ctx->args(std::min(chunk, steps - done));
            a.mode = 4;  // Alg 9 / Alg 10
            a.inv_temp = 1.0 / temperature;
            a.xbest = ctx->xbest;
            a.Ebest = ctx->Ebest;
            if (ctx->opt_classes.size() > 1 || (int64_t)k.chains.size() != C) a.chain_list = k.d_list;
            hipError_t e = launch_steps(ctx->qtype, ctx->htype, k.flav, true, k.tile.block, k.tile.groups,
                                        (int32_t)k.chains.size(), k.dyn, st, a);
            if (e != hipSuccess) return hip_fail(e, "optimization kernel launch");
        }
    }
    return PNS_OK;
}

int pns_read_best(pns_ctx* ctx, uint8_t* states, double* energies)
{
    g_error.clear();
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    if (!ctx->best_valid) return fail(PNS_EINVAL, "no optimization has run (pns_optimize)");
    int rc = pns_sync(ctx);
    if (rc) return rc;
    const int64_t C = ctx->num_chains;
    if (states) {
        std::vector<uint8_t> xp;
        if ((rc = d2h(xp, ctx->xbest, (size_t)ctx->fields))) return rc;
        std::vector<uint8_t> xs((size_t)ctx->h_offsets.back());
        for (int64_t c = 0; c < C; ++c)
            std::memcpy(&xs[ctx->h_offsets[c]], &xp[ctx->h_foff[c]], ctx->probs[ctx->h_chain_problem[c]].N);
        if ((rc = copy_out(states, xs.data(), xs.size()))) return rc;
    }
    if (energies) {
        std::vector<int64_t> eb;
        if ((rc = d2h(eb, ctx->Ebest, C))) return rc;
        std::vector<double> e = energies_to_double(ctx, eb);
        if ((rc = copy_out(energies, e.data(), C * 8))) return rc;
    }
    return PNS_OK;
}

int pns_adopt_best(pns_ctx* ctx)
{
    g_error.clear();
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    if (!ctx->best_valid) return fail(PNS_EINVAL, "no optimization has run (pns_optimize)");
    hipStream_t st = ctx->stream;
    const int64_t C = ctx->num_chains;
    HIP_TRY(hipMemcpyAsync(ctx->x, ctx->xbest, (size_t)ctx->fields, hipMemcpyDeviceToDevice, st), "adopt best");
    // fields and energies of the new states; budgets restart (a new block)
    InitArgs ia{};
    ia.problems = ctx->problems;
    ia.chain_problem = ctx->chain_problem;
    ia.foff = ctx->foff;
    ia.num_chains = (int32_t)C;
    ia.init = 2;
    ia.seed = ctx->seed;
    ia.chain_id = ctx->chain_id;
    ia.x = ctx->x;
    ia.h = ctx->h;
    ia.E = ctx->E;
    ia.last_E = ctx->last_E;
    hipError_t e = launch_init_with_map(ctx->qtype, ctx->htype, (int32_t)ctx->max_pitch, st, ia,
                                        ctx->h_chain_problem.data(), ctx->pitches().data());
    if (e != hipSuccess) return hip_fail(e, "recompute fields");
    std::vector<int64_t> Lv((size_t)C);
    for (int64_t c = 0; c < C; ++c) Lv[c] = ctx->probs[ctx->h_chain_problem[c]].L0;
    std::vector<int32_t> la((size_t)C, PNS_STAY);
    HIP_TRY(hipMemcpyAsync(ctx->L, Lv.data(), C * 8, hipMemcpyHostToDevice, st), "reset budgets");
    HIP_TRY(hipMemcpyAsync(ctx->last_action, la.data(), C * 4, hipMemcpyHostToDevice, st), "reset records");
    HIP_TRY(hipStreamSynchronize(st), "adopt best");
    return PNS_OK;
}

}  // extern "C"

extern "C" {

int pns_run_original(pns_ctx* ctx, int64_t original_steps)
{
    g_error.clear();
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    if (ctx->mode != PNS_MODE_RF && ctx->mode != PNS_MODE_BASIC)
        return fail(PNS_EINVAL, "runs of original samples need a Rejection-Free or Basic PNS context");
    if (original_steps < 0) return fail(PNS_EINVAL, "original_steps must be >= 0");
    if (original_steps == 0) return PNS_OK;
    // every record covers at least one original sample, so original_steps
    // records always reach the end
    return ctx->launch_chunk(original_steps, original_steps);
}

int pns_pt_swap(pns_ctx* ctx, int32_t temps, int64_t round, int32_t* accepted)
{
    g_error.clear();
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    const int64_t C = ctx->num_chains;
    if (temps < 2 || C % temps != 0) return fail(PNS_EINVAL, "temps must be >= 2 and divide the number of chains");
    if (round < 0) return fail(PNS_EINVAL, "round must be >= 0");
    for (int64_t g0 = 0; g0 < C; g0 += temps)
        if (ctx->h_chain_problem[g0] != ctx->h_chain_problem[g0 + temps - 1])
            return fail(PNS_EINVAL, "a tempering group spans two problems");
    hipStream_t st = ctx->stream;
    if (ctx->pt_T != temps) {
        // ladder: each group's chains ordered by their current beta
        std::vector<double> b;
        int rc = pns_sync(ctx);
        if (!rc) rc = d2h(b, ctx->beta, (size_t)C);
        if (rc) return rc;
        std::vector<int32_t> lad((size_t)C);
        for (int64_t g0 = 0; g0 < C; g0 += temps) {
            for (int32_t t = 0; t < temps; ++t) lad[g0 + t] = t;
            std::stable_sort(lad.begin() + g0, lad.begin() + g0 + temps,
                             [&](int32_t x, int32_t y) { return b[g0 + x] < b[g0 + y]; });
        }
        if (!ctx->pt_ladder && (rc = dev_alloc(&ctx->pt_ladder, (size_t)C))) return rc;
        if (!ctx->pt_accepted && (rc = dev_alloc(&ctx->pt_accepted, (size_t)C))) return rc;
        HIP_TRY(hipMemcpy(ctx->pt_ladder, lad.data(), C * sizeof(int32_t), hipMemcpyHostToDevice), "upload ladder");
        ctx->pt_T = temps;
    }
    const bool acc_dev = accepted && is_device_ptr(accepted);
    int32_t* dacc = accepted ? (acc_dev ? accepted : ctx->pt_accepted) : nullptr;
    if (dacc) {
        hipError_t e = launch_fill64(dacc, C / 2, 0, st);
        if (e != hipSuccess) return hip_fail(e, "clear accepted");
        if (C % 2) HIP_TRY(hipMemsetAsync(dacc + C - 1, 0, 4, st), "clear accepted");
    }
    hipError_t e = launch_pt_swap(ctx->E, ctx->qtype == Q_F32 ? 1 : 0, ctx->beta, ctx->pt_ladder,
                                  (int32_t)(C / temps), temps, ctx->seed, (uint64_t)round, dacc, st);
    if (e != hipSuccess) return hip_fail(e, "swap kernel");
    if (accepted && !acc_dev) {
        HIP_TRY(hipMemcpyAsync(accepted, dacc, C * sizeof(int32_t), hipMemcpyDeviceToHost, st), "download accepted");
        HIP_TRY(hipStreamSynchronize(st), "swap");
    }
    return PNS_OK;
}

int pns_read_betas(pns_ctx* ctx, double* betas)
{
    g_error.clear();
    if (!ctx || !betas) return fail(PNS_EINVAL, "NULL argument");
    int rc = pns_sync(ctx);
    if (rc) return rc;
    std::vector<double> b;
    if ((rc = d2h(b, ctx->beta, (size_t)ctx->num_chains))) return rc;
    return copy_out(betas, b.data(), b.size() * 8);
}

int pns_read_ladder(pns_ctx* ctx, int32_t* ladder)
{
    g_error.clear();
    if (!ctx || !ladder) return fail(PNS_EINVAL, "NULL argument");
    if (!ctx->pt_ladder) return fail(PNS_EINVAL, "no tempering ladder yet (pns_pt_swap)");
    int rc = pns_sync(ctx);
    if (rc) return rc;
    std::vector<int32_t> l;
    if ((rc = d2h(l, ctx->pt_ladder, (size_t)ctx->num_chains))) return rc;
    return copy_out(ladder, l.data(), l.size() * 4);
}

}  // extern "C"

// ---- field refresh ----

extern "C" int pns_refresh(pns_ctx* ctx)
{
    g_error.clear();
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    InitArgs ia{};
    ia.problems = ctx->problems;
    ia.chain_problem = ctx->chain_problem;
    ia.foff = ctx->foff;
    ia.num_chains = ctx->num_chains;
    ia.init = 2;
    ia.seed = ctx->seed;
    ia.chain_id = ctx->chain_id;
    ia.x = ctx->x;
    ia.h = ctx->h;
    ia.E = ctx->E;
    ia.last_E = nullptr;  // the last record keeps its energy
    hipError_t e = launch_init_with_map(ctx->qtype, ctx->htype, (int32_t)ctx->max_pitch, ctx->stream, ia,
                                        ctx->h_chain_problem.data(), ctx->pitches().data());
    if (e != hipSuccess) return hip_fail(e, "field refresh");
    return PNS_OK;
}

// ---- checkpoints (pns_save / pns_load) ----

namespace {

constexpr char kCkptMagic[8] = {'P', 'N', 'S', 'C', 'K', 'P', 'T', '1'};
constexpr uint32_t kCkptVersion = 1;

enum : uint32_t { kCkptRandSets = 1u, kCkptLadder = 2u, kCkptBest = 4u };

// Fixed-size header of a checkpoint; the problem descriptors, the state
// arrays and an FNV-1a checksum of everything before it follow.
struct CkptHeader {
    char magic[8];
    uint32_t version;
    uint32_t flags;
    int32_t mode, qtype, htype, num_chains;
    int32_t num_problems, pt_T;
    uint64_t seed;
    int64_t fields;
    int64_t total_bytes;
};

struct CkptProblem {
    int32_t N, n, layout, chains;
    int64_t L0, pitch;
};

uint64_t fnv1a(const uint8_t* p, size_t n)
{
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= p[i];
        h *= 1099511628211ull;
    }
    return h;
}

// One device array of the chain state: address and byte count.
struct CkptArray {
    void* dev;
    size_t bytes;
};

// The arrays a checkpoint holds, in their order in the blob.
std::vector<CkptArray> ckpt_arrays(pns_ctx* ctx, uint32_t flags)
{
    const size_t C = (size_t)ctx->num_chains, F = (size_t)ctx->fields;
    const size_t hb = ctx->htype == H_I32 ? 4 : 8;
    std::vector<CkptArray> a = {
        {ctx->x, F},          {ctx->h, F * hb},          {ctx->E, C * 8},          {ctx->L, C * 8},
        {ctx->sub, C * 8},    {ctx->step, C * 8},        {ctx->last_action, C * 4}, {ctx->last_M, C * 8},
        {ctx->last_E, C * 8}, {ctx->counters, C * 6 * 8}, {ctx->beta, C * 8},       {ctx->chain_id, C * 4},
    };
    if (flags & kCkptRandSets) a.push_back({ctx->rmem, F});
    if (flags & kCkptLadder) a.push_back({ctx->pt_ladder, C * 4});
    if (flags & kCkptBest) {
        a.push_back({ctx->xbest, F});
        a.push_back({ctx->Ebest, C * 8});
    }
    return a;
}

uint32_t ckpt_flags(const pns_ctx* ctx)
{
    return (ctx->rmem ? kCkptRandSets : 0u) | (ctx->pt_ladder ? kCkptLadder : 0u) |
           (ctx->best_valid ? kCkptBest : 0u);
}

size_t ckpt_size(pns_ctx* ctx, uint32_t flags)
{
    size_t n = sizeof(CkptHeader) + ctx->probs.size() * sizeof(CkptProblem) + 8;
    for (const CkptArray& a : ckpt_arrays(ctx, flags)) n += a.bytes;
    return n;
}

}  // namespace

extern "C" {

int pns_save(pns_ctx* ctx, void* buf, int64_t capacity, int64_t* size)
{
    g_error.clear();
    if (!ctx || !size) return fail(PNS_EINVAL, "NULL argument");
    const uint32_t flags = ckpt_flags(ctx);
    const size_t total = ckpt_size(ctx, flags);
    *size = (int64_t)total;
    if (!buf) return PNS_OK;
    if (capacity < (int64_t)total) return fail(PNS_EINVAL, "checkpoint needs %zu bytes, buffer holds %lld", total,
                                               (long long)capacity);
    int rc = pns_sync(ctx);
    if (rc) return rc;
    std::vector<uint8_t> blob(total);
    CkptHeader h{};
    std::memcpy(h.magic, kCkptMagic, 8);
    h.version = kCkptVersion;
    h.flags = flags;
    h.mode = ctx->mode;
    h.qtype = ctx->qtype;
    h.htype = ctx->htype;
    h.num_chains = ctx->num_chains;
    h.num_problems = (int32_t)ctx->probs.size();
    h.pt_T = ctx->pt_T;
    h.seed = ctx->seed;
    h.fields = ctx->fields;
    h.total_bytes = (int64_t)total;
    size_t off = 0;
    std::memcpy(&blob[off], &h, sizeof(h));
    off += sizeof(h);
    for (const ProblemRun& P : ctx->probs) {
        CkptProblem cp{P.N, P.n, P.layout, P.chains, P.L0, P.pitch};
        std::memcpy(&blob[off], &cp, sizeof(cp));
        off += sizeof(cp);
    }
    for (const CkptArray& a : ckpt_arrays(ctx, flags)) {
        HIP_TRY(hipMemcpy(&blob[off], a.dev, a.bytes, hipMemcpyDeviceToHost), "checkpoint download");
        off += a.bytes;
    }
    const uint64_t sum = fnv1a(blob.data(), off);
    std::memcpy(&blob[off], &sum, 8);
    return copy_out(buf, blob.data(), total);
}

int pns_load(pns_ctx* ctx, const void* buf, int64_t size)
{
    g_error.clear();
    if (!ctx || !buf) return fail(PNS_EINVAL, "NULL argument");
    if (size < (int64_t)sizeof(CkptHeader)) return fail(PNS_EINVAL, "checkpoint of %lld bytes is too short",
                                                         (long long)size);
    std::vector<uint8_t> blob((size_t)size);
    int rc = copy_in(blob.data(), buf, blob.size());
    if (rc) return rc;
    CkptHeader h;
    std::memcpy(&h, blob.data(), sizeof(h));
    if (std::memcmp(h.magic, kCkptMagic, 8) != 0 || h.version != kCkptVersion)
        return fail(PNS_EINVAL, "not a checkpoint of this library version");
    if (h.total_bytes != size) return fail(PNS_EINVAL, "checkpoint size %lld, header says %lld", (long long)size,
                                           (long long)h.total_bytes);
    uint64_t sum;
    std::memcpy(&sum, &blob[(size_t)size - 8], 8);
    if (sum != fnv1a(blob.data(), (size_t)size - 8)) return fail(PNS_EINVAL, "checkpoint checksum mismatch");
    if (h.mode != ctx->mode || h.qtype != ctx->qtype || h.htype != ctx->htype || h.num_chains != ctx->num_chains ||
        h.num_problems != (int32_t)ctx->probs.size() || h.seed != ctx->seed || h.fields != ctx->fields)
        return fail(PNS_EINVAL, "checkpoint is of a context with another mode, element type, chain count, "
                                "problem count or seed");
    size_t off = sizeof(h);
    for (const ProblemRun& P : ctx->probs) {
        CkptProblem cp;
        std::memcpy(&cp, &blob[off], sizeof(cp));
        off += sizeof(cp);
        if (cp.N != P.N || cp.n != P.n || cp.layout != P.layout || cp.chains != P.chains || cp.L0 != P.L0 ||
            cp.pitch != P.pitch)
            return fail(PNS_EINVAL, "checkpoint problem (N=%d, n=%d, L0=%lld, %d chains) differs from the "
                                    "context's (N=%d, n=%d, L0=%lld, %d chains)",
                        cp.N, cp.n, (long long)cp.L0, cp.chains, P.N, P.n, (long long)P.L0, P.chains);
    }
    if ((rc = pns_sync(ctx))) return rc;
    // the chain ids must be those of this context
    std::vector<uint32_t> cid;
    if ((rc = d2h(cid, ctx->chain_id, (size_t)ctx->num_chains))) return rc;
    {
        size_t o2 = off;
        for (const CkptArray& a : ckpt_arrays(ctx, 0)) {
            if (a.dev == ctx->chain_id) {
                if (std::memcmp(&blob[o2], cid.data(), a.bytes) != 0)
                    return fail(PNS_EINVAL, "checkpoint chain ids differ (another chain_id_base)");
                break;
            }
            o2 += a.bytes;
        }
    }
    // optional parts the context may not have yet
    if ((h.flags & kCkptLadder) && !ctx->pt_ladder) {
        if ((rc = dev_alloc(&ctx->pt_ladder, (size_t)ctx->num_chains))) return rc;
        if (!ctx->pt_accepted && (rc = dev_alloc(&ctx->pt_accepted, (size_t)ctx->num_chains))) return rc;
    }
    if ((h.flags & kCkptBest) && !ctx->xbest) {
        if ((rc = dev_alloc(&ctx->xbest, (size_t)ctx->fields))) return rc;
        if ((rc = dev_alloc(&ctx->Ebest, (size_t)ctx->num_chains))) return rc;
    }
    if ((h.flags & kCkptRandSets) && !ctx->rmem) return fail(PNS_EINVAL, "checkpoint holds random sets");
    for (const CkptArray& a : ckpt_arrays(ctx, h.flags)) {
        HIP_TRY(hipMemcpy(a.dev, &blob[off], a.bytes, hipMemcpyHostToDevice), "checkpoint upload");
        off += a.bytes;
    }
    ctx->pt_T = h.pt_T;
    ctx->best_valid = (h.flags & kCkptBest) != 0;
    return PNS_OK;
}

}  // extern "C"

// ---- continuous Unbiased PNS (Alg 7, donut target) ----

struct pns_cont {
    pns_cont_opts o{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int32_t C = 0, dim = 0;
    uint32_t* chain_id = nullptr;
    double* x = nullptr;
    double* lpx = nullptr;
    int64_t* L = nullptr;
    int64_t* set = nullptr;
    int64_t* step = nullptr;
    int64_t* counters = nullptr;
    double* sums = nullptr;
    int32_t* log_action = nullptr;
    int64_t* log_M = nullptr;
    double* log_lp = nullptr;
    double* log_p = nullptr;
    double* log_w = nullptr;

    ContArgs args(int64_t steps) const
    {
        ContArgs a{};
        a.dim = dim;
        a.pairs = o.pairs;
        a.mu0 = o.mu0;
        a.c = 1.0 / (2.0 * o.sigma * o.sigma);
        a.L0 = o.L0;
        a.seed = o.seed;
        a.num_chains = C;
        a.chain_id = chain_id;
        a.x = x;
        a.lpx = lpx;
        a.L = L;
        a.set = set;
        a.step = step;
        a.counters = counters;
        a.sums = sums;
        a.steps = steps;
        a.log_cap = o.log_capacity;
        a.log_action = log_action;
        a.log_M = log_M;
        a.log_lp = log_lp;
        a.log_p = log_p;
        a.log_w = log_w;
        return a;
    }

    void free_all()
    {
        void* ptrs[] = {chain_id, x, lpx, L, set, step, counters, sums, log_action, log_M, log_lp, log_p, log_w};
        for (void* p : ptrs)
            if (p) (void)hipFree(p);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

namespace {

constexpr int64_t kContChunk = 8192;  // records per chain per launch

int cont_sums_count(const pns_cont* ctx) { return 2 * (4 * ctx->dim + 1); }

}  // namespace

extern "C" {

void pns_cont_opts_default(pns_cont_opts* o)
{
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->dim = 2;
    o->pairs = 25;
    o->mu0 = 9.0;
    o->sigma = 0.1;
    o->L0 = 1000;
    o->num_chains = 1;
}

int pns_cont_create(pns_cont** out, const pns_cont_opts* o)
{
    g_error.clear();
    if (!out || !o) return fail(PNS_EINVAL, "NULL argument");
    *out = nullptr;
    if (o->dim < 1 || o->dim > 7) return fail(PNS_EINVAL, "dim must be in [1, 7]");
    if (o->pairs < 1 || o->pairs > 32) return fail(PNS_EINVAL, "pairs must be in [1, 32]");
    if (!(o->sigma > 0.0) || !std::isfinite(o->sigma)) return fail(PNS_EINVAL, "sigma must be finite and > 0");
    if (!std::isfinite(o->mu0)) return fail(PNS_EINVAL, "mu0 must be finite");
    if (!std::isfinite(1.0 / (2.0 * o->sigma * o->sigma)) || 2.0 * o->sigma * o->sigma == 0.0 ||
        !std::isfinite(2.0 * o->sigma * o->sigma))
        return fail(PNS_EINVAL, "2 sigma^2 and its reciprocal must be finite positive doubles");
    if (o->L0 < 1 || o->L0 > ((int64_t)1 << 53)) return fail(PNS_EINVAL, "L0 must be in [1, 2^53]");
    if (o->num_chains < 1) return fail(PNS_EINVAL, "num_chains must be >= 1");
    if (o->log_capacity < 0) return fail(PNS_EINVAL, "log_capacity must be >= 0");
    for (int r : o->reserved)
        if (r != 0) return fail(PNS_EINVAL, "reserved fields must be zero");
    const int64_t C = o->num_chains, d = o->dim;
    std::vector<double> x0((size_t)(C * d), 0.0);
    if (o->x0) {
        int rc = copy_in(x0.data(), o->x0, x0.size() * sizeof(double));
        if (rc) return rc;
        for (double v : x0)
            if (!std::isfinite(v)) return fail(PNS_EINVAL, "x0 must be finite");
    }
    pns_cont* ctx = new pns_cont();
    ctx->o = *o;
    ctx->o.x0 = nullptr;
    ctx->C = o->num_chains;
    ctx->dim = o->dim;
    auto fail_free = [&](int rc) {
        ctx->free_all();
        delete ctx;
        return rc;
    };
    if (o->stream) {
        ctx->stream = reinterpret_cast<hipStream_t>(o->stream);
    } else {
        hipError_t e = hipStreamCreate(&ctx->stream);
        if (e != hipSuccess) return fail_free(hip_fail(e, "hipStreamCreate"));
        ctx->own_stream = true;
    }
    const int ns = cont_sums_count(ctx);
    int rc = PNS_OK;
    if (!rc) rc = dev_alloc(&ctx->chain_id, (size_t)C);
    if (!rc) rc = dev_alloc(&ctx->x, (size_t)(C * d));
    if (!rc) rc = dev_alloc(&ctx->lpx, (size_t)C);
    if (!rc) rc = dev_alloc(&ctx->L, (size_t)C);
    if (!rc) rc = dev_alloc(&ctx->set, (size_t)C);
    if (!rc) rc = dev_alloc(&ctx->step, (size_t)C);
    if (!rc) rc = dev_alloc(&ctx->counters, (size_t)C * 2);
    if (!rc) rc = dev_alloc(&ctx->sums, (size_t)C * ns);
    if (!rc && o->log_capacity > 0) {
        const size_t n = (size_t)C * (size_t)o->log_capacity;
        if (!rc) rc = dev_alloc(&ctx->log_action, n);
        if (!rc) rc = dev_alloc(&ctx->log_M, n);
        if (!rc) rc = dev_alloc(&ctx->log_lp, n);
        if (!rc) rc = dev_alloc(&ctx->log_p, n);
        if (!rc) rc = dev_alloc(&ctx->log_w, n);
    }
    if (rc) return fail_free(rc);
    std::vector<uint32_t> cid((size_t)C);
    for (int64_t c = 0; c < C; ++c) cid[c] = o->chain_id_base + (uint32_t)c;
    std::vector<int64_t> Lv((size_t)C, o->L0), zeros((size_t)C * 2, 0);
    hipError_t e = hipMemcpy(ctx->chain_id, cid.data(), C * sizeof(uint32_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->x, x0.data(), x0.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->L, Lv.data(), C * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->set, zeros.data(), C * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->step, zeros.data(), C * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(ctx->counters, zeros.data(), C * 2 * sizeof(int64_t), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(ctx->sums, 0, (size_t)C * ns * sizeof(double));
    if (e == hipSuccess) e = launch_cont(ctx->args(0), true, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) return fail_free(hip_fail(e, "continuous sampler set-up"));
    *out = ctx;
    return PNS_OK;
}

int pns_cont_run(pns_cont* ctx, int64_t steps)
{
    g_error.clear();
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    if (steps < 0) return fail(PNS_EINVAL, "steps must be >= 0");
    for (int64_t done = 0; done < steps;) {
        const int64_t n = std::min(kContChunk, steps - done);
        hipError_t e = launch_cont(ctx->args(n), false, ctx->stream);
        if (e != hipSuccess) return hip_fail(e, "continuous step kernel launch");
        done += n;
    }
    return PNS_OK;
}

int pns_cont_read(pns_cont* ctx, double* states, double* log_density, int64_t* L, int64_t* set_index, int64_t* step)
{
    g_error.clear();
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(ctx->stream), "stream synchronize");
    const size_t C = (size_t)ctx->C;
    int rc = PNS_OK;
    auto out64 = [&](void* dst, const void* src, size_t count) {
        std::vector<int64_t> v;
        int r = d2h(v, src, count);
        return r ? r : copy_out(dst, v.data(), count * 8);
    };
    if (states && (rc = out64(states, ctx->x, C * ctx->dim))) return rc;
    if (log_density && (rc = out64(log_density, ctx->lpx, C))) return rc;
    if (L && (rc = out64(L, ctx->L, C))) return rc;
    if (set_index && (rc = out64(set_index, ctx->set, C))) return rc;
    if (step && (rc = out64(step, ctx->step, C))) return rc;
    return PNS_OK;
}

int pns_cont_read_log(pns_cont* ctx, int32_t* actions, int64_t* multiplicities, double* log_density, double* p,
                      double* weights)
{
    g_error.clear();
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    if (ctx->o.log_capacity == 0) return fail(PNS_EINVAL, "the per-step log is off (log_capacity = 0)");
    HIP_TRY(hipStreamSynchronize(ctx->stream), "stream synchronize");
    const size_t n = (size_t)ctx->C * (size_t)ctx->o.log_capacity;
    int rc = PNS_OK;
    if (actions) {
        std::vector<int32_t> v;
        if ((rc = d2h(v, ctx->log_action, n)) || (rc = copy_out(actions, v.data(), n * 4))) return rc;
    }
    auto out64 = [&](void* dst, const void* src) {
        std::vector<int64_t> v;
        int r = d2h(v, src, n);
        return r ? r : copy_out(dst, v.data(), n * 8);
    };
    if (multiplicities && (rc = out64(multiplicities, ctx->log_M))) return rc;
    if (log_density && (rc = out64(log_density, ctx->log_lp))) return rc;
    if (p && (rc = out64(p, ctx->log_p))) return rc;
    if (weights && (rc = out64(weights, ctx->log_w))) return rc;
    return PNS_OK;
}

int pns_cont_read_sums(pns_cont* ctx, double* sums)
{
    g_error.clear();
    if (!ctx || !sums) return fail(PNS_EINVAL, "NULL argument");
    HIP_TRY(hipStreamSynchronize(ctx->stream), "stream synchronize");
    const size_t n = (size_t)ctx->C * cont_sums_count(ctx);
    std::vector<double> v;
    int rc = d2h(v, ctx->sums, n);
    return rc ? rc : copy_out(sums, v.data(), n * 8);
}

int pns_cont_clear_sums(pns_cont* ctx)
{
    g_error.clear();
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    hipError_t e = launch_fill64(ctx->sums, (int64_t)ctx->C * cont_sums_count(ctx), 0, ctx->stream);
    if (e != hipSuccess) return hip_fail(e, "clear sums");
    return PNS_OK;
}

int pns_cont_stats(pns_cont* ctx, int64_t* jumps, int64_t* stays)
{
    g_error.clear();
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(ctx->stream), "stream synchronize");
    std::vector<int64_t> v;
    int rc = d2h(v, ctx->counters, (size_t)ctx->C * 2);
    if (rc) return rc;
    std::vector<int64_t> j((size_t)ctx->C), s((size_t)ctx->C);
    for (int32_t c = 0; c < ctx->C; ++c) {
        j[c] = v[(size_t)c * 2];
        s[c] = v[(size_t)c * 2 + 1];
    }
    if (jumps && (rc = copy_out(jumps, j.data(), j.size() * 8))) return rc;
    if (stays && (rc = copy_out(stays, s.data(), s.size() * 8))) return rc;
    return PNS_OK;
}

int pns_cont_sync(pns_cont* ctx)
{
    g_error.clear();
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    HIP_TRY(hipStreamSynchronize(ctx->stream), "stream synchronize");
    HIP_TRY(hipGetLastError(), "queued work");
    return PNS_OK;
}

int pns_cont_destroy(pns_cont* ctx)
{
    if (!ctx) return PNS_OK;
    (void)hipStreamSynchronize(ctx->stream);
    ctx->free_all();
    delete ctx;
    return PNS_OK;
}

}  // extern "C"
