// C-ABI runtime of the Partial Neighbor Search sampler (see include/pns.h).
//
// Owns the device memory of a sampler context, prepares the coefficient
// matrix (zero-diagonal off-diagonal part A with a padded pitch, diagonal
// split off, symmetry and field-bound checks), chooses the workgroup tile,
// queues the step kernels in the plain, persistent or HIP-graph form, and
// copies results out to host or device buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
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

#define HIP_TRY(call, what)                       \
    do {                                          \
        hipError_t e_ = (call);                   \
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

struct Tile {
    int32_t block, groups;
};

// Tile table: smallest capacity (block * 4 * groups) covering N.
Tile default_tile(int32_t N)
{
    if (N <= 256) return {64, 1};
    if (N <= 1024) return {256, 1};
    if (N <= 2048) return {256, 2};
    if (N <= 4096) return {512, 2};
    if (N <= 8192) return {512, 4};
    return {1024, 4};
}

}  // namespace

struct pns_ctx {
    int32_t N = 0, n = 0, mode = 0, qtype = 0, htype = 0, layout = 0;
    int32_t num_chains = 0;
    int32_t block = 0, groups = 0;
    int64_t pitch = 0;
    int32_t launch = PNS_LAUNCH_PERSISTENT;
    int32_t chunk = 0;
    uint64_t seed = 0;
    int64_t L0 = 100;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t dyn_lds = 0;
    // device memory
    void* A = nullptr;
    void* diag = nullptr;
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
    unsigned long long* hist_w = nullptr;
    unsigned long long* hist_v = nullptr;
    int32_t snap_every = 0, snap_cap = 0;
    uint8_t* snap_x = nullptr;
    int64_t* snap_M = nullptr;
    int64_t* snap_E = nullptr;
    int32_t* snap_count = nullptr;
    // graph cache
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    int64_t graph_steps = -1;

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
        a.log_cap = log_cap;
        a.hist_w = hist_w;
        a.hist_v = hist_v;
        a.snap_every = snap_every;
        a.snap_cap = snap_cap;
        a.snap_x = snap_x;
        a.snap_M = snap_M;
        a.snap_E = snap_E;
        a.snap_count = snap_count;
        a.snap_pitch = pitch;
        return a;
    }

    // How the step kernel forms the subset: 0 every bit, 1 systematic window,
    // 2 random subset drawn in LDS, 3 systematic window that reaches at most
    // one 4-bit group of any lane (weights kept for that group only).
    int32_t flavour() const
    {
        if (mode == PNS_MODE_RF) return 0;
        if (mode == PNS_MODE_BASIC) return n < N ? 2 : 0;
        if (mode == PNS_MODE_UNBIASED_SYS || n >= N) return window_compact_ok(N, n, block, groups) ? 3 : 1;
        return 2;
    }

    // True if no window of n cyclically consecutive bits holds bits of two
    // different 4-bit groups within one wave: the wave's lanes of group g
    // hold the contiguous range [(g*block + 64w)*4, +256) of bits.
    static bool window_compact_ok(int32_t N, int32_t n, int32_t block, int32_t groups)
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

    bool instrumented() const { return log_cap > 0 || hist_w != nullptr || snap_every > 0; }

    int launch_chunk(int64_t steps)
    {
        // host-side check that the launch matches what the kernel assumes
        if ((int64_t)block * 4 * groups < N || num_chains < 1 || !have_tile(qtype, htype, block, groups))
            return fail(PNS_EINVAL, "tile %dx%d does not cover N=%d", block, groups, N);
        const int32_t flav = flavour();
        const size_t dyn = flav == 2 ? (size_t)pitch * 4 : flav == 3 ? (size_t)pitch * 4 : 0;
        hipError_t e = launch_steps(qtype, htype, flav, instrumented(), block, groups, num_chains, dyn, stream,
                                    args(steps));
        if (e != hipSuccess) return hip_fail(e, "step kernel launch");
        return PNS_OK;
    }

    void free_all()
    {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        void* ptrs[] = {A, diag, problems, chain_problem, foff, beta, chain_id, x, h, rmem, E, L, sub, step,
                        last_action, last_M, last_E, counters, log_action, log_M, log_E, log_p, hist_w, hist_v,
                        snap_x, snap_M, snap_E, snap_count};
        for (void* p : ptrs)
            if (p) (void)hipFree(p);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

namespace {

size_t qsize(int32_t qtype) { return qtype == Q_I16 ? 2 : 4; }

// Build the zero-diagonal off-diagonal matrix A (pitch-padded) and the
// diagonal from the caller's Q, and bound the fields.
template <typename QT>
int prepare_matrix(const QT* Q, int32_t N, int32_t layout, int64_t pitch, std::vector<QT>& A,
                   std::vector<uint8_t>& diag_bytes, double* field_bound, double* diag_bound)
{
    A.assign((size_t)N * pitch, (QT)0);
    using DW = typename std::conditional<std::is_same<QT, float>::value, float, int32_t>::type;
    std::vector<DW> d((size_t)pitch, (DW)0);
    double fb = 0.0, db = 0.0;
    for (int32_t i = 0; i < N; ++i) {
        double rowsum = 0.0;
        for (int32_t j = 0; j < N; ++j) {
            QT v;
            if (i == j) {
                d[i] = (DW)Q[(size_t)i * N + i];
                db = std::max(db, std::fabs((double)d[i]));
                continue;
            }
            if (layout == PNS_SYMMETRIC) {
                v = Q[(size_t)i * N + j];
                if (!(v == Q[(size_t)j * N + i]))
                    return fail(PNS_EINVAL, "SYMMETRIC Q is not symmetric at (%d, %d)", i, j);
            } else {
                v = i < j ? Q[(size_t)i * N + j] : Q[(size_t)j * N + i];
            }
            if (std::is_same<QT, float>::value && !std::isfinite((double)v))
                return fail(PNS_EINVAL, "Q has a non-finite entry at (%d, %d)", i, j);
            A[(size_t)i * pitch + j] = v;
            rowsum += std::fabs((double)v);
        }
        fb = std::max(fb, rowsum);
    }
    diag_bytes.resize(d.size() * sizeof(DW));
    std::memcpy(diag_bytes.data(), d.data(), diag_bytes.size());
    *field_bound = fb;
    *diag_bound = db;
    return PNS_OK;
}

int check_opts(const pns_opts* o)
{
    for (int i = 0; i < 8; ++i)
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

}  // namespace

namespace {

template <typename T>
int d2h(std::vector<T>& v, const void* src, size_t count)
{
    v.resize(count);
    if (count == 0) return PNS_OK;
    HIP_TRY(hipMemcpy(v.data(), src, count * sizeof(T), hipMemcpyDeviceToHost), "download");
    return PNS_OK;
}

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

int compact_states(const pns_ctx* ctx, const std::vector<uint8_t>& xp, std::vector<uint8_t>& xs)
{
    const int64_t C = ctx->num_chains;
    xs.resize((size_t)C * ctx->N);
    for (int64_t c = 0; c < C; ++c) std::memcpy(&xs[c * ctx->N], &xp[c * ctx->pitch], ctx->N);
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

const char* pns_version(void) { return "0.1.0"; }

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
    if (mode < PNS_MODE_RF || mode > PNS_MODE_UNBIASED_RAND) return fail(PNS_EINVAL, "unknown mode %d", mode);
    const int32_t n = mode == PNS_MODE_RF ? N : subset_size;
    if (n < 1 || n > N) return fail(PNS_EINVAL, "subset size %d outside [1, %d]", subset_size, N);
    if (o.hist && N > 24) return fail(PNS_EINVAL, "histograms need N <= 24");
    std::vector<double> betas((size_t)o.num_chains, beta);
    if (o.betas) {
        for (int32_t c = 0; c < o.num_chains; ++c) betas[c] = o.betas[c];
    }
    for (double b : betas)
        if (!(b >= 0.0) || !std::isfinite(b)) return fail(PNS_EINVAL, "beta must be finite and >= 0");
    const Tile def = default_tile(N);
    Tile tile = def;
    if (o.block > 0 || o.groups > 0) {
        tile.block = o.block > 0 ? o.block : def.block;
        tile.groups = o.groups > 0 ? o.groups : std::max<int32_t>(1, (int32_t)((N + tile.block * 4 - 1) / (tile.block * 4)));
    }
    if ((int64_t)tile.block * 4 * tile.groups < N) {
        if (N > 16384) return fail(PNS_EUNSUPPORTED, "N=%d exceeds the largest tile (16384)", N);
        return fail(PNS_EINVAL, "tile %dx%d cannot hold N=%d", tile.block, tile.groups, N);
    }

    const int32_t qtype = o.dtype;
    const int64_t pitch = round_up(N, 64);
    const size_t qbytes = (size_t)N * N * qsize(qtype);

    // caller's Q into host memory
    std::vector<uint8_t> qhost(qbytes);
    rc = copy_in(qhost.data(), Q, qbytes);
    if (rc) return rc;

    std::vector<uint8_t> Abytes, dbytes;
    double fbound = 0.0, dbound = 0.0;
    if (qtype == Q_I16) {
        std::vector<int16_t> A;
        rc = prepare_matrix(reinterpret_cast<const int16_t*>(qhost.data()), N, o.layout, pitch, A, dbytes, &fbound, &dbound);
        if (rc) return rc;
        Abytes.resize(A.size() * 2);
        std::memcpy(Abytes.data(), A.data(), Abytes.size());
    } else if (qtype == Q_I32) {
        std::vector<int32_t> A;
        rc = prepare_matrix(reinterpret_cast<const int32_t*>(qhost.data()), N, o.layout, pitch, A, dbytes, &fbound, &dbound);
        if (rc) return rc;
        Abytes.resize(A.size() * 4);
        std::memcpy(Abytes.data(), A.data(), Abytes.size());
    } else {
        std::vector<float> A;
        rc = prepare_matrix(reinterpret_cast<const float*>(qhost.data()), N, o.layout, pitch, A, dbytes, &fbound, &dbound);
        if (rc) return rc;
        Abytes.resize(A.size() * 4);
        std::memcpy(Abytes.data(), A.data(), Abytes.size());
    }
    qhost.clear();
    qhost.shrink_to_fit();
    const int32_t s = o.layout == PNS_SYMMETRIC ? 2 : 1;
    int32_t htype;
    if (qtype == Q_F32) {
        htype = H_F64;
    } else {
        const double ebound = dbound + s * fbound;
        if (ebound * (double)N > 9.0e18) return fail(PNS_EINVAL, "energy bound of Q overflows int64");
        htype = (fbound < 2147483647.0 && ebound < 2147483647.0) ? H_I32 : H_I64;
        if (qtype == Q_I16) htype = H_I32;
    }
    if (!have_tile(qtype, htype, tile.block, tile.groups))
        return fail(PNS_EINVAL, "no kernel for tile %dx%d", tile.block, tile.groups);

    pns_ctx* ctx = new pns_ctx();
    ctx->N = N;
    ctx->n = n;
    ctx->mode = mode;
    ctx->qtype = qtype;
    ctx->htype = htype;
    ctx->layout = o.layout;
    ctx->num_chains = o.num_chains;
    ctx->block = tile.block;
    ctx->groups = tile.groups;
    ctx->pitch = pitch;
    ctx->launch = o.launch;
    ctx->chunk = o.chunk;
    ctx->seed = o.seed;
    ctx->L0 = o.L0;
    ctx->dyn_lds = ((mode == PNS_MODE_BASIC || mode == PNS_MODE_UNBIASED_RAND) && n < N) ? (size_t)pitch * 4 : 0;
    if (o.stream) {
        ctx->stream = reinterpret_cast<hipStream_t>(o.stream);
    } else {
        hipError_t e = hipStreamCreate(&ctx->stream);
        if (e != hipSuccess) {
            delete ctx;
            return hip_fail(e, "hipStreamCreate");
        }
        ctx->own_stream = true;
    }
    const int64_t C = o.num_chains;
    const size_t hbytes = htype == H_I32 ? 4 : 8;
    const size_t fields = (size_t)C * pitch;
#define ALLOC(ptr, type, count)                                   \
    do {                                                          \
        int r_ = dev_alloc(reinterpret_cast<type**>(&ptr), count); \
        if (r_) {                                                 \
            ctx->free_all();                                      \
            delete ctx;                                           \
            return r_;                                            \
        }                                                         \
    } while (0)
    ALLOC(ctx->A, uint8_t, Abytes.size());
    ALLOC(ctx->diag, uint8_t, dbytes.size());
    ALLOC(ctx->problems, Problem, 1);
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
    if (mode == PNS_MODE_UNBIASED_RAND) ALLOC(ctx->rmem, uint8_t, fields);
    if (o.log_capacity > 0) {
        ctx->log_cap = o.log_capacity;
        ALLOC(ctx->log_action, int32_t, (size_t)C * o.log_capacity);
        ALLOC(ctx->log_M, int64_t, (size_t)C * o.log_capacity);
        ALLOC(ctx->log_E, int64_t, (size_t)C * o.log_capacity);
        ALLOC(ctx->log_p, double, (size_t)C * o.log_capacity);
    }
    if (o.hist) {
        ALLOC(ctx->hist_w, unsigned long long, (size_t)1 << N);
        ALLOC(ctx->hist_v, unsigned long long, (size_t)1 << N);
    }
    if (o.snapshot_every > 0) {
        ctx->snap_every = o.snapshot_every;
        ctx->snap_cap = o.snapshot_capacity;
        ALLOC(ctx->snap_x, uint8_t, (size_t)C * o.snapshot_capacity * pitch);
        ALLOC(ctx->snap_M, int64_t, (size_t)C * o.snapshot_capacity);
        ALLOC(ctx->snap_E, int64_t, (size_t)C * o.snapshot_capacity);
        ALLOC(ctx->snap_count, int32_t, C);
    }
#undef ALLOC

    // host-side tables
    Problem P{};
    P.A = ctx->A;
    P.diag = ctx->diag;
    P.pitch = pitch;
    P.num_sets = N / gcd64(N, n);
    P.L0 = o.L0;
    P.N = N;
    P.n = n;
    P.s = s;
    P.qtype = qtype;
    std::vector<int32_t> cp((size_t)C, 0);
    std::vector<int64_t> fo((size_t)C);
    std::vector<uint32_t> cidv((size_t)C);
    for (int64_t c = 0; c < C; ++c) {
        fo[c] = c * pitch;
        cidv[c] = o.chain_id_base + (uint32_t)c;
    }
    std::vector<int64_t> Lv((size_t)C, o.L0), zeros64((size_t)C * 6, 0);
    std::vector<int32_t> la((size_t)C, PNS_STAY);
    auto fail_free = [&](int r) {
        ctx->free_all();
        delete ctx;
        return r;
    };
#define H2D(dst, src, bytes)                                                                   \
    do {                                                                                       \
        hipError_t e_ = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);                      \
        if (e_ != hipSuccess) return fail_free(hip_fail(e_, "upload"));                        \
    } while (0)
    H2D(ctx->A, Abytes.data(), Abytes.size());
    H2D(ctx->diag, dbytes.data(), dbytes.size());
    H2D(ctx->problems, &P, sizeof(P));
    H2D(ctx->chain_problem, cp.data(), C * sizeof(int32_t));
    H2D(ctx->foff, fo.data(), C * sizeof(int64_t));
    H2D(ctx->beta, betas.data(), C * sizeof(double));
    H2D(ctx->chain_id, cidv.data(), C * sizeof(uint32_t));
    H2D(ctx->L, Lv.data(), C * sizeof(int64_t));
    H2D(ctx->sub, zeros64.data(), C * sizeof(int64_t));
    H2D(ctx->step, zeros64.data(), C * sizeof(int64_t));
    H2D(ctx->last_action, la.data(), C * sizeof(int32_t));
    H2D(ctx->last_M, zeros64.data(), C * sizeof(int64_t));
    H2D(ctx->counters, zeros64.data(), C * 6 * sizeof(int64_t));
    if (ctx->snap_count) H2D(ctx->snap_count, zeros64.data(), C * sizeof(int32_t));
    if (ctx->hist_w) {
        hipError_t e1 = hipMemset(ctx->hist_w, 0, sizeof(unsigned long long) << N);
        hipError_t e2 = hipMemset(ctx->hist_v, 0, sizeof(unsigned long long) << N);
        if (e1 != hipSuccess || e2 != hipSuccess) return fail_free(hip_fail(e1 != hipSuccess ? e1 : e2, "hipMemset"));
    }
    if (ctx->rmem) {
        hipError_t e1 = hipMemset(ctx->rmem, 0, fields);
        if (e1 != hipSuccess) return fail_free(hip_fail(e1, "hipMemset"));
    }

    // initial state
    hipError_t e;
    if (o.init == PNS_INIT_GIVEN) {
        std::vector<uint8_t> x0((size_t)C * N), xp(fields, 0);
        rc = copy_in(x0.data(), o.x0, x0.size());
        if (rc) return fail_free(rc);
        for (int64_t c = 0; c < C; ++c)
            for (int32_t j = 0; j < N; ++j) xp[c * pitch + j] = x0[c * N + j] ? 1 : 0;
        H2D(ctx->x, xp.data(), fields);
    } else if (o.init == PNS_INIT_ZERO) {
        if ((e = hipMemset(ctx->x, 0, fields)) != hipSuccess) return fail_free(hip_fail(e, "hipMemset"));
    }
#undef H2D
    if (o.init == PNS_INIT_ZERO) {
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
        e = launch_init_with_map(qtype, htype, (int32_t)pitch, ctx->stream, ia, cp.data());
        if (e != hipSuccess) return fail_free(hip_fail(e, "init kernels"));
    }
    if ((e = hipDeviceSynchronize()) != hipSuccess) return fail_free(hip_fail(e, "create synchronize"));
    *out = ctx;
    return PNS_OK;
}

int pns_run(pns_ctx* ctx, int64_t steps)
{
    g_error.clear();
    if (!ctx) return fail(PNS_EINVAL, "ctx is NULL");
    if (steps < 0) return fail(PNS_EINVAL, "steps must be >= 0");
    if (steps == 0) return PNS_OK;
    if (ctx->launch == PNS_LAUNCH_PLAIN) {
        for (int64_t s = 0; s < steps; ++s) {
            int rc = ctx->launch_chunk(1);
            if (rc) return rc;
        }
        return PNS_OK;
    }
    const int64_t chunk = ctx->chunk > 0 ? std::min<int64_t>(ctx->chunk, steps) : steps;
    if (ctx->launch == PNS_LAUNCH_PERSISTENT) {
        for (int64_t done = 0; done < steps; done += chunk) {
            int rc = ctx->launch_chunk(std::min(chunk, steps - done));
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
        for (int64_t done = 0; done < steps && rc == PNS_OK; done += chunk) rc = ctx->launch_chunk(std::min(chunk, steps - done));
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
        std::vector<uint8_t> xp, xs;
        std::vector<int32_t> la;
        if ((rc = d2h(xp, ctx->x, (size_t)C * ctx->pitch))) return rc;
        if ((rc = d2h(la, ctx->last_action, C))) return rc;
        compact_states(ctx, xp, xs);
        for (int64_t c = 0; c < C; ++c)
            if (la[c] >= 0) xs[c * ctx->N + la[c]] ^= 1u;  // the record's state is before the last move
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
    if (block) *block = ctx->block;
    if (groups) *groups = ctx->groups;
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
        std::vector<uint8_t> xp, xs;
        if ((rc = d2h(xp, ctx->x, (size_t)C * ctx->pitch))) return rc;
        compact_states(ctx, xp, xs);
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
        std::vector<uint8_t> hp, hs((size_t)C * ctx->N * hb);
        if ((rc = d2h(hp, ctx->h, (size_t)C * ctx->pitch * hb))) return rc;
        for (int64_t c = 0; c < C; ++c) std::memcpy(&hs[c * ctx->N * hb], &hp[c * ctx->pitch * hb], ctx->N * hb);
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
    const size_t cnt = (size_t)1 << ctx->N;
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
    const int64_t cnt = (int64_t)1 << ctx->N;
    hipError_t e = launch_fill64(ctx->hist_w, cnt, 0, ctx->stream);
    if (e == hipSuccess) e = launch_fill64(ctx->hist_v, cnt, 0, ctx->stream);
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
    int32_t stored = S;
    for (int32_t v : cnt) stored = std::min<int32_t>(stored, v);
    if (count) *count = stored;
    if (states) {
        std::vector<uint8_t> xp, xs((size_t)C * S * ctx->N);
        if ((rc = d2h(xp, ctx->snap_x, (size_t)C * S * ctx->pitch))) return rc;
        for (int64_t r = 0; r < C * S; ++r) std::memcpy(&xs[r * ctx->N], &xp[r * ctx->pitch], ctx->N);
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
