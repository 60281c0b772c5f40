// Host side of the C interface in include/ecmg.h: problem validation, the level
// hierarchy resident in HBM, discretisation (Section 2), the Algorithm 4
// driver, and the per-level operators exposed for testing.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "ecmg_internal.h"

using namespace ecmg;

namespace {
thread_local std::string g_thread_error;
}

struct BatchPlan;
struct ecmg_ctx;
static void batch_plan_free(ecmg_ctx *c0, BatchPlan *P);
// generations are unique over all contexts of the process, so a plan never
// matches a context that replaced a destroyed one at the same address
static std::atomic<uint64_t> g_generation{0};

// ---------------------------------------------------------------------------
// Allocation-free reductions (ecmg_norms_noalloc): the block partials, the
// arrival counter and the two totals of the norm kernel live in this
// file-scope device array, one copy per GPU, held until the process ends.
// Host code never passes `scratch` itself (in host code the name is only a
// stand-in, not a device address): ecmg_create looks up each device's address
// once with hipGetSymbolAddress and every later use goes through it.
// ---------------------------------------------------------------------------
constexpr int NOALLOC_BLOCKS = 2048;                       // the norm kernel's most blocks
constexpr size_t NOALLOC_TOTALS = 2 * NOALLOC_BLOCKS;      // doubles: partials, then 2 totals
constexpr size_t NOALLOC_COUNTER = NOALLOC_TOTALS + 32;    // doubles: counter on its own 256-byte line
constexpr size_t NOALLOC_BYTES = 8 * (NOALLOC_COUNTER + 32);
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[NOALLOC_MAX_DEVICES];           // device address of `scratch`, per device

__global__ void k_noalloc_clear(unsigned *counter) {
    if (threadIdx.x == 0) *counter = 0u;
}

struct ecmg_ctx {
    ecmg_options opt{};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // device blocks by size: a set-up of a problem with the grids of the
    // previous one takes its arrays back instead of freeing and allocating
    std::unordered_map<void *, size_t> dsize;   // bytes of every live block
    std::multimap<size_t, void *> bin;          // blocks kept for reuse
    bool recycle = false;                       // dfree keeps blocks in the bin
    // level whose last JCG x update (x += alpha p) is still pending on the
    // device (c->sc, p0 / p1 hold it): a solve with EXP_true fuses the finest
    // level's update into EXP_true; anything else that reads that x or reuses
    // the JCG buffers applies it first (flush_x); -1: none
    int x_pending = -1;
    // set-up scratch (field samples of a slab or face; coordinates passed to
    // device callbacks): grown as needed, kept until the context is destroyed,
    // reused in stream order without host waits or frees
    double *stmp = nullptr, *scoord = nullptr;
    int64_t stmp_n = 0, scoord_n = 0;
    int device = 0;
    rocblas_handle blas = nullptr;            // dense DSOLVE factorisation (lazy)
    // batched solves led by this context: task and scalar arrays for the queue kernel
    PersistentTask *bt_tasks = nullptr;
    JcgScalars *bt_sc = nullptr, *bt_sc_host = nullptr;
    unsigned *bt_next = nullptr;              // queue counter
    unsigned *bt_bar = nullptr;               // 32 barrier words per box (error flag, counter)
    ExpTask *bt_exp = nullptr;                // batched EXP_finite / EXP_true boxes
    int bt_cap = 0;
    struct BatchPlan *bplan = nullptr;        // batched solves led by this context: plan and graph
    uint64_t gen = 0;                         // changes whenever the hierarchy or its JCG configuration does
    std::string err;
    std::vector<Level> lv;
    int nlev = 0;
    int face_type[6] = {};
    bool ready = false;        // setup done
    bool solved = false;       // u of every level available
    // shared JCG scratch, sized for the finest level
    double *r = nullptr, *p0 = nullptr, *p1 = nullptr, *q = nullptr;
    // mixed precision: FP32 work vectors of the inner JCG (finest size) and its scalars
    float *r32 = nullptr, *p32a = nullptr, *p32b = nullptr, *q32 = nullptr, *d32 = nullptr;
    JcgScalars *sc32 = nullptr;
    int64_t scratch_n = 0;
    JcgScalars *sc = nullptr;  // device
    JcgScalars *sc_host = nullptr;  // pinned
    double *partials = nullptr;
    int64_t partials_n = 0;
    unsigned *counters = nullptr;   // [0] stencil, [1] pass B, [2] norms
    double *dres = nullptr;         // device results of reductions [4]
    double *hres = nullptr;         // pinned host copy
    double *hstage = nullptr;       // pinned host staging for callback samples
    double *dstage = nullptr;       // device staging
    int64_t stage_n = 0;
    int KZ = 32;
    int kz_target = 1024;                      // tiled stencil: blocks aimed for per launch
    int fold_max = FOLD_MAX_BLOCKS;            // JCG scalar steps folded into the passes up to this many blocks
    int col_enable = 1;                        // column kernels for init / pass A on unfolded levels
    int64_t gather_max = GATHER_DEFAULT_NODES; // built-in rule: the gather path up to this many nodes
    int col_kz = 16;                           // planes per z-chunk of a column wave
    int col_order = 0;                         // wave order of the column kernels (col_waves)
    uint32_t timing_mask = 0;                  // kernel classes timed with HIP events (bit k = class k)
    // persistent JCG for grids of at most persist_max nodes (larger ones: the
    // tiled passes with folded scalar steps -- two launches per iteration,
    // whose boundaries cost about what one of the persistent kernel's three
    // device-wide barriers per iteration costs)
    int64_t persist_max = 20000;
    // ECMG_MIXED: levels up to this many nodes stay FP64 -- those whose JCG
    // passes fold their scalar steps (pass B of at most FOLD_MAX_BLOCKS blocks
    // of 2,048 nodes), where an iteration waits on launches, not bytes
    int64_t mixed_min = (int64_t)FOLD_MAX_BLOCKS * 2048;
                                               // (an explicit persistent_nodes sets it too)
    int persist_blocks = 0;                    // co-resident workgroups (0 = unavailable)
    int persist_seglen = 0;                    // persistent kernel: nodes per thread along z (0 = by size)
    int persist_nwg = 256;                     // persistent kernel: most workgroups per task
    int queue_blocks = 0;                      // co-resident workgroups of the queue kernel
    int batch_npw = 8192;                      // batched solves: nodes per workgroup of a box
    int batch_seg = 0;                         // batched solves: nodes per segment (0 = by size)
    PersistentTask *d_task = nullptr;          // device copy of one task
    std::string tune_cache;                    // tuning cache path ("" = none)
    std::string device_name;                   // "<arch> <CUs> CUs", recorded with tuning choices
    unsigned *d_bar = nullptr;                 // barrier words + error flag
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // a solve enqueues the levels without waiting for them: per level, its
    // final JCG scalars and persistent task (pinned; the stream copies them
    // when it gets there) and a start / end event pair
    JcgScalars *sc_lv = nullptr;
    JcgScalars *sc_lv_dev = nullptr;           // the same slots as kernels address them
    double *rrt_lv = nullptr;                  // per level ||F - A u||^2 (options.true_residual), pinned
    PersistentTask *task_lv = nullptr;
    int lv_cap = 0;
    std::vector<hipEvent_t> lv_ev;
    // kernel timing (options.timing)
    struct Rec { hipEvent_t a, b; int level, kind, iter; bool ext, valid; };
    std::vector<hipEvent_t> evpool;
    std::vector<Rec> recs;
    size_t evnext = 0;
};

// ---------------------------------------------------------------------------
// error helpers
// ---------------------------------------------------------------------------
static int fail(ecmg_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    g_thread_error = buf;
    return code;
}

#define HIPCHK(c, call)                                                                             \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess)                                                                       \
            return fail((c), ECMG_EDEVICE, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                                  \
    } while (0)

#define CHK(call)                     \
    do {                              \
        int s_ = (call);              \
        if (s_ != ECMG_OK) return s_; \
    } while (0)

static int dalloc(ecmg_ctx *c, void **p, size_t bytes) {
    if (bytes == 0) bytes = 8;
    auto it = c->bin.find(bytes);                // a kept block of this size
    if (it != c->bin.end()) {
        *p = it->second;
        c->bin.erase(it);
        return ECMG_OK;
    }
    if (c->opt.alloc) {                          // the caller's allocator (stream-ordered)
        *p = c->opt.alloc(bytes, (void *)c->stream, c->opt.alloc_user);
        if (!*p) return fail(c, ECMG_ENOMEM, "allocator hook returned NULL for %zu bytes", bytes);
        if ((uintptr_t)*p % 256 != 0) {
            c->opt.free(*p, (void *)c->stream, c->opt.alloc_user);
            *p = nullptr;
            return fail(c, ECMG_EINVAL, "allocator hook returned a pointer not aligned to 256 bytes");
        }
        c->dsize[*p] = bytes;
        return ECMG_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(c, ECMG_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    c->dsize[*p] = bytes;
    return ECMG_OK;
}
template <typename T>
static int dalloc_n(ecmg_ctx *c, T **p, int64_t n) {
    const size_t bytes = sizeof(T) * (size_t)std::max<int64_t>(n, 1);
    int rc = dalloc(c, (void **)p, bytes);
    if (rc != ECMG_OK) return rc;
    // every array starts zeroed (row padding must read as zero); ordered on the
    // library stream, which does not synchronise with the null stream
    if (hipMemsetAsync(*p, 0, bytes, c->stream) != hipSuccess) return fail(c, ECMG_EDEVICE, "hipMemsetAsync failed");
    return ECMG_OK;
}

// dense host node array <-> padded device node array of level geometry g,
// through the dense device buffer `dense` (one contiguous transfer, the row
// padding handled by a pack kernel: a pitched copy with short rows is slow)
static hipError_t copy_in(const Geom &g, double *dev, const double *host, double *dense, hipStream_t s,
                          hipMemcpyKind kind) {
    const hipError_t e = hipMemcpyAsync(dense, host, 8 * (size_t)g.nreal, kind, s);
    if (e != hipSuccess) return e;
    launch_unpack(g, dense, dev, s);
    return hipGetLastError();
}
static hipError_t copy_out(const Geom &g, double *host, const double *dev, double *dense, hipStream_t s) {
    launch_pack(g, dev, dense, s);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return hipMemcpyAsync(host, dense, 8 * (size_t)g.nreal, hipMemcpyDeviceToHost, s);
}
static void dfree(ecmg_ctx *c, void *p) {
    if (!p) return;
    auto it = c->dsize.find(p);
    if (c->recycle && it != c->dsize.end()) {    // kept for the set-up in progress
        c->bin.insert({it->second, p});
        return;
    }
    if (it != c->dsize.end()) c->dsize.erase(it);
    if (c->opt.free) c->opt.free(p, (void *)c->stream, c->opt.alloc_user);
    else (void)hipFree(p);
}

// free the kept blocks
static void bin_flush(ecmg_ctx *c) {
    const bool keep = c->recycle;
    c->recycle = false;
    for (auto &kv : c->bin) dfree(c, kv.second);
    c->bin.clear();
    c->recycle = keep;
}

// ---------------------------------------------------------------------------
// geometry
// ---------------------------------------------------------------------------
static Geom make_geom(const ecmg_problem *p, int l, double lo[3]) {
    Geom g{};
    g.nx = p->n0[0] << l;
    g.ny = p->n0[1] << l;
    g.nz = p->n0[2] << l;
    g.sx = row_pitch(g.nx + 1);
    g.sy = g.ny + 1;
    g.nnodes = (int64_t)g.sx * g.sy * (g.nz + 1);
    g.nreal = (int64_t)(g.nx + 1) * g.sy * (g.nz + 1);
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int d = 0; d < 3; ++d) {
        g.h[d] = (p->hi[d] - p->lo[d]) / (double)n[d];
        lo[d] = p->lo[d];
    }
    for (int f = 0; f < 6; ++f) g.ft[f] = p->face_type[f];
    // Q1 element stiffness classes: product over axes of 1-D stiffness
    // K1 = (+1 same node, -1 other)/h and 1-D mass M1 = h (1/3 same, 1/6 other),
    // summed over which axis carries the derivative.
    for (int m = 0; m < 8; ++m) {
        double s = 0.0;
        for (int dv = 0; dv < 3; ++dv) {
            double t = 1.0;
            for (int ax = 0; ax < 3; ++ax) {
                const bool other = (m >> ax) & 1;
                if (ax == dv) t *= (other ? -1.0 : 1.0) / g.h[ax];
                else t *= g.h[ax] * (other ? 1.0 / 6.0 : 1.0 / 3.0);
            }
            s += t;
        }
        g.C[m] = s;
    }
    for (int f = 0; f < 6; ++f) {
        const int ax = f / 2;
        const int pax = (ax == 0) ? 1 : 0, qax = (ax == 2) ? 1 : 2;
        const double A = g.h[pax] * g.h[qax];
        g.M[f][0] = A / 9.0;
        g.M[f][1] = A / 18.0;
        g.M[f][2] = A / 36.0;
    }
    return g;
}

static void face_axes_h(int f, int &p, int &q) {
    const int ax = f / 2;
    p = (ax == 0) ? 1 : 0;
    q = (ax == 2) ? 1 : 2;
}

// coordinates of the sampling sets along axis d of a level
static std::vector<double> node_coords(const Geom &g, const double lo[3], int d) {
    const int n[3] = {g.nx, g.ny, g.nz};
    std::vector<double> v(n[d] + 1);
    for (int i = 0; i <= n[d]; ++i) v[i] = lo[d] + (double)i * g.h[d];
    return v;
}
static std::vector<double> centroid_coords(const Geom &g, const double lo[3], int d) {
    const int n[3] = {g.nx, g.ny, g.nz};
    std::vector<double> v(n[d]);
    for (int i = 0; i < n[d]; ++i) v[i] = lo[d] + ((double)i + 0.5) * g.h[d];
    return v;
}
// two Gauss-Legendre points per element: origin + (1 -/+ 1/sqrt3) h/2
static std::vector<double> gauss_coords(const Geom &g, const double lo[3], int d) {
    const int n[3] = {g.nx, g.ny, g.nz};
    const double G = 1.0 / std::sqrt(3.0);
    std::vector<double> v(2 * (size_t)n[d]);
    for (int i = 0; i < n[d]; ++i) {
        const double e0 = lo[d] + (double)i * g.h[d];
        v[2 * i] = e0 + (1.0 - G) * g.h[d] / 2.0;
        v[2 * i + 1] = e0 + (1.0 + G) * g.h[d] / 2.0;
    }
    return v;
}

// ---------------------------------------------------------------------------
// field sampling: evaluates `fld` on x (fastest) by y by z into device memory
// `dout`, validating host samples.  check: 0 finite, 1 > 0, 2 >= 0.
// ---------------------------------------------------------------------------
static int ensure_stage(ecmg_ctx *c, int64_t n) {
    if (n <= c->stage_n) return ECMG_OK;
    if (c->hstage) (void)hipHostFree(c->hstage);
    dfree(c, c->dstage);
    c->hstage = nullptr;
    c->dstage = nullptr;
    c->stage_n = 0;
    HIPCHK(c, hipHostMalloc((void **)&c->hstage, sizeof(double) * (size_t)n, hipHostMallocDefault));
    CHK(dalloc_n(c, &c->dstage, n));
    c->stage_n = n;
    return ECMG_OK;
}

// a set-up scratch buffer of at least n doubles (grown: the old one freed)
static int ensure_scratch(ecmg_ctx *c, double **buf, int64_t *cap, int64_t n) {
    if (*cap >= n) return ECMG_OK;
    dfree(c, *buf);
    *buf = nullptr;
    *cap = 0;
    CHK(dalloc(c, (void **)buf, 8 * (size_t)std::max<int64_t>(n, 1)));
    *cap = n;
    return ECMG_OK;
}

static int sample(ecmg_ctx *c, const ecmg_field &fld, const char *name, int face, const std::vector<double> &x,
                  const std::vector<double> &y, const std::vector<double> &z, double *dout, int check) {
    const int64_t n = (int64_t)x.size() * (int64_t)y.size() * (int64_t)z.size();
    if (n == 0) return ECMG_OK;
    if (fld.device) {
        // coordinates in the context's scratch: the callback's work, this copy
        // and the next sample's copy are ordered on the stream, so nothing
        // waits on the host here
        CHK(ensure_scratch(c, &c->scoord, &c->scoord_n, (int64_t)(x.size() + y.size() + z.size())));
        double *dx = c->scoord, *dy = dx + x.size(), *dz = dy + y.size();
        HIPCHK(c, hipMemcpyAsync(dx, x.data(), 8 * x.size(), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(dy, y.data(), 8 * y.size(), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipMemcpyAsync(dz, z.data(), 8 * z.size(), hipMemcpyHostToDevice, c->stream));
        const int rc = fld.device(face, (int64_t)x.size(), (int64_t)y.size(), (int64_t)z.size(), dx, dy, dz, dout,
                                  (void *)c->stream, fld.user);
        if (rc != 0) return fail(c, ECMG_ECALLBACK, "device callback for %s returned %d", name, rc);
        return ECMG_OK;
    }
    if (!fld.host) {
        const double v = fld.value;
        if (!std::isfinite(v) || (check == 1 && !(v > 0)) || (check == 2 && !(v >= 0)))
            return fail(c, ECMG_EINVAL, "invalid constant %s = %g", name, v);
        launch_fill(dout, n, v, c->stream);
        HIPCHK(c, hipGetLastError());
        return ECMG_OK;
    }
    CHK(ensure_stage(c, n));
    HIPCHK(c, hipStreamSynchronize(c->stream));  // staging buffer may still be in use
    const int rc = fld.host(face, (int64_t)x.size(), (int64_t)y.size(), (int64_t)z.size(), x.data(), y.data(),
                            z.data(), c->hstage, fld.user);
    if (rc != 0) return fail(c, ECMG_ECALLBACK, "host callback for %s returned %d", name, rc);
    for (int64_t i = 0; i < n; ++i) {
        const double v = c->hstage[i];
        if (!std::isfinite(v) || (check == 1 && !(v > 0)) || (check == 2 && !(v >= 0)))
            return fail(c, ECMG_EINVAL, "invalid sample of %s: %g at point %lld", name, v, (long long)i);
    }
    HIPCHK(c, hipMemcpyAsync(dout, c->hstage, sizeof(double) * (size_t)n, hipMemcpyHostToDevice, c->stream));
    return ECMG_OK;
}

static const int64_t kBatchPoints = (int64_t)1 << 23;

// ---------------------------------------------------------------------------
// timing records
// ---------------------------------------------------------------------------
static int rec_flush(ecmg_ctx *c, int iter_limit);
thread_local ecmg::PendingTiming ecmg::g_pending_timing;

constexpr size_t NO_REC = ~(size_t)0;
static int rec_begin(ecmg_ctx *c, int level, int kind, int iter, size_t *slot) {
    *slot = NO_REC;
    if (!((c->timing_mask >> kind) & 1u)) return ECMG_OK;
    // bound the pending records (a long run of calls that never reach a
    // solve's final wait or a kernel-time query)
    if (c->recs.size() >= 65536) CHK(rec_flush(c, 1 << 30));
    if (c->evnext + 2 > c->evpool.size()) {
        for (int t = 0; t < 256; ++t) {
            hipEvent_t e;
            HIPCHK(c, hipEventCreate(&e));
            c->evpool.push_back(e);
        }
    }
    // the kernel's own start and end through the extended launch; the
    // cooperative launch of the persistent kernel (class 7) between markers
    const bool ext = kind != 7;
    ecmg_ctx::Rec r{c->evpool[c->evnext], c->evpool[c->evnext + 1], level, kind, iter, ext, true};
    c->evnext += 2;
    if (ext) g_pending_timing = PendingTiming{r.a, r.b};
    else HIPCHK(c, hipEventRecord(r.a, c->stream));
    *slot = c->recs.size();
    c->recs.push_back(r);
    return ECMG_OK;
}
static int rec_end(ecmg_ctx *c, size_t slot) {
    if (slot == NO_REC) return ECMG_OK;
    ecmg_ctx::Rec &r = c->recs[slot];
    if (!r.ext) {
        HIPCHK(c, hipEventRecord(r.b, c->stream));
    } else if (g_pending_timing.start || g_pending_timing.stop) {
        // nothing was launched, or a timed group without its last launch: no record
        g_pending_timing = PendingTiming{};
        r.valid = false;
    }
    return ECMG_OK;
}
// Fold the finished records.  A JCG pass launch (classes 0, 1, 5, 6) whose
// iteration index is at or beyond its level's limit (the iterations the level
// ran) found the `done` flag set and did no work; it is not counted.
static bool rec_is_pass(int kind) {
    return kind == 0 || kind == 1 || kind == 5 || kind == 6 || kind == 10 || kind == 11 || kind == 12;
}
static int rec_flush_levels(ecmg_ctx *c, const std::vector<int> &limit) {
    if (c->recs.empty()) return ECMG_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (auto &r : c->recs) {
        const int lim = r.level < (int)limit.size() ? limit[r.level] : 0;
        if (!r.valid || (rec_is_pass(r.kind) && r.iter >= lim)) continue;
        float ms = 0.f;
        HIPCHK(c, hipEventElapsedTime(&ms, r.a, r.b));
        c->lv[r.level].kt_ms[r.kind] += ms;
        c->lv[r.level].kt_n[r.kind] += 1;
    }
    c->recs.clear();
    c->evnext = 0;
    return ECMG_OK;
}
// the same with one limit for every level
static int rec_flush(ecmg_ctx *c, int iter_limit) {
    return rec_flush_levels(c, std::vector<int>(std::max(c->nlev, 1), iter_limit));
}

static int apply_tune_cache(ecmg_ctx *c);
static int dense_prepare(ecmg_ctx *c, int l);
static int ensure_partials(ecmg_ctx *c, int64_t n);

// ---------------------------------------------------------------------------
// JCG on one level (the JCG loop of Algorithm 4)
// ---------------------------------------------------------------------------
static StencilArgs<double> stencil_args(ecmg_ctx *c, Level &L) {
    StencilArgs<double> a{};
    a.g = L.g;
    a.KZ = (L.tune_path == 0 && L.tune_kz > 0) ? std::min(L.tune_kz, L.g.nz + 1) : stencil_kz(L.g, c->KZ, c->kz_target);
    stencil_blocks(L.g, a.KZ, &a.ntx, &a.nty, &a.nkz);
    a.beta = L.beta;
    for (int f = 0; f < 6; ++f) a.alpha[f] = L.alpha[f];
    a.dinv = L.dinv;
    a.F = L.F;
    a.sc = c->sc;
    a.partials = c->partials;
    return a;
}

// Enqueue JCG iterations (pass A, pass B) in chunks until the device sets
// `done`, with one status read after each chunk.  The first chunk follows the
// init pass without a status read (if init already met the tolerance its
// launches return at once); it is `hint` iterations (the count the level needed
// last time, so a repeated solve usually needs one status read) or 2; later
// chunks double from 2 up to 64.  Fixed-iteration mode enqueues all iterations
// at once.  Leaves the final scalars in c->sc_host.  kind_a / kind_b name the
// timing classes.  nowait: the first chunk only, with no status read (the
// caller checks `done` once the stream has run it).
template <typename T>
static int jcg_chunks(ecmg_ctx *c, int l, const StencilArgs<T> &a, const PassBArgs<T> &b, JcgScalars *sc,
                      int fixed, int kind_a, int kind_b, int hint, bool nowait = false, const ColArgs *col = nullptr,
                      int col_waves_n = 0) {
    int done_iters = 0;
    int next = 2;
    int chunk = c->opt.chunk > 0 ? c->opt.chunk : (hint > 0 ? hint : 2);
    if (fixed >= 0) chunk = std::max(fixed, 1);
    size_t slot = 0;
    for (bool first = true;; first = false) {
        if (!first) {
            HIPCHK(c, hipMemcpyAsync(c->sc_host, sc, sizeof(JcgScalars), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            if (c->sc_host->done) break;
            done_iters = c->sc_host->iter;
            if (c->opt.chunk <= 0 && fixed < 0) {
                chunk = next;
                next = std::min(next * 2, 64);
            }
        }
        for (int t = 0; t < chunk; ++t) {
            // iteration 0 from the p_0 init stored, when it did (its own timing class)
            const bool a0 = a.p_init && done_iters + t == 0;
            CHK(rec_begin(c, l, a0 ? 10 : col ? 11 : kind_a, done_iters + t, &slot));
            if (col) {
                // column levels: iteration 0 reads the p_0 init stored; later
                // iterations form p (and the x update) node-wise first, then
                // the column stencil reads it from the buffer of the
                // iteration's parity
                if constexpr (std::is_same<T, double>::value) {
                    if (!a0) launch_p_update(a.g, a.dinv, a.r, a.p0, a.p1, a.x, sc, c->stream);
                }
                if (launch_col(MODE_PASSA0, *col, c->stream) < 0)
                    return fail(c, ECMG_EINVAL, "column wave grid mismatch");
                CHK(rec_end(c, slot));
                launch_stencil_finish(MODE_PASSA, sc, col->partials, col_waves_n, c->stream);
            } else {
                launch_stencil<T>(a0 ? MODE_PASSA0 : MODE_PASSA, a, c->stream);
                CHK(rec_end(c, slot));
            }
            // the last pass B of a speculative FP64 chunk stores no r (see
            // PassBArgs::last): its own timing class
            PassBArgs<T> bt = b;
            bt.last = nowait && kind_b == 1 && t == chunk - 1;
            CHK(rec_begin(c, l, bt.last ? 12 : kind_b, done_iters + t, &slot));
            launch_passB<T>(bt, c->stream);
            CHK(rec_end(c, slot));
        }
        HIPCHK(c, hipGetLastError());
        if (nowait) break;
    }
    return ECMG_OK;
}

// The same with folded scalars (no finishing kernels): the launches form the
// sequence A0 B0 A1 B1 ..., each with its iteration index, and every chunk ends
// on a pass A, which takes the stop test of the pass B before it.  Pass A sums
// init's partials (nb_init pairs) at iteration 0 and pass B's after.
static int jcg_chunks_folded(ecmg_ctx *c, int l, StencilArgs<double> a, PassBArgs<double> b, int fixed, int hint,
                             int nb_init, int nb_b, bool nowait) {
    int next = 2;
    int chunk = c->opt.chunk > 0 ? c->opt.chunk : (hint > 0 ? hint : 2);
    if (fixed >= 0) chunk = std::max(fixed, 1);
    int64_t seq = 0;                     // next launch: even = pass A of seq / 2, odd = pass B
    size_t slot = 0;
    for (bool first = true;; first = false) {
        if (!first) {
            HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(JcgScalars), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            if (c->sc_host->done) break;
            if (c->opt.chunk <= 0 && fixed < 0) {
                chunk = next;
                next = std::min(next * 2, 64);
            }
        }
        const int64_t last = 2 * (seq / 2 + chunk);
        for (; seq <= last; ++seq) {
            const int it = (int)(seq / 2);
            if ((seq & 1) == 0) {
                a.it = it;
                a.fold_nb = it == 0 ? nb_init : nb_b;
                const bool a0 = a.p_init && it == 0;
                CHK(rec_begin(c, l, a0 ? 10 : 0, it, &slot));
                launch_stencil<double>(a0 ? MODE_PASSA0 : MODE_PASSA, a, c->stream);
            } else {
                b.it = it;
                CHK(rec_begin(c, l, 1, it, &slot));
                launch_passB<double>(b, c->stream);
            }
            CHK(rec_end(c, slot));
        }
        HIPCHK(c, hipGetLastError());
        if (nowait) break;
    }
    return ECMG_OK;
}

// The gather levels (folded scalars, one thread per node for the stencils):
// each iteration is the node-wise p update with the scalar step of the pass
// before (U), the gather stencil (G) and pass B; the launches form U0 G0 B0
// U1 G1 B1 ..., each with its iteration index, and every chunk ends on a U G
// pair, whose U takes the stop test of the pass B before it (as
// jcg_chunks_folded ends on a pass A).  U0 takes init's scalar step (nb_init
// pairs), later U the pass B's (nb_b); pass B sums the gather's p.q pairs.
static int jcg_chunks_gather(ecmg_ctx *c, int l, PUFoldArgs u, const ColArgs &ga, PassBArgs<double> b, int fixed,
                             int hint, int nb_init, int nb_b, bool nowait) {
    int next = 2;
    int chunk = c->opt.chunk > 0 ? c->opt.chunk : (hint > 0 ? hint : 2);
    if (fixed >= 0) chunk = std::max(fixed, 1);
    int64_t seq = 0;                     // next launch: seq % 3 = 0 U, 1 G, 2 B of iteration seq / 3
    size_t slot = 0;
    for (bool first = true;; first = false) {
        if (!first) {
            HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(JcgScalars), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            if (c->sc_host->done) break;
            if (c->opt.chunk <= 0 && fixed < 0) {
                chunk = next;
                next = std::min(next * 2, 64);
            }
        }
        const int64_t last = 3 * (seq / 3 + chunk) + 1;
        for (; seq <= last; ++seq) {
            const int it = (int)(seq / 3);
            const int ph = (int)(seq % 3);
            if (ph == 0) {
                u.it = it;
                u.fold_nb = it == 0 ? nb_init : nb_b;
                // the p update and the stencil timed as one pass A
                CHK(rec_begin(c, l, it == 0 ? 10 : 11, it, &slot));
                launch_p_update_fold(u, c->stream);
            } else if (ph == 1) {
                ColArgs gi = ga;
                gi.it = it;
                launch_gather_a(gi, c->stream);
                CHK(rec_end(c, slot));
            } else {
                b.it = it;
                CHK(rec_begin(c, l, 1, it, &slot));
                launch_passB<double>(b, c->stream);
                CHK(rec_end(c, slot));
            }
        }
        HIPCHK(c, hipGetLastError());
        if (nowait) break;
    }
    return ECMG_OK;
}

// Mixed precision (FP32 stencil and CG vectors, FP64 dot products, FP64
// residual and iterate): iterative refinement around an FP32 JCG.
//   r = F - A x in FP64 (the stop test of Algorithm 4 is taken on it);
//   s = ||r||_2;  FP32 JCG on A d = r / s from d = 0 until its residual is
//   below max(inner_tol, tol / (2 ||r||)) of the start;  x += s d in FP64.
static int run_jcg_mixed(ecmg_ctx *c, int l, double tol_abs, int max_iter, ecmg_level_info *info) {
    Level &L = c->lv[l];
    StencilArgs<double> a = stencil_args(c, L);
    a.v = L.x;
    a.r = c->r;
    StencilArgs<float> a32{};
    a32.g = L.g;
    a32.KZ = a.KZ;
    a32.ntx = a.ntx;
    a32.nty = a.nty;
    a32.nkz = a.nkz;
    a32.beta = L.beta32;
    for (int f = 0; f < 6; ++f) a32.alpha[f] = L.alpha32[f];
    a32.dinv = L.dinv32;
    a32.r = c->r32;
    a32.q = c->q32;
    a32.x = c->d32;
    a32.p0 = c->p32a;
    a32.p1 = c->p32b;
    a32.sc = c->sc32;
    a32.partials = c->partials;
    PassBArgs<float> b32{};
    b32.n = L.g.nnodes;
    b32.r = c->r32;
    b32.q = c->q32;
    b32.dinv = L.dinv32;
    b32.sc = c->sc32;
    b32.partials = c->partials;
    const int max_outer = 100;
    int inner_total = 0, outer = 0, status = ECMG_OK;
    double rn = 0.0;
    size_t slot = 0;
    launch_zero_pad(L.g, c->r, nullptr, nullptr, nullptr, c->stream);
    launch_zero_pad_f32(L.g, c->q32, c->p32a, c->p32b, c->stream);
    for (;;) {
        launch_jcg_reset(c->sc, tol_abs, 0, -1, c->stream);
        CHK(rec_begin(c, l, 2, 0, &slot));
        launch_stencil<double>(MODE_INIT, a, c->stream);
        CHK(rec_end(c, slot));
        HIPCHK(c, hipMemcpyAsync(c->sc_host, c->sc, sizeof(JcgScalars), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        rn = std::sqrt(c->sc_host->rr);
        if (!(rn > tol_abs)) break;
        if (!std::isfinite(rn)) {
            status = ECMG_EBREAKDOWN;
            break;
        }
        if (outer >= max_outer || inner_total >= max_iter) {
            status = ECMG_ENOTCONV;
            break;
        }
        const double tol_in = std::max(c->opt.inner_tol, 0.5 * tol_abs / rn);
        launch_jcg_reset(c->sc32, tol_in, max_iter - inner_total, -1, c->stream);
        CHK(rec_begin(c, l, 8, 0, &slot));
        launch_mixed_start(L.g, c->r, 1.0 / rn, L.dinv32, c->r32, c->d32, c->sc32, c->partials, c->counters + 3,
                           c->stream);
        CHK(rec_end(c, slot));
        HIPCHK(c, hipGetLastError());
        CHK(jcg_chunks<float>(c, l, a32, b32, c->sc32, -1, 5, 6, 0));
        const JcgScalars s = *c->sc_host;
        CHK(rec_begin(c, l, 9, 0, &slot));
        launch_mixed_update(L.g, L.x, rn, c->d32, c->p32a, c->p32b, c->sc32, c->stream);
        CHK(rec_end(c, slot));
        HIPCHK(c, hipGetLastError());
        CHK(rec_flush(c, s.iter));
        inner_total += s.iter;
        ++outer;
        if (s.done == DONE_BREAKDOWN) {
            status = ECMG_EBREAKDOWN;
            break;
        }
        if (s.iter == 0) {               // FP32 cannot reduce this residual further
            status = ECMG_ENOTCONV;
            break;
        }
    }
    CHK(rec_flush(c, 1));
    if (info) {
        info->iters = inner_total;
        info->outer_steps = outer;
        info->rre = (L.nf > 0) ? rn / L.nf : 0.0;
        info->nf = L.nf;
        info->status = status;
        info->path = ECMG_PATH_MIXED;
    }
    if (status == ECMG_EBREAKDOWN) return fail(c, status, "mixed JCG breakdown on level %d", l);
    if (status == ECMG_ENOTCONV)
        return fail(c, status, "mixed JCG did not reach the tolerance on level %d (rre %g after %d outer steps)", l,
                    rn / L.nf, outer);
    return ECMG_OK;
}

// The level's results from its final JCG scalars s: iterations, relative
// residual, status (breakdown / iteration cap reported as errors).
static int jcg_result(ecmg_ctx *c, int l, const JcgScalars &s, int max_iter, bool keep_hint, ecmg_level_info *info) {
    Level &L = c->lv[l];
    if (info) {
        info->iters = s.iter;
        info->rre = (L.nf > 0) ? std::sqrt(s.rr) / L.nf : 0.0;
        info->nf = L.nf;
        info->status = (s.done == DONE_BREAKDOWN) ? ECMG_EBREAKDOWN
                       : (s.done == DONE_MAXITER) ? ECMG_ENOTCONV : ECMG_OK;
        info->path = L.last_path;
    }
    if (s.done == DONE_BREAKDOWN) return fail(c, ECMG_EBREAKDOWN, "JCG breakdown on level %d (p.q = %g)", l, s.pq);
    if (s.done == DONE_MAXITER)
        return fail(c, ECMG_ENOTCONV, "JCG reached max_iter = %d on level %d (rre %g)", max_iter, l,
                    std::sqrt(s.rr) / L.nf);
    if (keep_hint && s.done == DONE_CONVERGED) {
        L.spec_hits = s.iter == L.last_iters ? std::min(L.spec_hits + 1, 1 << 20) : 0;
        L.last_iters = s.iter;
    }
    return ECMG_OK;
}

// The column kernels take grids whose arrays index with 32-bit offsets.
static bool col_usable(const ecmg_ctx *c, const Geom &g) {
    return c->col_enable && g.nnodes < ((int64_t)1 << 31) && (int64_t)g.nx * g.ny * g.nz < ((int64_t)1 << 31);
}

// Column-kernel arguments of level L (input, output and partials set by the
// caller); returns the partial pairs a launch writes (waves, then the blocks
// of the Robin faces).
static int col_args(ecmg_ctx *c, Level &L, int R, ColArgs *ca) {
    ColArgs &x = *ca;
    x.g = L.g;
    x.KZ = std::max(1, std::min(c->col_kz, L.g.nz + 1));
    x.order = c->col_order;
    x.R = R;
    const int waves = col_waves(L.g, x.KZ, x.order, R, &x.ntx, &x.nty, &x.nkz);
    x.beta = L.beta;
    for (int f = 0; f < 6; ++f) x.alpha[f] = L.alpha[f];
    x.F = L.F;
    x.dinv = L.dinv;
    x.plain_cg = c->opt.method == ECMG_CG;
    x.sc = c->sc;
    ColFaces fl;
    return waves + col_faces(L.g, &fl);
}

// the gather path fits level grid g: folded scalars (each pass at most
// fold_max blocks)
static bool gather_possible(const ecmg_ctx *c, const Geom &g) {
    return gather_blocks(g) <= c->fold_max && passB_blocks(g.nnodes) <= c->fold_max;
}
// the level runs the gather path: chosen by the tuner (path 3) or, with no
// tuned choice, up to options.gather_nodes nodes
static bool gather_level(const ecmg_ctx *c, const Level &L) {
    const bool want = L.tune_path == 3 || (L.tune_path < 0 && L.g.nreal <= c->gather_max);
    return want && gather_possible(c, L.g);
}

// Tiled JCG of level l, enqueued: init, the iterations (status reads only
// between chunks), the last x update (the kernel checks whether one is
// pending), which also copies the final scalars into the level's pinned slot;
// the slot holds them once the stream has passed it.  speculate: a level whose
// last two solves converged in the same number of iterations enqueues that
// many and reads no status (L.spec_live; the caller checks `done` in the slot).
static int enqueue_jcg(ecmg_ctx *c, int l, double tol_abs, int max_iter, int fixed, bool speculate = false,
                       bool defer_x = false) {
    Level &L = c->lv[l];
    L.spec_live = speculate && fixed < 0 && c->opt.chunk <= 0 && c->opt.speculate && L.last_iters > 0 &&
                  L.spec_hits >= 1;
    launch_jcg_reset(c->sc, tol_abs, max_iter, fixed, c->stream);
    launch_zero_pad(L.g, c->r, c->q, c->p0, c->p1, c->stream);
    StencilArgs<double> a = stencil_args(c, L);
    a.v = L.x;
    a.r = c->r;
    a.q = c->q;
    a.x = L.x;
    a.p0 = c->p0;
    a.p1 = c->p1;
    a.p_init = 1;
    PassBArgs<double> b{};
    b.n = L.g.nnodes;
    b.r = c->r;
    b.q = c->q;
    b.dinv = L.dinv;
    b.sc = c->sc;
    b.partials = c->partials;
    const int64_t nb_b = passB_blocks(L.g.nnodes);
    // the gather levels: init and the stencil of every pass A one thread per
    // node, the node-wise p update taking the folded scalar step
    if (gather_level(c, L)) {
        L.last_path = ECMG_PATH_GATHER;
        const int64_t nb_g = gather_blocks(L.g);
        CHK(ensure_partials(c, 2 * nb_g + 2 * std::max(nb_g, nb_b)));
        double *pq = c->partials, *p2 = c->partials + 2 * nb_g;   // gather p.q; init / pass B pairs
        ColArgs ga{};
        ga.g = L.g;
        ga.beta = L.beta;
        for (int f = 0; f < 6; ++f) ga.alpha[f] = L.alpha[f];
        ga.F = L.F;
        ga.dinv = L.dinv;
        ga.sc = c->sc;
        size_t slot = 0;
        CHK(rec_begin(c, l, 2, 0, &slot));
        ga.v = L.x;
        ga.out = c->r;
        ga.p_out = c->p1;                         // p_0 in p1, as the tiled and column paths keep it
        ga.p_init = 1;
        ga.partials = p2;
        launch_gather_init(ga, c->stream);
        CHK(rec_end(c, slot));
        ga.v = c->p1;                             // p in p1 at even, p0 at odd iterations
        ga.v_odd = c->p0;
        ga.out = c->q;
        ga.p_out = nullptr;
        ga.p_init = 0;
        ga.partials = pq;
        PUFoldArgs u{};
        u.n = L.g.nnodes;
        u.dinv = L.dinv;
        u.r = c->r;
        u.p0 = c->p0;
        u.p1 = c->p1;
        u.x = L.x;
        u.sc = c->sc;
        u.partials = p2;
        b.fold = 1;
        b.partials = p2;
        b.pq_partials = pq;
        b.nb_a = (int)nb_g;
        const int hint = fixed < 0 ? L.last_iters : 0;
        CHK(jcg_chunks_gather(c, l, u, ga, b, fixed, hint, (int)nb_g, (int)nb_b, L.spec_live));
        launch_final_x(L.g, L.x, c->p0, c->p1, c->sc, c->sc_lv_dev + l, c->stream, !defer_x);
        HIPCHK(c, hipGetLastError());
        if (defer_x) c->x_pending = l;
        return ECMG_OK;
    }
    // folded scalars when both passes have few blocks: pass A's p.q partials
    // at the start of the buffer, init's and pass B's (r.z, r.r) pairs after
    const int64_t nb_a = (int64_t)a.ntx * a.nty * a.nkz;
    const bool fold = nb_a <= c->fold_max && nb_b <= c->fold_max &&
                      2 * nb_a + 2 * std::max(nb_a, nb_b) <= c->partials_n;
    if (fold) {
        a.fold = b.fold = 1;
        a.partials2 = c->partials + 2 * nb_a;
        b.partials = a.partials2;
        b.pq_partials = c->partials;
        b.nb_a = (int)nb_a;
    }
    // the large (unfolded) levels: JCG init and the stencil of every pass A by
    // the column kernels (after the node-wise p update from iteration 1 on)
    ColArgs ca{};
    int cw = 0;
    const bool col = !fold && col_usable(c, L.g);
    L.last_path = fold ? ECMG_PATH_TILED : col ? ECMG_PATH_COLUMN : ECMG_PATH_TILED_UNFOLDED;
    ColArgs ca0{};                                // iteration 0 (its own rows per wave)
    int cw0 = 0;
    if (col) {
        cw = col_args(c, L, COL_R_INIT, &ca);
        cw0 = col_args(c, L, COL_R_A0, &ca0);
        CHK(ensure_partials(c, 2 * (int64_t)std::max(cw, cw0)));
        ca.partials = ca0.partials = c->partials;
        a.partials = c->partials;
        b.partials = c->partials;
    }
    size_t slot = 0;
    CHK(rec_begin(c, l, 2, 0, &slot));
    if (col) {
        ca.v = L.x;
        ca.out = c->r;
        ca.p_out = c->p1;
        ca.p_init = 1;
        if (launch_col(MODE_INIT, ca, c->stream) < 0) return fail(c, ECMG_EINVAL, "column wave grid mismatch");
        CHK(rec_end(c, slot));
        launch_stencil_finish(MODE_INIT, c->sc, c->partials, cw, c->stream);
        ca0.v = c->p1;                            // iteration 0: q = A p_0 (p_0 in p1)
        ca0.v_odd = c->p0;                        // later: p in p1 at even, p0 at odd iterations
        ca0.out = c->q;
        ca0.p_out = nullptr;
        ca0.p_init = 0;
    } else {
        launch_stencil<double>(MODE_INIT, a, c->stream);
        CHK(rec_end(c, slot));
    }
    HIPCHK(c, hipGetLastError());

    const int hint = fixed < 0 ? L.last_iters : 0;
    if (fold) CHK(jcg_chunks_folded(c, l, a, b, fixed, hint, (int)nb_a, (int)nb_b, L.spec_live));
    else CHK(jcg_chunks(c, l, a, b, c->sc, fixed, 0, 1, hint, L.spec_live, col ? &ca0 : nullptr, cw0));
    launch_final_x(L.g, L.x, c->p0, c->p1, c->sc, c->sc_lv_dev + l, c->stream, !defer_x);
    HIPCHK(c, hipGetLastError());
    if (defer_x) c->x_pending = l;
    return ECMG_OK;
}

// Apply a pending last x update (see ecmg_ctx::x_pending).
static int flush_x(ecmg_ctx *c) {
    if (!c || c->x_pending < 0) return ECMG_OK;
    const int l = c->x_pending;
    c->x_pending = -1;
    if (l >= c->nlev) return ECMG_OK;
    const Level &L = c->lv[l];
    launch_final_x(L.g, L.x, c->p0, c->p1, c->sc, c->sc_lv_dev + l, c->stream);
    HIPCHK(c, hipGetLastError());
    return ECMG_OK;
}

static int run_jcg(ecmg_ctx *c, int l, double tol_abs, int max_iter, int fixed, ecmg_level_info *info) {
    CHK(enqueue_jcg(c, l, tol_abs, max_iter, fixed));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const JcgScalars s = c->sc_lv[l];
    CHK(rec_flush(c, s.iter));
    return jcg_result(c, l, s, max_iter, fixed < 0, info);
}

// Whole JCG loop of one level in one cooperative launch (small grids),
// enqueued: the task goes from the level's pinned slot to the device, the final
// scalars come back into the level's scalar slot.
static int enqueue_jcg_persistent(ecmg_ctx *c, int l, double tol_abs, int max_iter, int fixed) {
    Level &L = c->lv[l];
    L.last_path = ECMG_PATH_PERSISTENT;
    PersistentTask &t = c->task_lv[l];
    t = PersistentTask{};
    t.g = L.g;
    t.beta = L.beta;
    for (int f = 0; f < 6; ++f) t.alpha[f] = L.alpha[f];
    t.F = L.F;
    t.dinv = L.dinv;
    t.x = L.x;
    t.r = c->r;
    t.q = c->q;
    t.p[0] = c->p0;
    t.p[1] = c->p1;
    t.partials = c->partials;
    t.err = (int *)c->d_bar;
    t.bar = c->d_bar + 16;
    t.sc = c->sc;
    t.tol = tol_abs;
    t.max_iter = max_iter;
    t.fixed = fixed;
    t.wg0 = 0;
    // one thread per column segment (2 nodes below 131072 nodes, else 4: short
    // segments spread small grids over more lanes, longer ones save halo
    // loads), at most persist_nwg workgroups (every barrier costs more with
    // more of them)
    const bool tuned = L.tune_path == 1 && L.tune_seg > 0 && L.tune_nwg > 0;
    const int seg = tuned ? L.tune_seg : c->persist_seglen > 0 ? c->persist_seglen : (L.g.nreal < 131072 ? 2 : 4);
    t.seglen = seg >= 4 ? 4 : (seg >= 2 ? 2 : 1);         // the kernel's instantiations
    const int64_t nseg = (L.g.nz + t.seglen) / t.seglen;
    const int64_t units = (int64_t)(L.g.nx + 1) * (L.g.ny + 1) * nseg;
    t.nwg = (int)std::max<int64_t>(
        1, std::min<int64_t>({(units + PERSIST_NTP - 1) / PERSIST_NTP, (int64_t)(tuned ? L.tune_nwg : c->persist_nwg),
                              (int64_t)c->persist_blocks}));
    HIPCHK(c, hipMemsetAsync(c->d_bar, 0, 32 * sizeof(unsigned), c->stream));
    HIPCHK(c, hipMemcpyAsync(c->d_task, &t, sizeof(t), hipMemcpyHostToDevice, c->stream));
    size_t slot = 0;
    CHK(rec_begin(c, l, 7, 0, &slot));
    HIPCHK(c, launch_jcg_persistent(c->d_task, 1, t.nwg, c->stream));
    CHK(rec_end(c, slot));
    HIPCHK(c, hipMemcpyAsync(c->sc_lv + l, c->sc, sizeof(JcgScalars), hipMemcpyDeviceToHost, c->stream));
    return ECMG_OK;
}

static int run_jcg_persistent(ecmg_ctx *c, int l, double tol_abs, int max_iter, int fixed, ecmg_level_info *info) {
    CHK(enqueue_jcg_persistent(c, l, tol_abs, max_iter, fixed));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    const JcgScalars s = c->sc_lv[l];
    CHK(rec_flush(c, 1));
    return jcg_result(c, l, s, max_iter, false, info);
}

// the persistent kernel can run the grid: co-resident workgroups exist and its
// 32-bit indices reach every node and element
static bool persist_possible(const ecmg_ctx *c, const Geom &g) {
    return c->persist_blocks > 0 && g.nnodes < ((int64_t)1 << 31) && (int64_t)g.nx * g.ny * g.nz < ((int64_t)1 << 31);
}

// The level's JCG path: the autotuned one if there is one, else the persistent
// kernel up to persist_max nodes.
static bool uses_persistent(const ecmg_ctx *c, int l) {
    const Level &L = c->lv[l];
    if (L.tune_path == 0 || L.tune_path == 3) return false;
    if (L.tune_path == 1) return persist_possible(c, L.g);
    return persist_possible(c, L.g) && L.g.nreal <= c->persist_max;
}

// Mixed precision applies to JCG levels (not DSOLVE) solved by the tiled
// kernels above mixed_min nodes; smaller levels are latency-bound (FP32 saves
// bytes they do not wait for, the outer FP64 steps add host round trips, and
// FP32 JCG needed up to 1.6x the FP64 iterations on a high-contrast problem)
// and stay FP64, as do the persistent ones.
static bool uses_mixed(const ecmg_ctx *c, int l) {
    return c->opt.precision == ECMG_MIXED && l >= 2 && !uses_persistent(c, l) && c->lv[l].g.nreal > c->mixed_min;
}

// ||F - A u_l||^2 over the free nodes of level l from its current iterate,
// enqueued: a JCG init pass into the scratch residual (its finishing step
// leaves the sum in the context's scalars, which the level no longer needs),
// copied into the level's pinned slot once the stream gets there.
static int enqueue_true_residual(ecmg_ctx *c, int l) {
    Level &L = c->lv[l];
    StencilArgs<double> a = stencil_args(c, L);
    a.v = L.x;
    a.r = c->r;
    a.p_init = 0;
    launch_stencil<double>(MODE_INIT, a, c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(c->rrt_lv + l, &c->sc->rr, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    return ECMG_OK;
}

// info->rre_true of level l from its pinned slot (after the stream has passed
// enqueue_true_residual), -1 when not requested
static void fill_true_residual(const ecmg_ctx *c, int l, ecmg_level_info *info) {
    const Level &L = c->lv[l];
    if (!c->opt.true_residual) info->rre_true = -1.0;
    else info->rre_true = L.nf > 0 ? std::sqrt(c->rrt_lv[l]) / L.nf : 0.0;
}

static int run_level_jcg(ecmg_ctx *c, int l, double tol_abs, int max_iter, int fixed, ecmg_level_info *info) {
    if (uses_mixed(c, l) && fixed < 0) return run_jcg_mixed(c, l, tol_abs, max_iter, info);
    if (uses_persistent(c, l)) return run_jcg_persistent(c, l, tol_abs, max_iter, fixed, info);
    return run_jcg(c, l, tol_abs, max_iter, fixed, info);
}

static int do_exp_finite(ecmg_ctx *c, int l) {
    Level &L = c->lv[l];
    size_t slot = 0;
    CHK(rec_begin(c, l, 3, 0, &slot));
    launch_exp_finite(L.g, c->lv[l - 1].g, c->lv[l - 1].x, c->lv[l - 2].x, L.x, L.W, c->opt.interp, c->stream);
    CHK(rec_end(c, slot));
    HIPCHK(c, hipGetLastError());
    return ECMG_OK;
}

static int do_exp_true(ecmg_ctx *c, int l) {
    Level &L = c->lv[l];
    if (!L.Ut) CHK(dalloc_n(c, &L.Ut, L.g.nnodes));
    size_t slot = 0;
    CHK(rec_begin(c, l, 4, 0, &slot));
    if (c->x_pending == l)        // U~ from x + alpha p, the update itself stays pending
        launch_exp_true(L.g, L.x, c->lv[l - 1].x, L.Ut, c->stream, c->sc, c->p0, c->p1);
    else
        launch_exp_true(L.g, L.x, c->lv[l - 1].x, L.Ut, c->stream);
    CHK(rec_end(c, slot));
    HIPCHK(c, hipGetLastError());
    return ECMG_OK;
}

// ---------------------------------------------------------------------------
// context lifetime
// ---------------------------------------------------------------------------
static void free_levels(ecmg_ctx *c) {
    for (auto &L : c->lv) {
        dfree(c, L.beta);
        dfree(c, L.F);
        dfree(c, L.x);
        dfree(c, L.dinv);
        dfree(c, L.W);
        dfree(c, L.Ut);
        dfree(c, L.beta32);
        dfree(c, L.dinv32);
        dfree(c, L.ainv);
        dfree(c, L.freeid);
        for (int f = 0; f < 6; ++f) {
            dfree(c, L.alpha[f]);
            dfree(c, L.alpha32[f]);
        }
    }
    c->lv.clear();
    dfree(c, c->r);
    dfree(c, c->p0);
    dfree(c, c->p1);
    dfree(c, c->q);
    dfree(c, c->partials);
    c->r = c->p0 = c->p1 = c->q = c->partials = nullptr;
    dfree(c, c->r32);
    dfree(c, c->p32a);
    dfree(c, c->p32b);
    dfree(c, c->q32);
    dfree(c, c->d32);
    c->r32 = c->p32a = c->p32b = c->q32 = c->d32 = nullptr;
    c->scratch_n = 0;
    c->partials_n = 0;
    c->nlev = 0;
    c->ready = c->solved = false;
}

extern "C" {

void ecmg_default_options(ecmg_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->precision = ECMG_FP64;
    o->max_iter = 20000;
    o->interp = ECMG_SERENDIPITY20;
    o->keep_w = 1;
    o->inner_tol = 1e-4;
    o->dsolve_tol = 1e-14;
    o->chunk = 0;
    o->timing = 0;
    o->hip_stream = nullptr;
    o->persistent_nodes = -1;
    o->dsolve_dense_max = DSOLVE_DENSE_LIMIT;
    o->autotune = 0;
    o->tune_cache = nullptr;
    o->method = ECMG_JCG;
    o->speculate = 1;
    o->fold_blocks = -1;
    o->true_residual = 0;
    o->batch_graph = 1;
    o->columns = 1;
    o->gather_nodes = -1;
    o->alloc = nullptr;
    o->free = nullptr;
    o->alloc_user = nullptr;
}

int ecmg_create(const ecmg_options *opt, ecmg_ctx **out) {
    if (!out) return fail(nullptr, ECMG_EINVAL, "ecmg_create: out is NULL");
    *out = nullptr;
    ecmg_options o;
    ecmg_default_options(&o);
    if (opt) o = *opt;
    if (o.precision != ECMG_FP64 && o.precision != ECMG_MIXED)
        return fail(nullptr, ECMG_EINVAL, "unknown precision %d", o.precision);
    if (o.interp != ECMG_SERENDIPITY20 && o.interp != ECMG_LAGRANGE27)
        return fail(nullptr, ECMG_EINVAL, "unknown interpolation %d", o.interp);
    if (o.method != ECMG_JCG && o.method != ECMG_CG) return fail(nullptr, ECMG_EINVAL, "unknown method %d", o.method);
    if (o.max_iter < 0) return fail(nullptr, ECMG_EINVAL, "max_iter < 0");
    if ((o.alloc == nullptr) != (o.free == nullptr))
        return fail(nullptr, ECMG_EINVAL, "options.alloc and options.free must be given together");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1)
        return fail(nullptr, ECMG_EDEVICE, "no HIP device available");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(nullptr, ECMG_EDEVICE, "hipGetDevice failed");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return fail(nullptr, ECMG_EDEVICE, "hipGetDeviceProperties failed");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, ECMG_EDEVICE, "device %d is %s; this library is built for gfx950", dev,
                    prop.gcnArchName);
    {
        // the device address of this GPU's copy of `scratch` (ecmg_norms_noalloc)
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (dev >= NOALLOC_MAX_DEVICES) return fail(nullptr, ECMG_EDEVICE, "device %d: too many devices", dev);
        if (!g_scratch_ptr[dev]) {
            void *ptr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr)
                return fail(nullptr, ECMG_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
            g_scratch_ptr[dev] = ptr;
        }
    }
    ecmg_ctx *c = new ecmg_ctx();
    c->device = dev;
    c->opt = o;
    c->timing_mask = o.timing ? ((1u << NKIND) - 1u) : 0u;
    if (o.tune_cache) c->tune_cache = o.tune_cache;
    else if (const char *tc = std::getenv("ECMG_TUNE_CACHE")) c->tune_cache = tc;
    c->opt.tune_cache = nullptr;              // the caller's string is not kept
    c->device_name = std::string(prop.gcnArchName) + " " + std::to_string(prop.multiProcessorCount) + " CUs";
    if (const char *kz = std::getenv("ECMG_KZ")) c->KZ = std::max(1, std::atoi(kz));
    if (const char *kt = std::getenv("ECMG_KZ_TARGET")) c->kz_target = std::max(1, std::atoi(kt));
    if (o.fold_blocks >= 0) c->fold_max = std::min<int>(o.fold_blocks, FOLD_MAX_BLOCKS);
    c->col_enable = o.columns != 0;
    if (o.gather_nodes >= 0) c->gather_max = o.gather_nodes;
    if (const char *v = std::getenv("ECMG_COL")) c->col_enable = std::atoi(v) != 0;
    if (const char *v = std::getenv("ECMG_COL_KZ")) c->col_kz = std::max(1, std::atoi(v));
    if (const char *v = std::getenv("ECMG_COL_ORDER")) c->col_order = std::min(2, std::max(0, std::atoi(v)));
    if (const char *v = std::getenv("ECMG_PERSIST_SEG")) c->persist_seglen = std::max(1, std::atoi(v));
    if (const char *v = std::getenv("ECMG_PERSIST_NWG")) c->persist_nwg = std::max(1, std::atoi(v));
    if (const char *v = std::getenv("ECMG_BATCH_NPW")) c->batch_npw = std::max(64, std::atoi(v));
    if (o.hip_stream) {
        c->stream = (hipStream_t)o.hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return fail(nullptr, ECMG_EDEVICE, "hipStreamCreate failed");
        }
        c->own_stream = true;
    }
    int rc = ECMG_OK;
    if ((rc = dalloc(c, (void **)&c->sc, sizeof(JcgScalars))) != ECMG_OK ||
        (rc = dalloc(c, (void **)&c->sc32, sizeof(JcgScalars))) != ECMG_OK ||
        (rc = dalloc(c, (void **)&c->counters, 16 * sizeof(unsigned))) != ECMG_OK ||
        (rc = dalloc(c, (void **)&c->dres, 8 * sizeof(double))) != ECMG_OK) {
        ecmg_destroy(c);
        return rc;
    }
    {
        int per_cu = 0, cus = 0;
        const int mb = persistent_max_blocks(&per_cu, &cus);
        c->persist_blocks = mb > 0 ? mb : 0;
        const int qb = queue_max_blocks();
        c->queue_blocks = qb > 0 ? qb : 0;
        if (o.persistent_nodes >= 0) c->persist_max = c->mixed_min = o.persistent_nodes;
    }
    // barrier words: error flag at 0, arrival counter at 16 (its own cache line)
    if ((rc = dalloc(c, (void **)&c->d_task, sizeof(PersistentTask))) != ECMG_OK ||
        (rc = dalloc(c, (void **)&c->d_bar, 32 * sizeof(unsigned))) != ECMG_OK) {
        ecmg_destroy(c);
        return rc;
    }
    if (hipMemsetAsync(c->counters, 0, 16 * sizeof(unsigned), c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess ||
        hipHostMalloc((void **)&c->sc_host, sizeof(JcgScalars), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&c->hres, 8 * sizeof(double), hipHostMallocDefault) != hipSuccess ||
        hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess) {
        ecmg_destroy(c);
        return fail(nullptr, ECMG_EDEVICE, "context initialisation failed");
    }
    *out = c;
    return ECMG_OK;
}

void ecmg_destroy(ecmg_ctx *c) {
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    free_levels(c);
    bin_flush(c);
    dfree(c, c->stmp);
    dfree(c, c->scoord);
    if (c->blas) (void)rocblas_destroy_handle(c->blas);
    batch_plan_free(c, c->bplan);
    c->bplan = nullptr;
    dfree(c, c->sc);
    dfree(c, c->sc32);
    dfree(c, c->bt_tasks);
    dfree(c, c->bt_sc);
    dfree(c, c->bt_next);
    dfree(c, c->bt_bar);
    dfree(c, c->bt_exp);
    if (c->bt_sc_host) (void)hipHostFree(c->bt_sc_host);
    dfree(c, c->d_task);
    dfree(c, c->d_bar);
    dfree(c, c->counters);
    dfree(c, c->dres);
    dfree(c, c->dstage);
    if (c->hstage) (void)hipHostFree(c->hstage);
    if (c->sc_host) (void)hipHostFree(c->sc_host);
    if (c->hres) (void)hipHostFree(c->hres);
    for (auto e : c->evpool) (void)hipEventDestroy(e);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->sc_lv) (void)hipHostFree(c->sc_lv);
    if (c->task_lv) (void)hipHostFree(c->task_lv);
    if (c->rrt_lv) (void)hipHostFree(c->rrt_lv);
    for (auto e : c->lv_ev) (void)hipEventDestroy(e);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

const char *ecmg_last_error(const ecmg_ctx *c) {
    if (c) return c->err.c_str();
    return g_thread_error.c_str();
}

static int validate(ecmg_ctx *c, const ecmg_problem *p) {
    if (!p) return fail(c, ECMG_EINVAL, "problem is NULL");
    for (int d = 0; d < 3; ++d) {
        if (!(p->lo[d] < p->hi[d]) || !std::isfinite(p->lo[d]) || !std::isfinite(p->hi[d]))
            return fail(c, ECMG_EINVAL, "box: lo[%d] = %g must be < hi[%d] = %g", d, p->lo[d], d, p->hi[d]);
        if (p->n0[d] < 1) return fail(c, ECMG_EINVAL, "n0[%d] = %d must be >= 1", d, p->n0[d]);
    }
    if (p->levels < 2 || p->levels > 16) return fail(c, ECMG_EINVAL, "levels = %d must be in [2, 16]", p->levels);
    for (int d = 0; d < 3; ++d) {
        const int64_t n = (int64_t)p->n0[d] << (p->levels - 1);
        if (n > (int64_t)1 << 20) return fail(c, ECMG_EINVAL, "finest grid too large on axis %d", d);
    }
    bool anyD = false;
    for (int f = 0; f < 6; ++f) {
        if (p->face_type[f] != ECMG_DIRICHLET && p->face_type[f] != ECMG_ROBIN)
            return fail(c, ECMG_EINVAL, "face_type[%d] = %d is neither Dirichlet nor Robin", f, p->face_type[f]);
        anyD |= p->face_type[f] == ECMG_DIRICHLET;
    }
    if (!anyD && !p->alpha.host && !p->alpha.device && !(p->alpha.value > 0))
        return fail(c, ECMG_EINVAL, "no Dirichlet face and alpha == 0: the system is singular");
    return ECMG_OK;
}

int ecmg_cascadic_schedule(int32_t levels, int32_t m_L, double beta, int32_t *iters) {
    if (!iters) return fail(nullptr, ECMG_EINVAL, "ecmg_cascadic_schedule: iters is NULL");
    if (levels < 3 || m_L < 1 || !(beta >= 1.0) || !std::isfinite(beta))
        return fail(nullptr, ECMG_EINVAL, "ecmg_cascadic_schedule: need levels >= 3, m_L >= 1, beta >= 1");
    // eq. ee: grid j of the L = levels - 2 fine grids (level j + 1) runs
    // ceil(m_L * beta^(L - j)) iterations; the power as repeated products
    const int L = levels - 2;
    iters[0] = iters[1] = 0;
    for (int j = 1; j <= L; ++j) {
        double m = (double)m_L;
        for (int e = 0; e < L - j; ++e) m *= beta;
        const double c = std::ceil(m);
        if (!(c <= 2147483647.0)) return fail(nullptr, ECMG_EINVAL, "ecmg_cascadic_schedule: count overflows");
        iters[j + 1] = (int32_t)c;
    }
    return ECMG_OK;
}

int ecmg_plan_bytes(const ecmg_problem *p, int32_t precision, size_t *bytes) {
    if (!bytes) return fail(nullptr, ECMG_EINVAL, "bytes is NULL");
    int rc = validate(nullptr, p);
    if (rc != ECMG_OK) return rc;
    size_t tot = 0;
    int64_t finest = 0;
    for (int l = 0; l < p->levels; ++l) {
        double lo[3];
        Geom g = make_geom(p, l, lo);
        const int64_t ne = (int64_t)g.nx * g.ny * g.nz;
        tot += 8 * (size_t)(5 * g.nnodes + ne);     // F, x, dinv, W, U~ + beta
        if (precision == ECMG_MIXED) tot += 4 * (size_t)(g.nnodes + ne);
        finest = g.nnodes;
    }
    tot += 8 * (size_t)(4 * finest);                // r, p0, p1, q
    if (precision == ECMG_MIXED) tot += 4 * (size_t)(5 * finest);
    *bytes = tot;
    return ECMG_OK;
}

int ecmg_setup(ecmg_ctx *c, const ecmg_problem *p) {
    if (!c) return fail(nullptr, ECMG_EINVAL, "ctx is NULL");
    CHK(validate(c, p));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->x_pending = -1;
    // the same grids as the current hierarchy: its blocks are kept and taken
    // back by size (the serving loop sets up one request after another on a
    // context); otherwise everything is freed first
    bool same = c->nlev == p->levels;
    for (int l = 0; same && l < p->levels; ++l) {
        double lo[3];
        const Geom g = make_geom(p, l, lo);
        same = g.nnodes == c->lv[l].g.nnodes && g.nx == c->lv[l].g.nx && g.ny == c->lv[l].g.ny;
    }
    if (!same) bin_flush(c);
    c->recycle = same;
    free_levels(c);
    c->recycle = false;
    c->nlev = p->levels;
    c->gen = ++g_generation;
    for (int f = 0; f < 6; ++f) c->face_type[f] = p->face_type[f];
    c->lv.resize(p->levels);
    if (c->lv_cap < p->levels) {
        if (c->sc_lv) (void)hipHostFree(c->sc_lv);
        if (c->task_lv) (void)hipHostFree(c->task_lv);
        if (c->rrt_lv) (void)hipHostFree(c->rrt_lv);
        c->sc_lv = c->sc_lv_dev = nullptr;
        c->task_lv = nullptr;
        c->rrt_lv = nullptr;
        c->lv_cap = 0;
        if (hipHostMalloc((void **)&c->sc_lv, sizeof(JcgScalars) * p->levels, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void **)&c->task_lv, sizeof(PersistentTask) * p->levels, hipHostMallocDefault) !=
                hipSuccess ||
            hipHostMalloc((void **)&c->rrt_lv, sizeof(double) * p->levels, hipHostMallocDefault) != hipSuccess)
            return fail(c, ECMG_ENOMEM, "pinned host allocation of %d level slots failed", p->levels);
        HIPCHK(c, hipHostGetDevicePointer((void **)&c->sc_lv_dev, c->sc_lv, 0));
        c->lv_cap = p->levels;
    }
    while (c->lv_ev.size() < 2 * (size_t)p->levels) {
        hipEvent_t e;
        HIPCHK(c, hipEventCreate(&e));
        c->lv_ev.push_back(e);
    }
    // scratch for the finest level and reduction partials
    {
        double lo[3];
        Geom gf = make_geom(p, p->levels - 1, lo);
        c->scratch_n = gf.nnodes;
        CHK(dalloc_n(c, &c->r, gf.nnodes));
        CHK(dalloc_n(c, &c->p0, gf.nnodes));
        CHK(dalloc_n(c, &c->p1, gf.nnodes));
        CHK(dalloc_n(c, &c->q, gf.nnodes));
        if (c->opt.precision == ECMG_MIXED) {
            CHK(dalloc_n(c, &c->r32, gf.nnodes));
            CHK(dalloc_n(c, &c->p32a, gf.nnodes));
            CHK(dalloc_n(c, &c->p32b, gf.nnodes));
            CHK(dalloc_n(c, &c->q32, gf.nnodes));
            CHK(dalloc_n(c, &c->d32, gf.nnodes));
        }
        // at least the two regions of folded scalar steps (pass A: 2 per block,
        // then init / pass B: 2 per block, each pass up to FOLD_MAX_BLOCKS)
        int64_t pn = std::max<int64_t>(4 * (int64_t)FOLD_MAX_BLOCKS, 3 * (int64_t)c->persist_blocks);
        for (int l = 0; l < p->levels; ++l) {
            Geom g = make_geom(p, l, lo);
            int a, b, d;
            pn = std::max<int64_t>(pn, 2 * (int64_t)stencil_blocks(g, stencil_kz(g, c->KZ, c->kz_target), &a, &b, &d));
            pn = std::max<int64_t>(pn, 2 * passB_blocks(g.nnodes));
            ColFaces fl;
            pn = std::max<int64_t>(pn, 2 * ((int64_t)col_waves(g, std::max(1, std::min(c->col_kz, g.nz + 1)), c->col_order, std::min(COL_R_INIT, COL_R_A0), &a, &b, &d) +
                                            col_faces(g, &fl)));
        }
        c->partials_n = pn;
        CHK(dalloc_n(c, &c->partials, pn));
    }
    for (int l = 0; l < p->levels; ++l) {
        Level &L = c->lv[l];
        L.g = make_geom(p, l, L.lo);
        const Geom &g = L.g;
        L.nelem = (int64_t)g.nx * g.ny * g.nz;
        CHK(dalloc_n(c, &L.beta, L.nelem));
        CHK(dalloc_n(c, &L.F, g.nnodes));
        CHK(dalloc_n(c, &L.x, g.nnodes));
        CHK(dalloc_n(c, &L.dinv, g.nnodes));
        if (c->opt.keep_w && l >= 2) CHK(dalloc_n(c, &L.W, g.nnodes));
        const std::vector<double> cx = centroid_coords(g, L.lo, 0), cy = centroid_coords(g, L.lo, 1),
                                  cz = centroid_coords(g, L.lo, 2);
        const std::vector<double> gx = gauss_coords(g, L.lo, 0), gy = gauss_coords(g, L.lo, 1),
                                  gz = gauss_coords(g, L.lo, 2);
        const std::vector<double> nx = node_coords(g, L.lo, 0), ny = node_coords(g, L.lo, 1),
                                  nz = node_coords(g, L.lo, 2);
        // beta at element centroids, in slabs of element layers
        {
            const int64_t per = (int64_t)g.nx * g.ny;
            const int step = (int)std::max<int64_t>(1, kBatchPoints / per);
            for (int k0 = 0; k0 < g.nz; k0 += step) {
                const int k1 = std::min(g.nz, k0 + step);
                std::vector<double> zz(cz.begin() + k0, cz.begin() + k1);
                CHK(sample(c, p->beta, "beta", -1, cx, cy, zz, L.beta + per * k0, 1));
            }
        }
        // load vector: f at 2x2x2 Gauss points, slab by slab
        launch_fill(L.F, g.nnodes, 0.0, c->stream);
        {
            const int64_t per = 8 * (int64_t)g.nx * g.ny;   // Gauss points per element layer
            const int step = (int)std::max<int64_t>(1, kBatchPoints / per);
            CHK(ensure_scratch(c, &c->stmp, &c->stmp_n, per * std::min(step, g.nz)));
            for (int e0 = 0; e0 < g.nz; e0 += step) {
                const int e1 = std::min(g.nz, e0 + step);
                std::vector<double> zz(gz.begin() + 2 * e0, gz.begin() + 2 * e1);
                CHK(sample(c, p->f, "f", -1, gx, gy, zz, c->stmp, 0));
                launch_load_volume(g, e0, e1, c->stmp, L.F, c->stream);
            }
        }
        // Robin faces: alpha at face-element centroids, g_R at face Gauss points
        launch_fill(L.x, g.nnodes, 0.0, c->stream);
        const int n3[3] = {g.nx, g.ny, g.nz};
        for (int f = 0; f < 6; ++f) {
            int pax, qax;
            face_axes_h(f, pax, qax);
            const int ax = f / 2;
            const double plane = (f & 1) ? p->hi[ax] : p->lo[ax];
            if (p->face_type[f] == ECMG_ROBIN) {
                L.nface[f] = (int64_t)n3[pax] * n3[qax];
                CHK(dalloc_n(c, &L.alpha[f], L.nface[f]));
                std::vector<double> s[3];
                s[ax] = {plane};
                s[pax] = centroid_coords(g, L.lo, pax);
                s[qax] = centroid_coords(g, L.lo, qax);
                CHK(sample(c, p->alpha, "alpha", f, s[0], s[1], s[2], L.alpha[f], 2));
                s[pax] = gauss_coords(g, L.lo, pax);
                s[qax] = gauss_coords(g, L.lo, qax);
                CHK(ensure_scratch(c, &c->stmp, &c->stmp_n, 4 * L.nface[f]));
                CHK(sample(c, p->g_R, "g_R", f, s[0], s[1], s[2], c->stmp, 0));
                launch_load_face(g, f, c->stmp, L.F, c->stream);
            }
        }
        // Dirichlet data at the nodes of Dirichlet faces
        for (int f = 0; f < 6; ++f) {
            if (p->face_type[f] != ECMG_DIRICHLET) continue;
            int pax, qax;
            face_axes_h(f, pax, qax);
            const int ax = f / 2;
            const std::vector<double> &nc = (ax == 0) ? nx : (ax == 1) ? ny : nz;
            std::vector<double> s[3];
            s[ax] = {(f & 1) ? nc.back() : nc.front()};
            s[pax] = node_coords(g, L.lo, pax);
            s[qax] = node_coords(g, L.lo, qax);
            CHK(ensure_scratch(c, &c->stmp, &c->stmp_n, (int64_t)s[pax].size() * s[qax].size()));
            CHK(sample(c, p->g_D, "g_D", f, s[0], s[1], s[2], c->stmp, 0));
            launch_scatter_face(g, f, c->stmp, L.x, c->stream);
        }
        const double *al[6];
        for (int f = 0; f < 6; ++f) al[f] = L.alpha[f];
        launch_dinv(g, L.beta, al, L.dinv, c->opt.method == ECMG_CG, c->stream);
        if (uses_mixed(c, l)) {           // FP32 copies for the inner JCG of the mixed form
            CHK(dalloc_n(c, &L.beta32, L.nelem));
            CHK(dalloc_n(c, &L.dinv32, g.nnodes));
            launch_to_f32(L.beta, L.beta32, L.nelem, c->stream);
            launch_to_f32(L.dinv, L.dinv32, g.nnodes, c->stream);
            for (int f = 0; f < 6; ++f) {
                if (!L.alpha[f]) continue;
                CHK(dalloc_n(c, &L.alpha32[f], L.nface[f]));
                launch_to_f32(L.alpha[f], L.alpha32[f], L.nface[f], c->stream);
            }
        }
        // ||f_h||: b = F - A x0 on free nodes (x0 = g_D on Dirichlet nodes, 0 elsewhere)
        StencilArgs<double> a = stencil_args(c, L);
        a.v = L.x;
        a.q = c->q;
        launch_stencil<double>(MODE_APPLY, a, c->stream);
        launch_rhs_norm(g, L.F, c->q, L.x, c->partials, c->counters + 2, c->dres, c->stream);
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipMemcpyAsync(c->hres, c->dres, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        L.nf = std::sqrt(c->hres[1]);
    }
    // DSOLVE (Algorithm 4, levels 0 and 1): the explicit inverse of A_FF is a
    // setup product, so every solve only applies it
    for (int l = 0; l < std::min(2, c->nlev); ++l) CHK(dense_prepare(c, l));
    if (c->opt.autotune == 1) CHK(apply_tune_cache(c));
    c->ready = true;
    c->solved = false;
    return ECMG_OK;
}

// ---------------------------------------------------------------------------
// DSOLVE as a direct solve (Algorithm 4, levels 0 and 1): the explicit inverse
// of A_FF from its Cholesky factor, built once per hierarchy by ecmg_setup, then
// x_F = A_FF^-1 (F - A_FD g_D) as one matrix-vector product per solve
// ---------------------------------------------------------------------------
static bool host_dir(const Geom &g, int i, int j, int k) {
    return (i == 0 && g.ft[0] == ECMG_DIRICHLET) || (i == g.nx && g.ft[1] == ECMG_DIRICHLET) ||
           (j == 0 && g.ft[2] == ECMG_DIRICHLET) || (j == g.ny && g.ft[3] == ECMG_DIRICHLET) ||
           (k == 0 && g.ft[4] == ECMG_DIRICHLET) || (k == g.nz && g.ft[5] == ECMG_DIRICHLET);
}

static int dense_prepare(ecmg_ctx *c, int l) {
    Level &L = c->lv[l];
    if (L.dense != 0) return ECMG_OK;
    L.dense = -1;
    const int64_t lim = std::min<int64_t>(c->opt.dsolve_dense_max, DSOLVE_DENSE_LIMIT);
    if (lim <= 0) return ECMG_OK;
    const Geom &g = L.g;
    std::vector<int> fmap((size_t)g.nnodes, -1), freeid;
    for (int k = 0; k <= g.nz; ++k)
        for (int j = 0; j <= g.ny; ++j)
            for (int i = 0; i <= g.nx; ++i) {
                if (host_dir(g, i, j, k)) continue;
                const int64_t pid = i + (int64_t)g.sx * (j + (int64_t)g.sy * k);
                fmap[(size_t)pid] = (int)freeid.size();
                freeid.push_back((int)pid);
            }
    const int nf = (int)freeid.size();
    if (nf == 0 || nf > lim) return ECMG_OK;
    int *d_fmap = nullptr, *d_info = nullptr;
    CHK(dalloc(c, (void **)&d_fmap, sizeof(int) * fmap.size()));
    CHK(dalloc(c, (void **)&d_info, sizeof(int)));
    CHK(dalloc(c, (void **)&L.freeid, sizeof(int) * (size_t)nf));
    CHK(dalloc_n(c, &L.ainv, (int64_t)nf * nf));
    HIPCHK(c, hipMemcpyAsync(d_fmap, fmap.data(), sizeof(int) * fmap.size(), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipMemcpyAsync(L.freeid, freeid.data(), sizeof(int) * (size_t)nf, hipMemcpyHostToDevice, c->stream));
    const double *al[6];
    for (int f = 0; f < 6; ++f) al[f] = L.alpha[f];
    launch_assemble_dense(g, L.beta, al, d_fmap, L.ainv, nf, c->stream);
    HIPCHK(c, hipGetLastError());
    if (!c->blas && rocblas_create_handle(&c->blas) != rocblas_status_success) {
        c->blas = nullptr;
        return fail(c, ECMG_EDEVICE, "rocblas_create_handle failed");
    }
    int info = 0;
    bool ok = rocblas_set_stream(c->blas, c->stream) == rocblas_status_success &&
              rocsolver_dpotrf(c->blas, rocblas_fill_lower, nf, L.ainv, nf, d_info) == rocblas_status_success &&
              hipMemcpyAsync(&info, d_info, sizeof(int), hipMemcpyDeviceToHost, c->stream) == hipSuccess &&
              hipStreamSynchronize(c->stream) == hipSuccess && info == 0;
    ok = ok && rocsolver_dpotri(c->blas, rocblas_fill_lower, nf, L.ainv, nf, d_info) == rocblas_status_success &&
         hipMemcpyAsync(&info, d_info, sizeof(int), hipMemcpyDeviceToHost, c->stream) == hipSuccess &&
         hipStreamSynchronize(c->stream) == hipSuccess && info == 0;
    if (ok) launch_symmetrize(L.ainv, nf, c->stream);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    dfree(c, d_fmap);
    dfree(c, d_info);
    if (!ok) {                                    // not factorable: keep the JCG DSOLVE
        dfree(c, L.ainv);
        dfree(c, L.freeid);
        L.ainv = nullptr;
        L.freeid = nullptr;
        return ECMG_OK;
    }
    L.nfree = nf;
    L.dense = 1;
    return ECMG_OK;
}

static int run_dsolve_dense(ecmg_ctx *c, int l, ecmg_level_info *info) {
    Level &L = c->lv[l];
    launch_zero_free(L.g, L.x, c->stream);       // x0: g_D on Dirichlet nodes, 0 elsewhere
    StencilArgs<double> a = stencil_args(c, L);
    a.v = L.x;
    a.q = c->q;
    launch_stencil<double>(MODE_APPLY, a, c->stream);
    launch_dsolve_gemv(L.nfree, L.ainv, L.freeid, L.F, c->q, L.x, c->stream);
    HIPCHK(c, hipGetLastError());
    if (info) {
        info->iters = 0;
        info->rre = 0.0;
        info->nf = L.nf;
        info->status = ECMG_OK;
        info->path = ECMG_PATH_DENSE;
    }
    return ECMG_OK;
}

// ---------------------------------------------------------------------------
// autotuner: per-level JCG configuration, timed on the device, cached in JSON
// ---------------------------------------------------------------------------
// partial-sum slots for at least n values (grown when a tuned z-chunk length
// gives a stencil pass more blocks than the built-in one)
static int ensure_partials(ecmg_ctx *c, int64_t n) {
    if (n <= c->partials_n) return ECMG_OK;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    dfree(c, c->partials);
    c->partials = nullptr;
    c->partials_n = 0;
    CHK(dalloc_n(c, &c->partials, n));
    c->partials_n = n;
    return ECMG_OK;
}

// the configuration the built-in rules give level l
static TuneEntry builtin_choice(const ecmg_ctx *c, int l) {
    const Level &L = c->lv[l];
    TuneEntry e;
    if (persist_possible(c, L.g) && L.g.nreal <= c->persist_max) {
        const int seg = c->persist_seglen > 0 ? c->persist_seglen : (L.g.nreal < 131072 ? 2 : 4);
        e.path = 1;
        e.seg = seg >= 4 ? 4 : (seg >= 2 ? 2 : 1);
        e.nwg = c->persist_nwg;
    } else if (L.g.nreal <= c->gather_max && gather_possible(c, L.g)) {
        e.path = 3;
    } else {
        e.path = 0;
        e.kz = stencil_kz(L.g, c->KZ, c->kz_target);
    }
    return e;
}

// level l runs configuration e from now on (path -1: the built-in rules)
static int apply_choice(ecmg_ctx *c, int l, int path, int kz, int seg, int nwg) {
    Level &L = c->lv[l];
    c->gen = ++g_generation;
    if (path == 1 && !persist_possible(c, L.g)) path = -1;
    L.tune_path = path;
    L.tune_kz = path == 0 ? std::max(1, std::min(kz, L.g.nz + 1)) : 0;
    L.tune_seg = path == 1 ? (seg >= 4 ? 4 : (seg >= 2 ? 2 : 1)) : 0;
    L.tune_nwg = path == 1 ? std::max(1, nwg) : 0;
    if (path == 0) {
        int a, b, d;
        CHK(ensure_partials(c, 2 * (int64_t)stencil_blocks(L.g, L.tune_kz, &a, &b, &d)));
    }
    return ECMG_OK;
}

// the cached choices for this hierarchy's JCG levels (ecmg_setup, autotune = 1)
static int apply_tune_cache(ecmg_ctx *c) {
    if (c->tune_cache.empty()) return ECMG_OK;
    std::map<std::string, TuneEntry> entries;
    std::string dev, err;
    const int rc = tune_cache_read(c->tune_cache, &dev, &entries, &err);
    if (rc == ECMG_ENOENT) return ECMG_OK;        // nothing tuned yet: built-in choices
    if (rc != ECMG_OK) return fail(c, rc, "%s", err.c_str());
    for (int l = 2; l < c->nlev; ++l) {
        const Level &L = c->lv[l];
        auto it = entries.find(tune_key(c->opt.precision, L.g.nx, L.g.ny, L.g.nz));
        if (it == entries.end() || it->second.path == 2) continue;
        const TuneEntry &e = it->second;
        CHK(apply_choice(c, l, e.path, e.kz, e.seg, e.nwg));
    }
    auto bt = entries.find(tune_key_batch(c->opt.precision));   // the batched solve's choice
    if (bt != entries.end() && bt->second.path == 2) {
        c->batch_npw = bt->second.nwg;
        c->batch_seg = bt->second.seg;
    }
    return ECMG_OK;
}

// Algorithm 4 over all levels.  Every level is enqueued without waiting for
// the one before (the stream orders them); the host waits only inside the
// tiled JCG loop (one status read per chunk) and once at the end, when the
// levels' results come out of their pinned slots.  A mixed-precision level
// drives its outer refinement from the host, so the levels before it are
// settled first.
static int solve_impl(ecmg_ctx *c, double rel_tol, const int32_t *fixed, ecmg_level_info *info,
                      const double *level_tol = nullptr, bool exp_true = false) {
    if (!c) return fail(nullptr, ECMG_EINVAL, "ctx is NULL");
    if (!c->ready) return fail(c, ECMG_ESTATE, "ecmg_solve before ecmg_setup");
    if (!fixed && !level_tol && !(rel_tol >= 0.0)) return fail(c, ECMG_EINVAL, "rel_tol = %g must be >= 0", rel_tol);
    const int n = c->nlev;
    if (level_tol)
        for (int l = 2; l < n; ++l)
            if (!(level_tol[l] >= 0.0)) return fail(c, ECMG_EINVAL, "rel_tol[%d] = %g must be >= 0", l, level_tol[l]);
    // every level is computed again (the finest from EXP_finite): a pending
    // update of the previous solve is void
    c->x_pending = -1;
    std::vector<ecmg_level_info> li(n);
    std::vector<char> deferred(n, 0);        // JCG results still in the level's slot
    std::vector<int> cap(n, 0);              // their iteration caps
    std::vector<int> limit(n, 1 << 30);      // timing: iterations each level ran
    int worst = ECMG_OK, settled = 0;
    int redo = -1;                           // first level whose speculative chunk fell short
    auto note = [&](int rc) {
        if (rc != ECMG_OK && worst == ECMG_OK) worst = rc;
    };
    // wait for the stream; results and times of levels settled .. upto-1.  A
    // level enqueued without status reads that is still running fell short:
    // it and every level after it are discarded (with their timing records)
    // and `redo` names it.
    auto settle = [&](int upto) -> int {
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int k = settled; k < upto; ++k) {
            if (deferred[k] && c->lv[k].spec_live && c->sc_lv[k].done == DONE_RUNNING) {
                c->lv[k].spec_hits = 0;
                redo = k;
                upto = k;
                c->recs.erase(std::remove_if(c->recs.begin(), c->recs.end(),
                                             [k](const ecmg_ctx::Rec &r) { return r.level >= k; }),
                              c->recs.end());
                break;
            }
            if (deferred[k]) {
                int rc = jcg_result(c, k, c->sc_lv[k], cap[k], fixed == nullptr, &li[k]);
                if (k < 2 && rc == ECMG_ENOTCONV) rc = ECMG_OK;   // DSOLVE: the iterate at the cap is kept
                note(rc);
                limit[k] = li[k].iters;
            }
            float ms = 0.f;
            HIPCHK(c, hipEventElapsedTime(&ms, c->lv_ev[2 * k], c->lv_ev[2 * k + 1]));
            li[k].ms = ms;
            fill_true_residual(c, k, &li[k]);
        }
        settled = upto;
        return rec_flush_levels(c, limit);
    };
    for (int l = 0;; ++l) {
        if (l == n) {
            // EXP_true on the finest level (the last step of Algorithm 4)
            // behind the cascade, before the one wait; again after a re-solve
            if (exp_true) CHK(do_exp_true(c, n - 1));
            CHK(settle(n));
            if (redo < 0) break;
            l = redo;
            redo = -1;
            c->x_pending = -1;                   // the finest level is solved again
        }
        Level &L = c->lv[l];
        li[l].level = l;
        li[l].nx = L.g.nx;
        li[l].ny = L.g.ny;
        li[l].nz = L.g.nz;
        HIPCHK(c, hipEventRecord(c->lv_ev[2 * l], c->stream));
        int rc = ECMG_OK;
        double tol = (level_tol && l >= 2 ? level_tol[l] : rel_tol) * L.nf;
        int max_iter = c->opt.max_iter, fx = fixed ? fixed[l] : -1;
        bool jcg = true;
        if (l < 2) {
            CHK(dense_prepare(c, l));
            if (L.dense == 1) {
                rc = run_dsolve_dense(c, l, &li[l]);
                jcg = false;
            } else {
                launch_zero_free(L.g, L.x, c->stream);
                tol = c->opt.dsolve_tol * L.nf;
                max_iter = 100000;
                fx = -1;
            }
        } else {
            CHK(do_exp_finite(c, l));
            if (uses_mixed(c, l) && fx < 0) {
                CHK(settle(l));
                if (redo >= 0) {                 // a level before this one runs again first
                    l = redo - 1;
                    redo = -1;
                    continue;
                }
                rc = run_jcg_mixed(c, l, tol, max_iter, &li[l]);
                jcg = false;
            }
        }
        c->lv[l].spec_live = false;
        if (jcg) {
            // the finest level's last x update goes into EXP_true, when nothing
            // reads that x in between (the true residual does)
            const bool defer_x = exp_true && l == n - 1 && !c->opt.true_residual;
            rc = uses_persistent(c, l) ? enqueue_jcg_persistent(c, l, tol, max_iter, fx)
                                       : enqueue_jcg(c, l, tol, max_iter, fx, fixed == nullptr, defer_x);
            deferred[l] = 1;
            cap[l] = max_iter;
        }
        HIPCHK(c, hipEventRecord(c->lv_ev[2 * l + 1], c->stream));
        if (rc == ECMG_EDEVICE) return rc;
        if (c->opt.true_residual) CHK(enqueue_true_residual(c, l));
        note(rc);
    }
    if (info)
        for (int l = 0; l < n; ++l) info[l] = li[l];
    c->solved = true;
    return worst;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched solves: many independent hierarchies, level by level, with the JCG
// of every box on one level in a single launch of the queue kernel
// ---------------------------------------------------------------------------
static int batch_reserve(ecmg_ctx *c, int n) {
    if (c->bt_cap >= n) return ECMG_OK;
    dfree(c, c->bt_tasks);
    dfree(c, c->bt_sc);
    if (c->bt_sc_host) (void)hipHostFree(c->bt_sc_host);
    c->bt_tasks = nullptr;
    c->bt_sc = c->bt_sc_host = nullptr;
    c->bt_cap = 0;
    if (!c->bt_next) CHK(dalloc(c, (void **)&c->bt_next, 64));
    dfree(c, c->bt_bar);
    c->bt_bar = nullptr;
    CHK(dalloc(c, (void **)&c->bt_bar, 32 * sizeof(unsigned) * (size_t)n));
    dfree(c, c->bt_exp);
    c->bt_exp = nullptr;
    CHK(dalloc(c, (void **)&c->bt_exp, sizeof(ExpTask) * (size_t)n));
    CHK(dalloc(c, (void **)&c->bt_tasks, sizeof(PersistentTask) * (size_t)n));
    CHK(dalloc(c, (void **)&c->bt_sc, sizeof(JcgScalars) * (size_t)n));
    if (hipHostMalloc((void **)&c->bt_sc_host, sizeof(JcgScalars) * (size_t)n, hipHostMallocDefault) != hipSuccess)
        return fail(c, ECMG_ENOMEM, "pinned host allocation of %d scalars failed", n);
    c->bt_cap = n;
    return ECMG_OK;
}

// The task of level l of context c as one workgroup of the queue kernel.
static PersistentTask batch_task(ecmg_ctx *c, int l, double tol_abs, int max_iter, JcgScalars *sc) {
    Level &L = c->lv[l];
    PersistentTask t{};
    t.g = L.g;
    t.beta = L.beta;
    for (int f = 0; f < 6; ++f) t.alpha[f] = L.alpha[f];
    t.F = L.F;
    t.dinv = L.dinv;
    t.x = L.x;
    t.r = c->r;
    t.q = c->q;
    t.p[0] = c->p0;
    t.p[1] = c->p1;
    t.partials = c->partials;
    t.err = (int *)c->d_bar;
    t.bar = c->d_bar + 16;
    t.sc = sc;
    t.tol = tol_abs;
    t.max_iter = max_iter;
    t.fixed = -1;
    t.wg0 = 0;
    // about batch_npw nodes per workgroup, at most 16 workgroups per box
    t.nwg = (int)std::max<int64_t>(1, std::min<int64_t>(L.g.nreal / c->batch_npw, 16));
    const int seg = c->batch_seg > 0 ? c->batch_seg
                    : c->persist_seglen > 0 ? c->persist_seglen : (L.g.nreal < 131072 ? 2 : 4);
    t.seglen = seg >= 4 ? 4 : (seg >= 2 ? 2 : 1);         // the kernel's instantiations
    return t;
}

// Runs fn(ctx) with ctx's work redirected to stream s.
template <typename Fn>
static int on_stream(ecmg_ctx *c, hipStream_t s, Fn fn) {
    hipStream_t keep = c->stream;
    c->stream = s;
    const int rc = fn(c);
    c->stream = keep;
    return rc;
}

// ---------------------------------------------------------------------------
// Batched cascade plan: every level's EXP_finite tasks and queue-kernel tasks
// (boxes sorted by node count, each with its own scalar slot and barrier
// words) uploaded once per set of boxes and tolerance, so that a solve is one
// fixed sequence of launches -- per level: a kernel that clears the barrier
// words and queue counter, the batched EXP_finite, the cooperative queue
// kernel -- and one copy of all scalars back to pinned memory.  That sequence
// is captured once into a HIP graph and replayed by later solves.
// ---------------------------------------------------------------------------
struct BatchPlan {
    struct Lv {
        int nt = 0, items = 0, nwg = 0, nex = 0;
        int64_t nb0 = 0;
        size_t task_off = 0, sc_off = 0, bar_off = 0, exp_off = 0;
        std::vector<int> owner;                  // sorted task k -> input box
    };
    std::vector<ecmg_ctx *> ctxs;
    std::vector<uint64_t> key;                   // per box: generation, batch_npw, batch_seg
    double rel_tol = 0.0;
    int n = 0, maxlev = 0;
    std::vector<Lv> lv;
    PersistentTask *d_tasks = nullptr;
    // the whole cascade as one launch of the queue kernel: every level's tasks
    // in level order (global work items), each box's level-l task (l >= 2)
    // waiting for its levels l-1 and l-2 and building its own x = W
    PersistentTask *d_tasks1 = nullptr;
    int items1 = 0, nwg1 = 0;
    JcgScalars *d_sc = nullptr;
    JcgScalars *h_sc = nullptr;                  // pinned
    unsigned *d_bar = nullptr;                   // per level: 32 words per box (error flag 0, done
                                                 // flag 8, counter 16), then 16 words of queue
                                                 // counter; at the end the single launch's counter
    ExpTask *d_exp = nullptr;
    size_t nsc = 0, nbar = 0;
    std::vector<hipEvent_t> ev;                  // level boundaries
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_state = 0;                         // 0 not tried, 1 captured, -1 not capturable (launch by launch)
    bool timed = true;                           // per-level events in the launch sequence

    bool matches(ecmg_ctx *const *cs, int m, double tol) const {
        if (m != n || tol != rel_tol) return false;
        for (int i = 0; i < m; ++i) {
            if (cs[i] != ctxs[i] || key[3 * i] != cs[i]->gen || key[3 * i + 1] != (uint64_t)cs[i]->batch_npw ||
                key[3 * i + 2] != (uint64_t)cs[i]->batch_seg)
                return false;
        }
        return true;
    }
};

static void batch_plan_free(ecmg_ctx *c0, BatchPlan *P) {
    if (!P) return;
    if (c0->stream) (void)hipStreamSynchronize(c0->stream);
    if (P->exec) (void)hipGraphExecDestroy(P->exec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    dfree(c0, P->d_tasks);
    dfree(c0, P->d_tasks1);
    dfree(c0, P->d_sc);
    dfree(c0, P->d_bar);
    dfree(c0, P->d_exp);
    if (P->h_sc) (void)hipHostFree(P->h_sc);
    for (auto e : P->ev) (void)hipEventDestroy(e);
    delete P;
}

static int batch_plan_build(ecmg_ctx *c0, ecmg_ctx *const *ctxs, int n, double rel_tol, BatchPlan **out) {
    BatchPlan *P = new BatchPlan();
    P->n = n;
    P->rel_tol = rel_tol;
    P->ctxs.assign(ctxs, ctxs + n);
    for (int i = 0; i < n; ++i) {
        P->key.push_back(ctxs[i]->gen);
        P->key.push_back((uint64_t)ctxs[i]->batch_npw);
        P->key.push_back((uint64_t)ctxs[i]->batch_seg);
        P->maxlev = std::max(P->maxlev, ctxs[i]->nlev);
    }
    P->lv.resize(P->maxlev);
    std::vector<PersistentTask> all_tasks;
    std::vector<ExpTask> all_exp;
    size_t nbar = 0;
    for (int l = 0; l < P->maxlev; ++l) {
        BatchPlan::Lv &V = P->lv[l];
        std::vector<PersistentTask> tasks;
        std::vector<int> owner;
        V.exp_off = all_exp.size();
        for (int i = 0; i < n; ++i) {
            ecmg_ctx *c = ctxs[i];
            if (l >= c->nlev) continue;
            Level &L = c->lv[l];
            if (l >= 2) {                 // EXP_finite of every box in one launch
                ExpTask e{};
                e.gf = L.g;
                e.g1 = c->lv[l - 1].g;
                e.U1 = c->lv[l - 1].x;
                e.U0 = c->lv[l - 2].x;
                e.x = L.x;
                e.W = L.W;
                e.variant = c->opt.interp;
                exp_task_blocks(e, 0);
                e.b0[0] = V.nb0;
                V.nb0 += e.nb[0];
                all_exp.push_back(e);
                ++V.nex;
            }
            const double tol = (l < 2 ? c->opt.dsolve_tol : rel_tol) * L.nf;
            const int max_iter = l < 2 ? 100000 : c->opt.max_iter;
            tasks.push_back(batch_task(c, l, tol, max_iter, nullptr));
            tasks.back().zero_x = l < 2;
            owner.push_back(i);
        }
        if (V.nb0 >= ((int64_t)1 << 31)) {
            delete P;
            return fail(c0, ECMG_EINVAL, "batched EXP_finite grid too large");
        }
        // longest first: order by node count, then by input position
        std::vector<int> order(tasks.size());
        for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
        std::stable_sort(order.begin(), order.end(),
                         [&](int a, int b) { return tasks[a].g.nreal > tasks[b].g.nreal; });
        V.nt = (int)tasks.size();
        V.task_off = all_tasks.size();
        V.sc_off = V.task_off;
        V.bar_off = nbar;
        for (size_t k = 0; k < order.size(); ++k) {
            PersistentTask t = tasks[order[k]];
            t.nwg = std::min(t.nwg, c0->queue_blocks);
            t.wg0 = V.items;
            V.items += t.nwg;
            all_tasks.push_back(t);
            V.owner.push_back(owner[order[k]]);
        }
        V.nwg = std::max(1, std::min(V.items, c0->queue_blocks));
        nbar += 32 * (size_t)V.nt + 16;
    }
    P->nsc = all_tasks.size();
    P->nbar = nbar + 16;                         // + the single launch's queue counter
    int rc = ECMG_OK;
    if ((rc = dalloc(c0, (void **)&P->d_tasks, sizeof(PersistentTask) * std::max<size_t>(1, P->nsc))) != ECMG_OK ||
        (rc = dalloc(c0, (void **)&P->d_tasks1, sizeof(PersistentTask) * std::max<size_t>(1, P->nsc))) != ECMG_OK ||
        (rc = dalloc(c0, (void **)&P->d_sc, sizeof(JcgScalars) * std::max<size_t>(1, P->nsc))) != ECMG_OK ||
        (rc = dalloc(c0, (void **)&P->d_bar, sizeof(unsigned) * P->nbar)) != ECMG_OK ||
        (rc = dalloc(c0, (void **)&P->d_exp, sizeof(ExpTask) * std::max<size_t>(1, all_exp.size()))) != ECMG_OK) {
        batch_plan_free(c0, P);
        return rc;
    }
    if (hipHostMalloc((void **)&P->h_sc, sizeof(JcgScalars) * std::max<size_t>(1, P->nsc), hipHostMallocDefault) !=
        hipSuccess) {
        P->h_sc = nullptr;
        batch_plan_free(c0, P);
        return fail(c0, ECMG_ENOMEM, "pinned host allocation of %zu scalars failed", P->nsc);
    }
    // every task's scalar slot and barrier words inside the plan's arrays
    for (int l = 0; l < P->maxlev; ++l) {
        const BatchPlan::Lv &V = P->lv[l];
        for (int k = 0; k < V.nt; ++k) {
            PersistentTask &t = all_tasks[V.task_off + k];
            t.sc = P->d_sc + V.sc_off + k;
            t.err = (int *)(P->d_bar + V.bar_off + 32 * (size_t)k);
            t.bar = P->d_bar + V.bar_off + 32 * (size_t)k + 16;
        }
    }
    // the single launch's tasks: global work items, dependencies on the box's
    // two coarser levels (their done flags), EXP_finite inside the task
    std::vector<PersistentTask> one(all_tasks);
    {
        std::vector<std::vector<int>> slot(P->maxlev, std::vector<int>(n, -1));   // (level, box) -> task
        std::vector<std::vector<int>> exi(P->maxlev, std::vector<int>(n, -1));    // (level, box) -> ExpTask
        for (int l = 0; l < P->maxlev; ++l) {
            const BatchPlan::Lv &V = P->lv[l];
            for (int k = 0; k < V.nt; ++k) slot[l][V.owner[k]] = k;
            int e = 0;
            for (int i = 0; i < n; ++i)
                if (l >= 2 && l < ctxs[i]->nlev) exi[l][i] = e++;
        }
        int base = 0;
        for (int l = 0; l < P->maxlev; ++l) {
            const BatchPlan::Lv &V = P->lv[l];
            for (int k = 0; k < V.nt; ++k) {
                PersistentTask &t = one[V.task_off + k];
                const int i = V.owner[k];
                t.wg0 += base;
                t.flag = P->d_bar + V.bar_off + 32 * (size_t)k + 8;
                // a box's levels share its context's JCG scratch (r, q, p), so
                // they run in order: level 1 after level 0, level l >= 2 after
                // l-1 and l-2 (whose solutions its EXP_finite reads)
                for (int d = 0; d < 2 && l - 1 - d >= 0; ++d) {
                    const BatchPlan::Lv &U = P->lv[l - 1 - d];
                    t.dep[d] = P->d_bar + U.bar_off + 32 * (size_t)slot[l - 1 - d][i] + 8;
                }
                if (l >= 2) t.exp = P->d_exp + V.exp_off + exi[l][i];
            }
            base += V.items;
        }
        P->items1 = base;
        P->nwg1 = std::max(1, std::min(base, c0->queue_blocks));
    }
    for (int l = 0; l <= P->maxlev; ++l) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) {
            batch_plan_free(c0, P);
            return fail(c0, ECMG_EDEVICE, "hipEventCreate failed");
        }
        P->ev.push_back(e);
    }
    hipStream_t s = c0->stream;
    if (hipMemcpyAsync(P->d_tasks, all_tasks.data(), sizeof(PersistentTask) * P->nsc, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipMemcpyAsync(P->d_tasks1, one.data(), sizeof(PersistentTask) * P->nsc, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        (!all_exp.empty() &&
         hipMemcpyAsync(P->d_exp, all_exp.data(), sizeof(ExpTask) * all_exp.size(), hipMemcpyHostToDevice, s) !=
             hipSuccess) ||
        hipStreamSynchronize(s) != hipSuccess) {
        batch_plan_free(c0, P);
        return fail(c0, ECMG_EDEVICE, "uploading the batched plan failed");
    }
    *out = P;
    return ECMG_OK;
}

// The plan's launch sequence on stream s (eager: the cooperative launch
// interface; under capture: the launch-attribute one, recorded as a kernel node
// with the cooperative attribute).  single: the whole cascade as one launch of
// the queue kernel; else level by level (EXP_finite of every box, then the
// queue kernel over the level's tasks), with an event after each level when
// the plan is timed.
static int batch_enqueue(ecmg_ctx *c0, BatchPlan *P, hipStream_t s, bool eager, bool single) {
    if (single) {
        launch_zero_u32(P->d_bar, (int64_t)P->nbar, s);        // barrier words, flags, queue counters
        HIPCHK(c0, hipGetLastError());
        unsigned *next = P->d_bar + P->nbar - 16;
        HIPCHK(c0, eager ? launch_jcg_queue(P->d_tasks1, (int)P->nsc, P->items1, P->nwg1, next, s)
                         : launch_jcg_queue_attr(P->d_tasks1, (int)P->nsc, P->items1, P->nwg1, next, s));
        HIPCHK(c0, hipMemcpyAsync(P->h_sc, P->d_sc, sizeof(JcgScalars) * P->nsc, hipMemcpyDeviceToHost, s));
        return ECMG_OK;
    }
    for (int l = 0; l < P->maxlev; ++l) {
        const BatchPlan::Lv &V = P->lv[l];
        unsigned *bar = P->d_bar + V.bar_off;
        unsigned *next = bar + 32 * (size_t)V.nt;
        launch_zero_u32(bar, 32 * (int64_t)V.nt + 16, s);       // barrier words and queue counter
        if (V.nex > 0) launch_exp_finite_batch(P->d_exp + V.exp_off, V.nex, V.nb0, s);
        HIPCHK(c0, hipGetLastError());
        const PersistentTask *tk = P->d_tasks + V.task_off;
        HIPCHK(c0, eager ? launch_jcg_queue(tk, V.nt, V.items, V.nwg, next, s)
                         : launch_jcg_queue_attr(tk, V.nt, V.items, V.nwg, next, s));
        if (P->timed) HIPCHK(c0, hipEventRecord(P->ev[l + 1], s));
    }
    HIPCHK(c0, hipMemcpyAsync(P->h_sc, P->d_sc, sizeof(JcgScalars) * P->nsc, hipMemcpyDeviceToHost, s));
    return ECMG_OK;
}

// Capture the launch sequence into a graph (without the per-level events:
// events recorded inside a captured graph cannot be timed); graph_state -1 if
// it cannot be captured.
static int batch_plan_capture(ecmg_ctx *c0, BatchPlan *P, hipStream_t s) {
    P->timed = false;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        const int rc = batch_enqueue(c0, P, s, false, true);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(s, &g);
        if (rc == ECMG_OK && e == hipSuccess && g) {
            hipGraphExec_t x = nullptr;
            if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) == hipSuccess && x) {
                P->graph = g;
                P->exec = x;
                P->graph_state = 1;
            }
        }
        if (P->graph_state != 1 && g) (void)hipGraphDestroy(g);
    }
    (void)hipGetLastError();                 // a refused capture leaves no error behind
    if (P->graph_state != 1) {
        P->graph_state = -1;
        P->timed = true;
        c0->err.clear();
    }
    return ECMG_OK;
}

extern "C" {

int ecmg_solve_batch(ecmg_ctx *const *ctxs, int32_t n, double rel_tol, ecmg_level_info *infos) {
    if (!ctxs || n < 1) return fail(nullptr, ECMG_EINVAL, "ctxs is NULL or n = %d < 1", n);
    ecmg_ctx *c0 = ctxs[0];
    if (!c0) return fail(nullptr, ECMG_EINVAL, "ctxs[0] is NULL");
    if (!(rel_tol >= 0.0)) return fail(c0, ECMG_EINVAL, "rel_tol = %g must be >= 0", rel_tol);
    std::vector<int64_t> info_off(n);
    int64_t off = 0;
    for (int i = 0; i < n; ++i) {
        ecmg_ctx *c = ctxs[i];
        if (!c) return fail(c0, ECMG_EINVAL, "ctxs[%d] is NULL", i);
        if (!c->ready) return fail(c0, ECMG_ESTATE, "ctxs[%d]: ecmg_solve_batch before ecmg_setup", i);
        if (c->device != c0->device) return fail(c0, ECMG_EINVAL, "ctxs[%d] is on another device", i);
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == c) return fail(c0, ECMG_EINVAL, "ctxs[%d] repeats ctxs[%d]", i, j);
        info_off[i] = off;
        off += c->nlev;
    }
    if (c0->queue_blocks < 1) return fail(c0, ECMG_EDEVICE, "the queue kernel cannot be resident");
    hipStream_t s = c0->stream;
    for (int i = 0; i < n; ++i) ctxs[i]->x_pending = -1;   // every level is computed again
    for (int i = 1; i < n; ++i)
        if (ctxs[i]->stream != s) HIPCHK(c0, hipStreamSynchronize(ctxs[i]->stream));
    BatchPlan *P = c0->bplan;
    if (!P || !P->matches(ctxs, n, rel_tol)) {
        if (P) batch_plan_free(c0, P);
        c0->bplan = nullptr;
        CHK(batch_plan_build(c0, ctxs, n, rel_tol, &P));
        c0->bplan = P;
    }
    // the whole cascade is enqueued at once (one host wait): from the plan's
    // graph when it could be captured, else launch by launch
    HIPCHK(c0, hipEventRecord(P->ev[0], s));
    if (c0->opt.batch_graph && P->graph_state == 0) CHK(batch_plan_capture(c0, P, s));
    if (P->graph_state == 1) HIPCHK(c0, hipGraphLaunch(P->exec, s));
    else CHK(batch_enqueue(c0, P, s, true, false));
    HIPCHK(c0, hipStreamSynchronize(s));
    int worst = ECMG_OK;
    for (int l = 0; l < P->maxlev; ++l) {
        const BatchPlan::Lv &V = P->lv[l];
        float ms = -1.f;                     // a replayed graph: per-level device time not observable
        if (P->timed) HIPCHK(c0, hipEventElapsedTime(&ms, P->ev[l], P->ev[l + 1]));
        for (int k = 0; k < V.nt; ++k) {
            ecmg_ctx *c = ctxs[V.owner[k]];
            const Level &L = c->lv[l];
            const JcgScalars &sc = P->h_sc[V.sc_off + k];
            ecmg_level_info li{};
            li.rre_true = -1.0;              // not computed by the batched form
            li.level = l;
            li.nx = L.g.nx;
            li.ny = L.g.ny;
            li.nz = L.g.nz;
            li.iters = sc.iter;
            li.rre = (L.nf > 0) ? std::sqrt(sc.rr) / L.nf : 0.0;
            li.nf = L.nf;
            li.ms = ms;
            int st = (sc.done == DONE_BREAKDOWN) ? ECMG_EBREAKDOWN : (sc.done == DONE_MAXITER) ? ECMG_ENOTCONV : ECMG_OK;
            if (l < 2 && st == ECMG_ENOTCONV) st = ECMG_OK;   // DSOLVE: the iterate at the cap is kept
            li.status = st;
            li.path = ECMG_PATH_QUEUE;
            if (infos) infos[info_off[V.owner[k]] + l] = li;
            if (st != ECMG_OK && worst == ECMG_OK) worst = st;
        }
    }
    for (int i = 0; i < n; ++i) {
        ctxs[i]->solved = true;
        CHK(on_stream(ctxs[i], s, [&](ecmg_ctx *cc) { return rec_flush(cc, 1); }));
    }
    if (worst != ECMG_OK) return fail(c0, worst, "batched solve: some box did not converge (see infos)");
    return ECMG_OK;
}

int ecmg_extrapolate_batch(ecmg_ctx *const *ctxs, int32_t n) {
    if (!ctxs || n < 1) return fail(nullptr, ECMG_EINVAL, "ctxs is NULL or n = %d < 1", n);
    ecmg_ctx *c0 = ctxs[0];
    if (!c0) return fail(nullptr, ECMG_EINVAL, "ctxs[0] is NULL");
    hipStream_t s = c0->stream;
    for (int i = 0; i < n; ++i) {
        ecmg_ctx *c = ctxs[i];
        if (!c || !c->ready) return fail(c0, ECMG_ESTATE, "ctxs[%d] is NULL or not set up", i);
        if (c->device != c0->device) return fail(c0, ECMG_EINVAL, "ctxs[%d] is on another device", i);
        if (c->nlev < 2) return fail(c0, ECMG_EINVAL, "ctxs[%d] has fewer than 2 levels", i);
        // U~ is allocated (and zeroed on ctx's own stream) before that stream
        // is waited for: the batched kernel below runs on ctxs[0]'s stream
        CHK(flush_x(c));
        Level &L = c->lv[c->nlev - 1];
        if (!L.Ut) CHK(dalloc_n(c, &L.Ut, L.g.nnodes));
        if (c->stream != s) HIPCHK(c0, hipStreamSynchronize(c->stream));
    }
    CHK(batch_reserve(c0, n));
    std::vector<ExpTask> ex(n);
    int64_t nb1 = 0;
    for (int i = 0; i < n; ++i) {
        ecmg_ctx *c = ctxs[i];
        Level &L = c->lv[c->nlev - 1];
        ExpTask &e = ex[i];
        e.gf = L.g;
        e.g1 = c->lv[c->nlev - 2].g;
        e.U1 = L.x;
        e.U0 = c->lv[c->nlev - 2].x;
        e.x = L.Ut;
        exp_task_blocks(e, 1);
        e.b0[1] = nb1;
        nb1 += e.nb[1];
    }
    if (nb1 >= ((int64_t)1 << 31)) return fail(c0, ECMG_EINVAL, "batched EXP_true grid too large");
    HIPCHK(c0, hipMemcpyAsync(c0->bt_exp, ex.data(), sizeof(ExpTask) * n, hipMemcpyHostToDevice, s));
    launch_exp_true_batch(c0->bt_exp, n, nb1, s);
    HIPCHK(c0, hipGetLastError());
    HIPCHK(c0, hipStreamSynchronize(s));
    return ECMG_OK;
}

int ecmg_solve(ecmg_ctx *c, double rel_tol, ecmg_level_info *info) { return solve_impl(c, rel_tol, nullptr, info); }

int ecmg_solve_extrapolated(ecmg_ctx *c, double rel_tol, ecmg_level_info *info) {
    return solve_impl(c, rel_tol, nullptr, info, nullptr, true);
}

int ecmg_solve_fixed(ecmg_ctx *c, const int32_t *iters, ecmg_level_info *info) {
    if (!iters) return fail(c, ECMG_EINVAL, "iters is NULL");
    return solve_impl(c, 0.0, iters, info);
}

int ecmg_solve_levels(ecmg_ctx *c, const double *rel_tol, ecmg_level_info *info) {
    if (!rel_tol) return fail(c, ECMG_EINVAL, "rel_tol is NULL");
    return solve_impl(c, 0.0, nullptr, info, rel_tol);
}

int ecmg_tolerance_schedule(int32_t levels, double eps_finest, double ratio, double *rel_tol) {
    if (!rel_tol) return fail(nullptr, ECMG_EINVAL, "ecmg_tolerance_schedule: rel_tol is NULL");
    if (levels < 3 || !(eps_finest > 0.0) || !(ratio >= 1.0) || !std::isfinite(eps_finest) || !std::isfinite(ratio))
        return fail(nullptr, ECMG_EINVAL, "ecmg_tolerance_schedule: need levels >= 3, eps_finest > 0, ratio >= 1");
    rel_tol[0] = rel_tol[1] = 0.0;                // DSOLVE grids: options.dsolve_tol applies
    for (int l = 2; l < levels; ++l) {
        double e = eps_finest;
        for (int k = l; k < levels - 1; ++k) e *= ratio;
        rel_tol[l] = std::min(e, 1.0);
    }
    return ECMG_OK;
}

static int check_level(ecmg_ctx *c, int32_t *level, int min_level) {
    if (!c) return fail(nullptr, ECMG_EINVAL, "ctx is NULL");
    if (!c->ready) return fail(c, ECMG_ESTATE, "call before ecmg_setup");
    if (*level < 0) *level = c->nlev - 1;
    if (*level < min_level || *level >= c->nlev)
        return fail(c, ECMG_EINVAL, "level %d out of range [%d, %d)", *level, min_level, c->nlev);
    return flush_x(c);               // the caller reads or replaces level data
}

int ecmg_extrapolate(ecmg_ctx *c, int32_t level, double *host_out) {
    CHK(check_level(c, &level, 1));
    CHK(do_exp_true(c, level));                   // its timing record is folded later (no wait here)
    Level &L = c->lv[level];
    if (host_out) {
        HIPCHK(c, copy_out(L.g, host_out, L.Ut, c->r, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return ECMG_OK;
}

int ecmg_prolongate(ecmg_ctx *c, int32_t level) {
    CHK(check_level(c, &level, 2));
    CHK(do_exp_finite(c, level));
    CHK(rec_flush(c, 1));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return ECMG_OK;
}

int ecmg_jcg(ecmg_ctx *c, int32_t level, double rel_tol, int32_t fixed_iters, ecmg_level_info *info) {
    CHK(check_level(c, &level, 0));
    Level &L = c->lv[level];
    ecmg_level_info li{};
    li.level = level;
    li.nx = L.g.nx;
    li.ny = L.g.ny;
    li.nz = L.g.nz;
    const int rc = run_level_jcg(c, level, rel_tol * L.nf, c->opt.max_iter, fixed_iters, &li);
    if (rc == ECMG_EDEVICE) return rc;
    if (c->opt.true_residual) CHK(enqueue_true_residual(c, level));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    fill_true_residual(c, level, &li);
    if (info) *info = li;
    return rc;
}

static double *vec_ptr(ecmg_ctx *c, Level &L, int which) {
    switch (which) {
        case ECMG_VEC_U: return L.x;
        case ECMG_VEC_W: return L.W;
        case ECMG_VEC_UTILDE: return L.Ut;
        case ECMG_VEC_F: return L.F;
        case ECMG_VEC_DINV: return L.dinv;
        default: return nullptr;
    }
}

int ecmg_get(ecmg_ctx *c, int32_t level, int32_t which, double *host_out) {
    CHK(check_level(c, &level, 0));
    if (!host_out) return fail(c, ECMG_EINVAL, "host_out is NULL");
    Level &L = c->lv[level];
    double *d = vec_ptr(c, L, which);
    if (!d) return fail(c, ECMG_EINVAL, "vector %d is not available on level %d", which, level);
    HIPCHK(c, copy_out(L.g, host_out, d, c->r, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return ECMG_OK;
}

int ecmg_set(ecmg_ctx *c, int32_t level, int32_t which, const double *host_in) {
    CHK(check_level(c, &level, 0));
    if (!host_in) return fail(c, ECMG_EINVAL, "host_in is NULL");
    Level &L = c->lv[level];
    if (which == ECMG_VEC_UTILDE && !L.Ut) CHK(dalloc_n(c, &L.Ut, L.g.nnodes));
    if (which == ECMG_VEC_W && !L.W) CHK(dalloc_n(c, &L.W, L.g.nnodes));
    double *d = vec_ptr(c, L, which);
    if (!d || which == ECMG_VEC_F || which == ECMG_VEC_DINV)
        return fail(c, ECMG_EINVAL, "vector %d cannot be set", which);
    HIPCHK(c, copy_in(L.g, d, host_in, c->r, c->stream, hipMemcpyHostToDevice));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return ECMG_OK;
}

int ecmg_device_view(ecmg_ctx *c, int32_t level, int32_t which, void **dptr, int64_t dims[3],
                     int64_t *row_pitch_out) {
    CHK(check_level(c, &level, 0));
    if (!dptr) return fail(c, ECMG_EINVAL, "dptr is NULL");
    Level &L = c->lv[level];
    double *d = vec_ptr(c, L, which);
    if (!d) return fail(c, ECMG_EINVAL, "vector %d is not available on level %d", which, level);
    *dptr = d;
    if (dims) {
        dims[0] = L.g.nx + 1;
        dims[1] = L.g.ny + 1;
        dims[2] = L.g.nz + 1;
    }
    if (row_pitch_out) *row_pitch_out = L.g.sx;
    return ECMG_OK;
}

int ecmg_apply(ecmg_ctx *c, int32_t level, const double *host_in, double *host_out) {
    CHK(check_level(c, &level, 0));
    if (!host_in || !host_out) return fail(c, ECMG_EINVAL, "NULL buffer");
    Level &L = c->lv[level];
    HIPCHK(c, copy_in(L.g, c->p0, host_in, c->r, c->stream, hipMemcpyHostToDevice));
    StencilArgs<double> a = stencil_args(c, L);
    a.v = c->p0;
    a.q = c->q;
    launch_stencil<double>(MODE_APPLY, a, c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, copy_out(L.g, host_out, c->q, c->r, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return ECMG_OK;
}

int ecmg_norms(ecmg_ctx *c, int32_t level, int32_t which, int32_t minus_which, const double *minus,
               int32_t minus_on_device, double out[2]) {
    CHK(check_level(c, &level, 0));
    if (!out) return fail(c, ECMG_EINVAL, "out is NULL");
    Level &L = c->lv[level];
    const double *a = vec_ptr(c, L, which);
    if (!a) return fail(c, ECMG_EINVAL, "vector %d is not available on level %d", which, level);
    const double *b = nullptr;
    if (minus_which != ECMG_VEC_NONE) {
        b = vec_ptr(c, L, minus_which);
        if (!b) return fail(c, ECMG_EINVAL, "vector %d is not available on level %d", minus_which, level);
    }
    const double *h = nullptr;
    if (minus) {   // dense node array (host or device) into the padded layout
        HIPCHK(c, copy_in(L.g, c->q, minus, c->r, c->stream,
                          minus_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice));
        h = c->q;
    }
    launch_norms(L.g, a, b, h, c->partials, c->counters + 2, c->dres, c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(c->hres, c->dres, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    out[0] = c->hres[0];
    out[1] = std::sqrt(c->hres[1] / (double)L.g.nreal);
    return ECMG_OK;
}

int ecmg_norms_noalloc(ecmg_ctx *c, int32_t level, int32_t which, int32_t minus_which, double out[2]) {
    CHK(check_level(c, &level, 0));
    if (!out) return fail(c, ECMG_EINVAL, "out is NULL");
    Level &L = c->lv[level];
    const double *a = vec_ptr(c, L, which);
    if (!a) return fail(c, ECMG_EINVAL, "vector %d is not available on level %d", which, level);
    const double *b = nullptr;
    if (minus_which != ECMG_VEC_NONE) {
        b = vec_ptr(c, L, minus_which);
        if (!b) return fail(c, ECMG_EINVAL, "vector %d is not available on level %d", minus_which, level);
    }
    if (reduce_blocks(L.g.nnodes) > NOALLOC_BLOCKS)
        return fail(c, ECMG_EINVAL, "level %d: %d reduction blocks exceed the static scratch (%d)", level,
                    reduce_blocks(L.g.nnodes), NOALLOC_BLOCKS);
    unsigned char *base = (unsigned char *)g_scratch_ptr[c->device];   // set by ecmg_create
    double *partials = (double *)base;
    double *totals = partials + NOALLOC_TOTALS;
    unsigned *counter = (unsigned *)(partials + NOALLOC_COUNTER);
    hipLaunchKernelGGL(k_noalloc_clear, dim3(1), dim3(64), 0, c->stream, counter);
    launch_norms(L.g, a, b, nullptr, partials, counter, totals, c->stream);
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(c->hres, totals, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    out[0] = c->hres[0];
    out[1] = std::sqrt(c->hres[1] / (double)L.g.nreal);
    return ECMG_OK;
}

int ecmg_level_dims(ecmg_ctx *c, int32_t level, int64_t n[3]) {
    CHK(check_level(c, &level, 0));
    if (!n) return fail(c, ECMG_EINVAL, "n is NULL");
    n[0] = c->lv[level].g.nx;
    n[1] = c->lv[level].g.ny;
    n[2] = c->lv[level].g.nz;
    return ECMG_OK;
}

int ecmg_kernel_times(ecmg_ctx *c, int32_t level, int32_t k, double out[2]) {
    CHK(check_level(c, &level, 0));
    if (k < 0 || k >= NKIND || !out) return fail(c, ECMG_EINVAL, "bad kernel class %d", k);
    CHK(rec_flush(c, 1 << 30));                   // records still pending (EXP_true, EXP_finite)
    out[0] = c->lv[level].kt_ms[k];
    out[1] = (double)c->lv[level].kt_n[k];
    return ECMG_OK;
}

int ecmg_reset_kernel_times(ecmg_ctx *c) {
    if (!c) return fail(nullptr, ECMG_EINVAL, "ctx is NULL");
    CHK(rec_flush(c, 1 << 30));                   // pending records belong before the reset
    for (auto &L : c->lv)
        for (int k = 0; k < NKIND; ++k) {
            L.kt_ms[k] = 0.0;
            L.kt_n[k] = 0;
        }
    return ECMG_OK;
}

int ecmg_set_timing(ecmg_ctx *c, int32_t mask) {
    if (!c) return fail(nullptr, ECMG_EINVAL, "ctx is NULL");
    c->timing_mask = (uint32_t)mask & ((1u << NKIND) - 1u);
    return ECMG_OK;
}

int ecmg_autotune(ecmg_ctx *c, int32_t iters, const char *cache_path, ecmg_tune_result *out) {
    if (!c) return fail(nullptr, ECMG_EINVAL, "ctx is NULL");
    if (!c->ready) return fail(c, ECMG_ESTATE, "ecmg_autotune before ecmg_setup");
    CHK(flush_x(c));
    const int fixed_iters = iters;
    const std::string path = cache_path ? std::string(cache_path) : c->tune_cache;
    std::map<std::string, TuneEntry> entries;
    if (!path.empty()) {
        std::string dev, err;
        // an unreadable or foreign file is replaced; entries of another device are dropped
        if (tune_cache_read(path, &dev, &entries, &err) != ECMG_OK || dev != c->device_name) entries.clear();
    }
    int64_t maxn = 0;
    for (int l = 2; l < c->nlev; ++l) maxn = std::max<int64_t>(maxn, c->lv[l].g.nnodes);
    // no per-launch event records while tuning: they would lengthen the
    // launch-bound candidates (and nothing the tuner runs is a solve to account)
    const uint32_t saved_mask = c->timing_mask;
    CHK(rec_flush(c, 1 << 30));
    c->timing_mask = 0;
    struct RestoreMask {
        ecmg_ctx *c;
        uint32_t m;
        ~RestoreMask() { c->timing_mask = m; }
    } restore_mask{c, saved_mask};
    double *save = nullptr;
    CHK(dalloc_n(c, &save, std::max<int64_t>(maxn, 1)));
    struct Cand { int path, kz, seg, nwg; };
    int rc = ECMG_OK;
    for (int l = 2; l < c->nlev && rc == ECMG_OK; ++l) {
        Level &L = c->lv[l];
        const size_t bytes = sizeof(double) * (size_t)L.g.nnodes;
        if (hipMemcpyAsync(save, L.x, bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess) {
            rc = fail(c, ECMG_EDEVICE, "autotune: copy of level %d failed", l);
            break;
        }
        // the run length: as asked, else the level's iterations in the last solve, else 8
        iters = fixed_iters > 0 ? fixed_iters : (L.last_iters > 0 ? std::min(L.last_iters, 4000) : 8);
        std::vector<Cand> cands{{-1, 0, 0, 0}};   // the built-in configuration first
        for (int kz : {1, 2, 4, 8, 16, 32, 64})
            if (kz <= L.g.nz + 1) cands.push_back({0, kz, 0, 0});
        if (gather_possible(c, L.g)) cands.push_back({3, 0, 0, 0});
        if (persist_possible(c, L.g) && L.g.nreal <= 20000000)
            for (int seg : {2, 4})
                for (int nwg : {32, 64, 128, 256})
                    if (nwg <= c->persist_blocks) cands.push_back({1, 0, seg, nwg});
        double best = 0.0, us_default = 0.0;
        int bi = -1;
        for (size_t ci = 0; ci < cands.size() && rc == ECMG_OK; ++ci) {
            const Cand &cd = cands[ci];
            if ((rc = apply_choice(c, l, cd.path, cd.kz, cd.seg, cd.nwg)) != ECMG_OK) break;
            double us = -1.0;
            for (int rep = 0; rep < 2; ++rep) {       // one untimed run, one timed
                if (hipMemcpyAsync(L.x, save, bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess ||
                    hipEventRecord(c->ev0, c->stream) != hipSuccess) {
                    rc = fail(c, ECMG_EDEVICE, "autotune: restore of level %d failed", l);
                    break;
                }
                ecmg_level_info li{};
                li.rre_true = -1.0;
                const int jr = run_level_jcg(c, l, 0.0, iters + 1, iters, &li);
                if (jr == ECMG_EDEVICE) {
                    rc = jr;
                    break;
                }
                float ms = 0.f;
                if (hipEventRecord(c->ev1, c->stream) != hipSuccess || hipEventSynchronize(c->ev1) != hipSuccess ||
                    hipEventElapsedTime(&ms, c->ev0, c->ev1) != hipSuccess) {
                    rc = fail(c, ECMG_EDEVICE, "autotune: timing of level %d failed", l);
                    break;
                }
                us = (jr == ECMG_OK && li.iters == iters) ? 1e3 * ms / iters : -1.0;   // breakdown: no time
            }
            if (rc != ECMG_OK) break;
            if (ci == 0) us_default = us;
            if (us > 0.0 && (bi < 0 || us < best)) {
                best = us;
                bi = (int)ci;
            }
        }
        if (rc == ECMG_OK) {
            // keep the fastest (as a concrete configuration); none timed: built-in
            TuneEntry e = builtin_choice(c, l);
            if (bi > 0) {
                e.path = cands[bi].path;
                e.kz = cands[bi].kz;
                e.seg = cands[bi].seg;
                e.nwg = cands[bi].nwg;
            }
            e.us_default = us_default;
            e.us_best = bi >= 0 ? best : us_default;
            rc = apply_choice(c, l, bi > 0 ? e.path : -1, e.kz, e.seg, e.nwg);
            if (bi >= 0) entries[tune_key(c->opt.precision, L.g.nx, L.g.ny, L.g.nz)] = e;
            if (out) {
                ecmg_tune_result &r = out[l - 2];
                r.level = l;
                r.path = e.path;
                r.kz = e.kz;
                r.seg = e.seg;
                r.nwg = e.nwg;
                r.candidates = (int32_t)cands.size();
                r.us_default = e.us_default;
                r.us_best = e.us_best;
            }
        }
        // the level's iterate as it was
        if (hipMemcpyAsync(L.x, save, bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess && rc == ECMG_OK)
            rc = fail(c, ECMG_EDEVICE, "autotune: restore of level %d failed", l);
    }
    if (hipStreamSynchronize(c->stream) != hipSuccess && rc == ECMG_OK)
        rc = fail(c, ECMG_EDEVICE, "autotune: stream synchronisation failed");
    dfree(c, save);
    c->solved = false;
    if (rc != ECMG_OK) return rc;
    if (!path.empty()) {
        std::string err;
        const int wr = tune_cache_write(path, c->device_name, entries, &err);
        if (wr != ECMG_OK) return fail(c, wr, "%s", err.c_str());
    }
    return ECMG_OK;
}

int ecmg_autotune_batch(ecmg_ctx *const *ctxs, int32_t n, double rel_tol, const char *cache_path,
                        ecmg_tune_result *out) {
    if (!ctxs || n < 1 || !ctxs[0]) return fail(nullptr, ECMG_EINVAL, "ctxs is NULL or n = %d < 1", n);
    ecmg_ctx *c0 = ctxs[0];
    for (int i = 0; i < n; ++i)
        if (!ctxs[i] || !ctxs[i]->ready) return fail(c0, ECMG_ESTATE, "ecmg_autotune_batch: ctxs[%d] not set up", i);
    const std::string path = cache_path ? std::string(cache_path) : c0->tune_cache;
    struct Cand { int npw, seg; };
    std::vector<Cand> cands{{c0->batch_npw, c0->batch_seg}};   // the current configuration first
    for (int npw : {2048, 4096, 8192, 16384, 32768})
        for (int seg : {2, 4}) cands.push_back({npw, seg});
    auto set_all = [&](const Cand &cd) {
        for (int i = 0; i < n; ++i) {
            ctxs[i]->batch_npw = cd.npw;
            ctxs[i]->batch_seg = cd.seg;
        }
    };
    double best = 0.0, us_default = 0.0;
    int bi = -1, rc = ECMG_OK;
    for (size_t ci = 0; ci < cands.size() && rc == ECMG_OK; ++ci) {
        set_all(cands[ci]);
        double us = -1.0;
        for (int rep = 0; rep < 2; ++rep) {          // one untimed solve, one timed (synchronous)
            const auto t0 = std::chrono::steady_clock::now();
            const int sr = ecmg_solve_batch(ctxs, n, rel_tol, nullptr);
            const auto t1 = std::chrono::steady_clock::now();
            if (sr == ECMG_EDEVICE || sr == ECMG_EINVAL || sr == ECMG_ESTATE || sr == ECMG_ENOMEM) {
                rc = sr;
                break;
            }
            us = sr == ECMG_OK ? std::chrono::duration<double, std::micro>(t1 - t0).count() : -1.0;
        }
        if (rc != ECMG_OK) break;
        if (ci == 0) us_default = us;
        if (us > 0.0 && (bi < 0 || us < best)) {
            best = us;
            bi = (int)ci;
        }
    }
    const Cand chosen = bi >= 0 ? cands[bi] : cands[0];
    set_all(chosen);
    if (rc != ECMG_OK) return rc;
    if (out) {
        *out = ecmg_tune_result{};
        out->level = -1;
        out->path = 2;
        out->seg = chosen.seg;
        out->nwg = chosen.npw;
        out->candidates = (int32_t)cands.size();
        out->us_default = us_default;
        out->us_best = bi >= 0 ? best : us_default;
    }
    if (!path.empty() && bi >= 0) {
        std::map<std::string, TuneEntry> entries;
        std::string dev, err;
        if (tune_cache_read(path, &dev, &entries, &err) != ECMG_OK || dev != c0->device_name) entries.clear();
        TuneEntry e;
        e.path = 2;
        e.seg = chosen.seg;                            // 0: by box size
        e.nwg = chosen.npw;
        e.us_default = us_default;
        e.us_best = best;
        entries[tune_key_batch(c0->opt.precision)] = e;
        const int wr = tune_cache_write(path, c0->device_name, entries, &err);
        if (wr != ECMG_OK) return fail(c0, wr, "%s", err.c_str());
    }
    return ECMG_OK;
}

int ecmg_tune_lookup(const char *path, int32_t precision, int32_t nx, int32_t ny, int32_t nz,
                     ecmg_tune_result *out) {
    if (!path || !out) return fail(nullptr, ECMG_EINVAL, "ecmg_tune_lookup: path or out is NULL");
    std::map<std::string, TuneEntry> entries;
    std::string dev, err;
    const int rc = tune_cache_read(path, &dev, &entries, &err);
    if (rc != ECMG_OK) return fail(nullptr, rc, "%s", err.c_str());
    auto it = entries.find(tune_key(precision, nx, ny, nz));
    if (it == entries.end())
        return fail(nullptr, ECMG_ENOENT, "no tuning entry for %s", tune_key(precision, nx, ny, nz).c_str());
    const TuneEntry &e = it->second;
    out->level = -1;
    out->path = e.path;
    out->kz = e.kz;
    out->seg = e.seg;
    out->nwg = e.nwg;
    out->candidates = 0;
    out->us_default = e.us_default;
    out->us_best = e.us_best;
    return ECMG_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// serving loop: continuous batching of independent requests
// ---------------------------------------------------------------------------
namespace {
using Clock = std::chrono::steady_clock;

// contexts of finished requests the server keeps per grid shape for reuse
constexpr int SERVER_IDLE_PER_SHAPE = 4;

struct ServerReq {
    uint64_t ticket = 0;
    ecmg_problem prob{};
    double rel_tol = 0.0;
    double *host_out = nullptr;
    size_t bytes = 0;
    ecmg_ctx *ctx = nullptr;
    int level = 0;                     // next level to solve
    int state = 0;                     // 0 queued, 1 running, 2 done, < 0 error status
    std::vector<ecmg_level_info> info;
    Clock::time_point t_submit, t_done;
};
}  // namespace

struct ecmg_server {
    ecmg_options opt{};
    std::string tune_cache;            // owned copy of opt.tune_cache (request contexts are created later)
    size_t budget = 0, used = 0;
    hipStream_t stream = nullptr;      // the solve steps of every request
    hipStream_t setup_stream = nullptr;  // discretisation of requests, beside the solve steps
    int device = 0;
    ecmg_ctx *lead = nullptr;          // holds the queue-kernel buffers
    std::mutex mu;                     // guards queue, ready, used, tickets and statistics
    std::condition_variable cv;        // queue, budget, ready or stop changed
    std::thread setup_thread;
    bool stop = false;
    int in_setup = 0;                  // requests the setup thread holds
    std::deque<ServerReq *> queue;
    std::deque<ServerReq *> ready;     // set up, joining the active set at the next step
    std::vector<ServerReq *> active;
    std::deque<uint64_t> finished;     // tickets done or failed, not yet drained
    // contexts of finished requests kept for the next request with the same
    // grids (its set-up takes the arrays back); their bytes stay in `used`
    struct Idle {
        ecmg_ctx *ctx;
        int32_t n0[3], levels;
        size_t bytes;
    };
    std::deque<Idle> idle;
    size_t idle_bytes = 0;
    // host time since creation or the last reset: set-up (set-up thread),
    // steps' level work and finishing (calling thread), in ms
    double t_setup = 0.0, t_tick = 0.0, t_finish = 0.0;
    std::unordered_map<uint64_t, ServerReq *> reqs;
    uint64_t next_ticket = 1;
    std::vector<double> lat_ms;
    bool have_t0 = false;
    Clock::time_point t0, t_last;
    int64_t ndone = 0;
};

// Finish a request: EXP_true on its finest level, U~ to the caller's buffer,
// hierarchy freed.
static int server_complete(ecmg_server *S, ServerReq *r) {
    ecmg_ctx *c = r->ctx;
    const int L = c->nlev - 1;
    int rc = ECMG_OK;
    if (L >= 1) rc = do_exp_true(c, L);
    if (rc == ECMG_OK && r->host_out) {
        const Level &F = c->lv[L];
        if (copy_out(F.g, r->host_out, F.Ut, c->r, c->stream) != hipSuccess)
            rc = fail(c, ECMG_EDEVICE, "copy of U~ failed");
    }
    if (rc == ECMG_OK && hipStreamSynchronize(c->stream) != hipSuccess) rc = fail(c, ECMG_EDEVICE, "sync failed");
    r->ctx = nullptr;
    bool keep = false;
    {
        std::lock_guard<std::mutex> g(S->mu);
        r->t_done = Clock::now();
        r->state = rc == ECMG_OK ? 2 : rc;
        S->finished.push_back(r->ticket);
        if (rc == ECMG_OK) {
            S->lat_ms.push_back(std::chrono::duration<double, std::milli>(r->t_done - r->t_submit).count());
            ++S->ndone;
            S->t_last = r->t_done;
        }
        int same = 0;
        for (const auto &e : S->idle)
            same += e.levels == r->prob.levels && e.n0[0] == r->prob.n0[0] && e.n0[1] == r->prob.n0[1] &&
                    e.n0[2] == r->prob.n0[2];
        keep = rc == ECMG_OK && same < SERVER_IDLE_PER_SHAPE;
        if (keep) {
            S->idle.push_back({c, {r->prob.n0[0], r->prob.n0[1], r->prob.n0[2]}, r->prob.levels, r->bytes});
            S->idle_bytes += r->bytes;
        } else {
            S->used -= r->bytes;
        }
    }
    if (!keep) ecmg_destroy(c);
    S->cv.notify_all();                // budget freed or a context to reuse
    return rc;
}

// The setup thread: admits queued requests first come first served while
// their hierarchies fit the budget and discretises each on the setup stream
// (field callbacks run on this thread), so that the set-up of new requests
// overlaps the solve steps of admitted ones.  A request joins the active set
// at the next step after its set-up has completed on the device.
static void server_setup_loop(ecmg_server *S) {
    (void)hipSetDevice(S->device);
    for (;;) {
        ServerReq *r = nullptr;
        ecmg_ctx *reuse = nullptr;
        std::vector<ecmg_ctx *> evict;
        {
            // the budget counts kept contexts, which can be given up
            std::unique_lock<std::mutex> g(S->mu);
            S->cv.wait(g, [S] {
                return S->stop ||
                       (!S->queue.empty() && S->used - S->idle_bytes + S->queue.front()->bytes <= S->budget);
            });
            if (S->stop) return;
            r = S->queue.front();
            S->queue.pop_front();
            for (auto it = S->idle.begin(); it != S->idle.end(); ++it)
                if (it->levels == r->prob.levels && it->n0[0] == r->prob.n0[0] && it->n0[1] == r->prob.n0[1] &&
                    it->n0[2] == r->prob.n0[2]) {
                    reuse = it->ctx;
                    S->used -= it->bytes;
                    S->idle_bytes -= it->bytes;
                    S->idle.erase(it);
                    break;
                }
            while (S->used + r->bytes > S->budget && !S->idle.empty()) {   // oldest kept contexts first
                evict.push_back(S->idle.front().ctx);
                S->used -= S->idle.front().bytes;
                S->idle_bytes -= S->idle.front().bytes;
                S->idle.pop_front();
            }
            S->used += r->bytes;
            ++S->in_setup;
        }
        const auto t_begin = Clock::now();
        for (ecmg_ctx *e : evict) ecmg_destroy(e);
        int rc = ECMG_OK;
        if (reuse) {
            r->ctx = reuse;
            r->ctx->stream = S->setup_stream;
        } else {
            ecmg_options o = S->opt;
            o.hip_stream = S->setup_stream;
            rc = ecmg_create(&o, &r->ctx);
        }
        if (rc == ECMG_OK) rc = ecmg_setup(r->ctx, &r->prob);
        if (rc == ECMG_OK && hipStreamSynchronize(S->setup_stream) != hipSuccess) rc = ECMG_EDEVICE;
        if (rc == ECMG_OK) {
            r->ctx->stream = S->stream;          // its solve steps run on the server's stream
        } else if (r->ctx) {
            ecmg_destroy(r->ctx);
            r->ctx = nullptr;
        }
        {
            std::lock_guard<std::mutex> g(S->mu);
            S->t_setup += std::chrono::duration<double, std::milli>(Clock::now() - t_begin).count();
            --S->in_setup;
            if (rc == ECMG_OK) {
                r->state = 1;
                S->ready.push_back(r);
            } else {
                r->state = rc;
                S->used -= r->bytes;
                S->finished.push_back(r->ticket);
            }
        }
        S->cv.notify_all();
    }
}

// One tick: the current level of every active request.  Levels the persistent
// kernel handles (small grids) of all requests run together in one launch of
// the queue kernel, after one batched EXP_finite launch; larger levels run the
// tiled JCG of their own request on the same stream.
static int server_tick(ecmg_server *S) {
    ecmg_ctx *c0 = S->lead;
    hipStream_t s = S->stream;
    std::vector<ServerReq *> small, big;
    for (ServerReq *r : S->active) (uses_persistent(r->ctx, r->level) ? small : big).push_back(r);
    const auto t_start = Clock::now();
    const int n = (int)small.size();
    std::vector<int> order(n);
    if (n > 0) {
        CHK(batch_reserve(c0, n));
        std::vector<PersistentTask> tasks(n);
        std::vector<ExpTask> ex;
        int64_t nb0 = 0;
        for (int k = 0; k < n; ++k) {
            ServerReq *r = small[k];
            ecmg_ctx *c = r->ctx;
            const int l = r->level;
            Level &L = c->lv[l];
            if (l >= 2) {
                ExpTask e{};
                e.gf = L.g;
                e.g1 = c->lv[l - 1].g;
                e.U1 = c->lv[l - 1].x;
                e.U0 = c->lv[l - 2].x;
                e.x = L.x;
                e.W = L.W;
                e.variant = c->opt.interp;
                exp_task_blocks(e, 0);
                e.b0[0] = nb0;
                nb0 += e.nb[0];
                ex.push_back(e);
            }
            const double tol = (l < 2 ? c->opt.dsolve_tol : r->rel_tol) * L.nf;
            tasks[k] = batch_task(c, l, tol, l < 2 ? 100000 : c->opt.max_iter, nullptr);
            tasks[k].zero_x = l < 2;
        }
        for (int k = 0; k < n; ++k) order[k] = k;
        std::stable_sort(order.begin(), order.end(),
                         [&](int x, int y) { return tasks[x].g.nreal > tasks[y].g.nreal; });
        std::vector<PersistentTask> sorted(n);
        int items = 0;
        for (int k = 0; k < n; ++k) {
            sorted[k] = tasks[order[k]];
            sorted[k].sc = c0->bt_sc + k;
            sorted[k].err = (int *)(c0->bt_bar + 32 * k);
            sorted[k].bar = c0->bt_bar + 32 * k + 16;
            sorted[k].nwg = std::min(sorted[k].nwg, c0->queue_blocks);
            sorted[k].wg0 = items;
            items += sorted[k].nwg;
        }
        if (!ex.empty()) {
            if (nb0 >= ((int64_t)1 << 31))
                return fail(c0, ECMG_EINVAL, "batched EXP_finite grid too large");
            HIPCHK(c0, hipMemcpyAsync(c0->bt_exp, ex.data(), sizeof(ExpTask) * ex.size(), hipMemcpyHostToDevice, s));
            launch_exp_finite_batch(c0->bt_exp, (int)ex.size(), nb0, s);
            HIPCHK(c0, hipGetLastError());
        }
        HIPCHK(c0, hipMemsetAsync(c0->bt_bar, 0, 32 * sizeof(unsigned) * (size_t)n, s));
        HIPCHK(c0, hipMemcpyAsync(c0->bt_tasks, sorted.data(), sizeof(PersistentTask) * n, hipMemcpyHostToDevice, s));
        HIPCHK(c0, hipMemsetAsync(c0->bt_next, 0, sizeof(unsigned), s));
        HIPCHK(c0, launch_jcg_queue(c0->bt_tasks, n, items, std::max(1, std::min(items, c0->queue_blocks)),
                                    c0->bt_next, s));
        HIPCHK(c0, hipMemcpyAsync(c0->bt_sc_host, c0->bt_sc, sizeof(JcgScalars) * n, hipMemcpyDeviceToHost, s));
    }
    // larger levels: the tiled path of each request (on the same stream)
    for (ServerReq *r : big) {
        ecmg_ctx *c = r->ctx;
        const int l = r->level;
        ecmg_level_info li{};
        li.rre_true = -1.0;
        li.level = l;
        li.nx = c->lv[l].g.nx;
        li.ny = c->lv[l].g.ny;
        li.nz = c->lv[l].g.nz;
        int rc;
        if (l >= 2) {
            CHK(do_exp_finite(c, l));
            rc = run_level_jcg(c, l, r->rel_tol * c->lv[l].nf, c->opt.max_iter, -1, &li);
        } else {
            launch_zero_free(c->lv[l].g, c->lv[l].x, s);
            rc = run_level_jcg(c, l, c->opt.dsolve_tol * c->lv[l].nf, 100000, -1, &li);
            if (rc == ECMG_ENOTCONV) rc = ECMG_OK;
        }
        if (rc == ECMG_EDEVICE) return rc;
        li.status = rc;
        r->info[l] = li;
    }
    HIPCHK(c0, hipStreamSynchronize(s));
    const float ms = (float)std::chrono::duration<double, std::milli>(Clock::now() - t_start).count();
    for (int k = 0; k < n; ++k) {
        ServerReq *r = small[order[k]];
        ecmg_ctx *c = r->ctx;
        const int l = r->level;
        const Level &L = c->lv[l];
        const JcgScalars &sc = c0->bt_sc_host[k];
        ecmg_level_info li{};
        li.rre_true = -1.0;
        li.level = l;
        li.nx = L.g.nx;
        li.ny = L.g.ny;
        li.nz = L.g.nz;
        li.iters = sc.iter;
        li.rre = (L.nf > 0) ? std::sqrt(sc.rr) / L.nf : 0.0;
        li.nf = L.nf;
        int st = (sc.done == DONE_BREAKDOWN) ? ECMG_EBREAKDOWN : (sc.done == DONE_MAXITER) ? ECMG_ENOTCONV : ECMG_OK;
        if (l < 2 && st == ECMG_ENOTCONV) st = ECMG_OK;
        li.status = st;
        li.path = ECMG_PATH_QUEUE;
        r->info[l] = li;
    }
    for (ServerReq *r : S->active) {
        r->info[r->level].ms = ms;
        ++r->level;
    }
    return ECMG_OK;
}

extern "C" {

int ecmg_server_create(const ecmg_options *opt, size_t hbm_budget_bytes, ecmg_server **out) {
    if (!out) return fail(nullptr, ECMG_EINVAL, "out is NULL");
    *out = nullptr;
    if (hbm_budget_bytes == 0) return fail(nullptr, ECMG_EINVAL, "hbm_budget_bytes is 0");
    ecmg_server *S = new ecmg_server();
    if (opt) S->opt = *opt;
    else ecmg_default_options(&S->opt);
    if (S->opt.tune_cache) {
        S->tune_cache = S->opt.tune_cache;
        S->opt.tune_cache = S->tune_cache.c_str();
    }
    if (S->opt.precision != ECMG_FP64) {
        delete S;
        return fail(nullptr, ECMG_EINVAL, "the server runs FP64 only");
    }
    S->opt.keep_w = 0;
    S->opt.timing = 0;
    S->opt.dsolve_dense_max = 0;       // DSOLVE levels run in the shared queue launches
    // coarse levels of all active requests share one queue launch: the
    // persistent form pays off up to larger grids there
    if (S->opt.persistent_nodes < 0) S->opt.persistent_nodes = 2400000;
    S->budget = hbm_budget_bytes;
    if (S->opt.hip_stream) {
        S->stream = (hipStream_t)S->opt.hip_stream;
    } else if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess) {
        delete S;
        return fail(nullptr, ECMG_EDEVICE, "hipStreamCreate failed");
    }
    ecmg_options lo = S->opt;
    lo.hip_stream = S->stream;
    int rc = ecmg_create(&lo, &S->lead);
    if (rc == ECMG_OK && (hipGetDevice(&S->device) != hipSuccess ||
                          hipStreamCreateWithFlags(&S->setup_stream, hipStreamNonBlocking) != hipSuccess))
        rc = fail(nullptr, ECMG_EDEVICE, "setup stream creation failed");
    if (rc != ECMG_OK) {
        if (S->lead) ecmg_destroy(S->lead);
        if (!S->opt.hip_stream) (void)hipStreamDestroy(S->stream);
        delete S;
        return rc;
    }
    S->setup_thread = std::thread(server_setup_loop, S);
    *out = S;
    return ECMG_OK;
}

int ecmg_server_submit(ecmg_server *S, const ecmg_problem *problem, double rel_tol, double *host_out,
                       uint64_t *ticket) {
    if (!S || !problem || !ticket) return fail(nullptr, ECMG_EINVAL, "NULL argument");
    if (!(rel_tol >= 0.0)) return fail(S->lead, ECMG_EINVAL, "rel_tol = %g must be >= 0", rel_tol);
    CHK(validate(S->lead, problem));
    size_t bytes = 0;
    CHK(ecmg_plan_bytes(problem, ECMG_FP64, &bytes));
    if (bytes > S->budget)
        return fail(S->lead, ECMG_ENOMEM, "request needs %zu bytes, above the budget of %zu", bytes, S->budget);
    ServerReq *r = new ServerReq();
    r->prob = *problem;
    r->rel_tol = rel_tol;
    r->host_out = host_out;
    r->bytes = bytes;
    r->info.assign(problem->levels, ecmg_level_info{});
    std::lock_guard<std::mutex> g(S->mu);
    r->t_submit = Clock::now();
    if (!S->have_t0) {
        S->t0 = r->t_submit;
        S->have_t0 = true;
    }
    r->ticket = S->next_ticket++;
    S->queue.push_back(r);
    S->reqs[r->ticket] = r;
    *ticket = r->ticket;
    S->cv.notify_all();
    return ECMG_OK;
}

int ecmg_server_step(ecmg_server *S, int32_t *n_done) {
    if (!S) return fail(nullptr, ECMG_EINVAL, "server is NULL");
    if (n_done) *n_done = 0;
    // requests whose set-up has completed join the active set; with none
    // active, wait (briefly, so the caller can keep submitting) for one
    {
        std::unique_lock<std::mutex> g(S->mu);
        if (S->active.empty() && S->ready.empty() && (S->in_setup > 0 || !S->queue.empty()))
            S->cv.wait_for(g, std::chrono::milliseconds(2), [S] { return !S->ready.empty(); });
        for (ServerReq *r : S->ready) S->active.push_back(r);
        S->ready.clear();
    }
    if (S->active.empty()) return ECMG_OK;
    const auto t0 = Clock::now();
    CHK(server_tick(S));
    const auto t1 = Clock::now();
    int32_t done = 0;
    std::vector<ServerReq *> keep;
    for (ServerReq *r : S->active) {
        if (r->level < r->ctx->nlev) {
            keep.push_back(r);
            continue;
        }
        const int rc = server_complete(S, r);
        if (rc == ECMG_EDEVICE) return rc;
        ++done;
    }
    S->active.swap(keep);
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->t_tick += std::chrono::duration<double, std::milli>(t1 - t0).count();
        S->t_finish += std::chrono::duration<double, std::milli>(Clock::now() - t1).count();
    }
    if (n_done) *n_done = done;
    return ECMG_OK;
}

int ecmg_server_poll(ecmg_server *S, uint64_t ticket, int32_t *state, ecmg_level_info *info) {
    if (!S || !state) return fail(nullptr, ECMG_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(S->lead, ECMG_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    ServerReq *r = it->second;
    *state = r->state;
    if (info && r->state == 2)
        for (size_t l = 0; l < r->info.size(); ++l) info[l] = r->info[l];
    return ECMG_OK;
}

int ecmg_server_stats(ecmg_server *S, double *p50_ms, double *p99_ms, double *solves_per_s, int64_t *done) {
    if (!S) return fail(nullptr, ECMG_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> g(S->mu);
    std::vector<double> v = S->lat_ms;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) {
        if (v.empty()) return 0.0;
        const size_t k = (size_t)std::min<double>((double)v.size() - 1, std::ceil(p * (double)v.size()) - 1);
        return v[k];
    };
    if (p50_ms) *p50_ms = pct(0.50);
    if (p99_ms) *p99_ms = pct(0.99);
    if (solves_per_s) {
        const double s = S->ndone > 0 ? std::chrono::duration<double>(S->t_last - S->t0).count() : 0.0;
        *solves_per_s = s > 0 ? (double)S->ndone / s : 0.0;
    }
    if (done) *done = S->ndone;
    return ECMG_OK;
}

int ecmg_server_completed(ecmg_server *S, uint64_t *tickets, int32_t cap, int32_t *n) {
    if (!S || !n || (cap > 0 && !tickets)) return fail(nullptr, ECMG_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(S->mu);
    int32_t k = 0;
    while (k < cap && !S->finished.empty()) {
        tickets[k++] = S->finished.front();
        S->finished.pop_front();
    }
    *n = k;
    return ECMG_OK;
}

int ecmg_server_times(ecmg_server *S, double *setup_ms, double *step_ms, double *finish_ms) {
    if (!S) return fail(nullptr, ECMG_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> g(S->mu);
    if (setup_ms) *setup_ms = S->t_setup;
    if (step_ms) *step_ms = S->t_tick;
    if (finish_ms) *finish_ms = S->t_finish;
    return ECMG_OK;
}

int ecmg_server_reset_stats(ecmg_server *S) {
    if (!S) return fail(nullptr, ECMG_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> g(S->mu);
    S->t_setup = S->t_tick = S->t_finish = 0.0;
    S->lat_ms.clear();
    S->ndone = 0;
    S->have_t0 = true;
    S->t0 = Clock::now();
    return ECMG_OK;
}

void ecmg_server_destroy(ecmg_server *S) {
    if (!S) return;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
    }
    S->cv.notify_all();
    if (S->setup_thread.joinable()) S->setup_thread.join();   // finishes the set-up it holds
    for (ServerReq *r : S->active)
        if (r->ctx) ecmg_destroy(r->ctx);
    for (ServerReq *r : S->ready)
        if (r->ctx) ecmg_destroy(r->ctx);
    for (auto &e : S->idle) ecmg_destroy(e.ctx);
    for (auto &kv : S->reqs) delete kv.second;
    if (S->lead) ecmg_destroy(S->lead);
    if (!S->opt.hip_stream && S->stream) (void)hipStreamDestroy(S->stream);
    if (S->setup_stream) (void)hipStreamDestroy(S->setup_stream);
    delete S;
}

}  // extern "C"
