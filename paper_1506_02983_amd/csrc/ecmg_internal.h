// Internal declarations of the MI355X ECMG_jcg library: level geometry, device
// argument blocks, kernel launchers.  Host code and kernels include this; the
// public interface is include/ecmg.h.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "ecmg.h"

namespace ecmg {

// ---- stencil tile shape ------------------------------------------------------
// A block of TX x TY threads owns a TX x (TY*RY) tile of an x-y node plane and
// marches through KZ planes in z.  Lanes run along x (one 64-wide wavefront per
// row: coalesced, each z-plane contiguous in HBM); each wave handles RY rows.
// 64 x 8 tiles of 512 threads: two blocks share a CU, so one computes while the
// other waits at its per-plane barrier for the next plane's loads.
#ifndef ECMG_TILE_TY
#define ECMG_TILE_TY 8
#endif
#ifndef ECMG_TILE_RY
#define ECMG_TILE_RY 1
#endif
#ifndef ECMG_PREFETCH
#define ECMG_PREFETCH 1
#endif
constexpr int TX = 64;
constexpr int TY = ECMG_TILE_TY;
constexpr int RY = ECMG_TILE_RY;
constexpr int TYT = TY * RY;          // tile height in nodes
constexpr int NT = TX * TY;           // threads per block
constexpr int PF = ECMG_PREFETCH;     // z-steps between issuing a plane's loads and using them
// waves per SIMD the stencil kernel is compiled for: 4 x 64 lanes x 4 SIMDs =
// 1024 threads per CU, one 1024-thread block or two 512-thread blocks (caps
// registers at 128 per lane)
constexpr int STENCIL_WAVES_PER_EU = 4;
constexpr int NXCD = 8;               // MI355X: 8 XCDs, each with its own L2

// Non-temporal (streaming) 16-byte accesses for the passes that read and write
// every node once with fully coalesced 2-vectors: on the finest grids it raises
// JCG pass B from 4.7 to 5.8 TB/s.  HIP's double2 / float2 are structs, the
// builtins take native vectors.  (Not for stores that cover half of each
// 32-byte chunk per instruction: those lose the L2's merging of the halves.)
template <typename E> struct NativeVec2 { typedef E type __attribute__((ext_vector_type(2))); };
template <typename V> __device__ __forceinline__ V nt_load2(const V *p) {
    using E = decltype(p->x);
    const typename NativeVec2<E>::type v = __builtin_nontemporal_load((const typename NativeVec2<E>::type *)p);
    V r;
    r.x = v.x;
    r.y = v.y;
    return r;
}
template <typename V> __device__ __forceinline__ void nt_store2(const V &v, V *p) {
    using E = decltype(p->x);
    typename NativeVec2<E>::type w;
    w.x = v.x;
    w.y = v.y;
    __builtin_nontemporal_store(w, (typename NativeVec2<E>::type *)p);
}

// The streaming hint pays only where a pass's vectors would not stay in the
// 256 MB last-level cache until the next pass reads them.  On smaller grids the
// node-wise passes (pass B, the p and x updates) use ordinary accesses, which
// keep those vectors cached between the passes of an iteration: measured per
// level, 129^3 nodes 0.44 -> 0.40 ms and 65^3 1.20 -> 1.16 ms with them, while
// 257^3 (136 MB per vector) went from 0.79 to 0.89 ms.
constexpr int64_t STREAM_MIN_NODES = int64_t(1) << 23;
template <bool NT, typename V> __device__ __forceinline__ V ld2(const V *p) {
    if constexpr (NT) {
        return nt_load2(p);
    } else {
        using E = decltype(p->x);
        const typename NativeVec2<E>::type v = *(const typename NativeVec2<E>::type *)p;
        V r;
        r.x = v.x;
        r.y = v.y;
        return r;
    }
}
// one element (the compiler merges a run-time choice between the two forms of
// the same access into the ordinary one, so the choice is a template argument)
template <bool NT, typename T> __device__ __forceinline__ T ld1(const T *p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, typename T> __device__ __forceinline__ void st1(T v, T *p) {
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}
template <bool NT, typename V> __device__ __forceinline__ void st2(const V &v, V *p) {
    if constexpr (NT) {
        nt_store2(v, p);
    } else {
        using E = decltype(p->x);
        typename NativeVec2<E>::type w;
        w.x = v.x;
        w.y = v.y;
        *(typename NativeVec2<E>::type *)p = w;
    }
}

// HIP events for the next timed launch, set by the library's kernel-time
// records.  launch_timed() hands them to the extended launch, which stamps
// them with that kernel's own start and end (no marker packets between
// kernels, so timing does not lengthen launch-bound levels), and clears them.
struct PendingTiming {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local PendingTiming g_pending_timing;
template <typename F, typename... Args>
inline void launch_timed(F kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t s, Args... args) {
    const PendingTiming t = g_pending_timing;
    g_pending_timing = PendingTiming{};
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, t.start, t.stop, 0u, args...);
}
// The first launch of a group timed as one (start of the first kernel to the
// end of the last): takes the start event and leaves the stop event to the
// group's last launch, made by launch_timed.
template <typename F, typename... Args>
inline void launch_timed_first(F kernel, dim3 grid, dim3 block, uint32_t shmem, hipStream_t s, Args... args) {
    hipEvent_t start = g_pending_timing.start;
    g_pending_timing.start = nullptr;
    hipExtLaunchKernelGGL(kernel, grid, block, shmem, s, start, nullptr, 0u, args...);
}

// Geometry of one level, passed to kernels by value.
// Node arrays in HBM: node (i,j,k) at i + sx*(j + sy*k), rows padded to a
// multiple of 16 doubles (128 bytes) so every tile row starts on a cache-line
// boundary; padding entries (i > nx) hold zeros.
constexpr int ROW_ALIGN = 16;
__host__ __device__ inline int row_pitch(int nodes_x) { return (nodes_x + ROW_ALIGN - 1) / ROW_ALIGN * ROW_ALIGN; }

struct Geom {
    int nx, ny, nz;                   // elements per axis
    int sx, sy;                       // row pitch (>= nx+1, padded) / rows per plane (ny+1)
    int64_t nnodes;                   // allocated entries sx*sy*(nz+1)
    int64_t nreal;                    // nodes (nx+1)(ny+1)(nz+1)
    double h[3];
    int ft[6];                        // face types (0 Dirichlet, 1 Robin)
    // Q1 stiffness entry / beta between local nodes differing on the axes of
    // mask m (bit 0 = x, 1 = y, 2 = z): tensor products of the 1-D stiffness
    // (1,-1)/h and mass h(1/3, 1/6) (Section 2, bilinear form a(u,v)).
    double C[8];
    // Robin face mass / alpha for face f between face nodes differing on c in-
    // face axes: hp*hq*(1/9, 1/18, 1/36).
    double M[6][3];
};

// Device-side JCG state: scalars of the current iteration and stop control.
struct JcgScalars {
    double rho;        // r.z of the current residual
    double rr;         // ||r||^2
    double alpha;      // step length of the last completed pass A
    double beta;       // rho_k / rho_{k-1} for the next search direction
    double pq;         // p.q of the last pass A
    double tol;        // eps * ||f_h|| (stop when !(||r|| > tol))
    int iter;          // completed iterations
    int done;          // 0 running, 1 converged, 2 max_iter, 3 breakdown
    int max_iter;
    int fixed;         // >= 0: run exactly this many iterations
    int pending;       // x += alpha p of the last iteration still to apply
    int brk;           // folded scalars: pass B found p.q <= 0 (the next pass A sets done)
    double rho_f[2];   // folded scalars: rho of iteration k in slot k & 1
};

enum { DONE_RUNNING = 0, DONE_CONVERGED = 1, DONE_MAXITER = 2, DONE_BREAKDOWN = 3 };

// Arguments of the tiled stencil kernels (apply, JCG init, JCG pass A).
template <typename T>
struct StencilArgs {
    Geom g;
    int ntx, nty, nkz, KZ;            // tiles in x, y; z-chunks and planes per chunk
    const T *beta;                    // element coefficients
    const T *alpha[6];                // Robin face-element coefficients (or null)
    const T *v;                       // apply/init: input vector
    T *q;                             // apply: output; pass A: q = A p
    const T *F;                       // init: load vector
    const T *dinv;                    // init / pass A: 1/diag, 0 on Dirichlet nodes
    T *r;                             // init: output residual; pass A: input
    T *x;                             // pass A: iterate (deferred update)
    T *p0, *p1;                       // pass A: search directions (ping-pong)
    JcgScalars *sc;
    double *partials;                 // per-block partial sums (2 per block)
    int p_init;                       // init also stores p_0 = D^-1 r into p1, and pass A's
                                      // iteration 0 (MODE_PASSA0) reads it there
    // Folded scalars (no finishing kernels): init stores its (r.z, r.r) block
    // partials in partials2; pass A of iteration `it` sums the fold_nb pairs
    // there (init's or pass B's) itself, takes the stop test and beta, and
    // stores its p.q partials in partials.
    int fold, it, fold_nb;
    double *partials2;
};

template <typename T>
struct PassBArgs {
    int64_t n;
    T *r;
    const T *q;
    const T *dinv;
    JcgScalars *sc;
    double *partials;                 // 2 * passB_blocks(n)
    // folded scalars: pass B of iteration `it` sums pass A's nb_a p.q partials
    // (stride 2) itself and takes alpha = rho_it / p.q
    int fold, it, nb_a;
    const double *pq_partials;
    // unfolded only: the pass B a speculative chunk expects to be its level's
    // last.  Computes r - alpha q and ||r||^2 for the stop test but stores
    // no r and forms no r.z (no 1/D read): if the test passes nothing reads
    // them, and if it fails the level is solved again from its start.
    int last;
};

// Largest pass (blocks) whose partials every block of the next pass sums
// itself instead of a one-block finishing kernel.
constexpr int FOLD_MAX_BLOCKS = 4096;
// Built-in limit of the gather path (one thread per node for the stencil
// passes, folded scalars): grids up to FOLD_MAX_BLOCKS blocks of 256 nodes.
constexpr int64_t GATHER_DEFAULT_NODES = (int64_t)FOLD_MAX_BLOCKS * 256;

// the Robin faces of a grid and the first thread of each in the face blocks
struct ColFaces {
    int nf;
    int face[6];
    int64_t start[7];
};
// Column stencil kernels (col_kernels.hip): one wave per (62-node x-segment,
// R rows, z-chunk of KZ planes), planes in registers, x neighbours by DPP,
// then one thread per Robin-face node in the launch's last blocks.
// Used for JCG init and the stencil of pass A on levels whose passes run
// with one-block finishing kernels (the large grids).  Rows per wave: init
// keeps 2 (its epilogue inputs and outputs fill the registers: 4 rows would
// leave 2 waves per SIMD and ran slower; so did 3), the stencil of pass A
// takes 4 (halo rows 1.5x instead of 2x its output rows: 513^3 0.75 -> 0.69
// ms; 6 rows: no net change).
constexpr int COL_R_INIT = 2, COL_R_A0 = 4;
struct ColArgs {
    Geom g;
    int ntx, nty, nkz, KZ;            // waves: x-segments, row groups, z-chunks; planes per chunk
    int order;                        // wave order (col_waves)
    int R;                            // node rows per wave (COL_R_INIT or COL_R_A0)
    const double *beta;
    const double *alpha[6];
    const double *v;                  // input: APPLY v, INIT x, PASSA0 p (p_0 at iteration 0)
    const double *v_odd;              // PASSA0: the input p at odd iterations (NULL: always v)
    double *out;                      // APPLY / PASSA0: q; INIT: r
    const double *F, *dinv;           // INIT epilogue inputs
    double *p_out;                    // INIT with p_init: p_0 = D^-1 r
    int p_init;
    int plain_cg;                     // INIT: M^-1 = 1 (ECMG_CG) instead of 1/diag from beta
    JcgScalars *sc;                   // PASSA0: returns when done is set
    int it;                           // gather pass A: the iteration (its p buffer), set per launch
    double *partials;                 // 2 per wave, then 2 per Robin-face block
    int ncb;                          // column blocks (set by launch_col)
    ColFaces fl;                      // Robin faces (set by launch_col)
};
// waves of a column launch for z-chunks of KZ planes
int col_waves(const Geom &g, int KZ, int order, int R, int *ntx, int *nty, int *nkz);
// Robin-face blocks of a column launch
int col_faces(const Geom &g, ColFaces *fl);
// the column launch (column blocks, then Robin-face blocks); returns the
// partial pairs written (waves, then face blocks), which the finishing kernel
// sums in that order, or -1 (nothing launched) if a.R is not the mode's rows
// per wave
int launch_col(int mode, const ColArgs &a, hipStream_t s);
// One thread per node (the gather levels: small grids, folded scalars).
// Init: the ColArgs fields of MODE_INIT (v = x, out = r, p_out, p_init,
// partials: r.z, r.r pairs).  Stencil of pass A: q = A p into out, p from v
// (even iterations) or v_odd (odd, by a.it), p.q pairs into partials; stores
// nothing when sc->done is set.  Both return the partial pairs
// written (one per block of 256 nodes).
int gather_blocks(const Geom &g);
int launch_gather_init(const ColArgs &a, hipStream_t s);
int launch_gather_a(const ColArgs &a, hipStream_t s);
// pass A of iteration `it` on the gather levels, node-wise part: the folded
// scalar step of the previous pass from its fold_nb partial pairs, then (it
// >= 1) p = D^-1 r + beta p_old, x += alpha p_old (the first launch of a
// timed group)
struct PUFoldArgs {
    int64_t n;
    const double *dinv, *r;
    double *p0, *p1, *x;
    JcgScalars *sc;
    const double *partials;
    int fold_nb, it;
};
void launch_p_update_fold(const PUFoldArgs &a, hipStream_t s);

// One independent JCG solve inside the persistent kernel: a grid, its arrays,
// its stop control, and the contiguous range of workgroups that works on it.
struct ExpTask;
struct PersistentTask {
    Geom g;
    const double *beta;
    const double *alpha[6];
    const double *F;
    const double *dinv;
    double *x, *r, *q;
    double *p[2];                     // search directions, ping-pong: iteration k writes p[(k+1)&1]
    double *partials;                 // 3 * nwg
    unsigned *bar;                    // arrival counter, zero before launch
    int *err;                         // set when a barrier wait exceeds its budget
    JcgScalars *sc;                   // result: iterations, ||r||^2, status
    double tol;                       // stop when !(||r|| > tol)
    int max_iter, fixed;
    int wg0, nwg;
    int seglen;                       // z-march length: the nodes of a column are cut into segments
    int zero_x;                       // 1: start from x = 0 on free nodes (DSOLVE), keep g_D
    // the whole batched cascade in one launch: wait until the tasks of the
    // box's coarser levels (one or two) have set their flags, build x = W by
    // EXP_finite (exp non-NULL), solve, then set this task's flag (all NULL
    // otherwise)
    const unsigned *dep[2];
    const ExpTask *exp;
    unsigned *flag;
};

// Modes of the tiled stencil kernel.
enum { MODE_APPLY = 0, MODE_INIT = 1, MODE_PASSA = 2, MODE_PASSA0 = 3 };

// ---- host-side level and context -------------------------------------------------
// kernel classes timed per level: 0 pass A, 1 pass B, 2 JCG init, 3 EXP_finite,
// 4 EXP_true, 5 pass A FP32, 6 pass B FP32, 7 persistent JCG, 8 mixed start,
// 9 mixed update
constexpr int NKIND = 13;

struct Level {
    Geom g;
    double lo[3];
    int64_t nelem;
    int64_t nface[6];                 // face elements per face (0 if not Robin)
    double *beta = nullptr;           // [nelem]
    double *alpha[6] = {};            // Robin faces
    double *F = nullptr;              // load vector
    double *x = nullptr;              // u_l (g_D on Dirichlet nodes)
    double *dinv = nullptr;
    double *W = nullptr;              // EXP_finite output (optional)
    double *Ut = nullptr;             // EXP_true output (lazy)
    double *ainv = nullptr;           // DSOLVE levels: explicit inverse of A_FF (lazy), nfree^2
    int *freeid = nullptr;            // padded node index of each free node
    int nfree = 0;
    int dense = 0;                    // 0 not tried, 1 ready, -1 not used
    float *beta32 = nullptr;          // mixed precision copies (lazy)
    float *alpha32[6] = {};
    float *dinv32 = nullptr;
    double nf = 0.0;                  // ||f_h||_2 of the stopping test
    int last_iters = -1;              // JCG iterations of the last converged solve (first chunk)
    int last_path = -1;               // ECMG_PATH_* of the last JCG enqueued on the level
    int spec_hits = 0;                // consecutive solves that converged in exactly last_iters
    bool spec_live = false;           // the enqueued solve reads no status (its chunk is last_iters)
    // autotuned JCG configuration (tune_path -1: the built-in rules)
    int tune_path = -1;               // 0 tiled passes, 1 persistent kernel, 3 gather stencil
    int tune_kz = 0;                  // tiled: planes per z-chunk
    int tune_seg = 0, tune_nwg = 0;   // persistent: nodes per segment, most workgroups
    // timing accumulators per kernel class
    double kt_ms[NKIND] = {};
    int64_t kt_n[NKIND] = {};
};

struct Ctx;

// ---- autotuner: per-level choices and their JSON cache (tune_cache.cpp) ----
struct TuneEntry {
    int path = 0;                     // 0 tiled passes, 1 persistent kernel, 2 batched solve,
                                      // 3 gather stencil (one thread per node)
    int kz = 0;                       // tiled: planes per z-chunk
    int seg = 0, nwg = 0;             // persistent: nodes per segment, most workgroups;
                                      // batched: nodes per segment (0: by box size),
                                      // nodes per workgroup
    double us_default = 0.0;          // microseconds per JCG iteration (batched: per
    double us_best = 0.0;             // batch solve), built-in and chosen configuration
};
// cache key of a JCG level: precision and elements per axis
std::string tune_key(int precision, int nx, int ny, int nz);
// cache key of the batched solve's configuration
std::string tune_key_batch(int precision);
// ECMG_OK, ECMG_ENOENT (no file) or ECMG_EINVAL (not a tuning cache); entries
// are added to *out, the device string of the file goes to *device
int tune_cache_read(const std::string &path, std::string *device, std::map<std::string, TuneEntry> *out,
                    std::string *err);
int tune_cache_write(const std::string &path, const std::string &device,
                     const std::map<std::string, TuneEntry> &entries, std::string *err);

// ---- launchers (kernels.hip / extrap.hip / setup.hip) ---------------------------
int stencil_blocks(const Geom &g, int KZ, int *ntx, int *nty, int *nkz);
// planes per z-chunk of the tiled stencil: about target_blocks blocks, at most kz_max
int stencil_kz(const Geom &g, int kz_max, int target_blocks);

template <typename T>
void launch_stencil(int mode, const StencilArgs<T> &a, hipStream_t s);
// the one-block finishing kernel of a stencil pass over nb partial pairs
// (MODE_INIT: rho, ||r||^2 and the first stop test; MODE_PASSA: p.q and alpha)
void launch_stencil_finish(int mode, JcgScalars *sc, const double *partials, int nb, hipStream_t s);
template <typename T>
void launch_passB(const PassBArgs<T> &a, hipStream_t s);
// blocks of pass B for n nodes (its partial slots: twice as many)
int64_t passB_blocks(int64_t n);
// x += alpha p of the last iteration if pending (update = false: only the copy
// of the final scalars to `out`, the update left to the caller)
void launch_final_x(const Geom &g, double *x, const double *p0, const double *p1, const JcgScalars *sc,
                    JcgScalars *out, hipStream_t s, bool update = true);
// pass A of iteration >= 1 on the column-kernel levels, node-wise part:
// p = D^-1 r + beta p_old, x += alpha p_old (the first launch of a timed group)
void launch_p_update(const Geom &g, const double *dinv, const double *r, double *p0, double *p1, double *x,
                     const JcgScalars *sc, hipStream_t s);
// mixed precision: r32 = r64 / s, d32 = 0, JCG start scalars (FP64 sums)
void launch_mixed_start(const Geom &g, const double *r64, double inv_s, const float *dinv32, float *r32, float *d32,
                        JcgScalars *sc, double *partials, unsigned *counter, hipStream_t s);
// mixed precision: x64 += s * (d32 + alpha p_last) (the deferred last update included)
void launch_mixed_update(const Geom &g, double *x, double sc_s, const float *d32, const float *p0, const float *p1,
                         const JcgScalars *sc, hipStream_t s);
void launch_to_f32(const double *a, float *b, int64_t n, hipStream_t s);
void launch_jcg_reset(JcgScalars *sc, double tol, int max_iter, int fixed, hipStream_t s);

void launch_exp_finite(const Geom &gf, const Geom &g1, const double *U1, const double *U0, double *x, double *W,
                       int variant, hipStream_t s);
// sc non-NULL: the fine solution is U1 + alpha p with the pending last update
// of the JCG solve whose scalars are sc and search directions p0 / p1
void launch_exp_true(const Geom &gf, const double *U1, const double *U0, double *Ut, hipStream_t s,
                     const JcgScalars *sc = nullptr, const double *p0 = nullptr, const double *p1 = nullptr);

// One box of a batched EXP_finite (U1 = u_{l-1}, U0 = u_{l-2}, x and optional
// W on level l) or EXP_true (U1 = u_l, U0 = u_{l-1}, result into x).  b0 / nb:
// first flat block and block count of the box ([0] EXP_finite, [1] EXP_true);
// gx / gy: EXP_true blocks along x and y (a block is 64 node pairs by 4 row
// pairs marching up a chunk of coarse planes).
struct ExpTask {
    Geom gf, g1;
    const double *U1, *U0;
    double *x, *W;
    int variant;
    int gx[2], gy[2];
    int tkz;                          // EXP_true: coarse planes per block
    int64_t nb[2], b0[2];
};
// kind 0: EXP_finite (one thread per coarse element; blocks in nb[0], b0[0]),
// 1: EXP_true (64 x 4 node-pair columns per block; nb[1], b0[1])
void exp_task_blocks(ExpTask &t, int kind);
void launch_exp_finite_batch(const ExpTask *d_tasks, int n, int64_t nb, hipStream_t s);
void launch_exp_true_batch(const ExpTask *d_tasks, int n, int64_t nb1, hipStream_t s);
void launch_zero_pad(const Geom &g, double *a, double *b, double *c, double *d, hipStream_t s);
void launch_zero_pad_f32(const Geom &g, float *a, float *b, float *c, hipStream_t s);

void launch_fill(double *p, int64_t n, double v, hipStream_t s);
// dense DSOLVE: A_FF (row-major, free nodes numbered by fmap), its inverse made
// full after the Cholesky routines, and x_F = A_FF^-1 (F - q) at the free nodes
constexpr int DSOLVE_DENSE_LIMIT = 8192;   // right-hand side in 64 KB of LDS
void launch_assemble_dense(const Geom &g, const double *beta, const double *const *alpha, const int *fmap,
                           double *A, int nf, hipStream_t s);
void launch_symmetrize(double *A, int n, hipStream_t s);
void launch_dsolve_gemv(int nf, const double *Ainv, const int *freeid, const double *F, const double *q, double *x,
                        hipStream_t s);
// dense (n_x+1)(n_y+1)(n_z+1) node array <-> padded level layout
void launch_pack(const Geom &g, const double *padded, double *dense, hipStream_t s);
void launch_unpack(const Geom &g, const double *dense, double *padded, hipStream_t s);
void launch_zero_free(const Geom &g, double *x, hipStream_t s);
void launch_load_volume(const Geom &g, int e0, int e1, const double *fg, double *F, hipStream_t s);
void launch_load_face(const Geom &g, int face, const double *gR, double *F, hipStream_t s);
void launch_scatter_face(const Geom &g, int face, const double *vals, double *x, hipStream_t s);
void launch_dinv(const Geom &g, const double *beta, const double *const *alpha, double *dinv, int plain_cg,
                 hipStream_t s);
void launch_rhs_norm(const Geom &g, const double *F, const double *Ax0, const double *x0, double *partials,
                     unsigned *counter, double *out, hipStream_t s);
void launch_norms(const Geom &g, const double *a, const double *b, const double *c, double *partials,
                  unsigned *counter, double *out, hipStream_t s);

#ifndef ECMG_PERSIST_NTP
#define ECMG_PERSIST_NTP 512
#endif
constexpr int PERSIST_NTP = ECMG_PERSIST_NTP;  // threads per workgroup of the persistent kernel
int persistent_max_blocks(int *per_cu, int *cus);
hipError_t launch_jcg_persistent(const PersistentTask *d_tasks, int ntasks, int total_wg, hipStream_t s);
// tasks with their own workgroup ranges [wg0, wg0 + nwg) over nitems work items,
// taken from the queue counter *next (zero at launch) by nwg resident workgroups
int queue_max_blocks();
hipError_t launch_jcg_queue(const PersistentTask *d_tasks, int ntasks, int nitems, int nwg, unsigned *next,
                            hipStream_t s);
// the same cooperative launch through hipLaunchKernelExC (recordable by stream capture)
hipError_t launch_jcg_queue_attr(const PersistentTask *d_tasks, int ntasks, int nitems, int nwg, unsigned *next,
                                 hipStream_t s);
// zero n 32-bit words with a kernel (a fill kernel, not a memset node, when captured)
void launch_zero_u32(unsigned *p, int64_t n, hipStream_t s);

// Block count of the 1-D reduction kernels (fixed so reductions are deterministic).
int reduce_blocks(int64_t n);

}  // namespace ecmg
