// Persistent JCG: the whole JCG loop of Algorithm 4 for one or
// many independent grids ("tasks") in a single cooperative launch.
//
// Small grids (the DSOLVE levels, coarse JCG levels, and the boxes of a
// batched solve) are latency-bound when every iteration costs kernel launches
// and host round trips.  Here each task owns a fixed set of workgroups that
// stay resident for the whole solve; the phases of an iteration are separated
// by task-wide barriers:
//   A  x += alpha_{k-1} p_{k-1};  p_k = D^-1 r + beta_k p_{k-1};  q = A p_k;
//      partial p.q                                      -> alpha_k
//   B  r -= alpha_k q;  partials r.D^-1 r, r.r          -> beta_{k+1}, stop test
// Work is cut into column segments (x-y column (i,j), planes k0..k1-1); in the
// stencil pass a thread marches up its segment holding three planes of the
// 3x3 neighbourhood in registers.  p ping-pongs between two arrays.  Phase A
// either stores p_k in an own-node pass and applies the stencil after a
// barrier.  Segments are 1, 2 or 4 nodes long (a template parameter), and every
// pass issues all loads of a segment before using any.
// Every workgroup of a task sums the per-workgroup partials itself in the same
// fixed order, so all of them take the same decision and the result does not
// depend on which other tasks share the launch (batch invariance).
//
// Waits are bounded: a barrier that does not complete within a spin budget
// sets the task's error flag and every workgroup leaves the loop.
#include "ecmg_internal.h"
#include "exp_finite.h"

#include <cmath>

namespace ecmg {

// The integers of a task's grid that the march needs; face types as bit masks
// (bit f = face f) so that few scalar registers hold them.
struct PGeom {
    int nx, ny, nz, sx, sxy, nxy;
    unsigned dir, robin;
};

__device__ __forceinline__ bool pdir(const PGeom &g, int i, int j, int k) {
    return (i == 0 && (g.dir & 1u)) || (i == g.nx && (g.dir & 2u)) || (j == 0 && (g.dir & 4u)) ||
           (j == g.ny && (g.dir & 8u)) || (k == 0 && (g.dir & 16u)) || (k == g.nz && (g.dir & 32u));
}

constexpr int NTP = PERSIST_NTP;
constexpr long SPIN_LIMIT = 1L << 22; // polls of the arrival counter before giving up

// Global-memory (address space 1) doubles: the task pointers are loaded from
// memory, so without this the compiler can only emit flat accesses.
typedef __attribute__((address_space(1))) double gdouble;

// Barrier over the nwg workgroups of one task: a monotonic arrival counter
// (zero at launch); barrier number gen completes when it reaches gen * nwg.
// The comparison is wrap-safe.
__device__ __forceinline__ void task_barrier(const PersistentTask &t, int nwg, unsigned gen, int *s_err) {
    __syncthreads();
    if (nwg > 1 && threadIdx.x == 0) {
        // release on arrival (the workgroup's writes, ordered before this by
        // the barrier above, become visible device-wide), acquire after the
        // wait: one L2 write-back and one invalidate per barrier
        __hip_atomic_fetch_add(t.bar, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned target = gen * (unsigned)nwg;
        long n = 0;
        while ((int)(__hip_atomic_load(t.bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
            __builtin_amdgcn_s_sleep(1);
            if ((++n & 63) == 0 &&
                (n > SPIN_LIMIT || __hip_atomic_load(t.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                *s_err = 1;
                __hip_atomic_store(t.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// Wait until the flags of the tasks this one depends on are set (bounded: the
// error flag instead of a hang), then acquire what those tasks wrote.
__device__ __forceinline__ void wait_deps(const PersistentTask &t, int *s_err) {
    if (threadIdx.x == 0) {
        for (int d = 0; d < 2; ++d) {
            if (!t.dep[d]) continue;
            long n = 0;
            while (__hip_atomic_load(t.dep[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) {
                __builtin_amdgcn_s_sleep(2);
                if ((++n & 63) == 0 &&
                    (n > SPIN_LIMIT || __hip_atomic_load(t.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                    *s_err = 1;
                    __hip_atomic_store(t.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// Load element idx of a uniform base pointer with a 32-bit byte offset, the
// form the SGPR-base global load takes: one VGPR per address instead of two.
// The caller guarantees idx * 8 < 2^32.
__device__ __forceinline__ double ldg(const gdouble *base, int idx) {
    return *(const gdouble *)((const __attribute__((address_space(1))) char *)base + (unsigned)idx * 8u);
}

// Arrays of one task as global-memory pointers.
struct TaskArrays {
    gdouble *X, *R, *Q, *PO, *PN;     // PO = p_{k-1} (read), PN = p_k (written)
    const gdouble *F, *DI, *BE;
    const gdouble *AL[6];
};

enum { MARCH_INIT = 0, MARCH_APPLY = 2 };

// One column segment of SEG nodes: node (i, j, k) for k in [k0, k0 + SEG),
// those above the grid (k > nz, last segment of a column) skipped.
//   MARCH_INIT: r = F - A x on free nodes (0 on Dirichlet); acc += (r.D^-1 r, r.r)
//   MARCH_APPLY: q = A p_k on free nodes (0 on Dirichlet); acc[0] += p_k.q
// Every load of the segment (SEG + 2 planes of the 3x3 neighbourhood, SEG + 1
// element slabs, the epilogue inputs) is issued before the first value is
// used, so a segment costs one memory latency rather than one per node.  The
// Q1 stencil is written per plane offset: the elements of the slab below and
// above the node, summed over the 2x2 element columns that hold both the node
// and each of the 3x3 in-plane neighbours.
template <int MODE, int SEG>
__device__ __forceinline__ void march(const PGeom &g, const double *sC_, const double (*sM_)[3], const TaskArrays &A,
                                      int i, int j, int k0, double (&acc)[2]) {
    // coefficients re-read from LDS at each use (a broadcast read) rather than
    // held in 26 register pairs for the whole kernel
    const volatile double *sC = sC_;
    const volatile double(*sM)[3] = sM_;
    const int sx = g.sx, sxy = g.sxy;
    const int nx = g.nx, ny = g.ny, nz = g.nz, nxy = g.nxy;
    const int ox[3] = {i > 0 ? -1 : 0, 0, i < nx ? 1 : 0};
    const int oy[3] = {j > 0 ? -sx : 0, 0, j < ny ? sx : 0};
    const int base = i + sx * j;
    const bool ex[2] = {i > 0, i < nx}, ey[2] = {j > 0, j < ny};
    const int bx[2] = {max(i - 1, 0), min(i, nx - 1)};
    const int by[2] = {nx * max(j - 1, 0), nx * min(j, ny - 1)};
    const gdouble *__restrict__ V = (MODE == MARCH_INIT) ? A.X : A.PN;

    // planes k0-1 .. k0+SEG (clamped into the grid; out-of-grid neighbours get
    // zero weight) and slabs k0-1 .. k0+SEG-1 (zero outside 0..nz-1)
    double P[SEG + 2][9], Bt[SEG + 1][4];
#pragma unroll
    for (int pl = 0; pl < SEG + 2; ++pl) {
        const int b = base + sxy * min(max(k0 - 1 + pl, 0), nz);
#pragma unroll
        for (int cy = 0; cy < 3; ++cy)
#pragma unroll
            for (int cx = 0; cx < 3; ++cx) P[pl][3 * cy + cx] = ldg(V, b + ox[cx] + oy[cy]);
    }
#pragma unroll
    for (int sl = 0; sl < SEG + 1; ++sl) {
        const int kz = k0 - 1 + sl;
        const bool okz = kz >= 0 && kz < nz;
        const int bz = nxy * min(max(kz, 0), nz - 1);
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const double v = ldg(A.BE, bx[dx] + by[dy] + bz);
                Bt[sl][2 * dy + dx] = (okz && ex[dx] && ey[dy]) ? v : 0.0;
            }
    }
    double E0[SEG], E1[SEG];                    // init: F and 1/D of the segment's nodes
    if (MODE == MARCH_INIT) {
#pragma unroll
        for (int kk = 0; kk < SEG; ++kk) {
            const int id = base + sxy * min(k0 + kk, nz);
            E0[kk] = ldg(A.F, id);
            E1[kk] = ldg(A.DI, id);
        }
    }
    // sum of a slab's elements that hold both the node and in-plane neighbour (cx, cy)
    auto wsum2 = [](const double(&b)[4], int cx, int cy) -> double {
        double w = 0.0;
#pragma unroll
        for (int dy = (cy == 2); dy <= (cy == 0 ? 0 : 1); ++dy)
#pragma unroll
            for (int dx = (cx == 2); dx <= (cx == 0 ? 0 : 1); ++dx) w += b[2 * dy + dx];
        return w;
    };
    // Robin face mass of face f over the 2x2 face elements around the node;
    // the in-face neighbour (cp, cq) is read by vat(cp, cq).
    auto robin = [&](int f, int pi, int np, int qi, int nq, auto vat) -> double {
        const bool fp[2] = {pi > 0, pi < np}, fq[2] = {qi > 0, qi < nq};
        const int ap[2] = {max(pi - 1, 0), min(pi, np - 1)};
        const int aq[2] = {np * max(qi - 1, 0), np * min(qi, nq - 1)};
        double a[2][2];
#pragma unroll
        for (int dq = 0; dq < 2; ++dq)
#pragma unroll
            for (int dp = 0; dp < 2; ++dp) {
                const double v = A.AL[f][ap[dp] + aq[dq]];
                a[dq][dp] = (fp[dp] && fq[dq]) ? v : 0.0;
            }
        double s = 0.0;
#pragma unroll
        for (int cq = 0; cq < 3; ++cq)
#pragma unroll
            for (int cp = 0; cp < 3; ++cp) {
                double w = 0.0;
#pragma unroll
                for (int dq = (cq == 2); dq <= (cq == 0 ? 0 : 1); ++dq)
#pragma unroll
                    for (int dp = (cp == 2); dp <= (cp == 0 ? 0 : 1); ++dp) w += a[dq][dp];
                s += sM[f][(cp != 1) + (cq != 1)] * w * vat(cp, cq);
            }
        return s;
    };

#pragma unroll
    for (int kk = 0; kk < SEG; ++kk) {
        const int k = k0 + kk;
        if (k > nz) break;
        const double(&vm)[9] = P[kk];
        const double(&v0)[9] = P[kk + 1];
        const double(&vp)[9] = P[kk + 2];
        const int id = base + sxy * k;
        double q = 0.0;
        const bool dir = pdir(g, i, j, k);
        if (!dir) {
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                const int m = ((c % 3) != 1) | (((c / 3) != 1) << 1);
                const double wm = wsum2(Bt[kk], c % 3, c / 3), wp = wsum2(Bt[kk + 1], c % 3, c / 3);
                q += sC[m | 4] * (wm * vm[c] + wp * vp[c]) + sC[m] * ((wm + wp) * v0[c]);
            }
            // x faces: in-face axes (y, z); y faces: (x, z); z faces: (x, y)
            auto vyz = [&](int cp, int cq) {
                return cq == 0 ? vm[3 * cp + 1] : cq == 1 ? v0[3 * cp + 1] : vp[3 * cp + 1];
            };
            auto vxz = [&](int cp, int cq) { return cq == 0 ? vm[3 + cp] : cq == 1 ? v0[3 + cp] : vp[3 + cp]; };
            auto vxy = [&](int cp, int cq) { return v0[3 * cq + cp]; };
            if (i == 0 && (g.robin & 1u)) q += robin(0, j, ny, k, nz, vyz);
            if (i == nx && (g.robin & 2u)) q += robin(1, j, ny, k, nz, vyz);
            if (j == 0 && (g.robin & 4u)) q += robin(2, i, nx, k, nz, vxz);
            if (j == ny && (g.robin & 8u)) q += robin(3, i, nx, k, nz, vxz);
            if (k == 0 && (g.robin & 16u)) q += robin(4, i, nx, j, ny, vxy);
            if (k == nz && (g.robin & 32u)) q += robin(5, i, nx, j, ny, vxy);
        }
        if (MODE == MARCH_INIT) {
            const double rv = dir ? 0.0 : E0[kk] - q;
            A.R[id] = rv;
            acc[0] += rv * (E1[kk] * rv);
            acc[1] += rv * rv;
        } else {
            A.Q[id] = q;
            acc[0] += v0[4] * q;
        }
    }
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over the workgroup, result broadcast to every thread.
template <int NV>
__device__ __forceinline__ void wg_sum(double (&v)[NV], double (*red)[NTP / 64]) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wsum(v[i]);
    __syncthreads();
    if ((tid & 63) == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) red[i][tid >> 6] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double s = red[i][0];
        for (int w = 1; w < NTP / 64; ++w) s += red[i][w];
        v[i] = s;
    }
}

// Task total of NV values: workgroup sums, exchange through the task's partial
// slots [slot .. slot+NV) x nwg, then the same fixed-order sum in every workgroup.
template <int NV>
__device__ __forceinline__ void task_sum(const PersistentTask &t, int w, int nwg, unsigned &gen, int slot,
                                         double (&v)[NV], double (*red)[NTP / 64], int *s_err) {
    wg_sum<NV>(v, red);
    if (nwg == 1) return;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i)
            __hip_atomic_store(t.partials + (int64_t)(slot + i) * nwg + w, v[i], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    task_barrier(t, nwg, ++gen, s_err);
    double s[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) s[i] = 0.0;
    for (int b = threadIdx.x; b < nwg; b += NTP) {
#pragma unroll
        for (int i = 0; i < NV; ++i)
            s[i] += __hip_atomic_load(t.partials + (int64_t)(slot + i) * nwg + b, __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_AGENT);
    }
    wg_sum<NV>(s, red);
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = s[i];
}

// The JCG solve of one task by workgroup w of its nwg workgroups.  LDS: red
// (reductions), s_err (barrier failure), sC / sM (coefficients).
template <int SEG>
__device__ __forceinline__ void jcg_task(const PersistentTask &t, int w, int nwg, double (*red)[NTP / 64],
                                         int &s_err, double *sC, double (*sM)[3]) {
    // stencil and face-mass coefficients in LDS (uniform reads), the rest of
    // the grid as a few integers
    if (threadIdx.x < 8) sC[threadIdx.x] = t.g.C[threadIdx.x];
    if (threadIdx.x < 18) sM[threadIdx.x / 3][threadIdx.x % 3] = t.g.M[threadIdx.x / 3][threadIdx.x % 3];
    PGeom g;
    g.nx = t.g.nx;
    g.ny = t.g.ny;
    g.nz = t.g.nz;
    g.sx = t.g.sx;
    g.sxy = t.g.sx * t.g.sy;
    g.nxy = t.g.nx * t.g.ny;
    g.dir = 0;
    g.robin = 0;
    for (int f = 0; f < 6; ++f) {
        if (t.g.ft[f] == ECMG_DIRICHLET) g.dir |= 1u << f;
        if (t.g.ft[f] == ECMG_ROBIN) g.robin |= 1u << f;
    }
    if (threadIdx.x == 0) s_err = 0;
    __syncthreads();

    TaskArrays A;
    A.X = (gdouble *)t.x;
    A.R = (gdouble *)t.r;
    A.Q = (gdouble *)t.q;
    A.F = (const gdouble *)t.F;
    A.DI = (const gdouble *)t.dinv;
    A.BE = (const gdouble *)t.beta;
#pragma unroll
    for (int f = 0; f < 6; ++f) A.AL[f] = (const gdouble *)t.alpha[f];

    // work units: (column, segment), columns fastest so that neighbouring
    // lanes take neighbouring x
    const int width = g.nx + 1;
    const int ncol = width * (g.ny + 1);
    const int nseg = (g.nz + SEG) / SEG;
    const int nunits = ncol * nseg;
    const int stride = nwg * NTP;
    const int sx = g.sx, sxy = g.sxy;
#define FOR_UNITS(...)                                                                    \
    for (int u = w * NTP + (int)threadIdx.x; u < nunits; u += stride) {                   \
        const int c = u % ncol, sg = u / ncol;                                            \
        const int i = c % width, j = c / width;                                           \
        const int k0 = sg * SEG;                                                          \
        __VA_ARGS__                                                                       \
    }

    // own-node loops over a segment: loads of all its nodes first
#define FOR_SEG(kk) _Pragma("unroll") for (int kk = 0; kk < SEG; ++kk)
    unsigned gen = 0;                  // barriers passed by this workgroup
    if (t.dep[0] || t.dep[1]) wait_deps(t, &s_err);
    if (t.exp && !s_err) {             // x = W from the box's two coarser levels
        const ExpTask &e = *t.exp;
        const int64_t ne = (int64_t)(e.gf.nx / 4) * (e.gf.ny / 4) * (e.gf.nz / 4);
        for (int64_t k = (int64_t)w * NTP + threadIdx.x; k < ne; k += (int64_t)nwg * NTP)
            exp_finite_elem<false>(e.gf, e.g1, e.U1, e.U0, e.x, e.W, e.variant, k, nullptr);
        task_barrier(t, nwg, ++gen, &s_err);
    }
    if (t.zero_x) {                    // x = 0 on free nodes, g_D stays on Dirichlet nodes
        FOR_UNITS({
            FOR_SEG(kk) {
                const int k = k0 + kk;
                if (k <= g.nz && !pdir(g, i, j, k)) A.X[i + sx * j + sxy * k] = 0.0;
            }
        })
        task_barrier(t, nwg, ++gen, &s_err);
    }
    double acc[2] = {0.0, 0.0};
    FOR_UNITS(march<MARCH_INIT, SEG>(g, sC, sM, A, i, j, k0, acc);)
    task_sum<2>(t, w, nwg, gen, 1, acc, red, &s_err);
    double rho = acc[0], rr = acc[1], alpha = 0.0, beta = 0.0;
    int it = 0, done = 0;
    const int fixed = t.fixed, max_iter = t.max_iter;
    auto stop = [&](double rrv) -> int {
        const double rn = sqrt(rrv);
        if (fixed >= 0) return it >= fixed ? DONE_CONVERGED : DONE_RUNNING;
        if (!(rn > t.tol)) return DONE_CONVERGED;
        return it >= max_iter ? DONE_MAXITER : DONE_RUNNING;
    };
    done = stop(rr);
    while (!done && !s_err) {
        // A: x, p (own nodes), then q = A p, p.q
        // (a select, not an index: indexing would put the task copy in scratch)
        A.PO = (gdouble *)((it & 1) ? t.p[1] : t.p[0]);
        A.PN = (gdouble *)((it & 1) ? t.p[0] : t.p[1]);
        double pq[2] = {0.0, 0.0};
        FOR_UNITS({
            gdouble *__restrict__ Xr = A.X;
            gdouble *__restrict__ Pn = A.PN;
            const gdouble *__restrict__ Po = A.PO;
            const gdouble *__restrict__ Rr = A.R;
            const gdouble *__restrict__ Dr = A.DI;
            const int id0 = i + sx * j + sxy * k0;
            double z[SEG], po[SEG], xv[SEG];
            FOR_SEG(kk) {
                const int id = id0 + sxy * min(kk, g.nz - k0);
                z[kk] = ldg(Dr, id) * ldg(Rr, id);
                if (it > 0) {
                    po[kk] = ldg(Po, id);
                    xv[kk] = ldg(Xr, id);
                }
            }
            FOR_SEG(kk) {
                if (k0 + kk > g.nz) break;
                const int id = id0 + sxy * kk;
                if (it == 0) {
                    Pn[id] = z[kk];
                } else {
                    Xr[id] = xv[kk] + alpha * po[kk];
                    Pn[id] = fma(beta, po[kk], z[kk]);
                }
            }
        })
        task_barrier(t, nwg, ++gen, &s_err);
        FOR_UNITS(march<MARCH_APPLY, SEG>(g, sC, sM, A, i, j, k0, pq);)
        double pqs[1] = {pq[0]};
        task_sum<1>(t, w, nwg, gen, 0, pqs, red, &s_err);
        if (!(pqs[0] > 0.0) || !isfinite(pqs[0])) { done = DONE_BREAKDOWN; break; }
        alpha = rho / pqs[0];
        // B: r -= alpha q; r.D^-1 r, r.r
        double s2[2] = {0.0, 0.0};
        FOR_UNITS({
            gdouble *__restrict__ Rr = A.R;
            const gdouble *__restrict__ Qr = A.Q;
            const gdouble *__restrict__ Dr = A.DI;
            const int id0 = i + sx * j + sxy * k0;
            double rv[SEG], qv[SEG], dv[SEG];
            FOR_SEG(kk) {
                const int id = id0 + sxy * min(kk, g.nz - k0);
                rv[kk] = ldg(Rr, id);
                qv[kk] = ldg(Qr, id);
                dv[kk] = ldg(Dr, id);
            }
            FOR_SEG(kk) {
                if (k0 + kk > g.nz) break;
                const double r1 = rv[kk] - alpha * qv[kk];
                Rr[id0 + sxy * kk] = r1;
                s2[0] += r1 * (dv[kk] * r1);
                s2[1] += r1 * r1;
            }
        })
        task_sum<2>(t, w, nwg, gen, 1, s2, red, &s_err);
        ++it;
        beta = s2[0] / rho;
        rho = s2[0];
        rr = s2[1];
        done = stop(rr);
    }
    if (it > 0 && done != DONE_BREAKDOWN) {   // x += alpha p of the last completed iteration
        const gdouble *__restrict__ PL = (const gdouble *)((it & 1) ? t.p[1] : t.p[0]);
        FOR_UNITS({
            gdouble *__restrict__ Xr = A.X;
            const int id0 = i + sx * j + sxy * k0;
            double pv[SEG], xv[SEG];
            FOR_SEG(kk) {
                const int id = id0 + sxy * min(kk, g.nz - k0);
                pv[kk] = ldg(PL, id);
                xv[kk] = ldg(Xr, id);
            }
            FOR_SEG(kk) {
                if (k0 + kk > g.nz) break;
                Xr[id0 + sxy * kk] = xv[kk] + alpha * pv[kk];
            }
        })
    }
#undef FOR_SEG
#undef FOR_UNITS
    if (w == 0 && threadIdx.x == 0) {
        JcgScalars *sc = t.sc;
        sc->iter = it;
        sc->rr = rr;
        sc->rho = rho;
        sc->alpha = alpha;
        sc->done = s_err ? DONE_BREAKDOWN : done;
        sc->pending = 0;
        sc->tol = t.tol;
    }
    if (t.flag) {
        // every workgroup's x is written (barrier), then the flag, released:
        // set whatever happened, so no dependent task waits in vain
        task_barrier(t, nwg, ++gen, &s_err);
        if (w == 0 && threadIdx.x == 0) __hip_atomic_store(t.flag, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();                   // LDS is reused by the next task of this workgroup
}

// The task's segment length selects the instantiation (1, 2 or 4 nodes).
__device__ __forceinline__ void run_task(const PersistentTask &t, int w, int nwg, double (*red)[NTP / 64], int &s_err,
                                         double *sC, double (*sM)[3]) {
    if (t.seglen >= 4) jcg_task<4>(t, w, nwg, red, s_err, sC, sM);
    else if (t.seglen == 2) jcg_task<2>(t, w, nwg, red, s_err, sC, sM);
    else jcg_task<1>(t, w, nwg, red, s_err, sC, sM);
}

// One or more tasks, each on its own contiguous range of workgroups
// (cooperative launch: all workgroups of a task must be resident together).
__global__ void __launch_bounds__(NTP) k_jcg_persistent(const PersistentTask *__restrict__ tasks, int ntasks) {
    __shared__ double red[3][NTP / 64];
    __shared__ int s_err;
    __shared__ double sC[8], sM[6][3];
    // locate this workgroup's task (tasks hold contiguous workgroup ranges)
    int lo = 0, hi = ntasks - 1;
    const int bid = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (tasks[mid].wg0 <= bid) lo = mid; else hi = mid - 1;
    }
    const PersistentTask &t = tasks[lo];
    run_task(t, bid - t.wg0, t.nwg, red, s_err, sC, sM);
}

// Many tasks taken from a queue.  Task i owns the work items [wg0, wg0 + nwg)
// (contiguous, tasks in order); every workgroup takes the next item from an
// atomic counter (zero at launch), works on its task as workgroup
// item - wg0 of nwg, and takes another until none is left.  Deadlock-free when
// every workgroup of the launch is resident (cooperative launch) and no task
// has more workgroups than the launch: items are taken in order, so when a
// workgroup waits at a task barrier, every item before its partners' has been
// taken by a workgroup whose own task can complete.  Tasks sorted by
// decreasing work keep the longest ones from starting last.
__global__ void __launch_bounds__(NTP) k_jcg_queue(const PersistentTask *__restrict__ tasks, int ntasks,
                                                   int nitems, unsigned *next) {
    __shared__ double red[3][NTP / 64];
    __shared__ int s_err;
    __shared__ double sC[8], sM[6][3];
    __shared__ int s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(next, 1u);
        __syncthreads();
        const int item = s_item;
        __syncthreads();
        if (item >= nitems) break;
        int lo = 0, hi = ntasks - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (tasks[mid].wg0 <= item) lo = mid; else hi = mid - 1;
        }
        const PersistentTask &t = tasks[lo];
        run_task(t, item - t.wg0, t.nwg, red, s_err, sC, sM);
    }
}

int persistent_max_blocks(int *per_cu, int *cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return -1;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_jcg_persistent, NTP, 0) != hipSuccess) return -1;
    *per_cu = nb;
    *cus = prop.multiProcessorCount;
    return nb * prop.multiProcessorCount;
}

hipError_t launch_jcg_persistent(const PersistentTask *d_tasks, int ntasks, int total_wg, hipStream_t s) {
    void *args[] = {(void *)&d_tasks, (void *)&ntasks};
    return hipLaunchCooperativeKernel((const void *)k_jcg_persistent, dim3(total_wg), dim3(NTP), args, 0, s);
}

int queue_max_blocks() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return -1;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return -1;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_jcg_queue, NTP, 0) != hipSuccess) return -1;
    return nb * prop.multiProcessorCount;
}

hipError_t launch_jcg_queue(const PersistentTask *d_tasks, int ntasks, int nitems, int nwg, unsigned *next,
                            hipStream_t s) {
    void *args[] = {(void *)&d_tasks, (void *)&ntasks, (void *)&nitems, (void *)&next};
    return hipLaunchCooperativeKernel((const void *)k_jcg_queue, dim3(nwg), dim3(NTP), args, 0, s);
}

// The same launch through the launch-attribute interface (cooperative
// attribute), which stream capture records into a graph kernel node.
hipError_t launch_jcg_queue_attr(const PersistentTask *d_tasks, int ntasks, int nitems, int nwg, unsigned *next,
                                 hipStream_t s) {
    void *args[] = {(void *)&d_tasks, (void *)&ntasks, (void *)&nitems, (void *)&next};
    hipLaunchAttribute attr[1];
    attr[0].id = hipLaunchAttributeCooperative;
    attr[0].val.cooperative = 1;
    hipLaunchConfig_t cfg{};
    cfg.gridDim = dim3(nwg);
    cfg.blockDim = dim3(NTP);
    cfg.dynamicSmemBytes = 0;
    cfg.stream = s;
    cfg.attrs = attr;
    cfg.numAttrs = 1;
    return hipLaunchKernelExC(&cfg, (const void *)k_jcg_queue, args);
}

}  // namespace ecmg
