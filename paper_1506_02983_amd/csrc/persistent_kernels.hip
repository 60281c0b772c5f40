// Persistent JCG: the whole JCG loop of Algorithm 4 (lines 7-9) for one or
// many independent grids ("tasks") in a single cooperative launch.
//
// Small grids (the DSOLVE levels, coarse JCG levels, and the boxes of a
// batched solve) are latency-bound when every iteration costs kernel launches
// and host round trips.  Here each task owns a fixed set of workgroups that
// stay resident for the whole solve; the phases of one iteration are separated
// by a task-local barrier (a single workgroup uses __syncthreads only):
//   A1  x += alpha_{k-1} p_{k-1};  p = D^-1 r + beta_k p          (own nodes)
//   A2  q = A p (27-point gather from L2), partial p.q  -> alpha_k
//   B   r -= alpha_k q;  z = D^-1 r;  partials r.z, r.r  -> beta_{k+1}, stop test
// Every workgroup of a task sums the per-workgroup partials itself in the same
// fixed order, so all of them take the same decision and the result does not
// depend on which other tasks share the launch (batch invariance).
//
// Waits are bounded: a barrier that does not complete within a spin budget
// sets the task's error flag and every workgroup leaves the loop.
#include "ecmg_internal.h"

#include <cmath>

namespace ecmg {

__device__ __forceinline__ bool pdir(const Geom &g, int i, int j, int k) {
    return (i == 0 && g.ft[0] == ECMG_DIRICHLET) || (i == g.nx && g.ft[1] == ECMG_DIRICHLET) ||
           (j == 0 && g.ft[2] == ECMG_DIRICHLET) || (j == g.ny && g.ft[3] == ECMG_DIRICHLET) ||
           (k == 0 && g.ft[4] == ECMG_DIRICHLET) || (k == g.nz && g.ft[5] == ECMG_DIRICHLET);
}

// (A v)_i for node (i,j,k) (not Dirichlet) with neighbours read from global
// memory: the same Q1 stencil as the tiled kernels (beta per element, Robin
// face mass), for grids that live in L2 / the Infinity Cache.  Out-of-grid
// neighbours are read at clamped addresses and masked, so all 35 loads of a
// node are independent and in flight together.
__device__ double stencil_gather(const Geom &g, const double *__restrict__ v, const double *__restrict__ beta,
                                 const double *const *alpha, int i, int j, int k) {
    const int64_t sx = g.sx, sxy = (int64_t)g.sx * g.sy;
    const int64_t ex = g.nx, exy = (int64_t)g.nx * g.ny;
    double b[2][2][2];                                   // [dz][dy][dx]: element (i-1+dx, j-1+dy, k-1+dz)
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy)
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                const int ie = i - 1 + dx, je = j - 1 + dy, ke = k - 1 + dz;
                const bool ok = ie >= 0 && ie < g.nx && je >= 0 && je < g.ny && ke >= 0 && ke < g.nz;
                const double val = beta[min(max(ie, 0), g.nx - 1) + ex * min(max(je, 0), g.ny - 1) +
                                        exy * min(max(ke, 0), g.nz - 1)];
                b[dz][dy][dx] = ok ? val : 0.0;
            }
    double q = 0.0;
#pragma unroll
    for (int oz = -1; oz <= 1; ++oz) {
        const int kk = min(max(k + oz, 0), g.nz);
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy) {
            const int jj = min(max(j + oy, 0), g.ny);
#pragma unroll
            for (int ox = -1; ox <= 1; ++ox) {
                const int ii = min(max(i + ox, 0), g.nx);
                double w = 0.0;
#pragma unroll
                for (int dz = (oz > 0); dz <= (oz < 0 ? 0 : 1); ++dz)
#pragma unroll
                    for (int dy = (oy > 0); dy <= (oy < 0 ? 0 : 1); ++dy)
#pragma unroll
                        for (int dx = (ox > 0); dx <= (ox < 0 ? 0 : 1); ++dx) w += b[dz][dy][dx];
                // a neighbour outside the grid only meets elements outside the
                // grid, whose beta is 0: w == 0 there, so the clamped value is
                // multiplied by zero
                const int m = (ox != 0) | ((oy != 0) << 1) | ((oz != 0) << 2);
                q += g.C[m] * w * v[ii + sx * jj + sxy * kk];
            }
        }
    }
    // Robin faces through the node
    const int idx[3] = {i, j, k};
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int f = 0; f < 6; ++f) {
        if (g.ft[f] != ECMG_ROBIN) continue;
        const int ax = f / 2;
        if (idx[ax] != ((f & 1) ? n[ax] : 0)) continue;
        const int pax = (ax == 0) ? 1 : 0, qax = (ax == 2) ? 1 : 2;
        const int pi = idx[pax], qi = idx[qax], np = n[pax], nq = n[qax];
        double s = 0.0;
        for (int dq = 0; dq < 2; ++dq) {
            const int eq = qi - 1 + dq;
            if (eq < 0 || eq >= nq) continue;
            for (int dp = 0; dp < 2; ++dp) {
                const int ep = pi - 1 + dp;
                if (ep < 0 || ep >= np) continue;
                const double a = alpha[f][ep + (int64_t)np * eq];
                double t = 0.0;
                for (int bq = 0; bq < 2; ++bq)
                    for (int bp = 0; bp < 2; ++bp) {
                        int c3[3] = {i, j, k};
                        c3[pax] = ep + bp;
                        c3[qax] = eq + bq;
                        const int c = (bp != 1 - dp) + (bq != 1 - dq);
                        t += g.M[f][c] * v[c3[0] + sx * c3[1] + sxy * c3[2]];
                    }
                s += a * t;
            }
        }
        q += s;
    }
    return q;
}

constexpr int NTP = 1024;             // threads per workgroup
constexpr long SPIN_LIMIT = 1L << 24; // polls of a barrier before giving up

// Barrier over the nwg workgroups of one task: sense by generation count.
__device__ __forceinline__ void task_barrier(const PersistentTask &t, int nwg, int *s_err) {
    __syncthreads();
    if (nwg > 1 && threadIdx.x == 0) {
        unsigned *cnt = t.bar, *gen = t.bar + 1;
        __threadfence();
        const unsigned g0 = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned arrived = atomicAdd(cnt, 1u);
        if (arrived == (unsigned)(nwg - 1)) {
            __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __threadfence();
            atomicAdd(gen, 1u);
        } else {
            long n = 0;
            while (__hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0) {
                __builtin_amdgcn_s_sleep(2);
                if (++n > SPIN_LIMIT) {
                    *s_err = 1;
                    __hip_atomic_store(t.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
        __threadfence();
        if (__hip_atomic_load(t.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) *s_err = 1;
    }
    __syncthreads();
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
__device__ __forceinline__ void task_sum(const PersistentTask &t, int w, int nwg, int slot, double (&v)[NV],
                                         double (*red)[NTP / 64], int *s_err) {
    wg_sum<NV>(v, red);
    if (nwg == 1) return;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i)
            __hip_atomic_store(t.partials + (int64_t)(slot + i) * nwg + w, v[i], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    }
    task_barrier(t, nwg, s_err);
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

__global__ void __launch_bounds__(NTP) k_jcg_persistent(const PersistentTask *__restrict__ tasks, int ntasks) {
    __shared__ double red[3][NTP / 64];
    __shared__ int s_err;
    // locate this workgroup's task (tasks hold contiguous workgroup ranges)
    int lo = 0, hi = ntasks - 1;
    const int bid = blockIdx.x;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (tasks[mid].wg0 <= bid) lo = mid; else hi = mid - 1;
    }
    const PersistentTask t = tasks[lo];
    const int w = bid - t.wg0, nwg = t.nwg;
    const Geom &g = t.g;
    if (threadIdx.x == 0) s_err = 0;
    __syncthreads();

    // rows [r0, r1) of this workgroup; row = j + sy*k
    const int64_t rows = (int64_t)g.sy * (g.nz + 1);
    const int64_t r0 = rows * w / nwg, r1 = rows * (w + 1) / nwg;
    const int64_t sx = g.sx;
    const int width = g.nx + 1;
    const int64_t n_own = (r1 - r0) * width;

    // init: r = F - A x on free nodes, z = D^-1 r; rho = r.z, rr = r.r
    double acc[2] = {0.0, 0.0};
    for (int64_t e = threadIdx.x; e < n_own; e += NTP) {
        const int64_t row = r0 + e / width;
        const int i = (int)(e % width), j = (int)(row % g.sy), k = (int)(row / g.sy);
        const int64_t id = i + sx * row;
        double rv = 0.0;
        if (!pdir(g, i, j, k)) rv = t.F[id] - stencil_gather(g, t.x, t.beta, t.alpha, i, j, k);
        t.r[id] = rv;
        acc[0] += rv * (t.dinv[id] * rv);
        acc[1] += rv * rv;
    }
    task_sum<2>(t, w, nwg, 1, acc, red, &s_err);
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
    int pending = 0;
    while (!done && !s_err) {
        // A1: deferred x update and the new search direction, own nodes
        for (int64_t e = threadIdx.x; e < n_own; e += NTP) {
            const int64_t row = r0 + e / width;
            const int64_t id = (e % width) + sx * row;
            const double z = t.dinv[id] * t.r[id];
            if (it == 0) {
                t.p[id] = z;
            } else {
                const double po = t.p[id];
                t.x[id] += alpha * po;
                t.p[id] = z + beta * po;
            }
        }
        pending = 0;
        task_barrier(t, nwg, &s_err);
        // A2: q = A p, p.q
        double pq[1] = {0.0};
        for (int64_t e = threadIdx.x; e < n_own; e += NTP) {
            const int64_t row = r0 + e / width;
            const int i = (int)(e % width), j = (int)(row % g.sy), k = (int)(row / g.sy);
            const int64_t id = i + sx * row;
            double qv = 0.0;
            if (!pdir(g, i, j, k)) qv = stencil_gather(g, t.p, t.beta, t.alpha, i, j, k);
            t.q[id] = qv;
            pq[0] += t.p[id] * qv;
        }
        task_sum<1>(t, w, nwg, 0, pq, red, &s_err);
        if (!(pq[0] > 0.0) || !isfinite(pq[0])) { done = DONE_BREAKDOWN; break; }
        alpha = rho / pq[0];
        // B: r -= alpha q; z = D^-1 r; r.z, r.r
        double s2[2] = {0.0, 0.0};
        for (int64_t e = threadIdx.x; e < n_own; e += NTP) {
            const int64_t row = r0 + e / width;
            const int64_t id = (e % width) + sx * row;
            const double rv = t.r[id] - alpha * t.q[id];
            t.r[id] = rv;
            s2[0] += rv * (t.dinv[id] * rv);
            s2[1] += rv * rv;
        }
        task_sum<2>(t, w, nwg, 1, s2, red, &s_err);
        ++it;
        beta = s2[0] / rho;
        rho = s2[0];
        rr = s2[1];
        pending = 1;
        done = stop(rr);
    }
    if (pending) {                     // x += alpha p of the last iteration
        for (int64_t e = threadIdx.x; e < n_own; e += NTP) {
            const int64_t row = r0 + e / width;
            const int64_t id = (e % width) + sx * row;
            t.x[id] += alpha * t.p[id];
        }
    }
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

}  // namespace ecmg
