// Discretisation kernels (Section 2): load vector assembly from field samples
// at Gauss points, Dirichlet data scatter, the Jacobi diagonal, the norm of the
// right-hand side used by the stopping test, and the error norms of Section 5.
#include "ecmg_internal.h"

#include <cmath>

namespace ecmg {

__device__ __forceinline__ bool dir_node(const Geom &g, int i, int j, int k) {
    return (i == 0 && g.ft[0] == ECMG_DIRICHLET) || (i == g.nx && g.ft[1] == ECMG_DIRICHLET) ||
           (j == 0 && g.ft[2] == ECMG_DIRICHLET) || (j == g.ny && g.ft[3] == ECMG_DIRICHLET) ||
           (k == 0 && g.ft[4] == ECMG_DIRICHLET) || (k == g.nz && g.ft[5] == ECMG_DIRICHLET);
}

// In-face axes of face f: p, q; normal axis f/2.
__host__ __device__ __forceinline__ void face_axes(int f, int &p, int &q) {
    const int ax = f / 2;
    p = (ax == 0) ? 1 : 0;
    q = (ax == 2) ? 1 : 2;
}

// 1-D Q1 basis at a 2-point Gauss abscissa: node c (0/1) of the element, Gauss
// point gq (0 = nearer node 0).  (1 + xi_c s)/2 with xi_c = 2c-1, s = -+1/sqrt3.
__device__ __forceinline__ double phi1(int c, int gq) {
    const double G = 0.57735026918962576451;  // 1/sqrt(3)
    return (c == gq) ? 0.5 * (1.0 + G) : 0.5 * (1.0 - G);
}

__global__ void k_fill(double *p, int64_t n, double v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

__global__ void k_zero_free(const Geom g, double *x) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= g.nnodes) return;
    const int i = (int)(id % g.sx);
    if (i > g.nx) return;
    const int64_t t = id / g.sx;
    const int j = (int)(t % g.sy), k = (int)(t / g.sy);
    if (!dir_node(g, i, j, k)) x[id] = 0.0;
}

// F += int f phi_i over the elements of layers [e0, e1): fg holds f at the
// 2x2x2 Gauss points of those layers, (2(e1-e0)) x (2ny) x (2nx), x fastest.
__global__ void k_load_volume(const Geom g, int e0, int e1, const double *__restrict__ fg, double *F) {
    const int64_t nplane = (int64_t)g.sx * g.sy;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int kmax = min(e1, g.nz);
    if (tid >= nplane * (kmax - e0 + 1)) return;
    const int i = (int)(tid % g.sx);
    const int j = (int)((tid / g.sx) % g.sy);
    const int k = e0 + (int)(tid / nplane);
    const double w = g.h[0] * g.h[1] * g.h[2] / 8.0;
    const int64_t gx = 2 * (int64_t)g.nx, gy = 2 * (int64_t)g.ny;
    double s = 0.0;
    for (int ke = k - 1; ke <= k; ++ke) {
        if (ke < e0 || ke >= e1 || ke >= g.nz) continue;
        for (int je = j - 1; je <= j; ++je) {
            if (je < 0 || je >= g.ny) continue;
            for (int ie = i - 1; ie <= i; ++ie) {
                if (ie < 0 || ie >= g.nx) continue;
                const int cx = i - ie, cy = j - je, cz = k - ke;
                for (int qz = 0; qz < 2; ++qz)
                    for (int qy = 0; qy < 2; ++qy)
                        for (int qx = 0; qx < 2; ++qx) {
                            const double phi = phi1(cx, qx) * phi1(cy, qy) * phi1(cz, qz);
                            const double fv = fg[(2 * (int64_t)(ke - e0) + qz) * gy * gx + (2 * (int64_t)je + qy) * gx +
                                                 (2 * (int64_t)ie + qx)];
                            s += w * fv * phi;
                        }
            }
        }
    }
    F[i + g.sx * (int64_t)j + nplane * k] += s;
}

// F += int_f g_R phi_i over Robin face f: gR holds g_R at the face's 2x2 Gauss
// points, (2nq) x (2np), p fastest.
__global__ void k_load_face(const Geom g, int f, const double *__restrict__ gR, double *F) {
    int pax, qax;
    face_axes(f, pax, qax);
    const int n[3] = {g.nx, g.ny, g.nz};
    const int np = n[pax], nq = n[qax];
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (int64_t)(np + 1) * (nq + 1)) return;
    const int pi = (int)(tid % (np + 1)), qi = (int)(tid / (np + 1));
    const double w = g.h[pax] * g.h[qax] / 4.0;
    double s = 0.0;
    for (int eq = qi - 1; eq <= qi; ++eq) {
        if (eq < 0 || eq >= nq) continue;
        for (int ep = pi - 1; ep <= pi; ++ep) {
            if (ep < 0 || ep >= np) continue;
            const int cp = pi - ep, cq = qi - eq;
            for (int gq = 0; gq < 2; ++gq)
                for (int gp = 0; gp < 2; ++gp)
                    s += w * gR[(2 * (int64_t)eq + gq) * (2 * (int64_t)np) + 2 * ep + gp] * (phi1(cp, gp) * phi1(cq, gq));
        }
    }
    int idx[3];
    idx[f / 2] = (f & 1) ? n[f / 2] : 0;
    idx[pax] = pi;
    idx[qax] = qi;
    F[idx[0] + g.sx * ((int64_t)idx[1] + (int64_t)g.sy * idx[2])] += s;
}

// x = vals on the nodes of face f ((np+1) x (nq+1), p fastest).
__global__ void k_scatter_face(const Geom g, int f, const double *__restrict__ vals, double *x) {
    int pax, qax;
    face_axes(f, pax, qax);
    const int n[3] = {g.nx, g.ny, g.nz};
    const int np = n[pax], nq = n[qax];
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (int64_t)(np + 1) * (nq + 1)) return;
    const int pi = (int)(tid % (np + 1)), qi = (int)(tid / (np + 1));
    int idx[3];
    idx[f / 2] = (f & 1) ? n[f / 2] : 0;
    idx[pax] = pi;
    idx[qax] = qi;
    x[idx[0] + g.sx * ((int64_t)idx[1] + (int64_t)g.sy * idx[2])] = vals[tid];
}

// 1/diag(A) on free nodes, 0 on Dirichlet nodes.  diag(A)_i = C[0] * (sum of
// beta over the elements around i) + sum over Robin faces through i of
// hp*hq/9 * (sum of alpha over the face elements around i).
struct AlphaPtrs { const double *a[6]; };

// The preconditioner M^-1 of the level's CG iterations, one value per node:
// ECMG_jcg (Section 4.1) takes M = diag(A), so 1 / A_ii; ECMG_cg (plain CG,
// the variant Section 4.1 names for comparison) takes M = I, so 1 on free
// nodes.  Dirichlet nodes and row padding hold 0, which keeps them out of
// every search direction.
__global__ void k_dinv(const Geom g, const double *__restrict__ beta, const AlphaPtrs al, double *dinv, int plain_cg) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= g.nnodes) return;
    const int i = (int)(id % g.sx);
    const int64_t t = id / g.sx;
    const int j = (int)(t % g.sy), k = (int)(t / g.sy);
    if (i > g.nx || dir_node(g, i, j, k)) { dinv[id] = 0.0; return; }
    if (plain_cg) { dinv[id] = 1.0; return; }
    double s8 = 0.0;
    for (int ke = k - 1; ke <= k; ++ke) {
        if (ke < 0 || ke >= g.nz) continue;
        for (int je = j - 1; je <= j; ++je) {
            if (je < 0 || je >= g.ny) continue;
            for (int ie = i - 1; ie <= i; ++ie) {
                if (ie < 0 || ie >= g.nx) continue;
                s8 += beta[ie + (int64_t)g.nx * (je + (int64_t)g.ny * ke)];
            }
        }
    }
    double d = g.C[0] * s8;
    const int idx[3] = {i, j, k};
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int f = 0; f < 6; ++f) {
        if (g.ft[f] != ECMG_ROBIN) continue;
        if (idx[f / 2] != ((f & 1) ? n[f / 2] : 0)) continue;
        int pax, qax;
        face_axes(f, pax, qax);
        const int pi = idx[pax], qi = idx[qax], np = n[pax], nq = n[qax];
        double sa = 0.0;
        for (int eq = qi - 1; eq <= qi; ++eq) {
            if (eq < 0 || eq >= nq) continue;
            for (int ep = pi - 1; ep <= pi; ++ep) {
                if (ep < 0 || ep >= np) continue;
                sa += al.a[f][ep + (int64_t)np * eq];
            }
        }
        d += g.M[f][0] * sa;
    }
    dinv[id] = 1.0 / d;
}

__device__ __forceinline__ double wsum_dense(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---- dense direct solve of the coarse levels (DSOLVE) -------------------------
// Row fi of A_FF (free node `id`): for every free neighbour, the Q1 stiffness
// class coefficient times the sum of beta over the elements holding both nodes,
// plus the Robin face mass times the sum of alpha over the face elements holding
// both (when both lie on a Robin face).  Row-major, A[fi * nf + fj].
__device__ __forceinline__ void elem_range(int i, int d, int n, int &lo, int &hi) {
    lo = d > 0 ? i : i - 1;                      // elements along one axis holding i and i + d
    hi = d < 0 ? i - 1 : i;
    lo = max(lo, 0);
    hi = min(hi, n - 1);
}

__global__ void k_assemble_dense(const Geom g, const double *__restrict__ beta, const AlphaPtrs al,
                                 const int *__restrict__ fmap, double *__restrict__ A, int nf) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= g.nnodes) return;
    const int fi = fmap[id];
    if (fi < 0) return;
    const int i = (int)(id % g.sx);
    const int64_t t = id / g.sx;
    const int j = (int)(t % g.sy), k = (int)(t / g.sy);
    const int idx[3] = {i, j, k};
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int d[3] = {dx, dy, dz};
                const int ii = i + dx, jj = j + dy, kk = k + dz;
                if (ii < 0 || ii > g.nx || jj < 0 || jj > g.ny || kk < 0 || kk > g.nz) continue;
                const int fj = fmap[ii + (int64_t)g.sx * (jj + (int64_t)g.sy * kk)];
                if (fj < 0) continue;
                int lo[3], hi[3];
                for (int a = 0; a < 3; ++a) elem_range(idx[a], d[a], n[a], lo[a], hi[a]);
                double wb = 0.0;
                for (int ez = lo[2]; ez <= hi[2]; ++ez)
                    for (int ey = lo[1]; ey <= hi[1]; ++ey)
                        for (int ex = lo[0]; ex <= hi[0]; ++ex)
                            wb += beta[ex + (int64_t)g.nx * (ey + (int64_t)g.ny * ez)];
                const int m = (dx != 0) | ((dy != 0) << 1) | ((dz != 0) << 2);
                double v = g.C[m] * wb;
                for (int f = 0; f < 6; ++f) {
                    if (g.ft[f] != ECMG_ROBIN) continue;
                    const int ax = f / 2;
                    if (idx[ax] != ((f & 1) ? n[ax] : 0) || d[ax] != 0) continue;
                    int pax, qax;
                    face_axes(f, pax, qax);
                    int plo, phi, qlo, qhi;
                    elem_range(idx[pax], d[pax], n[pax], plo, phi);
                    elem_range(idx[qax], d[qax], n[qax], qlo, qhi);
                    double wa = 0.0;
                    for (int eq = qlo; eq <= qhi; ++eq)
                        for (int ep = plo; ep <= phi; ++ep) wa += al.a[f][ep + (int64_t)n[pax] * eq];
                    v += g.M[f][(d[pax] != 0) + (d[qax] != 0)] * wa;
                }
                A[(int64_t)fi * nf + fj] = v;
            }
}

// Copy the lower triangle (column-major: element (r, c), r > c, at r + c n) to
// the upper one, making the explicit inverse of the Cholesky routines full.
__global__ void k_symmetrize(double *A, int n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n * n) return;
    const int r = (int)(t % n), c = (int)(t / n);
    if (r < c) A[t] = A[c + (int64_t)r * n];
}

// x at the free nodes = A_FF^-1 (F - A x0) (x0 = g_D on Dirichlet nodes, 0 on
// free ones; q = A x0 on free rows).  Each workgroup gathers the right-hand
// side into LDS; a wave per row, lanes across the (symmetric, so row-major)
// inverse, fixed-order reduction.
constexpr int GEMV_NT = 512;

__global__ void __launch_bounds__(GEMV_NT) k_dsolve_gemv(int nf, const double *__restrict__ Ainv,
                                                         const int *__restrict__ freeid,
                                                         const double *__restrict__ F, const double *__restrict__ q,
                                                         double *__restrict__ x) {
    extern __shared__ double rhs[];
    for (int c = threadIdx.x; c < nf; c += GEMV_NT) {
        const int id = freeid[c];
        rhs[c] = F[id] - q[id];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int row = blockIdx.x * (GEMV_NT / 64) + wave; row < nf; row += gridDim.x * (GEMV_NT / 64)) {
        const double *Ar = Ainv + (int64_t)row * nf;
        double s = 0.0;
        for (int c = lane; c < nf; c += 64) s += Ar[c] * rhs[c];
        s = wsum_dense(s);
        if (lane == 0) x[freeid[row]] = s;
    }
}

void launch_assemble_dense(const Geom &g, const double *beta, const double *const *alpha, const int *fmap,
                           double *A, int nf, hipStream_t s) {
    AlphaPtrs al;
    for (int f = 0; f < 6; ++f) al.a[f] = alpha[f];
    hipLaunchKernelGGL(k_assemble_dense, dim3((unsigned)((g.nnodes + 255) / 256)), dim3(256), 0, s, g, beta, al, fmap,
                       A, nf);
}

void launch_symmetrize(double *A, int n, hipStream_t s) {
    const int64_t t = (int64_t)n * n;
    hipLaunchKernelGGL(k_symmetrize, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, A, n);
}

void launch_dsolve_gemv(int nf, const double *Ainv, const int *freeid, const double *F, const double *q, double *x,
                        hipStream_t s) {
    const int rows_per_block = GEMV_NT / 64;
    const int nb = std::max(1, std::min((nf + rows_per_block - 1) / rows_per_block, 1024));
    hipLaunchKernelGGL(k_dsolve_gemv, dim3(nb), dim3(GEMV_NT), sizeof(double) * nf, s, nf, Ainv, freeid, F, q, x);
}

// ---- reductions over node arrays (deterministic, last block finalises) ----------
__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// out[0] = max |v|, out[1] = sum v^2 with v supplied per node by `val`.
template <typename Val>
__device__ void reduce_max_sum(Val val, int64_t n, double *partials, unsigned *counter, double *out) {
    __shared__ double red[2][4];
    __shared__ int s_last;
    const int tid = threadIdx.x;
    double mx = 0.0, sm = 0.0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + tid; i < n; i += stride) {
        const double v = val(i);
        mx = fmax(mx, fabs(v));
        sm += v * v;
    }
    mx = wmax(mx);
    sm = wsum(sm);
    if ((tid & 63) == 0) { red[0][tid >> 6] = mx; red[1][tid >> 6] = sm; }
    __syncthreads();
    if (tid == 0) {
        double m = red[0][0], s = red[1][0];
        for (int w = 1; w < 4; ++w) { m = fmax(m, red[0][w]); s += red[1][w]; }
        __hip_atomic_store(partials + 2 * blockIdx.x, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(partials + 2 * blockIdx.x + 1, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        s_last = (atomicAdd(counter, 1u) == gridDim.x - 1);
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    mx = 0.0;
    sm = 0.0;
    for (int b = tid; b < (int)gridDim.x; b += blockDim.x) {
        mx = fmax(mx, __hip_atomic_load(partials + 2 * b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        sm += __hip_atomic_load(partials + 2 * b + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    mx = wmax(mx);
    sm = wsum(sm);
    __syncthreads();
    if ((tid & 63) == 0) { red[0][tid >> 6] = mx; red[1][tid >> 6] = sm; }
    __syncthreads();
    if (tid == 0) {
        double m = red[0][0], s = red[1][0];
        for (int w = 1; w < 4; ++w) { m = fmax(m, red[0][w]); s += red[1][w]; }
        out[0] = m;
        out[1] = s;
        __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void __launch_bounds__(256) k_rhs_norm(const Geom g, const double *F, const double *Ax0,
                                                  const double *x0, double *partials, unsigned *counter,
                                                  double *out) {
    auto val = [&](int64_t id) -> double {
        const int i = (int)(id % g.sx);
        if (i > g.nx) return 0.0;
        const int64_t t = id / g.sx;
        const int j = (int)(t % g.sy), k = (int)(t / g.sy);
        return dir_node(g, i, j, k) ? x0[id] : F[id] - Ax0[id];
    };
    reduce_max_sum(val, g.nnodes, partials, counter, out);
}

__global__ void __launch_bounds__(256) k_norms(const Geom g, const double *a, const double *b, const double *c,
                                               double *partials, unsigned *counter, double *out) {
    auto val = [&](int64_t i) -> double {
        if ((int)(i % g.sx) > g.nx) return 0.0;
        double v = a[i];
        if (b) v -= b[i];
        if (c) v -= c[i];
        return v;
    };
    reduce_max_sum(val, g.nnodes, partials, counter, out);
}

// ---- launchers ----------------------------------------------------------------
static inline unsigned nblk(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

__global__ void k_zero_u32(unsigned *p, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = 0u;
}

void launch_zero_u32(unsigned *p, int64_t n, hipStream_t s) {
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(nblk(n), 1024));
    hipLaunchKernelGGL(k_zero_u32, dim3(nb), dim3(256), 0, s, p, n);
}

void launch_fill(double *p, int64_t n, double v, hipStream_t s) {
    const unsigned nb = (unsigned)std::min<int64_t>(nblk(n), 8192);
    hipLaunchKernelGGL(k_fill, dim3(nb > 0 ? nb : 1), dim3(256), 0, s, p, n, v);
}

void launch_zero_free(const Geom &g, double *x, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_free, dim3(nblk(g.nnodes)), dim3(256), 0, s, g, x);
}

void launch_load_volume(const Geom &g, int e0, int e1, const double *fg, double *F, hipStream_t s) {
    const int kmax = std::min(e1, g.nz);
    const int64_t n = (int64_t)g.sx * g.sy * (kmax - e0 + 1);
    hipLaunchKernelGGL(k_load_volume, dim3(nblk(n)), dim3(256), 0, s, g, e0, e1, fg, F);
}

void launch_load_face(const Geom &g, int face, const double *gR, double *F, hipStream_t s) {
    int p, q;
    face_axes(face, p, q);
    const int n[3] = {g.nx, g.ny, g.nz};
    hipLaunchKernelGGL(k_load_face, dim3(nblk((int64_t)(n[p] + 1) * (n[q] + 1))), dim3(256), 0, s, g, face, gR, F);
}

void launch_scatter_face(const Geom &g, int face, const double *vals, double *x, hipStream_t s) {
    int p, q;
    face_axes(face, p, q);
    const int n[3] = {g.nx, g.ny, g.nz};
    hipLaunchKernelGGL(k_scatter_face, dim3(nblk((int64_t)(n[p] + 1) * (n[q] + 1))), dim3(256), 0, s, g, face,
                       vals, x);
}

void launch_dinv(const Geom &g, const double *beta, const double *const *alpha, double *dinv, int plain_cg,
                 hipStream_t s) {
    AlphaPtrs ap;
    for (int f = 0; f < 6; ++f) ap.a[f] = alpha[f];
    hipLaunchKernelGGL(k_dinv, dim3(nblk(g.nnodes)), dim3(256), 0, s, g, beta, ap, dinv, plain_cg);
}

void launch_rhs_norm(const Geom &g, const double *F, const double *Ax0, const double *x0, double *partials,
                     unsigned *counter, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_rhs_norm, dim3(reduce_blocks(g.nnodes)), dim3(256), 0, s, g, F, Ax0, x0, partials,
                       counter, out);
}

void launch_norms(const Geom &g, const double *a, const double *b, const double *c, double *partials,
                  unsigned *counter, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_norms, dim3(reduce_blocks(g.nnodes)), dim3(256), 0, s, g, a, b, c, partials, counter, out);
}

// dense node array (x fastest, no padding) <-> padded level layout
__global__ void k_pack(const Geom g, const double *__restrict__ padded, double *__restrict__ dense, int unpack) {
    const int w = g.nx + 1;
    const int64_t rows = (int64_t)g.sy * (g.nz + 1);
    for (int64_t row = blockIdx.x; row < rows; row += gridDim.x) {
        const int64_t d0 = row * w, p0 = row * g.sx;
        for (int i = threadIdx.x; i < w; i += blockDim.x) {
            if (unpack) ((double *)padded)[p0 + i] = dense[d0 + i];
            else dense[d0 + i] = padded[p0 + i];
        }
    }
}

void launch_pack(const Geom &g, const double *padded, double *dense, hipStream_t s) {
    const int64_t nb = std::max<int64_t>(1, std::min<int64_t>((int64_t)g.sy * (g.nz + 1), 65536));
    hipLaunchKernelGGL(k_pack, dim3((unsigned)nb), dim3(256), 0, s, g, padded, dense, 0);
}

void launch_unpack(const Geom &g, const double *dense, double *padded, hipStream_t s) {
    const int64_t nb = std::max<int64_t>(1, std::min<int64_t>((int64_t)g.sy * (g.nz + 1), 65536));
    hipLaunchKernelGGL(k_pack, dim3((unsigned)nb), dim3(256), 0, s, g, (const double *)padded, (double *)dense, 1);
}

}  // namespace ecmg
