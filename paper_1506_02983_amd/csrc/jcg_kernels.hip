// JCG kernels for gfx950: the matrix-free Q1 stencil (operator apply, JCG
// initialisation, fused JCG pass A), JCG pass B, the deferred x update, and
// the deterministic reductions that drive the relative-residual stop of
// Algorithm 4.
//
// Operator (Section 2, a(u,v) = int beta grad u.grad v + int_R alpha u v): with
// beta constant per element, the row of node i is
//   (A v)_i = sum_{o in {-1,0,1}^3} C[mask(o)] * (sum of beta over the elements
//             containing both i and i+o) * v_{i+o}  +  Robin face-mass terms,
// where mask(o) marks the axes on which o is nonzero and C holds the Q1 element
// stiffness classes (tensor products of 1-D stiffness and mass).
//
// JCG (Section 4.1: CG preconditioned with M = diag(A)) is split into two
// streaming passes per iteration k:
//   pass A: x += alpha_{k-1} p_{k-1};  p_k = D^-1 r_k + beta_k p_{k-1};
//           q = A p_k;  partial p_k.q            (last block: alpha_k = rho_k/p.q)
//   pass B: r_{k+1} = r_k - alpha_k q;  z = D^-1 r_{k+1};  partials r.z, r.r
//           (last block: beta_{k+1} = rho_{k+1}/rho_k and the stop test
//            ||r_{k+1}|| <= eps ||f_h||, the `while` of Algorithm 4)
// Every kernel reads the device `done` flag first and returns if it is set, so
// the host can enqueue iterations in chunks and the iterate freezes exactly at
// the stopping iteration.
//
// Data layout in HBM: node (i,j,k) at i + sx*(j + sy*k) (x fastest, each
// z-plane contiguous); element arrays likewise over nx*ny*nz.  The stencil
// kernels tile x-y planes (TX lanes along x, coalesced rows) and march through
// KZ planes in z with a rolling 3-plane buffer of the input vector and a
// 2-layer buffer of element coefficients in LDS, so each HBM byte is read once
// per pass apart from tile halos.
#include "ecmg_internal.h"

#include <cmath>

namespace ecmg {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------

// Consecutive workgroups are dispatched round-robin over the 8 XCDs.  Map them
// so that each XCD receives one contiguous range of tiles (neighbouring tiles
// then share halo lines in that XCD's L2).
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int per = nb / NXCD;
    if (b < per * NXCD) return (b % NXCD) * per + b / NXCD;
    return b;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ void store_agent(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_agent(const double *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum NV values over the block in a fixed order (lane shuffles, then waves in
// index order).  Result valid in thread 0.
template <int NV, int NTHREADS>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*red)[NTHREADS / 64]) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    if ((tid & 63) == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) red[i][tid >> 6] = v[i];
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            double s = red[i][0];
            for (int w = 1; w < NTHREADS / 64; ++w) s += red[i][w];
            v[i] = s;
        }
    }
    __syncthreads();
}

// Two-stage deterministic reduction: every block stores its partials, the last
// block to arrive sums all partials in block order.  Returns true in the last
// block, where tot[] (thread 0) holds the totals.
template <int NV, int NTHREADS>
__device__ __forceinline__ bool last_block_total(double (&acc)[NV], double (*red)[NTHREADS / 64], int *s_last,
                                                 double *partials, unsigned *counter, int bid, int nb,
                                                 double (&tot)[NV]) {
    block_sum<NV, NTHREADS>(acc, red);
    const int tid = threadIdx.x;
    if (tid == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) store_agent(partials + (int64_t)NV * bid + i, acc[i]);
        __threadfence();
        const unsigned prev = atomicAdd(counter, 1u);
        *s_last = (prev == (unsigned)(nb - 1));
    }
    __syncthreads();
    if (!*s_last) return false;
    __threadfence();
#pragma unroll
    for (int i = 0; i < NV; ++i) tot[i] = 0.0;
    for (int b = tid; b < nb; b += NTHREADS) {
#pragma unroll
        for (int i = 0; i < NV; ++i) tot[i] += load_agent(partials + (int64_t)NV * b + i);
    }
    block_sum<NV, NTHREADS>(tot, red);
    if (tid == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
}

__device__ __forceinline__ bool is_dirichlet(const Geom &g, int i, int j, int k) {
    return (i == 0 && g.ft[0] == ECMG_DIRICHLET) || (i == g.nx && g.ft[1] == ECMG_DIRICHLET) ||
           (j == 0 && g.ft[2] == ECMG_DIRICHLET) || (j == g.ny && g.ft[3] == ECMG_DIRICHLET) ||
           (k == 0 && g.ft[4] == ECMG_DIRICHLET) || (k == g.nz && g.ft[5] == ECMG_DIRICHLET);
}

// Robin face-mass term of face F (axis AX = F/2) at a node whose in-face
// coordinates are (pi, qi), using the 3x3x3 neighbourhood v (index [oz][oy][ox]).
// Face elements around the node: (ep, eq) = (pi-1+dp, qi-1+dq); the node sits
// at local corner (1-dp, 1-dq) of each; the face mass couples it to the face
// element's 4 corners with hp*hq*(1/9, 1/18, 1/36) by the number of differing
// in-face axes.
template <int AX, typename T>
__device__ __forceinline__ T robin_term(const Geom &g, int face, const T *al, int pi, int qi, int np, int nq,
                                        const T (&v)[3][3][3]) {
    T s = 0;
#pragma unroll
    for (int dq = 0; dq < 2; ++dq) {
        const int eq = qi - 1 + dq;
        if (eq < 0 || eq >= nq) continue;
#pragma unroll
        for (int dp = 0; dp < 2; ++dp) {
            const int ep = pi - 1 + dp;
            if (ep < 0 || ep >= np) continue;
            const T a = al[ep + (int64_t)np * eq];
            T t = 0;
#pragma unroll
            for (int bq = 0; bq < 2; ++bq)
#pragma unroll
                for (int bp = 0; bp < 2; ++bp) {
                    const int op = dp - 1 + bp, oq = dq - 1 + bq;
                    const int c = (bp != 1 - dp) + (bq != 1 - dq);
                    T vv;
                    if (AX == 0) vv = v[oq + 1][op + 1][1];
                    else if (AX == 1) vv = v[oq + 1][1][op + 1];
                    else vv = v[1][oq + 1][op + 1];
                    t += (T)g.M[face][c] * vv;
                }
            s += a * t;
        }
    }
    return s;
}

// ---------------------------------------------------------------------------
// tiled stencil kernel: MODE_APPLY (q = A v), MODE_INIT (r = F - A x, r.z, r.r),
// MODE_PASSA (fused JCG pass A)
// ---------------------------------------------------------------------------

template <typename T, int MODE>
__global__ void __launch_bounds__(NT) k_stencil(const StencilArgs<T> a) {
    __shared__ T sv[3][TYT + 2][TX + 2];   // input vector, planes k-1, k, k+1 (+ halo)
    __shared__ T sb[2][TYT + 1][TX + 1];   // beta of element layers k-1, k (+ halo)
    __shared__ double red[2][NT / 64];
    __shared__ int s_last;

    const Geom &g = a.g;
    const int tid = threadIdx.x, tx = tid & (TX - 1), ty = tid / TX;
    const int w = xcd_remap(blockIdx.x, gridDim.x);
    const int bx = w % a.ntx;
    const int byz = w / a.ntx;
    const int by = byz % a.nty;
    const int bz = byz / a.nty;
    const int i0 = bx * TX, j0 = by * TYT;
    const int k0 = bz * a.KZ;
    const int k1 = min(k0 + a.KZ, g.nz + 1);

    bool first = true;
    T alpha_prev = 0, betak = 0;
    const T *pin = a.p0;
    T *pout = a.p1;
    if (MODE == MODE_PASSA) {
        const JcgScalars *sc = a.sc;
        if (sc->done) return;                     // uniform over the grid
        const int it = sc->iter;
        first = (it == 0);
        alpha_prev = (T)sc->alpha;
        betak = (T)sc->beta;
        pin = (it & 1) ? a.p1 : a.p0;
        pout = (it & 1) ? a.p0 : a.p1;
    }

    const int64_t sx = g.sx, sxy = (int64_t)g.sx * g.sy;
    T pold_next[RY], pold_cur[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) pold_next[r] = pold_cur[r] = 0;

    // value of the stencil input at node (i,j,k): v, or for pass A the new
    // search direction D^-1 r + beta p_old; 0 outside the grid
    auto node_val = [&](int i, int j, int k, T &pold) -> T {
        if (i < 0 || i > g.nx || j < 0 || j > g.ny || k < 0 || k > g.nz) { pold = 0; return 0; }
        const int64_t id = i + sx * j + sxy * k;
        if (MODE == MODE_PASSA) {
            const T z = a.dinv[id] * a.r[id];
            if (first) { pold = 0; return z; }
            pold = pin[id];
            return z + betak * pold;
        } else {
            pold = 0;
            return a.v[id];
        }
    };
    auto load_plane = [&](int k, int slot) {
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int jj = ty + TY * r;
            T po;
            sv[slot][jj + 1][tx + 1] = node_val(i0 + tx, j0 + jj, k, po);
            pold_next[r] = po;
        }
        constexpr int NH = 2 * (TX + 2) + 2 * TYT;
        for (int h = tid; h < NH; h += NT) {
            int li, lj;
            if (h < TX + 2) { lj = 0; li = h; }
            else if (h < 2 * (TX + 2)) { lj = TYT + 1; li = h - (TX + 2); }
            else if (h < 2 * (TX + 2) + TYT) { li = 0; lj = 1 + h - 2 * (TX + 2); }
            else { li = TX + 1; lj = 1 + h - 2 * (TX + 2) - TYT; }
            T po;
            sv[slot][lj][li] = node_val(i0 + li - 1, j0 + lj - 1, k, po);
        }
    };
    auto elem_val = [&](int ie, int je, int ke) -> T {
        if (ie < 0 || ie >= g.nx || je < 0 || je >= g.ny || ke < 0 || ke >= g.nz) return 0;
        return a.beta[ie + (int64_t)g.nx * (je + (int64_t)g.ny * ke)];
    };
    auto load_beta = [&](int ke, int slot) {
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int jj = ty + TY * r;
            sb[slot][jj + 1][tx + 1] = elem_val(i0 + tx, j0 + jj, ke);
        }
        constexpr int NHB = (TX + 1) + TYT;
        for (int h = tid; h < NHB; h += NT) {
            int li, lj;
            if (h < TX + 1) { lj = 0; li = h; }
            else { li = 0; lj = 1 + h - (TX + 1); }
            sb[slot][lj][li] = elem_val(i0 + li - 1, j0 + lj - 1, ke);
        }
    };
    auto vslot = [](int k) { return (k + 3) % 3; };
    auto bslot = [](int k) { return (k + 2) & 1; };

    T C[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) C[m] = (T)g.C[m];

    double acc0 = 0.0, acc1 = 0.0;

    load_plane(k0 - 1, vslot(k0 - 1));
    load_plane(k0, vslot(k0));
    load_beta(k0 - 1, bslot(k0 - 1));

    for (int k = k0; k < k1; ++k) {
#pragma unroll
        for (int r = 0; r < RY; ++r) pold_cur[r] = pold_next[r];
        load_plane(k + 1, vslot(k + 1));
        load_beta(k, bslot(k));
        __syncthreads();

        const int s0 = vslot(k - 1), s1 = vslot(k), s2 = vslot(k + 1);
        const int b0 = bslot(k - 1), b1 = bslot(k);
        const int i = i0 + tx;
#pragma unroll
        for (int r = 0; r < RY; ++r) {
            const int jj = ty + TY * r;
            const int j = j0 + jj;
            const int li = tx + 1, lj = jj + 1;
            T v[3][3][3];
#pragma unroll
            for (int oy = 0; oy < 3; ++oy)
#pragma unroll
                for (int ox = 0; ox < 3; ++ox) {
                    v[0][oy][ox] = sv[s0][lj - 1 + oy][li - 1 + ox];
                    v[1][oy][ox] = sv[s1][lj - 1 + oy][li - 1 + ox];
                    v[2][oy][ox] = sv[s2][lj - 1 + oy][li - 1 + ox];
                }
            T b[2][2][2];
#pragma unroll
            for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                for (int dx = 0; dx < 2; ++dx) {
                    b[0][dy][dx] = sb[b0][lj - 1 + dy][li - 1 + dx];
                    b[1][dy][dx] = sb[b1][lj - 1 + dy][li - 1 + dx];
                }
            // partial sums of beta over x, then y (elements sharing an edge/face)
            T q = 0;
#pragma unroll
            for (int oz = -1; oz <= 1; ++oz)
#pragma unroll
                for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
                    for (int ox = -1; ox <= 1; ++ox) {
                        T wsum = 0;
#pragma unroll
                        for (int dz = (oz > 0); dz <= (oz < 0 ? 0 : 1); ++dz)
#pragma unroll
                            for (int dy = (oy > 0); dy <= (oy < 0 ? 0 : 1); ++dy)
#pragma unroll
                                for (int dx = (ox > 0); dx <= (ox < 0 ? 0 : 1); ++dx) wsum += b[dz][dy][dx];
                        const int m = (ox != 0) | ((oy != 0) << 1) | ((oz != 0) << 2);
                        q += C[m] * wsum * v[oz + 1][oy + 1][ox + 1];
                    }
            if (i > g.nx || j > g.ny) continue;
            // Robin faces
            if (i == 0 && g.ft[0] == ECMG_ROBIN) q += robin_term<0>(g, 0, a.alpha[0], j, k, g.ny, g.nz, v);
            if (i == g.nx && g.ft[1] == ECMG_ROBIN) q += robin_term<0>(g, 1, a.alpha[1], j, k, g.ny, g.nz, v);
            if (j == 0 && g.ft[2] == ECMG_ROBIN) q += robin_term<1>(g, 2, a.alpha[2], i, k, g.nx, g.nz, v);
            if (j == g.ny && g.ft[3] == ECMG_ROBIN) q += robin_term<1>(g, 3, a.alpha[3], i, k, g.nx, g.nz, v);
            if (k == 0 && g.ft[4] == ECMG_ROBIN) q += robin_term<2>(g, 4, a.alpha[4], i, j, g.nx, g.ny, v);
            if (k == g.nz && g.ft[5] == ECMG_ROBIN) q += robin_term<2>(g, 5, a.alpha[5], i, j, g.nx, g.ny, v);
            const bool dir = is_dirichlet(g, i, j, k);
            const int64_t id = i + sx * j + sxy * k;
            if (MODE == MODE_APPLY) {
                a.q[id] = dir ? (T)0 : q;
            } else if (MODE == MODE_INIT) {
                const T rv = dir ? (T)0 : a.F[id] - q;
                a.r[id] = rv;
                const T z = a.dinv[id] * rv;
                acc0 += (double)rv * (double)z;
                acc1 += (double)rv * (double)rv;
            } else {
                const T pc = v[1][1][1];
                const T qv = dir ? (T)0 : q;
                pout[id] = pc;
                a.q[id] = qv;
                if (!first) a.x[id] += alpha_prev * pold_cur[r];
                acc0 += (double)pc * (double)qv;
            }
        }
        __syncthreads();
    }

    if (MODE == MODE_APPLY) return;

    if (MODE == MODE_INIT) {
        double acc[2] = {acc0, acc1}, tot[2];
        if (last_block_total<2, NT>(acc, red, &s_last, a.partials, a.counter, blockIdx.x, gridDim.x, tot) &&
            tid == 0) {
            JcgScalars *sc = a.sc;
            sc->rho = tot[0];
            sc->rr = tot[1];
            sc->iter = 0;
            sc->alpha = 0.0;
            sc->beta = 0.0;
            sc->pending = 0;
            const double rn = sqrt(tot[1]);
            if (sc->fixed >= 0) sc->done = (sc->fixed == 0) ? DONE_CONVERGED : DONE_RUNNING;
            else if (!(rn > sc->tol)) sc->done = DONE_CONVERGED;
            else sc->done = (sc->max_iter <= 0) ? DONE_MAXITER : DONE_RUNNING;
        }
    } else {
        double acc[1] = {acc0}, tot[1];
        if (last_block_total<1, NT>(acc, red, &s_last, a.partials, a.counter, blockIdx.x, gridDim.x, tot) &&
            tid == 0) {
            JcgScalars *sc = a.sc;
            const double pq = tot[0];
            sc->pq = pq;
            sc->pending = 0;
            if (!(pq > 0.0) || !isfinite(pq)) sc->done = DONE_BREAKDOWN;
            else sc->alpha = sc->rho / pq;
        }
    }
}

// ---------------------------------------------------------------------------
// pass B: r -= alpha q; z = D^-1 r; r.z, r.r; stop test
// ---------------------------------------------------------------------------
constexpr int NTB = 256;

template <typename T>
__global__ void __launch_bounds__(NTB) k_passB(const PassBArgs<T> a) {
    __shared__ double red[2][NTB / 64];
    __shared__ int s_last;
    JcgScalars *sc = a.sc;
    if (sc->done) return;
    const T al = (T)sc->alpha;
    const int64_t stride = (int64_t)gridDim.x * NTB;
    double rz = 0.0, rr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NTB + threadIdx.x; i < a.n; i += stride) {
        const T rv = a.r[i] - al * a.q[i];
        a.r[i] = rv;
        const T z = a.dinv[i] * rv;
        rz += (double)rv * (double)z;
        rr += (double)rv * (double)rv;
    }
    double acc[2] = {rz, rr}, tot[2];
    if (last_block_total<2, NTB>(acc, red, &s_last, a.partials, a.counter, blockIdx.x, gridDim.x, tot) &&
        threadIdx.x == 0) {
        const int it = sc->iter + 1;
        sc->iter = it;
        const double rho_old = sc->rho;
        sc->beta = tot[0] / rho_old;
        sc->rho = tot[0];
        sc->rr = tot[1];
        sc->pending = 1;
        const double rn = sqrt(tot[1]);
        if (sc->fixed >= 0) sc->done = (it >= sc->fixed) ? DONE_CONVERGED : DONE_RUNNING;
        else if (!(rn > sc->tol)) sc->done = DONE_CONVERGED;
        else if (it >= sc->max_iter) sc->done = DONE_MAXITER;
    }
}

// x += alpha p of the last iteration (after the host has seen `done`).
template <typename T>
__global__ void k_final_x(int64_t n, T *x, const T *p0, const T *p1, const JcgScalars *sc) {
    if (!sc->pending) return;
    const T al = (T)sc->alpha;
    const T *p = (sc->iter & 1) ? p1 : p0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] += al * p[i];
}

__global__ void k_jcg_reset(JcgScalars *sc, double tol, int max_iter, int fixed) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        sc->rho = sc->rr = sc->alpha = sc->beta = sc->pq = 0.0;
        sc->tol = tol;
        sc->iter = 0;
        sc->done = 0;
        sc->max_iter = max_iter;
        sc->fixed = fixed;
        sc->pending = 0;
        sc->pad = 0;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

int stencil_blocks(const Geom &g, int KZ, int *ntx, int *nty, int *nkz) {
    *ntx = (g.sx + TX - 1) / TX;
    *nty = (g.sy + TYT - 1) / TYT;
    *nkz = (g.nz + 1 + KZ - 1) / KZ;
    return (*ntx) * (*nty) * (*nkz);
}

template <typename T>
void launch_stencil(int mode, const StencilArgs<T> &a, hipStream_t s) {
    const int nb = a.ntx * a.nty * a.nkz;
    if (mode == MODE_APPLY) hipLaunchKernelGGL((k_stencil<T, MODE_APPLY>), dim3(nb), dim3(NT), 0, s, a);
    else if (mode == MODE_INIT) hipLaunchKernelGGL((k_stencil<T, MODE_INIT>), dim3(nb), dim3(NT), 0, s, a);
    else hipLaunchKernelGGL((k_stencil<T, MODE_PASSA>), dim3(nb), dim3(NT), 0, s, a);
}

template <typename T>
void launch_passB(const PassBArgs<T> &a, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL((k_passB<T>), dim3(nblocks), dim3(NTB), 0, s, a);
}

void launch_final_x(const Geom &g, double *x, const double *p0, const double *p1, const JcgScalars *sc,
                    hipStream_t s) {
    const int nb = (int)std::min<int64_t>((g.nnodes + 255) / 256, 4096);
    hipLaunchKernelGGL((k_final_x<double>), dim3(nb), dim3(256), 0, s, g.nnodes, x, p0, p1, sc);
}

void launch_jcg_reset(JcgScalars *sc, double tol, int max_iter, int fixed, hipStream_t s) {
    hipLaunchKernelGGL(k_jcg_reset, dim3(1), dim3(64), 0, s, sc, tol, max_iter, fixed);
}

int reduce_blocks(int64_t n) {
    const int64_t per = (int64_t)NTB * 8;
    int64_t nb = (n + per - 1) / per;
    if (nb < 1) nb = 1;
    if (nb > 2048) nb = 2048;
    return (int)nb;
}

template void launch_stencil<double>(int, const StencilArgs<double> &, hipStream_t);
template void launch_passB<double>(const PassBArgs<double> &, int, hipStream_t);

}  // namespace ecmg
