// Inter-level kernels: EXP_finite (Sections 4.2.2-4.3) and EXP_true (Section
// 4.2.1 and the end of Section 4.3).
//
// EXP_finite builds W on level l from U1 = u_{l-1} and U0 = u_{l-2}.  Each
// coarse (level l-2) element holds 5x5x5 fine nodes at local offsets (a,b,c) in
// {0..4}^3; the 27 offsets in {0,2,4}^3 are level l-1 nodes.  Nodal values at
// those 27 offsets:
//   corners      W = (5 U1 - U0) / 4                           (eq. jiedian)
//   mid-edges    W = U1 + (U1 - U0 at both ends) / 8           (eq. zhongdian)
//   face/body centres:
//     serendipity form: the value the 20-node serendipity interpolant (eq.
//       inter) takes there, -1/4 sum(face corners) + 1/2 sum(face mid-edges) and
//       -1/4 sum(8 corners) + 1/4 sum(12 mid-edges);
//     Lagrange form (the Remark): the mean of eq. zhongdian along the 2 face
//       diagonals or the 4 space diagonals.
// Every other fine node is the tri-quadratic Lagrange interpolant of the 27
// values.  For the serendipity form this equals eq. inter exactly, because the
// serendipity interpolant is itself tri-quadratic and so is reproduced by
// 27-node Lagrange interpolation of its own values; the tensor-product form
// skips the vanishing 1-D weights instead of evaluating 20 three-dimensional
// shape functions.  A fine node on a face shared by two coarse elements belongs
// to the lower-index element (both give the same value up to rounding).
//
// The 27 nodal values sit on level l-1 nodes and each depends only on its own
// edge, face or element, so phase 1 computes them once per level l-1 node (into
// scratch) and phase 2 interpolates every fine node from them.
#include "ecmg_internal.h"

namespace ecmg {

// 1-D quadratic Lagrange weights at natural coordinate t = a/2 - 1, a in 0..4,
// for the nodes t = -1, 0, 1.
__device__ __forceinline__ void lagrange3(int a, double (&L)[3]) {
    switch (a) {
        case 0: L[0] = 1.0; L[1] = 0.0; L[2] = 0.0; break;
        case 1: L[0] = 0.375; L[1] = 0.75; L[2] = -0.125; break;
        case 2: L[0] = 0.0; L[1] = 1.0; L[2] = 0.0; break;
        case 3: L[0] = -0.125; L[1] = 0.75; L[2] = 0.375; break;
        default: L[0] = 0.0; L[1] = 0.0; L[2] = 1.0; break;
    }
}

__device__ __forceinline__ bool is_dir(const Geom &g, int i, int j, int k) {
    return (i == 0 && g.ft[0] == ECMG_DIRICHLET) || (i == g.nx && g.ft[1] == ECMG_DIRICHLET) ||
           (j == 0 && g.ft[2] == ECMG_DIRICHLET) || (j == g.ny && g.ft[3] == ECMG_DIRICHLET) ||
           (k == 0 && g.ft[4] == ECMG_DIRICHLET) || (k == g.nz && g.ft[5] == ECMG_DIRICHLET);
}

// Phase 1 of EXP_finite, on the level l-1 grid (node (p,q,r), level l-2 nodes
// at even indices): the 27-point nodal value V of the level l-2 element(s)
// containing the node.  Every such value depends only on the node's own edge,
// face or element, so it is single-valued across neighbouring coarse elements.
__device__ __forceinline__ double u_at(const double *U, int64_t sx, int64_t sxy, int p, int q, int r) {
    return U[p + sx * q + sxy * r];
}

__device__ __forceinline__ void exp_finite_nodal_block(const Geom &g1, const double *__restrict__ U1,
                                                       const double *__restrict__ U0, double *__restrict__ V,
                                                       int variant, int bx, int by, int bz) {
    const int p = bx * 64 + threadIdx.x;
    const int q = by * 4 + threadIdx.y, r = bz;
    if (p > g1.nx || q > g1.ny || r > g1.nz) return;
    const int64_t s1 = g1.sx, s1y = (int64_t)g1.sx * g1.sy;
    const int64_t s0 = row_pitch(g1.nx / 2 + 1), s0y = s0 * (g1.ny / 2 + 1);
    // eq. jiedian at a level l-2 node (all indices even)
    auto Wc = [&](int pp, int qq, int rr) {
        return (5.0 * u_at(U1, s1, s1y, pp, qq, rr) - u_at(U0, s0, s0y, pp >> 1, qq >> 1, rr >> 1)) / 4.0;
    };
    auto del = [&](int pp, int qq, int rr) {
        return u_at(U1, s1, s1y, pp, qq, rr) - u_at(U0, s0, s0y, pp >> 1, qq >> 1, rr >> 1);
    };
    // eq. zhongdian at the midpoint (pp,qq,rr) of the edge along axis ax
    auto Wm = [&](int pp, int qq, int rr, int ax) {
        const int dp = ax == 0, dq = ax == 1, dr = ax == 2;
        return u_at(U1, s1, s1y, pp, qq, rr) + (del(pp - dp, qq - dq, rr - dr) + del(pp + dp, qq + dq, rr + dr)) / 8.0;
    };
    const int op = p & 1, oq = q & 1, orr = r & 1;
    const int nodd = op + oq + orr;
    double v;
    if (nodd == 0) {
        v = Wc(p, q, r);
    } else if (nodd == 1) {
        v = Wm(p, q, r, op ? 0 : (oq ? 1 : 2));
    } else if (nodd == 2) {
        // face centre; in-face axes A < B (the two odd ones)
        const int A = op ? 0 : 1, B = orr ? 2 : 1;
        auto at = [&](int sa, int sb) {                  // offset sa along A, sb along B
            int3 c = make_int3(p, q, r);
            if (A == 0) c.x += sa; else c.y += sa;
            if (B == 1) c.y += sb; else c.z += sb;
            return c;
        };
        if (variant == ECMG_SERENDIPITY20) {
            // value of the face's 8-node serendipity interpolant at its centre:
            // -1/4 (4 corners) + 1/2 (4 mid-edges)
            double sc = 0.0, sm = 0.0;
            for (int sb = -1; sb <= 1; sb += 2)
                for (int sa = -1; sa <= 1; sa += 2) {
                    const int3 c = at(sa, sb);
                    sc += Wc(c.x, c.y, c.z);
                }
            for (int s = -1; s <= 1; s += 2) {
                const int3 ea = at(0, s);                // edge along A at B offset s
                const int3 eb = at(s, 0);                // edge along B at A offset s
                sm += Wm(ea.x, ea.y, ea.z, A) + Wm(eb.x, eb.y, eb.z, B);
            }
            v = -0.25 * sc + 0.5 * sm;
        } else {
            // mean of eq. zhongdian along the two face diagonals
            const double u = u_at(U1, s1, s1y, p, q, r);
            const int3 a0 = at(-1, -1), a1 = at(1, 1), b0 = at(-1, 1), b1 = at(1, -1);
            v = ((u + (del(a0.x, a0.y, a0.z) + del(a1.x, a1.y, a1.z)) / 8.0) +
                 (u + (del(b0.x, b0.y, b0.z) + del(b1.x, b1.y, b1.z)) / 8.0)) / 2.0;
        }
    } else {
        if (variant == ECMG_SERENDIPITY20) {
            // -1/4 (8 corners) + 1/4 (12 mid-edges)
            double sc = 0.0, sm = 0.0;
            for (int c = -1; c <= 1; c += 2)
                for (int b = -1; b <= 1; b += 2)
                    for (int a = -1; a <= 1; a += 2) sc += Wc(p + a, q + b, r + c);
            for (int t = -1; t <= 1; t += 2)
                for (int u2 = -1; u2 <= 1; u2 += 2)
                    sm += Wm(p, q + t, r + u2, 0) + Wm(p + t, q, r + u2, 1) + Wm(p + t, q + u2, r, 2);
            v = -0.25 * sc + 0.25 * sm;
        } else {
            // mean of eq. zhongdian along the 4 space diagonals
            const double m = u_at(U1, s1, s1y, p, q, r);
            double sum = 0.0;
            for (int b = -1; b <= 1; b += 2)
                for (int c = -1; c <= 1; c += 2)
                    sum += m + (del(p - 1, q - b, r - c) + del(p + 1, q + b, r + c)) / 8.0;
            v = sum / 4.0;
        }
    }
    V[p + s1 * q + s1y * r] = v;
}

__global__ void __launch_bounds__(256) k_exp_finite_nodal(const Geom g1, const double *__restrict__ U1,
                                                          const double *__restrict__ U0, double *__restrict__ V,
                                                          int variant) {
    exp_finite_nodal_block(g1, U1, U0, V, variant, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Phase 2: every fine node of level l is the tri-quadratic Lagrange
// interpolant of the 27 nodal values of its owner coarse element.  A thread
// takes one coarse element I along x and one fine row (j, k): the 4 fine
// nodes 4I..4I+3 (and 4I+4 at the end of the row).  For each coarse row with a
// nonzero y / z weight (1, 3 or 9 of them, uniform over the wave) it loads the
// element's 3 nodal values with one 16-byte and one 8-byte load and folds
// them into 3 x-column sums; the fine nodes are then fixed combinations of the
// column sums, written as 16-byte stores.  Few wide loads per node matter:
// the inter-level kernels are bound by address processing, not bytes.
__device__ __forceinline__ void exp_finite_interp_block(const Geom &gf, const double *__restrict__ V,
                                                        double *__restrict__ x, double *__restrict__ W, int bx,
                                                        int by, int bz) {
    const int NX = gf.nx / 4, NY = gf.ny / 4, NZ = gf.nz / 4;
    const int I = bx * 64 + threadIdx.x;
    const int j = by * 4 + threadIdx.y, k = bz;
    if (I >= NX || j > gf.ny || k > gf.nz) return;
    const int J = min(j / 4, NY - 1), K = min(k / 4, NZ - 1);
    const int b = j - 4 * J, c = k - 4 * K;
    const int64_t s1 = row_pitch(gf.nx / 2 + 1), s1y = s1 * (gf.ny / 2 + 1);
    double Ly[3], Lz[3];
    lagrange3(b, Ly);
    lagrange3(c, Lz);
    const double *Vb = V + (2 * I) + s1 * (2 * J) + s1y * (2 * K);
    double w0 = 0.0, w1 = 0.0, w2 = 0.0;                  // weighted sums of the 3 x-columns
    for (int cc = 0; cc < 3; ++cc) {
        if (Lz[cc] == 0.0) continue;                      // uniform over the wave
        double t0 = 0.0, t1 = 0.0, t2 = 0.0;
        for (int bb = 0; bb < 3; ++bb) {
            if (Ly[bb] == 0.0) continue;                  // uniform over the wave
            const double *Vr = Vb + s1 * bb + s1y * cc;
            const double2 v01 = *(const double2 *)Vr;     // 2I is even: 16-byte aligned
            const double v2 = Vr[2];
            t0 += Ly[bb] * v01.x;
            t1 += Ly[bb] * v01.y;
            t2 += Ly[bb] * v2;
        }
        w0 += Lz[cc] * t0;
        w1 += Lz[cc] * t1;
        w2 += Lz[cc] * t2;
    }
    // x weights at a = 0..4 (natural coordinate a/2 - 1): (1,0,0), (3/8,3/4,-1/8),
    // (0,1,0), (-1/8,3/4,3/8), (0,0,1)
    double out[5];
    out[0] = w0;
    out[1] = 0.375 * w0 + 0.75 * w1 - 0.125 * w2;
    out[2] = w1;
    out[3] = -0.125 * w0 + 0.75 * w1 + 0.375 * w2;
    out[4] = w2;
    const int i0 = 4 * I;
    const int64_t id = i0 + (int64_t)gf.sx * j + (int64_t)gf.sx * gf.sy * k;
    const bool dj = (j == 0 && gf.ft[2] == ECMG_DIRICHLET) || (j == gf.ny && gf.ft[3] == ECMG_DIRICHLET) ||
                    (k == 0 && gf.ft[4] == ECMG_DIRICHLET) || (k == gf.nz && gf.ft[5] == ECMG_DIRICHLET);
    const int na = (I == NX - 1) ? 5 : 4;
    if (W) {
        *(double2 *)(W + id) = make_double2(out[0], out[1]);   // 4I: 32-byte aligned
        *(double2 *)(W + id + 2) = make_double2(out[2], out[3]);
        if (na == 5) W[id + 4] = out[4];
    }
    if (dj) return;                                       // the whole row is Dirichlet
    const bool d0 = (i0 == 0 && gf.ft[0] == ECMG_DIRICHLET);
    const bool d4 = (i0 + 4 == gf.nx && gf.ft[1] == ECMG_DIRICHLET);
    if (!d0) {
        *(double2 *)(x + id) = make_double2(out[0], out[1]);
    } else {
        x[id + 1] = out[1];
    }
    *(double2 *)(x + id + 2) = make_double2(out[2], out[3]);
    if (na == 5 && !d4) x[id + 4] = out[4];
}

__global__ void __launch_bounds__(256) k_exp_finite_interp(const Geom gf, const double *__restrict__ V,
                                                           double *__restrict__ x, double *__restrict__ W) {
    exp_finite_interp_block(gf, V, x, W, blockIdx.x, blockIdx.y, blockIdx.z);
}

// U~ = U1 + (1/3) T[U1 - U0]: eq. t1 at coarse nodes ((4 U1 - U0)/3), eq.
// chenlin at edge midpoints (U1 + (d_a + d_b)/6), and the mean of chenlin along
// the 2 face diagonals (U1 + sum(4 d)/12) or the 4 space diagonals (U1 +
// sum(8 d)/24) at face and body centres.  A thread takes a pair of fine nodes
// (2p, 2p+1) of one row; the coarse differences d = U1 - U0 at the even x
// positions of the 1, 2 or 4 contributing rows (row parities are uniform over
// the wave) are loaded once per lane, and the odd node takes the difference at
// 2p+2 from the next lane.  A wave covers 63 pairs: its last lane only supplies
// that neighbour value.
__device__ __forceinline__ void exp_true_block(const Geom &gf, const double *__restrict__ U1,
                                               const double *__restrict__ U0, double *__restrict__ Ut, int bx,
                                               int by, int bz) {
    const int lane = threadIdx.x;                         // one wave per row (blockDim.x == 64)
    const int npair = gf.nx / 2 + 1;                      // pair p: nodes 2p and 2p + 1 <= nx
    const int p = bx * 63 + lane;
    const int j = by * 4 + threadIdx.y, k = bz;
    if (j > gf.ny || k > gf.nz) return;                   // whole rows only: the shuffles below stay wave-wide
    const int pc = min(p, npair - 1);                     // clamped for the loads
    const int i0 = 2 * pc;
    const int64_t sx = gf.sx, sxy = (int64_t)gf.sx * gf.sy;
    const int64_t cx = row_pitch(gf.nx / 2 + 1), cxy = cx * (gf.ny / 2 + 1);
    const int64_t id = i0 + sx * j + sxy * k;
    const bool has_odd = i0 + 1 <= gf.nx;
    double u_e, u_o = 0.0;
    if (has_odd) {
        const double2 v = *(const double2 *)(U1 + id);    // i0 even, rows 16-byte aligned
        u_e = v.x;
        u_o = v.y;
    } else {
        u_e = U1[id];
    }
    const int oj = j & 1, ok = k & 1;
    double se = 0.0, so = 0.0, c_own = 0.0;
    for (int dk = 0; dk <= ok; ++dk) {
        const int kk = k - ok + 2 * dk;
        for (int dj = 0; dj <= oj; ++dj) {
            const int jj = j - oj + 2 * dj;
            const double c0 = U0[pc + cx * (jj >> 1) + cxy * (kk >> 1)];
            const double d0 = U1[i0 + sx * jj + sxy * kk] - c0;
            const double d2 = __shfl_down(d0, 1, 64);     // the difference at 2p + 2
            c_own = c0;
            se += d0;
            so += d0 + d2;
        }
    }
    if (lane == 63 || p >= npair) return;
    const int ne = oj + ok;
    double ve;
    if (ne == 0) ve = (4.0 * u_e - c_own) / 3.0;
    else ve = u_e + se / (ne == 1 ? 6.0 : 12.0);
    if (has_odd) {
        const double vo = u_o + so / (ne == 0 ? 6.0 : (ne == 1 ? 12.0 : 24.0));
        *(double2 *)(Ut + id) = make_double2(ve, vo);
    } else {
        Ut[id] = ve;
    }
}

__global__ void __launch_bounds__(256) k_exp_true(const Geom gf, const double *__restrict__ U1,
                                                  const double *__restrict__ U0, double *__restrict__ Ut) {
    exp_true_block(gf, U1, U0, Ut, blockIdx.x, blockIdx.y, blockIdx.z);
}

// ---------------------------------------------------------------------------
// batched forms: one launch covers the grids of many boxes; box t owns the
// flat blocks [b0, b0 + gx * gy) of the launch (tasks in order of b0)
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_box(const ExpTask *__restrict__ t, int n, int64_t b, int phase) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (t[mid].b0[phase] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(256) k_exp_finite_nodal_batch(const ExpTask *__restrict__ tasks, int n) {
    const int64_t b = blockIdx.x;
    const ExpTask &t = tasks[find_box(tasks, n, b, 0)];
    const int64_t lb = b - t.b0[0];
    const int64_t pl = lb / t.gx[0];
    exp_finite_nodal_block(t.g1, t.U1, t.U0, t.V, t.variant, (int)(lb - pl * t.gx[0]), (int)(pl % t.gy[0]), (int)(pl / t.gy[0]));
}

__global__ void __launch_bounds__(256) k_exp_finite_interp_batch(const ExpTask *__restrict__ tasks, int n) {
    const int64_t b = blockIdx.x;
    const ExpTask &t = tasks[find_box(tasks, n, b, 1)];
    const int64_t lb = b - t.b0[1];
    const int64_t pl = lb / t.gx[1];
    exp_finite_interp_block(t.gf, t.V, t.x, t.W, (int)(lb - pl * t.gx[1]), (int)(pl % t.gy[1]), (int)(pl / t.gy[1]));
}

__global__ void __launch_bounds__(256) k_exp_true_batch(const ExpTask *__restrict__ tasks, int n) {
    const int64_t b = blockIdx.x;
    const ExpTask &t = tasks[find_box(tasks, n, b, 1)];
    const int64_t lb = b - t.b0[1];
    const int64_t pl = lb / t.gx[1];
    exp_true_block(t.gf, t.U1, t.U0, t.x, (int)(lb - pl * t.gx[1]), (int)(pl % t.gy[1]), (int)(pl / t.gy[1]));
}

// Block counts of a box: phase 0 over the level l-1 grid g1, phase 1 over the
// fine grid gf (64 x 4 nodes per block).
int exp_interp_gx(const Geom &gf) { return (gf.nx / 4 + 63) / 64; }
int exp_true_gx(const Geom &gf) { return (gf.nx / 2 + 1 + 62) / 63; }

void exp_task_blocks(ExpTask &t, int kind) {
    t.gx[0] = (t.g1.nx + 1 + 63) / 64;
    t.gx[1] = kind == 0 ? exp_interp_gx(t.gf) : exp_true_gx(t.gf);
    t.gy[0] = (t.g1.ny + 1 + 3) / 4;
    t.gy[1] = (t.gf.ny + 1 + 3) / 4;
    t.nb[0] = (int64_t)t.gx[0] * t.gy[0] * (t.g1.nz + 1);
    t.nb[1] = (int64_t)t.gx[1] * t.gy[1] * (t.gf.nz + 1);
}

void launch_exp_finite_batch(const ExpTask *d_tasks, int n, int64_t nb0, int64_t nb1, hipStream_t s) {
    if (nb0 > 0) hipLaunchKernelGGL(k_exp_finite_nodal_batch, dim3((unsigned)nb0), dim3(64, 4), 0, s, d_tasks, n);
    if (nb1 > 0) hipLaunchKernelGGL(k_exp_finite_interp_batch, dim3((unsigned)nb1), dim3(64, 4), 0, s, d_tasks, n);
}

void launch_exp_true_batch(const ExpTask *d_tasks, int n, int64_t nb1, hipStream_t s) {
    if (nb1 > 0) hipLaunchKernelGGL(k_exp_true_batch, dim3((unsigned)nb1), dim3(64, 4), 0, s, d_tasks, n);
}

void launch_exp_finite(const Geom &gf, const Geom &g1, const double *U1, const double *U0, double *V, double *x,
                       double *W, int variant, hipStream_t s) {
    const dim3 blk(64, 4);
    const dim3 g1grid((g1.nx + 1 + 63) / 64, (g1.ny + 1 + 3) / 4, g1.nz + 1);
    hipLaunchKernelGGL(k_exp_finite_nodal, g1grid, blk, 0, s, g1, U1, U0, V, variant);
    const dim3 gfgrid(exp_interp_gx(gf), (gf.ny + 1 + 3) / 4, gf.nz + 1);
    hipLaunchKernelGGL(k_exp_finite_interp, gfgrid, blk, 0, s, gf, V, x, W);
}

// Zero the row padding (i > nx) of up to four node arrays of a level; the JCG
// scratch arrays are shared by all levels, so padding left over from another
// level's layout is cleared before a level's streaming passes read it.
__global__ void k_zero_pad(const Geom g, double *a, double *b, double *c, double *d) {
    const int pad = g.sx - g.nx - 1;
    const int64_t rows = (int64_t)g.sy * (g.nz + 1);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pad <= 0 || t >= rows * pad) return;
    const int64_t id = (t / pad) * g.sx + g.nx + 1 + (t % pad);
    if (a) a[id] = 0.0;
    if (b) b[id] = 0.0;
    if (c) c[id] = 0.0;
    if (d) d[id] = 0.0;
}

void launch_zero_pad(const Geom &g, double *a, double *b, double *c, double *d, hipStream_t s) {
    const int64_t n = (int64_t)g.sy * (g.nz + 1) * (g.sx - g.nx - 1);
    if (n <= 0) return;
    hipLaunchKernelGGL(k_zero_pad, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, a, b, c, d);
}

__global__ void k_zero_pad_f32(const Geom g, float *a, float *b, float *c) {
    const int pad = g.sx - g.nx - 1;
    const int64_t rows = (int64_t)g.sy * (g.nz + 1);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (pad <= 0 || t >= rows * pad) return;
    const int64_t id = (t / pad) * g.sx + g.nx + 1 + (t % pad);
    if (a) a[id] = 0.0f;
    if (b) b[id] = 0.0f;
    if (c) c[id] = 0.0f;
}

void launch_zero_pad_f32(const Geom &g, float *a, float *b, float *c, hipStream_t s) {
    const int64_t n = (int64_t)g.sy * (g.nz + 1) * (g.sx - g.nx - 1);
    if (n <= 0) return;
    hipLaunchKernelGGL(k_zero_pad_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, a, b, c);
}

void launch_exp_true(const Geom &gf, const double *U1, const double *U0, double *Ut, hipStream_t s) {
    const dim3 grid(exp_true_gx(gf), (gf.ny + 1 + 3) / 4, gf.nz + 1);
    hipLaunchKernelGGL(k_exp_true, grid, dim3(64, 4), 0, s, gf, U1, U0, Ut);
}

}  // namespace ecmg
