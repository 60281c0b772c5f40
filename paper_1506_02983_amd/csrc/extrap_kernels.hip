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
// Each of the 27 nodal values of a coarse element depends only on that
// element's own 27 level l-1 values and 8 level l-2 corner values (its edge,
// face or the element itself), so one thread per coarse element loads those 35
// values, forms the 27 nodal values in registers and writes the element's 4x4x4
// fine nodes (one more layer on the grid's upper faces).  A nodal value on a
// face or edge shared with a neighbouring element is computed by both from the
// same inputs with the same expression, so it is single-valued.
#include "ecmg_internal.h"
#include "exp_finite.h"

#include <algorithm>

namespace ecmg {

template <bool WIDE>
__global__ void __launch_bounds__(256) k_exp_finite(const Geom gf, const Geom g1, const double *__restrict__ U1,
                                                    const double *__restrict__ U0, double *__restrict__ x,
                                                    double *__restrict__ W, int variant) {
    __shared__ double stage[WIDE ? 4 : 1][WIDE ? 256 : 1];
    exp_finite_elem<WIDE>(gf, g1, U1, U0, x, W, variant, (int64_t)blockIdx.x * 256 + threadIdx.x,
                          stage[WIDE ? threadIdx.x / 64 : 0]);
}

// U~ = U1 + (1/3) T[U1 - U0]: eq. t1 at coarse nodes ((4 U1 - U0)/3), eq.
// chenlin at edge midpoints (U1 + (d_a + d_b)/6), and the mean of chenlin along
// the 2 face diagonals (U1 + sum(4 d)/12) or the 4 space diagonals (U1 +
// sum(8 d)/24) at face and body centres, d = U1 - U0 at the coarse nodes.
// A thread takes node pair p (fine x = 2p, 2p+1) of row pair J (fine y = 2J,
// 2J+1) and marches up tkz coarse planes K (fine z = 2K, 2K+1): the 4 coarse
// differences on the upper plane 2K+2 are carried to the next step as its
// lower plane, so every input is read about once.  The last pair / row pair /
// plane of the grid has only its even node.  tkz (at most 16) leaves about
// 2048 blocks per launch: small grids do not march, large ones amortise the
// re-read chunk boundary.

// The fine solution read by EXP_true: U1 itself, or (FUSE) U1 + alpha p, the
// last x update of the JCG solve that produced U1 when it is still pending
// (the finest level of a solve with EXP_true applies it here instead of
// storing it: x is read once either way, and p is read instead of x being
// written back and read again).
struct FineRead {
    const double *__restrict__ U1;
    const double *__restrict__ P;     // FUSE: the search direction of the last iteration
    double al;                        // its step length, 0 if no update is pending
    template <bool FUSE>
    __device__ __forceinline__ double at(int64_t i) const {
        return FUSE ? fma(al, P[i], U1[i]) : U1[i];
    }
    template <bool FUSE>
    __device__ __forceinline__ double2 at2(int64_t i) const {
        double2 v = *(const double2 *)(U1 + i);
        if (FUSE) {
            const double2 q = *(const double2 *)(P + i);
            v.x = fma(al, q.x, v.x);
            v.y = fma(al, q.y, v.y);
        }
        return v;
    }
};

template <bool FUSE = false>
__device__ __forceinline__ void exp_true_block(const Geom &gf, const FineRead &U, const double *__restrict__ U0,
                                               double *__restrict__ Ut, int tkz, int bx, int by, int bz) {
    const int NX1 = gf.nx / 2, NY1 = gf.ny / 2, NZ1 = gf.nz / 2;   // coarse elements per axis
    const int p = bx * 64 + threadIdx.x, J = by * 4 + threadIdx.y;
    if (p > NX1 || J > NY1) return;
    const int K0 = bz * tkz, K1 = min(K0 + tkz, NZ1 + 1);
    const int64_t sx = gf.sx, sxy = (int64_t)gf.sx * gf.sy;
    const int64_t cx = row_pitch(NX1 + 1), cxy = cx * (NY1 + 1);
    const bool hx = p < NX1, hy = J < NY1;                        // odd x node / odd row exist
    const int p2 = min(p + 1, NX1), J2 = min(J + 1, NY1);          // clamped: used only where they exist
    // On coarse plane kc: the fine pair (2p, 2p + 1) of row 2J (kept: it is
    // also the first output row of the step on plane kc), the coarse
    // differences d at x = 2p (dx 0) and 2p + 2 (dx 1) of rows 2J (dj 0) and
    // 2J + 2 (dj 1), and U0 at (p, J, kc).  Row 2J + 2 is the lead row of the
    // thread of row J + 1 on the same plane, so its lines are read by both at
    // about the same time.
    auto lead = [&](int kc, double2 &e0, double (&d)[2][2], double &c00) {
        const int64_t f = sxy * (2 * (int64_t)kc), c = cxy * (int64_t)kc;
        const int64_t fr0 = f + sx * (2 * (int64_t)J), cr0 = c + cx * J;
        if (hx) {
            e0 = U.at2<FUSE>(fr0 + 2 * p);                // 2p even, rows 16-byte aligned
        } else {
            e0.x = U.at<FUSE>(fr0 + 2 * p);
            e0.y = 0.0;
        }
        c00 = U0[cr0 + p];
        d[0][0] = e0.x - c00;
        d[0][1] = U.at<FUSE>(fr0 + 2 * p2) - U0[cr0 + p2];
        const int64_t fr1 = f + sx * (2 * (int64_t)J2), cr1 = c + cx * J2;
        d[1][0] = U.at<FUSE>(fr1 + 2 * p) - U0[cr1 + p];
        d[1][1] = U.at<FUSE>(fr1 + 2 * p2) - U0[cr1 + p2];
    };
    double dlo[2][2], dhi[2][2], clo, chi;
    double2 elo, ehi;
    lead(K0, elo, dlo, clo);
    for (int K = K0; K < K1; ++K) {
        const bool hz = K < NZ1;
        if (hz) lead(K + 1, ehi, dhi, chi);
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            if (c == 1 && !hz) break;
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                if (b == 1 && !hy) break;
                const int64_t id = 2 * p + sx * (2 * (int64_t)J + b) + sxy * (2 * (int64_t)K + c);
                double u_e, u_o = 0.0;
                if (b == 0 && c == 0) {
                    u_e = elo.x;
                    u_o = elo.y;
                } else if (hx) {
                    const double2 v = U.at2<FUSE>(id);
                    u_e = v.x;
                    u_o = v.y;
                } else {
                    u_e = U.at<FUSE>(id);
                }
                // sums over the contributing coarse rows (planes outer, rows inner)
                double se = 0.0, so = 0.0;
#pragma unroll
                for (int dk = 0; dk <= c; ++dk)
#pragma unroll
                    for (int dj = 0; dj <= b; ++dj) {
                        const double d0 = dk ? dhi[dj][0] : dlo[dj][0];
                        const double d2 = dk ? dhi[dj][1] : dlo[dj][1];
                        se += d0;
                        so += d0 + d2;
                    }
                const int ne = b + c;
                double ve;
                if (ne == 0) ve = (4.0 * u_e - clo) / 3.0;
                else ve = u_e + se / (ne == 1 ? 6.0 : 12.0);
                if (hx) {
                    const double vo = u_o + so / (ne == 0 ? 6.0 : (ne == 1 ? 12.0 : 24.0));
                    nt_store2(make_double2(ve, vo), (double2 *)(Ut + id));   // streamed: read by nothing here
                } else {
                    Ut[id] = ve;
                }
            }
        }
        if (hz) {
#pragma unroll
            for (int dj = 0; dj < 2; ++dj) {
                dlo[dj][0] = dhi[dj][0];
                dlo[dj][1] = dhi[dj][1];
            }
            clo = chi;
            elo = ehi;
        }
    }
}

__global__ void __launch_bounds__(256) k_exp_true(const Geom gf, const double *__restrict__ U1,
                                                  const double *__restrict__ U0, double *__restrict__ Ut, int tkz) {
    const FineRead U{U1, nullptr, 0.0};
    exp_true_block<false>(gf, U, U0, Ut, tkz, blockIdx.x, blockIdx.y, blockIdx.z);
}

// EXP_true from x + alpha p (the JCG scalars say whether an update is pending
// and which of the two search-direction buffers holds p)
__global__ void __launch_bounds__(256) k_exp_true_fused(const Geom gf, const double *__restrict__ X,
                                                        const double *__restrict__ U0, double *__restrict__ Ut,
                                                        int tkz, const JcgScalars *__restrict__ sc,
                                                        const double *__restrict__ p0, const double *__restrict__ p1) {
    const FineRead U{X, (sc->iter & 1) ? p1 : p0, sc->pending ? sc->alpha : 0.0};
    exp_true_block<true>(gf, U, U0, Ut, tkz, blockIdx.x, blockIdx.y, blockIdx.z);
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

__global__ void __launch_bounds__(256) k_exp_finite_batch(const ExpTask *__restrict__ tasks, int n) {
    const int64_t b = blockIdx.x;
    const ExpTask &t = tasks[find_box(tasks, n, b, 0)];
    exp_finite_elem<false>(t.gf, t.g1, t.U1, t.U0, t.x, t.W, t.variant, (b - t.b0[0]) * 256 + threadIdx.x, nullptr);
}

__global__ void __launch_bounds__(256) k_exp_true_batch(const ExpTask *__restrict__ tasks, int n) {
    const int64_t b = blockIdx.x;
    const ExpTask &t = tasks[find_box(tasks, n, b, 1)];
    const int64_t lb = b - t.b0[1];
    const int64_t pl = lb / t.gx[1];
    const FineRead U{t.U1, nullptr, 0.0};
    exp_true_block<false>(t.gf, U, t.U0, t.x, t.tkz, (int)(lb - pl * t.gx[1]), (int)(pl % t.gy[1]),
                          (int)(pl / t.gy[1]));
}

// Block counts of a box: EXP_finite one thread per coarse element (256 per
// block, [0]); EXP_true 64 node pairs x 4 row pairs x tkz coarse planes per
// block ([1]).
int exp_true_gx(const Geom &gf) { return (gf.nx / 2 + 1 + 63) / 64; }
int exp_true_gy(const Geom &gf) { return (gf.ny / 2 + 1 + 3) / 4; }
int exp_true_tkz(const Geom &gf) {
    const int64_t t = (int64_t)exp_true_gx(gf) * exp_true_gy(gf) * (gf.nz / 2 + 1) / 2048;
    return (int)std::max<int64_t>(1, std::min<int64_t>(16, t));
}
int exp_true_gz(const Geom &gf, int tkz) { return (gf.nz / 2 + 1 + tkz - 1) / tkz; }

void exp_task_blocks(ExpTask &t, int kind) {
    t.gx[0] = t.gy[0] = 0;
    t.nb[0] = 0;
    t.gx[1] = t.gy[1] = 0;
    t.nb[1] = 0;
    if (kind == 0) {
        t.nb[0] = ((int64_t)(t.gf.nx / 4) * (t.gf.ny / 4) * (t.gf.nz / 4) + 255) / 256;
    } else {
        t.gx[1] = exp_true_gx(t.gf);
        t.gy[1] = exp_true_gy(t.gf);
        t.tkz = exp_true_tkz(t.gf);
        t.nb[1] = (int64_t)t.gx[1] * t.gy[1] * exp_true_gz(t.gf, t.tkz);
    }
}

void launch_exp_finite_batch(const ExpTask *d_tasks, int n, int64_t nb, hipStream_t s) {
    if (nb > 0) hipLaunchKernelGGL(k_exp_finite_batch, dim3((unsigned)nb), dim3(256), 0, s, d_tasks, n);
}

void launch_exp_true_batch(const ExpTask *d_tasks, int n, int64_t nb1, hipStream_t s) {
    if (nb1 > 0) hipLaunchKernelGGL(k_exp_true_batch, dim3((unsigned)nb1), dim3(64, 4), 0, s, d_tasks, n);
}

void launch_exp_finite(const Geom &gf, const Geom &g1, const double *U1, const double *U0, double *x, double *W,
                       int variant, hipStream_t s) {
    const int64_t ne = (int64_t)(gf.nx / 4) * (gf.ny / 4) * (gf.nz / 4);
    if (ne <= 0) return;
    // whole waves on one element row when NX is a multiple of 64 (then every
    // 64-thread wave holds 64 consecutive elements of one row)
    if ((gf.nx / 4) % 64 == 0)
        launch_timed(k_exp_finite<true>, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, gf, g1, U1, U0, x, W,
                     variant);
    else
        launch_timed(k_exp_finite<false>, dim3((unsigned)((ne + 255) / 256)), dim3(256), 0, s, gf, g1, U1, U0, x, W,
                     variant);
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

void launch_exp_true(const Geom &gf, const double *U1, const double *U0, double *Ut, hipStream_t s,
                     const JcgScalars *sc, const double *p0, const double *p1) {
    const int tkz = exp_true_tkz(gf);
    const dim3 grid(exp_true_gx(gf), exp_true_gy(gf), exp_true_gz(gf, tkz));
    if (sc) launch_timed(k_exp_true_fused, grid, dim3(64, 4), 0, s, gf, U1, U0, Ut, tkz, sc, p0, p1);
    else launch_timed(k_exp_true, grid, dim3(64, 4), 0, s, gf, U1, U0, Ut, tkz);
}

}  // namespace ecmg
