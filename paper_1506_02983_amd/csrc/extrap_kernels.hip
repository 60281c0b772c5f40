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
// costs 39 multiply-adds per node instead of 20 three-dimensional shape
// functions.  A fine node on a face shared by two coarse elements belongs to
// the lower-index element (both give the same value up to rounding).
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

__global__ void __launch_bounds__(256) k_exp_finite(const Geom gf, const double *__restrict__ U1,
                                                    const double *__restrict__ U0, double *__restrict__ x,
                                                    double *__restrict__ W, int variant) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= gf.nnodes) return;
    const int i = (int)(id % gf.sx);
    const int64_t t = id / gf.sx;
    const int j = (int)(t % gf.sy);
    const int k = (int)(t / gf.sy);
    const int NX = gf.nx / 4, NY = gf.ny / 4, NZ = gf.nz / 4;
    const int I = min(i / 4, NX - 1), J = min(j / 4, NY - 1), K = min(k / 4, NZ - 1);
    const int a = i - 4 * I, b = j - 4 * J, c = k - 4 * K;
    const int64_t n1x = gf.nx / 2 + 1, n1y = gf.ny / 2 + 1;
    const int64_t n0x = NX + 1, n0y = NY + 1;

    double u1[3][3][3];
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
#pragma unroll
        for (int bb = 0; bb < 3; ++bb)
#pragma unroll
            for (int aa = 0; aa < 3; ++aa)
                u1[cc][bb][aa] = U1[(2 * I + aa) + n1x * ((2 * J + bb) + n1y * (int64_t)(2 * K + cc))];
    double u0[2][2][2], d[2][2][2];
#pragma unroll
    for (int cc = 0; cc < 2; ++cc)
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int aa = 0; aa < 2; ++aa) {
                u0[cc][bb][aa] = U0[(I + aa) + n0x * ((J + bb) + n0y * (int64_t)(K + cc))];
                d[cc][bb][aa] = u1[2 * cc][2 * bb][2 * aa] - u0[cc][bb][aa];
            }

    double V[3][3][3];
    // corners (eq. jiedian)
#pragma unroll
    for (int cc = 0; cc < 2; ++cc)
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int aa = 0; aa < 2; ++aa)
                V[2 * cc][2 * bb][2 * aa] = (5.0 * u1[2 * cc][2 * bb][2 * aa] - u0[cc][bb][aa]) / 4.0;
    // mid-edges (eq. zhongdian)
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            V[2 * q][2 * p][1] = u1[2 * q][2 * p][1] + (d[q][p][0] + d[q][p][1]) / 8.0;   // along x
            V[2 * q][1][2 * p] = u1[2 * q][1][2 * p] + (d[q][0][p] + d[q][1][p]) / 8.0;   // along y
            V[1][2 * q][2 * p] = u1[1][2 * q][2 * p] + (d[0][q][p] + d[1][q][p]) / 8.0;   // along z
        }
    if (variant == ECMG_SERENDIPITY20) {
        // face centres: -1/4 (4 face corners) + 1/2 (4 face mid-edges)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int e = 2 * s;
            V[1][1][e] = -0.25 * (V[0][0][e] + V[0][2][e] + V[2][0][e] + V[2][2][e]) +
                         0.5 * (V[0][1][e] + V[2][1][e] + V[1][0][e] + V[1][2][e]);
            V[1][e][1] = -0.25 * (V[0][e][0] + V[0][e][2] + V[2][e][0] + V[2][e][2]) +
                         0.5 * (V[0][e][1] + V[2][e][1] + V[1][e][0] + V[1][e][2]);
            V[e][1][1] = -0.25 * (V[e][0][0] + V[e][0][2] + V[e][2][0] + V[e][2][2]) +
                         0.5 * (V[e][0][1] + V[e][2][1] + V[e][1][0] + V[e][1][2]);
        }
        double sc = 0.0, sm = 0.0;
#pragma unroll
        for (int cc = 0; cc < 2; ++cc)
#pragma unroll
            for (int bb = 0; bb < 2; ++bb)
#pragma unroll
                for (int aa = 0; aa < 2; ++aa) sc += V[2 * cc][2 * bb][2 * aa];
#pragma unroll
        for (int p = 0; p < 2; ++p)
#pragma unroll
            for (int q = 0; q < 2; ++q) sm += V[2 * q][2 * p][1] + V[2 * q][1][2 * p] + V[1][2 * q][2 * p];
        V[1][1][1] = -0.25 * sc + 0.25 * sm;
    } else {
        // face centres: mean of eq. zhongdian along the two face diagonals
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int e = 2 * s;
            V[1][1][e] = ((u1[1][1][e] + (d[0][0][s] + d[1][1][s]) / 8.0) +
                          (u1[1][1][e] + (d[0][1][s] + d[1][0][s]) / 8.0)) / 2.0;
            V[1][e][1] = ((u1[1][e][1] + (d[0][s][0] + d[1][s][1]) / 8.0) +
                          (u1[1][e][1] + (d[0][s][1] + d[1][s][0]) / 8.0)) / 2.0;
            V[e][1][1] = ((u1[e][1][1] + (d[s][0][0] + d[s][1][1]) / 8.0) +
                          (u1[e][1][1] + (d[s][0][1] + d[s][1][0]) / 8.0)) / 2.0;
        }
        // body centre: mean along the 4 space diagonals
        const double m = u1[1][1][1];
        V[1][1][1] = ((m + (d[0][0][0] + d[1][1][1]) / 8.0) + (m + (d[0][0][1] + d[1][1][0]) / 8.0) +
                      (m + (d[0][1][0] + d[1][0][1]) / 8.0) + (m + (d[0][1][1] + d[1][0][0]) / 8.0)) / 4.0;
    }

    double w;
    if (!(a & 1) && !(b & 1) && !(c & 1)) {
        w = V[c >> 1][b >> 1][a >> 1];
    } else {
        double Lx[3], Ly[3], Lz[3];
        lagrange3(a, Lx);
        lagrange3(b, Ly);
        lagrange3(c, Lz);
        w = 0.0;
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            double sy = 0.0;
#pragma unroll
            for (int bb = 0; bb < 3; ++bb) {
                const double sxv = Lx[0] * V[cc][bb][0] + Lx[1] * V[cc][bb][1] + Lx[2] * V[cc][bb][2];
                sy += Ly[bb] * sxv;
            }
            w += Lz[cc] * sy;
        }
    }
    if (W) W[id] = w;
    if (!is_dir(gf, i, j, k)) x[id] = w;
}

// U~ = U1 + (1/3) T[U1 - U0]: eq. t1 at coarse nodes ((4 U1 - U0)/3), eq.
// chenlin at edge midpoints (U1 + (d_a + d_b)/6), and the mean of chenlin along
// the 2 face diagonals (U1 + sum(4 d)/12) or the 4 space diagonals (U1 +
// sum(8 d)/24) at face and body centres.
__global__ void __launch_bounds__(256) k_exp_true(const Geom gf, const double *__restrict__ U1,
                                                  const double *__restrict__ U0, double *__restrict__ Ut) {
    const int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= gf.nnodes) return;
    const int i = (int)(id % gf.sx);
    const int64_t t = id / gf.sx;
    const int j = (int)(t % gf.sy);
    const int k = (int)(t / gf.sy);
    const int64_t sx = gf.sx, sxy = (int64_t)gf.sx * gf.sy;
    const int64_t cx = gf.nx / 2 + 1, cxy = cx * (gf.ny / 2 + 1);
    const double u1 = U1[id];
    const int oi = i & 1, oj = j & 1, ok = k & 1;
    if (!(oi | oj | ok)) {
        Ut[id] = (4.0 * u1 - U0[(i >> 1) + cx * (j >> 1) + cxy * (k >> 1)]) / 3.0;
        return;
    }
    double s = 0.0;
#pragma unroll
    for (int dk = 0; dk < 2; ++dk) {
        if (dk && !ok) break;
        const int kk = k - ok + 2 * dk;
#pragma unroll
        for (int dj = 0; dj < 2; ++dj) {
            if (dj && !oj) break;
            const int jj = j - oj + 2 * dj;
#pragma unroll
            for (int di = 0; di < 2; ++di) {
                if (di && !oi) break;
                const int ii = i - oi + 2 * di;
                s += U1[ii + sx * jj + sxy * kk] - U0[(ii >> 1) + cx * (jj >> 1) + cxy * (kk >> 1)];
            }
        }
    }
    const int nodd = oi + oj + ok;
    const double denom = nodd == 1 ? 6.0 : (nodd == 2 ? 12.0 : 24.0);
    Ut[id] = u1 + s / denom;
}

void launch_exp_finite(const Geom &gf, const double *U1, const double *U0, double *x, double *W, int variant,
                       hipStream_t s) {
    const int64_t nb = (gf.nnodes + 255) / 256;
    hipLaunchKernelGGL(k_exp_finite, dim3((unsigned)nb), dim3(256), 0, s, gf, U1, U0, x, W, variant);
}

void launch_exp_true(const Geom &gf, const double *U1, const double *U0, double *Ut, hipStream_t s) {
    const int64_t nb = (gf.nnodes + 255) / 256;
    hipLaunchKernelGGL(k_exp_true, dim3((unsigned)nb), dim3(256), 0, s, gf, U1, U0, Ut);
}

}  // namespace ecmg
