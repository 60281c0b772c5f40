// EXP_finite of one coarse element (Sections 4.2.2-4.3), shared by the
// inter-level kernels (extrap_kernels.hip) and the queue kernel of the batched
// cascade (persistent_kernels.hip), which runs it inside each box's level task.
// The formulas and the element decomposition are described in
// extrap_kernels.hip.
#pragma once
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

// EXP_finite of coarse (level l-2) element e = I + NX (J + NY K) of the fine
// grid gf (NX = nx/4 ...): local level l-1 nodes (a,b,c) in {0,1,2}^3 are the
// global ones (2I+a, 2J+b, 2K+c); level l-2 corners (a/2, b/2, c/2).  Fine rows
// are written with 16-byte stores (4I is a multiple of 4 and rows are 16-byte
// aligned); lanes take consecutive I, so a wave writes contiguous row segments.
// WIDE: every wave holds 64 consecutive elements of one element row (the
// caller guarantees NX % 64 == 0, 64-thread-aligned waves): each fine row's
// 256 values go through the wave's LDS buffer `stage` (256 doubles), so that
// every store instruction writes 1 KB contiguous instead of 16 bytes per
// 32-byte chunk.
template <bool WIDE>
__device__ __forceinline__ void exp_finite_elem(const Geom &gf, const Geom &g1, const double *__restrict__ U1,
                                                const double *__restrict__ U0, double *__restrict__ x,
                                                double *__restrict__ W, int variant, int64_t e,
                                                double *__restrict__ stage) {
    const int NX = gf.nx / 4, NY = gf.ny / 4, NZ = gf.nz / 4;
    if (e >= (int64_t)NX * NY * NZ) return;
    const int I = (int)(e % NX);
    const int64_t ejk = e / NX;
    const int J = (int)(ejk % NY), K = (int)(ejk / NY);
    const int64_t s1 = g1.sx, s1y = (int64_t)g1.sx * g1.sy;
    const int64_t s0 = row_pitch(g1.nx / 2 + 1), s0y = s0 * (g1.ny / 2 + 1);

    // the element's level l-1 values u[c][b][a] and level l-2 corners u0[c][b][a]
    double u[3][3][3], u0[2][2][2];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const double *row = U1 + 2 * I + s1 * (2 * J + b) + s1y * (2 * K + c);
            const double2 v01 = *(const double2 *)row;   // 2I is even: 16-byte aligned
            u[c][b][0] = v01.x;
            u[c][b][1] = v01.y;
            u[c][b][2] = row[2];
        }
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) u0[c][b][a] = U0[(I + a) + s0 * (J + b) + s0y * (K + c)];

    // nodal values N[c][b][a]
    double N[3][3][3];
    auto del = [&](int a, int b, int c) { return u[c][b][a] - u0[c >> 1][b >> 1][a >> 1]; };
#pragma unroll
    for (int c = 0; c < 3; c += 2)                     // corners: eq. jiedian
#pragma unroll
        for (int b = 0; b < 3; b += 2)
#pragma unroll
            for (int a = 0; a < 3; a += 2) N[c][b][a] = (5.0 * u[c][b][a] - u0[c >> 1][b >> 1][a >> 1]) / 4.0;
    // mid-edges along axis ax: eq. zhongdian
    auto Wm = [&](int a, int b, int c, int ax) {
        const int da = ax == 0, db = ax == 1, dc = ax == 2;
        return u[c][b][a] + (del(a - da, b - db, c - dc) + del(a + da, b + db, c + dc)) / 8.0;
    };
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if ((a & 1) + (b & 1) + (c & 1) == 1) N[c][b][a] = Wm(a, b, c, (a & 1) ? 0 : ((b & 1) ? 1 : 2));
    // face centres: in-face axes A < B (the two odd ones); offset (sa, sb)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if ((a & 1) + (b & 1) + (c & 1) != 2) continue;
                const int A = (a & 1) ? 0 : 1, B = (c & 1) ? 2 : 1;
                auto at = [&](int sa, int sb, int &pa, int &pb, int &pc) {
                    pa = a + (A == 0 ? sa : 0);
                    pb = b + (A == 1 ? sa : 0) + (B == 1 ? sb : 0);
                    pc = c + (B == 2 ? sb : 0);
                };
                int xa, xb, xc, ya, yb, yc;
                double v;
                if (variant == ECMG_SERENDIPITY20) {
                    // the face's 8-node serendipity interpolant at its centre:
                    // -1/4 (4 corners) + 1/2 (4 mid-edges)
                    double sc = 0.0, sm = 0.0;
#pragma unroll
                    for (int sb = -1; sb <= 1; sb += 2)
#pragma unroll
                        for (int sa = -1; sa <= 1; sa += 2) {
                            at(sa, sb, xa, xb, xc);
                            sc += N[xc][xb][xa];
                        }
#pragma unroll
                    for (int s2 = -1; s2 <= 1; s2 += 2) {
                        at(0, s2, xa, xb, xc);           // edge along A at B offset s2
                        at(s2, 0, ya, yb, yc);           // edge along B at A offset s2
                        sm += N[xc][xb][xa] + N[yc][yb][ya];
                    }
                    v = -0.25 * sc + 0.5 * sm;
                } else {
                    // mean of eq. zhongdian along the two face diagonals
                    const double um = u[c][b][a];
                    int pa, pb, pc, qa, qb, qc;
                    at(-1, -1, xa, xb, xc);
                    at(1, 1, ya, yb, yc);
                    at(-1, 1, pa, pb, pc);
                    at(1, -1, qa, qb, qc);
                    v = ((um + (del(xa, xb, xc) + del(ya, yb, yc)) / 8.0) +
                         (um + (del(pa, pb, pc) + del(qa, qb, qc)) / 8.0)) / 2.0;
                }
                N[c][b][a] = v;
            }
    // element centre
    if (variant == ECMG_SERENDIPITY20) {
        // -1/4 (8 corners) + 1/4 (12 mid-edges)
        double sc = 0.0, sm = 0.0;
#pragma unroll
        for (int c = -1; c <= 1; c += 2)
#pragma unroll
            for (int b = -1; b <= 1; b += 2)
#pragma unroll
                for (int a = -1; a <= 1; a += 2) sc += N[1 + c][1 + b][1 + a];
#pragma unroll
        for (int t = -1; t <= 1; t += 2)
#pragma unroll
            for (int u2 = -1; u2 <= 1; u2 += 2)
                sm += N[1 + u2][1 + t][1] + N[1 + u2][1][1 + t] + N[1][1 + u2][1 + t];
        N[1][1][1] = -0.25 * sc + 0.25 * sm;
    } else {
        // mean of eq. zhongdian along the 4 space diagonals
        const double m = u[1][1][1];
        double sum = 0.0;
#pragma unroll
        for (int b = -1; b <= 1; b += 2)
#pragma unroll
            for (int c = -1; c <= 1; c += 2) sum += m + (del(0, 1 - b, 1 - c) + del(2, 1 + b, 1 + c)) / 8.0;
        N[1][1][1] = sum / 4.0;
    }

    // fine rows (j, k) = (4J + bf, 4K + cf): tensor-product quadratic
    // interpolation, z then y weights folded into 3 x-column sums
    const bool lastx = I == NX - 1, lasty = J == NY - 1, lastz = K == NZ - 1;
    const bool d0 = I == 0 && gf.ft[0] == ECMG_DIRICHLET;
    const bool d4 = lastx && gf.ft[1] == ECMG_DIRICHLET;
    const int64_t sx = gf.sx, sxy = (int64_t)gf.sx * gf.sy;
#pragma unroll
    for (int cf = 0; cf < 5; ++cf) {
        if (cf == 4 && !lastz) break;
        double Lz[3];
        lagrange3(cf, Lz);
        const int k = 4 * K + cf;
#pragma unroll
        for (int bf = 0; bf < 5; ++bf) {
            if (bf == 4 && !lasty) break;
            double Ly[3];
            lagrange3(bf, Ly);
            const int j = 4 * J + bf;
            double w0 = 0.0, w1 = 0.0, w2 = 0.0;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                if (Lz[cc] == 0.0) continue;
                double t0 = 0.0, t1 = 0.0, t2 = 0.0;
#pragma unroll
                for (int bb = 0; bb < 3; ++bb) {
                    if (Ly[bb] == 0.0) continue;
                    t0 += Ly[bb] * N[cc][bb][0];
                    t1 += Ly[bb] * N[cc][bb][1];
                    t2 += Ly[bb] * N[cc][bb][2];
                }
                w0 += Lz[cc] * t0;
                w1 += Lz[cc] * t1;
                w2 += Lz[cc] * t2;
            }
            // x weights at a = 0..4: (1,0,0), (3/8,3/4,-1/8), (0,1,0),
            // (-1/8,3/4,3/8), (0,0,1)
            const double o1 = 0.375 * w0 + 0.75 * w1 - 0.125 * w2;
            const double o3 = -0.125 * w0 + 0.75 * w1 + 0.375 * w2;
            const int64_t id = 4 * I + sx * j + sxy * k;
            const bool drow = (j == 0 && gf.ft[2] == ECMG_DIRICHLET) || (j == gf.ny && gf.ft[3] == ECMG_DIRICHLET) ||
                              (k == 0 && gf.ft[4] == ECMG_DIRICHLET) || (k == gf.nz && gf.ft[5] == ECMG_DIRICHLET);
            if (WIDE) {
                // the wave's 256 fine nodes of this row start at 4 * (I - lane)
                const int lane = (int)(threadIdx.x & 63);
                const int64_t row0 = id - 4 * lane;
                const bool dw = (I - lane) == 0 && gf.ft[0] == ECMG_DIRICHLET;   // node x = 0 keeps g_D
                *(double2 *)(stage + 4 * lane) = make_double2(w0, o1);
                *(double2 *)(stage + 4 * lane + 2) = make_double2(w1, o3);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                const double2 v0 = *(const double2 *)(stage + 2 * lane);
                const double2 v1 = *(const double2 *)(stage + 128 + 2 * lane);
                if (W) {
                    *(double2 *)(W + row0 + 2 * lane) = v0;
                    *(double2 *)(W + row0 + 128 + 2 * lane) = v1;
                    if (lastx) W[id + 4] = w2;
                }
                if (!drow) {
                    if (dw && lane == 0) x[row0 + 1] = v0.y;
                    else *(double2 *)(x + row0 + 2 * lane) = v0;
                    *(double2 *)(x + row0 + 128 + 2 * lane) = v1;
                    if (lastx && !d4) x[id + 4] = w2;
                }
                // the buffer is rewritten by the next row
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                continue;
            }
            if (W) {
                *(double2 *)(W + id) = make_double2(w0, o1);
                *(double2 *)(W + id + 2) = make_double2(w1, o3);
                if (lastx) W[id + 4] = w2;
            }
            if (drow) continue;                               // the whole row is Dirichlet (g_D stays)
            if (!d0) *(double2 *)(x + id) = make_double2(w0, o1);
            else x[id + 1] = o1;
            *(double2 *)(x + id + 2) = make_double2(w1, o3);
            if (lastx && !d4) x[id + 4] = w2;
        }
    }
}

}  // namespace ecmg
