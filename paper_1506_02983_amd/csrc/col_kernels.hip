// Column stencil kernels for the large JCG levels (gfx950): operator apply,
// JCG initialisation and pass A of iteration 0, each a matrix-free 27-point
// apply of the Q1 operator with one beta per element (Section 2), without LDS
// and without block barriers.
//
// One wavefront owns a column of nodes: 64 lanes along x (x = 62 tx - 1 + lane;
// lanes 1..62 produce outputs, lanes 0 and 63 only carry the x-halo), R rows in
// y and a chunk of KZ planes in z that it marches through.  Each lane keeps
// its R + 2 rows (the R output rows and their y-halo) of the planes k-1, k, k+1
// and the elements of the layers k-1, k in registers, in rings of four planes
// and layers so that the loads of plane k+2 (and layer k+1, and the epilogue
// inputs of plane k+1) are in flight while plane k is computed.  The x
// neighbours come from the adjacent lanes through DPP wavefront shifts (a VALU
// operand modifier, no LDS traffic): the exchange through LDS, not HBM, bounded
// the tiled kernels.  Every load is branch-free (clamped index, the value
// zeroed afterwards), so the compiler waits for exactly the loads a step uses.
//
// Reductions: each wave sums its lanes' partials with shuffles and stores one
// pair; the one-block finishing kernels of jcg_kernels.hip (fixed order) take
// the scalar steps, so results are bitwise reproducible.
#include "ecmg_internal.h"

namespace ecmg {

namespace {

// lane i receives lane i-1 (DPP wave_shr:1); lane 0 receives 0
__device__ __forceinline__ double from_left(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)__double2loint(v), 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)__double2hiint(v), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
// lane i receives lane i+1 (DPP wave_shl:1); lane 63 receives 0
__device__ __forceinline__ double from_right(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, (int)__double2loint(v), 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)__double2hiint(v), 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ bool dir_node(const Geom &g, int i, int j, int k) {
    return (i == 0 && g.ft[0] == ECMG_DIRICHLET) || (i == g.nx && g.ft[1] == ECMG_DIRICHLET) ||
           (j == 0 && g.ft[2] == ECMG_DIRICHLET) || (j == g.ny && g.ft[3] == ECMG_DIRICHLET) ||
           (k == 0 && g.ft[4] == ECMG_DIRICHLET) || (k == g.nz && g.ft[5] == ECMG_DIRICHLET);
}

// Robin face-mass term of face F at in-face coordinates (pi, qi) (face element
// counts np, nq): the node is corner (1-dp, 1-dq) of each surrounding face
// element (ep, eq) = (pi-1+dp, qi-1+dq), coupled to that element's 4 corners
// with hp*hq*(1/9, 1/18, 1/36) by the number of differing in-face axes; nb(op,
// oq) is the input value at in-face offset (op, oq).
template <typename NB>
__device__ __forceinline__ double robin_col(const Geom &g, int face, const double *__restrict__ al, int pi, int qi,
                                            int np, int nq, NB nb) {
    double s = 0.0;
#pragma unroll
    for (int dq = 0; dq < 2; ++dq) {
        const int eq = qi - 1 + dq;
        if (eq < 0 || eq >= nq) continue;
#pragma unroll
        for (int dp = 0; dp < 2; ++dp) {
            const int ep = pi - 1 + dp;
            if (ep < 0 || ep >= np) continue;
            const double a = al[ep + (int64_t)np * eq];
            double t = 0.0;
#pragma unroll
            for (int bq = 0; bq < 2; ++bq)
#pragma unroll
                for (int bp = 0; bp < 2; ++bp) {
                    const int c = (bp != 1 - dp) + (bq != 1 - dq);
                    t += g.M[face][c] * nb(dp - 1 + bp, dq - 1 + bq);
                }
            s += a * t;
        }
    }
    return s;
}

// register rings of one wave lane
template <int R>
struct ColRegs {
    double P[4][R + 2];    // input planes: rows j0-1 .. j0+R
    double B[4][R + 1];    // element layers: element rows j0-1 .. j0+R-1, element x = i
    double E[2][1][R];     // epilogue input of the output rows (INIT: F)
};

// One z-step: output plane k from the planes Pm (k-1), P0 (k), Pp (k+1) and the
// layers Bl (k-1), Bu (k); first issues the loads of plane k+2 into Pn, layer
// k+1 into Bn and the epilogue inputs of plane k+1 into En.
template <int MODE, int R>
__device__ __forceinline__ void col_step(const ColArgs &a, int i, int j0, int k, int k1, bool out_lane, bool iok,
                                         bool ieok, bool dir_i, bool rob_i, double (&Pm)[R + 2], double (&P0)[R + 2],
                                         double (&Pp)[R + 2],
                                         double (&Pn)[R + 2], double (&Bl)[R + 1], double (&Bu)[R + 1],
                                         double (&Bn)[R + 1], double (&Ec)[1][R], double (&En)[1][R], double &acc0,
                                         double &acc1) {
    const Geom &g = a.g;
    const int sx = g.sx, sxy = g.sx * g.sy, exy = g.nx * g.ny;
    const int ic = min(max(i, 0), g.nx), ie = min(max(i, 0), g.nx - 1);
    const bool dir_k = (k == 0 && g.ft[4] == ECMG_DIRICHLET) || (k == g.nz && g.ft[5] == ECMG_DIRICHLET);
    const bool rob_k = (k == 0 && g.ft[4] == ECMG_ROBIN) || (k == g.nz && g.ft[5] == ECMG_ROBIN);
    {   // prefetch: plane k+2 (inside the chunk and its upper halo plane), layer k+1, epilogue of plane k+1
        const int kp = k + 2, kb = k + 1, ke = k + 1;
#pragma unroll
        for (int r = 0; r < R + 2; ++r) {
            const int jj = j0 - 1 + r;
            const bool ok = iok && jj >= 0 && jj <= g.ny && kp <= g.nz && kp <= k1;
            const double v = a.v[ic + sx * min(max(jj, 0), g.ny) + sxy * min(kp, g.nz)];
            Pn[r] = ok ? v : 0.0;
        }
#pragma unroll
        for (int r = 0; r < R + 1; ++r) {
            const int jj = j0 - 1 + r;
            const bool ok = ieok && jj >= 0 && jj < g.ny && kb < g.nz && kb < k1;
            const double v = a.beta[ie + g.nx * min(max(jj, 0), g.ny - 1) + exy * min(kb, g.nz - 1)];
            Bn[r] = ok ? v : 0.0;
        }
        if (MODE == MODE_INIT) {
#pragma unroll
            for (int r = 0; r < R; ++r) En[0][r] = __builtin_nontemporal_load(a.F + ic + sx * min(j0 + r, g.ny) +
                                                                              sxy * min(ke, g.nz));
        }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = j0 + r;
        // beta of the 8 elements around the node: layer below (k-1, Bl) and
        // above (k, Bu); in-plane [dy][dx] = element (i-1+dx, j-1+dy)
        const double l01 = Bl[r], l11 = Bl[r + 1], u01 = Bu[r], u11 = Bu[r + 1];
        const double l00 = from_left(l01), l10 = from_left(l11), u00 = from_left(u01), u10 = from_left(u11);
        double q = 0.0;
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy) {
            const int rr = r + 1 + oy;
#pragma unroll
            for (int ox = -1; ox <= 1; ++ox) {
                double sl, su;
                if (oy < 0 && ox < 0) { sl = l00; su = u00; }
                else if (oy < 0 && ox > 0) { sl = l01; su = u01; }
                else if (oy > 0 && ox < 0) { sl = l10; su = u10; }
                else if (oy > 0 && ox > 0) { sl = l11; su = u11; }
                else if (oy < 0) { sl = l00 + l01; su = u00 + u01; }
                else if (oy > 0) { sl = l10 + l11; su = u10 + u11; }
                else if (ox < 0) { sl = l00 + l10; su = u00 + u10; }
                else if (ox > 0) { sl = l01 + l11; su = u01 + u11; }
                else { sl = (l00 + l01) + (l10 + l11); su = (u00 + u01) + (u10 + u11); }
                const int m = (ox != 0) | ((oy != 0) << 1);
                double vm = Pm[rr], v0 = P0[rr], vp = Pp[rr];
                if (ox < 0) { vm = from_left(vm); v0 = from_left(v0); vp = from_left(vp); }
                if (ox > 0) { vm = from_right(vm); v0 = from_right(v0); vp = from_right(vp); }
                // neighbours in planes k-1 / k+1 share only the layer between;
                // neighbours in plane k are shared by both layers
                q += g.C[m | 4] * (sl * vm + su * vp) + g.C[m] * ((sl + su) * v0);
            }
        }
        // nodes on a Robin face (and on no Dirichlet face) are the face kernel's
        const bool dir = dir_i || (j == 0 && g.ft[2] == ECMG_DIRICHLET) || (j == g.ny && g.ft[3] == ECMG_DIRICHLET) ||
                         dir_k;
        const bool rob = rob_i || (j == 0 && g.ft[2] == ECMG_ROBIN) || (j == g.ny && g.ft[3] == ECMG_ROBIN) || rob_k;
        if (!out_lane || j > g.ny || (rob && !dir)) continue;
        const int id = i + sx * j + sxy * k;
        if (MODE == MODE_APPLY) {
            __builtin_nontemporal_store(dir ? 0.0 : q, a.out + id);
        } else if (MODE == MODE_INIT) {
            const double rv = dir ? 0.0 : Ec[0][r] - q;
            __builtin_nontemporal_store(rv, a.out + id);
            // M^-1 from the beta already in registers: the diagonal C[0] * (sum of
            // the 8 element betas, in the order the setup's 1/D uses), so z is
            // what the stored 1/D gives, bit for bit (no Robin term here)
            double z;
            if (a.plain_cg) {
                z = rv;
            } else {
                const double s8 = ((((((l00 + l01) + l10) + l11) + u00) + u01) + u10) + u11;
                z = (1.0 / (g.C[0] * s8)) * rv;
            }
            if (a.p_init) __builtin_nontemporal_store(z, a.p_out + id);     // p_0 for iteration 0
            acc0 += rv * z;
            acc1 += rv * rv;
        } else {                                  // MODE_PASSA0: q = A p_0, p_0 . q
            const double qv = dir ? 0.0 : q;
            __builtin_nontemporal_store(qv, a.out + id);
            acc0 += P0[r + 1] * qv;
        }
    }
}

// WPE: waves per SIMD the register budget is set for (iteration 0 and apply:
// 3, with a few bytes of spills, measured faster than 2 without; init keeps 2,
// where 3 would spill 128 bytes per lane)
template <int MODE, int R, int WPE>
__global__ void __launch_bounds__(256, WPE) k_col(const ColArgs a) {
    const Geom &g = a.g;
    if (MODE == MODE_PASSA0 && a.sc->done) return;      // uniform over the grid
    const int lane = threadIdx.x & 63;
    // consecutive waves take consecutive x-segments of the same rows (blocks go
    // round-robin over the XCDs; a contiguous range per XCD was measured slower)
    const int wid = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int total = a.ntx * a.nty * a.nkz;
    double acc0 = 0.0, acc1 = 0.0;
    if (wid < total) {
        const int tx = wid % a.ntx, t2 = wid / a.ntx, ty = t2 % a.nty, tz = t2 / a.nty;
        const int i = 62 * tx - 1 + lane;
        const int j0 = ty * R;
        const int k0 = tz * a.KZ, k1 = min(k0 + a.KZ, g.nz + 1);
        const bool iok = i >= 0 && i <= g.nx, ieok = i >= 0 && i < g.nx;
        const bool out_lane = lane >= 1 && lane <= 62 && iok;
        const int sx = g.sx, sxy = g.sx * g.sy, exy = g.nx * g.ny;
        const int ic = min(max(i, 0), g.nx), ie = min(max(i, 0), g.nx - 1);
        ColRegs<R> S;
        // prologue: planes k0-1, k0, k0+1, layers k0-1, k0, epilogue of plane k0
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int kk = k0 - 1 + c;
#pragma unroll
            for (int r = 0; r < R + 2; ++r) {
                const int jj = j0 - 1 + r;
                const bool ok = iok && jj >= 0 && jj <= g.ny && kk >= 0 && kk <= g.nz && kk <= k1;
                const double v = a.v[ic + sx * min(max(jj, 0), g.ny) + sxy * min(max(kk, 0), g.nz)];
                S.P[c][r] = ok ? v : 0.0;
            }
        }
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int kk = k0 - 1 + c;
#pragma unroll
            for (int r = 0; r < R + 1; ++r) {
                const int jj = j0 - 1 + r;
                const bool ok = ieok && jj >= 0 && jj < g.ny && kk >= 0 && kk < g.nz;
                const double v = a.beta[ie + g.nx * min(max(jj, 0), g.ny - 1) + exy * min(max(kk, 0), g.nz - 1)];
                S.B[c][r] = ok ? v : 0.0;
            }
        }
        if (MODE == MODE_INIT) {
#pragma unroll
            for (int r = 0; r < R; ++r) S.E[0][0][r] = a.F[ic + sx * min(j0 + r, g.ny) + sxy * k0];
        }
        const bool dir_i = (i == 0 && g.ft[0] == ECMG_DIRICHLET) || (i == g.nx && g.ft[1] == ECMG_DIRICHLET);
        const bool rob_i = (i == 0 && g.ft[0] == ECMG_ROBIN) || (i == g.nx && g.ft[1] == ECMG_ROBIN);
        int k = k0;
        for (; k + 3 < k1; k += 4) {
            col_step<MODE, R>(a, i, j0, k, k1, out_lane, iok, ieok, dir_i, rob_i, S.P[0], S.P[1], S.P[2], S.P[3], S.B[0], S.B[1],
                              S.B[2], S.E[0], S.E[1], acc0, acc1);
            col_step<MODE, R>(a, i, j0, k + 1, k1, out_lane, iok, ieok, dir_i, rob_i, S.P[1], S.P[2], S.P[3], S.P[0], S.B[1],
                              S.B[2], S.B[3], S.E[1], S.E[0], acc0, acc1);
            col_step<MODE, R>(a, i, j0, k + 2, k1, out_lane, iok, ieok, dir_i, rob_i, S.P[2], S.P[3], S.P[0], S.P[1], S.B[2],
                              S.B[3], S.B[0], S.E[0], S.E[1], acc0, acc1);
            col_step<MODE, R>(a, i, j0, k + 3, k1, out_lane, iok, ieok, dir_i, rob_i, S.P[3], S.P[0], S.P[1], S.P[2], S.B[3],
                              S.B[0], S.B[1], S.E[1], S.E[0], acc0, acc1);
        }
        if (k < k1)
            col_step<MODE, R>(a, i, j0, k, k1, out_lane, iok, ieok, dir_i, rob_i, S.P[0], S.P[1], S.P[2], S.P[3], S.B[0], S.B[1],
                              S.B[2], S.E[0], S.E[1], acc0, acc1);
        if (k + 1 < k1)
            col_step<MODE, R>(a, i, j0, k + 1, k1, out_lane, iok, ieok, dir_i, rob_i, S.P[1], S.P[2], S.P[3], S.P[0], S.B[1],
                              S.B[2], S.B[3], S.E[1], S.E[0], acc0, acc1);
        if (k + 2 < k1)
            col_step<MODE, R>(a, i, j0, k + 2, k1, out_lane, iok, ieok, dir_i, rob_i, S.P[2], S.P[3], S.P[0], S.P[1], S.B[2],
                              S.B[3], S.B[0], S.E[0], S.E[1], acc0, acc1);
    }
    if (MODE == MODE_APPLY || wid >= total) return;
    // wave partials in lane order (fixed), one pair per wave
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        acc0 += __shfl_xor(acc0, off, 64);
        acc1 += __shfl_xor(acc1, off, 64);
    }
    if (lane == 0) {
        a.partials[2 * (int64_t)wid] = acc0;
        if (MODE == MODE_INIT) a.partials[2 * (int64_t)wid + 1] = acc1;
    }
}

// The nodes on a Robin face (and on no Dirichlet face), which the column
// kernel leaves out: each is taken by the first Robin face (in face order) that
// holds it, one thread per node, with its full row -- the 27-point stencil read
// from global memory plus the face-mass terms of every Robin face it lies on --
// and the column kernel's epilogue; block partials follow the waves' partials.
template <int MODE>
__global__ void __launch_bounds__(256) k_col_face(const ColArgs a, const ColFaces fl, int part_off) {
    const Geom &g = a.g;
    __shared__ double red[2][4];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double acc0 = 0.0, acc1 = 0.0;
    if (t < fl.start[fl.nf]) {
        int s = 0;
        while (t >= fl.start[s + 1]) ++s;
        const int f = fl.face[s], ax = f / 2;
        const int pa = ax == 0 ? 1 : 0, qa = ax == 2 ? 1 : 2;
        const int n3[3] = {g.nx, g.ny, g.nz};
        const int64_t loc = t - fl.start[s];
        int ijk[3];
        ijk[ax] = (f & 1) ? n3[ax] : 0;
        ijk[pa] = (int)(loc % (n3[pa] + 1));
        ijk[qa] = (int)(loc / (n3[pa] + 1));
        const int i = ijk[0], j = ijk[1], k = ijk[2];
        bool skip = dir_node(g, i, j, k);
        for (int f2 = 0; f2 < f; ++f2)           // an earlier Robin face takes the node
            if (g.ft[f2] == ECMG_ROBIN && ijk[f2 / 2] == ((f2 & 1) ? n3[f2 / 2] : 0)) skip = true;
        if (!skip) {
            const int sx = g.sx, sxy = g.sx * g.sy;
            auto v = [&](int ii, int jj, int kk) -> double {
                if (ii < 0 || ii > g.nx || jj < 0 || jj > g.ny || kk < 0 || kk > g.nz) return 0.0;
                return a.v[ii + sx * jj + sxy * kk];
            };
            auto be = [&](int ii, int jj, int kk) -> double {
                if (ii < 0 || ii >= g.nx || jj < 0 || jj >= g.ny || kk < 0 || kk >= g.nz) return 0.0;
                return a.beta[ii + g.nx * jj + g.nx * g.ny * kk];
            };
            const double l00 = be(i - 1, j - 1, k - 1), l01 = be(i, j - 1, k - 1), l10 = be(i - 1, j, k - 1),
                         l11 = be(i, j, k - 1);
            const double u00 = be(i - 1, j - 1, k), u01 = be(i, j - 1, k), u10 = be(i - 1, j, k), u11 = be(i, j, k);
            double q = 0.0;
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    double sl, su;
                    if (oy < 0 && ox < 0) { sl = l00; su = u00; }
                    else if (oy < 0 && ox > 0) { sl = l01; su = u01; }
                    else if (oy > 0 && ox < 0) { sl = l10; su = u10; }
                    else if (oy > 0 && ox > 0) { sl = l11; su = u11; }
                    else if (oy < 0) { sl = l00 + l01; su = u00 + u01; }
                    else if (oy > 0) { sl = l10 + l11; su = u10 + u11; }
                    else if (ox < 0) { sl = l00 + l10; su = u00 + u10; }
                    else if (ox > 0) { sl = l01 + l11; su = u01 + u11; }
                    else { sl = (l00 + l01) + (l10 + l11); su = (u00 + u01) + (u10 + u11); }
                    const int m = (ox != 0) | ((oy != 0) << 1);
                    q += g.C[m | 4] * (sl * v(i + ox, j + oy, k - 1) + su * v(i + ox, j + oy, k + 1)) +
                         g.C[m] * ((sl + su) * v(i + ox, j + oy, k));
                }
            for (int f2 = 0; f2 < 6; ++f2) {     // face-mass terms of every Robin face the node is on
                const int a2 = f2 / 2;
                if (g.ft[f2] != ECMG_ROBIN || ijk[a2] != ((f2 & 1) ? n3[a2] : 0)) continue;
                const int p2 = a2 == 0 ? 1 : 0, q2 = a2 == 2 ? 1 : 2;
                auto nb = [&](int op, int oq) -> double {
                    int c[3] = {i, j, k};
                    c[p2] += op;
                    c[q2] += oq;
                    return v(c[0], c[1], c[2]);
                };
                q += robin_col(g, f2, a.alpha[f2], ijk[p2], ijk[q2], n3[p2], n3[q2], nb);
            }
            const int id = i + sx * j + sxy * k;
            if (MODE == MODE_APPLY) {
                __builtin_nontemporal_store(q, a.out + id);
            } else if (MODE == MODE_INIT) {
                const double rv = a.F[id] - q;
                __builtin_nontemporal_store(rv, a.out + id);
                const double z = a.dinv[id] * rv;           // 1/D with the Robin terms
                if (a.p_init) __builtin_nontemporal_store(z, a.p_out + id);
                acc0 += rv * z;
                acc1 += rv * rv;
            } else {
                __builtin_nontemporal_store(q, a.out + id);
                acc0 += a.v[id] * q;
            }
        }
    }
    if (MODE == MODE_APPLY) return;
    // block partials in a fixed order: lanes, then the 4 waves
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        acc0 += __shfl_xor(acc0, off, 64);
        acc1 += __shfl_xor(acc1, off, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = acc0;
        red[1][w] = acc1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        a.partials[2 * ((int64_t)part_off + blockIdx.x)] = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
        if (MODE == MODE_INIT)
            a.partials[2 * ((int64_t)part_off + blockIdx.x) + 1] = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
    }
}

}  // namespace

int col_waves(const Geom &g, int KZ, int *ntx, int *nty, int *nkz) {
    *ntx = (g.nx + 1 + 61) / 62;
    *nty = (g.ny + 1 + COL_R - 1) / COL_R;
    *nkz = (g.nz + 1 + KZ - 1) / KZ;
    return (*ntx) * (*nty) * (*nkz);
}

int col_faces(const Geom &g, ColFaces *fl) {
    const int n3[3] = {g.nx, g.ny, g.nz};
    fl->nf = 0;
    fl->start[0] = 0;
    for (int f = 0; f < 6; ++f) {
        if (g.ft[f] != ECMG_ROBIN) continue;
        const int ax = f / 2, pa = ax == 0 ? 1 : 0, qa = ax == 2 ? 1 : 2;
        fl->face[fl->nf] = f;
        fl->start[fl->nf + 1] = fl->start[fl->nf] + (int64_t)(n3[pa] + 1) * (n3[qa] + 1);
        ++fl->nf;
    }
    return (int)((fl->start[fl->nf] + 255) / 256);
}

int launch_col(int mode, const ColArgs &a, hipStream_t s) {
    const int waves = a.ntx * a.nty * a.nkz;
    const int nb = (waves + 3) / 4;
    if (mode == MODE_APPLY) launch_timed(k_col<MODE_APPLY, COL_R, 3>, dim3(nb), dim3(256), 0, s, a);
    else if (mode == MODE_INIT) launch_timed(k_col<MODE_INIT, COL_R, 2>, dim3(nb), dim3(256), 0, s, a);
    else launch_timed(k_col<MODE_PASSA0, COL_R, 3>, dim3(nb), dim3(256), 0, s, a);
    ColFaces fl;
    const int fb = col_faces(a.g, &fl);
    if (fb > 0) {
        if (mode == MODE_APPLY) hipLaunchKernelGGL(k_col_face<MODE_APPLY>, dim3(fb), dim3(256), 0, s, a, fl, waves);
        else if (mode == MODE_INIT) hipLaunchKernelGGL(k_col_face<MODE_INIT>, dim3(fb), dim3(256), 0, s, a, fl, waves);
        else hipLaunchKernelGGL(k_col_face<MODE_PASSA0>, dim3(fb), dim3(256), 0, s, a, fl, waves);
    }
    return waves + fb;
}

}  // namespace ecmg
