// Column stencil kernels for the large JCG levels (gfx950): operator apply,
// JCG initialisation and the stencil part of pass A (q = A p, p.q; at
// iterations >= 1 after the node-wise p update), each a matrix-free 27-point
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
// neighbours come from the adjacent lanes through DPP wavefront shifts (no LDS
// traffic: the exchange through LDS, not HBM, bounded the tiled kernels); each
// lane computes its column's parts of its own node and of both neighbours'
// nodes, so a node needs two shifted partial sums and the shifted betas of one
// element column rather than nine shifted plane values.  Every load is
// branch-free (clamped index; betas outside the grid zeroed afterwards), so the
// compiler waits for exactly the loads a step uses.
//
// Reductions: each wave sums its lanes' partials with shuffles and stores one
// pair; the one-block finishing kernels of jcg_kernels.hip (fixed order) take
// the scalar steps, so results are bitwise reproducible.
#include "ecmg_internal.h"

namespace ecmg {

namespace {

// the iteration index (x) and the `done` flag (y) of the JCG scalars in one
// load (a launch's first dependent read: one round trip instead of two)
__device__ __forceinline__ int2 iter_done(const JcgScalars *sc) {
    static_assert(offsetof(JcgScalars, done) == offsetof(JcgScalars, iter) + 4 && offsetof(JcgScalars, iter) % 8 == 0,
                  "iter and done adjacent");
    // an atomic 64-bit load, which the compiler cannot split into two
    const unsigned long long w = __hip_atomic_load(reinterpret_cast<const unsigned long long *>(&sc->iter),
                                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_int2((int)(unsigned)w, (int)(unsigned)(w >> 32));
}

// lane i receives lane i-1 (DPP wave_shr:1); lane 0 receives 0 (bound_ctrl)
__device__ __forceinline__ double from_left(double v) {
    const int lo = __builtin_amdgcn_mov_dpp((int)__double2loint(v), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)__double2hiint(v), 0x138, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}
// lane i receives lane i+1 (DPP wave_shl:1); lane 63 receives 0 (bound_ctrl)
__device__ __forceinline__ double from_right(double v) {
    const int lo = __builtin_amdgcn_mov_dpp((int)__double2loint(v), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)__double2hiint(v), 0x130, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

// block b of nb (dispatched round-robin over the 8 XCDs) -> the logical block
// that gives every XCD a contiguous range
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int per = nb >> 3;
    return b < (per << 3) ? (b & 7) * per + (b >> 3) : b;
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

// register rings of one wave lane, NR = D + 3 slots for a prefetch distance
// of D z-steps (planes k-1, k, k+1 in use and D in flight; the layer and
// epilogue rings use NR slots too, so that one unrolled pass of NR steps
// returns every ring to its first slot)
template <int R, int NR>
struct ColRegs {
    double P[NR][R + 2];   // input planes: rows j0-1 .. j0+R
    double B[NR][R + 1];   // element layers: element rows j0-1 .. j0+R-1, element x = i
    double E[NR][R];       // epilogue input of the output rows (INIT: F)
};

// The 27-point row of node (i, j, k) split by neighbour column: the centre
// column i (elements of x-index i-1 and i), column i-1 (elements i-1 only)
// and column i+1 (elements i only).  Lane i holds column i and the elements
// of x-index i, so it computes the centre part of its own node and, from its
// column, the part of node i+1 (weights from its own elements: `tr`) and of
// node i-1 (weights from the elements of x-index i-1, the left lane's: `tl`);
// node i adds the neighbours' parts with one wave shift each.  A neighbour in
// plane k-1 (k+1) couples through the lower (upper) layer's elements only, one
// in plane k through both: with sl, su the beta sums of the shared elements
// below and above, a neighbour row contributes
//   sl (Cz vm + C v0) + su (Cz vp + C v0),
// C, Cz the entries for the differing in-plane axes without / with z, each
// product accumulated by a fused multiply-add.  The two side parts share those
// plane combinations.
// L, Rt: the elements of x-index i-1 and i of the lower layer (rows j0-1 ..);
// LU, RU of the upper layer; r: the output row's index in the wave's rows.
template <int R>
__device__ __forceinline__ void col_row(const Geom &g, int r, const double (&L)[R + 1], const double (&Rt)[R + 1],
                                        const double (&LU)[R + 1], const double (&RU)[R + 1],
                                        const double (&Pm)[R + 2], const double (&P0)[R + 2],
                                        const double (&Pp)[R + 2], double &qc, double &tr, double &tl) {
    qc = 0.0;
    tr = 0.0;
    tl = 0.0;
#pragma unroll
    for (int oy = -1; oy <= 1; ++oy) {
        const int t = r + 1 + oy;                 // plane row of the neighbour row
        const int mo = (oy != 0) << 1;
        // element rows below (row j-1) / above (row j) the node row
        const double lL = oy > 0 ? L[r + 1] : oy < 0 ? L[r] : L[r] + L[r + 1];
        const double lR = oy > 0 ? Rt[r + 1] : oy < 0 ? Rt[r] : Rt[r] + Rt[r + 1];
        const double uL = oy > 0 ? LU[r + 1] : oy < 0 ? LU[r] : LU[r] + LU[r + 1];
        const double uR = oy > 0 ? RU[r + 1] : oy < 0 ? RU[r] : RU[r] + RU[r + 1];
        const double c0 = g.C[mo] * P0[t], s0 = g.C[mo | 1] * P0[t];
        const double ac = fma(g.C[mo | 4], Pm[t], c0), bc = fma(g.C[mo | 4], Pp[t], c0);
        const double as = fma(g.C[mo | 5], Pm[t], s0), bs = fma(g.C[mo | 5], Pp[t], s0);
        qc = fma(lL + lR, ac, qc);
        qc = fma(uL + uR, bc, qc);
        tr = fma(lR, as, tr);
        tr = fma(uR, bs, tr);
        tl = fma(lL, as, tl);
        tl = fma(uL, bs, tl);
    }
}

// One z-step: output plane k from the planes Pm (k-1), P0 (k), Pp (k+1) and the
// layers Bl (k-1), Bu (k); first issues the loads of plane k+1+D into Pn, layer
// k+D into Bn and the epilogue inputs of plane k+D into En.  Plane values of
// columns or rows outside the grid are clamped loads of grid nodes: every
// element holding such a neighbour lies outside the grid and carries beta = 0,
// so its weight is 0.
template <int MODE, int R, int D>
__device__ __forceinline__ void col_step(const ColArgs &a, const double *__restrict__ vin, int i, int j0, int k,
                                         int k1, bool out_lane,
                                         bool ieok, bool dir_i, bool rob_i, double (&Pm)[R + 2], double (&P0)[R + 2],
                                         double (&Pp)[R + 2],
                                         double (&Pn)[R + 2], double (&Bl)[R + 1], double (&Bu)[R + 1],
                                         double (&Bn)[R + 1], double (&Ec)[R], double (&En)[R], double &acc0,
                                         double &acc1) {
    const Geom &g = a.g;
    const int sx = g.sx, sxy = g.sx * g.sy, exy = g.nx * g.ny;
    const int ic = min(max(i, 0), g.nx), ie = min(max(i, 0), g.nx - 1);
    const bool dir_k = (k == 0 && g.ft[4] == ECMG_DIRICHLET) || (k == g.nz && g.ft[5] == ECMG_DIRICHLET);
    const bool rob_k = (k == 0 && g.ft[4] == ECMG_ROBIN) || (k == g.nz && g.ft[5] == ECMG_ROBIN);
    {   // prefetch: plane k+1+D, layer k+D, epilogue of plane k+D
        const int kp = k + 1 + D, kb = k + D, ke = k + D;
#pragma unroll
        for (int r = 0; r < R + 2; ++r) {
            const int jj = j0 - 1 + r;
            Pn[r] = vin[ic + sx * min(max(jj, 0), g.ny) + sxy * min(kp, g.nz)];
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
            for (int r = 0; r < R; ++r) En[r] = __builtin_nontemporal_load(a.F + ic + sx * min(j0 + r, g.ny) +
                                                                           sxy * min(ke, g.nz));
        }
    }
    // elements of x-index i-1 (the left lane's)
    double BlL[R + 1], BuL[R + 1];
#pragma unroll
    for (int r = 0; r < R + 1; ++r) {
        BlL[r] = from_left(Bl[r]);
        BuL[r] = from_left(Bu[r]);
    }
    double qc[R], tr[R], tl[R];
#pragma unroll
    for (int r = 0; r < R; ++r) col_row<R>(g, r, BlL, Bl, BuL, Bu, Pm, P0, Pp, qc[r], tr[r], tl[r]);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int j = j0 + r;
        const double q = qc[r] + from_left(tr[r]) + from_right(tl[r]);
        // nodes on a Robin face (and on no Dirichlet face) are the face blocks'
        const bool dir = dir_i || (j == 0 && g.ft[2] == ECMG_DIRICHLET) || (j == g.ny && g.ft[3] == ECMG_DIRICHLET) ||
                         dir_k;
        const bool rob = rob_i || (j == 0 && g.ft[2] == ECMG_ROBIN) || (j == g.ny && g.ft[3] == ECMG_ROBIN) || rob_k;
        if (!out_lane || j > g.ny || (rob && !dir)) continue;
        const int id = i + sx * j + sxy * k;
        if (MODE == MODE_APPLY) {
            __builtin_nontemporal_store(dir ? 0.0 : q, a.out + id);
        } else if (MODE == MODE_INIT) {
            const double rv = dir ? 0.0 : Ec[r] - q;
            __builtin_nontemporal_store(rv, a.out + id);
            // M^-1 from the beta already in registers: the diagonal C[0] * (sum of
            // the 8 element betas, in the order the setup's 1/D uses), so z is
            // what the stored 1/D gives, bit for bit (no Robin term here)
            double z;
            if (a.plain_cg) {
                z = rv;
            } else {
                const double s8 = ((((((BlL[r] + Bl[r]) + BlL[r + 1]) + Bl[r + 1]) + BuL[r]) + Bu[r]) + BuL[r + 1]) +
                                  Bu[r + 1];
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

// The 27-point row of node (i, j, k), read from global memory through v(idx)
// (the input value at flat node index idx): the stencil with the betas of the
// 8 surrounding elements plus the face-mass terms of every Robin face the
// node lies on.  Neighbour indices are clamped to the grid (an outside
// neighbour couples only through outside elements, whose beta is 0).
template <class V>
__device__ __forceinline__ double gather_q(const ColArgs &a, int i, int j, int k, V v) {
    const Geom &g = a.g;
    const int sx = g.sx, sxy = g.sx * g.sy, exy = g.nx * g.ny;
    int xo[3], yo[3], zo[3];
#pragma unroll
    for (int o = 0; o < 3; ++o) {
        xo[o] = min(max(i - 1 + o, 0), g.nx);
        yo[o] = sx * min(max(j - 1 + o, 0), g.ny);
        zo[o] = sxy * min(max(k - 1 + o, 0), g.nz);
    }
    auto be = [&](int ii, int jj, int kk) -> double {
        const bool ok = ii >= 0 && ii < g.nx && jj >= 0 && jj < g.ny && kk >= 0 && kk < g.nz;
        const double b = a.beta[min(max(ii, 0), g.nx - 1) + g.nx * min(max(jj, 0), g.ny - 1) +
                                exy * min(max(kk, 0), g.nz - 1)];
        return ok ? b : 0.0;
    };
    const double l00 = be(i - 1, j - 1, k - 1), l01 = be(i, j - 1, k - 1), l10 = be(i - 1, j, k - 1),
                 l11 = be(i, j, k - 1);
    const double u00 = be(i - 1, j - 1, k), u01 = be(i, j - 1, k), u10 = be(i - 1, j, k), u11 = be(i, j, k);
    // all 27 values loaded before any is used: one memory round trip
    double pv[3][3][3];                           // [z][y][x] offsets + 1
#pragma unroll
    for (int oz = 0; oz < 3; ++oz)
#pragma unroll
        for (int oy = 0; oy < 3; ++oy)
#pragma unroll
            for (int ox = 0; ox < 3; ++ox) pv[oz][oy][ox] = v(xo[ox] + yo[oy] + zo[oz]);
    // keep the scheduler from interleaving the loads with their uses (it
    // otherwise splits them into two dependent rounds)
    __builtin_amdgcn_sched_barrier(0);
    double q = 0.0;
#pragma unroll
    for (int oy = -1; oy <= 1; ++oy)
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
            q += g.C[m | 4] * (sl * pv[0][oy + 1][ox + 1] + su * pv[2][oy + 1][ox + 1]) +
                 g.C[m] * ((sl + su) * pv[1][oy + 1][ox + 1]);
        }
    const int ijk[3] = {i, j, k}, n3[3] = {g.nx, g.ny, g.nz};
    for (int f = 0; f < 6; ++f) {
        const int ax = f / 2;
        if (g.ft[f] != ECMG_ROBIN || ijk[ax] != ((f & 1) ? n3[ax] : 0)) continue;
        const int pa = ax == 0 ? 1 : 0, qa = ax == 2 ? 1 : 2;
        auto nb = [&](int op, int oq) -> double {
            int c[3] = {i, j, k};
            c[pa] += op;
            c[qa] += oq;
            return v(c[0] + sx * c[1] + sxy * c[2]);
        };
        q += robin_col(g, f, a.alpha[f], ijk[pa], ijk[qa], n3[pa], n3[qa], nb);
    }
    return q;
}

// block partials in a fixed order (lanes, then the 4 waves): acc0 (and acc1
// if TWO) of the block into slot[0] (slot[1])
template <bool TWO>
__device__ __forceinline__ void block_partials(double acc0, double acc1, double *slot, double (*red)[4]) {
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
        slot[0] = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
        if (TWO) slot[1] = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
    }
}

// node of thread t of a launch over the grid's nodes (x fastest); false past the end
__device__ __forceinline__ bool gather_node(const Geom &g, int64_t t, int &i, int &j, int &k) {
    const int nxp = g.nx + 1, nyp = g.ny + 1;
    if (t >= (int64_t)nxp * nyp * (g.nz + 1)) return false;
    i = (int)(t % nxp);
    const int64_t rw = t / nxp;
    j = (int)(rw % nyp);
    k = (int)(rw / nyp);
    return true;
}

// The nodes on a Robin face (and on no Dirichlet face), which the column
// waves leave out: each is taken by the first Robin face (in face order) that
// holds it, one thread per node, with its full row -- the 27-point stencil read
// from global memory plus the face-mass terms of every Robin face it lies on --
// and the column epilogue.  These blocks follow the column blocks in the same
// launch; block partials follow the waves' partials (part_off of them).
template <int MODE>
__device__ __forceinline__ void col_face_block(const ColArgs &a, const double *__restrict__ vin, int bid,
                                               int part_off) {
    const Geom &g = a.g;
    const ColFaces &fl = a.fl;
    __shared__ double red[2][4];
    const int64_t t = (int64_t)bid * 256 + threadIdx.x;
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
            const double q = gather_q(a, i, j, k, [&](int idx) { return vin[idx]; });
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
                acc0 += vin[id] * q;
            }
        }
    }
    if (MODE == MODE_APPLY) return;
    block_partials<MODE == MODE_INIT>(acc0, acc1, a.partials + 2 * ((int64_t)part_off + bid), red);
}

// WPE: waves per SIMD the register budget is set for (init, 2 rows: 150
// VGPRs, 3 waves fit; the stencil of pass A, 4 rows: about 200 VGPRs, 2
// waves); D: prefetch distance in z-steps
template <int MODE, int R, int WPE, int D>
__global__ void __launch_bounds__(256, WPE) k_col(const ColArgs a) {
    constexpr int NR = D + 3;
    const Geom &g = a.g;
    const int2 itd = MODE == MODE_PASSA0 ? iter_done(a.sc) : make_int2(0, 0);
    if (itd.y) return;                            // done: uniform over the grid
    // iterations >= 1 alternate the direction buffers (the iteration's parity)
    const double *__restrict__ vin = (MODE == MODE_PASSA0 && a.v_odd && (itd.x & 1)) ? a.v_odd : a.v;
    if ((int)blockIdx.x >= a.ncb) {               // the Robin-face blocks (uniform per block)
        col_face_block<MODE>(a, vin, (int)blockIdx.x - a.ncb, a.ntx * a.nty * a.nkz);
        return;
    }
    const int cb = blockIdx.x;                    // column block
    const int lane = threadIdx.x & 63;
    const int wid = cb * 4 + (threadIdx.x >> 6);             // partial slot
    const int total = a.ntx * a.nty * a.nkz;
    int tx, ty, tz;
    if (a.order == 0) {
        // consecutive waves take consecutive x-segments of the same rows
        tx = wid % a.ntx;
        const int t2 = wid / a.ntx;
        ty = t2 % a.nty;
        tz = t2 / a.nty;
    } else {
        // the 4 waves of a block take 4 consecutive row groups of one x-segment,
        // so the y-halo rows they share are fetched once into the CU's caches;
        // order 2 also gives each XCD a contiguous range of blocks (blocks are
        // dispatched round-robin over the XCDs), so the halo rows between
        // neighbouring blocks are shared through that XCD's L2
        const int b = a.order == 2 ? xcd_block(cb, a.ncb) : cb;
        const int nty4 = a.nty >> 2;
        tx = b % a.ntx;
        const int t2 = b / a.ntx;
        ty = 4 * (t2 % nty4) + (threadIdx.x >> 6);
        tz = t2 / nty4;
    }
    double acc0 = 0.0, acc1 = 0.0;
    if (wid < total) {
        const int i = 62 * tx - 1 + lane;
        const int j0 = ty * R;
        const int k0 = tz * a.KZ, k1 = min(k0 + a.KZ, g.nz + 1);
        const bool iok = i >= 0 && i <= g.nx, ieok = i >= 0 && i < g.nx;
        const bool out_lane = lane >= 1 && lane <= 62 && iok;
        const int sx = g.sx, sxy = g.sx * g.sy, exy = g.nx * g.ny;
        const int ic = min(max(i, 0), g.nx), ie = min(max(i, 0), g.nx - 1);
        ColRegs<R, NR> S;
        // prologue: planes k0-1 .. k0+D, layers k0-1 .. k0+D-1, epilogue of
        // planes k0 .. k0+D-1
#pragma unroll
        for (int c = 0; c < D + 2; ++c) {
            const int kk = k0 - 1 + c;
#pragma unroll
            for (int r = 0; r < R + 2; ++r) {
                const int jj = j0 - 1 + r;
                S.P[c][r] = vin[ic + sx * min(max(jj, 0), g.ny) + sxy * min(max(kk, 0), g.nz)];
            }
        }
#pragma unroll
        for (int c = 0; c < D + 1; ++c) {
            const int kk = k0 - 1 + c;
#pragma unroll
            for (int r = 0; r < R + 1; ++r) {
                const int jj = j0 - 1 + r;
                const bool ok = ieok && jj >= 0 && jj < g.ny && kk >= 0 && kk < g.nz && kk < k1;
                const double v = a.beta[ie + g.nx * min(max(jj, 0), g.ny - 1) + exy * min(max(kk, 0), g.nz - 1)];
                S.B[c][r] = ok ? v : 0.0;
            }
        }
        if (MODE == MODE_INIT) {
#pragma unroll
            for (int c = 0; c < D; ++c)
#pragma unroll
                for (int r = 0; r < R; ++r)
                    S.E[c][r] = a.F[ic + sx * min(j0 + r, g.ny) + sxy * min(k0 + c, g.nz)];
        }
        const bool dir_i = (i == 0 && g.ft[0] == ECMG_DIRICHLET) || (i == g.nx && g.ft[1] == ECMG_DIRICHLET);
        const bool rob_i = (i == 0 && g.ft[0] == ECMG_ROBIN) || (i == g.nx && g.ft[1] == ECMG_ROBIN);
        // step s of a pass of NR steps: planes in slots s, s+1, s+2, the load
        // into s+2+D; layers in s, s+1, the load into s+1+D; epilogue in s,
        // the load into s+D (all mod NR)
        int k = k0;
        for (; k + NR - 1 < k1; k += NR) {
#pragma unroll
            for (int t = 0; t < NR; ++t)
                col_step<MODE, R, D>(a, vin, i, j0, k + t, k1, out_lane, ieok, dir_i, rob_i, S.P[t % NR],
                                     S.P[(t + 1) % NR], S.P[(t + 2) % NR], S.P[(t + 2 + D) % NR], S.B[t % NR],
                                     S.B[(t + 1) % NR], S.B[(t + 1 + D) % NR], S.E[t % NR], S.E[(t + D) % NR], acc0,
                                     acc1);
        }
#pragma unroll
        for (int t = 0; t < NR - 1; ++t)
            if (k + t < k1)
                col_step<MODE, R, D>(a, vin, i, j0, k + t, k1, out_lane, ieok, dir_i, rob_i, S.P[t % NR],
                                     S.P[(t + 1) % NR], S.P[(t + 2) % NR], S.P[(t + 2 + D) % NR], S.B[t % NR],
                                     S.B[(t + 1) % NR], S.B[(t + 1 + D) % NR], S.E[t % NR], S.E[(t + D) % NR], acc0,
                                     acc1);
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

// JCG init one thread per node: r = F - A x, z = D^-1 r (p_0 = z stored if
// p_init), r.z and r.r block partials.  For the small grids, whose vectors
// stay in the caches between passes: there a block's march through its
// planes is a chain of memory latencies, and one thread per node has none.
__global__ void __launch_bounds__(256) k_gather_init(const ColArgs a) {
    __shared__ double red[2][4];
    const Geom &g = a.g;
    double acc0 = 0.0, acc1 = 0.0;
    int i, j, k;
    if (gather_node(g, (int64_t)blockIdx.x * 256 + threadIdx.x, i, j, k)) {
        const int id = i + g.sx * j + g.sx * g.sy * k;
        const double *__restrict__ x = a.v;
        const bool dir = dir_node(g, i, j, k);
        const double fv = a.F[id], dv = a.dinv[id];   // issued with the row's loads
        const double q = dir ? 0.0 : gather_q(a, i, j, k, [&](int idx) { return x[idx]; });
        const double rv = dir ? 0.0 : fv - q;
        __builtin_nontemporal_store(rv, a.out + id);
        const double z = dv * rv;
        if (a.p_init) __builtin_nontemporal_store(z, a.p_out + id);
        acc0 += rv * z;
        acc1 += rv * rv;
    }
    block_partials<true>(acc0, acc1, a.partials + 2 * (int64_t)blockIdx.x, red);
}

// The stencil of pass A one thread per node: q = A p and p.q block partials,
// p read from the buffer of the iteration's parity (a.it, the iteration whose
// node-wise p update ran just before).  A version that formed
// p at the 27 neighbours itself (one launch per pass A, three loads per
// neighbour) ran 1.6x slower on 65^3 than the p update plus this kernel.
__global__ void __launch_bounds__(256) k_gather_a(const ColArgs a) {
    __shared__ double red[2][4];
    const Geom &g = a.g;
    // the iteration comes with the launch, so the row's loads depend on no
    // other load; `done` (which this iteration's p update may have set) is
    // loaded alongside them and checked before any store
    const int dn = a.sc->done;
    const double *__restrict__ vin = (a.v_odd && (a.it & 1)) ? a.v_odd : a.v;
    double acc0 = 0.0, qv = 0.0, pv = 0.0;
    int64_t id = -1;
    int i, j, k;
    if (gather_node(g, (int64_t)blockIdx.x * 256 + threadIdx.x, i, j, k)) {
        id = i + g.sx * j + (int64_t)g.sx * g.sy * k;
        const bool dir = dir_node(g, i, j, k);
        qv = dir ? 0.0 : gather_q(a, i, j, k, [&](int idx) { return vin[idx]; });
        pv = vin[id];
    }
    if (dn) return;                               // uniform over the grid
    if (id >= 0) {
        __builtin_nontemporal_store(qv, a.out + id);
        acc0 += pv * qv;
    }
    block_partials<false>(acc0, 0.0, a.partials + 2 * (int64_t)blockIdx.x, red);
}

}  // namespace

// wave grid: x-segments of 62 nodes, row groups of R rows, z-chunks of KZ
// planes.  order 0: waves in x-segment order; 1: the 4 waves of a block in
// row-group order (row groups padded to a multiple of 4; the padding waves
// produce nothing and store zero partials); 2: as 1, blocks contiguous per XCD.
int col_waves(const Geom &g, int KZ, int order, int R, int *ntx, int *nty, int *nkz) {
    *ntx = (g.nx + 1 + 61) / 62;
    *nty = (g.ny + 1 + R - 1) / R;
    if (order != 0) *nty = (*nty + 3) & ~3;
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
    // the wave grid (a.nty) was laid out for a.R rows per wave
    if (a.R != (mode == MODE_PASSA0 ? COL_R_A0 : COL_R_INIT)) return -1;
    const int waves = a.ntx * a.nty * a.nkz;
    ColArgs b = a;
    b.ncb = (waves + 3) / 4;
    const int fb = col_faces(a.g, &b.fl);
    // the face blocks after the column blocks, where they fill the launch's
    // tail (spread among the column blocks they ran slower)
    const dim3 grid(b.ncb + fb);
    // one z-step of prefetch: two steps, or 4 waves per SIMD for the stencil
    // of pass A, measured no faster on 513^3
    if (mode == MODE_APPLY) launch_timed(k_col<MODE_APPLY, COL_R_INIT, 3, 1>, grid, dim3(256), 0, s, b);
    else if (mode == MODE_INIT) launch_timed(k_col<MODE_INIT, COL_R_INIT, 2, 1>, grid, dim3(256), 0, s, b);
    else launch_timed(k_col<MODE_PASSA0, COL_R_A0, 2, 1>, grid, dim3(256), 0, s, b);
    return waves + fb;
}

int gather_blocks(const Geom &g) {
    return (int)(((int64_t)(g.nx + 1) * (g.ny + 1) * (g.nz + 1) + 255) / 256);
}

int launch_gather_init(const ColArgs &a, hipStream_t s) {
    const int nb = gather_blocks(a.g);
    launch_timed(k_gather_init, dim3(nb), dim3(256), 0, s, a);
    return nb;
}

int launch_gather_a(const ColArgs &a, hipStream_t s) {
    const int nb = gather_blocks(a.g);
    launch_timed(k_gather_a, dim3(nb), dim3(256), 0, s, a);
    return nb;
}

}  // namespace ecmg
