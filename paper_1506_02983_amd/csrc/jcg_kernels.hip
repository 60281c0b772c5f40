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
// The scalar steps run either in one-block finishing kernels after each pass,
// or -- when a pass has few blocks, where launches rather than bytes set the
// time -- folded into the next pass: every block of pass A sums the (r.z, r.r)
// partials of pass B (or init) itself, in one fixed order, so all blocks take
// the same stop decision and the same beta; every block of pass B likewise sums
// pass A's p.q partials for alpha.  Block 0 publishes the scalars.  Values that
// block 0 writes are never read by the other blocks of the same launch: the
// iteration index is a launch argument, rho alternates between two slots, and
// a breakdown found in pass B is handed to the next pass A.
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

constexpr int NTF = 1024;              // threads of a one-block finishing kernel


// 2-vector of T for 16-byte (double) / 8-byte (float) accesses
template <typename T> struct Vec2;
template <> struct Vec2<double> { using type = double2; };
template <> struct Vec2<float> { using type = float2; };

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

// Sum over blocks b < nb of partials[2 b + i] (i < NV) by one block of NTF
// threads: 8 independent loads in flight per thread, then a fixed-order
// combination, so the total does not depend on timing.  Result in thread 0.
template <int NV>
__device__ __forceinline__ void sum_partials(const double *__restrict__ partials, int nb, double (&tot)[NV],
                                             double (*red)[NTF / 64]) {
    constexpr int U = 8;
    double acc[U][NV];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[u][i] = 0.0;
    int b = threadIdx.x;
    for (; b + (U - 1) * NTF < nb; b += U * NTF) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int i = 0; i < NV; ++i) acc[u][i] += partials[2 * (int64_t)(b + u * NTF) + i];
    }
    for (; b < nb; b += NTF)
#pragma unroll
        for (int i = 0; i < NV; ++i) acc[0][i] += partials[2 * (int64_t)b + i];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double t = acc[0][i];
#pragma unroll
        for (int u = 1; u < U; ++u) t += acc[u][i];
        tot[i] = t;
    }
    block_sum<NV, NTF>(tot, red);
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
// coordinates are (pi, qi); neighbours come from the LDS planes (slots s0, s1,
// s2 = planes k-1, k, k+1) around LDS position (lj, li).  Face elements around
// the node: (ep, eq) = (pi-1+dp, qi-1+dq); the node sits at local corner
// (1-dp, 1-dq) of each; the face mass couples it to the face element's 4
// corners with hp*hq*(1/9, 1/18, 1/36) by the number of differing in-face axes.
template <int AX, typename T, typename Planes>
__device__ __forceinline__ T robin_term(const Geom &g, int face, const T *al, int pi, int qi, int np, int nq,
                                     Planes sv, int s0, int s1, int s2, int lj, int li) {
    T s = 0;
    for (int dq = 0; dq < 2; ++dq) {
        const int eq = qi - 1 + dq;
        if (eq < 0 || eq >= nq) continue;
        for (int dp = 0; dp < 2; ++dp) {
            const int ep = pi - 1 + dp;
            if (ep < 0 || ep >= np) continue;
            const T a = al[ep + (int64_t)np * eq];
            T t = 0;
            for (int bq = 0; bq < 2; ++bq)
                for (int bp = 0; bp < 2; ++bp) {
                    const int op = dp - 1 + bp, oq = dq - 1 + bq;
                    const int c = (bp != 1 - dp) + (bq != 1 - dq);
                    T vv;
                    if (AX == 0) vv = sv[oq < 0 ? s0 : (oq > 0 ? s2 : s1)][lj + op][li];        // (p,q) = (y,z)
                    else if (AX == 1) vv = sv[oq < 0 ? s0 : (oq > 0 ? s2 : s1)][lj][li + op];   // (p,q) = (x,z)
                    else vv = sv[s1][lj + oq][li + op];                                         // (p,q) = (x,y)
                    t += (T)g.M[face][c] * vv;
                }
            s += a * t;
        }
    }
    return s;
}

// ---------------------------------------------------------------------------
// tiled stencil kernel: MODE_APPLY (q = A v), MODE_INIT (r = F - A x, r.z, r.r),
// MODE_PASSA (fused JCG pass A), MODE_PASSA0 (its iteration 0 from a stored p_0)
// ---------------------------------------------------------------------------

// Rolling LDS buffers: 4 node planes and 3 element layers, so the plane being
// filled never aliases the three planes being read and one barrier per z-step
// suffices.  Declared by the kernel, once for both forms of the body.
template <typename T, int TYv>
struct StencilLds {
    T sv[4][TYT + 2][TX + 2];
    T sb[3][TYT + 1][TX + 1];
    double red[2][TX * TYv / 64];
    double s_beta;
    int s_flag;
};

// NT: streaming hints on the vector accesses (grids of STREAM_MIN_NODES nodes
// or more)
template <typename T, int MODE, int TYv, int RYv, bool NT>
__device__ __forceinline__ void stencil_body(const StencilArgs<T> &a, StencilLds<T, TYv> &L) {
    constexpr int NTv = TX * TYv;
    static_assert(TYv * RYv == TYT, "a block shape covers the tile height");
    auto &sv = L.sv;
    auto &sb = L.sb;
    auto &red = L.red;
    double &s_beta = L.s_beta;
    int &s_flag = L.s_flag;
    constexpr int NH = 2 * (TX + 2) + 2 * TYT;   // halo nodes of a plane tile
    constexpr int NHB = (TX + 1) + TYT;          // halo elements of a layer tile
    static_assert(NH <= NTv && NHB <= NTv, "one halo value per thread");

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

    // MODE_PASSA0: pass A of iteration 0 when init has stored p_0 = D^-1 r_0
    // in p1: the stencil input is p_0 itself (no r, 1/D loads, no p store)
    constexpr bool PA = MODE == MODE_PASSA || MODE == MODE_PASSA0;
    bool first = true;
    T alpha_prev = 0, betak = 0;
    const T *pin = a.p0;
    T *pout = a.p1;
    // Folded scalar step (pass A): the iteration index and the buffers come
    // with the launch; the sums of the previous pass's partials are loaded here
    // and resolved after the first planes' loads are issued, so one memory
    // round trip covers both.
    double fold_t[2] = {0.0, 0.0};
    // the scalars the folded step reads, loaded here with the partials: no
    // block of this launch writes them, except `done` (block 0 may set it),
    // which each block takes from thread 0 through LDS below
    int f_done = 0, f_brk = 0, f_fixed = 0, f_maxit = 0;
    double f_tol = 0.0, f_rho_prev = 1.0, f_alpha = 0.0;
    if (PA && a.fold) {
        const int it = a.it;
        first = (it == 0);
        pin = (it & 1) ? a.p1 : a.p0;
        pout = (it & 1) ? a.p0 : a.p1;
        const JcgScalars *scf = a.sc;
        f_done = scf->done;
        f_brk = scf->brk;
        f_fixed = scf->fixed;
        f_maxit = scf->max_iter;
        f_tol = scf->tol;
        f_alpha = scf->alpha;
        if (it > 0) f_rho_prev = scf->rho_f[(it - 1) & 1];
        for (int b = tid; b < a.fold_nb; b += NTv) {
            fold_t[0] += a.partials2[2 * b];
            fold_t[1] += a.partials2[2 * b + 1];
        }
    } else if (PA) {
        const JcgScalars *sc = a.sc;
        if (sc->done) return;                     // uniform over the grid
        const int it = MODE == MODE_PASSA0 ? 0 : sc->iter;
        first = (it == 0);
        alpha_prev = (T)sc->alpha;
        betak = (T)sc->beta;
        pin = (it & 1) ? a.p1 : a.p0;
        pout = (it & 1) ? a.p0 : a.p1;
    }
    const int64_t sxy = (int64_t)g.sx * g.sy;
    const int64_t exy = (int64_t)g.nx * g.ny;
    const int i = i0 + tx;

    // Per-thread positions, fixed for the whole z-march: in-plane offsets of
    // this thread's RYv interior nodes and elements and of its halo node and
    // halo element (-1 when outside the grid).
    int off[RYv], eoff[RYv];
#pragma unroll
    for (int r = 0; r < RYv; ++r) {
        const int j = j0 + ty + TYv * r;
        off[r] = (i <= g.nx && j <= g.ny) ? i + g.sx * j : -1;
        eoff[r] = (i < g.nx && j < g.ny) ? i + g.nx * j : -1;
    }
    int hli = 0, hlj = 0, hoff = -1, bli = 0, blj = 0, beoff = -1;
    if (tid < NH) {
        const int h = tid;
        if (h < TX + 2) { hlj = 0; hli = h; }
        else if (h < 2 * (TX + 2)) { hlj = TYT + 1; hli = h - (TX + 2); }
        else if (h < 2 * (TX + 2) + TYT) { hli = 0; hlj = 1 + h - 2 * (TX + 2); }
        else { hli = TX + 1; hlj = 1 + h - 2 * (TX + 2) - TYT; }
        const int ii = i0 + hli - 1, jj = j0 + hlj - 1;
        if (ii >= 0 && ii <= g.nx && jj >= 0 && jj <= g.ny) hoff = ii + g.sx * jj;
    }
    if (tid < NHB) {
        if (tid < TX + 1) { blj = 0; bli = tid; }
        else { bli = 0; blj = 1 + tid - (TX + 1); }
        const int ie = i0 + bli - 1, je = j0 + blj - 1;
        if (ie >= 0 && ie < g.nx && je >= 0 && je < g.ny) beoff = ie + g.nx * je;
    }

    // ---- raw loads into registers, issued PF z-steps before they are used ----
    // A register set holds, for one z-step k: the raw inputs of plane k+1 (pass
    // A: 1/D, r, p_old; apply/init: v) for this thread's interior and halo
    // nodes, beta of element layer k, and the epilogue inputs of output plane k
    // (pass A: x; init: F and 1/D).  With PF = 1 the loads of step k+1 are in
    // flight while step k computes; PF = 2 alternates two sets.
    struct RegSet {
        T ra[RYv], rb[RYv], rc[RYv], ha, hb, hc, bb[RYv], bh, ea[RYv], eb[RYv];
    };
    RegSet SA, SB;
    auto fetch_node = [&](int o, int kk, T &va, T &vb, T &vc) {
        va = vb = vc = 0;
        if (o < 0 || kk < 0 || kk > g.nz) return;
        const int64_t id = (int64_t)o + sxy * kk;
        if (MODE == MODE_PASSA0) {
            va = pout[id];
        } else if (MODE == MODE_PASSA) {
            va = a.dinv[id];
            vb = a.r[id];
            if (!first) vc = pin[id];
        } else {
            va = a.v[id];
        }
    };
    // fill set S for z-step k: plane k+1, layer k, epilogue of plane k
    auto fetch_set = [&](RegSet &S, int k) {
#pragma unroll
        for (int r = 0; r < RYv; ++r) fetch_node(off[r], k + 1, S.ra[r], S.rb[r], S.rc[r]);
        fetch_node(hoff, k + 1, S.ha, S.hb, S.hc);
        const bool ok = k >= 0 && k < g.nz;
#pragma unroll
        for (int r = 0; r < RYv; ++r) S.bb[r] = (ok && eoff[r] >= 0) ? a.beta[eoff[r] + exy * k] : (T)0;
        S.bh = (ok && beoff >= 0) ? a.beta[beoff + exy * k] : (T)0;
#pragma unroll
        for (int r = 0; r < RYv; ++r) {
            S.ea[r] = S.eb[r] = 0;
            if (MODE == MODE_APPLY || MODE == MODE_PASSA0 || off[r] < 0 || k < 0 || k > g.nz) continue;
            const int64_t id = (int64_t)off[r] + sxy * k;
            // epilogue inputs are read once: non-temporal on large grids
            if (MODE == MODE_PASSA) {
                if (!first) S.ea[r] = ld1<NT>(a.x + id);
            } else {
                S.ea[r] = ld1<NT>(a.F + id);
                S.eb[r] = ld1<NT>(a.dinv + id);
            }
        }
    };
    // value stored in LDS: v, or the pass-A search direction D^-1 r + beta p_old
    auto node_value = [&](T va, T vb, T vc) -> T {
        if (MODE == MODE_PASSA) {
            const T z = va * vb;
            return first ? z : z + betak * vc;
        }
        return va;                                // apply / init: v; MODE_PASSA0: p_0
    };
    auto vslot = [](int k) { return (k + 4) & 3; };
    auto bslot = [](int k) { return (k + 3) % 3; };
    T pold_next[RYv], pold_cur[RYv], xa_cur[RYv], xb_cur[RYv];
    // plane k+1 and layer k of set S into LDS
    auto commit_set = [&](const RegSet &S, int k) {
        const int slot = vslot(k + 1);
#pragma unroll
        for (int r = 0; r < RYv; ++r) {
            sv[slot][ty + TYv * r + 1][tx + 1] = node_value(S.ra[r], S.rb[r], S.rc[r]);
            pold_next[r] = S.rc[r];
        }
        if (tid < NH) sv[slot][hlj][hli] = node_value(S.ha, S.hb, S.hc);
        const int bs = bslot(k);
#pragma unroll
        for (int r = 0; r < RYv; ++r) sb[bs][ty + TYv * r + 1][tx + 1] = S.bb[r];
        if (tid < NHB) sb[bs][blj][bli] = S.bh;
    };

    T C[8];
#pragma unroll
    for (int m = 0; m < 8; ++m) C[m] = (T)g.C[m];

    double acc0 = 0.0, acc1 = 0.0;

    // prologue: planes k0-1 and k0 (sets SA and SB as steps k0-2 and k0-1),
    // both in flight together
    fetch_set(SA, k0 - 2);           // plane k0-1, layer k0-2 (unused), epilogue k0-2 (unused)
    fetch_set(SB, k0 - 1);           // plane k0, layer k0-1
    if (PA && a.fold) {
        // resolve the folded scalar step of the previous pass B (or init).
        // Block 0 of this launch may set `done`, so each block reads it once,
        // through LDS; every block sums the same partials in the same order.
        JcgScalars *sc = a.sc;
        const int it = a.it;
        if (tid == 0) s_flag = f_done ? -1 : (f_brk ? -2 : 0);
        __syncthreads();
        const int pre = s_flag;
        if (pre == -1) return;                    // stopped by an earlier launch
        block_sum<2, NTv>(fold_t, red);
        if (tid == 0) {
            int dn;
            double bk = 0.0;
            if (pre == -2) {
                dn = DONE_BREAKDOWN;              // the previous pass B found p.q <= 0
            } else {
                const double rz = fold_t[0], rr = fold_t[1], rn = sqrt(rr);
                if (f_fixed >= 0) dn = (it >= f_fixed) ? DONE_CONVERGED : DONE_RUNNING;
                else if (!(rn > f_tol)) dn = DONE_CONVERGED;
                else if (it >= f_maxit) dn = DONE_MAXITER;
                else dn = DONE_RUNNING;
                if (it > 0) bk = rz / f_rho_prev;
                if (blockIdx.x == 0) {
                    sc->iter = it;
                    sc->rho = rz;
                    sc->rho_f[it & 1] = rz;
                    sc->rr = rr;
                    sc->beta = bk;
                    // stopping after a pass B leaves that iteration's x update
                    sc->pending = (dn != DONE_RUNNING && it > 0) ? 1 : 0;
                }
            }
            if (blockIdx.x == 0 && dn != DONE_RUNNING) sc->done = dn;
            s_beta = bk;
            s_flag = dn;
        }
        __syncthreads();
        if (s_flag != DONE_RUNNING) return;
        alpha_prev = (T)f_alpha;
        betak = (T)s_beta;
    }
    commit_set(SA, k0 - 2);
    commit_set(SB, k0 - 1);
    fetch_set(SA, k0);
    if (PF == 2) fetch_set(SB, k0 + 1);

    // one z-step: output plane k from planes k-1, k, k+1 (S holds plane k+1)
    auto step = [&](RegSet &S, int k) {
#pragma unroll
        for (int r = 0; r < RYv; ++r) {
            pold_cur[r] = pold_next[r];
            xa_cur[r] = S.ea[r];
            xb_cur[r] = S.eb[r];
        }
        commit_set(S, k);
        __syncthreads();
        if (k + PF < k1) fetch_set(S, k + PF);

        const int s0 = vslot(k - 1), s1 = vslot(k), s2 = vslot(k + 1);
        const int b0 = bslot(k - 1), b1 = bslot(k);
#pragma unroll
        for (int r = 0; r < RYv; ++r) {
            const int jj = ty + TYv * r;
            const int j = j0 + jj;
            const int li = tx + 1, lj = jj + 1;
            // beta of the 8 elements around the node: layer below (k-1) and
            // above (k), in-plane offsets [dy][dx] (element i-1+dx, j-1+dy)
            const T l00 = sb[b0][lj - 1][li - 1], l01 = sb[b0][lj - 1][li];
            const T l10 = sb[b0][lj][li - 1], l11 = sb[b0][lj][li];
            const T u00 = sb[b1][lj - 1][li - 1], u01 = sb[b1][lj - 1][li];
            const T u10 = sb[b1][lj][li - 1], u11 = sb[b1][lj][li];
            // For in-plane neighbour offset (oy, ox), the elements of one layer
            // that contain both the node and the neighbour column: one element
            // (diagonal), two (edge) or all four (centre).
            T q = 0;
#pragma unroll
            for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
                for (int ox = -1; ox <= 1; ++ox) {
                    T sl, su;
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
                    const T vm = sv[s0][lj + oy][li + ox];
                    const T v0 = sv[s1][lj + oy][li + ox];
                    const T vp = sv[s2][lj + oy][li + ox];
                    // neighbours in planes k-1 / k+1 share only the layer between;
                    // neighbours in plane k are shared by both layers
                    q += C[m | 4] * (sl * vm + su * vp) + C[m] * ((sl + su) * v0);
                }
            if (i > g.nx || j > g.ny) continue;
            // Robin faces (face-mass terms, rare: boundary nodes only)
            if (i == 0 && g.ft[0] == ECMG_ROBIN) q += robin_term<0>(g, 0, a.alpha[0], j, k, g.ny, g.nz, sv, s0, s1, s2, lj, li);
            if (i == g.nx && g.ft[1] == ECMG_ROBIN) q += robin_term<0>(g, 1, a.alpha[1], j, k, g.ny, g.nz, sv, s0, s1, s2, lj, li);
            if (j == 0 && g.ft[2] == ECMG_ROBIN) q += robin_term<1>(g, 2, a.alpha[2], i, k, g.nx, g.nz, sv, s0, s1, s2, lj, li);
            if (j == g.ny && g.ft[3] == ECMG_ROBIN) q += robin_term<1>(g, 3, a.alpha[3], i, k, g.nx, g.nz, sv, s0, s1, s2, lj, li);
            if (k == 0 && g.ft[4] == ECMG_ROBIN) q += robin_term<2>(g, 4, a.alpha[4], i, j, g.nx, g.ny, sv, s0, s1, s2, lj, li);
            if (k == g.nz && g.ft[5] == ECMG_ROBIN) q += robin_term<2>(g, 5, a.alpha[5], i, j, g.nx, g.ny, sv, s0, s1, s2, lj, li);
            const bool dir = is_dirichlet(g, i, j, k);
            const int64_t id = (int64_t)off[r] + sxy * k;
            // outputs: coalesced rows, written once per pass (non-temporal on large grids)
            if (MODE == MODE_APPLY) {
                st1<NT>(dir ? (T)0 : q, a.q + id);
            } else if (MODE == MODE_INIT) {
                const T rv = dir ? (T)0 : xa_cur[r] - q;
                st1<NT>(rv, a.r + id);
                const T z = xb_cur[r] * rv;
                if (a.p_init) st1<NT>(z, a.p1 + id);   // p_0 for MODE_PASSA0
                acc0 += (double)rv * (double)z;
                acc1 += (double)rv * (double)rv;
            } else {
                const T pc = sv[s1][lj][li];
                const T qv = dir ? (T)0 : q;
                if (MODE == MODE_PASSA) st1<NT>(pc, pout + id);
                st1<NT>(qv, a.q + id);
                if (MODE == MODE_PASSA && !first) st1<NT>(xa_cur[r] + alpha_prev * pold_cur[r], a.x + id);
                acc0 += (double)pc * (double)qv;
            }
        }
    };

    if (PF == 1) {
        for (int k = k0; k < k1; ++k) step(SA, k);
    } else {
        for (int k = k0; k < k1; k += 2) {
            step(SA, k);
            if (k + 1 < k1) step(SB, k + 1);
        }
    }

    if (MODE == MODE_APPLY) return;

    // block partials, plain stores: a one-block kernel takes the totals
    double acc[2] = {acc0, acc1};
    block_sum<2, NTv>(acc, red);
    if (tid == 0) {
        double *out = (MODE == MODE_INIT && a.fold) ? a.partials2 : a.partials;
        out[2 * (int64_t)blockIdx.x] = acc[0];
        if (MODE == MODE_INIT) out[2 * (int64_t)blockIdx.x + 1] = acc[1];
    }
}

// Block shape per instantiation: TYv rows of TX threads, RYv node rows per
// thread (TYv * RYv == TYT, so every shape tiles the plane alike and the host's
// tile counts and partial slots do not depend on it), WPE waves per SIMD.  The
// grid's size picks the form of the body.
template <typename T, int MODE, int TYv, int RYv, int WPE>
__global__ void __launch_bounds__(TX * TYv, WPE) k_stencil(const StencilArgs<T> a) {
    __shared__ StencilLds<T, TYv> lds;
    if (a.g.nnodes >= STREAM_MIN_NODES) stencil_body<T, MODE, TYv, RYv, true>(a, lds);
    else stencil_body<T, MODE, TYv, RYv, false>(a, lds);
}

// Totals of the stencil pass's nb block partials (fixed order), then the
// scalar step: init sets rho = r.z, ||r||^2 and the first stop test; pass A
// sets p.q and alpha = rho / p.q (or flags a breakdown).
template <int MODE>
__global__ void __launch_bounds__(NTF) k_stencil_finish(JcgScalars *sc, const double *__restrict__ partials, int nb) {
    __shared__ double red[2][NTF / 64];
    if (MODE != MODE_INIT && sc->done) return;
    double tot[2] = {0.0, 0.0};
    if (MODE == MODE_INIT) {
        sum_partials<2>(partials, nb, tot, red);
    } else {
        double t1[1];
        sum_partials<1>(partials, nb, t1, red);
        tot[0] = t1[0];
    }
    if (threadIdx.x != 0) return;
    if (MODE == MODE_INIT) {
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
    } else {
        const double pq = tot[0];
        sc->pq = pq;
        sc->pending = 0;
        if (!(pq > 0.0) || !isfinite(pq)) sc->done = DONE_BREAKDOWN;
        else sc->alpha = sc->rho / pq;
    }
}

// ---------------------------------------------------------------------------
// pass B: r -= alpha q; z = D^-1 r; r.z, r.r; stop test
// ---------------------------------------------------------------------------
// A streaming kernel in which every block takes one contiguous chunk of UB x NTB
// node pairs (16-byte accesses, non-temporal on grids of STREAM_MIN_NODES nodes
// or more; node arrays have an even length and 16-byte alignment) and stores
// its two partial sums, then a one-block kernel that sums
// the partials in block order and takes the scalar step.  Many short-lived
// blocks with contiguous chunks stream faster than a grid-stride loop, and
// plain partial stores avoid a device-scope fence and atomic per block.
constexpr int NTB = 256;
constexpr int UB = 4;

template <typename T, bool LAST, bool NT>
__device__ __forceinline__ void passB_body(const PassBArgs<T> &a) {
    __shared__ double red[2][NTB / 64];
    __shared__ double s_alpha;
    __shared__ int s_bad;
    JcgScalars *sc = a.sc;
    // never set during a pass B; folded, the check waits until the loads below
    // are issued (a launch after `done` then only reads, on a small grid)
    if (!a.fold && sc->done) return;
    using V2 = typename Vec2<T>::type;
    const int64_t n2 = a.n / 2;
    const V2 *__restrict__ r2 = (const V2 *)a.r;
    const V2 *__restrict__ q2 = (const V2 *)a.q;
    const V2 *__restrict__ d2 = (const V2 *)a.dinv;
    V2 *__restrict__ w2 = (V2 *)a.r;
    const int64_t base = (int64_t)blockIdx.x * (UB * NTB) + threadIdx.x;
    V2 rv[UB], qv[UB], dv[UB];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
        const int64_t i = base + u * NTB;
        if (i < n2) {
            rv[u] = ld2<NT>(r2 + i);
            qv[u] = ld2<NT>(q2 + i);
            if (!LAST) dv[u] = ld2<NT>(d2 + i);
        }
    }
    T al;
    if (a.fold) {
        // folded: alpha = rho_it / p.q from pass A's partials (every block the
        // same sum, while its own loads are in flight); a breakdown goes to
        // `brk`, which the next pass A turns into `done`
        const int dn = sc->done;
        const double rho_it = sc->rho_f[a.it & 1];
        double t[1] = {0.0};
        for (int b = threadIdx.x; b < a.nb_a; b += NTB) t[0] += a.pq_partials[2 * b];
        if (dn) return;                           // uniform: no pass B writes it
        block_sum<1, NTB>(t, red);
        if (threadIdx.x == 0) {
            const double pq = t[0];
            const bool bad = !(pq > 0.0) || !isfinite(pq);
            const double alpha = bad ? 0.0 : rho_it / pq;
            if (blockIdx.x == 0) {
                sc->pq = pq;
                if (bad) sc->brk = 1;
                else sc->alpha = alpha;
            }
            s_alpha = alpha;
            s_bad = bad;
        }
        __syncthreads();
        if (s_bad) return;
        al = (T)s_alpha;
    } else {
        al = (T)sc->alpha;
    }
    double rz = 0.0, rr = 0.0;
#pragma unroll
    for (int u = 0; u < UB; ++u) {
        const int64_t i = base + u * NTB;
        if (i < n2) {
            V2 x;
            x.x = rv[u].x - al * qv[u].x;
            x.y = rv[u].y - al * qv[u].y;
            if (!LAST) {
                st2<NT>(x, w2 + i);
                const T z0 = dv[u].x * x.x, z1 = dv[u].y * x.y;
                rz += (double)x.x * (double)z0 + (double)x.y * (double)z1;
            }
            rr += (double)x.x * (double)x.x + (double)x.y * (double)x.y;
        }
    }
    double acc[2] = {rz, rr};
    block_sum<2, NTB>(acc, red);
    if (threadIdx.x == 0) {
        a.partials[2 * (int64_t)blockIdx.x] = acc[0];
        a.partials[2 * (int64_t)blockIdx.x + 1] = acc[1];
    }
}

template <typename T, bool LAST>
__global__ void __launch_bounds__(NTB) k_passB(const PassBArgs<T> a) {
    if (a.n >= STREAM_MIN_NODES) passB_body<T, LAST, true>(a);
    else passB_body<T, LAST, false>(a);
}

// Totals of pass B's nb block partials (fixed order), then beta, rho, ||r||^2
// and the stop test.
__global__ void __launch_bounds__(NTF) k_passB_finish(JcgScalars *sc, const double *__restrict__ partials, int nb) {
    __shared__ double red[2][NTF / 64];
    if (sc->done) return;
    double tot[2];
    sum_partials<2>(partials, nb, tot, red);
    if (threadIdx.x == 0) {
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

// x += alpha p of the last iteration (after the host has seen `done`, or
// enqueued right behind the iterations): one contiguous chunk of UB x 256 node
// pairs per block, 16-byte accesses.  Thread 0 of block 0 also copies the
// final scalars to `out` (pinned host memory, read by the host once the stream
// has passed this launch).
template <typename T, bool NT>
__device__ __forceinline__ void final_x_body(int64_t n, T *x, const T *p0, const T *p1, const JcgScalars *sc) {
    using V2 = typename Vec2<T>::type;
    const T al = (T)sc->alpha;
    const V2 *__restrict__ p = (const V2 *)((sc->iter & 1) ? p1 : p0);
    V2 *__restrict__ x2 = (V2 *)x;
    const int64_t n2 = n / 2;
    const int64_t base = (int64_t)blockIdx.x * (UB * 256) + threadIdx.x;
    V2 xv[UB], pv[UB];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
        const int64_t i = base + u * 256;
        if (i < n2) {
            xv[u] = ld2<NT>(x2 + i);
            pv[u] = ld2<NT>(p + i);
        }
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
        const int64_t i = base + u * 256;
        if (i < n2) {
            xv[u].x += al * pv[u].x;
            xv[u].y += al * pv[u].y;
            st2<NT>(xv[u], x2 + i);
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_final_x(int64_t n, T *x, const T *p0, const T *p1, const JcgScalars *sc,
                                                 JcgScalars *out) {
    static_assert(sizeof(JcgScalars) % 8 == 0, "scalars copied as 8-byte words");
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // system-scope stores: the words reach host memory without an L2 write-back
        const unsigned long long *src = (const unsigned long long *)sc;
        unsigned long long *dst = (unsigned long long *)out;
        for (int w = 0; w < (int)(sizeof(JcgScalars) / 8); ++w)
            __hip_atomic_store(dst + w, src[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    if (!sc->pending) return;
    if (n >= STREAM_MIN_NODES) final_x_body<T, true>(n, x, p0, p1, sc);
    else final_x_body<T, false>(n, x, p0, p1, sc);
}

// Pass A of iteration it >= 1 split for the column stencil (the grids too
// large for folded scalars): the node-wise part, the search direction
// p = D^-1 r + beta p_old and the previous iteration's x += alpha p_old, with
// the same roundings as the fused tiled pass A; the column kernel then forms
// q = A p and p.q.  One contiguous chunk of UB x 256 node pairs per block,
// 16-byte accesses over the whole array (padding entries are zero in every
// input and stay zero).
template <bool NT>
__device__ __forceinline__ void p_update_body(int64_t n, const double *__restrict__ dinv,
                                              const double *__restrict__ r, double *p0, double *p1, double *x,
                                              const JcgScalars *sc) {
    const int it = sc->iter;
    const double bk = sc->beta, al = sc->alpha;
    const bool first = it == 0;
    const double2 *__restrict__ pin = (const double2 *)((it & 1) ? p1 : p0);
    double2 *__restrict__ pout = (double2 *)((it & 1) ? p0 : p1);
    const double2 *__restrict__ d2 = (const double2 *)dinv;
    const double2 *__restrict__ r2 = (const double2 *)r;
    double2 *__restrict__ x2 = (double2 *)x;
    const int64_t n2 = n / 2;
    const int64_t base = (int64_t)blockIdx.x * (UB * 256) + threadIdx.x;
    double2 dv[UB], rv[UB], pv[UB], xv[UB];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
        const int64_t i = base + u * 256;
        if (i < n2) {
            dv[u] = ld2<NT>(d2 + i);
            rv[u] = ld2<NT>(r2 + i);
            if (!first) {
                pv[u] = ld2<NT>(pin + i);
                xv[u] = ld2<NT>(x2 + i);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
        const int64_t i = base + u * 256;
        if (i < n2) {
            double2 pn;
            const double z0 = dv[u].x * rv[u].x, z1 = dv[u].y * rv[u].y;
            pn.x = first ? z0 : z0 + bk * pv[u].x;
            pn.y = first ? z1 : z1 + bk * pv[u].y;
            st2<NT>(pn, pout + i);
            if (!first) {
                double2 xn;
                xn.x = xv[u].x + al * pv[u].x;
                xn.y = xv[u].y + al * pv[u].y;
                st2<NT>(xn, x2 + i);
            }
        }
    }
}

__global__ void __launch_bounds__(256) k_p_update(int64_t n, const double *__restrict__ dinv,
                                                  const double *__restrict__ r, double *p0, double *p1, double *x,
                                                  const JcgScalars *sc) {
    if (sc->done) return;                         // uniform over the grid
    if (n >= STREAM_MIN_NODES) p_update_body<true>(n, dinv, r, p0, p1, x, sc);
    else p_update_body<false>(n, dinv, r, p0, p1, x, sc);
}

// The same node-wise part of pass A for the gather levels, whose scalar steps
// are folded: iteration `it` (a launch argument) first takes the scalar step
// of the pass before (init at it = 0, pass B after): every block sums that
// pass's fold_nb partial pairs in one fixed order, then the stop test and
// beta = rho_it / rho_{it-1}; block 0 stores the scalars (as the folded
// tiled pass A does).  While running, it >= 1 forms p and x += alpha p_old;
// at it = 0 init has stored p_0 already.
template <bool NT>
__device__ __forceinline__ void p_update_fold_body(const PUFoldArgs &a) {
    __shared__ double red[2][4];
    __shared__ double s_beta;
    __shared__ int s_flag;
    JcgScalars *sc = a.sc;
    const int it = a.it, tid = threadIdx.x;
    // the scalars the step reads; `done` (which block 0 may set in this
    // launch) only through thread 0 and LDS
    const int f_done = sc->done, f_brk = sc->brk, f_fixed = sc->fixed, f_maxit = sc->max_iter;
    const double f_tol = sc->tol, f_alpha = sc->alpha;
    const double f_rho_prev = it > 0 ? sc->rho_f[(it - 1) & 1] : 1.0;
    double ft[2] = {0.0, 0.0};
    for (int b = tid; b < a.fold_nb; b += 256) {
        ft[0] += a.partials[2 * b];
        ft[1] += a.partials[2 * b + 1];
    }
    // the vector loads (iterations >= 1) in flight during the scalar step
    const bool first = it == 0;
    const double2 *__restrict__ pin = (const double2 *)((it & 1) ? a.p1 : a.p0);
    double2 *__restrict__ pout = (double2 *)((it & 1) ? a.p0 : a.p1);
    const double2 *__restrict__ d2 = (const double2 *)a.dinv;
    const double2 *__restrict__ r2 = (const double2 *)a.r;
    double2 *__restrict__ x2 = (double2 *)a.x;
    const int64_t n2 = a.n / 2;
    const int64_t base = (int64_t)blockIdx.x * (UB * 256) + tid;
    double2 dv[UB], rv[UB], pv[UB], xv[UB];
    if (!first) {
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const int64_t i = base + u * 256;
            if (i < n2) {
                dv[u] = ld2<NT>(d2 + i);
                rv[u] = ld2<NT>(r2 + i);
                pv[u] = ld2<NT>(pin + i);
                xv[u] = ld2<NT>(x2 + i);
            }
        }
    }
    if (tid == 0) s_flag = f_done ? -1 : (f_brk ? -2 : 0);
    __syncthreads();
    const int pre = s_flag;
    if (pre == -1) return;                        // stopped by an earlier launch
    block_sum<2, 256>(ft, red);
    if (tid == 0) {
        int dn;
        double bk = 0.0;
        if (pre == -2) {
            dn = DONE_BREAKDOWN;                  // the previous pass B found p.q <= 0
        } else {
            const double rz = ft[0], rr = ft[1], rn = sqrt(rr);
            if (f_fixed >= 0) dn = (it >= f_fixed) ? DONE_CONVERGED : DONE_RUNNING;
            else if (!(rn > f_tol)) dn = DONE_CONVERGED;
            else if (it >= f_maxit) dn = DONE_MAXITER;
            else dn = DONE_RUNNING;
            if (it > 0) bk = rz / f_rho_prev;
            if (blockIdx.x == 0) {
                sc->iter = it;
                sc->rho = rz;
                sc->rho_f[it & 1] = rz;
                sc->rr = rr;
                sc->beta = bk;
                // stopping after a pass B leaves that iteration's x update
                sc->pending = (dn != DONE_RUNNING && it > 0) ? 1 : 0;
            }
        }
        if (blockIdx.x == 0 && dn != DONE_RUNNING) sc->done = dn;
        s_beta = bk;
        s_flag = dn;
    }
    __syncthreads();
    if (s_flag != DONE_RUNNING || first) return;
    const double bk = s_beta;
#pragma unroll
    for (int u = 0; u < UB; ++u) {
        const int64_t i = base + u * 256;
        if (i < n2) {
            double2 pn, xn;
            const double z0 = dv[u].x * rv[u].x, z1 = dv[u].y * rv[u].y;
            pn.x = z0 + bk * pv[u].x;
            pn.y = z1 + bk * pv[u].y;
            st2<NT>(pn, pout + i);
            xn.x = xv[u].x + f_alpha * pv[u].x;
            xn.y = xv[u].y + f_alpha * pv[u].y;
            st2<NT>(xn, x2 + i);
        }
    }
}

__global__ void __launch_bounds__(256) k_p_update_fold(const PUFoldArgs a) {
    if (a.n >= STREAM_MIN_NODES) p_update_fold_body<true>(a);
    else p_update_fold_body<false>(a);
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
        sc->brk = 0;
        sc->rho_f[0] = sc->rho_f[1] = 0.0;
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

int stencil_kz(const Geom &g, int kz_max, int target_blocks) {
    // Planes per z-chunk: long chunks amortise the two halo planes, but small
    // grids need short chunks so that enough blocks run concurrently (the
    // planes of one chunk are processed in sequence by one block).  At least 4:
    // below that the halo planes dominate and the extra blocks of a small grid
    // queue behind each other instead of overlapping.
    const int64_t tiles = (int64_t)((g.sx + TX - 1) / TX) * ((g.sy + TYT - 1) / TYT);
    int64_t kz = tiles * (g.nz + 1) / std::max(1, target_blocks);
    if (kz < 4) kz = 4;
    if (kz > kz_max) kz = kz_max;
    if (kz > g.nz + 1) kz = g.nz + 1;
    return (int)std::max<int64_t>(kz, 1);
}

// Block shape of pass A's iteration 0: it reads only p_0 and beta, so a z-step
// carries little work for its memory latency; 256-thread blocks with two node
// rows per thread at 2 waves per SIMD (164 registers, no spills) run it 8-11 %
// faster on 513^3 than the 512-thread shape the other passes use (for them the
// same shape was measured slower).
#ifndef ECMG_PA0_TY
#define ECMG_PA0_TY 4
#endif
#ifndef ECMG_PA0_RY
#define ECMG_PA0_RY 2
#endif
#ifndef ECMG_PA0_WPE
#define ECMG_PA0_WPE 2
#endif

template <typename T>
void launch_stencil(int mode, const StencilArgs<T> &a, hipStream_t s) {
    const int nb = a.ntx * a.nty * a.nkz;
    if (mode == MODE_APPLY) {
        launch_timed(k_stencil<T, MODE_APPLY, TY, RY, STENCIL_WAVES_PER_EU>, dim3(nb), dim3(NT), 0, s, a);
    } else if (mode == MODE_INIT) {
        launch_timed(k_stencil<T, MODE_INIT, TY, RY, STENCIL_WAVES_PER_EU>, dim3(nb), dim3(NT), 0, s, a);
        if (!a.fold)
            hipLaunchKernelGGL(k_stencil_finish<MODE_INIT>, dim3(1), dim3(NTF), 0, s, a.sc,
                               (const double *)a.partials, nb);
    } else {
        if (mode == MODE_PASSA0)
            launch_timed(k_stencil<T, MODE_PASSA0, ECMG_PA0_TY, ECMG_PA0_RY, ECMG_PA0_WPE>, dim3(nb),
                         dim3(TX * ECMG_PA0_TY), 0, s, a);
        else
            launch_timed(k_stencil<T, MODE_PASSA, TY, RY, STENCIL_WAVES_PER_EU>, dim3(nb), dim3(NT), 0, s, a);
        if (!a.fold)
            hipLaunchKernelGGL(k_stencil_finish<MODE_PASSA>, dim3(1), dim3(NTF), 0, s, a.sc,
                               (const double *)a.partials, nb);
    }
}

void launch_stencil_finish(int mode, JcgScalars *sc, const double *partials, int nb, hipStream_t s) {
    if (mode == MODE_INIT) hipLaunchKernelGGL(k_stencil_finish<MODE_INIT>, dim3(1), dim3(NTF), 0, s, sc, partials, nb);
    else hipLaunchKernelGGL(k_stencil_finish<MODE_PASSA>, dim3(1), dim3(NTF), 0, s, sc, partials, nb);
}

int64_t passB_blocks(int64_t n) { return std::max<int64_t>(1, (n / 2 + UB * NTB - 1) / (UB * NTB)); }

template <typename T>
void launch_passB(const PassBArgs<T> &a, hipStream_t s) {
    const int64_t nb = passB_blocks(a.n);
    if (a.last && !a.fold) launch_timed(k_passB<T, true>, dim3((unsigned)nb), dim3(NTB), 0, s, a);
    else launch_timed(k_passB<T, false>, dim3((unsigned)nb), dim3(NTB), 0, s, a);
    if (!a.fold) hipLaunchKernelGGL(k_passB_finish, dim3(1), dim3(NTF), 0, s, a.sc, (const double *)a.partials, (int)nb);
}

void launch_final_x(const Geom &g, double *x, const double *p0, const double *p1, const JcgScalars *sc,
                    JcgScalars *out, hipStream_t s, bool update) {
    const int64_t n = update ? g.nnodes : 0;
    const int64_t nb = std::max<int64_t>(1, (n / 2 + UB * 256 - 1) / (UB * 256));
    hipLaunchKernelGGL((k_final_x<double>), dim3((unsigned)nb), dim3(256), 0, s, n, x, p0, p1, sc, out);
}

void launch_p_update(const Geom &g, const double *dinv, const double *r, double *p0, double *p1, double *x,
                     const JcgScalars *sc, hipStream_t s) {
    const int64_t nb = std::max<int64_t>(1, (g.nnodes / 2 + UB * 256 - 1) / (UB * 256));
    launch_timed_first(k_p_update, dim3((unsigned)nb), dim3(256), 0, s, g.nnodes, dinv, r, p0, p1, x, sc);
}

void launch_p_update_fold(const PUFoldArgs &a, hipStream_t s) {
    const int64_t nb = std::max<int64_t>(1, (a.n / 2 + UB * 256 - 1) / (UB * 256));
    launch_timed_first(k_p_update_fold, dim3((unsigned)nb), dim3(256), 0, s, a);
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

// ---------------------------------------------------------------------------
// mixed precision (outer FP64 residual / iterative refinement around an FP32
// JCG on the correction)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(NTB) k_mixed_start(int64_t n, const double *r64, double inv_s, const float *dinv32,
                                                     float *r32, float *d32, JcgScalars *sc, double *partials,
                                                     unsigned *counter) {
    __shared__ double red[2][NTB / 64];
    __shared__ int s_last;
    const int64_t stride = (int64_t)gridDim.x * NTB;
    double rz = 0.0, rr = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NTB + threadIdx.x; i < n; i += stride) {
        const float rv = (float)(r64[i] * inv_s);
        r32[i] = rv;
        d32[i] = 0.0f;
        const float z = dinv32[i] * rv;
        rz += (double)rv * (double)z;
        rr += (double)rv * (double)rv;
    }
    double acc[2] = {rz, rr}, tot[2];
    if (last_block_total<2, NTB>(acc, red, &s_last, partials, counter, blockIdx.x, gridDim.x, tot) &&
        threadIdx.x == 0) {
        sc->rho = tot[0];
        sc->rr = tot[1];
        sc->iter = 0;
        sc->alpha = 0.0;
        sc->beta = 0.0;
        sc->pending = 0;
        const double rn = sqrt(tot[1]);
        if (!(rn > sc->tol)) sc->done = DONE_CONVERGED;
        else sc->done = (sc->max_iter <= 0) ? DONE_MAXITER : DONE_RUNNING;
    }
}

__global__ void k_mixed_update(int64_t n, int sx, int width, double *x, double s, const float *d32, const float *p0,
                               const float *p1, const JcgScalars *sc) {
    const float al = sc->pending ? (float)sc->alpha : 0.0f;
    const float *p = (sc->iter & 1) ? p1 : p0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        if ((int)(i % sx) < width) x[i] += s * (double)(d32[i] + al * p[i]);
}

__global__ void k_to_f32(const double *a, float *b, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) b[i] = (float)a[i];
}

void launch_mixed_start(const Geom &g, const double *r64, double inv_s, const float *dinv32, float *r32, float *d32,
                        JcgScalars *sc, double *partials, unsigned *counter, hipStream_t s) {
    launch_timed(k_mixed_start, dim3(reduce_blocks(g.nnodes)), dim3(NTB), 0, s, g.nnodes, r64, inv_s, dinv32,
                       r32, d32, sc, partials, counter);
}

void launch_mixed_update(const Geom &g, double *x, double sc_s, const float *d32, const float *p0, const float *p1,
                         const JcgScalars *sc, hipStream_t s) {
    const int64_t nb = std::min<int64_t>((g.nnodes + 255) / 256, 8192);
    launch_timed(k_mixed_update, dim3(nb), dim3(256), 0, s, g.nnodes, g.sx, g.nx + 1, x, sc_s, d32, p0, p1, sc);
}

void launch_to_f32(const double *a, float *b, int64_t n, hipStream_t s) {
    const int64_t nb = std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192));
    hipLaunchKernelGGL(k_to_f32, dim3(nb), dim3(256), 0, s, a, b, n);
}

template void launch_stencil<double>(int, const StencilArgs<double> &, hipStream_t);
template void launch_passB<double>(const PassBArgs<double> &, hipStream_t);
template void launch_stencil<float>(int, const StencilArgs<float> &, hipStream_t);
template void launch_passB<float>(const PassBArgs<float> &, hipStream_t);

}  // namespace ecmg
