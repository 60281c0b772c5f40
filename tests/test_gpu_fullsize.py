"""Parity at the benchmark's full sizes, in the configuration bench.py times
(device-sampled fields, the same solver options, the autotuned per-level
configuration), on outputs the oracle can compute one by one:

* the operator (A u)_r at sampled rows of the finest level (tile edges, the
  ragged x-tail, z-chunk edges, faces, edges, corners, random rows) against the
  oracle's row-wise apply with its own coefficients;
* EXP_finite (raw W) and EXP_true at sampled nodes against the oracle's
  point-wise formulas applied to the GPU's own coarse-level solutions;
* the two DSOLVE levels against the oracle's direct solve;
* properties at any size: g_D on Dirichlet nodes to a few ulps, the reported relative
  residual below eps on every JCG level, and (smooth solution) the FE error of
  the finest level at least halving from the next coarser level."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

CASES = {
    "variable-beta-robin-513": lambda: workloads.variable_beta_robin_cube(levels=7, eps=1e-8),
    "high-contrast-513x257x257": lambda: workloads.high_contrast_singular_box(levels=6, eps=1e-8),
}


@pytest.fixture(scope="module")
def ecmg():
    import paper_1506_02983_amd as E
    E.load_library()
    return E


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _sample(n, rng, extra=2000):
    """Dense node indices: boundary, tile and chunk edges, the ragged tail, random."""
    def marks(m, edges):
        s = {0, 1, 2, m - 2, m - 1, m}
        for e in edges:
            for d in (-1, 0, 1):
                if 0 <= e + d <= m:
                    s.add(e + d)
        return sorted(s)
    xs = marks(n[0], range(64, n[0] + 1, 64))[::3] + [n[0]]
    ys = marks(n[1], range(16, n[1] + 1, 16))[::5] + [n[1]]
    zs = marks(n[2], range(32, n[2] + 1, 32))[::5] + [n[2]]
    ii, jj, kk = np.meshgrid(np.array(sorted(set(xs))), np.array(sorted(set(ys))), np.array(sorted(set(zs))),
                             indexing="ij")
    pts = (ii + (n[0] + 1) * (jj + (n[1] + 1) * kk)).ravel()
    rnd = rng.integers(0, (n[0] + 1) * (n[1] + 1) * (n[2] + 1), size=extra)
    return np.unique(np.concatenate([pts, rnd])).astype(np.int64)


@pytest.mark.parametrize("name", sorted(CASES))
def test_fullsize_sampled_parity(orc, ecmg, name):
    p = CASES[name]()
    L = p.levels - 1
    n = p.n_at(L)
    rng = np.random.default_rng(11)
    with ecmg.Solver(keep_w=True) as s:
        s.setup(p, device_fields=True)
        # the configuration bench.py times: a warm-up solve, then the autotuner
        # over each level's iteration count
        s.solve(p.eps)
        tuned = s.autotune(iters=0)
        print("fullsize %s: tuned %s" % (name, [(r["level"], r["path"], r["kz"]) for r in tuned]), flush=True)
        infos = s.solve(p.eps)
        print("fullsize %s: iterations %s" % (name, [i["iters"] for i in infos]), flush=True)
        for l in range(2, p.levels):
            assert infos[l]["status"] == 0 and infos[l]["rre"] <= p.eps, infos[l]
        s.extrapolate(L, out=False)
        u = {l: s.get(l, ecmg.VEC_U) for l in (0, 1, L - 2, L - 1, L)}
        W = s.get(L, ecmg.VEC_W)
        Ut = s.get(L, ecmg.VEC_UTILDE)
        Au = s.apply(L, u[L])
        dinv = s.get(L, ecmg.VEC_DINV)
    # DSOLVE levels against the oracle's direct solve
    for l in (0, 1):
        ref = orc.dsolve(orc.discretize(p, l))
        assert _rel(u[l], ref) <= 1e-12, (name, l, _rel(u[l], ref))
    pts = _sample(n, rng)
    print("fullsize %s: %d sampled nodes" % (name, pts.size), flush=True)
    # operator rows with the oracle's own coefficients
    grid = orc.grid_of(p, L)
    beta, alpha = orc.coefficients(p, grid)
    ref = orc.apply_rows(grid, beta, alpha, u[L], pts)
    # (A u)_r nearly cancels (it approximates the load, O(h^3)), so the bound is
    # set by the size of the summed terms: sum_j |A_rj||u_j| <= 2 D_r max|u|
    # (D_r the diagonal; the GPU's 1/D only sizes the tolerance here)
    free = dinv[pts] != 0.0
    assert np.all(Au[pts][~free] == 0.0) and np.all(ref[~free] == 0.0)
    tol = 1e-14 * 2.0 * np.abs(u[L]).max() / dinv[pts][free]
    err = np.abs(Au[pts][free] - ref[free])
    assert np.all(err <= tol), (name, float((err / tol).max()))
    del beta, alpha
    # EXP_finite (raw, before g_D) and EXP_true from the GPU's coarse solutions
    wref = orc.exp_finite_points(n, u[L - 1], u[L - 2], pts)
    assert _rel(W[pts], wref) <= 1e-14, name
    tref = orc.exp_true_points(n, u[L], u[L - 1], pts)
    assert _rel(Ut[pts], tref) <= 1e-14, name
    # g_D on Dirichlet nodes (sampled): the fields are evaluated on the device
    # (its pow / atan2 / sin), so agreement is to a few ulps, not bitwise
    ue = orc.exact_nodes(p, grid)
    dmask = orc.dirichlet_mask(grid)
    dpts = pts[dmask[pts] == 1]
    assert dpts.size > 0
    assert np.all(np.abs(u[L][dpts] - ue[dpts]) <= 8 * np.finfo(np.float64).eps * np.abs(ue[dpts]) + 1e-300)
    # FE error of the finest level: O(h^2) from the next coarser level
    e_fine = float(np.abs(u[L] - ue).max())
    ue1 = orc.exact_nodes(p, orc.grid_of(p, L - 1))
    e_coarse = float(np.abs(u[L - 1] - ue1).max())
    print("fullsize %s: |U-u| %.3e (finest) %.3e (coarser), |U~-u| %.3e" %
          (name, e_fine, e_coarse, float(np.abs(Ut - ue).max())), flush=True)
    if name == "variable-beta-robin-513":       # smooth u: second order; r^(2/3) is singular
        assert e_fine <= 0.5 * e_coarse


@pytest.mark.parametrize("interp", ["serendipity", "lagrange"])
def test_exp_finite_wide_rows_against_points(orc, ecmg, interp):
    """EXP_finite on a grid whose element rows fill whole waves (257^3: 64 coarse
    elements per row, the form that stages each row through LDS): with zero JCG
    iterations u_L is EXP_finite's output with g_D on Dirichlet nodes, and W its
    raw form; both at sampled nodes (row ends, the Dirichlet x faces) against the
    oracle's point-wise formula on the GPU's own coarser solutions."""
    p = workloads.variable_beta_robin_cube(levels=6)
    L = p.levels - 1
    n = p.n_at(L)
    variant = ecmg.LAGRANGE27 if interp == "lagrange" else ecmg.SERENDIPITY20
    with ecmg.Solver(keep_w=True, interp=variant) as s:
        s.setup(p, device_fields=True)
        s.solve_fixed([0] * p.levels)
        u1, u0, uL = s.get(L - 1, ecmg.VEC_U), s.get(L - 2, ecmg.VEC_U), s.get(L, ecmg.VEC_U)
        W = s.get(L, ecmg.VEC_W)
    rng = np.random.default_rng(5)
    pts = _sample(n, rng, extra=4000)
    ovar = orc.LAGRANGE27 if interp == "lagrange" else orc.SERENDIPITY20
    wref = orc.exp_finite_points(n, u1, u0, pts, variant=ovar)
    assert _rel(W[pts], wref) <= 1e-14
    grid = orc.grid_of(p, L)
    dmask = orc.dirichlet_mask(grid)[pts] == 1
    assert dmask.any() and (~dmask).any()
    assert _rel(uL[pts][~dmask], wref[~dmask]) <= 1e-14
    ue = orc.exact_nodes(p, grid)[pts][dmask]
    assert np.all(np.abs(uL[pts][dmask] - ue) <= 8 * np.finfo(np.float64).eps * np.abs(ue) + 1e-300)
