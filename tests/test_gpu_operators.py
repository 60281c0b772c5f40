"""GPU parity of the single operators against the oracle on identical seeded
inputs: the matrix-free stencil (Section 2), the discretisation (load vector,
Jacobi diagonal, ||f_h||), EXP_finite (both interpolation forms) and EXP_true.

Tolerances follow from the arithmetic: each output is a sum of at most ~64
products of O(1) factors in a different order on the two sides, so the
difference is bounded by a few dozen units in the last place of the largest
term: 1e-14 relative to the largest magnitude involved."""
import itertools

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ecmg():
    import paper_1506_02983_amd as E
    E.load_library()
    return E


def _rel(a, b, scale=None):
    s = np.abs(b).max() if scale is None else scale
    return float(np.abs(a - b).max() / max(s, 1e-300))


def _mixed_problem(n0=(3, 2, 5), levels=3, faces=(0, 0, 1, 1, 1, 1), lo=(0.0, -0.5, 0.25), hi=(1.0, 0.7, 1.5)):
    p = workloads.variable_beta_robin_cube(levels=levels)
    return p.with_(n0=n0, lo=lo, hi=hi, face_type=faces, alpha=lambda x, y, z, face=-1: 1.0 + 0.5 * x * x + 0 * y * z)


@pytest.mark.parametrize("case", ["robin-var", "dirichlet", "anisotropic"])
def test_stencil_apply_parity(orc, ecmg, case):
    if case == "robin-var":
        p = _mixed_problem()
    elif case == "dirichlet":
        p = workloads.smooth_dirichlet_cube(levels=3)
    else:
        p = _mixed_problem(n0=(5, 2, 3), faces=(1, 0, 1, 0, 1, 1), lo=(0, 0, 0), hi=(3.0, 0.2, 0.9))
    with ecmg.Solver() as s:
        s.setup(p)
        for level in range(p.levels):
            lv = orc.discretize(p, level)
            v = workloads.random_vector(lv.grid.num_nodes, seed=100 + level)
            got = s.apply(level, v)
            want = orc.spmv(lv, v)
            assert _rel(got, want) <= 1e-14, (case, level)


def test_stencil_apply_all_face_masks(orc, ecmg):
    base = _mixed_problem(n0=(3, 4, 2), levels=2)
    for mask in itertools.product((0, 1), repeat=6):
        p = base.with_(face_type=mask)
        with ecmg.Solver() as s:
            s.setup(p)
            lv = orc.discretize(p, 1)
            v = workloads.random_vector(lv.grid.num_nodes, seed=7)
            assert _rel(s.apply(1, v), orc.spmv(lv, v)) <= 1e-14, mask


def test_stencil_multi_tile_ragged(orc, ecmg):
    """Grids spanning several 64 x 16 tiles and z-chunks with ragged tails."""
    p = _mixed_problem(n0=(35, 9, 17), levels=2, faces=(1, 0, 1, 1, 0, 1))
    with ecmg.Solver() as s:
        s.setup(p)
        for level in (0, 1):
            lv = orc.discretize(p, level)
            v = workloads.random_vector(lv.grid.num_nodes, seed=3)
            assert _rel(s.apply(level, v), orc.spmv(lv, v)) <= 1e-14


def test_discretisation_parity(orc, ecmg):
    p = _mixed_problem(n0=(4, 3, 2), levels=3, faces=(0, 1, 1, 0, 1, 1))
    with ecmg.Solver() as s:
        s.setup(p)
        for level in range(p.levels):
            lv = orc.discretize(p, level)
            F = s.get(level, ecmg.VEC_F)
            assert _rel(F, lv.F) <= 1e-14
            dinv = s.get(level, ecmg.VEC_DINV)
            want = np.where(lv.dmask == 1, 0.0, 1.0 / np.where(lv.D == 0, 1.0, lv.D))
            assert _rel(dinv, want) <= 1e-14
            u = s.get(level, ecmg.VEC_U)
            assert np.array_equal(u[lv.dmask == 1], lv.gD[lv.dmask == 1])


@pytest.mark.parametrize("variant", [0, 1])
def test_exp_finite_parity(orc, ecmg, variant):
    p = _mixed_problem(n0=(3, 2, 4), levels=4, faces=(0, 1, 0, 1, 1, 0))
    with ecmg.Solver(interp=variant) as s:
        s.setup(p)
        for level in (2, 3):
            n1, n0 = p.n_at(level - 1), p.n_at(level - 2)
            U1 = workloads.random_vector((n1[0] + 1) * (n1[1] + 1) * (n1[2] + 1), seed=level)
            U0 = workloads.random_vector((n0[0] + 1) * (n0[1] + 1) * (n0[2] + 1), seed=50 + level)
            s.set(level - 1, ecmg.VEC_U, U1)
            s.set(level - 2, ecmg.VEC_U, U0)
            s.prolongate(level)
            g = orc.grid_of(p, level)
            W = orc.exp_finite(g, U1, U0, variant)
            assert _rel(s.get(level, ecmg.VEC_W), W) <= 1e-14
            dm = orc.dirichlet_mask(g)
            gD = orc.discretize(p, level).gD
            x = s.get(level, ecmg.VEC_U)
            assert _rel(x, np.where(dm == 1, gD, W), np.abs(W).max()) <= 1e-14
            assert np.array_equal(x[dm == 1], gD[dm == 1])


def test_exp_true_parity(orc, ecmg):
    p = _mixed_problem(n0=(3, 5, 2), levels=3)
    with ecmg.Solver() as s:
        s.setup(p)
        for level in (1, 2):
            n1, n0 = p.n_at(level), p.n_at(level - 1)
            U1 = workloads.random_vector((n1[0] + 1) * (n1[1] + 1) * (n1[2] + 1), seed=level + 11)
            U0 = workloads.random_vector((n0[0] + 1) * (n0[1] + 1) * (n0[2] + 1), seed=level + 21)
            s.set(level, ecmg.VEC_U, U1)
            s.set(level - 1, ecmg.VEC_U, U0)
            got = s.extrapolate(level)
            want = orc.exp_true(orc.grid_of(p, level), U1, U0)
            assert _rel(got, want) <= 1e-14


def test_rhs_norm_parity(orc, ecmg):
    """||f_h|| of the stopping test: the relative residual reported after zero
    iterations is ||b - A x0|| / ||f_h||, checked through a JCG call that stops
    immediately (fixed_iters = 0)."""
    p = workloads.paper_problem3(levels=2)
    with ecmg.Solver() as s:
        s.setup(p)
        lv = orc.discretize(p, 1)
        s.set(1, ecmg.VEC_U, lv.gD)
        info = s.jcg(1, 1e-3, fixed_iters=0)
        assert info["nf"] == pytest.approx(lv.nf, rel=1e-14)
        assert info["rre"] == pytest.approx(lv.nb / lv.nf, rel=1e-13)
