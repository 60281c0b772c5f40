"""Pins the oracle's DSOLVE (banded Cholesky) and JCG against a dense direct
solve with numpy on grids of at most 5^3 elements, for every Dirichlet/Robin
face pattern, with and without a Robin coefficient."""
import itertools

import numpy as np
import pytest

import workloads


def _small(faces, alpha, n=(3, 4, 2), beta_var=True):
    p = workloads.variable_beta_robin_cube(levels=1)
    p = p.with_(n0=n, face_type=faces, alpha=workloads._const(alpha))
    if not beta_var:
        p = p.with_(beta=workloads._const(1.0))
    return p


MASKS = list(itertools.product((0, 1), repeat=6))


@pytest.mark.parametrize("mask", MASKS, ids=lambda m: "".join(map(str, m)))
def test_direct_and_jcg_vs_dense(orc, mask):
    alpha = 0.0 if sum(mask) % 2 else 1.3
    if all(t == 1 for t in mask) and alpha == 0.0:
        alpha = 0.8          # pure Neumann is singular; keep the problem well posed
    p = _small(mask, alpha)
    lv = orc.discretize(p, 0)
    A = lv.dense()
    free = lv.dmask == 0
    Aff = A[np.ix_(free, free)]
    assert np.allclose(Aff, Aff.T, atol=1e-14)
    assert np.linalg.eigvalsh(Aff)[0] > 0
    ref = lv.gD.copy()
    ref[free] = np.linalg.solve(Aff, lv.b[free])
    x = orc.dsolve(lv)
    scale = np.abs(ref).max()
    assert np.abs(x - ref).max() <= 1e-13 * scale
    jr = orc.jcg(lv, lv.gD.copy(), 1e-14)
    assert jr.status == 0
    assert np.abs(jr.x - ref).max() <= 1e-11 * scale
    assert jr.rre <= 1e-14


def test_jcg_energy_error_monotone(orc):
    """PCG minimises the A-norm error over growing Krylov spaces: it decreases
    monotonically."""
    p = _small((0, 1, 0, 1, 1, 0), 1.0, n=(5, 5, 5))
    lv = orc.discretize(p, 0)
    A = lv.dense()
    free = lv.dmask == 0
    xs = orc.dsolve(lv)
    prev = np.inf
    for k in range(0, 25):
        x = orc.jcg(lv, lv.gD.copy(), 0.0, fixed_iters=k).x
        e = (x - xs)[free]
        en = float(e @ A[np.ix_(free, free)] @ e)
        assert en <= prev * (1 + 1e-12)
        prev = en


def test_jcg_stops_before_first_step_when_converged(orc):
    """Algorithm 4 tests the residual before iterating: a converged start takes
    0 steps."""
    p = _small((0,) * 6, 0.0)
    lv = orc.discretize(p, 0)
    xs = orc.dsolve(lv)
    jr = orc.jcg(lv, xs, 1e-8)
    assert jr.iters == 0


def test_jcg_not_converged_status(orc):
    p = _small((0,) * 6, 0.0)
    lv = orc.discretize(p, 0)
    jr = orc.jcg(lv, lv.gD.copy(), 1e-14, max_iter=1)
    assert jr.status == -3 and jr.iters == 1


def test_stopping_norm_includes_dirichlet_rows(orc):
    """||f_h|| of the stopping test is the norm of b on free nodes and g_D on
    Dirichlet nodes (the system with Dirichlet identity rows)."""
    p = workloads.paper_problem3(levels=1)
    lv = orc.discretize(p, 0)
    want = np.sqrt(np.sum(lv.b[lv.dmask == 0] ** 2) + np.sum(lv.gD[lv.dmask == 1] ** 2))
    assert lv.nf == pytest.approx(want, rel=1e-14)
