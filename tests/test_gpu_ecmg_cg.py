"""GPU: ECMG_cg (Algorithm 4 with plain CG, Section 4.1) and the original ECMG
of Algorithm 3 (fixed counts of eq. ee), both through the C ABI with
options.method = ECMG_CG, against the oracle and the paper's ECMG_cg column."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ecmg():
    import paper_1506_02983_amd as E
    E.load_library()
    return E


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("persistent", [300000, 0], ids=["persistent", "tiled"])
@pytest.mark.parametrize("eps,paper", [(1e-8, [58, 82]), (1e-10, [76, 124])], ids=["eps1e-8", "eps1e-10"])
def test_ecmg_cg_paper_counts_and_oracle(orc, ecmg, persistent, eps, paper):
    """Section 5, Problem 1, Tables iterations8 and iterations10 (ECMG_cg
    column): the GPU takes the paper's counts, and its iterates match the
    oracle's CG on every level."""
    p = workloads.paper_problem1(levels=4, eps=eps)
    ref = orc.cascade(p, variant=orc.LAGRANGE27, method=orc.CG_METHOD, errors=False)
    with ecmg.Solver(interp=ecmg.LAGRANGE27, method=ecmg.CG, persistent_nodes=persistent) as s:
        s.setup(p)
        infos = s.solve(eps)
        got = [i["iters"] for i in infos]
        u = [s.get(l, ecmg.VEC_U) for l in range(p.levels)]
        minv = s.get(p.levels - 1, ecmg.VEC_DINV)
    assert got[2:] == paper == [r.iters for r in ref[2:]], (got, paper)
    d = [_rel(u[l], ref[l].u) for l in range(p.levels)]
    print("ECMG_cg eps %g: iterate differences per level %s" % (eps, d))
    assert max(d) <= 1e-12, d
    # M^-1 of plain CG: 1 on free nodes, 0 on Dirichlet nodes
    assert set(np.unique(minv).tolist()) <= {0.0, 1.0}


@pytest.mark.parametrize("method", ["cg", "jcg"])
def test_algorithm3_fixed_schedule(orc, ecmg, method):
    """Algorithm 3: EXP_finite then m_j = 4 * 4^(L-j) CG steps per grid (no
    stopping test); the same schedule under JCG for comparison."""
    p = workloads.variable_beta_robin_cube(levels=5)
    sched = ecmg.cascadic_schedule(p.levels, 4, 4.0)
    assert sched == [0, 0, 64, 16, 4]
    m_orc = orc.CG_METHOD if method == "cg" else orc.JCG_METHOD
    ref = orc.cascade(p, fixed_iters=sched, method=m_orc, errors=False)
    with ecmg.Solver(method=ecmg.CG if method == "cg" else ecmg.JCG, persistent_nodes=0) as s:
        s.setup(p)
        infos = s.solve_fixed(sched)
        u = [s.get(l, ecmg.VEC_U) for l in range(p.levels)]
    assert [i["iters"] for i in infos[2:]] == sched[2:]
    d = [_rel(u[l], ref[l].u) for l in range(p.levels)]
    print("Algorithm 3 (%s): iterate differences per level %s" % (method, d))
    assert max(d) <= 1e-12, d


def test_unknown_method_is_rejected(ecmg):
    with pytest.raises(ecmg.EcmgError):
        ecmg.Solver(method=7)
