"""GPU parity of JCG and the whole Algorithm 4 cascade against the oracle.

Fixed-iteration mode runs the oracle's per-level iteration counts on the GPU,
so both sides perform the same arithmetic steps in different summation orders;
the iterates must agree to 1e-12 relative in the max norm.  Normal mode must
reproduce the oracle's iteration counts and the paper's (Section 5 tables)."""
import json
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_tables.json")


@pytest.fixture(scope="module")
def ecmg():
    import paper_1506_02983_amd as E
    E.load_library()
    return E


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


# The JCG drivers: the whole-loop persistent kernel (forced on every grid it
# can take); with the scalar steps folded into the passes, the gather path
# (one thread per node for the stencils after a node-wise p / x update: what
# grids of up to 1,048,576 nodes use) and the tiled two-pass kernels (what the
# grids up to 4096 blocks per pass use beyond that); and the passes with
# one-block finishing kernels, forced here with fold_blocks = 0: by the column
# kernels (init, and pass A as the node-wise p / x update plus the column
# stencil: what the 257^3 and 513^3 grids use) or by the tiled kernels.
DRIVERS = {"persistent": dict(persistent_nodes=300000), "gather": dict(persistent_nodes=0),
           "tiled": dict(persistent_nodes=0, gather_nodes=0),
           "column-unfolded": dict(persistent_nodes=0, fold_blocks=0),
           "tiled-unfolded": dict(persistent_nodes=0, fold_blocks=0, columns=False)}


@pytest.mark.parametrize("driver", list(DRIVERS))
def test_jcg_fixed_iterations_single_level(orc, ecmg, driver):
    p = workloads.variable_beta_robin_cube(levels=3)
    lv = orc.discretize(p, 2)
    x0 = np.where(lv.dmask == 1, lv.gD, workloads.random_vector(lv.grid.num_nodes, seed=5))
    with ecmg.Solver(**DRIVERS[driver]) as s:
        s.setup(p)
        for k in (1, 2, 7, 25):
            s.set(2, ecmg.VEC_U, x0)
            info = s.jcg(2, 0.0, fixed_iters=k)
            ref = orc.jcg(lv, x0, 0.0, fixed_iters=k)
            assert info["iters"] == k
            assert _rel(s.get(2, ecmg.VEC_U), ref.x) <= 1e-12, k
            assert info["rre"] == pytest.approx(ref.rre, rel=1e-9)


# (problem, EXP_finite form, iterate parity bound).  The bound is 1e-12; for
# the paper's Problem 2 at eps = 1e-12 the iterates are converged to the level
# where two FP64 runs of the same cascade separate when only their summation
# order differs: the oracle against itself with reversed dot products and
# reversed row sums separates by 7.5e-13 (55 iterations) and 9.2e-13 (81), the
# GPU by 1.1e-12 and 1.3e-12, so its bound is 5e-12.  (The same experiment on
# the other cases, including the per-level schedule, ECMG_cg and Algorithm 3,
# separates by at most 3e-15, and their bound is 1e-12.)
CASES = {
    "smooth-dirichlet": lambda: (workloads.smooth_dirichlet_cube(levels=4), 0, 1e-12),
    "variable-beta-robin": lambda: (workloads.variable_beta_robin_cube(levels=4), 0, 1e-12),
    "paper-p2-lagrange": lambda: (workloads.paper_problem2(levels=4), 1, 5e-12),
    "singular-contrast": lambda: (workloads.high_contrast_singular_box(levels=3), 0, 1e-12),
}


@pytest.mark.parametrize("driver", list(DRIVERS))
def test_level_info_names_the_driver(ecmg, driver):
    """ecmg_level_info.path reports the kernels each level ran on."""
    p = workloads.variable_beta_robin_cube(levels=4)
    want = {"persistent": ecmg.PATH_PERSISTENT, "gather": ecmg.PATH_GATHER, "tiled": ecmg.PATH_TILED,
            "column-unfolded": ecmg.PATH_COLUMN, "tiled-unfolded": ecmg.PATH_TILED_UNFOLDED}[driver]
    with ecmg.Solver(**DRIVERS[driver]) as s:
        s.setup(p)
        infos = s.solve(1e-8)
    assert [i["path"] for i in infos] == [ecmg.PATH_DENSE] * 2 + [want] * (p.levels - 2)


@pytest.mark.parametrize("driver", list(DRIVERS))
@pytest.mark.parametrize("name", list(CASES))
def test_cascade_fixed_iterations(orc, ecmg, name, driver):
    """Every JCG driver (DRIVERS) with device-side stop control."""
    p, variant, bound = CASES[name]()
    ref = orc.cascade(p, variant=variant)
    iters = [r.iters for r in ref]
    rows = []
    with ecmg.Solver(interp=variant, **DRIVERS[driver]) as s:
        s.setup(p)
        s.solve_fixed(iters)
        for l in range(p.levels):
            row = {"level": l, "iters": iters[l], "u": _rel(s.get(l, ecmg.VEC_U), ref[l].u)}
            if l >= 2:
                row["W"] = _rel(s.get(l, ecmg.VEC_W), ref[l].W)
            if l >= 1:
                row["Ut"] = _rel(s.extrapolate(l), ref[l].Ut)
            rows.append(row)
    print(name, rows)
    for row in rows:
        for k in ("u", "W", "Ut"):
            if k in row:
                assert row[k] <= bound, (name, row)


@pytest.mark.parametrize("driver", list(DRIVERS))
@pytest.mark.parametrize("name", list(CASES))
def test_cascade_normal_mode(orc, ecmg, name, driver):
    p, variant, bound = CASES[name]()
    ref = orc.cascade(p, variant=variant)
    with ecmg.Solver(interp=variant, true_residual=True, **DRIVERS[driver]) as s:
        s.setup(p)
        infos = s.solve(p.eps)
        for l in range(2, p.levels):
            r = ref[l]
            # identical counts unless the oracle stopped within 0.1% of the threshold
            near = abs(r.rre / p.eps - 1.0) < 1e-3
            assert abs(infos[l]["iters"] - r.iters) <= (1 if near else 0), (name, l, infos[l]["iters"], r.iters)
            assert infos[l]["rre"] <= p.eps
            if infos[l]["iters"] == r.iters:
                assert _rel(s.get(l, ecmg.VEC_U), r.u) <= bound
                # the true residual ||F - A u|| / ||f_h|| of the final iterate
                # against the oracle's.  Iterates that agree to `bound` give
                # residuals that differ by about cond(A) * bound relative, so
                # this checks the quantity, not the rounding: 2 %.
                assert infos[l]["rre_true"] == pytest.approx(r.rre_true, rel=2e-2), (l, infos[l], r.rre_true)
            ue = orc.exact_nodes(p, orc.grid_of(p, l))
            e_max, e_l2 = s.norms(l, ecmg.VEC_U, minus=ue)
            assert e_max == pytest.approx(r.err["U_max"], rel=1e-3)
            assert e_l2 == pytest.approx(r.err["U_l2"], rel=1e-3)
            s.extrapolate(l)
            t_max, t_l2 = s.norms(l, ecmg.VEC_UTILDE, minus=ue)
            assert t_max == pytest.approx(r.err["Ut_max"], rel=1e-3)
            w_max, w_l2 = s.norms(l, ecmg.VEC_W, ecmg.VEC_U)
            assert w_l2 == pytest.approx(r.err["WU_l2"], rel=1e-3)


def test_paper_iteration_counts_on_gpu(ecmg):
    """Every iteration count of the golden tables, reproduced on the GPU with the
    paper's (27-node Lagrange) initial guess."""
    with open(GOLDEN) as fh:
        cases = json.load(fh)["cases"]
    for case in cases:
        mk = {1: workloads.paper_problem1, 2: workloads.paper_problem2, 3: workloads.paper_problem3}[case["problem"]]
        p = mk(levels=case["levels"], eps=case["eps"])
        with ecmg.Solver(interp=ecmg.LAGRANGE27) as s:
            s.setup(p)
            infos = s.solve(case["eps"])
            for row, info in zip(case["rows"], infos[2:]):
                assert info["iters"] == row["iters"], (case["cite"], row["mesh"], info["iters"])


@pytest.mark.parametrize("driver", list(DRIVERS))
def test_deterministic(ecmg, driver):
    p = workloads.variable_beta_robin_cube(levels=4)
    with ecmg.Solver(**DRIVERS[driver]) as s:
        s.setup(p)
        s.solve(p.eps)
        a = s.extrapolate()
        s.solve(p.eps)
        b = s.extrapolate()
        assert np.array_equal(a, b)


@pytest.mark.parametrize("persistent", [300000, 0], ids=["persistent", "tiled"])
def test_not_converged_and_errors(ecmg, persistent):
    p = workloads.smooth_dirichlet_cube(levels=3)
    with ecmg.Solver(max_iter=1, persistent_nodes=persistent) as s:
        s.setup(p)
        infos = s.solve(1e-12, allow_fail=True)
        assert infos[2]["status"] == ecmg.ENOTCONV and infos[2]["iters"] == 1
    with ecmg.Solver() as s:
        with pytest.raises(ecmg.EcmgError) as e:
            s.solve(1e-8)
        assert e.value.code == ecmg.ESTATE
        bad = p.with_(beta=lambda x, y, z, face=-1: -1.0 + 0 * x * y * z)
        with pytest.raises(ecmg.EcmgError) as e:
            s.setup(bad)
        assert e.value.code == ecmg.EINVAL


def test_dsolve_dense_matches_jcg_dsolve(orc, ecmg):
    """The direct DSOLVE (explicit inverse of A_FF) and the FP64-JCG DSOLVE give
    the same coarse solutions and the same cascade (both are held to the
    oracle's banded Cholesky above)."""
    p = workloads.variable_beta_robin_cube(levels=4)
    out = {}
    for dense in (8192, 0):
        with ecmg.Solver(dsolve_dense_max=dense) as s:
            s.setup(p)
            infos = s.solve(1e-10)
            out[dense] = ([i["iters"] for i in infos], [s.get(l, ecmg.VEC_U) for l in range(p.levels)])
    assert out[8192][0][:2] == [0, 0] and min(out[0][0][:2]) > 0
    assert out[8192][0][2:] == out[0][0][2:]
    for l in range(p.levels):
        assert _rel(out[8192][1][l], out[0][1][l]) <= 1e-12, l
    ref = orc.dsolve(orc.discretize(p, 1))
    assert _rel(out[8192][1][1], ref) <= 1e-12


@pytest.mark.parametrize("driver", list(DRIVERS))
def test_per_level_tolerance_schedule(orc, ecmg, driver):
    """ecmg_solve_levels with a schedule tightened towards the finest grid
    takes the oracle's per-level iteration counts and iterates."""
    p = workloads.variable_beta_robin_cube(levels=5)
    sched = ecmg.tolerance_schedule(p.levels, 1e-11, 16.0)
    ref = orc.cascade(p, eps=sched, errors=False)
    with ecmg.Solver(**DRIVERS[driver]) as s:
        s.setup(p)
        infos = s.solve_levels(sched)
        u = [s.get(l, ecmg.VEC_U) for l in range(p.levels)]
    assert [i["iters"] for i in infos[2:]] == [r.iters for r in ref[2:]]
    d = [_rel(u[l], ref[l].u) for l in range(2, p.levels)]
    print("schedule: iterate differences per level", d)
    for l in range(2, p.levels):
        assert infos[l]["rre"] <= sched[l]
    assert max(d) <= 1e-12, d


def test_resetup_same_grids_matches_fresh(ecmg):
    """A second set-up of a problem with the same grids takes the context's
    device arrays back (by size) instead of freeing and allocating them; the
    solve then equals a fresh context's bit for bit, also after a set-up of
    other grids in between."""
    rng = np.random.default_rng(5)
    mk = lambda n: workloads.serving_request(n, rng.uniform(0, 1, 3), rng.uniform(1, 3, 3), rng.integers(0, 2, 6))
    a, b, c = mk(32), mk(32), mk(64)

    def solve(s, p):
        s.setup(p)
        s.solve(1e-8)
        return s.extrapolate()

    with ecmg.Solver(keep_w=True) as s:
        solve(s, a)
        got_b = solve(s, b)
        solve(s, c)
        got_b2 = solve(s, b)
    with ecmg.Solver(keep_w=True) as f:
        ref_b = solve(f, b)
    assert np.array_equal(got_b, ref_b) and np.array_equal(got_b2, ref_b)
