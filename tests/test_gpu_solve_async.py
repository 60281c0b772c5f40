"""GPU: the solve enqueues every level without waiting and starts each tiled
JCG level with the iteration count it needed in the previous solve.  Whatever
that first chunk is -- too long (its extra launches find `done` set and return
at once) or too short (the loop goes on) -- the iterates must be those of a
fresh context, bit for bit, with the same per-level iteration counts."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ecmg():
    import paper_1506_02983_amd as E
    E.load_library()
    return E


def _solve(ecmg, s, p, eps):
    infos = s.solve(eps)
    return [i["iters"] for i in infos], {l: s.get(l, ecmg.VEC_U) for l in range(p.levels)}


@pytest.mark.parametrize("persistent", [0, -1, 300000], ids=["no-persistent", "default", "persistent"])
def test_repeated_solves_match_fresh_context(ecmg, persistent):
    p = workloads.variable_beta_robin_cube(levels=5)
    fresh = {}
    for eps in (1e-6, 1e-10):
        with ecmg.Solver(persistent_nodes=persistent) as s:
            s.setup(p)
            fresh[eps] = _solve(ecmg, s, p, eps)
    assert fresh[1e-10][0][2:] != fresh[1e-6][0][2:]       # the hint differs between the two
    with ecmg.Solver(persistent_nodes=persistent) as s:
        s.setup(p)
        for eps in (1e-6, 1e-10, 1e-10, 1e-6):               # too short, exact, too long
            iters, u = _solve(ecmg, s, p, eps)
            assert iters == fresh[eps][0], (eps, iters, fresh[eps][0])
            for l in range(p.levels):
                assert np.array_equal(u[l], fresh[eps][1][l]), (eps, l)


def test_kernel_times_count_working_launches(ecmg):
    """Pass A / pass B launches that found `done` set are not counted: after a
    solve whose first chunk was too long, each tiled level counts exactly its
    iterations (pass A: iteration 0 in class 10, the others in class 0)."""
    p = workloads.variable_beta_robin_cube(levels=5)
    with ecmg.Solver(persistent_nodes=0, gather_nodes=0, timing=True) as s:
        s.setup(p)
        s.solve(1e-10)
        s.reset_kernel_times()
        infos = s.solve(1e-6)                                 # hints from the 1e-10 solve
        for l in range(2, p.levels):
            it = infos[l]["iters"]
            counts = {k: s.kernel_times(l, k)[1] for k in (0, 1, 10)}
            assert counts[10] == min(it, 1) and counts[0] == max(it - 1, 0), (l, counts, it)
            assert counts[1] == it, (l, counts, it)


def test_set_timing_selects_classes(ecmg):
    """Only the selected kernel classes are timed; -1 times every class again."""
    p = workloads.variable_beta_robin_cube(levels=5)
    with ecmg.Solver(persistent_nodes=0, timing=True) as s:
        s.setup(p)
        s.solve(1e-8)
        s.set_timing([2])                                     # JCG init only
        s.reset_kernel_times()
        infos = s.solve(1e-8)
        for l in range(2, p.levels):
            assert s.kernel_times(l, 2)[1] == 1, l
            for k in (0, 1, 10):
                assert s.kernel_times(l, k)[1] == 0, (l, k)
        s.set_timing(-1)
        s.reset_kernel_times()
        infos = s.solve(1e-8)
        for l in range(2, p.levels):
            assert s.kernel_times(l, 1)[1] == infos[l]["iters"], l
        s.set_timing(0)
        s.reset_kernel_times()
        s.solve(1e-8)
        assert all(s.kernel_times(l, k)[1] == 0 for l in range(p.levels) for k in (0, 1, 2, 10))


def _stable(ecmg, s, p, eps, times=3):
    # the same solve a few times: every tiled level's iteration count repeats,
    # so the next solve enqueues each of them without a status read
    for _ in range(times):
        s.solve(eps)


# the drivers a speculative level can run: tiled or gather with folded scalar
# steps, the persistent kernel where it is the default, and the unfolded column
# path of the large grids (forced with fold_blocks = 0), whose last speculative
# pass B stores no residual
SPEC_DRIVERS = {"tiled": dict(persistent_nodes=0, gather_nodes=0), "gather": dict(persistent_nodes=0),
                "default": dict(persistent_nodes=-1), "unfolded": dict(persistent_nodes=0, fold_blocks=0)}


@pytest.mark.parametrize("driver", list(SPEC_DRIVERS))
def test_speculative_chunk_shortfall_matches_fresh_context(ecmg, driver):
    """A level enqueued with its previous count and no status read that then
    falls short of a tighter tolerance is solved again, with every finer level,
    from its EXP_finite start: iterates and counts equal a fresh context's."""
    p = workloads.variable_beta_robin_cube(levels=5)
    with ecmg.Solver(**SPEC_DRIVERS[driver]) as s:
        s.setup(p)
        fresh = _solve(ecmg, s, p, 1e-10)
    with ecmg.Solver(**SPEC_DRIVERS[driver]) as s:
        s.setup(p)
        _stable(ecmg, s, p, 1e-6)
        for _ in range(2):                                    # short speculation, then no speculation
            iters, u = _solve(ecmg, s, p, 1e-10)
            assert iters == fresh[0], (iters, fresh[0])
            for l in range(p.levels):
                assert np.array_equal(u[l], fresh[1][l]), l


@pytest.mark.parametrize("driver", ["tiled", "gather", "unfolded"])
def test_speculative_shortfall_on_a_middle_level(ecmg, driver):
    """Only level 3's tolerance tightens: level 2 keeps its speculative result,
    levels 3 and 4 are solved again; the same as a fresh context."""
    p = workloads.variable_beta_robin_cube(levels=5)
    loose = [1e-6] * p.levels
    tight = list(loose)
    tight[3] = 1e-11
    with ecmg.Solver(**SPEC_DRIVERS[driver]) as s:
        s.setup(p)
        s.solve_levels(loose)
        ref = s.solve_levels(tight)
        ref_u = {l: s.get(l, ecmg.VEC_U) for l in range(p.levels)}
    with ecmg.Solver(timing=True, **SPEC_DRIVERS[driver]) as s:
        s.setup(p)
        for _ in range(3):
            base = s.solve_levels(loose)
        s.reset_kernel_times()
        infos = s.solve_levels(tight)
        assert [i["iters"] for i in infos] == [i["iters"] for i in ref]
        assert infos[2]["iters"] == base[2]["iters"] and infos[3]["iters"] > base[3]["iters"]
        for l in range(p.levels):
            assert np.array_equal(s.get(l, ecmg.VEC_U), ref_u[l]), l
        # the discarded attempt leaves no kernel times: each tiled level counts
        # exactly the iterations of its kept solve
        # (unfolded: pass A of iterations >= 1 is class 11, and the last pass B
        # of a kept speculative level class 12)
        for l in range(2, p.levels):
            it = infos[l]["iters"]
            counts = {k: s.kernel_times(l, k)[1] for k in (0, 1, 10, 11, 12)}
            assert counts[10] == min(it, 1) and counts[0] + counts[11] == max(it - 1, 0), (l, counts, it)
            assert counts[1] + counts[12] == it, (l, counts, it)
            # level 3 fell short and ran again with status reads; levels 2 and 4
            # ran speculatively
            assert counts[12] == (1 if driver == "unfolded" and l != 3 else 0), (l, counts)


@pytest.mark.parametrize("driver", ["tiled", "gather", "unfolded"])
def test_speculation_off_gives_the_same_iterates(ecmg, driver):
    p = workloads.variable_beta_robin_cube(levels=5)
    out = []
    for spec in (True, False):
        with ecmg.Solver(speculate=spec, **SPEC_DRIVERS[driver]) as s:
            s.setup(p)
            _stable(ecmg, s, p, 1e-8)
            out.append(_solve(ecmg, s, p, 1e-8))
    assert out[0][0] == out[1][0]
    for l in range(p.levels):
        assert np.array_equal(out[0][1][l], out[1][1][l]), l


def test_solve_extrapolated_matches_solve_then_extrapolate(ecmg):
    """ecmg_solve_extrapolated (EXP_true enqueued behind the cascade, one wait;
    the finest level's last x update fused into EXP_true and applied to x only
    when x is read) leaves the U~ and U of ecmg_solve + ecmg_extrapolate, also
    when a speculative level falls short and the finest levels are solved
    again, and when the next call reads x (get, norms, extrapolate, a JCG
    continuation) or replaces it (solve)."""
    p = workloads.variable_beta_robin_cube(levels=5)
    L = p.levels - 1
    ref, refu, refj = {}, {}, None
    with ecmg.Solver(persistent_nodes=0) as s:
        s.setup(p)
        for eps in (1e-6, 1e-10):
            s.solve(eps)
            refu[eps] = s.get(L, ecmg.VEC_U)
            s.extrapolate(L, out=False)
            ref[eps] = s.get(L, ecmg.VEC_UTILDE)
        refn = s.norms(L, ecmg.VEC_U)
        s.jcg(L, 1e-12)
        refj = s.get(L, ecmg.VEC_U)
    with ecmg.Solver(persistent_nodes=0) as s:
        s.setup(p)
        for eps in (1e-6, 1e-6, 1e-6, 1e-10):                 # the last one falls short
            infos = s.solve(eps, extrapolate=True)
            assert all(i["status"] == ecmg.OK for i in infos)
            assert np.array_equal(s.get(L, ecmg.VEC_UTILDE), ref[eps]), eps
            assert np.array_equal(s.get(L, ecmg.VEC_U), refu[eps]), eps
        s.solve(1e-10, extrapolate=True)
        assert s.norms(L, ecmg.VEC_U) == refn                 # norms apply the pending update first
        s.solve(1e-10, extrapolate=True)
        s.jcg(L, 1e-12)                                        # so does a JCG continuation
        assert np.array_equal(s.get(L, ecmg.VEC_U), refj)
        s.solve(1e-10, extrapolate=True)
        assert np.array_equal(s.extrapolate(L), ref[1e-10])
