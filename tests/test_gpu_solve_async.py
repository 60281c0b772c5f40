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


@pytest.mark.parametrize("persistent", [0, -1, 300000], ids=["tiled", "default", "persistent"])
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
    with ecmg.Solver(persistent_nodes=0, timing=True) as s:
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
