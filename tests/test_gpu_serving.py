"""GPU serving loop (continuous batching): requests of different sizes,
coefficients and boundary types admitted as they arrive and by device-memory
budget, advanced one level per step with the small levels of all requests in
one launch.

A request's result must be the same alone and in the mix: each request's
levels run with the same workgroup decomposition whatever else is admitted,
so the check is bitwise.  Against the single-problem solver (different
summation order) the normal-mode rule applies: equal per-level iteration
counts and U~ within 1e-12 relative in the max norm."""
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


@pytest.fixture(scope="module")
def requests():
    rng = np.random.default_rng(7)
    out = []
    for n in (32, 64, 32, 64, 32, 64):
        phi = rng.uniform(0, 1, 3)
        k = rng.uniform(1, 3, 3)
        faces = rng.integers(0, 2, 6)
        out.append(workloads.serving_request(n, phi, k, faces))
    return out


def _run(ecmg, probs, budget=1 << 40, stagger=None, **opts):
    with ecmg.Server(budget, **opts) as srv:
        tickets = []
        pending = list(probs)
        first = pending if stagger is None else pending[:stagger]
        for p in first:
            tickets.append(srv.submit(p, 1e-8))
        rest = [] if stagger is None else pending[stagger:]
        steps = 0
        while True:
            srv.step()
            steps += 1
            if rest:
                tickets.append(srv.submit(rest.pop(0), 1e-8))
                continue
            if all(srv.poll(t)[0] == 2 for t in tickets):
                break
            assert steps < 1000
        res = [(srv.result(t).copy(), srv.poll(t)[1]) for t in tickets]
        stats = srv.stats()
    return res, stats


@pytest.mark.parametrize("persistent", [-1, 5000], ids=["queue", "queue+tiled"])
def test_request_same_alone_and_in_mix(ecmg, requests, persistent):
    mix, stats = _run(ecmg, requests, stagger=2, persistent_nodes=persistent)
    assert stats["done"] == len(requests) and stats["p99_ms"] >= stats["p50_ms"] > 0
    for i in (0, 3, 5):
        alone, _ = _run(ecmg, [requests[i]], persistent_nodes=persistent)
        assert [x["iters"] for x in alone[0][1]] == [x["iters"] for x in mix[i][1]]
        assert np.array_equal(alone[0][0], mix[i][0]), i
        # the levels in the shared queue launches, and the larger ones (queue+tiled)
        # on their own kernels: the gather path at these sizes
        p = requests[i]
        want = [ecmg.PATH_QUEUE if persistent < 0 or p.nodes_at(l) <= persistent else ecmg.PATH_GATHER
                for l in range(p.levels)]
        assert [x["path"] for x in mix[i][1]] == want, (i, [x["path"] for x in mix[i][1]])


def test_budget_admission_queues_and_matches(ecmg, requests):
    free, _ = _run(ecmg, requests)
    need = max(ecmg.plan_bytes(p) for p in requests)
    tight, stats = _run(ecmg, requests, budget=need)      # one hierarchy at a time at most
    assert stats["done"] == len(requests)
    for a, b in zip(free, tight):
        assert np.array_equal(a[0], b[0])


def test_matches_single_solver(ecmg, requests):
    mix, _ = _run(ecmg, requests)
    for i, p in enumerate(requests):
        with ecmg.Solver() as s:
            s.setup(p, device_fields=True)
            infos = s.solve(1e-8)
            s.extrapolate(p.levels - 1, out=False)
            ut = s.get(p.levels - 1, ecmg.VEC_UTILDE)
        assert [x["iters"] for x in infos[2:]] == [x["iters"] for x in mix[i][1][2:]], i
        assert _rel(mix[i][0].ravel(), ut.ravel()) <= 1e-12, i


def test_over_budget_rejected(ecmg, requests):
    with ecmg.Server(1 << 20) as srv:
        with pytest.raises(ecmg.EcmgError) as e:
            srv.submit(requests[1], 1e-8)
        assert e.value.code == ecmg.ENOMEM


def test_served_requests_match_oracle(orc, ecmg, requests):
    """Three served requests (finest 32^3 and 64^3, mixed Dirichlet / Robin
    faces) against the oracle's cascade (Algorithm 4 with EXP_true): per-level
    JCG counts equal, U~ within 1e-12 relative in the max norm.  The server's
    DSOLVE levels run JCG to round-off, the oracle's a direct solve; the
    difference is far below the bound."""
    picked = [requests[0], requests[1], requests[3]]
    mix, _ = _run(ecmg, picked)
    for i, p in enumerate(picked):
        ref = orc.cascade(p, eps=1e-8, keep_vectors=True, errors=False)
        L = p.levels - 1
        assert [r.iters for r in ref[2:]] == [x["iters"] for x in mix[i][1][2:]], i
        assert _rel(mix[i][0].ravel(), np.asarray(ref[L].Ut).ravel()) <= 1e-12, i


def test_completed_drains_each_ticket_once(ecmg, requests):
    """ecmg_server_completed hands out every finished ticket once, in finishing
    order; a context kept from a finished request serves the next request of
    the same grids bit for bit like a fresh server."""
    with ecmg.Server(1 << 40) as srv:
        tickets = [srv.submit(p, 1e-8) for p in requests]
        seen = []
        while len(seen) < len(tickets):
            srv.step()
            got = srv.completed()
            assert all(srv.poll(t)[0] == 2 for t in got)
            seen += got
        assert sorted(seen) == sorted(tickets) and srv.completed() == []
        again = srv.submit(requests[0], 1e-8)       # reuses a kept 32^3 context
        while srv.poll(again)[0] != 2:
            srv.step()
        assert srv.completed() == [again]
        fresh, _ = _run(ecmg, [requests[0]])
        assert np.array_equal(srv.result(again), fresh[0][0])
        assert np.array_equal(srv.result(tickets[0]), fresh[0][0])


def test_release_refuses_unfinished(ecmg, requests):
    with ecmg.Server(1 << 40) as srv:
        t = srv.submit(requests[0], 1e-8)
        with pytest.raises(ecmg.EcmgError) as e:
            srv.release(t)
        assert e.value.code == ecmg.ESTATE
        while srv.poll(t)[0] != 2:
            srv.step()
        srv.release(t)
