"""GPU autotuner: times the JCG configurations of every JCG level, keeps the
fastest, writes the JSON cache, and a context created with autotune = 1 applies
the cached choices.  The configuration changes how the JCG loop runs, not its
recurrence: per-level iteration counts are those of the built-in
configuration and the iterates agree to 1e-12 relative (summation order); the
same cached configuration gives the same iterates bit for bit."""
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


def _solve(ecmg, s, p):
    infos = s.solve(1e-9)
    return [i["iters"] for i in infos], [s.get(l, ecmg.VEC_U) for l in range(p.levels)]


def test_autotune_cache_roundtrip(ecmg, tmp_path):
    p = workloads.variable_beta_robin_cube(levels=5)
    cache = str(tmp_path / "tune.json")
    with ecmg.Solver() as s:
        s.setup(p)
        ref_iters, ref_u = _solve(ecmg, s, p)
    with ecmg.Solver() as s:
        s.setup(p)
        res = s.autotune(iters=4, cache=cache)
        assert [r["level"] for r in res] == list(range(2, p.levels))
        for r in res:
            assert r["candidates"] >= 2 and 0 < r["us_best"] <= r["us_default"] * (1 + 1e-12), r
            n = p.n_at(r["level"])
            hit = ecmg.tune_lookup(cache, n)
            assert hit is not None and (hit["path"], hit["kz"], hit["seg"], hit["nwg"]) == \
                (r["path"], r["kz"], r["seg"], r["nwg"])
        iters, u = _solve(ecmg, s, p)
    assert iters == ref_iters
    for l in range(2, p.levels):
        assert _rel(u[l], ref_u[l]) <= 1e-12, l
    with ecmg.Solver(autotune=1, tune_cache=cache) as s:
        s.setup(p)
        iters2, u2 = _solve(ecmg, s, p)
    assert iters2 == iters
    for l in range(p.levels):
        assert np.array_equal(u2[l], u[l]), l


def test_autotune_before_setup_is_an_error(ecmg):
    with ecmg.Solver() as s:
        with pytest.raises(ecmg.EcmgError) as e:
            s.autotune()
        assert e.value.code == ecmg.ESTATE
