"""ecmg_norms_noalloc, the allocation-free variant of ecmg_norms (its reduction
scratch in the library's static device array), against ecmg_norms itself and
against the same norms taken on the host: two calls in a row, the second on a
smaller level, so the second call runs on the array the first one left."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ecmg():
    import paper_1506_02983_amd as E
    E.load_library()
    return E


def test_norms_noalloc_matches_norms(ecmg):
    p = workloads.variable_beta_robin_cube(levels=5)          # finest 129^3: 1,024 reduction blocks
    with ecmg.Solver() as s:
        s.setup(p)
        s.solve(p.eps)
        s.extrapolate()
        cases = [(4, ecmg.VEC_U, ecmg.VEC_W),                 # the finest level, then a smaller one
                 (2, ecmg.VEC_U, ecmg.VEC_NONE),
                 (4, ecmg.VEC_UTILDE, ecmg.VEC_U)]
        for level, which, minus in cases:
            got = s.norms_noalloc(level, which, minus)
            ref = s.norms(level, which, minus)
            assert got == ref, (level, which, minus, got, ref)          # same kernel, same order
            v = s.get(level, which) - (s.get(level, minus) if minus != ecmg.VEC_NONE else 0.0)
            assert got[0] == pytest.approx(float(np.abs(v).max()), rel=1e-15, abs=0.0)
            assert got[1] == pytest.approx(float(np.sqrt(np.dot(v, v) / v.size)), rel=1e-13)


def test_norms_noalloc_errors(ecmg):
    with ecmg.Solver() as s:
        with pytest.raises(ecmg.EcmgError) as e:
            s.norms_noalloc(0, ecmg.VEC_U)
        assert e.value.code == ecmg.ESTATE
        s.setup(workloads.smooth_dirichlet_cube(levels=3))
        with pytest.raises(ecmg.EcmgError) as e:
            s.norms_noalloc(2, ecmg.VEC_UTILDE)                # not computed yet
        assert e.value.code == ecmg.EINVAL
