"""GPU batched form: many independent three-level ECMG_jcg solves, the JCG of
every box on a level in one launch of the queue kernel.

Checks: a box's result in the batch equals the same box solved in a batch of
its own bit for bit (batch invariance); against the single-problem solver
(multi-workgroup persistent kernel, different summation order) and the oracle
the per-level iteration counts agree and the iterates match to 1e-12 relative
in the max norm, the normal-mode parity rule."""
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
def boxes():
    # the first 12 boxes of the batched mix (seed 0): uneven shapes 16..64
    return workloads.batched_mix(12, seed=0)


def _solve_batch(ecmg, probs, eps):
    solvers = [ecmg.Solver().setup(p) for p in probs]
    infos = ecmg.solve_batch(solvers, eps)
    ecmg.extrapolate_batch(solvers)
    out = [(s.get(p.levels - 1, ecmg.VEC_U), s.get(p.levels - 1, ecmg.VEC_UTILDE)) for s, p in zip(solvers, probs)]
    for s in solvers:
        s.close()
    return infos, out


def test_batch_invariance(ecmg, boxes):
    infos, out = _solve_batch(ecmg, boxes, 1e-8)
    for i in (0, 5, 11):
        infos1, out1 = _solve_batch(ecmg, [boxes[i]], 1e-8)
        assert [x["iters"] for x in infos1[0]] == [x["iters"] for x in infos[i]]
        assert np.array_equal(out1[0][0], out[i][0]), i
        assert np.array_equal(out1[0][1], out[i][1]), i


def test_batch_matches_single_solver(ecmg, boxes):
    infos, out = _solve_batch(ecmg, boxes, 1e-8)
    for i, p in enumerate(boxes):
        with ecmg.Solver() as s:
            s.setup(p)
            ref = s.solve(1e-8)
            assert [x["iters"] for x in ref[2:]] == [x["iters"] for x in infos[i][2:]], i
            assert _rel(out[i][0], s.get(2, ecmg.VEC_U)) <= 1e-12, i
            s.extrapolate(2, out=False)
            assert _rel(out[i][1], s.get(2, ecmg.VEC_UTILDE)) <= 1e-12, i
        assert all(x["status"] == 0 for x in infos[i])


def test_batch_parity_with_oracle(orc, ecmg, boxes):
    small = [p for p in boxes if p.nodes_at(2) <= 40000][:3]
    assert small
    infos, out = _solve_batch(ecmg, small, 1e-8)
    for i, p in enumerate(small):
        res = orc.cascade(p, eps=1e-8, keep_vectors=True, errors=False)
        assert res[2].iters == infos[i][2]["iters"], (i, res[2].iters, infos[i][2])
        assert _rel(out[i][0], res[2].u) <= 1e-12, i
        assert _rel(out[i][1], res[2].Ut) <= 1e-12, i


def test_batch_errors(ecmg, boxes):
    s = ecmg.Solver().setup(boxes[0])
    t = ecmg.Solver()
    with pytest.raises(ecmg.EcmgError) as e:
        ecmg.solve_batch([s, t], 1e-8)
    assert e.value.code == ecmg.ESTATE
    with pytest.raises(ecmg.EcmgError) as e:
        ecmg.solve_batch([s, s], 1e-8)
    assert e.value.code == ecmg.EINVAL
    s.close()
    t.close()
