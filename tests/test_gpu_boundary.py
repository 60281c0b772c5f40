"""The C interface's options that do not change the arithmetic: the device
allocator hook (PyTorch's caching allocator backing the hierarchy) and the
true residual report."""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ecmg():
    import paper_1506_02983_amd as E
    E.load_library()
    return E


def _run(ecmg, p, **opts):
    with ecmg.Solver(**opts) as s:
        s.setup(p)
        infos = s.solve(p.eps)
        return [i["iters"] for i in infos], [s.get(l) for l in range(p.levels)], s.extrapolate()


def test_torch_allocator_hook(ecmg):
    """Every device allocation of a context comes from PyTorch's caching
    allocator when the hook is set, the results are bit for bit those of the
    library's own hipMalloc, and closing the context gives the memory back."""
    import torch

    p = workloads.variable_beta_robin_cube(levels=4)
    base = _run(ecmg, p)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    with ecmg.Solver(torch_allocator=True) as s:
        s.setup(p)
        during = torch.cuda.memory_allocated()
        infos = s.solve(p.eps)
        got = ([i["iters"] for i in infos], [s.get(l) for l in range(p.levels)], s.extrapolate())
    torch.cuda.synchronize()
    after = torch.cuda.memory_allocated()
    # the finest level alone holds x, F, 1/D, W and four work vectors of 65^3 nodes
    assert during - before >= 8 * 8 * 65 ** 3
    assert after == before
    assert got[0] == base[0]
    for a, b in zip(got[1], base[1]):
        assert np.array_equal(a, b)
    assert np.array_equal(got[2], base[2])


def test_true_residual_matches_host(ecmg, orc):
    """info.rre_true is ||F - A u||_2 / ||f_h||_2 over the free nodes of the
    final iterate: recomputed here from the library's operator apply, F and the
    Dirichlet mask of the oracle."""
    p = workloads.variable_beta_robin_cube(levels=4)
    with ecmg.Solver(true_residual=True) as s:
        s.setup(p)
        infos = s.solve(p.eps)
        for l in range(p.levels):
            u = s.get(l)
            Au = s.apply(l, u)
            F = s.get(l, ecmg.VEC_F)
            free = orc.dirichlet_mask(orc.grid_of(p, l)) == 0
            r = np.linalg.norm((F - Au)[free]) / infos[l]["nf"]
            if l < 2:       # the direct DSOLVE: a residual of rounding size
                assert infos[l]["rre_true"] < 1e-13 and r < 1e-13, (l, infos[l], r)
                continue
            assert infos[l]["rre_true"] == pytest.approx(r, rel=1e-6), (l, infos[l], r)
            assert infos[l]["rre_true"] <= 1.1 * p.eps
    with ecmg.Solver() as s:
        s.setup(p)
        infos = s.solve(p.eps)
        assert all(i["rre_true"] == -1.0 for i in infos)
