"""Element-wise oracle parity and the paper's own numbers at the benchmark's
largest sizes.

* The 513^3 workload's hierarchy cut at six grids (finest 256^3 elements,
  16,974,593 nodes), the largest the oracle runs in seconds, in the
  configuration bench.py times: device-sampled fields and the autotuned
  per-level JCG configuration.  There the 257^3 level's passes have more than
  4,096 blocks, so it runs the tiled passes with one-block finishing kernels,
  the driver of the benchmark's two finest levels.  Fixed-iteration mode with
  the oracle's per-level counts: u, W and U~ of every level, element by
  element, to 1e-12 relative in the max norm; then normal mode: the same
  counts, iterates and true residuals.
* The paper's Problem 1 on its seven grids 8^3 .. 512^3 (Section 5, Tables
  iterations8-10, table11, table22, table1, table2): the counts of the grids
  up to 128^3 are the oracle's (or stop where the oracle's residual stalls
  within 1.5x of the threshold), those of 256^3 and 512^3 are within 2 of the
  printed ones (summation order moves a count when the residual stops near the
  threshold) whenever the coarser counts are the printed ones, and the errors
  of the 512^3 grid agree with the printed ones."""
import json
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
GOLDEN_512 = os.path.join(os.path.dirname(__file__), "golden", "paper_problem1_512.json")


@pytest.fixture(scope="module")
def ecmg():
    import paper_1506_02983_amd as E
    E.load_library()
    return E


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def ref257(orc):
    p = workloads.variable_beta_robin_cube(levels=6, eps=1e-8)
    print("oracle: variable-beta Robin cascade 8^3 -> 256^3", flush=True)
    return p, orc.cascade(p)


def _bench_config_solver(ecmg, p):
    """A context in bench.py's configuration: device fields, a warm-up solve,
    then the autotuner over each level's own iteration count."""
    s = ecmg.Solver(keep_w=True, true_residual=True)
    s.setup(p, device_fields=True)
    s.solve(p.eps)
    tuned = s.autotune(iters=0)
    print("tuned", [(r["level"], r["path"], r["kz"]) for r in tuned], flush=True)
    return s


@pytest.mark.timeout(900)
def test_cascade_257_fixed_iterations(ecmg, ref257):
    p, ref = ref257
    iters = [r.iters for r in ref]
    print("oracle iterations", iters, flush=True)
    with _bench_config_solver(ecmg, p) as s:
        s.solve_fixed(iters)
        for l in range(p.levels):
            du = _rel(s.get(l, ecmg.VEC_U), ref[l].u)
            dw = _rel(s.get(l, ecmg.VEC_W), ref[l].W) if l >= 2 else 0.0
            dt = _rel(s.extrapolate(l), ref[l].Ut) if l >= 1 else 0.0
            print("level %d: u %.2e  W %.2e  U~ %.2e" % (l, du, dw, dt), flush=True)
            assert du <= 1e-12 and dw <= 1e-12 and dt <= 1e-12, (l, du, dw, dt)


@pytest.mark.timeout(900)
def test_cascade_257_normal_mode(ecmg, ref257):
    p, ref = ref257
    with _bench_config_solver(ecmg, p) as s:
        infos = s.solve(p.eps)
        got = [i["iters"] for i in infos]
        print("GPU iterations", got, "oracle", [r.iters for r in ref], flush=True)
        for l in range(2, p.levels):
            r = ref[l]
            near = abs(r.rre / p.eps - 1.0) < 1e-3
            assert abs(got[l] - r.iters) <= (1 if near else 0), (l, got[l], r.iters)
            assert infos[l]["rre"] <= p.eps
            if got[l] == r.iters:
                assert _rel(s.get(l, ecmg.VEC_U), r.u) <= 1e-12, l
                assert infos[l]["rre_true"] == pytest.approx(r.rre_true, rel=2e-2), (l, infos[l], r.rre_true)
        assert _rel(s.extrapolate(), ref[-1].Ut) <= 1e-12


def _golden_512():
    with open(GOLDEN_512) as fh:
        return json.load(fh)["cases"]


def _digits(got, want, tol=0.006):
    return abs(got / want - 1.0) <= tol


@pytest.mark.timeout(600)
@pytest.mark.parametrize("case", _golden_512(), ids=lambda c: "eps%g" % c["eps"])
def test_paper_problem1_512(orc, ecmg, case):
    import torch

    eps = case["eps"]
    p = workloads.paper_problem1(levels=7, eps=eps)
    # the grids up to 128^3 against the oracle (a five-grid run computes the
    # same first five levels); the printed counts there are pinned to the
    # oracle on the CPU, including the two 128^3 counts this reading does not
    # reproduce
    p5 = workloads.paper_problem1(levels=5, eps=eps)
    lv5 = [orc.discretize(p5, l) for l in range(5)]
    ref = orc.cascade(p5, levels=lv5, variant=orc.LAGRANGE27, errors=False)
    with ecmg.Solver(interp=ecmg.LAGRANGE27, keep_w=True) as s:
        s.setup(p, device_fields=True)
        infos = s.solve(eps)
        got = [i["iters"] for i in infos[2:]]
        want = [row["iters"] for row in case["rows"]]
        print("eps %g: GPU iterations %s, oracle (to 128^3) %s, paper %s"
              % (eps, got, [r.iters for r in ref[2:]], want), flush=True)
        for l in range(2, 5):
            if got[l - 2] == ref[l].iters:
                continue
            # A different count is allowed only where the residual stalls at
            # the threshold: there two summation orders cross it several
            # iterations apart (at eps = 1e-10 on 128^3 the oracle's residual
            # needs five iterations to fall from 1.2 to 0.9 times it).  The
            # oracle's own residual at the GPU's count must be within 1.5x of
            # the threshold.
            lv = lv5[l]
            x0 = np.where(lv.dmask == 1, lv.gD, ref[l].W)
            k = got[l - 2]
            hist = orc.jcg(lv, x0, 0.0, fixed_iters=k).hist
            thr = eps * lv.nf
            print("level %d: oracle residual at the GPU's count %d: %.3f x threshold"
                  % (l, k, hist[k] / thr), flush=True)
            assert hist[k] <= 1.5 * thr and hist[k - 1] > thr / 1.5, (l, k, ref[l].iters, hist[k] / thr)
        # the two finest grids against the paper, when they start from the
        # paper's coarse solutions (every coarser count printed)
        if got[:3] == want[:3]:
            for g_, w_, row in zip(got[3:], want[3:], case["rows"][3:]):
                assert abs(g_ - w_) <= 2, (case["cite"], row["mesh"], g_, w_)
        s.extrapolate()
        # exact solution at the 513^3 nodes, on the device (dense node order)
        n = p.n_at(6)
        dev = torch.device("cuda")
        ax = [torch.arange(n[d] + 1, dtype=torch.float64, device=dev) / n[d] for d in range(3)]
        S = [torch.sin(0.5 * np.pi * a) for a in ax]
        ue = (S[2][:, None, None] * S[1][None, :, None] * S[0][None, None, :]).contiguous()
        err = {}
        err["U_max"], err["U_l2"] = s.norms(6, ecmg.VEC_U, minus=ue)
        err["Ut_max"], err["Ut_l2"] = s.norms(6, ecmg.VEC_UTILDE, minus=ue)
        err["WU_max"], err["WU_l2"] = s.norms(6, ecmg.VEC_W, ecmg.VEC_U)
        del ue
        row = case["rows"][-1]
        print("eps %g: 512^3 errors %s, rre %.3e" % (eps, err, infos[6]["rre"]), flush=True)
        # the FE error and the initial guess's distance are set by the grid and
        # the interpolation: 3 digits whatever the algebraic error
        for k in ("U_max", "U_l2", "WU_max", "WU_l2"):
            if k in row:
                assert _digits(err[k], row[k]), (case["cite"], k, err[k], row[k])
        # U~ differences two grid solutions, so its error follows the algebraic
        # error of both: 3 digits when every count is the paper's
        if "Ut_max" in row:
            tol = 0.006 if got == want else 0.25
            for k in ("Ut_max", "Ut_l2"):
                assert _digits(err[k], row[k], tol), (case["cite"], k, err[k], row[k], got)
