#!/usr/bin/env python3
"""ECMG_jcg benchmark on one MI355X.

One step = the whole hot path on the workload: Algorithm 4 (DSOLVE on the two
coarsest grids, EXP_finite + JCG on every finer grid) plus the final EXP_true on
the finest grid, with every input already resident in HBM (setup is timed
separately).  value = finest-grid unknowns (all nodes, as the paper counts them)
per second of wall time of that step.

Prints one JSON line.  After the warm-up (and the autotuner), two untimed steps
with HIP events around every launch give the per-kernel breakdown and name the
dominant kernel (largest total time); the timed steps run without events (a
timed launch costs about 5 us more, which the launch-bound levels would add to
the step); the same number of steps follows with events, stamped by each launch
of the dominant kernel itself on the library's stream, around that kernel only,
which give the roofline's average duration.  Algorithmic bytes per launch follow
the per-node traffic model of each kernel (algorithmic_bytes below).  The CPU baseline times the oracle on a
bounded sample of the same workload (fewer levels) on the host cores.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "unknowns/s to 4th-order accuracy (FP64 vs mixed); JCG HBM GB/s; serve p50/p99"
HBM_PEAK_GBS = 8000.0   # MI355X HBM3E
KIND_NAMES = {0: "jcg_pass_a", 1: "jcg_pass_b", 2: "jcg_init", 3: "exp_finite", 4: "exp_true",
              5: "jcg_pass_a_fp32", 6: "jcg_pass_b_fp32", 7: "jcg_persistent", 10: "jcg_pass_a0",
              11: "jcg_pass_a_col", 12: "jcg_pass_b_last"}
# kernel names as rocprofv3 reports them (stencil: <type, mode, rows of
# threads, rows per thread, waves per SIMD>; column kernels: <mode, node rows
# per wave, waves per SIMD, prefetch distance>, whose last blocks take the
# Robin-face nodes).  A class runs different kernels on levels that ran
# different paths (ecmg_level_info.path): the tiled kernels with folded or
# unfolded scalar steps, the column kernels on the large grids, the gather
# kernels (one thread per node) on the small ones.  There pass A is a
# node-wise p / x update followed by the stencil, timed as one (class 10 at
# iteration 0, 11 after); class 12 is the pass B a speculative chunk expects
# to be the level's last (stop test only, no r stored).
def kernel_symbol(kind, path, nx, E):
    col, gat = path == E.PATH_COLUMN, path == E.PATH_GATHER
    if kind == 0:
        return "k_stencil<double, 2, 8, 1, 4>"
    if kind == 1:
        return "k_passB<double, false>"
    if kind == 2:
        return "k_col<1, 2, 2, 1>" if col else "k_gather_init" if gat else "k_stencil<double, 1, 8, 1, 4>"
    if kind == 3:
        return "k_exp_finite<%s>" % ("true" if (nx // 4) % 64 == 0 else "false")
    if kind == 4:
        return "k_exp_true_fused"
    if kind == 5:
        return "k_stencil<float, 2, 8, 1, 4>"
    if kind == 6:
        return "k_passB<float, false>"
    if kind == 7:
        return "k_jcg_persistent"
    if kind == 10:
        return "k_col<3, 4, 2, 1>" if col else "k_p_update_fold + k_gather_a" if gat else \
            "k_stencil<double, 3, 4, 2, 2>"
    if kind == 11:
        return "k_p_update_fold + k_gather_a" if gat else "k_p_update + k_col<3, 4, 2, 1>"
    if kind == 12:
        return "k_passB<double, true>"
    return KIND_NAMES.get(kind, "?")


def workload(name):
    import workloads
    if name == "variable-beta-robin-513":
        return (workloads.variable_beta_robin_cube(levels=7, eps=1e-8),
                "variable-beta Robin cube, beta=1+0.5 sin(pi x)sin(pi y)sin(pi z), u=S+xyz, Dirichlet x-faces, "
                "Robin alpha=1 elsewhere; 8^3 -> 512^3 elements (7 levels, 513^3 = 135,005,697 nodes); eps=1e-8")
    if name == "smooth-dirichlet-33":
        return (workloads.smooth_dirichlet_cube(levels=4, eps=1e-10),
                "beta=1, u=exp(x+y+z), Dirichlet cube; 4^3 -> 32^3 elements (35,937 nodes); eps=1e-10")
    if name == "high-contrast-513x257x257":
        return (workloads.high_contrast_singular_box(levels=6, eps=1e-8),
                "box [0,2]x[0,1]^2, beta=exp(4 sin 2pi x cos 2pi y), u=r^(2/3), Dirichlet; 16x8x8 -> 512x256x256 "
                "(6 levels, 33,883,137 nodes); eps=1e-8")
    raise SystemExit("unknown workload %s" % name)


def algorithmic_bytes(kind, n, e, n1, n0, iters=0):
    """HBM bytes a launch must move at minimum (8-byte values; n nodes, e
    elements of the level; n1, n0 nodes of the two coarser levels; iters JCG
    iterations inside one persistent launch)."""
    if kind in (0, 11):
        return 8 * (6 * n + e)          # iterations >= 1: read r, p_old, x, beta; write p, q, x
    if kind == 10:
        return 8 * (2 * n + e)          # iteration 0: read p_0 (stored by init), beta; write q
    if kind == 1:
        return 8 * 4 * n                # read r, q, 1/D; write r
    if kind == 12:
        return 8 * 2 * n                # the expected last pass B: read r, q (stop test only)
    if kind == 2:
        return 8 * (4 * n + e)          # read x, F, beta; write r, p_0 = D^-1 r (D from beta: 40 B/node)
    if kind == 3:
        return 8 * (n + n1 + n0)        # write x; read u_{l-1}, u_{l-2} (the W copy is off when timed)
    if kind == 4:
        # a solve with EXP_true applies the finest level's last JCG update
        # x += alpha p inside EXP_true (x is stored only when read later):
        # read x, p, u_{l-1}; write U~
        return 8 * (3 * n + n1)
    if kind == 5:
        return 4 * (6 * n + e)
    if kind == 6:
        return 4 * 4 * n
    if kind == 7:
        # init: read x, F, 1/D, beta, write r; per iteration: read r, 1/D, x,
        # p_old, write x, p (own-node pass; the first iteration reads neither
        # x nor p_old and writes no x), read p, beta, write q (stencil), read
        # r, q, 1/D, write r; final x update: read x, p, write x
        if iters <= 0:
            return 8 * (4 * n + e)
        return 8 * ((4 * n + e) + (9 * n + e) + (iters - 1) * (12 * n + e) + 3 * n)
    return 0


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("jcg_kernels.hip", "col_kernels.hip", "persistent_kernels.hip", "extrap_kernels.hip",
              "ecmg_internal.h"):
        with open(os.path.join(ROOT, "paper_1506_02983_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(symbol, launches_per_step):
    """HBM bytes per launch: the kernel's HBM bytes per step from the committed
    rocprofv3 counter summary (every dispatch of the kernel name, or of the
    pair timed as one; launches that find the `done` flag set move next to
    nothing) over its working launches per step, if the summary was taken on
    the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    k = t.get("kernels", {}).get(symbol)
    if not k or not launches_per_step:
        return None
    return float(k["bytes_per_step"]) / launches_per_step


def exact_on_device(problem, n):
    import torch
    lo, hi = problem.lo, problem.hi
    ax = [lo[d] + torch.arange(n[d] + 1, dtype=torch.float64, device="cuda") * ((hi[d] - lo[d]) / n[d])
          for d in range(3)]
    v = problem.u(ax[0][None, None, :], ax[1][None, :, None], ax[2][:, None, None], -1)
    return torch.as_tensor(v, dtype=torch.float64, device="cuda").expand(n[2] + 1, n[1] + 1, n[0] + 1).contiguous()


def cpu_baseline(problem, levels, precision_interp=0, min_seconds=10.0):
    """The oracle's cascade (discretisation excluded, as on the GPU) on the same
    workload with fewer levels, repeated until at least min_seconds of CPU work
    have been timed."""
    import oracle
    p = problem.with_(levels=levels)
    lvls = [oracle.discretize(p, l) for l in range(levels)]
    reps, dt, res = 0, 0.0, None
    while reps == 0 or dt < min_seconds:
        t0 = time.perf_counter()
        res = oracle.cascade(p, levels=lvls, errors=False, keep_vectors=False, variant=precision_interp)
        dt += time.perf_counter() - t0
        reps += 1
    nodes = p.nodes_at(levels - 1)
    cores = oracle.num_threads()
    # the same region on one core, on the small smooth Dirichlet workload
    m1, m1_desc = workload("smooth-dirichlet-33")
    lv1 = [oracle.discretize(m1, l) for l in range(m1.levels)]
    reps1, dt1 = 0, 0.0
    oracle.set_num_threads(1)
    try:
        while reps1 == 0 or dt1 < 1.0:
            t0 = time.perf_counter()
            oracle.cascade(m1, levels=lv1, errors=False, keep_vectors=False)
            dt1 += time.perf_counter() - t0
            reps1 += 1
    finally:
        oracle.set_num_threads(cores)
    n1 = m1.nodes_at(m1.levels - 1)
    return {"value": nodes * reps / dt, "unit": "unknowns/s", "cores": cores, "kind": "oracle",
            "sample": "same workload on %d levels (finest %s elements, %d nodes): oracle DSOLVE + EXP_finite + "
                      "JCG + EXP_true region, %d repetitions, %.1f s, iterations %s" % (
                          levels, "x".join(map(str, p.n_at(levels - 1))), nodes, reps, dt,
                          [r.iters for r in res]),
            "host": host_cpu(),
            "one_core": {"value": n1 * reps1 / dt1, "unit": "unknowns/s", "cores": 1,
                         "sample": "%s: the same region, %d repetitions, %.2f s" % (m1_desc, reps1, dt1)}}


def host_cpu():
    """CPU model, sockets and logical CPUs of the host (and those this process may use)."""
    model, sockets = "unknown", set()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name") and model == "unknown":
                    model = line.split(":", 1)[1].strip()
                elif line.startswith("physical id"):
                    sockets.add(line.split(":", 1)[1].strip())
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"model": model, "sockets": max(1, len(sockets)), "logical_cpus": os.cpu_count(),
            "usable_cpus": usable}


def _finest_orders(E, s, problem, levels):
    """Max-norm errors of U and U~ on the given levels and the observed orders."""
    err = {}
    for l in levels:
        ue = exact_on_device(problem, problem.n_at(l))
        err["U_max_L%d" % l], _ = s.norms(l, E.VEC_U, minus=ue)
        s.extrapolate(l, out=False)
        err["Ut_max_L%d" % l], _ = s.norms(l, E.VEC_UTILDE, minus=ue)
        del ue
    a, b = levels[-2], levels[-1]
    return err, math.log2(err["Ut_max_L%d" % a] / err["Ut_max_L%d" % b])


def _timed_solves(torch, fn, reps=2):
    fn()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out = None
    for _ in range(reps):
        out = fn()
    torch.cuda.synchronize()
    return out, (time.perf_counter() - t1) / reps


def fourth_order_search(E, torch, s, problem, desc, nodes):
    """Uniform eps from 1e-9 down to 1e-15 until U~ on the finest grid is fourth
    order (log2 of the max-error ratio to the next coarser grid >= 3.8) or stops
    changing (converged: the discretisation limits it); then the same finest
    tolerance as per-level schedules (each coarser grid 4x and 16x looser)."""
    L = problem.levels - 1
    s.set_timing(0)                      # no kernel events in these timings
    out = {"workload": desc, "uniform": []}
    prev = None
    for e4 in (1e-9, 1e-10, 1e-11, 1e-12, 1e-13, 1e-14, 1e-15):
        inf4, dt4 = _timed_solves(torch, lambda: s.solve(e4, extrapolate=True))
        err4, order = _finest_orders(E, s, problem, [L - 1, L])
        row = {"eps": e4, "ms_per_step": 1e3 * dt4, "value": nodes / dt4, "Ut_order_max": order,
               "iters": [i["iters"] for i in inf4], **err4}
        out["uniform"].append(row)
        print("bench: eps %g: %.2f ms/step, Ut order %.2f" % (e4, 1e3 * dt4, order), file=sys.stderr, flush=True)
        ut = err4["Ut_max_L%d" % L]
        if order >= 3.8:
            out["reached"] = row
            break
        if prev is not None and abs(ut / prev - 1.0) < 1e-3:
            out["converged"] = row          # U~ no longer moves with eps
            break
        prev = ut
    last = out.get("reached") or out.get("converged") or out["uniform"][-1]
    for ratio in (4.0, 16.0):
        sched = E.tolerance_schedule(problem.levels, last["eps"], ratio)

        def run():
            r = s.solve_levels(sched)
            s.extrapolate(L, out=False)
            return r
        infs, dts = _timed_solves(torch, run)
        errs, order = _finest_orders(E, s, problem, [L - 1, L])
        out["schedule%d" % ratio] = {"rel_tol": sched, "ms_per_step": 1e3 * dts, "value": nodes / dts,
                                     "Ut_order_max": order, "iters": [i["iters"] for i in infs], **errs}
        print("bench: schedule (finest eps %g, ratio %g): %.2f ms/step, Ut order %.2f" %
              (last["eps"], ratio, 1e3 * dts, order), file=sys.stderr, flush=True)
    torch.cuda.empty_cache()
    return out


def fourth_order_problem1(E, torch):
    """The paper's Problem 1 (beta = 1, three Neumann faces) on its seven grids
    8^3 .. 512^3 (Section 5): the loosest eps at which U~ is fourth order on the
    512^3 grid, with unknowns/s at that eps (solve + EXP_true, device fields)."""
    import workloads
    p = workloads.paper_problem1(levels=7, eps=1e-10)
    L = p.levels - 1
    nodes = p.nodes_at(L)
    out = {"workload": "Problem 1 of Section 5: -Laplace u = f, u = sin(pi x/2) sin(pi y/2) sin(pi z/2), "
                       "Dirichlet on x=0, y=0, z=0, Neumann elsewhere; 8^3 -> 512^3 elements (7 levels)",
           "uniform": []}
    with E.Solver(keep_w=False) as s:
        s.setup(p, device_fields=True)
        s.solve(1e-10, extrapolate=True)
        s.autotune(iters=0)
        for e4 in (1e-10, 1e-11, 1e-12, 1e-13, 1e-14):
            inf4, dt4 = _timed_solves(torch, lambda: s.solve(e4, extrapolate=True))
            err4, order = _finest_orders(E, s, p, [L - 1, L])
            row = {"eps": e4, "ms_per_step": 1e3 * dt4, "value": nodes / dt4, "Ut_order_max": order,
                   "iters": [i["iters"] for i in inf4], **err4}
            out["uniform"].append(row)
            print("bench: problem 1 eps %g: %.2f ms/step, Ut order %.2f" % (e4, 1e3 * dt4, order),
                  file=sys.stderr, flush=True)
            if order >= 3.8:
                out["reached"] = row
                break
    torch.cuda.empty_cache()
    return out


def precision_comparison(E, torch, name="high-contrast-513x257x257", steps=3):
    """FP64 and mixed precision on the same GPU and workload: ms per step
    (solve + finest EXP_true) and max-norm errors of U and U~ vs the exact
    solution on the finest grid."""
    problem, desc = workload(name)
    L = problem.levels - 1
    nodes = problem.nodes_at(L)
    res = {"workload": desc}
    for prec, tag in ((E.FP64, "fp64"), (E.MIXED, "mixed")):
        with E.Solver(precision=prec, keep_w=False) as s:
            s.setup(problem, device_fields=True)
            s.solve(problem.eps, extrapolate=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                infos = s.solve(problem.eps, extrapolate=True)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            ue = exact_on_device(problem, problem.n_at(L))
            eu, _ = s.norms(L, E.VEC_U, minus=ue)
            et, _ = s.norms(L, E.VEC_UTILDE, minus=ue)
            del ue
            res[tag] = {"ms_per_step": 1e3 * dt, "value": nodes / dt, "U_max": eu, "Ut_max": et,
                        "iters": [i["iters"] for i in infos], "outer_steps": [i["outer_steps"] for i in infos]}
        torch.cuda.empty_cache()
        print("bench: %s on %s: %.2f ms/step, |U-u| %.3e, |U~-u| %.3e" % (tag, name, 1e3 * dt, eu, et),
              file=sys.stderr, flush=True)
    res["speedup_mixed"] = res["fp64"]["ms_per_step"] / res["mixed"]["ms_per_step"]
    res["error_ratio_U"] = res["mixed"]["U_max"] / res["fp64"]["U_max"]
    res["error_ratio_Ut"] = res["mixed"]["Ut_max"] / res["fp64"]["Ut_max"]
    return res


def method_comparison(E, torch, problem, desc, steps=3):
    """ECMG_jcg and ECMG_cg (Algorithm 4 with plain CG, the comparison of the
    paper's Tables iterations8-10) on the same workload and GPU: ms per step
    (solve + finest EXP_true), CG iterations per level, finest-grid errors."""
    L = problem.levels - 1
    nodes = problem.nodes_at(L)
    res = {"workload": desc}
    for method, tag in ((E.JCG, "ecmg_jcg"), (E.CG, "ecmg_cg")):
        with E.Solver(method=method, keep_w=False) as s:
            s.setup(problem, device_fields=True)
            s.solve(problem.eps, extrapolate=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                infos = s.solve(problem.eps, extrapolate=True)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            ue = exact_on_device(problem, problem.n_at(L))
            eu, _ = s.norms(L, E.VEC_U, minus=ue)
            et, _ = s.norms(L, E.VEC_UTILDE, minus=ue)
            del ue
            res[tag] = {"ms_per_step": 1e3 * dt, "value": nodes / dt, "U_max": eu, "Ut_max": et,
                        "iters": [i["iters"] for i in infos]}
        torch.cuda.empty_cache()
        print("bench: %s: %.2f ms/step, iterations %s, |U~-u| %.3e" % (tag, 1e3 * dt, res[tag]["iters"], et),
              file=sys.stderr, flush=True)
    res["speedup_jcg"] = res["ecmg_cg"]["ms_per_step"] / res["ecmg_jcg"]["ms_per_step"]
    return res


def batched(E, torch, n_boxes=512, steps=3):
    """512 independent three-level solves (uneven boxes) through the batched
    API: one step = ecmg_solve_batch + ecmg_extrapolate_batch over all boxes,
    replayed from the HIP graph the first solve captures; the same steps launch
    by launch (a leading context with options.batch_graph = 0) for the per-level
    device times."""
    import tempfile
    import workloads
    probs = workloads.batched_mix(n_boxes, seed=0)
    t0 = time.perf_counter()
    solvers = [E.Solver(keep_w=False, dsolve_dense_max=0).setup(p, device_fields=True) for p in probs]
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    nodes = sum(p.nodes_at(p.levels - 1) for p in probs)
    eps = probs[0].eps
    cache = os.path.join(tempfile.mkdtemp(prefix="ecmg_batch_"), "tune.json")
    t0 = time.perf_counter()
    tuned = E.autotune_batch(solvers, eps, cache=cache)   # untimed: every box takes the fastest setting
    tune_s = time.perf_counter() - t0
    print("bench: batched autotune %.2f s: %d nodes per workgroup, segments of %d (%.1f -> %.1f ms)" % (
        tune_s, tuned["nodes_per_workgroup"], tuned["seg"], tuned["us_default"] / 1e3, tuned["us_best"] / 1e3),
        file=sys.stderr, flush=True)

    def timed(lst):
        E.solve_batch(lst, eps)                          # captures the graph (or not) and warms up
        E.extrapolate_batch(lst)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        inf = None
        for _ in range(steps):
            inf = E.solve_batch(lst, eps)
            E.extrapolate_batch(lst)
        torch.cuda.synchronize()
        return inf, (time.perf_counter() - t1) / steps

    infos, dt = timed(solvers)
    lead = E.Solver(keep_w=False, dsolve_dense_max=0, batch_graph=False, autotune=1, tune_cache=cache)
    lead.setup(probs[0], device_fields=True)
    infos_e, dt_e = timed([lead] + solvers[1:])
    lead.close()
    # the same boxes one by one through ecmg_solve (a sample of 64) for context
    t0 = time.perf_counter()
    for sv in solvers[:64]:
        sv.solve(eps, extrapolate=True)
    torch.cuda.synchronize()
    seq = (time.perf_counter() - t0) * n_boxes / 64
    it = [i[-1]["iters"] for i in infos]
    for sv in solvers:
        sv.close()
    return {"boxes": n_boxes, "finest_nodes_total": nodes, "setup_s": setup_s, "ms_per_step": 1e3 * dt,
            "boxes_per_s": n_boxes / dt, "unknowns_per_s": nodes / dt,
            "graph": "replayed HIP graph of one cooperative launch that runs every box's three levels "
                     "(captured by the first solve)",
            "ms_per_step_launch_by_launch": 1e3 * dt_e,
            "level_ms": [infos_e[0][l]["ms"] for l in range(3)],
            "finest_iters_mean": sum(it) / len(it), "finest_iters_max": max(it),
            "sequential_ms_estimate": 1e3 * seq, "speedup_vs_sequential": seq / dt, "autotune": tuned}


def serving(E, n_measured=2000, n_warmup=100, rate=50.0, budget=200 * 10 ** 9):
    """Replay a seeded Poisson stream of requests (finest 32^3..256^3,
    random coefficients and faces) against the serving loop; latency is from
    each request's scheduled arrival to its U~ on the host."""
    import workloads
    stream = workloads.serving_stream(n_measured + n_warmup, rate, seed=1)
    lat, sizes = [], []
    t_submit = t_step = 0.0
    with E.Server(budget) as srv:
        t0 = time.perf_counter()
        nxt, live, t_first = 0, {}, None
        while nxt < len(stream) or live:
            now = time.perf_counter() - t0
            while nxt < len(stream) and stream[nxt].arrival_s <= now:
                live[srv.submit(stream[nxt].problem, stream[nxt].problem.eps)] = nxt
                nxt += 1
            t_submit += time.perf_counter() - t0 - now
            if not live:
                time.sleep(max(0.0, stream[nxt].arrival_s - (time.perf_counter() - t0)))
                continue
            ts = time.perf_counter()
            srv.step()
            t_step += time.perf_counter() - ts
            tnow = time.perf_counter() - t0
            for t in srv.completed():
                k = live[t]
                st, _ = srv.poll(t)
                if st == 2 or st < 0:
                    if st < 0:
                        raise RuntimeError("request %d failed with status %d" % (k, st))
                    if k >= n_warmup:
                        lat.append(1e3 * (tnow - stream[k].arrival_s))
                        sizes.append(stream[k].problem.nodes_at(stream[k].problem.levels - 1))
                        if t_first is None:
                            t_first = stream[k].arrival_s
                        if len(lat) % 500 == 0:
                            print("bench: serving %d of %d measured requests done (%.1f s)"
                                  % (len(lat), n_measured, tnow), file=sys.stderr, flush=True)
                    srv.release(t)
                    del live[t]
        t_end = time.perf_counter() - t0
        internal = srv.stats()
    lat = sorted(lat)
    pct = lambda q: lat[min(len(lat) - 1, max(0, int(math.ceil(q * len(lat))) - 1))]
    span = t_end - t_first
    return {"requests": n_measured, "warmup": n_warmup, "rate_per_s": rate, "budget_bytes": budget,
            "p50_ms": pct(0.5), "p99_ms": pct(0.99), "max_ms": lat[-1],
            "solves_per_s": n_measured / span, "unknowns_per_s": sum(sizes) / span,
            "latency_from": "scheduled arrival to U~ on the host (setup included)",
            "driver_s": {"submit": t_submit, "step": t_step, "total": t_end},
            "server_internal": internal}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="variable-beta-robin-513")
    ap.add_argument("--eps", type=float, default=None)
    ap.add_argument("--interp", type=int, default=0)
    ap.add_argument("--host-fields", action="store_true", help="sample fields with numpy on the host")
    ap.add_argument("--cpu-levels", type=int, default=6, help="levels of the oracle CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", type=int, default=1, choices=(0, 1),
                    help="time the JCG configurations of every level after the warm-up (untimed) and keep the "
                         "fastest; 0 = the built-in heuristics")
    ap.add_argument("--tune-cache", default=None, help="JSON tuning cache to merge the choices into")
    ap.add_argument("--tuned-from", default=None, metavar="CACHE",
                    help="apply the choices of an existing tuning cache at setup instead of tuning (profiled runs: "
                         "no candidate launches)")
    ap.add_argument("--no-errors", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run one device copy kernel (read BYTES, write BYTES) and exit: the reference "
                         "for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE")
    ap.add_argument("--no-method-comparison", action="store_true",
                    help="skip ECMG_jcg vs ECMG_cg (plain CG) on the same workload")
    ap.add_argument("--no-precision-comparison", action="store_true",
                    help="skip the FP64 vs mixed comparison on the high-contrast workload")
    ap.add_argument("--batch-boxes", type=int, default=512, help="boxes of the batched workload (0 = skip)")
    ap.add_argument("--serve-requests", type=int, default=2000,
                    help="measured requests of the serving replay (0 = skip), after 100 warm-up requests")
    ap.add_argument("--roofline-kernel", default=None, metavar="SYMBOL",
                    help="the roofline kernel (as the bench line names it) instead of the one with the largest "
                         "total time, e.g. the choice of an unprofiled run when this run is profiled")
    ap.add_argument("--no-fourth-order", action="store_true",
                    help="skip the search for the eps that keeps the extrapolation fourth order")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the solver runs on a single GPU (one device per context); "
              "--gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        n = args.copy_calibration // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": 8 * n, "kernel": "torch.mul(src, 1.0, out=dst)"}))
        return
    import paper_1506_02983_amd as E

    problem, desc = workload(args.workload)
    eps = problem.eps if args.eps is None else args.eps
    torch.cuda.init()
    L = problem.levels - 1
    n = problem.n_at(L)
    nodes = problem.nodes_at(L)
    elems = n[0] * n[1] * n[2]

    if args.tuned_from:
        args.autotune = 0
        s = E.Solver(interp=args.interp, timing=True, keep_w=False, autotune=1, tune_cache=args.tuned_from)
    else:
        s = E.Solver(interp=args.interp, timing=True, keep_w=False)
    t0 = time.perf_counter()
    s.setup(problem, device_fields=not args.host_fields)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    print("bench: setup %.2f s (%s fields)" % (setup_s, "host" if args.host_fields else "device"),
          file=sys.stderr, flush=True)

    for _ in range(max(args.warmup, 1 if args.autotune else 0)):
        s.solve(eps, extrapolate=True)
    tuned = None
    if args.autotune:
        # each level timed over its iteration count in the warm-up solve
        t0 = time.perf_counter()
        tuned = s.autotune(iters=0, cache=args.tune_cache)
        print("bench: autotune %.2f s: %s" % (time.perf_counter() - t0, ", ".join(
            "L%d %s" % (r["level"], ("tiled kz=%d" % r["kz"]) if r["path"] == "tiled" else "gather"
                        if r["path"] == "gather" else "persistent seg=%d nwg=%d" % (r["seg"], r["nwg"]))
            for r in tuned)), file=sys.stderr, flush=True)
        s.solve(eps, extrapolate=True)
    # per-kernel breakdown: two untimed steps with every kernel class timed
    # (HIP events around each launch, which lengthen the launch-bound levels)
    s.set_timing(-1)
    torch.cuda.synchronize()
    s.reset_kernel_times()
    for _ in range(2):
        infos_b = s.solve(eps, extrapolate=True)
    kernels = []
    for l in range(problem.levels):
        nl = problem.n_at(l)
        nn = problem.nodes_at(l)
        ee = nl[0] * nl[1] * nl[2]
        n1 = problem.nodes_at(l - 1) if l >= 1 else 0
        n0 = problem.nodes_at(l - 2) if l >= 2 else 0
        for k in sorted(KIND_NAMES):
            ms, cnt = s.kernel_times(l, k)
            if cnt == 0:
                continue
            b = algorithmic_bytes(k, nn, ee, n1, n0, infos_b[l]["iters"])
            kernels.append({"level": l, "kernel": KIND_NAMES[k], "kind": k,
                            "symbol": kernel_symbol(k, infos_b[l]["path"], nl[0], E), "launches": cnt,
                            "total_ms": ms, "avg_us": 1e3 * ms / cnt, "bytes_per_launch": b,
                            "gbs": b / (ms / cnt * 1e-3) / 1e9, "nodes": nn})
    # the dominant kernel: largest total time, summed over all its launches
    # (every level it runs on), as rocprofv3 reports it per kernel name
    by_sym = {}
    for r in kernels:
        by_sym[r["symbol"]] = by_sym.get(r["symbol"], 0.0) + r["total_ms"]
    dsym = args.roofline_kernel if args.roofline_kernel in by_sym else max(by_sym, key=by_sym.get)
    # the (level, class) pairs it ran as (a pair of kernels can serve two classes)
    dpairs = sorted({(r["level"], r["kind"]) for r in kernels if r["symbol"] == dsym})
    dkinds = sorted({k for _, k in dpairs})

    # timed region: no events (a timed launch costs about 5 us more, which the
    # launch-bound levels would add to the step)
    s.set_timing(0)
    torch.cuda.synchronize()
    infos = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos = s.solve(eps, extrapolate=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = 1e3 * dt / args.steps
    value = nodes * args.steps / dt
    print("bench: %.3f ms/step, %.3e unknowns/s" % (ms_per_step, value), file=sys.stderr, flush=True)

    # roofline region: the same steps again with events (stamped by each
    # launch of the dominant kernel itself) around that kernel only
    s.set_timing(dkinds)
    s.reset_kernel_times()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos_r = s.solve(eps, extrapolate=True)
    torch.cuda.synchronize()
    region_ms = 1e3 * (time.perf_counter() - t0) / args.steps

    d = {"total_ms": 0.0, "launches": 0, "bytes": 0.0}
    for l, dkind in dpairs:
        ms, cnt = s.kernel_times(l, dkind)
        if cnt == 0:
            continue
        nl = problem.n_at(l)
        b = algorithmic_bytes(dkind, problem.nodes_at(l), nl[0] * nl[1] * nl[2],
                              problem.nodes_at(l - 1) if l >= 1 else 0, problem.nodes_at(l - 2) if l >= 2 else 0,
                              infos_r[l]["iters"])
        d["total_ms"] += ms
        d["launches"] += cnt
        d["bytes"] += b * cnt
    s.set_timing(-1)
    achieved = d["bytes"] / (d["total_ms"] * 1e-3) / 1e9
    traffic = measured_traffic(dsym, d["launches"] / args.steps)
    traffic = round(traffic) if traffic else None
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": dsym, "classes": [KIND_NAMES[k] for k in dkinds],
                "levels": sorted({l for l, _ in dpairs}), "launches": d["launches"],
                "avg_us": round(1e3 * d["total_ms"] / d["launches"], 2),
                "bytes_per_launch": round(d["bytes"] / d["launches"]),
                "region": "%d steps after the timed ones, HIP events only around this kernel's launches "
                          "(%.3f ms/step)" % (args.steps, region_ms)}
    # the finest level's kernels against the same HBM peak (from the breakdown
    # steps: every launch stamped; algorithmic bytes as above)
    finest = [{"kernel": r["kernel"], "symbol": r["symbol"], "launches": r["launches"],
               "avg_us": round(r["avg_us"], 2), "achieved": round(r["gbs"], 1),
               "frac": round(r["gbs"] / HBM_PEAK_GBS, 4), "bytes_per_launch": r["bytes_per_launch"]}
              for r in kernels if r["level"] == L]
    jcg_fin = [r for r in kernels if r["level"] == L and r["kind"] in (0, 1, 10, 11, 12)]
    jcg_gbs = None
    if jcg_fin:
        tb = sum(r["bytes_per_launch"] * r["launches"] for r in jcg_fin)
        tt = sum(r["total_ms"] for r in jcg_fin) * 1e-3
        jcg_gbs = tb / tt / 1e9

    errors = {}
    if not args.no_errors:
        for l in (L - 1, L):
            ue = exact_on_device(problem, problem.n_at(l))
            errors["U_max_L%d" % l], errors["U_l2_L%d" % l] = s.norms(l, E.VEC_U, minus=ue)
            s.extrapolate(l, out=False)
            errors["Ut_max_L%d" % l], errors["Ut_l2_L%d" % l] = s.norms(l, E.VEC_UTILDE, minus=ue)
            del ue
        errors["U_order_max"] = math.log2(errors["U_max_L%d" % (L - 1)] / errors["U_max_L%d" % L])
        errors["Ut_order_max"] = math.log2(errors["Ut_max_L%d" % (L - 1)] / errors["Ut_max_L%d" % L])
        torch.cuda.empty_cache()

    # if eps loses fourth order on the finest grid (the stop test is relative to
    # ||f_h||, reading of Section 5), search tighter tolerances: the first that
    # keeps it, or the point where U~ stops changing (the algebraic error is
    # gone and the discretisation sets the order)
    fourth = None
    if not args.no_errors and errors.get("Ut_order_max", 0.0) < 3.8 and not args.no_fourth_order:
        fourth = fourth_order_search(E, torch, s, problem, desc, nodes)
    s.close()
    torch.cuda.empty_cache()
    if not args.no_errors and not args.no_fourth_order:
        p1 = fourth_order_problem1(E, torch)
        if fourth is None:
            fourth = {}
        fourth["problem1"] = p1
    prec_cmp = None
    if not args.no_precision_comparison:
        prec_cmp = precision_comparison(E, torch)
    meth_cmp = None
    if not args.no_method_comparison:
        meth_cmp = method_comparison(E, torch, problem.with_(eps=eps), desc)

    batch = None
    if args.batch_boxes > 0:
        batch = batched(E, torch, args.batch_boxes)
        print("bench: batched %d boxes: %.2f ms/step, %.0f boxes/s" % (batch["boxes"], batch["ms_per_step"],
                                                                     batch["boxes_per_s"]),
              file=sys.stderr, flush=True)
        torch.cuda.empty_cache()

    serve = None
    if args.serve_requests > 0:
        serve = serving(E, n_measured=args.serve_requests)
        print("bench: serving p50 %.1f ms, p99 %.1f ms, %.1f solves/s" % (serve["p50_ms"], serve["p99_ms"],
                                                                          serve["solves_per_s"]),
              file=sys.stderr, flush=True)
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(problem.with_(eps=eps), min(args.cpu_levels, problem.levels), args.interp)
        print("bench: cpu baseline %.3e unknowns/s on %d threads" % (cpu["value"], cpu["cores"]),
              file=sys.stderr, flush=True)

    out = {
        "metric": METRIC, "value": value, "unit": "unknowns/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic (closed-form manufactured solution)",
        "config": {"workload": desc, "levels": problem.levels, "finest_elements": list(n), "finest_nodes": nodes,
                   "eps": eps, "precision": "fp64",
                   "interp": "lagrange27" if args.interp else "serendipity20", "parallelism": "single GPU",
                   "jcg_configuration": ("from tuning cache" if args.tuned_from else
                                         "autotuned" if args.autotune else "built-in")},
        "autotune": tuned,
        "roofline": roofline,
        "roofline_finest": {"level": L, "bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s", "kernels": finest},
        "cpu_baseline": cpu,
        "jcg_hbm_gbs_finest": jcg_gbs,
        "fourth_order": fourth,
        "precision_comparison": prec_cmp,
        "method_comparison": meth_cmp,
        "batched": batch,
        "serving": serve,
        "setup_s": setup_s,
        "levels": [{"level": i["level"], "n": [i["nx"], i["ny"], i["nz"]], "iters": i["iters"],
                    "rre": i["rre"], "ms": i["ms"]} for i in infos],
        "errors": errors,
        "kernels_note": "per-kernel breakdown from 2 untimed steps with every kernel class timed; the timed "
                        "steps record no events, the roofline region's only around the roofline kernel",
        "kernels": [{k: (round(v, 3) if isinstance(v, float) else v) for k, v in r.items()} for r in kernels],
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
