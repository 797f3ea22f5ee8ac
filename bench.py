"""PDHG throughput of the gfx950 PDLP solver on the large plain LP (m=1e6, n=2e6, Zipf(1.5)
column counts, nnz ~1.35e8), one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-batched]
                    [--no-unroll] [--no-truncated] [--no-pagerank] [--no-policies]
                    [--no-ablations] [--only-large | --only-lp truncated|pagerank | --only-unroll]
                    [--calibrate-copy]
    python bench.py --summarize-profile DIR     # text summary of the rocprofv3 runs in DIR
    python bench.py --summarize-unroll DIR      # the same for a trace of --only-unroll

A step is one accepted PDHG iteration of Algorithm 1 on the whole LP: the K~^T product fused
with the primal step, the K~ product fused with the dual step and the step-size rule, and
(every 40 steps) the restart / termination check.  The LP is resident in HBM before timing
starts.  Prints one JSON line.  Progress goes to stderr.

Three timed windows per LP, one after the other on the same solver:
  * the headline: W warmup steps, then exactly K steps as pdlp_solve runs them (whole blocks of
    40 attempt slots replayed as HIP graphs, a block cut short at the iteration limit), wall
    clock bracketed by device synchronisation; `value` = K / seconds;
  * kernel timing: the next K steps with HIP events around every pass of every attempt slot
    (kernel by kernel, one block at a time), giving each pass's average duration over the
    slots that ran: the `roofline` of the dominant kernel;
  * whole check blocks: from the next multiple of 40, max(5, ceil(K / 40)) blocks of 40 steps,
    each ending with its restart / termination check: `check_inclusive`.
Beside the headline the line carries the same figures for the same shape with column counts
truncated to [1,190] and for the PageRank LP on 5e6 nodes, a whole solve of the tiny LP, the
constant-step and Malitsky-Pock policies, the ablation switches' steps to KKT 1e-8 on two
small LPs, the batched solver, the unrolled PDHG and its adjoint, and the oracle's rate on
the host.
"""
from __future__ import annotations

import argparse
import glob
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, vendor figure
CHECK_EVERY = 40


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


# rocprofv3 summaries of the step passes per workload (bench.py --summarize-profile)
PROFILES = {"large": os.path.join(ROOT, "profiles", "pdlp_step_passes_large_plain_lp.txt"),
            "truncated": os.path.join(ROOT, "profiles", "pdlp_step_passes_truncated_large_lp.txt"),
            "pagerank": os.path.join(ROOT, "profiles", "pdlp_step_passes_pagerank_5m.txt")}

# Sources that define the timed step kernels and their launches (the batched solver and the
# unrolled adjoint live in files of their own and do not take part in the timed step).
STEP_SOURCES = ["pdlp_kernels.hip", "pdlp_solver.hip", "pdlp_device.h", "pdlp_internal.h",
                "host_prep.cpp", "host_prep.h"]

PASS_NAMES = ["primal_pass1", "primal_combine", "dual_pass1", "dual_combine"]
PASS_DOC = {
    "primal_pass1": "K~^T y product, first pass (k_lds_rows<1>: panel rows of LDS slices of y; "
                    "k_panel_rows<1> without the stage)",
    "primal_combine": "panel partials of K~^T y added per row, primal update of Eq. (3) and its "
                      "reductions (k_primal_combine; k_primal in the plain layout does both passes)",
    "dual_pass1": "K~ x' product, first pass (k_lds_rows<0>: XCD panels, hottest x' entries staged "
                  "in LDS; k_panel_rows<0> without the stage)",
    "dual_combine": "panel partials of K~ x' added per row, dual update of Eq. (3), the Eq. (5) "
                    "reductions and the step-size tail (k_dual_combine + k_tail; k_dual in the plain "
                    "layout does both passes)",
}
# kernel symbol of each pass per copy layout (1 panels, 2 slices, 3 panels with a stage)
PASS_KERNELS = {
    "primal_pass1": {1: "k_panel_rows<1>", 2: "k_lds_rows<1>", 3: "k_lds_rows<1>"},
    "primal_combine": {0: "k_primal", 1: "k_primal_combine", 2: "k_primal_combine", 3: "k_primal_combine"},
    "dual_pass1": {1: "k_panel_rows<0>", 2: "k_lds_rows<0>", 3: "k_lds_rows<0>"},
    "dual_combine": {0: "k_dual", 1: "k_dual_combine", 2: "k_dual_combine", 3: "k_dual_combine"},
}


def kernel_sources_digest():
    """sha256 over the sources of the timed step kernels (names and contents)."""
    import hashlib
    h = hashlib.sha256()
    for f in [os.path.join(ROOT, "paper_2106_04756_amd", "csrc", f) for f in STEP_SOURCES]:
        h.update(os.path.relpath(f, ROOT).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_bytes(which="large"):
    """HBM bytes per product dispatch of each step kernel on one workload, from the rocprofv3
    byte counters in its committed profile summary; None when the summary was taken on other
    kernel sources."""
    try:
        with open(PROFILES[which]) as fh:
            for line in fh:
                if line.startswith("bench-traffic: "):
                    d = json.loads(line[len("bench-traffic: "):])
                    if d["sources_sha256"] == kernel_sources_digest():
                        return d["bytes_per_dispatch"]
    except (OSError, ValueError, KeyError):
        pass
    return None


def host_cpu():
    """CPU model and the cores this process may run on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "host_cores": len(os.sched_getaffinity(0))}


def cpu_baseline(lp, budget_s=20.0):
    """The oracle's PDHG attempts (Eq. (3) + Algorithm 2 rule) on the same LP, single thread,
    timed on a bounded sample of iterations."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import pdlp_oracle as O

    K = lp.K()
    KT = K.T.tocsr()
    x = np.clip(np.zeros(lp.n), lp.l, lp.u)
    y = np.zeros(lp.m)
    eta = 1.0 / float(np.max(np.abs(K.data)))
    omega = O.initial_primal_weight(lp.c, lp.q, 1e-10)
    iters = 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while True:
            xp, yp = O.pdhg_step(x, y, eta, omega, lp.c, K, KT, lp.q, lp.l, lp.u, lp.m1)
            eta_bar = O.step_size_limit(xp - x, yp - y, omega, K)
            eta_next = O.next_step_size(eta_bar, eta, iters + 1)
            if eta <= eta_bar:
                x, y = xp, yp
                iters += 1
            eta = eta_next
            el = time.perf_counter() - t0
            if el >= budget_s or iters >= 50:
                break
    out = dict(value=iters / el, unit="PDHG iters/s", cores=1, kind="oracle",
               sample=f"{iters} accepted oracle PDHG steps (Eq. (3) + Algorithm 2, unpreconditioned, "
                      f"scipy CSR products, 1 thread; the step-size limit forms K dx as a third "
                      f"product) on the same LP, {el:.1f} s")
    out.update(host_cpu())
    return out


def pass_bytes(lp):
    """Algorithmic bytes of one launch of each pass when it forms its product (int64 row
    offsets, int32 columns and float64 values of the CSR copy, the gathered vector once, each
    other vector once): the first passes move the matrix and the gathered vector, the combines
    the vectors of the update (primal: read x, c, l, u, S_x, write x', S_x, K~^T y; dual: read
    y, q, K~x, S_y, write y', K~x', S_y)."""
    m, n, nnz = lp.m, lp.n, lp.nnz
    return {"primal_pass1": 12.0 * nnz + 8.0 * (n + 1) + 8.0 * m, "primal_combine": 64.0 * n,
            "dual_pass1": 12.0 * nnz + 8.0 * (m + 1) + 8.0 * n, "dual_combine": 56.0 * m}


def measure_lp(P, torch, lp, W, K, tol=1e-8, label="lp"):
    """The three timed windows of the module docstring on one LP.  Returns a dict."""
    t = time.time()
    s = P.Solver.from_lp(lp)
    inf = s.info()
    log(f"{label}: created solver in {time.time() - t:.1f}s (library create {inf['create_seconds']:.1f}s); "
        f"layouts K~ {inf['layout_K']} ({inf['panels_K']} panels), K~^T {inf['layout_KT']} ({inf['panels_KT']} panels)")
    s.solve(tol, W)
    # 1. headline window: exactly K steps as a solve runs them
    i0 = s.info()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = s.solve(tol, i0["iterations"] + K)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    i1 = s.info()
    steps = i1["iterations"] - i0["iterations"]
    log(f"{label}: headline {steps} steps in {dt:.4f}s = {steps / dt:.1f} iters/s "
        f"(status {P.STATUS_NAMES[st]}, checks {i1['checks'] - i0['checks']})")
    # 2. kernel timing over the next K steps
    s.set_kernel_timing(True)
    s.reset_kernel_times()
    j0 = s.info()
    s.solve(tol, j0["iterations"] + K)
    j1 = s.info()
    s.set_kernel_timing(False)
    tms, cnt = s.pass_times()
    d_att = j1["attempts"] - j0["attempts"]
    d_chk = j1["checks"] - j0["checks"]
    # products formed by the timed slots: a check forms two K~^T products (of the average and
    # of the current y) and one K~ product; the primal step skips its product when y has not
    # changed since it was formed (after a rejected attempt, and after a check)
    prim_products = (j1["spmv_KT"] - j0["spmv_KT"]) - 2 * d_chk
    dual_products = (j1["spmv_K"] - j0["spmv_K"]) - d_chk
    pb = pass_bytes(lp)
    plain_T, plain_K = inf["layout_KT"] == 0, inf["layout_K"] == 0
    alg = {"primal_pass1": 0.0 if plain_T else prim_products * pb["primal_pass1"],
           "primal_combine": cnt[1] * pb["primal_combine"] + (prim_products * pb["primal_pass1"] if plain_T else 0.0),
           "dual_pass1": 0.0 if plain_K else dual_products * pb["dual_pass1"],
           "dual_combine": cnt[3] * pb["dual_combine"] + (dual_products * pb["dual_pass1"] if plain_K else 0.0)}
    passes = {}
    for j, name in enumerate(PASS_NAMES):
        launches = int(cnt[j])
        ms = float(tms[j]) / max(launches, 1)
        bpl = alg[name] / max(launches, 1)
        passes[name] = {"avg_us": 1e3 * ms, "launches": launches, "algorithmic_bytes_per_launch": bpl,
                        "algorithmic_bytes_per_product": pb[name] + (pb[name.replace("combine", "pass1")]
                                                                     if (name == "primal_combine" and plain_T)
                                                                     or (name == "dual_combine" and plain_K) else 0.0),
                        "achieved_gbs": bpl / (ms * 1e-3) / 1e9 if ms > 0 else None}
    slots = {}
    for slot, (a, b) in (("primal", ("primal_pass1", "primal_combine")), ("dual", ("dual_pass1", "dual_combine"))):
        ms = (tms[PASS_NAMES.index(a)] + tms[PASS_NAMES.index(b)]) / max(int(cnt[0]), 1)
        by = (alg[a] + alg[b]) / max(int(cnt[0]), 1)
        slots[slot] = {"avg_us": 1e3 * ms, "algorithmic_bytes_per_launch": by,
                       "achieved_gbs": by / (ms * 1e-3) / 1e9 if ms > 0 else None,
                       "frac": (by / (ms * 1e-3) / 1e9) / HBM_PEAK_GBS if ms > 0 else None}
    dom = max(PASS_NAMES, key=lambda nm: tms[PASS_NAMES.index(nm)])
    lay = inf["layout_KT"] if dom.startswith("primal") else inf["layout_K"]
    roof = {"bound": "hbm", "kernel": PASS_KERNELS[dom].get(lay, "?") + ": " + PASS_DOC[dom],
            "achieved": passes[dom]["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": (passes[dom]["achieved_gbs"] or 0.0) / HBM_PEAK_GBS, "traffic": None,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled)",
            "avg_launch_ms": passes[dom]["avg_us"] * 1e-3, "launches": passes[dom]["launches"],
            "algorithmic_bytes_per_launch": passes[dom]["algorithmic_bytes_per_launch"],
            "pass": dom, "timing": f"HIP events on the solver's stream around each pass of the {d_att} attempt "
                                   f"slots that ran in the {K} steps after the headline window"}
    log(f"{label}: passes " + ", ".join(f"{k} {v['avg_us']:.1f}us" for k, v in passes.items())
        + f"; dominant {dom} at {roof['frac'] * 100:.1f}% of HBM peak")
    # 3. whole check blocks
    k = s.info()["iterations"]
    start = -(-k // CHECK_EVERY) * CHECK_EVERY
    s.solve(tol, start)
    nb = max(5, -(-K // CHECK_EVERY))
    c0 = s.info()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.solve(tol, c0["iterations"] + nb * CHECK_EVERY)
    torch.cuda.synchronize()
    cdt = time.perf_counter() - t0
    c1 = s.info()
    csteps = c1["iterations"] - c0["iterations"]
    check_incl = {"iters_per_s": csteps / cdt, "steps": csteps, "checks": c1["checks"] - c0["checks"],
                  "seconds": cdt, "first_step": c0["iterations"] + 1}
    log(f"{label}: {csteps} steps with {check_incl['checks']} checks in {cdt:.4f}s = {csteps / cdt:.1f} iters/s")
    kkt = c1["kkt"][3]
    s.close()
    return {"steps_taken": steps, "seconds": dt, "iters_per_s": steps / dt, "roofline": roof,
            "passes": passes, "slots": slots, "check_inclusive": check_incl,
            "step_gbs_algorithmic": inf["step_bytes"] * steps / dt / 1e9, "kkt_at_end": kkt,
            "attempts_per_step_timed": d_att / max(j1["iterations"] - j0["iterations"], 1),
            "create_seconds": inf["create_seconds"],
            "layouts": {"K": inf["layout_K"], "KT": inf["layout_KT"]}}


def attach_traffic(r, lp, which="large"):
    """roofline.traffic of the dominant pass: the HBM bytes per product dispatch of its kernel
    in the committed profile, scaled to the timed launches (a first pass after a rejected
    attempt returns at once: it moves no matrix); null when the profile was taken on other
    kernel sources or does not cover the kernel."""
    prof = profiled_bytes(which)
    roof = r["roofline"]
    kern = _match_kernel(roof["kernel"].split(":")[0], prof or {})
    if not kern:
        return
    name = roof["pass"]
    full = pass_bytes(lp)[name]
    per_launch = r["passes"][name]["algorithmic_bytes_per_launch"]
    frac = per_launch / full if name.endswith("pass1") else 1.0
    roof["traffic"] = prof[kern] * frac
    roof["traffic_over_algorithmic"] = roof["traffic"] / per_launch if per_launch else None


def bench_batched(P, lpgen, count, iter_limit, sample=32, oracle_budget_s=20.0, tune_steps=200):
    """LPs/s to KKT 1e-8 of the batched solver (one persistent launch per size class, one
    workgroup per LP, the workgroup size of each class picked by pdlp_batch_tune) on the
    batched workload; a loop of single-LP solves and the oracle on stratified samples of the
    same members, extrapolated to the whole workload."""
    import numpy as np
    t = time.time()
    lps = [lpgen.batched_instance(i) for i in range(count)]
    log(f"generated {count} batched members in {time.time() - t:.1f}s")
    b = P.Batch(lps)
    default_sizes, members = b.schedule()
    sizes = b.tune(tune_steps)
    tune_s = b.tune_seconds()
    log(f"batched: tuned schedules (threads x rows per thread) {sizes} for classes of {members} members "
        f"in {tune_s:.2f}s")
    secs = b.solve(1e-8, iter_limit)
    _, _, st, it, kkt = b.get()
    b.close()
    conv = int((st == P.OPTIMAL).sum())
    # stratified sample: evenly spaced in the order of m
    order = np.argsort([lp.m for lp in lps], kind="stable")
    idx = [int(order[int(i)]) for i in np.linspace(0, count - 1, sample)]
    t0 = time.perf_counter()
    pconv = 0
    for i in idx:
        s = P.Solver.from_lp(lps[i])
        pconv += s.solve(1e-8, iter_limit) == P.OPTIMAL
        s.close()
    pdt = time.perf_counter() - t0
    plain_est = pdt / len(idx) * count
    log(f"batched: {conv}/{count} at KKT 1e-8 in {secs:.2f}s; plain loop on {len(idx)} members "
        f"{pdt:.2f}s ({pconv} converged), {plain_est:.0f}s estimated for all {count}")
    out = {"workload": f"{count} LPs, m log-uniform in [50,2000], n = U[2,3] m, 3-8 nonzeros per "
                       f"column, seeds 3000+i", "tol": 1e-8, "iter_limit": iter_limit,
           "schedule": {"class_nonzeros": ["<2^11", "2^11..2^13", "2^13..2^15", ">=2^15"],
                        "members": members, "threads_x_rows": sizes, "untuned": default_sizes,
                        "tune_steps": tune_steps, "tune_seconds": tune_s},
           "seconds": secs, "count": count, "converged": conv, "not_converged": count - conv,
           "lps_per_s": count / secs if conv == count else None,
           "converged_per_s": conv / secs,
           "median_iterations": float(np.median(it)), "max_iterations": int(it.max()),
           "max_kkt_converged": float(kkt[st == 0, 3].max()) if conv else None,
           "plain_loop": {"sample": len(idx), "seconds": pdt, "converged": pconv,
                          "seconds_per_lp": pdt / len(idx), "estimated_seconds_all": plain_est},
           "speedup_vs_plain_loop_estimate": plain_est / secs}
    out["oracle"] = batched_oracle(lps, idx, oracle_budget_s, count)
    return out


def _oracle_member(lp):
    from threadpoolctl import threadpool_limits

    from oracle import pdlp_oracle as O
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        r = O.solve_lp(lp, tol=1e-8, iter_limit=20000)
        return time.perf_counter() - t0, int(r.status == O.OPTIMAL), int(r.k)


def batched_oracle(lps, idx, budget_s, count):
    """The oracle on members of the stratified sample: one thread (members in turn, within
    the budget) and a process pool over all host cores (one member per process)."""
    import multiprocessing as mp
    cpu = host_cpu()
    one = []
    t0 = time.perf_counter()
    for i in idx[::-1]:                                  # small members last
        if time.perf_counter() - t0 > budget_s and one:
            break
        one.append(_oracle_member(lps[i]))
    secs1 = sum(a for a, _, _ in one)
    cores = cpu["host_cores"]
    sub = [lps[i] for i in idx[: max(cores, 1) * 2]]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_member, sub, chunksize=1)
    secsN = time.perf_counter() - t0
    out = {"one_thread": {"members": len(one), "seconds": secs1, "converged": sum(c for _, c, _ in one),
                          "lps_per_s": len(one) / secs1 if secs1 > 0 else None},
           "all_cores": {"members": len(sub), "seconds": secsN, "processes": cores,
                         "converged": sum(c for _, c, _ in res), "lps_per_s": len(sub) / secsN},
           "note": "members from the stratified sample (largest first for one thread, smallest first "
                   "on all cores); iteration limit 20000", **cpu}
    log(f"batched oracle: 1 thread {len(one)} members in {secs1:.1f}s; {cores} processes {len(sub)} "
        f"members in {secsN:.1f}s")
    return out


def bench_step_policies(P, torch, lp, W=100, K=400):
    """PDHG iters/s on the bench LP under the other step policies (constant step, the
    Malitsky-Pock line search of Appendix C), each timed over K steps after W, with the
    attempts (line-search trials) per accepted step."""
    out = {}
    for name, kw in (("constant", dict(step_policy=1)), ("malitsky_pock", dict(step_policy=2))):
        s = P.Solver.from_lp(lp, **kw)
        s.solve(1e-8, W)
        i0 = s.info()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.solve(1e-8, W + K)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        i1 = s.info()
        s.close()
        steps = i1["iterations"] - i0["iterations"]
        out[name] = {"iters_per_s": steps / dt, "steps": steps, "seconds": dt,
                     "attempts_per_step": (i1["attempts"] - i0["attempts"]) / max(steps, 1)}
        log(f"step policy {name}: {steps / dt:.1f} iters/s, "
            f"{out[name]['attempts_per_step']:.2f} attempts per step")
    return out


# The switches of the paper's ablations (Appendix C), as solver options.
ABLATIONS = {
    "pdlp": {},
    "constant_step": dict(step_policy=1),
    "no_restarts": dict(adaptive_restarts=0),
    "no_restarts_weight_at_2j": dict(adaptive_restarts=0, pw_power_of_two=1),
    "restart_theory": dict(beta_sufficient=0.37, beta_necessary=0.37, restart_to_current=0),
    "fixed_weight": dict(primal_weight_update=0),
    "no_scaling": dict(ruiz_iters=0, pock_chambolle=0),
    "ruiz_only": dict(pock_chambolle=0),
    "pock_chambolle_only": dict(ruiz_iters=0),
    "malitsky_pock": dict(step_policy=2),
}


def bench_ablations(P, lpgen, tol=1e-8, iter_limit=50000):
    """The ablation switches on two synthetic LPs: PDHG steps (K~ and K~^T products) and seconds
    to the relative KKT error tol, or the iteration limit."""
    lps = {"tiny": lpgen.tiny_lp(),
           "pagerank_2e4": lpgen.pagerank_lp(2, 20000, name="PageRank LP 2e4 nodes out-degree 8")}
    out = {"tol": tol, "iter_limit": iter_limit,
           "workloads": {k: f"{lp.name} (nnz {lp.nnz})" for k, lp in lps.items()}, "runs": {}}
    for name, kw in ABLATIONS.items():
        row = {}
        for key, lp in lps.items():
            s = P.Solver.from_lp(lp, **kw)
            t0 = time.perf_counter()
            st = s.solve(tol, iter_limit)
            dt = time.perf_counter() - t0
            inf = s.info()
            s.close()
            row[key] = {"status": P.STATUS_NAMES[st], "iterations": inf["iterations"],
                        "spmv": inf["spmv_K"] + inf["spmv_KT"], "kkt": inf["kkt"][3], "seconds": dt}
        out["runs"][name] = row
        log(f"ablation {name}: " + ", ".join(f"{k} {v['status']} {v['iterations']} steps {v['seconds']:.2f}s"
                                             for k, v in row.items()))
    return out


def bench_unroll(P, lpgen, T=500, segment=50, reps=5):
    """Unrolled PDHG on the unroll LP (m=2e4, n=5e4, 6 nonzeros per column): wall time of the
    forward pass (T fixed steps) and of the adjoint (with checkpoint recomputation), median of
    reps, and the same with every step's masks kept (segment 0: no recomputation); the
    oracle's NumPy forward + reverse pass timed once beside it (1 thread)."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    lp, x_tgt = lpgen.unroll_lp()
    s = P.Solver.from_lp(lp)
    res = {}
    for seg in (segment, 0):
        f, b = [], []
        for r in range(reps + 1):
            x, _ = s.unroll_forward(lp.c, lp.q, T, seg)
            s.unroll_backward(2.0 * (x - x_tgt))
            inf = s.unroll_info()
            if r:
                f.append(inf["forward_seconds"])
                b.append(inf["backward_seconds"])
        fm, bm = float(np.median(f)), float(np.median(b))
        res[seg] = dict(forward_ms=fm * 1e3, backward_ms=bm * 1e3, forward_steps_per_s=T / fm,
                        fwd_plus_adjoint_over_fwd=(fm + bm) / fm,
                        recomputed_steps=inf["recomputed_steps"], device_bytes=inf["device_bytes"])
    eta, omega = inf["eta"], inf["omega"]
    s.close()
    from oracle import pdlp_oracle as O
    Kt, ct, qt, lt, ut, D1, D2 = O.precondition(lp.K(), lp.c, lp.q, lp.l, lp.u)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        xs, ys = O.unroll_forward(Kt, ct, qt, lt, ut, lp.m1, eta, omega, T)
        t1 = time.perf_counter()
        O.unroll_backward(Kt, lt, ut, lp.m1, eta, omega, xs, ys, D2 * 2.0 * (D2 * xs[-1] - x_tgt))
        t2 = time.perf_counter()
    log(f"unroll T={T}: forward {res[segment]['forward_ms']:.2f} ms, adjoint {res[segment]['backward_ms']:.2f} ms "
        f"(segment {segment}); oracle {1e3 * (t1 - t0):.0f} + {1e3 * (t2 - t1):.0f} ms")
    return {"workload": f"{lp.name}, T={T}", "segment": segment, "checkpointed": res[segment],
            "all_masks_kept": res[0], "oracle_forward_ms": 1e3 * (t1 - t0),
            "oracle_adjoint_ms": 1e3 * (t2 - t1), "oracle_cores": 1}


def measure_copy_gbs(torch, nbytes=2 << 30, reps=10):
    """Device-to-device copy bandwidth (bytes read + written per second) on this GPU."""
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * nbytes * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    log(f"device copy: {gbs:.0f} GB/s (read + write)")
    return gbs


def calibrate_copy(nbytes=1 << 30):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "device copy", "bytes_read": nbytes, "bytes_written": nbytes,
                      "launches": 3}), flush=True)


# ---------------------------------------------------------------------------------------------
# rocprofv3 summaries (text for profiles/)
# ---------------------------------------------------------------------------------------------

def _short_kernel(name):
    """'void pdlp::k_lds_rows<1>(pdlp::CsrDev, ...)' -> 'k_lds_rows<1>'."""
    import re
    n = name.strip().strip('"')
    n = re.sub(r"^void\s+", "", n)
    n = n.split("(")[0]
    n = re.sub(r"pdlp::(\(anonymous namespace\)::)?", "", n)
    n = re.sub(r"<(\d+), (\d+)>", r"<\1, \2>", n)
    return n


def _match_kernel(kern, names):
    """The profiled kernel name that a PASS_KERNELS entry denotes: 'k_panel_rows<1>' matches
    'k_panel_rows<1, 8>' (the entry count per lane is a second template argument)."""
    if kern in names:
        return kern
    hits = [k for k in names if kern.endswith(">") and k.startswith(kern[:-1] + ",")]
    return hits[0] if len(hits) == 1 else None


def _read_csv(path):
    import csv
    with open(path, newline="") as fh:
        return list(csv.DictReader(fh))


def summarize_profile(d):
    """Summary of the rocprofv3 runs under d: d/trace (kernel trace + stats), d/fetch and
    d/write (FETCH_SIZE / WRITE_SIZE of the bench run), d/copy_fetch and d/copy_write (the same
    counters on the calibration copy).  Prints text; its last line is machine-readable."""
    import numpy as np

    def find(sub, suffix):
        hits = sorted(glob.glob(os.path.join(d, sub, "**", f"*{suffix}"), recursive=True))
        return hits[0] if hits else None

    title = "the large plain LP (m=1e6, n=2e6, nnz=1.354e8)"
    bj0 = {}
    bl = os.path.join(d, "bench_trace.json")
    if os.path.exists(bl):
        with open(bl) as fh:
            lines = [ln for ln in fh if ln.startswith("{")]
        if lines:
            bj0 = json.loads(lines[-1])
            title = bj0.get("workload") or bj0.get("config", {}).get("workload", title)
    print(f"rocprofv3 profile: PDLP step passes on {title}, one MI355X")
    print(f"step-kernel sources sha256 {kernel_sources_digest()} (bench.STEP_SOURCES under paper_2106_04756_amd/csrc)")
    print()
    trace = find("trace", "kernel_trace.csv")
    if trace:
        rows = _read_csv(trace)
        per = {}
        for r in rows:
            k = _short_kernel(r["Kernel_Name"])
            per.setdefault(k, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
        print("1. Kernel trace of the run (durations in us; 'ran' = dispatches longer than 20% of the kernel's")
        print("   longest, i.e. those that formed a product or ran their update rather than returning at once)")
        print(f"{'kernel':34s} {'calls':>7s} {'avg_us':>9s} {'ran':>7s} {'ran_avg_us':>11s} {'total_ms':>9s}")
        tot = sum(sum(v) for v in per.values())
        for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1]))[:18]:
            a = np.array(v)
            ran = a[a > 0.2 * a.max()]
            print(f"{k:34s} {a.size:7d} {a.mean():9.1f} {ran.size:7d} {ran.mean():11.1f} {a.sum() * 1e-3:9.2f}")
        print(f"   all kernels: {tot * 1e-3:.1f} ms")
        print()
    cal = {}
    for cnt in ("FETCH_SIZE", "WRITE_SIZE"):
        f = find(f"copy_{cnt.split('_')[0].lower()}", "counter_collection.csv")
        if f:
            vals = [float(r["Counter_Value"]) for r in _read_csv(f)
                    if r["Counter_Name"].startswith(cnt) and "copy" in r["Kernel_Name"].lower()]
            if vals:
                cal[cnt] = float(np.median(vals))
    nbytes = 1 << 30
    scale = {c: (nbytes / (cal[c] * 1024.0) if cal.get(c) else None) for c in ("FETCH_SIZE", "WRITE_SIZE")}
    bl = os.path.join(d, "bench_trace.json")
    if os.path.exists(bl):
        with open(bl) as fh:
            line = [ln for ln in fh if ln.startswith("{")][-1]
        bj = json.loads(line)
        print("   bench.py line of the traced run: " + f"{bj['value']:.1f} iters/s; HIP-event averages of the passes "
              "that ran (us): " + ", ".join(f"{k} {v['avg_us']:.1f}" for k, v in bj["passes"].items()))
        print()
    print("2. Counter calibration: a 1 GiB device copy (1 GiB read, 1 GiB written) gives "
          + ", ".join(f"{c} {cal.get(c, float('nan')):.0f} KiB" for c in ("FETCH_SIZE", "WRITE_SIZE"))
          + " per dispatch,")
    print("   so HBM bytes = " + " + ".join(f"{c} x {scale[c]:.3f} KiB" for c in scale if scale[c]))
    print()
    byk = {}
    for cnt, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        f = find(sub, "counter_collection.csv")
        if not f or not scale[cnt]:
            continue
        for r in _read_csv(f):
            if not r["Counter_Name"].startswith(cnt):
                continue
            k = _short_kernel(r["Kernel_Name"])
            if not k.startswith("k_"):
                continue   # the solver's kernels only (not the copy-rate probe's)
            byk.setdefault(k, {}).setdefault(cnt, []).append(float(r["Counter_Value"]) * 1024.0 * scale[cnt])
    print("3. HBM bytes per dispatch that formed its product (dispatches above 20% of the kernel's largest")
    print("   fetch; the median of those), scaled by the calibration:")
    print(f"{'kernel':34s} {'dispatches':>10s} {'fetch_MB':>9s} {'write_MB':>9s} {'total_MB':>9s}")
    per_dispatch = {}
    for k in sorted(byk):
        fe = np.array(byk[k].get("FETCH_SIZE", [0.0]))
        wr = np.array(byk[k].get("WRITE_SIZE", [0.0]))
        if fe.max() <= 0:
            continue
        sel = fe > 0.2 * fe.max()
        fmed = float(np.median(fe[sel]))
        wmed = float(np.median(wr[: fe.size][sel[: wr.size]])) if wr.size == fe.size else float(np.median(wr))
        per_dispatch[k] = fmed + wmed
        if fmed + wmed > 1e6:
            print(f"{k:34s} {int(sel.sum()):10d} {fmed / 1e6:9.1f} {wmed / 1e6:9.1f} {(fmed + wmed) / 1e6:9.1f}")
    print()
    import re
    sizes = re.search(r"m=(\d+) n=(\d+) nnz=(\d+)", title)
    if bj0.get("layouts") and sizes:
        lay = bj0["layouts"]

        class _Sz:
            m, n, nnz = (int(v) for v in sizes.groups())
        pb = pass_bytes(_Sz)
        print("4. The passes of the timed step: HBM bytes per dispatch that formed its product against the")
        print("   algorithmic bytes of one product (bench.pass_bytes), and the kernel's average duration here")
        print(f"{'pass':16s} {'kernel':22s} {'measured_MB':>12s} {'algorithmic_MB':>15s} {'ratio':>6s} {'trace_us':>9s}")
        for name, v in bj0.get("passes", {}).items():
            lk = lay.get("KT" if name.startswith("primal") else "K", 0)
            kern = _match_kernel(PASS_KERNELS[name].get(lk, ""), per_dispatch)
            if not kern:
                continue
            alg = pb[name]
            if (name == "primal_combine" and lay.get("KT") == 0) or (name == "dual_combine" and lay.get("K") == 0):
                alg += pb[name.replace("combine", "pass1")]
            tr = per.get(kern) if trace else None
            tr_us = float(np.mean([t for t in tr if t > 0.2 * max(tr)])) if tr else float("nan")
            print(f"{name:16s} {kern:22s} {per_dispatch[kern] / 1e6:12.1f} {alg / 1e6:15.1f} "
                  f"{per_dispatch[kern] / alg:6.2f} {tr_us:9.1f}")
        print()
    cmd = os.path.join(d, "commands.txt")
    if os.path.exists(cmd):
        print("Commands (R = the repository root; run from /tmp after `export TMPDIR=/tmp`):")
        with open(cmd) as fh:
            for ln in fh:
                print("  " + ln.rstrip())
        print()
    print("bench-traffic: " + json.dumps({"sources_sha256": kernel_sources_digest(),
                                         "bytes_per_dispatch": {k: round(v) for k, v in per_dispatch.items()
                                                                if v > 1e6}}))


def summarize_unroll(d):
    """Summary of the rocprofv3 kernel trace of `bench.py --only-unroll` under d/trace (kernel
    statistics of the unrolled-PDHG kernels) with that run's bench line (d/bench_trace.json)."""
    trace = sorted(glob.glob(os.path.join(d, "trace", "**", "*kernel_stats.csv"), recursive=True))
    bl = os.path.join(d, "bench_trace.json")
    bj = {}
    if os.path.exists(bl):
        with open(bl) as fh:
            lines = [ln for ln in fh if ln.startswith("{")]
        if lines:
            bj = json.loads(lines[-1])
    print(f"rocprofv3 profile: unrolled PDHG kernels on {bj.get('workload', 'the unroll LP')}, one MI355X")
    print(f"step-kernel sources sha256 {kernel_sources_digest()} (bench.STEP_SOURCES under paper_2106_04756_amd/csrc)")
    print()
    print("Kernel statistics (one forward step = UFwdPrimal + UFwdDual, one adjoint step = UBwdPrimal +")
    print("UBwdDual; the run makes 6 forward and 6 backward passes with segment 50, then 6 with every")
    print("step's masks kept):")
    print(f"{'kernel':32s} {'calls':>7s} {'avg_us':>8s} {'min_us':>8s} {'max_us':>8s} {'total_ms':>9s}")
    if trace:
        rows = [r for r in _read_csv(trace[0]) if "unroll" in r["Name"]]
        for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
            print(f"{_short_kernel(r['Name']):32s} {int(r['Calls']):7d} {float(r['AverageNs']) * 1e-3:8.1f} "
                  f"{float(r['MinNs']) * 1e-3:8.1f} {float(r['MaxNs']) * 1e-3:8.1f} "
                  f"{float(r['TotalDurationNs']) * 1e-6:9.2f}")
    print()
    if bj:
        c, a = bj["checkpointed"], bj["all_masks_kept"]
        print(f"bench.py unroll line of the traced run: forward {c['forward_ms']:.2f} ms "
              f"({c['forward_steps_per_s']:.0f} steps/s), adjoint {c['backward_ms']:.2f} ms, "
              f"(forward + adjoint) / forward = {c['fwd_plus_adjoint_over_fwd']:.2f} (segment {bj['segment']}); "
              f"all masks kept: {a['fwd_plus_adjoint_over_fwd']:.2f}")
        print()
    print("Commands (R = the repository root; run from /tmp after `export TMPDIR=/tmp`):")
    print("  rocprofv3 --kernel-trace --stats --output-format csv -d trace -o run -- python3 R/bench.py "
          "--only-unroll > bench_trace.json")
    print("  python3 R/bench.py --summarize-unroll <this directory>")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-unroll", action="store_true")
    ap.add_argument("--no-truncated", action="store_true",
                    help="skip the large LP with column counts truncated to [1,190]")
    ap.add_argument("--no-pagerank", action="store_true", help="skip the PageRank LP on 5e6 nodes")
    ap.add_argument("--no-policies", action="store_true", help="skip the other step policies")
    ap.add_argument("--no-ablations", action="store_true", help="skip the ablation switches")
    ap.add_argument("--only-large", action="store_true", help="only the large plain LP (profiling runs)")
    ap.add_argument("--only-lp", choices=["truncated", "pagerank"],
                    help="only the truncated large LP or the PageRank LP, headline windows as for the "
                         "large LP (profiling runs; the JSON line carries that LP's figures)")
    ap.add_argument("--only-unroll", action="store_true",
                    help="only the unrolled PDHG measurement (profiling runs; prints its JSON object)")
    ap.add_argument("--summarize-unroll", metavar="DIR")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--batch-iter-limit", type=int, default=100000)
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--summarize-profile", metavar="DIR")
    args = ap.parse_args()
    if args.summarize_profile:
        summarize_profile(args.summarize_profile)
        return
    if args.summarize_unroll:
        summarize_unroll(args.summarize_unroll)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU layout is described in the design notes, not built).", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.only_large:
        args.no_truncated = args.no_pagerank = args.no_policies = args.no_ablations = True
        args.no_batched = args.no_unroll = args.no_cpu_baseline = True

    import torch

    import paper_2106_04756_amd as P
    from workloads import lpgen

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.only_unroll:
        print(json.dumps(bench_unroll(P, lpgen)), flush=True)
        return
    if args.only_lp:
        t = time.time()
        lpo = lpgen.large_lp_truncated(args.seed) if args.only_lp == "truncated" else lpgen.pagerank_5m()
        log(f"generated {lpo.name}: nnz={lpo.nnz} in {time.time() - t:.1f}s")
        ro = measure_lp(P, torch, lpo, args.warmup, args.steps, label=args.only_lp)
        attach_traffic(ro, lpo, args.only_lp)
        print(json.dumps({"workload": f"{lpo.name}, m={lpo.m} n={lpo.n} nnz={lpo.nnz}", "value": ro["iters_per_s"],
                          "steps": args.steps, "warmup": args.warmup, **ro}), flush=True)
        return
    t = time.time()
    lp = lpgen.large_lp(args.seed)
    log(f"generated {lp.name}: m={lp.m} n={lp.n} nnz={lp.nnz} in {time.time() - t:.1f}s")
    W, K = args.warmup, args.steps
    r = measure_lp(P, torch, lp, W, K, label="large LP")
    attach_traffic(r, lp)
    copy_gbs = measure_copy_gbs(torch)
    roof = r["roofline"]
    roof["measured_copy_gbs"] = copy_gbs
    roof["frac_of_measured_copy"] = (roof["achieved"] or 0.0) / copy_gbs
    m, n, nnz = lp.m, lp.n, lp.nnz
    out = {
        "metric": "PDHG iters/s",
        "value": r["iters_per_s"],
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": r["seconds"] / max(r["steps_taken"], 1) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"large plain LP m={m} n={n} nnz={nnz} (Zipf(1.5) column counts, "
                               f"30% equality rows, mixed bounds), seed {args.seed}",
                   "tol": 1e-8, "steps_taken": r["steps_taken"],
                   "timed": "exactly K steps of pdlp_solve after W warmup steps (captured HIP graphs per "
                            "block of 40 attempt slots; checks fall where k is a multiple of 40)"},
        "roofline": roof,
        "check_inclusive": r["check_inclusive"],
        "passes": r["passes"],
        "slots": r["slots"],
        "step_gbs_algorithmic": r["step_gbs_algorithmic"],
        "create_seconds": r["create_seconds"],
        "layouts": r["layouts"],
    }
    if not args.no_truncated:
        lpb = lpgen.large_lp_truncated(args.seed)
        log(f"generated {lpb.name}: nnz={lpb.nnz}")
        rb = measure_lp(P, torch, lpb, W, K, label="truncated LP")
        attach_traffic(rb, lpb, "truncated")
        out["large_lp_truncated"] = {
            "workload": f"large plain LP m={lpb.m} n={lpb.n} nnz={lpb.nnz} (Zipf(1.5) column "
                        f"counts truncated to [1,190]), seed {args.seed}", **rb}
    if not args.no_pagerank:
        t = time.time()
        lpr = lpgen.pagerank_5m()
        log(f"generated {lpr.name}: nnz={lpr.nnz} in {time.time() - t:.1f}s")
        rp = measure_lp(P, torch, lpr, W, K, label="PageRank LP")
        attach_traffic(rp, lpr, "pagerank")
        out["pagerank_5m"] = {"workload": f"{lpr.name}, m={lpr.m} n={lpr.n} nnz={lpr.nnz}", **rp}
        del lpr
    # the tiny plain LP (launch-bound regime): wall time of a whole solve to KKT 1e-8
    tiny = lpgen.tiny_lp()
    st0 = P.Solver.from_lp(tiny)
    st0.solve(1e-8, 1)          # first launches / module load outside the timing
    st0.close()
    st0 = P.Solver.from_lp(tiny)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc0 = st0.solve(1e-8, 100000)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    i0 = st0.info()
    out["tiny_lp_solve"] = {"workload": tiny.name, "status": P.STATUS_NAMES[rc0], "iterations": i0["iterations"],
                            "seconds": t1 - t0, "iters_per_s": i0["iterations"] / (t1 - t0),
                            "kkt": i0["kkt"][3]}
    st0.close()
    log(f"tiny LP: {i0['iterations']} iterations to KKT {i0['kkt'][3]:.2e} in {t1 - t0:.3f}s")
    if not args.no_policies:
        out["step_policies"] = bench_step_policies(P, torch, lp)
    if not args.no_ablations:
        out["ablations"] = bench_ablations(P, lpgen)
    if not args.no_batched:
        out["batched"] = bench_batched(P, lpgen, args.batch_count, args.batch_iter_limit)
    if not args.no_unroll:
        out["unroll"] = bench_unroll(P, lpgen)
    if not args.no_cpu_baseline:
        log("timing the oracle sample on the host")
        out["cpu_baseline"] = cpu_baseline(lp)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
