"""PDHG throughput of the gfx950 PDLP solver on the large plain LP (m=1e6, n=2e6, Zipf(1.5)
column counts, nnz ~1.35e8), one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-batched]
                    [--no-unroll] [--no-truncated] [--no-policies] [--no-ablations]
                    [--calibrate-copy]

A step is one accepted PDHG iteration of Algorithm 1 on the whole LP: the K~^T product fused
with the primal step, the K~ product fused with the dual step and the step-size rule, and
(every 40 steps) the restart / termination check.  The LP is resident in HBM before timing
starts.  Prints one JSON line.  Progress goes to stderr.  Beside the headline figures the line
carries: the same shape with column counts truncated to [1,190]; a whole solve of the tiny LP;
the constant-step and Malitsky-Pock policies on the large LP; the ablation switches' steps to
KKT 1e-8 on two small LPs; the batched solver; the unrolled PDHG and its adjoint; the oracle's
rate on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, vendor figure


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


PROFILE = os.path.join(ROOT, "profiles", "pdlp_step_large_plain_lp.txt")


# Sources that define the timed step kernels and their launches (the batched solver and the
# unrolled adjoint live in files of their own and do not take part in the timed step).
STEP_SOURCES = ["pdlp_kernels.hip", "pdlp_solver.hip", "pdlp_device.h", "pdlp_internal.h",
                "host_prep.cpp", "host_prep.h"]


def kernel_sources_digest():
    """sha256 over the sources of the timed step kernels (names and contents)."""
    import hashlib
    h = hashlib.sha256()
    for f in [os.path.join(ROOT, "paper_2106_04756_amd", "csrc", f) for f in STEP_SOURCES]:
        h.update(os.path.relpath(f, ROOT).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(steps, warmup):
    """HBM bytes per step slot (primal, dual) that the rocprofv3 byte counters gave for this
    very source tree and bench configuration, read from the committed profile summary; None
    when the kernels or the configuration differ from the profiled ones."""
    try:
        with open(PROFILE) as fh:
            for line in fh:
                if line.startswith("bench-traffic: "):
                    d = json.loads(line[len("bench-traffic: "):])
                    if (d["sources_sha256"] == kernel_sources_digest() and d["steps"] == steps
                            and d["warmup"] == warmup):
                        return d["bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    return None


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
    return dict(value=iters / el, unit="PDHG iters/s", cores=1, kind="oracle",
                sample=f"{iters} accepted oracle PDHG steps (Eq. (3) + Algorithm 2, unpreconditioned, "
                       f"scipy CSR products, 1 thread) on the same LP, {el:.1f} s")


def bench_batched(P, lpgen, count, iter_limit, plain_sample=16):
    """LPs/s to KKT 1e-8 of the batched solver (one launch, one workgroup per LP) on the
    batched workload, against a loop of single-LP solves on an evenly spaced sample."""
    import numpy as np
    t = time.time()
    lps = [lpgen.batched_instance(i) for i in range(count)]
    log(f"generated {count} batched members in {time.time() - t:.1f}s")
    b = P.Batch(lps)
    secs = b.solve(1e-8, iter_limit)
    _, _, st, it, kkt = b.get()
    b.close()
    conv = int((st == P.OPTIMAL).sum())
    idx = list(range(0, count, max(1, count // plain_sample)))[:plain_sample]
    t0 = time.perf_counter()
    pconv = 0
    for i in idx:
        s = P.Solver.from_lp(lps[i])
        pconv += s.solve(1e-8, iter_limit) == P.OPTIMAL
        s.close()
    pdt = time.perf_counter() - t0
    log(f"batched: {conv}/{count} at KKT 1e-8 in {secs:.2f}s; plain loop {pconv}/{len(idx)} in {pdt:.2f}s")
    return {"workload": f"{count} LPs, m log-uniform in [50,2000], n = U[2,3] m, 3-8 nonzeros per "
                        f"column, seeds 3000+i", "tol": 1e-8, "iter_limit": iter_limit,
            "seconds": secs, "converged": conv, "count": count, "lps_per_s": conv / secs,
            "median_iterations": float(np.median(it)), "max_kkt_converged": float(kkt[st == 0, 3].max()) if conv else None,
            "plain_loop_lps_per_s": pconv / pdt, "plain_sample": len(idx), "plain_converged": pconv,
            "speedup_vs_plain": (conv / secs) / (pconv / pdt) if pconv else None}


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


def measure_steps(P, torch, lp, W, K):
    """Warm up W accepted steps, then time K more of Algorithm 1 (HIP events around every step
    kernel) and account the algorithmic bytes of the timed step kernels.  Returns (dict, solver)."""
    t = time.time()
    s = P.Solver.from_lp(lp, time_kernels=1)
    info = s.info()
    log(f"created solver in {time.time() - t:.1f}s (library create {info['create_seconds']:.1f}s)")
    st = s.solve(1e-8, W)
    log(f"warmup {W} steps: status {P.STATUS_NAMES[st]}")
    s.reset_kernel_times()
    i0 = s.info()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = s.solve(1e-8, W + K)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    info = s.info()
    steps = info["iterations"] - i0["iterations"]
    dt = t1 - t0
    log(f"timed {steps} steps in {dt:.3f}s: status {P.STATUS_NAMES[st]}, attempts {info['attempts']}, "
        f"restarts {info['restarts']}, kkt {info['kkt'][3]:.3e}")
    # Algorithmic bytes of the timed step kernels.  The primal step skips its K~^T y product
    # when y is unchanged since that product was last formed (after a rejected attempt, and
    # after a check, which forms it), and a slot whose attempt does not run (a check pending)
    # does nothing; so count the products from the solver's counters: each check forms two
    # K~^T products (of the average and of the current y) and one K~ product.
    times, counts = s.kernel_times()
    m, n, nnz = lp.m, lp.n, lp.nnz
    d_att = info["attempts"] - i0["attempts"]
    d_chk = info["checks"] - i0["checks"]
    prim_products = (info["spmv_KT"] - i0["spmv_KT"]) - 2 * d_chk
    dual_products = (info["spmv_K"] - i0["spmv_K"]) - d_chk
    bytes_primal = 8.0 * (n + 1) + 12.0 * nnz + 8.0 * m + 64.0 * n     # K~^T y, then 8 n-vectors
    bytes_primal_epi = 64.0 * n                                         # the same without the product
    bytes_dual = 8.0 * (m + 1) + 12.0 * nnz + 8.0 * n + 56.0 * m        # K~ x', then 7 m-vectors
    total_bytes = [prim_products * bytes_primal + (d_att - prim_products) * bytes_primal_epi,
                   dual_products * bytes_dual]
    dom = 0 if times[0] >= times[1] else 1
    name = ["primal step: K~^T y product fused with the primal update (first pass k_lds_rows<1> with "
            "the operand staged in LDS, else k_panel_rows<1>, then k_primal_combine; k_primal in the "
            "plain layout)",
            "dual step: K~ x' product fused with the dual update and the step rule (first pass "
            "k_lds_rows<0> with the operand staged in LDS, else k_panel_rows<0>, then k_dual_combine; "
            "k_dual in the plain layout)"][dom]
    avg_ms = times[dom] / counts[dom]
    bpl = total_bytes[dom] / counts[dom]
    achieved = bpl / (avg_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "kernel": name, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled)",
            "avg_launch_ms": avg_ms, "launches": int(counts[dom]),
            "products": int([prim_products, dual_products][dom]), "attempts": int(d_att),
            "algorithmic_bytes_per_launch": bpl, "slot": ["primal", "dual"][dom]}
    return ({"steps_taken": steps, "seconds": dt, "roofline": roof,
             "step_gbs_algorithmic": info["step_bytes"] * steps / dt / 1e9,
             "step_avg_ms": {"primal": times[0] / counts[0], "dual": times[1] / counts[1]},
             "algorithmic_bytes_per_slot": {"primal": total_bytes[0] / counts[0],
                                            "dual": total_bytes[1] / counts[1]}}, s)


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
    ap.add_argument("--no-policies", action="store_true", help="skip the other step policies")
    ap.add_argument("--no-ablations", action="store_true", help="skip the ablation switches")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--batch-iter-limit", type=int, default=20000)
    ap.add_argument("--calibrate-copy", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU layout is described in the design notes, not built).", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return

    import torch

    import paper_2106_04756_amd as P
    from workloads import lpgen

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t = time.time()
    lp = lpgen.large_lp(args.seed)
    log(f"generated {lp.name}: m={lp.m} n={lp.n} nnz={lp.nnz} in {time.time() - t:.1f}s")
    W, K = args.warmup, args.steps
    r, s = measure_steps(P, torch, lp, W, K)
    steps, dt = r["steps_taken"], r["seconds"]
    m, n, nnz = lp.m, lp.n, lp.nnz
    traffic = profiled_traffic(K, W)
    roof = r["roofline"]
    roof["traffic"] = (traffic or {}).get(roof.pop("slot"))
    copy_gbs = measure_copy_gbs(torch)
    roof["measured_copy_gbs"] = copy_gbs
    roof["frac_of_measured_copy"] = roof["achieved"] / copy_gbs
    out = {
        "metric": "PDHG iters/s",
        "value": steps / dt,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": dt / max(steps, 1) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"large plain LP m={m} n={n} nnz={nnz} (Zipf(1.5) column counts, "
                               f"30% equality rows, mixed bounds), seed {args.seed}",
                   "tol": 1e-8, "steps_taken": steps},
        "roofline": roof,
        "step_gbs_algorithmic": r["step_gbs_algorithmic"],
        "step_avg_ms": r["step_avg_ms"],
        "algorithmic_bytes_per_slot": r["algorithmic_bytes_per_slot"],
    }
    s.close()
    if not args.no_truncated:
        # the same shape with column counts truncated to [1, 190] (nnz ~2.1e7)
        lpb = lpgen.large_lp_truncated(args.seed)
        log(f"generated {lpb.name}: nnz={lpb.nnz}")
        rb, sb = measure_steps(P, torch, lpb, W, K)
        sb.close()
        rb["roofline"].pop("slot")
        out["large_lp_truncated"] = {
            "workload": f"large plain LP m={lpb.m} n={lpb.n} nnz={lpb.nnz} (Zipf(1.5) column "
                        f"counts truncated to [1,190]), seed {args.seed}",
            "iters_per_s": rb["steps_taken"] / rb["seconds"], "steps": rb["steps_taken"],
            "roofline": rb["roofline"], "step_gbs_algorithmic": rb["step_gbs_algorithmic"]}
        log(f"large_lp_truncated: {out['large_lp_truncated']['iters_per_s']:.1f} iters/s, "
            f"{rb['roofline']['frac'] * 100:.1f}% of HBM peak")
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
        s.close()
        out["cpu_baseline"] = cpu_baseline(lp)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
