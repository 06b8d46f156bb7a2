"""Benchmark: combined-preconditioned CG solve on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one whole solve (PCG with the combined ILU(0) + AMG preconditioner, the
complete hot path) of the 3-D 128x128x64 TPFA pressure system to relative residual
1e-8, with the matrix hierarchy and the right-hand side already resident in HBM.
value = the method's bytes of one solve / solve time (GB/s): every matrix read once
per pass the algorithm makes over it, every vector read or written once per step,
whatever form evaluates a Gauss-Seidel sweep; ms_per_step = solve time. The roofline
object is for the kernel family that takes the most time per iteration, measured
live; the same system is also solved with the FP32 preconditioner (speedup and error
against the FP64 oracle); the CPU baseline is the oracle solving the system on the
host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from pathlib import Path

ROOT = Path(__file__).resolve().parent
sys.path.insert(0, str(ROOT))

HBM_PEAK_GBS = 8000.0
# candidates for the roofline object: the two families that hold most of the solve
# time (level-scheduled triangular sweeps, explicit-inverse products), with the kernel
# each launches, its source and the committed counter passes for it
FAMILIES = {
    "sweep": {"kernel": "tri_wave_kernel", "source": "wave_sweep.hip",
              "what": "level-scheduled triangular solves: forward/backward Gauss-Seidel sweeps on the levels "
                      "smoothed that way (both V-cycles) and the ILU(0) L and U solves of one PCG iteration"},
    "dense_gemv": {"kernel": "gemv_tri_rows_kernel", "source": "dense_tri.hip",
                   "what": "products with the explicit inverses of D+L or of its diagonal blocks, both "
                           "directions, every level smoothed that way (one V-cycle)"},
}
# other families reported with their method GB/s (one V-cycle's launches, or one PCG
# step for the finest-level product)
OTHER_FAMILIES = ["spmv_pq", "residual", "restrict", "prolong"]
CSRC = ROOT / "paper_1205_6113_amd" / "csrc"


def traffic_file(kernel: str) -> Path:
    return ROOT / "profiles" / f"traffic_{kernel}_c2.txt"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name: str):
    import gen
    if name == "c2":
        return gen.config2(), "3d-128x128x64-tpfa-corr-sigma2-kz0.1-2wells (1,048,448 unknowns), B_co PCG to 1e-8"
    if name == "c3":
        return gen.config3(), "3d-60x220x85-tpfa-layered-channels-kz0.01 (1,122,000 unknowns), B_co PCG to 1e-8"
    if name == "c1":
        return gen.config1(), "2d-64x64-tpfa-lognormal (4096 unknowns), B_co PCG to 1e-8"
    raise SystemExit(f"unknown workload {name}")


def cpu_baseline(p, iters_gpu):
    """The oracle (single-threaded C, FP64) on the same system: setup untimed, one
    full solve to the same tolerance timed."""
    import numpy as np
    import oracle
    t = time.perf_counter()
    h = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val)
    setup_s = time.perf_counter() - t
    t = time.perf_counter()
    r = h.pcg(oracle.PREC_COMBINED, p.b, p.tol, 10000)
    solve_s = time.perf_counter() - t
    return h, r, setup_s, solve_s, np


def chain_latency(dev, reps):
    """Dependent-step latencies of the one-wave sweep kernel on a chain (tridiagonal
    matrix, one row per level set): with the whole chain in one block every step is an
    in-block step (t_step); with two-row blocks every second step waits for another
    workgroup's store (t_hop, the cross-workgroup hand-off beyond an in-block step)."""
    import numpy as np
    import paper_1205_6113_amd as cpc
    n = 8192  # the largest one-block sweep with a forced block size
    rp = np.concatenate([[0], np.cumsum([2] + [3] * (n - 2) + [2])]).astype(np.int32)
    ci, v = [], []
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                ci.append(j)
                v.append(2.5 if j == i else -1.0)
    ci = np.array(ci, np.int32)
    v = np.array(v)
    ms = {}
    for R in (n, 2):
        with cpc.Solver(n, rp, ci, v, device=dev, sweep_block_rows=R, dense_smoother="never") as s:
            ms[R] = s.time_kernel("fgs", level=0, reps=reps)["avg_ms"]
    t_step = 1000.0 * ms[n] / n
    t_hop = 2.0 * 1000.0 * ms[2] / n - 2.0 * t_step
    return {"t_step_us": round(t_step, 4), "t_hop_us": round(t_hop, 4), "chain_rows": n,
            "one_block_ms": round(ms[n], 4), "two_row_blocks_ms": round(ms[2], 4)}


def sweep_roofs(solver, info, lat, reps):
    """Both roofs of every level smoothed by level-scheduled sweeps: the HBM floor (the
    forward sweep's method bytes at 8 TB/s) and the latency floor (dependency depth times
    the in-block step latency; depth times step plus hand-off if every level crossed a
    workgroup), beside the measured forward sweep."""
    rows = []
    for d in range(info["nlev"] - 1):
        if info["smoother"][d] != "sweep":
            continue
        tk = solver.time_kernel("fgs", level=d, reps=reps)
        depth = info["depth"][d]
        rows.append({"level": d, "rows": info["n"][d], "depth": depth, "measured_ms": round(tk["avg_ms"], 4),
                     "method_bytes": tk["bytes"], "hbm_floor_ms": round(tk["bytes"] / (HBM_PEAK_GBS * 1e9) * 1e3, 4),
                     "latency_floor_ms": round(depth * lat["t_step_us"] / 1000.0, 4),
                     "all_hops_ms": round(depth * (lat["t_step_us"] + lat["t_hop_us"]) / 1000.0, 4)})
    return rows


def bench_batch(args):
    """Batch of 64 independent TPFA systems (edges 32..96) in one batched solve, against
    the same 64 systems solved one after the other with single-system handles."""
    import numpy as np
    import torch
    import gen
    import paper_1205_6113_amd as cpc
    probs = gen.config4()
    n_tot = sum(p.n for p in probs)
    log(f"workload c4: {len(probs)} systems, {n_tot} unknowns in all")
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    bs = cpc.BatchSolver([(p.n, p.row_ptr, p.col, p.val) for p in probs], device=dev, verbose=True,
                         tune=not args.rules)
    setup_s = time.perf_counter() - t0
    log(f"batch setup {setup_s:.1f}s")
    b = torch.as_tensor(np.concatenate([p.b for p in probs]), device=dev)
    tol = probs[0].tol
    for w in range(args.warmup):
        x, its, rels, st = bs.solve(b, tol=tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        x, its, rels, st = bs.solve(b, tol=tol)
    torch.cuda.synchronize()
    ms_batch = 1000.0 * (time.perf_counter() - t0) / args.steps
    stats = bs.stats()
    log(f"batch: {ms_batch:.1f} ms per batch solve, iterations {int(its.min())}..{int(its.max())}")
    # the same systems one by one (setups untimed): every 4th system, times 4
    seq_ms, errs = 0.0, []
    offs = bs.offsets
    sample = [] if args.no_sequential else list(range(0, len(probs), 4))
    for k in sample:
        p = probs[k]
        log(f"single system {k}: n={p.n}")
        s1 = cpc.Solver(p.n, p.row_ptr, p.col, p.val, device=dev)
        b1 = torch.as_tensor(p.b, device=dev)
        x1, it1, rel1, st1 = s1.solve(b1, tol=tol)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x1, it1, rel1, st1 = s1.solve(b1, tol=tol)
        torch.cuda.synchronize()
        seq_ms += 1000.0 * (time.perf_counter() - t0)
        xb = x[offs[k]:offs[k] + p.n]
        errs.append(float(torch.linalg.norm(xb - x1) / torch.linalg.norm(x1)))
        s1.close()
    if sample:
        seq_ms *= len(probs) / len(sample)
        log(f"sequential: {seq_ms:.1f} ms for the {len(probs)} single-system solves (from {len(sample)} of them)")
    else:
        seq_ms = None
    # method bytes: each system's own iterations (the per-iteration figure of the batch
    # is the sum over systems, so weight it by the systems' share of the unknowns); the
    # forms' bytes: the batched preconditioner runs over every system until the last stops
    ns = np.array([p.n for p in probs], dtype=np.float64)
    it_w = float((ns * its.astype(np.float64)).sum() / ns.sum())
    method_batch = stats["method_bytes_per_iter"] * it_w + stats["method_bytes_initial"]
    form_batch = stats["bytes_per_iter"] * int(its.max()) + stats["bytes_initial"]
    # x against the oracle on a sample of the systems (smallest, median, largest)
    order = np.argsort(ns)
    osample = sorted({int(order[0]), int(order[len(order) // 2]), int(order[-1])})
    oerr = {}
    if not args.no_cpu_baseline:
        import oracle
        for k in osample:
            p = probs[k]
            log(f"oracle system {k}: n={p.n}")
            hk = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val)
            rk = hk.pcg(oracle.PREC_COMBINED, p.b, tol, 1000)
            xb = x[offs[k]:offs[k] + p.n].cpu().numpy()
            oerr[k] = {"n": p.n, "iters_oracle": int(rk["iters"]), "iters_batch": int(its[k]),
                       "x_relerr": float(np.linalg.norm(xb - rk["x"]) / np.linalg.norm(rk["x"]))}
            log(f"oracle system {k}: {oerr[k]}")
    out = {
        "metric": "combined-PCG solve s + HBM GB/s to 1e-8 rel res; FP32-precond vs FP64",
        "value": round(method_batch / (ms_batch / 1000.0) / 1e9, 3),
        "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_batch, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"batch of {len(probs)} 3-d TPFA systems, edges 32..96 ({n_tot} unknowns), "
                               "B_co PCG to 1e-8",
                   "systems": len(probs), "unknowns": n_tot, "setup_s": round(setup_s, 3),
                   "solves_per_s": round(len(probs) / (ms_batch / 1000.0), 2),
                   "iters_min": int(its.min()), "iters_max": int(its.max()), "iters_mean": float(its.mean()),
                   "relres_max": float(rels.max()), "sequential_ms": round(seq_ms, 3) if seq_ms else None,
                   "sequential_sample": (f"every 4th system ({len(sample)}), scaled by {len(probs) / len(sample):g}"
                                         if sample else None),
                   "speedup_vs_sequential": round(seq_ms / ms_batch, 3) if seq_ms else None,
                   "x_relerr_batch_vs_single_max": max(errs) if errs else None,
                   "method_bytes_per_batch_solve": method_batch, "form_bytes_per_batch_solve": form_batch,
                   "oracle_sample": oerr},
    }
    print(json.dumps(out), flush=True)
    bs.close()


def bench_adjoint(args):
    """Differentiable solve on C5: forward (assembly, setup, PCG) and backward (adjoint
    PCG, gradient assembly) times; gradient against the oracle and central differences."""
    import numpy as np
    import torch
    import gen
    from paper_1205_6113_amd import adjoint as adj
    p = gen.config5()
    nx, ny, nz = p.dims
    dev = torch.device("cuda:0")
    grid = adj.TpfaGrid(nx, ny, nz, p.kz_ratio, p.dirichlet_x)
    obs = torch.as_tensor(p.meta["obs"], device=dev)
    d = torch.as_tensor(p.meta["d"], device=dev)
    tol = 1e-10
    times = []
    for k in range(args.warmup + args.steps):
        logk = torch.as_tensor(p.logk.ravel(), device=dev).requires_grad_(True)
        b = torch.as_tensor(p.b, device=dev).requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x = adj.tpfa_solve(logk, b, grid, tol=tol, tune=False)  # rule-based setup (no timing)
        L = 0.5 * ((x[obs] - d) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if k >= args.warmup:
            times.append((t1 - t0, t2 - t1))
    fwd = float(np.mean([t[0] for t in times]))
    bwd = float(np.mean([t[1] for t in times]))
    g_logk = logk.grad.cpu().numpy()
    g_b = b.grad.cpu().numpy()
    log(f"forward {fwd:.3f}s backward {bwd:.3f}s")
    res = {"forward_s": round(fwd, 4), "backward_s": round(bwd, 4), "loss": float(L.item())}
    # the same differentiable solve at nearby log k (log k + 0.02 N(0,1), a new draw per
    # step) with the preconditioner set up once at log k (tpfa_solve's `setup`)
    fz0 = adj.FrozenPreconditionerSolve(torch.as_tensor(p.logk.ravel(), device=dev), grid, tune=False)
    rng = np.random.default_rng(3)
    rtimes = []
    for k in range(args.warmup + args.steps):
        lk = torch.as_tensor(p.logk.ravel() + 0.02 * rng.standard_normal(p.n), device=dev).requires_grad_(True)
        bb = torch.as_tensor(p.b, device=dev).requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xr = adj.tpfa_solve(lk, bb, grid, tol=tol, setup=fz0)
        Lr = 0.5 * ((xr[obs] - d) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        Lr.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if k >= args.warmup:
            rtimes.append((t1 - t0, t2 - t1))
    fz0.close()
    res["forward_reused_setup_s"] = round(float(np.mean([t[0] for t in rtimes])), 4)
    res["backward_reused_setup_s"] = round(float(np.mean([t[1] for t in rtimes])), 4)
    res["reused_setup_at"] = "log k + 0.02 N(0,1), preconditioner of log k"
    log(f"with the setup reused: forward {res['forward_reused_setup_s']}s backward {res['backward_reused_setup_s']}s")
    # central differences with the preconditioner frozen at log k, 20 cells
    fz = adj.FrozenPreconditionerSolve(logk.detach(), grid)
    h = 1e-6
    fd_err = []
    for c in p.meta["fd_cells"]:
        vals = []
        for sgn in (1.0, -1.0):
            lk = logk.detach().clone()
            lk[int(c)] += sgn * h
            xs, it, rel, st = fz.solve(lk, b.detach(), tol=1e-13)
            vals.append(0.5 * float(((xs[obs] - d) ** 2).sum()))
        g_fd = (vals[0] - vals[1]) / (2 * h)
        fd_err.append(abs(g_fd - g_logk[c]) / max(abs(g_logk[c]), 1e-3 * np.abs(g_logk).max()))
    fz.close()
    res["fd_cells"] = len(fd_err)
    res["fd_relerr_max"] = float(max(fd_err))
    if not args.no_cpu_baseline:
        import oracle
        hh = oracle.Hierarchy(p.n, p.row_ptr, p.col, p.val)
        ref = oracle.misfit_gradient(p, hh, tol=tol)
        res["grad_logk_relerr_vs_oracle"] = float(np.linalg.norm(g_logk - ref["grad_logk"]) /
                                                  np.linalg.norm(ref["grad_logk"]))
        res["grad_b_relerr_vs_oracle"] = float(np.linalg.norm(g_b - ref["grad_b"]) / np.linalg.norm(ref["grad_b"]))
    log(f"gradient check: {res}")
    out = {
        "metric": "combined-PCG solve s + HBM GB/s to 1e-8 rel res; FP32-precond vs FP64",
        "value": None, "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1000.0 * (fwd + bwd), 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "differentiable 3-d 96x96x48 TPFA solve (442,368 unknowns), forward + adjoint, "
                               "PCG to 1e-10", **res},
    }
    print(json.dumps(out), flush=True)


def bench_table(args):
    """The comparison of Table 5.2 on a synthetic workload: iterations and solve time of
    PCG with each preconditioner (one handle for the ILU(0)-based ones, one with ILU(1)
    as B), setup time per handle. Prints one JSON line of its own."""
    import torch
    import paper_1205_6113_amd as cpc
    p, desc = workload(args.workload)
    dev = torch.device("cuda:0")
    b = torch.as_tensor(p.b, device=dev)
    rows = []
    for fill, entries in ((0, [("ILU(0)", "ilu"), ("AMG(GS)", "amg"), ("AMG(ILU(0))", "amg_ilu"),
                               ("additive B^", "additive"), ("B_co (multiplicative)", "combined"),
                               ("wrong-order B-bar", "bbar")]),
                          (1, [("ILU(1)", "ilu"), ("B_co with ILU(1)", "combined")])):
        t0 = time.perf_counter()
        s = cpc.Solver(p.n, p.row_ptr, p.col, p.val, device=dev, precision=args.precision,
                       tune=not args.rules, ilu_fill=fill)
        setup_s = time.perf_counter() - t0
        log(f"handle with ILU({fill}): setup {setup_s:.2f}s")
        for name, prec in entries:
            x, it, rel, st = s.solve(b, tol=p.tol, maxit=10000, prec=prec)
            times = []
            for _ in range(max(1, args.steps)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x, it, rel, st = s.solve(b, tol=p.tol, maxit=10000, prec=prec)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            times.sort()
            ms = 1000.0 * times[len(times) // 2]
            rows.append({"preconditioner": name, "ilu_fill": fill, "iters": it, "status": st, "relres": rel,
                         "solve_ms": round(ms, 3), "setup_s": round(setup_s, 3)})
            log(f"{name}: {it} iterations, status {st}, {ms:.2f} ms")
        s.close()
    out = {"metric": "Table 5.2 analogue: PCG iterations and solve time per preconditioner",
           "unit": "ms", "n_gpus": 1, "data": "synthetic", "dtype": "f64" if args.precision == "fp64" else
           "f64-pcg/f32-precond", "config": {"workload": desc, "n": p.n, "nnz": p.nnz, "tol": p.tol}, "rows": rows}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--roofline-reps", type=int, default=5)
    ap.add_argument("--no-compare-precision", action="store_true",
                    help="skip the solve with the preconditioner in the other precision")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="copy MB megabytes device to device once (a plain copy of known size for "
                         "calibrating memory counters)")
    ap.add_argument("--rules", action="store_true", help="rule-based setup instead of the timing tuner")
    ap.add_argument("--no-sequential", action="store_true",
                    help="c4: skip the single-system solves the batch is compared with (profiling runs)")
    ap.add_argument("--verbose", action="store_true", help="print setup progress")
    ap.add_argument("--table", action="store_true",
                    help="instead of the benchmark line, the Table 5.2 comparison of preconditioners")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU form is "
              "not built (see the sharding design).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1205_6113_amd as cpc

    if args.table:
        return bench_table(args)
    if args.workload == "c4":
        return bench_batch(args)
    if args.workload == "c5":
        return bench_adjoint(args)
    p, desc = workload(args.workload)
    log(f"workload {desc}: n={p.n} nnz={p.nnz}")
    torch.cuda.init()
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    solver = cpc.Solver(p.n, p.row_ptr, p.col, p.val, device=dev, precision=args.precision,
                        tune=not args.rules, verbose=args.verbose)
    setup_s = time.perf_counter() - t0
    info = solver.hierarchy()
    log(f"setup {setup_s:.2f}s levels={info['nlev']} n={info['n']}")
    b = torch.as_tensor(p.b, device=dev)
    x = torch.zeros_like(b)
    it = 0
    for w in range(args.warmup):
        x, it, rel, st = solver.solve(b, x=x, tol=p.tol, maxit=10000)
        log(f"warmup {w}: iters={it} relres={rel:.3e} status={st}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        x, it, rel, st = solver.solve(b, x=x, tol=p.tol, maxit=10000)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = 1000.0 * elapsed / args.steps
    stats = solver.stats()
    method_solve = stats["method_bytes_per_iter"] * it + stats["method_bytes_initial"]
    form_solve = stats["bytes_per_iter"] * it + stats["bytes_initial"]
    value = method_solve / (ms_per_step / 1000.0) / 1e9
    log(f"timed {args.steps} solves: {ms_per_step:.3f} ms/solve iters={it} relres={rel:.3e} -> {value:.1f} GB/s "
        f"(method bytes {method_solve / 1e9:.2f} GB; the forms the setup chose move {form_solve / 1e9:.2f} GB)")

    # kernel families, timed live on the solver's stream (HIP events); per iteration the
    # sweep mix runs once, the V-cycle families twice (two V-cycles per B_co application)
    fam = {}
    for name in list(FAMILIES) + OTHER_FAMILIES:
        try:
            tk = solver.time_kernel(name, level=-1, reps=args.roofline_reps)
        except Exception as e:  # a family the chosen forms do not use
            log(f"family {name}: not timed ({e})")
            continue
        per_rep = tk["launches"] / args.roofline_reps
        reps_per_iter = 1 if name in ("sweep", "spmv_pq") else 2
        fam[name] = {"avg_launch_us": round(1000.0 * tk["avg_ms"], 3), "launches_per_iter": per_rep * reps_per_iter,
                     "ms_per_iter": round(tk["avg_ms"] * per_rep * reps_per_iter, 4),
                     "method_bytes_per_launch": tk["bytes"], "form_bytes_per_launch": tk["form_bytes"],
                     "method_gbs": round(tk["bytes"] / (tk["avg_ms"] / 1000.0) / 1e9, 2),
                     "form_gbs": round(tk["form_bytes"] / (tk["avg_ms"] / 1000.0) / 1e9, 2),
                     "launches_timed": tk["launches"]}
        log(f"family {name}: {fam[name]}")
    dom = max((k for k in FAMILIES if k in fam), key=lambda k: fam[k]["ms_per_iter"])
    fd = fam[dom]
    achieved = fd["method_gbs"]
    # counted HBM bytes per launch from the committed rocprofv3 counter passes, only if
    # they were taken on this workload, precision and kernel source
    traffic = None
    tf = traffic_file(FAMILIES[dom]["kernel"])
    if tf.exists():
        try:
            import hashlib
            tr = json.loads(tf.read_text())
            src = hashlib.sha256((CSRC / FAMILIES[dom]["source"]).read_bytes()).hexdigest()
            if (tr.get("workload") == args.workload and tr.get("precision") == args.precision
                    and tr.get("kernel_source_sha256") == src):
                traffic = tr.get("bytes_per_launch")
        except Exception:
            traffic = None
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                "kernel": f"{FAMILIES[dom]['kernel']} ({FAMILIES[dom]['what']})",
                "avg_launch_us": fd["avg_launch_us"], "bytes_per_launch": fd["method_bytes_per_launch"],
                "form_bytes_per_launch": fd["form_bytes_per_launch"], "launches_timed": fd["launches_timed"]}
    log(f"roofline {dom}: {fd['avg_launch_us']:.2f} us/launch, {fd['method_bytes_per_launch'] / 1e6:.3f} MB "
        f"method bytes/launch -> {achieved:.1f} GB/s")
    # the sweeps' two roofs (HBM bytes and dependency latency)
    lat = chain_latency(dev, args.roofline_reps)
    sroofs = sweep_roofs(solver, info, lat, args.roofline_reps)
    log(f"sweep latency: {lat}; levels: {sroofs}")
    # after the timed launches, so that the copy's write-backs do not land on them
    if args.copy_calibration > 0:
        nbytes = args.copy_calibration * (1 << 20)
        src = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {nbytes} bytes")
        del src, dst

    # the same system with the preconditioner in the other precision
    compare = None
    x_other = None
    if not args.no_compare_precision:
        other = "fp64" if args.precision == "fp32" else "fp32"
        t0 = time.perf_counter()
        s2 = cpc.Solver(p.n, p.row_ptr, p.col, p.val, device=dev, precision=other, tune=not args.rules)
        setup2 = time.perf_counter() - t0
        x2 = torch.zeros_like(b)
        for w in range(args.warmup):
            x2, it2, rel2, st2 = s2.solve(b, x=x2, tol=p.tol, maxit=10000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            x2, it2, rel2, st2 = s2.solve(b, x=x2, tol=p.tol, maxit=10000)
        torch.cuda.synchronize()
        ms2 = 1000.0 * (time.perf_counter() - t0) / args.steps
        st2s = s2.stats()
        m2 = st2s["method_bytes_per_iter"] * it2 + st2s["method_bytes_initial"]
        x64, x32 = (x2, x) if other == "fp64" else (x, x2)
        x_other = x2
        diff = float(torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64))
        compare = {"precision": other, "ms_per_solve": round(ms2, 4), "iters": it2, "relres": rel2,
                   "setup_s": round(setup2, 3), "method_gbs": round(m2 / (ms2 / 1000.0) / 1e9, 3),
                   "speedup_fp32_vs_fp64": round((ms2 / ms_per_step) if other == "fp64" else (ms_per_step / ms2), 4),
                   "x_relerr_fp32_vs_fp64": diff}
        log(f"{other}: {ms2:.3f} ms/solve iters={it2}; fp32 vs fp64 solution {diff:.2e}")
        s2.close()

    out = {
        "metric": "combined-PCG solve s + HBM GB/s to 1e-8 rel res; FP32-precond vs FP64",
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f64-pcg/f32-precond",
        "data": "synthetic",
        "config": {"workload": desc, "n": p.n, "nnz": p.nnz, "iters": it, "relres": rel,
                   "solve_s": round(ms_per_step / 1000.0, 6), "setup_s": round(setup_s, 3),
                   "levels": info["nlev"], "level_n": info["n"], "level_nnz": info["nnz"],
                   "level_depth": info["depth"], "level_smoother": info["smoother"],
                   "level_block_rows": info["block_rows"],
                   "level_inverse_bytes": info["inverse_bytes"],
                   "inverse_bytes_total": int(sum(info["inverse_bytes"])),
                   "matrix_bytes_total": int(sum(12 * z + 4 * (m + 1) for m, z in zip(info["n"], info["nnz"]))),
                   "method_bytes_per_solve": method_solve, "form_bytes_per_solve": form_solve,
                   "precision": args.precision},
        "roofline": roofline,
        "families": fam,
        "sweep_roofs": {"latency": lat, "levels": sroofs},
    }
    if compare:
        out["config"]["compare"] = compare
    if not args.no_cpu_baseline:
        h, r, osetup, osolve, _ = cpu_baseline(p, it)
        ob = stats["method_bytes_per_iter"] * r["iters"] + stats["method_bytes_initial"]
        if args.precision != "fp64":
            ob = None  # the oracle runs in FP64: its bytes are those of the FP64 method
        xo = r["x"]
        err = float(np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo))
        out["cpu_baseline"] = {"value": round(ob / osolve / 1e9, 4) if ob else None, "unit": "GB/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"one full solve of the same workload to 1e-8 on the host (setup "
                                         f"{osetup:.1f}s untimed); solve {osolve:.2f}s, {r['iters']} iterations; "
                                         f"GB/s on the method bytes of the FP64 solve",
                               "solve_s": round(osolve, 3), "setup_s": round(osetup, 3), "iters": r["iters"],
                               "host_cpus": os.cpu_count()}
        out["config"]["x_relerr_vs_oracle"] = err
        if compare and x_other is not None:
            xc = x_other.cpu().numpy()
            compare[f"x_relerr_{compare['precision']}_vs_fp64_oracle"] = float(np.linalg.norm(xc - xo) /
                                                                               np.linalg.norm(xo))
            import scipy.sparse as sp
            A = sp.csr_matrix((p.val, p.col, p.row_ptr), shape=(p.n, p.n))
            compare["true_relres"] = float(np.linalg.norm(p.b - A @ xc) / np.linalg.norm(p.b))
        log(f"oracle: {osolve:.2f}s {r['iters']} iters; GPU x vs oracle {err:.2e}")
    print(json.dumps(out), flush=True)
    solver.close()


if __name__ == "__main__":
    main()
