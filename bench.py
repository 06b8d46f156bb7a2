"""Benchmark: combined-preconditioned CG solve on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

A step is one whole solve (PCG with the combined ILU(0) + AMG preconditioner, the
complete hot path) of the 3-D 128x128x64 TPFA pressure system to relative residual
1e-8, with the matrix hierarchy and the right-hand side already resident in HBM.
value = algorithmic HBM bytes of one solve / solve time (GB/s); ms_per_step = solve
time. The roofline object is for the kernel that dominates the solve time; the CPU
baseline is the oracle solving the same system on the host.
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
# kernel reported in the roofline object (the kernel that dominates the solve time in
# the committed kernel-trace summary) and the committed traffic counters for it
ROOFLINE_KERNEL = "dense_gemv"
ROOFLINE_NAME = "gemv_tri_rows_kernel"
TRAFFIC_FILE = ROOT / "profiles" / "traffic_gemv_tri_rows_c2.txt"
KERNEL_SOURCE = ROOT / "paper_1205_6113_amd" / "csrc" / "dense_tri.hip"


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--roofline-reps", type=int, default=5)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU form is "
              "not built (see the sharding design).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1205_6113_amd as cpc

    p, desc = workload(args.workload)
    log(f"workload {desc}: n={p.n} nnz={p.nnz}")
    torch.cuda.init()
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    solver = cpc.Solver(p.n, p.row_ptr, p.col, p.val, device=dev, precision=args.precision)
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
    bytes_solve = stats["bytes_per_iter"] * it + stats["bytes_initial"]
    value = bytes_solve / (ms_per_step / 1000.0) / 1e9
    log(f"timed {args.steps} solves: {ms_per_step:.3f} ms/solve iters={it} relres={rel:.3e} -> {value:.1f} GB/s")

    # roofline of the dominant kernel family (HIP events on the solver's stream)
    tk = solver.time_kernel(ROOFLINE_KERNEL, level=-1, reps=args.roofline_reps)
    achieved = tk["bytes"] / (tk["avg_ms"] / 1000.0) / 1e9
    # counted HBM bytes per launch from the committed rocprofv3 counter passes, only if
    # they were taken on this workload, precision and kernel source
    traffic = None
    if TRAFFIC_FILE.exists():
        try:
            import hashlib
            tr = json.loads(TRAFFIC_FILE.read_text())
            src = hashlib.sha256(KERNEL_SOURCE.read_bytes()).hexdigest()
            if (tr.get("workload") == args.workload and tr.get("precision") == args.precision
                    and tr.get("kernel_source_sha256") == src):
                traffic = tr.get("bytes_per_launch")
        except Exception:
            traffic = None
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                "kernel": f"{ROOFLINE_NAME} (products with the explicit inverses of D+L or of its diagonal "
                          "blocks, both directions, every level smoothed that way)",
                "avg_launch_us": round(1000.0 * tk["avg_ms"], 3), "bytes_per_launch": tk["bytes"],
                "launches_timed": tk["launches"]}
    log(f"roofline {ROOFLINE_KERNEL}: {1000 * tk['avg_ms']:.2f} us/launch, {tk['bytes'] / 1e6:.2f} MB/launch "
        f"-> {achieved:.1f} GB/s")

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
                   "bytes_per_solve": bytes_solve, "precision": args.precision},
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        h, r, osetup, osolve, _ = cpu_baseline(p, it)
        ob = stats["bytes_per_iter"] * r["iters"] + stats["bytes_initial"]
        xo = r["x"]
        err = float(np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo))
        out["cpu_baseline"] = {"value": round(ob / osolve / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
                               "sample": f"one full solve of the same workload to 1e-8 on the host (setup "
                                         f"{osetup:.1f}s untimed); solve {osolve:.2f}s, {r['iters']} iterations",
                               "solve_s": round(osolve, 3), "iters": r["iters"],
                               "host_cpus": os.cpu_count()}
        out["config"]["x_relerr_vs_oracle"] = err
        log(f"oracle: {osolve:.2f}s {r['iters']} iters; GPU x vs oracle {err:.2e}")
    print(json.dumps(out), flush=True)
    solver.close()


if __name__ == "__main__":
    main()
