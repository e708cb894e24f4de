"""Benchmark of restarted PDHG with online preconditioning on one MI355X.

One step is one launch sequence of the hot path: the KKT evaluation with
its restart / termination decision, then 64 step attempts, each the
CSR(A^T) SpMV fused with the primal step, the CSR(A) SpMV fused with the
dual step and the adaptive step decision, and the AdaGrad learner on update
iterations (every 20th). The LP never terminates during timing (tol 0), so
every step does the full work.

Default workload: the badly scaled LP (m = 50k rows, 40% equality, n = 100k
columns, power-law column degree on 2..2000 with exponent 2.2, ~0.7M
nonzeros, row scales log-uniform in [1e-3, 1e3]), synthetic and seeded.

The printed JSON line reports accepted PDHG iterations per second
(whole-job throughput, data resident in HBM), the achieved bandwidth of
the dominant kernel against the HBM roofline (algorithmic bytes / kernel
time measured with HIP events on the solver's stream), and the FP64 CPU
oracle timed on a bounded sample of the same LP on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32|fp64]
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def primal_kernel_bytes(lp, vbytes: int) -> float:
    """Algorithmic bytes of one launch of the primal kernel.

    CSR(A^T): nnz values + nnz int32 column indices + (n+1) int32 row
    pointers; the gathered y read once (m values); the primal vectors:
    read x, c, l, u, T and the running sum, write x' and the new sum
    (8 n values).
    """
    nnz, m, n = lp.nnz, lp.m, lp.n
    return nnz * (vbytes + 4) + 4.0 * (n + 1) + vbytes * m + 8.0 * vbytes * n


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def oracle_baseline(lp, lr: float, phi: int, seconds: float) -> dict:
    """The FP64 oracle as it stands, single-threaded, on a bounded sample:
    as many accepted iterations of the same LP as fit in ~`seconds`."""
    import oracle
    from oracle.params import default_params
    # calibrate with a short run, then time a run sized to the budget
    t0 = time.perf_counter()
    r = oracle.solve(lp, default_params(tol=0.0, max_iter=4, lr=lr, phi=phi))
    per_it = max((time.perf_counter() - t0) / max(r.iterations, 1), 1e-4)
    iters = int(max(8, min(2000, seconds / per_it)))
    t0 = time.perf_counter()
    r = oracle.solve(lp, default_params(tol=0.0, max_iter=iters, lr=lr, phi=phi))
    dt = time.perf_counter() - t0
    return {
        "value": r.iterations / dt,
        "unit": "PDHG iters/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"first {r.iterations} iterations of the same LP (FP64, single thread, "
                  f"includes rescaling and setup), {dt:.1f} s on {cpu_model()} "
                  f"({os.cpu_count()} logical CPUs on the host)",
    }


def run(args) -> dict:
    import torch
    import paper_2506_17650_amd as P
    from lpgen import config_lp
    from lpgen.generators import summary

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    P.load()
    t = time.perf_counter()
    lp = config_lp(args.workload, scale=args.scale)
    shape = summary(lp)
    log(f"[bench] workload {args.workload} m={lp.m} n={lp.n} nnz={lp.nnz} "
        f"generated in {time.perf_counter() - t:.1f}s")
    prec = P.OPDHG_FP32 if args.precision == "fp32" else P.OPDHG_FP64
    vbytes = 4 if prec == P.OPDHG_FP32 else 8
    params = P.opdhg_default_params(precision=prec, tol=0.0, max_iter=10**12, lr=args.lr,
                                    phi=args.phi, normalize=1, time_limit_s=1e9,
                                    tile_nnz=args.tile_nnz, lanes=args.lanes,
                                    workgroups=args.workgroups)
    t = time.perf_counter()
    sess = P.Session(lp, params)
    log(f"[bench] session ready in {time.perf_counter() - t:.1f}s")
    sess.replay(args.warmup)
    torch.cuda.synchronize()
    _, _, _, _, st0 = sess.state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sess.replay(args.steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _, _, _, _, st1 = sess.state()
    iters = st1.k - st0.k
    attempts = st1.attempts - st0.attempts
    log(f"[bench] {args.steps} steps, {iters} iterations, {attempts} attempts in {dt:.3f}s; "
        f"status {st1.status}")
    if st1.status != P.capi.OPDHG_STATUS_RUNNING:
        raise SystemExit(f"solver stopped during timing (status {st1.status})")
    # dominant kernel: CSR(A^T) SpMV fused with the primal step
    reps = max(20, args.kernel_reps)
    ms = sess.time_primal_kernel(reps)
    kbytes = primal_kernel_bytes(lp, vbytes)
    achieved = kbytes / (ms * 1e-3) / 1e9
    sess.close()
    out = {
        "metric": "PDHG iters/s + SpMV HBM GB/s; LP solves/s and p99 latency at rel KKT 1e-4",
        "value": iters / dt,
        "unit": "PDHG iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == P.OPDHG_FP32 else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: badly scaled random LP, power-law column degree"
                        if args.workload == "cfg1" else args.workload,
            "m": lp.m, "n": lp.n, "nnz": lp.nnz,
            "row_len_mean": round(shape["row_len_mean"], 2),
            "col_len_max": shape["col_len_max"],
            "precision": args.precision + (" (reductions, steps, KKT in f64)"
                                           if prec == P.OPDHG_FP32 else ""),
            "attempts_per_step": 64,
            "tile_nnz": args.tile_nnz, "lanes": args.lanes, "workgroups": args.workgroups,
            "lr": args.lr, "phi": args.phi, "normalize": True,
            "attempts_per_s": attempts / dt,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "kernel": "k_primal (CSR(A^T) SpMV + primal step)",
            "bytes_per_launch": kbytes,
            "avg_launch_ms": ms,
        },
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle")
        out["cpu_baseline"] = oracle_baseline(lp, args.lr, args.phi, args.cpu_seconds)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="cfg1")
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--lr", type=float, default=1e-5)
    ap.add_argument("--phi", type=int, default=20)
    ap.add_argument("--kernel-reps", type=int, default=100)
    ap.add_argument("--tile-nnz", type=int, default=0, help="SpMV tile target (0: automatic)")
    ap.add_argument("--lanes", type=int, default=0, help="lanes per row (0: per tile)")
    ap.add_argument("--workgroups", type=int, default=0, help="workgroups per launch (0: auto)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: every LP here is solved on a single device "
              "(no multi-GPU path is built); run it with --gpus 1", file=sys.stderr)
        raise SystemExit(2)
    print(json.dumps(run(args)), flush=True)


if __name__ == "__main__":
    main()
