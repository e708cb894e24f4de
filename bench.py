"""Benchmark of restarted PDHG with online preconditioning on one MI355X.

One step is one launch sequence of the hot path on the resident LP: the KKT
evaluation with its restart / termination decision, then 64 step-attempt
slots, each the CSR(A^T) SpMV fused with the primal step, the CSR(A) SpMV
fused with the dual step, and the adaptive step decision, with a guarded
evaluation after every 16 slots and the AdaGrad learner on update
iterations (every 20th). The LP never terminates during timing (tol 0), so
every step does the full work.

Headline: accepted PDHG iterations per second on the block-angular LP
(64 blocks of 30k rows x 80k columns with 6 +-1 entries per column, plus
2,000 linking >= rows of ~2,140 N(0,1) entries; m = 1.922M, n = 5.12M,
35M nonzeros; synthetic, seeded), FP32 storage and SpMV with FP64
reductions, data resident in HBM. The same JSON line carries:
  roofline      the dominant kernel (the windowed primal step, k_primal_win):
                algorithmic bytes per launch / average launch time (HIP
                events on the solver's stream) against 8 TB/s, HBM traffic
                from rocprofv3 counters when a counter summary for the
                current kernel source exists; beside it the dual side and
                the whole iteration
  cpu_baseline  the FP64 oracle on a bounded sample of the same LP
  cfg1          the badly scaled power-law LP (50k x 100k, ~0.7M nonzeros)
                in FP32 and in FP64
  batch         256 LPs solved to relative KKT 1e-4 in one packed launch
                set (FP32), against plain FP64 PDHG (lr 0) one at a time,
                with the FP32 error against FP64 per result and the batch's
                bytes per batch-attempt against the HBM roofline
  serving       a Poisson stream of serving requests through the
                continuous-batching server (FP32), against plain FP64 PDHG
                served first-in first-out one at a time through the same
                server machinery (one LP at a time); p50 / p99 latency
  cfg2lit       (on request: --sections ...,cfg2lit) the block-angular LP
                with linking rows of the literal 2% density (102,400
                nonzeros each, nnz ~235M; minutes to generate)
  variants      (on request: --sections ...,variants) the paper's variant
                matrix with #Opt, SGM10 / mean iterations, GM / mean time
                and #Imp / #Wors on a mixed synthetic set, for restarted
                adaptive PDHG and for vanilla PDHG

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
                       [--sections cfg1,batch,serving[,cfg2lit][,variants]]
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
METRIC = "PDHG iters/s + SpMV HBM GB/s; LP solves/s and p99 latency at rel KKT 1e-4"
SECTIONS = ("cfg1", "batch", "serving")
SLOTS_PER_STEP = 64  # step-attempt slots per launch sequence
KERNEL_SOURCE = os.path.join(ROOT, "paper_2506_17650_amd", "csrc", "kernels.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------------------
# algorithmic bytes
# ---------------------------------------------------------------------------

def primal_kernel_bytes(lp, vbytes: int) -> float:
    """Algorithmic bytes of one launch of the primal kernel.

    CSR(A^T): nnz values + nnz int32 column indices + (n+1) int32 row
    pointers; the gathered y read once (m values); the primal vectors:
    read x, c, l, u, T and the running sum, write x' and the new sum
    (8 n values).
    """
    nnz, m, n = lp.nnz, lp.m, lp.n
    return nnz * (vbytes + 4) + 4.0 * (n + 1) + vbytes * m + 8.0 * vbytes * n


def dual_kernel_bytes(lp, vbytes: int) -> float:
    """Algorithmic bytes of one launch of the dual kernel.

    CSR(A): nnz values + indices + (m+1) row pointers; the gathered x' read
    once (n values); the dual vectors: read y, b, Sigma, A x and the running
    sum, write y', A x' and the new sum (8 m values), and the row senses
    (m bytes).
    """
    nnz, m, n = lp.nnz, lp.m, lp.n
    return nnz * (vbytes + 4) + 4.0 * (m + 1) + vbytes * n + 8.0 * vbytes * m + m


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def kernel_source_hash() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def counter_traffic(kernel: str, workload: str, precision: str):
    """HBM bytes per launch from a committed rocprofv3 counter summary.

    profiles/<kernel>_<workload>_<precision>_counters.txt holds the
    FETCH_SIZE and WRITE_SIZE readings of the kernel and of a device copy
    of known size, and the SHA-256 of the kernel source they were taken
    with. Returns None when the file is absent or the source has changed.
    """
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{precision}_counters.txt")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("kernel_source_sha256") != kernel_source_hash():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v, dtype=float), q)) if len(v) else None


# ---------------------------------------------------------------------------
# sections
# ---------------------------------------------------------------------------

def iterate_section(P, lp, prec, args, steps, warmup, reps):
    """Replays of the resident LP: iterations/s and kernel times."""
    params = P.opdhg_default_params(precision=prec, tol=0.0, max_iter=10**12, lr=args.lr,
                                    phi=args.phi, normalize=1, time_limit_s=1e9,
                                    tile_nnz=args.tile_nnz, lanes=args.lanes,
                                    workgroups=args.workgroups)
    import torch
    t = time.perf_counter()
    sess = P.Session(lp, params)
    log(f"[bench]   session ready in {time.perf_counter() - t:.1f}s")
    sess.replay(warmup)
    _, _, _, _, st0 = sess.state()
    torch.cuda.synchronize()
    # the K timed replays in up to 5 runs of consecutive replays, each
    # bracketed by a synchronization, for the spread of the rate
    nrun = max(1, min(5, steps))
    sizes = [steps // nrun + (1 if r < steps % nrun else 0) for r in range(nrun)]
    run_ms = []
    t0 = time.perf_counter()
    for sz in sizes:
        ta = time.perf_counter()
        sess.replay(sz)
        torch.cuda.synchronize()
        run_ms.append((time.perf_counter() - ta) * 1e3 / sz)
    dt = time.perf_counter() - t0
    _, _, _, _, st1 = sess.state()
    if st1.status != P.capi.OPDHG_STATUS_RUNNING:
        raise SystemExit(f"solver stopped during timing (status {st1.status})")
    primal_ms, dual_ms = sess.time_kernels(reps)
    sess.close()
    vb = 4 if prec == P.OPDHG_FP32 else 8
    kb = {"primal": primal_kernel_bytes(lp, vb), "dual": dual_kernel_bytes(lp, vb)}
    km = {"primal": primal_ms, "dual": dual_ms}
    import numpy as np
    runs = {"runs": len(run_ms), "ms_per_step_median": float(np.median(run_ms)),
            "ms_per_step_min": min(run_ms), "ms_per_step_max": max(run_ms)}
    return {
        "iters": st1.k - st0.k, "attempts": st1.attempts - st0.attempts, "seconds": dt,
        "runs": runs,
        "kernels": {k: {"avg_launch_ms": km[k], "bytes_per_launch": kb[k],
                        "achieved_GBs": kb[k] / (km[k] * 1e-3) / 1e9,
                        "frac": kb[k] / (km[k] * 1e-3) / 1e9 / HBM_PEAK_GBS}
                    for k in km},
    }


def section_headline(P, args):
    """The block-angular LP in FP32 (windowed products): the headline."""
    from lpgen import config_lp
    from lpgen.generators import summary
    t = time.perf_counter()
    lp = config_lp("cfg2")
    log(f"[bench] headline: cfg2 m={lp.m} n={lp.n} nnz={lp.nnz} "
        f"(generated in {time.perf_counter() - t:.1f}s)")
    r = iterate_section(P, lp, P.OPDHG_FP32, args, args.steps, args.warmup, args.kernel_reps)
    log(f"[bench] headline: {r['iters'] / r['seconds']:.0f} iters/s, "
        f"{r['attempts'] / args.steps:.2f} attempts per step of {SLOTS_PER_STEP} slots, primal "
        f"{r['kernels']['primal']['achieved_GBs']:.0f} GB/s, dual "
        f"{r['kernels']['dual']['achieved_GBs']:.0f} GB/s")
    # HBM traffic of each side from the committed counter summaries: the
    # primal side is the windowed kernel alone; the dual side is the windowed
    # kernel and the finish of the segmented rows (the linking rows, and the
    # few block rows that no chunk takes); no A row is left in tiles
    parts = {"primal": ["k_primal_win"], "dual": ["k_dual_win", "k_dual_seg"]}
    for side, names in parts.items():
        vals = [counter_traffic(nm, "cfg2", "fp32") for nm in names]
        k = r["kernels"][side]
        k["kernels"] = names
        k["traffic"] = None if any(v is None for v in vals) else sum(vals)
        if k["traffic"] is not None:
            k["traffic_GBs"] = k["traffic"] / (k["avg_launch_ms"] * 1e-3) / 1e9
    return lp, summary(lp), r


def section_cfg1(P, args):
    """The badly scaled power-law LP (MALL-resident) in FP32 and FP64."""
    from lpgen import config_lp
    from lpgen.generators import summary
    t = time.perf_counter()
    lp = config_lp("cfg1")
    shape = summary(lp)
    log(f"[bench] cfg1: m={lp.m} n={lp.n} nnz={lp.nnz} "
        f"(generated in {time.perf_counter() - t:.1f}s)")
    out = {"workload": "cfg1: badly scaled random LP, power-law column degree",
           "m": lp.m, "n": lp.n, "nnz": lp.nnz,
           "row_len_mean": round(shape["row_len_mean"], 2), "col_len_max": shape["col_len_max"],
           "note": "the matrix (5.6 MB in FP32) stays in the 256 MB MALL: GB/s here are "
                   "algorithmic bytes over kernel time, not HBM traffic"}
    precs = {"f32": P.OPDHG_FP32, "f64": P.OPDHG_FP64}
    for name in [q for q in args.cfg1_precisions.split(",") if q in precs]:
        prec = precs[name]
        r = iterate_section(P, lp, prec, args, args.cfg1_steps, args.warmup, args.kernel_reps)
        log(f"[bench] cfg1 {name}: {r['iters'] / r['seconds']:.0f} iters/s, "
            f"{r['attempts'] / args.cfg1_steps:.2f} attempts per step")
        out[name] = {"value": r["iters"] / r["seconds"], "unit": "PDHG iters/s",
                     "attempts_per_s": r["attempts"] / r["seconds"],
                     "attempts_per_step": r["attempts"] / args.cfg1_steps,
                     "slots_per_step": SLOTS_PER_STEP,
                     "executed_fraction": r["attempts"] / (args.cfg1_steps * SLOTS_PER_STEP),
                     "steps": args.cfg1_steps, "timing_runs": r["runs"], "kernels": r["kernels"]}
    return out


def section_cfg2lit(P, args):
    """cfg2 with linking rows of the literal 2% density (102,400 nonzeros
    each, nnz ~235M): the long rows run as segments of the windowed chunks.
    Opt-in (--sections ...,cfg2lit): generating it takes minutes."""
    from lpgen import config_lp
    from lpgen.generators import summary
    t = time.perf_counter()
    lp = config_lp("cfg2lit", log=lambda msg: log(f"[bench] cfg2lit: {msg} "
                                                  f"({time.perf_counter() - t:.0f}s)"))
    log(f"[bench] cfg2lit: m={lp.m} n={lp.n} nnz={lp.nnz} "
        f"(generated in {time.perf_counter() - t:.1f}s)")
    steps = max(2, args.steps // 4)
    r = iterate_section(P, lp, P.OPDHG_FP32, args, steps, 1, max(3, args.kernel_reps // 10))
    b_att = r["kernels"]["primal"]["bytes_per_launch"] + r["kernels"]["dual"]["bytes_per_launch"]
    att_s = r["attempts"] / r["seconds"]
    log(f"[bench] cfg2lit: {r['iters'] / r['seconds']:.0f} iters/s, primal "
        f"{r['kernels']['primal']['achieved_GBs']:.0f} GB/s, dual "
        f"{r['kernels']['dual']['achieved_GBs']:.0f} GB/s")
    shape = summary(lp)
    return {"workload": "cfg2 with 2% dense linking rows (102,400 nonzeros each)",
            "m": lp.m, "n": lp.n, "nnz": lp.nnz, "row_len_max": shape.get("row_len_max"),
            "value": r["iters"] / r["seconds"], "unit": "PDHG iters/s", "dtype": "f32",
            "steps": steps, "attempts_per_s": att_s, "timing_runs": r["runs"],
            "kernels": r["kernels"],
            "iteration": {"bytes_per_attempt": b_att, "achieved_GBs": b_att * att_s / 1e9,
                          "frac": b_att * att_s / 1e9 / HBM_PEAK_GBS}}


def section_batch(P, args):
    import numpy as np
    from lpgen import batch_lps
    t = time.perf_counter()
    lps = batch_lps(args.batch_size)
    nnz = sum(lp.nnz for lp in lps)
    log(f"[bench] batch: {len(lps)} cfg3 LPs, {nnz} nonzeros "
        f"(generated in {time.perf_counter() - t:.1f}s)")
    p32 = P.opdhg_default_params(precision=P.OPDHG_FP32, tol=1e-4, max_iter=200000,
                                 lr=args.lr, phi=args.phi, time_limit_s=600)
    p64 = P.opdhg_default_params(precision=P.OPDHG_FP64, tol=1e-4, max_iter=200000, lr=0.0,
                                 time_limit_s=600)
    import torch
    t0 = time.perf_counter()
    tun, p32 = P.opdhg_autotune(lps, p32, replays=args.tune_replays)
    log(f"[bench] batch: autotuned tile {tun.tile_nnz}, workgroups {tun.workgroups}: "
        f"{tun.attempts_per_s:.0f} attempts/s (automatic tiling {tun.default_attempts_per_s:.0f}), "
        f"{100 * tun.executed_fraction:.1f}% of slots executed; "
        f"{time.perf_counter() - t0:.1f}s")
    # the batch against the HBM roofline: one batch-attempt moves every LP's
    # primal- and dual-kernel bytes once (V = 4); the tuner's replays keep
    # all LPs running, so batch-attempts/s is the attempts/s over the count
    b_att = sum(primal_kernel_bytes(lp, 4) + dual_kernel_bytes(lp, 4) for lp in lps)
    ba_per_s = tun.attempts_per_s / len(lps)
    batch_gbs = b_att * ba_per_s / 1e9
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res32 = P.opdhg_solve_batch(lps, p32)
    wall32 = time.perf_counter() - t0
    loop32 = max(r.solve_seconds for _, _, r in res32)
    opt32 = sum(r.status == P.capi.OPDHG_STATUS_OPTIMAL for _, _, r in res32)
    log(f"[bench] batch: FP32 packed: {opt32}/{len(lps)} optimal in {wall32:.1f}s "
        f"(loop {loop32:.1f}s)")
    # plain FP64 PDHG one at a time on an evenly spaced sample of the batch
    idx = list(range(0, len(lps), max(1, len(lps) // args.batch_baseline)))[: args.batch_baseline]
    wall64, loop64, opt64, errs = 0.0, 0.0, 0, []
    for i in idx:
        t0 = time.perf_counter()
        x, y, r = P.opdhg_solve(lps[i], p64)
        wall64 += time.perf_counter() - t0
        loop64 += r.solve_seconds
        opt64 += r.status == P.capi.OPDHG_STATUS_OPTIMAL
        r32 = res32[i][2]
        errs.append(abs(r32.primal_obj - r.primal_obj) / (1.0 + abs(r.primal_obj)))
    log(f"[bench] batch: FP64 one at a time: {opt64}/{len(idx)} optimal in {wall64:.1f}s")
    kkt32 = [r.rel_kkt for _, _, r in res32]
    return {
        "workload": f"cfg3: {len(lps)} LPs, m log-uniform in [1k, 50k], n=2m, 3..8 per column",
        "lps": len(lps), "nnz_total": nnz, "dtype": "f32",
        "solves_per_s": opt32 / wall32, "solves_per_s_loop": opt32 / loop32,
        "optimal": opt32, "wall_s": wall32, "loop_s": loop32,
        "autotune": {"tile_nnz": tun.tile_nnz, "lanes": tun.lanes, "workgroups": tun.workgroups,
                     "candidates": tun.candidates, "replays": args.tune_replays,
                     "attempts_per_s": tun.attempts_per_s,
                     "automatic_tiling_attempts_per_s": tun.default_attempts_per_s,
                     "executed_fraction": tun.executed_fraction},
        "roofline": {"bound": "hbm", "achieved": batch_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": batch_gbs / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_batch_attempt": b_att, "batch_attempts_per_s": ba_per_s,
                     "note": "whole step (primal, dual and decision kernels of every LP) "
                             "over the tuner's timed replays; bytes from the per-kernel "
                             "algorithmic model (primal_kernel_bytes + dual_kernel_bytes), "
                             "V = 4"},
        "fp32_rel_kkt_max": max(kkt32),
        "baseline": {
            "kind": "plain FP64 PDHG (lr 0), one LP at a time, same GPU",
            "sample": f"{len(idx)} LPs evenly spaced in the batch", "optimal": opt64,
            "solves_per_s": opt64 / wall64, "solves_per_s_loop": opt64 / loop64,
        },
        "speedup_solves_per_s": (opt32 / wall32) / (opt64 / wall64) if opt64 else None,
        "fp32_vs_fp64_rel_objective_error": {
            "per_result": errs, "max": max(errs), "median": pct(errs, 50),
            "note": "|p32 - p64| / (1 + |p64|) on the sampled LPs; both at rel KKT <= 1e-4"},
    }


def section_serving(P, args):
    """Open-loop Poisson arrivals through the continuous-batching server.

    The first `serve_warmup` requests measure plain FP64 one-at-a-time
    throughput (mu_plain) and warm the server up; then `serve_requests`
    further requests arrive at rate 0.7 mu_plain and are served twice with
    the same arrival times: by the FP32 server (continuous batching, up to
    256 resident LPs, with the FP64 fallback for requests whose FP32 solve
    ends short of the tolerance) and by plain FP64 PDHG (lr 0) one LP at a
    time through the same server machinery (max_active 1, first in first
    out). Latency runs from submit to the result on the host.
    """
    import numpy as np
    from lpgen import config_lp
    from lpgen.generators import serving_requests
    nw, n = args.serve_warmup, args.serve_requests
    t = time.perf_counter()
    reqs = [config_lp("cfg4", index=i) for i in range(nw + n)]
    warm, meas = reqs[:nw], reqs[nw:]
    log(f"[bench] serving: {nw} warm-up + {n} measured cfg4 requests, nnz "
        f"{min(r.nnz for r in reqs)}..{max(r.nnz for r in reqs)} "
        f"(generated in {time.perf_counter() - t:.1f}s)")
    p32 = P.opdhg_default_params(precision=P.OPDHG_FP32, tol=1e-4, max_iter=200000,
                                 lr=args.lr, phi=args.phi, time_limit_s=600)
    p64 = P.opdhg_default_params(precision=P.OPDHG_FP64, tol=1e-4, max_iter=200000, lr=0.0,
                                 time_limit_s=600)
    # plain FP64 one at a time on the warm-up requests: mu_plain
    t0 = time.perf_counter()
    for lp in warm:
        P.opdhg_solve(lp, p64)
    mu_plain = nw / (time.perf_counter() - t0)
    rate = 0.7 * mu_plain
    arrivals, _ = serving_requests(n, rate)
    arrivals = np.asarray(arrivals) - arrivals[0]
    log(f"[bench] serving: FP64 one at a time: mu {mu_plain:.2f}/s; arrivals at {rate:.2f}/s")
    import torch
    free, _ = torch.cuda.mem_get_info()
    arena = int(min(args.serve_budget_gb * 1e9, 0.8 * free))

    def open_loop(srv, params):
        tickets = [None] * n
        t0 = time.perf_counter()

        def feed():
            for i, lp in enumerate(meas):
                d = arrivals[i] - (time.perf_counter() - t0)
                if d > 0:
                    time.sleep(d)
                tickets[i] = srv.submit(lp, params)

        th = threading.Thread(target=feed)
        th.start()
        th.join()
        res, lat, prec = [], [], []
        for x in tickets:
            res.append(srv.wait(x)[2])
            lat.append(srv.latency(x))
            prec.append(srv.precision(x))
        return res, lat, prec, time.perf_counter() - t0

    with P.Server(arena, precision=P.OPDHG_FP32, max_active=256,
                  fallback=P.OPDHG_FALLBACK_FP64) as srv:
        # warm-up, closed loop: every warm-up request at once
        t0 = time.perf_counter()
        for x in [srv.submit(lp, p32) for lp in warm]:
            srv.wait(x)
        mu_srv = nw / (time.perf_counter() - t0)
        log(f"[bench] serving: server closed loop (warm-up set) mu {mu_srv:.2f}/s")
        res32, lat32, prec32, span32 = open_loop(srv, p32)
        st = srv.stats()
    del srv
    torch.cuda.empty_cache()  # the FP32 server's arena goes back to the device
    ok32 = sum(r.status == P.capi.OPDHG_STATUS_OPTIMAL for r in res32)
    fell = [i for i in range(n) if prec32[i] == P.OPDHG_FP64]
    log(f"[bench] serving: FP32 server: {ok32}/{n} optimal ({len(fell)} solved again in FP64), "
        f"p50 {pct(lat32, 50):.3f}s p99 {pct(lat32, 99):.3f}s")
    # one LP at a time needs room for the largest request only (plus tables)
    one = max(P.opdhg_workspace_bytes(lp, p64) for lp in meas)
    with P.Server(min(arena, 4 * one + (256 << 20)), precision=P.OPDHG_FP64,
                  max_active=1) as srv:
        res64, lat64, _, span64 = open_loop(srv, p64)
    del srv
    torch.cuda.empty_cache()
    ok64 = sum(r.status == P.capi.OPDHG_STATUS_OPTIMAL for r in res64)
    log(f"[bench] serving: FP64 one at a time: {ok64}/{n} optimal, p50 {pct(lat64, 50):.3f}s "
        f"p99 {pct(lat64, 99):.3f}s")
    errs = [abs(a.primal_obj - b.primal_obj) / (1.0 + abs(b.primal_obj))
            for a, b, q in zip(res32, res64, prec32)
            if a.status == b.status == P.capi.OPDHG_STATUS_OPTIMAL and q == P.OPDHG_FP32]

    def statuses(res):
        out = {}
        for r in res:
            k = P.opdhg_status_name(r.status)
            out[k] = out.get(k, 0) + 1
        return out
    not_opt = [{"request": i, "status": P.opdhg_status_name(r.status), "nnz": meas[i].nnz,
                "iterations": r.iterations, "rel_kkt": r.rel_kkt}
               for i, r in enumerate(res32) if r.status != P.capi.OPDHG_STATUS_OPTIMAL]
    # preparation of the largest request, on the host and on the device
    # (session creation: validation, structure, rescaling, upload, initial
    # products), the best of three creations of each
    big = max(reqs, key=lambda lp: lp.nnz)
    prep = {}
    for name, mode in (("host", P.OPDHG_PREP_HOST), ("device", P.OPDHG_PREP_DEVICE)):
        q = P.opdhg_default_params(precision=P.OPDHG_FP32, prep=mode, lr=args.lr, phi=args.phi)
        for _ in range(3):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sess = P.Session(big, q)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            sess.close()
            prep[name] = min(prep.get(name, dt), dt)
    log(f"[bench] serving: preparing the largest request ({big.nnz} nonzeros): host "
        f"{prep['host']:.3f}s, device {prep['device']:.3f}s")
    return {
        "workload": f"cfg4: {n} measured requests after {nw} warm-up, m log-uniform in "
                    "[500, 500k], n=2.5m, power-law degree 4..10, Poisson arrivals",
        "requests": n, "warmup_requests": nw, "rate_per_s": rate,
        "rate_rule": "0.7 x plain FP64 one-at-a-time throughput on the warm-up requests",
        "arena_bytes": arena, "peak_bytes": st.peak_bytes, "dtype": "f32",
        "optimal": ok32, "statuses": statuses(res32), "not_optimal": not_opt,
        "fallback": "OPDHG_FALLBACK_FP64: a request whose FP32 solve ends short of its "
                    "tolerance is solved again in FP64 by the server",
        "fell_back": [{"request": i, "nnz": meas[i].nnz, "status": P.opdhg_status_name(res32[i].status),
                       "fp64_iterations": res32[i].iterations, "latency_s": lat32[i]}
                      for i in fell],
        "solves_per_s": ok32 / span32,
        "closed_loop_solves_per_s_warmup": mu_srv,
        "latency_p50_s": pct(lat32, 50), "latency_p99_s": pct(lat32, 99),
        "latency_max_s": max(lat32),
        "fp32_vs_fp64_rel_objective_error": {
            "compared": len(errs), "max": max(errs) if errs else None,
            "median": pct(errs, 50), "p99": pct(errs, 99),
            "note": "|p32 - p64| / (1 + |p64|) per request solved in FP32, both at rel KKT "
                    "<= 1e-4"},
        "largest_request_prep_s": {"nnz": big.nnz, "host": prep["host"], "device": prep["device"],
                                   "note": "session creation, best of three; requests of 2^20 nonzeros or more "
                                           "are prepared on the device in the server runs"},
        "baseline": {
            "kind": "plain FP64 PDHG (lr 0) served one LP at a time, first in first out, by the "
                    "same server (max_active 1) at the same arrival times on the same GPU",
            "optimal": ok64, "statuses": statuses(res64), "solves_per_s": ok64 / span64,
            "closed_loop_solves_per_s": mu_plain,
            "latency_p50_s": pct(lat64, 50), "latency_p99_s": pct(lat64, 99),
            "latency_max_s": max(lat64)},
    }


def section_variants(P, args):
    """The paper's variant matrix on a seeded synthetic instance set.

    Restarted adaptive PDHG (the cuPDLP.jl-style runs of Section 4.3): lr 0
    against NoNorm/Norm x Freq/Infreq, the rate chosen per instance from
    {1e-5, 1e-6, 1e-7}. Vanilla PDHG (Section 4.2): lr 0 against the
    normalized, every-iteration variant with the rate chosen per instance
    from {1e-1, 1e-2, 1e-3}, 5e4 iterations at most. Iteration counts come
    from packed batch solves (bit-identical to solo solves); times are the
    iteration-loop seconds of solo solves of the baseline and of each
    variant at its chosen rates. FP64 throughout. A third table compares the
    learning-rate schedules (AdaGrad per coordinate, AdaGrad on the norm,
    constant) and the preconditioner-weighted step rule on the restarted
    solver; its fixed-rate rows show each schedule with one rate for every
    instance (no per-instance tuning).
    """
    from lpgen import study_lps
    from paper_2506_17650_amd.metrics import best_over_grid, compare
    t = time.perf_counter()
    lps = study_lps(args.study_size)
    log(f"[bench] variants: {len(lps)} instances, {sum(lp.nnz for lp in lps)} nonzeros "
        f"(generated in {time.perf_counter() - t:.1f}s)")
    OPT = P.capi.OPDHG_STATUS_OPTIMAL

    def rec(r, timed):
        return {"optimal": r.status == OPT, "iterations": int(r.iterations),
                "seconds": r.solve_seconds if timed else None}

    def batch(params):
        return [rec(r, False) for _, _, r in P.opdhg_solve_batch(lps, params)]

    def solo(plist):
        return [rec(P.opdhg_solve(lp, q)[2], True) for lp, q in zip(lps, plist)]

    def study(make, grid, variants, base):
        t0 = time.perf_counter()
        methods = {"lr=0": solo([make(0.0, *base)] * len(lps))}
        fixed, chosen, mismatch = {}, {}, 0
        for name, kw in variants.items():
            by_rate = {lr: batch(make(lr, *kw)) for lr in grid}
            runs, rates = best_over_grid(by_rate)
            timed = solo([make(r if r is not None else grid[0], *kw) for r in rates])
            mismatch += sum(a["iterations"] != b["iterations"] for a, b in zip(runs, timed))
            methods[name] = timed
            chosen[name] = [r for r in rates]
            for lr in grid:
                fixed[f"{name} lr={lr:g}"] = compare(
                    {"lr=0": methods["lr=0"], "v": by_rate[lr]}, "lr=0")["rows"]["v"]
        table = compare(methods, "lr=0")
        for name, row in table["rows"].items():
            log(f"[bench]   {name:14s} opt {row['optimal']:3d}  SGM10 {row['iter_sgm10']:9.1f}  "
                f"mean {row['iter_mean']:9.1f}  imp {row['improved']:3d}  wors {row['worsened']:3d}")
        return {"table": table, "fixed_rate_rows": fixed, "chosen_rates": chosen,
                "batch_vs_solo_iteration_mismatches": mismatch,
                "seconds": time.perf_counter() - t0}, methods["lr=0"]

    def pdlp(lr, norm, phi):
        return P.opdhg_default_params(precision=P.OPDHG_FP64, tol=1e-4, lr=lr, normalize=norm,
                                      phi=phi, max_iter=args.study_max_iter, time_limit_s=600)

    def vanilla(lr, norm, phi):
        return P.opdhg_vanilla_params(lr, precision=P.OPDHG_FP64, normalize=norm, phi=phi)

    log("[bench] variants: restarted adaptive PDHG, rates {1e-5, 1e-6, 1e-7}")
    restarted, _ = study(pdlp, (1e-5, 1e-6, 1e-7),
                         {"NoNorm-Freq": (0, 1), "Norm-Freq": (1, 1), "NoNorm-Infreq": (0, 20),
                          "Norm-Infreq": (1, 20)}, (1, 20))
    log("[bench] variants: vanilla PDHG, rates {1e-1, 1e-2, 1e-3}")
    van, _ = study(vanilla, (1e-1, 1e-2, 1e-3), {"Norm-Freq": (1, 1)}, (1, 1))

    # step-rule norms and learning-rate schedules on the restarted solver
    # (Norm-Infreq): per-instance rates, and one rate for every instance
    def sched(lr, schedule, step_norm):
        return P.opdhg_default_params(precision=P.OPDHG_FP64, tol=1e-4, lr=lr, normalize=1,
                                      phi=20, schedule=schedule, step_norm=step_norm,
                                      max_iter=args.study_max_iter, time_limit_s=600)

    log("[bench] variants: schedules and step norms (restarted, Norm-Infreq)")
    schedules, base_runs = study(sched, (1e-5, 1e-6, 1e-7),
                                 {"AdaGrad-diag": (0, 0), "AdaGrad-norm": (1, 0),
                                  "constant": (2, 0), "AdaGrad-diag weighted-step": (0, 1)},
                                 (0, 0))
    # the weighted rule alone (lr 0 keeps T = S = I: it must equal the plain rule)
    weighted_lr0 = solo([sched(0.0, 0, 1)] * len(lps))
    schedules["weighted_step_lr0"] = compare({"lr=0": base_runs, "w": weighted_lr0},
                                             "lr=0")["rows"]["w"]
    return {"workload": "mixed synthetic set: cfg0-, cfg1-, cfg3- and cfg4-shaped LPs "
                        "(stand-in for the paper's benchmark collections)",
            "instances": len(lps), "dtype": "f64", "max_iter_restarted": args.study_max_iter,
            "restarted": restarted, "vanilla": van, "schedules": schedules}


def oracle_baseline(lp, lr: float, phi: int, seconds: float) -> dict:
    """The FP64 oracle as it stands, single-threaded, on a bounded sample of
    the same LP: its rescaling and start, the evaluation and first iteration
    at k = 0, then as many further iterations as fit in ~`seconds` (no
    evaluation falls among them), which give the rate."""
    import oracle
    from oracle import pdhg as OP
    from oracle.params import default_params
    p = default_params(tol=0.0, max_iter=10**9, lr=lr, phi=phi)
    t0 = time.perf_counter()
    slp = oracle.rescale(lp, p.ruiz_iters, p.pc_beta, p.l2_rescale)
    st = OP.initial_state(slp, p)
    setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    OP.solve_from_state(slp, st, p, stop_k=1)
    first = time.perf_counter() - t0
    # sized from the first iteration, which also carried the k = 0 evaluation
    # (about three more sparse products): a plain iteration costs less
    iters = int(max(2, min(p.eval_every - 2, seconds / max(first / 1.5, 1e-4))))
    t0 = time.perf_counter()
    r = OP.solve_from_state(slp, st, p, stop_k=1 + iters)
    dt = time.perf_counter() - t0
    done = r.iterations - 1
    return {
        "value": done / dt,
        "unit": "PDHG iters/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"iterations 2..{r.iterations} of the same LP (FP64, single thread): "
                  f"{done} iterations in {dt:.1f} s on {cpu_model()} ({os.cpu_count()} logical "
                  f"CPUs on the host); its rescaling and start ({setup:.1f} s) and the first "
                  f"iteration with the k = 0 evaluation ({first:.1f} s) ran before and are not "
                  f"in the rate",
    }


def run(args) -> dict:
    import torch
    import paper_2506_17650_amd as P

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    P.load()
    if args.copy_probe_mb > 0:
        # a device-to-device copy of known size, outside every timed region:
        # profiler counter runs scale the solver kernels' byte counters by it
        nb = int(args.copy_probe_mb * 2**20)
        src = torch.ones(nb, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"[bench] copy probe: {nb} bytes device to device")
    sections = [s for s in args.sections.split(",") if s]
    lp, shape, main = section_headline(P, args)
    ker = main["kernels"]
    prim = ker["primal"]
    # one attempt moves the primal and the dual kernel's bytes once (the
    # decision kernel reads partial sums only); the whole-step rate counts
    # every attempt, evaluations and decisions included in the time
    b_att = prim["bytes_per_launch"] + ker["dual"]["bytes_per_launch"]
    att_s = main["attempts"] / main["seconds"]
    whole = b_att * att_s / 1e9
    out = {
        "metric": METRIC,
        "value": main["iters"] / main["seconds"],
        "unit": "PDHG iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main["seconds"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "cfg2: block-angular LP, 64 blocks of 30k x 80k (6 +-1 per column) "
                        "+ 2k linking rows of ~2,140 N(0,1) entries",
            "m": lp.m, "n": lp.n, "nnz": lp.nnz,
            "row_len_mean": round(shape["row_len_mean"], 2), "col_len_max": shape["col_len_max"],
            "precision": "f32 A, vectors and SpMV; f64 reductions, steps and KKT",
            "slots_per_step": SLOTS_PER_STEP,
            "attempts_per_step": main["attempts"] / args.steps,
            "executed_fraction": main["attempts"] / (args.steps * SLOTS_PER_STEP),
            "attempts_per_s": att_s,
            "timing_runs": main["runs"],
            "windows": "automatic (every A^T row windowed; every A row in a windowed chunk or a "
                       "segment of one)",
            "lr": args.lr, "phi": args.phi, "normalize": True,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": prim["achieved_GBs"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": prim["frac"],
            "traffic": prim.get("traffic"),
            "kernel": "k_primal_win",
            "bytes_per_launch": prim["bytes_per_launch"],
            "avg_launch_ms": prim["avg_launch_ms"],
            "sides": ker,
            "iteration": {"bytes_per_attempt": b_att, "attempts_per_s": att_s,
                          "achieved_GBs": whole, "frac": whole / HBM_PEAK_GBS,
                          "note": "both sparse-product sides' algorithmic bytes per attempt x "
                                  "attempts/s over the timed replays (decisions, evaluations "
                                  "and launch gaps in the time)"},
        },
    }
    if "cfg1" in sections:
        out["cfg1"] = section_cfg1(P, args)
    if "cfg2lit" in sections:
        out["cfg2lit"] = section_cfg2lit(P, args)
    if "batch" in sections:
        out["batch"] = section_batch(P, args)
    if "serving" in sections:
        out["serving"] = section_serving(P, args)
    if "variants" in sections:
        out["variants"] = section_variants(P, args)
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle")
        out["cpu_baseline"] = oracle_baseline(lp, args.lr, args.phi, args.cpu_seconds)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--sections", default=",".join(SECTIONS))
    ap.add_argument("--lr", type=float, default=1e-5)
    ap.add_argument("--phi", type=int, default=20)
    ap.add_argument("--kernel-reps", type=int, default=100)
    ap.add_argument("--tile-nnz", type=int, default=0, help="SpMV tile target (0: automatic)")
    ap.add_argument("--lanes", type=int, default=0, help="lanes per row (0: per tile)")
    ap.add_argument("--workgroups", type=int, default=0, help="workgroups per launch (0: auto)")
    ap.add_argument("--cfg1-steps", type=int, default=20)
    ap.add_argument("--cfg1-precisions", default="f32,f64",
                    help="precisions of the power-law LP section (f32, f64 or both)")
    ap.add_argument("--batch-size", type=int, default=256)
    ap.add_argument("--batch-baseline", type=int, default=16)
    ap.add_argument("--tune-replays", type=int, default=4)
    ap.add_argument("--serve-warmup", type=int, default=24)
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--study-size", type=int, default=24)
    ap.add_argument("--study-max-iter", type=int, default=100000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mb", type=float, default=0.0,
                    help="copy this many MiB device to device first (counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: every LP here is solved on a single device "
              "(no multi-GPU path is built); run it with --gpus 1", file=sys.stderr)
        raise SystemExit(2)
    print(json.dumps(run(args)), flush=True)


if __name__ == "__main__":
    main()
