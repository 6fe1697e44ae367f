#!/usr/bin/env python3
"""Time-to-solution benchmark of M-IHS ridge regression on one MI355X.

Workload (synthetic, seeded): A = G diag(sigma) Q, n = 2^18, d = 2048, FP64,
sigma_i = exp(-8 i / d), lambda chosen for statistical dimension 512, b = A x0 + 1%
noise; SRHT sketch with m = 2048 rows; Corollary 4 momentum (beta = 512/2048).

One step = one whole solve from A, b resident in HBM: mihs_sketch + mihs_solve
until the stop rule fires.  The timed region covers K steps of the mixed path
(SRHT in FP32, FP32 inner CG, FP64 outer gradient) and, separately, K steps of
the plain FP64 path; each result's error against the closed-form solution is
checked to be <= 1e-10 after timing.

Prints ONE JSON line.  --gpus above 1 is refused: this build measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="srht_2p18x2048")
    ap.add_argument("--tol", type=float, default=5e-11)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-rows", type=int, default=1 << 15)
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(w, lam, rows):
    """The oracle (numpy FP64) on a bounded sample: the same workload recipe with
    the first `rows` rows (same d, m, lambda), sketch + M-IHS to 1e-10; the
    measured time is scaled by n / rows (both the sketch and the per-iteration
    pass are linear in n)."""
    import numpy as np
    import workloads as W
    from oracle import sketches, solver as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    P = W.make_problem(rows, w.d, w.sigma, w.sd_target, w.data_seed + 1)
    t0 = time.perf_counter()
    SA = sketches.sketch(P.A, w.sketch, w.m, w.sketch_seed, w.m2)
    a, b = O.momentum_cor4(w.sd_target, w.m)
    r = O.mihs(P.A, P.b, lam, SA, a, b, inner="cg", eps_sub=w.eps_sub, tol=1e-10)
    dt = time.perf_counter() - t0
    scale = w.n / rows
    return {"value": dt * scale * 1e3, "unit": "ms", "cores": cores, "kind": "oracle",
            "sample": (f"oracle sketch+solve of a {rows}x{w.d} instance of the same recipe "
                       f"({r.outer} outer / {sum(r.inner)} inner iterations, {dt:.1f} s), "
                       f"scaled by n/rows = {scale:g}")}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1912_03514_amd as mihs
    import workloads as W
    from oracle import solver as O

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    mihs.load_library()
    dev = torch.device("cuda", 0)
    w = W.workload(args.workload)
    lam = w.lam
    alpha, beta = mihs.momentum(w.sd_target, w.m)

    log(f"drawing {w.name}: n={w.n} d={w.d} ({w.a_dtype}) on the GPU")
    A, b, _x0, _ = W.make_problem_torch(w.n, w.d, w.sigma, w.sd_target, w.data_seed, dev,
                                        w.a_dtype)
    torch.cuda.synchronize()

    # closed-form reference on the host (the oracle's plain definition)
    log("closed-form reference on the host")
    A_h = A.cpu().numpy()
    b_h = b.cpu().numpy()
    t0 = time.perf_counter()
    x_ref = O.ridge_cholesky(A_h, b_h, lam)
    log(f"  reference in {time.perf_counter() - t0:.1f}s")

    stream = torch.cuda.current_stream(dev)

    def run(precision, steps, record):
        ws = mihs.SolveWorkspace(w.n, w.d, w.m, precision, dev)
        kind = w.sketch
        times, sk_ms, sv_ms, infos, xs = [], [], [], [], []
        for s in range(steps):
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            e0.record(stream)
            SA = mihs.mihs_sketch(A, kind, w.m, w.sketch_seed, precision=precision, m2=w.m2)
            e1.record(stream)
            x, info_raw = mihs.mihs_solve(A, b, lam, SA, alpha, beta, eps_sub=w.eps_sub,
                                          tol=args.tol, max_outer=300, max_inner=2000,
                                          precision=precision, workspace=ws, sync=False)
            e2.record(stream)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if record:
                times.append((t1 - t0) * 1e3)
                sk_ms.append(e0.elapsed_time(e1))
                sv_ms.append(e1.elapsed_time(e2))
                infos.append(mihs.info_to_dict(info_raw)[0])
                xs.append(x)
            del SA
        return times, sk_ms, sv_ms, infos, xs

    out = {}
    for precision in ("mixed", "plain"):
        log(f"{precision}: warmup {args.warmup}")
        run(precision, args.warmup, False)
        log(f"{precision}: timing {args.steps} steps")
        torch.cuda.synchronize()
        times, sk, sv, infos, xs = run(precision, args.steps, True)
        errs = [float(np.linalg.norm(x.cpu().numpy() - x_ref) / np.linalg.norm(x_ref)) for x in xs]
        out[precision] = dict(ms=float(np.mean(times)), sketch_ms=float(np.mean(sk)),
                              solve_ms=float(np.mean(sv)), infos=infos, errs=errs)
        log(f"  {precision}: {np.mean(times):.2f} ms/solve (sketch {np.mean(sk):.2f}, solve "
            f"{np.mean(sv):.2f}); outer {infos[-1]['outer_iters']}, inner "
            f"{infos[-1]['inner_iters_total']}; max err {max(errs):.2e}")

    mx, pl = out["mixed"], out["plain"]
    info = mx["infos"][-1]
    s_a = 8 if w.a_dtype == "f64" else 4
    apass_bytes = w.n * w.d * s_a + w.n * 8
    sa_bytes = w.m * w.d * 4  # mixed: FP32 sketch
    outer = info["outer_iters"]
    inner = info["inner_iters_total"]
    solve_bytes = outer * apass_bytes + inner * sa_bytes
    achieved = solve_bytes / (mx["solve_ms"] * 1e-3) / 1e9
    result = {
        "metric": "time-to-1e-10 rel.err per ridge solve (M-IHS, mixed precision; SRHT sketch + solve)",
        "value": round(mx["ms"], 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mx["ms"], 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 outer / f32 inner",
        "data": "synthetic (seeded A = G diag(sigma) Q, 1% noise)",
        "config": {"workload": w.name, "n": w.n, "d": w.d, "a_dtype": w.a_dtype,
                   "sketch": w.sketch, "m": w.m, "sd": w.sd_target, "lambda": lam,
                   "eps_sub": w.eps_sub, "tol": args.tol, "alpha": alpha, "beta": beta},
        "plain_fp64_ms": round(pl["ms"], 3),
        "mixed_speedup_vs_plain": round(pl["ms"] / mx["ms"], 3),
        "mixed": {"sketch_ms": round(mx["sketch_ms"], 3), "solve_ms": round(mx["solve_ms"], 3),
                  "outer_iters": outer, "inner_iters": inner,
                  "max_rel_err": max(mx["errs"])},
        "plain": {"sketch_ms": round(pl["sketch_ms"], 3), "solve_ms": round(pl["solve_ms"], 3),
                  "outer_iters": pl["infos"][-1]["outer_iters"],
                  "inner_iters": pl["infos"][-1]["inner_iters_total"],
                  "max_rel_err": max(pl["errs"])},
        "a_pass_bytes": apass_bytes,
        "roofline": {"bound": "hbm", "kernel": "solve_kernel (mixed)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
        "accuracy_ok": max(mx["errs"]) <= 1e-10 and max(pl["errs"]) <= 1e-10,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a bounded sample)")
        result["cpu_baseline"] = cpu_baseline(w, lam, args.cpu_sample_rows)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
