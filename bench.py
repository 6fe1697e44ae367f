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

Prints ONE JSON line.  --gpus above 1 is refused: the solver runs on one GPU.

Other workloads (opt-in, one JSON line each): --workload small_gauss (4096 x 256,
Gaussian m = 256), batched_lambda_path (256 problems x 16 lambdas, Gaussian
sketches, one launch), diff_2p18x1024 (64 right-hand sides, forward + adjoint
backward through the autograd op), count_2p20x4096 (FP32 A, CountSketch ->
Gaussian), dual_4096x2p16 (under-determined, Dual M-IHS), pd_16384x4096
(square-like, Primal-Dual M-IHS).
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
    ap.add_argument("--tol", type=float, default=None,
                    help="relative-step stop tolerance (default: per workload, chosen so "
                         "that the result is within 1e-10 of x*)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true",
                    help="batched workload: skip the after-timing check of all 4096 results "
                         "against QR closed forms (for profiler runs: its ~2 million library "
                         "launches end them before they write their output); the line then "
                         "says the results were not checked")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the 2^20 x 4096 CountSketch workload of the default line")
    ap.add_argument("--large-steps", type=int, default=1)
    ap.add_argument("--tol-large", type=float, default=None)
    ap.add_argument("--cpu-sample-rows", type=int, default=0,
                    help="rows of the oracle's CPU baseline instance (0: the full workload)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy three times (the reference "
                         "kernel for scaling HBM byte counters) and exit")
    return ap.parse_args()


# HBM bytes per launch of the persistent solve kernel, from two rocprofv3 --pmc
# runs (FETCH_SIZE, then WRITE_SIZE, each scaled by what the counter reads for a
# plain 1 GiB device copy: x1.99992 for FETCH_SIZE, x1.000 for WRITE_SIZE); see
# profiles/solve_kernel_srht_2p18x2048.md.  Valid for the kernel as profiled, on
# the launch of 35 outer / 342 inner iterations.
MEASURED_TRAFFIC = {("srht_2p18x2048", "mixed"): 151142182626}

# Stop-rule tolerance per workload: the relative-step rule estimates the error
# from the Corollary 4 rate sqrt(beta); where the observed rate is slower (the
# two-stage sketch of the ill-conditioned FP32 workload, the batched paths) the
# tolerance is tighter.  The headline stops at the metric's own 1e-10, the rule
# its CPU baseline (the oracle) uses too; every workload's final error is
# checked against 1e-10 after timing.
DEFAULT_TOL = {"count_2p20x4096": 2e-12, "batched_lambda_path": 3e-12, "srht_2p18x2048": 1e-10}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# ---- reference solutions for the accuracy checks ----------------------------
# Plain closed forms written here (independent of the library under test):
# x* = (A^T A + lambda I)^{-1} A^T b by Cholesky of the Gram matrix, and the dense
# adjoint gradient.  For ill-conditioned workloads the Cholesky solution is
# refined with residual gradients accumulated in extended (long double) precision.

def ref_ridge(A, B, lam):
    """numpy FP64: (A^T A + lam I)^{-1} A^T B."""
    import numpy as np
    import scipy.linalg as sl
    A = np.asarray(A, dtype=np.float64)
    H = A.T @ A + lam * np.eye(A.shape[1])
    return sl.cho_solve(sl.cho_factor(H), A.T @ B)


def ref_backward(A, lam, X, gbar):
    """W = (A^T A + lam I)^{-1} gbar, dB = A W, dlam = -sum X .* W (dense FP64)."""
    import numpy as np
    import scipy.linalg as sl
    A = np.asarray(A, dtype=np.float64)
    H = A.T @ A + lam * np.eye(A.shape[1])
    Wm = sl.cho_solve(sl.cho_factor(H), gbar)
    return Wm, A @ Wm, -float(np.sum(X * Wm))


def ref_ridge_device(A, b, lam, refine=0, chunk=1 << 16):
    """Closed form on the GPU with torch FP64 (Gram in row chunks, Cholesky), then
    `refine` steps x += (A^T A + lam I)^{-1} (A^T (b - A x) - lam x) with A^T r
    accumulated on the host in long double.  Returns a host FP64 vector."""
    import concurrent.futures as cf
    import numpy as np
    import torch
    n, d = A.shape
    dev = A.device
    H = torch.zeros(d, d, dtype=torch.float64, device=dev)
    Atb = torch.zeros(d, dtype=torch.float64, device=dev)
    for r0 in range(0, n, chunk):
        Ac = A[r0:r0 + chunk].double()
        H += Ac.T @ Ac
        Atb += Ac.T @ b[r0:r0 + chunk]
        del Ac
    H += lam * torch.eye(d, dtype=torch.float64, device=dev)
    Lc = torch.linalg.cholesky(H)
    x = torch.cholesky_solve(Atb[:, None], Lc)[:, 0]
    del H, Atb
    for step in range(refine):
        r = torch.empty(n, dtype=torch.float64, device=dev)
        for r0 in range(0, n, chunk):
            r[r0:r0 + chunk] = b[r0:r0 + chunk] - A[r0:r0 + chunk].double() @ x
        rh = r.cpu().numpy()
        rows = 1 << 14

        def part(r0):
            Ac = A[r0:r0 + rows].cpu().numpy().astype(np.longdouble)
            return Ac.T @ rh[r0:r0 + rows].astype(np.longdouble)

        with cf.ThreadPoolExecutor(max_workers=8) as ex:
            parts = list(ex.map(part, range(0, n, rows)))
        atr = np.zeros(d, dtype=np.longdouble)
        for q in parts:  # fixed order
            atr += q
        g = atr - np.longdouble(lam) * x.cpu().numpy().astype(np.longdouble)
        gd = torch.from_numpy(g.astype(np.float64)).to(dev)
        dx = torch.cholesky_solve(gd[:, None], Lc)[:, 0]
        log(f"  refinement step {step + 1}: |dx|/|x| = {float(dx.norm() / x.norm()):.2e}")
        x = x + dx
    return x.cpu().numpy()


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, lam, A_dev, b_dev, rows):
    """The oracle (numpy/scipy FP64, as it stands) timed on the host cores:
    sketch + M-IHS with its CG inner solver to 1e-10.  rows = n (the default) is
    the full workload, on the same A and b the GPU solved (copied to the host
    before timing); a smaller `rows` times a seeded instance of that many rows
    drawn from the same recipe and scales the time by n / rows (both the sketch
    and the per-iteration pass are linear in n)."""
    import workloads as W
    from oracle import sketches, solver as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:  # pragma: no cover
        cores = os.cpu_count() or 1
    if rows >= w.n:
        A, b = A_dev.cpu().numpy(), b_dev.cpu().numpy()
        what = f"the full {w.n}x{w.d} workload (the GPU's A and b)"
        scale = 1.0
    else:
        P = W.make_problem(rows, w.d, w.sigma, w.sd_target, w.data_seed + 1)
        A, b = P.A, P.b
        scale = w.n / rows
        what = (f"a {rows}x{w.d} instance of the same recipe, scaled by n/rows = {scale:g}")
    t0 = time.perf_counter()
    SA = sketches.sketch(A, w.sketch, w.m, w.sketch_seed, w.m2)
    a, be = O.momentum_cor4(w.sd_target, w.m_out)
    r = O.mihs(A, b, lam, SA, a, be, inner="cg", eps_sub=w.eps_sub, tol=1e-10)
    dt = time.perf_counter() - t0
    return {"value": round(dt * scale * 1e3, 1), "unit": "ms", "cores": cores, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": (f"oracle sketch + M-IHS (CG inner) to 1e-10 on {what}: "
                       f"{r.outer} outer / {sum(r.inner)} inner iterations, {dt:.1f} s")}


def timed(fn, steps, warmup, stream):
    """Run fn warmup + steps times; return per-step wall ms (synchronised) and results."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    times, outs = [], []
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs.append(fn())
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t0) * 1e3)
    return times, outs


def ridge_path_qr(A, b, lams):
    """Closed forms of one problem's lambda-path on the device with torch
    (Householder QR of A, then a small QR of [R; sqrt(lam) I] per lambda;
    backward stable, independent of the library).  Returns host d x k."""
    import numpy as np
    import torch
    n, d = A.shape
    Q, R = torch.linalg.qr(A.to(torch.float64))
    c = Q.transpose(0, 1).contiguous() @ b.to(torch.float64)
    del Q
    lam = torch.as_tensor(np.asarray(lams, dtype=np.float64), device=A.device)
    k = lam.numel()
    eye = torch.eye(d, dtype=torch.float64, device=A.device)
    M = torch.cat([R.expand(k, d, d), torch.sqrt(lam)[:, None, None] * eye], dim=1).contiguous()
    rhs = torch.cat([c.expand(k, d), torch.zeros(k, d, dtype=torch.float64, device=A.device)],
                    dim=1)[:, :, None].contiguous()
    Q2, R2 = torch.linalg.qr(M)
    x = torch.linalg.solve_triangular(R2, Q2.transpose(1, 2).contiguous() @ rhs, upper=True)
    return x[:, :, 0].transpose(0, 1).contiguous().cpu().numpy()


def run_batched(args):
    """256 problems x 16 lambdas (n_k in [4096, 65536], d_k in [64, 512], FP64 A),
    one Gaussian sketch per problem, then all 4096 lambda-path solves in one
    launch of the block kernel.  One step (the 256 sketches round-robin on four
    streams, i.e. four branches of the graph, x^1 = 0 and the batched launch) is
    captured in a HIP graph and the timed steps are graph replays.

    Three configurations, each tuned by the library's autotuner (untimed, once):
      mixed  BF16 sketches, the decomposition-free inner CG of Algorithm 1 (the
             headline `value`);
      plain  FP64 sketches on the FP64 matrix cores, inner CG: the plain FP64
             GPU baseline;
      exact  BF16 sketches, exact sub-solves (Exact M-IHS, one Cholesky factor
             per column), reported beside the others.
    Every one of the 4096 results of the headline run is checked against its
    QR closed form after timing."""
    import numpy as np
    import torch
    import paper_1912_03514_amd as mihs
    import workloads as W
    dev = torch.device("cuda", 0)
    specs = W.batched_specs()
    log(f"drawing {len(specs)} problems on the GPU")
    probs = []
    for s in specs:
        sig = W.sigma_profile("exp", s.d, 6.0)
        A, b, _, _ = W.make_problem_torch(s.n, s.d, sig, s.d / 2, s.seed, dev, "f64")
        ld = (s.d + 1) // 2 * 2  # 16-byte rows, so nothing is copied inside the step
        Ab = torch.zeros((s.n, ld), dtype=torch.float64, device=dev)
        Ab[:, :s.d] = A
        del A
        probs.append((Ab[:, :s.d], b))
    torch.cuda.synchronize()
    nlam = len(specs[0].lambdas)
    lam = np.stack([s.lambdas for s in specs])
    sds = np.stack([[W.nominal_sd(W.sigma_profile("exp", s.d, 6.0), float(l)) for l in s.lambdas]
                    for s in specs])
    ms = np.array([s.m for s in specs], dtype=np.float64)
    betas = np.minimum(sds / ms[:, None], 0.95)
    alphas = (1.0 - betas) ** 2
    lam_d = torch.as_tensor(lam, device=dev)
    al_d = torch.as_tensor(alphas, device=dev)
    be_d = torch.as_tensor(betas, device=dev)
    eps_sub = 0.1
    nsk = 4
    sk_streams = [torch.cuda.Stream(device=dev) for _ in range(nsk)]

    def make_sketches(precision):
        dt = torch.float32 if precision == "mixed" else torch.float64
        per = 4 if precision == "mixed" else 2
        sks = [torch.zeros((s.m, (s.d + per - 1) // per * per), dtype=dt, device=dev)[:, :s.d]
               for s in specs]
        wsb = max(mihs.sketch_workspace_bytes(s.n, s.d, s.m, "gaussian", precision)
                  for s in specs)
        wss = [torch.empty(wsb, dtype=torch.uint8, device=dev) for _ in range(nsk)]
        return sks, wss

    def sketch_all(precision, sks, wss):
        main = torch.cuda.current_stream()
        for st in sk_streams:
            st.wait_stream(main)
        for i, ((A, b), s) in enumerate(zip(probs, specs)):
            with torch.cuda.stream(sk_streams[i % nsk]):
                mihs.mihs_sketch(A, "gaussian", s.m, 10 + i, precision=precision, out=sks[i],
                                 workspace=wss[i % nsk])
        for st in sk_streams:
            main.wait_stream(st)

    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]

    def configuration(name, precision, allow_exact, steps, warmup):
        sks, wss = make_sketches(precision)
        sketch_all(precision, sks, wss)
        solver = mihs.BatchedSolver([(A, b, SA) for (A, b), SA in zip(probs, sks)], lam_d, al_d,
                                    be_d, eps_sub=eps_sub, tol=args.tol, max_outer=400,
                                    max_inner=2000)
        log(f"{name}: autotuning the launch shape (exact sub-solves "
            f"{'allowed' if allow_exact else 'not allowed'})")
        t0 = time.perf_counter()
        tune = solver.tune(trial_outer=8, allow_exact=allow_exact)
        tune["wall_s"] = round(time.perf_counter() - t0, 2)
        log(f"  {tune}")

        def eager_step():
            ev[0].record()
            sketch_all(precision, sks, wss)
            ev[1].record()
            solver.run()
            ev[2].record()
            torch.cuda.synchronize()
            return ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])

        eager_times, eager_outs = timed(eager_step, 1, 1, None)
        sketch_ms, solve_ms = eager_outs[-1]
        graph = torch.cuda.CUDAGraph()
        cs = torch.cuda.Stream(device=dev)
        cs.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(cs):
            with torch.cuda.graph(graph, stream=cs):
                sketch_all(precision, sks, wss)
                solver.run()
        torch.cuda.current_stream().wait_stream(cs)
        torch.cuda.synchronize()
        times, _ = timed(graph.replay, steps, warmup, None)
        infos = solver.infos()
        outer = np.array([[r["outer_iters"] for r in inf] for inf in infos])
        inner = np.array([[r["inner_iters_total"] for r in inf] for inf in infos])
        status = np.array([[r["status"] for r in inf] for inf in infos])
        out = {"ms": float(np.mean(times)), "eager_step_ms": float(np.mean(eager_times)),
               "solve_ms": solve_ms, "sketch_ms": sketch_ms, "tuning": tune,
               "outer_iters_max": int(outer.max()), "outer_iters_mean": float(outer.mean()),
               "inner_iters_mean": float(inner.mean()),
               "all_converged": bool((status == 0).all()), "outer": outer,
               "xs": [x.clone() for x in solver.xs],
               "elapsed_ms": np.array([inf[0]["elapsed_us"] for inf in infos]) * 1e-3}
        log(f"  {name}: {out['ms']:.2f} ms/step (sketches {sketch_ms:.2f}, solve {solve_ms:.2f}); "
            f"outer max {out['outer_iters_max']}, mean {out['outer_iters_mean']:.1f}")
        del graph
        solver.close()
        del solver, sks, wss
        torch.cuda.synchronize()
        return out

    res = {"mixed": configuration("mixed, inner CG", "mixed", False, args.steps, args.warmup)}
    short = max(1, min(args.steps, 3))
    res["plain"] = configuration("plain FP64, inner CG", "plain", False, short, 1)
    res["exact"] = configuration("mixed, exact sub-solves", "mixed", True, short, 1)

    worst = {k: 0.0 for k in res}
    if args.no_check:
        log("results not checked (--no-check)")
    else:
        log("checking all 4096 results of every configuration against QR closed forms")
    for i, ((A, b), s) in enumerate(zip(probs, specs) if not args.no_check else []):
        ref = ridge_path_qr(A, b, s.lambdas)
        nrm = np.linalg.norm(ref, axis=0)
        for k, r in res.items():
            X = r["xs"][i].cpu().numpy()
            e = float(np.max(np.linalg.norm(X - ref, axis=0) / nrm))
            worst[k] = max(worst[k], e)
    if not args.no_check:
        log(f"  worst relative errors {worst}")
    mx = res["mixed"]
    apass = sum(s.n * s.d * 8 for s in specs)
    # per-problem outer counts: every entry passes over its A once per outer
    # iteration of its slowest column, with 16 columns per pass (4 n d x 16 flops)
    flops = sum(4.0 * s.n * s.d * 16 * int(mx["outer"][i].max()) for i, s in enumerate(specs))
    bytes_moved = sum(s.n * s.d * 8 * int(mx["outer"][i].max()) for i, s in enumerate(specs))
    tf = flops / (mx["solve_ms"] * 1e-3) / 1e12
    slow = np.argsort(-mx["elapsed_ms"])[:5]
    clean = lambda r: {k: (round(v, 3) if isinstance(v, float) else v) for k, v in r.items()
                       if k not in ("outer", "xs", "elapsed_ms")}
    value = mx["ms"]
    return {
        "metric": "time to solve 256 ridge problems x 16 lambdas to 1e-10 (sketch + batched "
                  "M-IHS, inner CG)",
        "value": round(value, 3), "unit": "ms", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(value, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 outer (BF16 sketches)", "data": "synthetic",
        "config": {"workload": "batched_lambda_path", "problems": len(specs), "nlam": nlam,
                   "n_range": [4096, 65536], "d_range": [64, 512], "eps_sub": eps_sub,
                   "tol": args.tol, "a_bytes_total": apass},
        "timing": "HIP-graph replay of one step (256 sketches + batched launch)",
        "mixed_cg": clean(mx),
        "plain_fp64_cg": clean(res["plain"]),
        "plain_fp64_ms": round(res["plain"]["ms"], 3),
        "mixed_speedup_vs_plain": round(res["plain"]["ms"] / value, 3),
        "exact_subsolves": clean(res["exact"]),
        "max_rel_err_all_4096": None if args.no_check else worst,
        "accuracy_ok": None if args.no_check else all(v <= 1e-10 for v in worst.values()),
        "slowest_entries": [{"problem": int(i), "n": specs[i].n, "d": specs[i].d,
                             "ms": round(float(mx["elapsed_ms"][i]), 2),
                             "outer_max": int(mx["outer"][i].max())} for i in slow],
        "roofline": {"bound": "mfma", "kernel": "batched_kernel (mixed, inner CG)",
                     "achieved": round(tf, 2), "peak": 78.6, "unit": "TFLOP/s",
                     "frac": round(tf / 78.6, 4), "traffic": None,
                     "a_pass_gbs": round(bytes_moved / (mx["solve_ms"] * 1e-3) / 1e9, 1)},
    }


def run_diff(args):
    """n = 2^18, d = 1024, FP32 A, 64 right-hand sides: forward (multi-RHS M-IHS on an
    SRHT sketch) + backward (adjoint M-IHS) of L = sum_j ||C x*_j - y_j||^2 through
    the autograd op; dL/dB and dL/dlog(lambda) checked against the dense FP64 gradient."""
    import numpy as np
    import torch
    import paper_1912_03514_amd as mihs
    import workloads as W
    dev = torch.device("cuda", 0)
    w = W.workload("diff_2p18x1024")
    log("drawing the differentiation workload on the GPU")
    A, B, _, lam = W.make_problem_torch(w.n, w.d, w.sigma, w.sd_target, w.data_seed, dev,
                                        w.a_dtype, nrhs=w.nrhs)
    g = torch.Generator(device=dev).manual_seed(w.data_seed + 1)
    C = torch.randn(128, w.d, generator=g, dtype=torch.float64, device=dev)
    Y = torch.randn(128, w.nrhs, generator=g, dtype=torch.float64, device=dev)
    alpha, beta = mihs.momentum(w.sd_target, w.m_out)
    kw = dict(eps_sub=w.eps_sub, tol=1e-12, max_outer=300)
    ll0 = math.log(lam)

    def step():
        SA = mihs.mihs_sketch(A, "srht", w.m, w.sketch_seed)
        Bt = B.clone().requires_grad_(True)
        ll = torch.tensor(ll0, dtype=torch.float64, device=dev, requires_grad=True)
        X = mihs.MIHSRidge.apply(Bt, ll, A, SA, alpha, beta, kw)
        L = ((C @ X - Y) ** 2).sum()
        L.backward()
        return X.detach(), Bt.grad, ll.grad

    times, outs = timed(step, args.steps, args.warmup, None)
    X, dB, dll = outs[-1]
    log("dense FP64 reference gradient on the host")
    A64 = A.double().cpu().numpy()
    Bh = B.cpu().numpy()
    Xs = ref_ridge(A64, Bh, lam)
    Ch, Yh = C.cpu().numpy(), Y.cpu().numpy()
    gbar = 2 * Ch.T @ (Ch @ Xs - Yh)
    _, dBref, dlref = ref_backward(A64, lam, Xs, gbar)
    ex = float(np.linalg.norm(X.cpu().numpy() - Xs) / np.linalg.norm(Xs))
    eb = float(np.linalg.norm(dB.cpu().numpy() - dBref) / np.linalg.norm(dBref))
    el = abs(float(dll) - lam * dlref) / abs(lam * dlref)
    # matrix-core work of one step: every block-kernel entry (16 columns) passes over A
    # once per outer iteration with 4 n d x 16 flops (U = C - A X and A^T U), forward and
    # adjoint, plus dB = A W (2 n d x 64); the outer counts come from an untimed repeat
    SA = mihs.mihs_sketch(A, "srht", w.m, w.sketch_seed)
    _, finf = mihs.mihs_solve_multi(A, B, lam, SA, alpha, beta, **kw)
    _, _, _, binf = mihs.mihs_solve_backward(A, SA, lam, X.contiguous(),
                                             torch.as_tensor(gbar, device=dev), alpha, beta,
                                             want_dB=True, **kw)
    passes = 0
    for inf in (finf, binf):
        outer = [r["outer_iters"] for r in inf]
        passes += sum(max(outer[g:g + 16]) for g in range(0, len(outer), 16))
    flops = passes * 4.0 * w.n * w.d * 16 + 2.0 * w.n * w.d * w.nrhs
    tf = flops / (float(np.mean(times)) * 1e-3) / 1e12
    return {
        "metric": "forward + backward time of a 64-RHS ridge layer (M-IHS + adjoint M-IHS)",
        "value": round(float(np.mean(times)), 3), "unit": "ms", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(float(np.mean(times)), 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic", "config": {"workload": w.name, "n": w.n, "d": w.d, "a_dtype": w.a_dtype,
                                        "nrhs": w.nrhs, "sketch": "srht", "m": w.m, "lambda": lam},
        "rel_err_X": ex, "rel_err_dB": eb, "rel_err_dloglam": el,
        "a_passes": passes,
        "roofline": {"bound": "mfma", "kernel": "batched_kernel (forward + adjoint, whole step)",
                     "achieved": round(tf, 2), "peak": 78.6, "unit": "TFLOP/s",
                     "frac": round(tf / 78.6, 4), "traffic": None},
    }


def run_dual(args):
    """Dual M-IHS (Algorithm 2) on the under-determined workload: A is 4096 x 2^16
    (A^T stored, FP64), SRHT m = 4096 on A^T; one step = sketch + dual solve +
    x = A^T nu, mixed and plain; error against the closed form
    nu* = (A A^T + lambda I)^{-1} b, x* = A^T nu*."""
    import numpy as np
    import torch
    import paper_1912_03514_amd as mihs
    import workloads as W
    dev = torch.device("cuda", 0)
    w = W.workload("dual_4096x2p16")
    At, b, lam = W.make_dual_problem_torch(w.n, w.d, w.sigma, w.sd_target, w.data_seed, dev,
                                           w.a_dtype)
    log("closed form on the host")
    Ath = At.cpu().numpy()
    nu_s = np.linalg.solve(Ath.T @ Ath + lam * np.eye(w.n), b.cpu().numpy())
    xs = Ath @ nu_s
    alpha, beta = mihs.momentum(w.sd_target, w.m_out)
    stream = torch.cuda.current_stream(dev)
    out = {}
    for prec in ("mixed", "plain"):
        def step():
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record(stream)
            SAt = mihs.mihs_sketch(At, w.sketch, w.m, w.sketch_seed, precision=prec)
            e1.record(stream)
            x, nu, info = mihs.mihs_solve_dual(At, b, lam, SAt, alpha, beta, eps_sub=w.eps_sub,
                                               tol=args.tol, max_outer=300, max_inner=2000,
                                               precision=prec, sync=False)
            e2.record(stream)
            torch.cuda.synchronize()
            return x, mihs.info_to_dict(info[0])[0], e0.elapsed_time(e1), e1.elapsed_time(e2)
        times, outs = timed(step, args.steps, args.warmup, None)
        x, info, sk, sv = outs[-1]
        err = float(np.linalg.norm(x.cpu().numpy() - xs) / np.linalg.norm(xs))
        out[prec] = dict(ms=float(np.mean(times)), sketch_ms=sk, solve_ms=sv, info=info, err=err)
        log(f"  {prec}: {out[prec]['ms']:.2f} ms (sketch {sk:.2f}, solve {sv:.2f}); outer "
            f"{info['outer_iters']}, inner {info['inner_iters_total']}; err {err:.2e}")
    mx = out["mixed"]
    pass_bytes = w.d * w.n * 8
    cg_bytes = w.n * w.n * 4
    algo = mx["info"]["outer_iters"] * pass_bytes + mx["info"]["inner_iters_total"] * cg_bytes
    achieved = algo / (mx["solve_ms"] * 1e-3) / 1e9
    return {
        "metric": "time-to-1e-10 rel.err per under-determined ridge solve (Dual M-IHS, mixed; "
                  "SRHT sketch + solve)",
        "value": round(mx["ms"], 3), "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(mx["ms"], 3), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64 outer / f32 inner",
        "data": "synthetic", "config": {"workload": w.name, "n": w.n, "d": w.d, "m": w.m,
                                        "sd": w.sd_target, "lambda": lam, "tol": args.tol},
        "plain_fp64_ms": round(out["plain"]["ms"], 3),
        "mixed": {k: (round(v, 3) if isinstance(v, float) and k != "err" else v)
                  for k, v in mx.items()},
        "plain": {k: (round(v, 3) if isinstance(v, float) and k != "err" else v)
                  for k, v in out["plain"].items()},
        "roofline": {"bound": "hbm", "kernel": "solve_kernel on A^T (mixed)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
        "accuracy_ok": mx["err"] <= 1e-10 and out["plain"]["err"] <= 1e-10,
    }


def run_pd(args):
    """Primal-Dual M-IHS (Algorithm 4) on the square-like workload: A 16384 x 4096
    (FP64), SRHT m1 = 2048 of A, SRHT m2 = 2048 of Q = (SA)^T, M = 25 dual steps
    with AAb_Solver (eps_sub = 0.1) per outer step; one step = both sketches +
    the solve; error against the closed form."""
    import numpy as np
    import torch
    import paper_1912_03514_amd as mihs
    import workloads as W
    dev = torch.device("cuda", 0)
    w = W.workload("pd_16384x4096")
    A, b, _x0, _ = W.make_problem_torch(w.n, w.d, w.sigma, w.sd_target, w.data_seed, dev,
                                        w.a_dtype)
    lam = w.lam
    log("closed-form reference")
    xs = ref_ridge_device(A, b, lam)
    a1, b1 = mihs.momentum(w.sd_target, w.m)
    a2, b2 = mihs.momentum(w.sd_target, w.m2)
    M = 25
    stream = torch.cuda.current_stream(dev)
    out = {}
    for prec, inner in (("plain", "aab"), ("mixed", "aab"), ("plain", "cg")):
        def step():
            e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
            e0.record(stream)
            Q, WQ = mihs.mihs_sketch_two_stage(A, w.sketch, w.m, w.sketch_seed, w.sketch,
                                               w.m2, w.sketch_seed + 1, precision=prec)
            e1.record(stream)
            x, info = mihs.mihs_solve_pd(A, b, lam, Q, WQ, a1, b1, a2, b2, M=M,
                                         eps_sub=w.eps_sub, tol=args.tol, max_outer=60,
                                         precision=prec, sync=False, inner=inner)
            e2.record(stream)
            torch.cuda.synchronize()
            return x, mihs.info_to_dict(info[0])[0], e0.elapsed_time(e1), e1.elapsed_time(e2)
        times, outs = timed(step, args.steps, args.warmup, None)
        x, info, sk, sv = outs[-1]
        err = float(np.linalg.norm(x.cpu().numpy() - xs) / np.linalg.norm(xs))
        key = prec if inner == "aab" else f"{prec}_cg"
        out[key] = dict(ms=float(np.mean(times)), sketch_ms=sk, solve_ms=sv, info=info, err=err)
        log(f"  {key}: {out[key]['ms']:.2f} ms (sketches {sk:.2f}, solve {sv:.2f}); outer "
            f"{info['outer_iters']}, {inner} steps {info['inner_iters_total']}; err {err:.2e}")
    pl = out["plain"]
    outer = pl["info"]["outer_iters"]
    # per outer step: A and b once; per dual step: Q (d x m1) once; per AAb step: WQ once
    # (M v and M^T y come from the same pass over its rows)
    algo = (outer * (w.n * w.d * 8 + w.n * 8) + outer * M * (w.d * w.m * 8)
            + pl["info"]["inner_iters_total"] * (w.m2 * w.m * 8))
    achieved = algo / (pl["solve_ms"] * 1e-3) / 1e9
    rnd = lambda dct: {k: (round(v, 3) if isinstance(v, float) and k != "err" else v)
                       for k, v in dct.items()}
    return {
        "metric": "time-to-1e-10 rel.err per square-like ridge solve (Primal-Dual M-IHS, "
                  "FP64; two-stage SRHT + solve)",
        "value": round(pl["ms"], 3), "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(pl["ms"], 3), "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "n": w.n, "d": w.d, "m1": w.m, "m2": w.m2, "M": M,
                   "sd": w.sd_target, "lambda": lam, "tol": args.tol, "inner": "aab"},
        "plain": rnd(pl), "mixed": rnd(out["mixed"]), "plain_cg_inner": rnd(out["plain_cg"]),
        "roofline": {"bound": "hbm", "kernel": "Primal-Dual solve (all kernels, plain)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "algorithmic_bytes_per_launch": algo},
        "accuracy_ok": all(o["err"] <= 1e-10 for o in out.values()),
    }


def run_small(args):
    import numpy as np
    import torch
    import paper_1912_03514_amd as mihs
    import workloads as W
    dev = torch.device("cuda", 0)
    w = W.workload("small_gauss")
    P = w.draw()
    A, b = torch.from_numpy(P.A).to(dev), torch.from_numpy(P.b).to(dev)
    alpha, beta = mihs.momentum(w.sd_target, w.m_out)
    ws = mihs.SolveWorkspace(w.n, w.d, w.m, "plain", dev)

    def step():
        SA = mihs.mihs_sketch(A, "gaussian", w.m, w.sketch_seed)
        return mihs.mihs_solve(A, b, P.lam, SA, alpha, beta, eps_sub=w.eps_sub, tol=args.tol,
                               max_outer=200, max_inner=2000, workspace=ws)

    times, outs = timed(step, args.steps, args.warmup, None)
    x, info = outs[-1]
    xs = ref_ridge(P.A, P.b, P.lam)
    err = float(np.linalg.norm(x.cpu().numpy() - xs) / np.linalg.norm(xs))
    return {
        "metric": "time-to-1e-10 rel.err per ridge solve (M-IHS, plain FP64; Gaussian sketch + solve)",
        "value": round(float(np.mean(times)), 3), "unit": "ms", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(float(np.mean(times)), 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic", "config": {"workload": w.name, "n": w.n, "d": w.d, "m": w.m},
        "outer_iters": info["outer_iters"], "inner_iters": info["inner_iters_total"],
        "rel_err": err, "roofline": None,
    }


def copy_calibration():
    """A plain copy of known size: 1 GiB read + 1 GiB written per call."""
    import torch
    n = 1 << 27  # doubles
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "calls": 3}))


def run_ridge(args, wname, steps, warmup, full=True):
    """One ridge workload: the sketch + solve step of the mixed and the plain
    FP64 path, timed over `steps` steps after `warmup`, each result checked
    against the closed form after timing; with `full`, also the sd estimate
    (Algorithm 5), the AAb_Solver inner solver and the oracle's CPU baseline."""
    import numpy as np
    import torch

    import paper_1912_03514_amd as mihs
    import workloads as W

    dev = torch.device("cuda", 0)
    w = W.workload(wname)
    lam = w.lam
    alpha, beta = mihs.momentum(w.sd_target, w.m_out)

    log(f"drawing {w.name}: n={w.n} d={w.d} ({w.a_dtype}) on the GPU")
    A, b, _x0, _ = W.make_problem_torch(w.n, w.d, w.sigma, w.sd_target, w.data_seed, dev,
                                        w.a_dtype)
    torch.cuda.synchronize()

    # closed-form reference (torch FP64 Gram + Cholesky; refined in extended
    # precision when the problem is too ill-conditioned for FP64 normal equations)
    log("closed-form reference")
    t0 = time.perf_counter()
    x_ref = ref_ridge_device(A, b, lam, refine=2 if w.a_dtype == "f32" and w.d >= 4096 else 0)
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

    def solve_overhead_ms(precision):
        """Time of mihs_solve with zero outer iterations (Gram matrix, barrier
        reset, a kernel that returns at once): subtracted from the solve time to
        get the persistent kernel's own duration."""
        ws = mihs.SolveWorkspace(w.n, w.d, w.m, precision, dev)
        SA = mihs.mihs_sketch(A, w.sketch, w.m, w.sketch_seed, precision=precision, m2=w.m2)
        ts = []
        for _ in range(4):
            e0, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
            torch.cuda.synchronize()
            e0.record(stream)
            mihs.mihs_solve(A, b, lam, SA, alpha, beta, eps_sub=w.eps_sub, tol=args.tol,
                            max_outer=0, max_inner=2000, precision=precision, workspace=ws,
                            sync=False)
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.mean(ts[1:]))

    out = {}
    for precision in ("mixed", "plain"):
        log(f"{w.name} {precision}: warmup {warmup}")
        run(precision, warmup, False)
        log(f"{w.name} {precision}: timing {steps} steps")
        torch.cuda.synchronize()
        times, sk, sv, infos, xs = run(precision, steps, True)
        errs = [float(np.linalg.norm(x.cpu().numpy() - x_ref) / np.linalg.norm(x_ref)) for x in xs]
        out[precision] = dict(ms=float(np.mean(times)), sketch_ms=float(np.mean(sk)),
                              solve_ms=float(np.mean(sv)), infos=infos, errs=errs,
                              overhead_ms=solve_overhead_ms(precision))
        log(f"  {precision}: {np.mean(times):.2f} ms/solve (sketch {np.mean(sk):.2f}, solve "
            f"{np.mean(sv):.2f}); outer {infos[-1]['outer_iters']}, inner "
            f"{infos[-1]['inner_iters_total']}; max err {max(errs):.2e}")

    def sd_estimate(precision, T=2, eps_tr=0.5, reps=5):
        """Algorithm 5 on this workload's sketch (the paper's T = 2, eps_tr = 0.5):
        the estimate, its inner CG steps and its time next to one outer iteration."""
        SA = mihs.mihs_sketch(A, w.sketch, w.m, w.sketch_seed, precision=precision, m2=w.m2)
        ts = []
        for _ in range(reps):
            e0, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
            torch.cuda.synchronize()
            e0.record(stream)
            est, infos = mihs.mihs_estimate_sd(SA, lam, T=T, seed=17, eps_tr=eps_tr)
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return {"estimate": round(est, 2), "T": T, "eps_tr": eps_tr,
                "inner_iters": [i["inner_iters_total"] for i in infos],
                "ms": round(float(np.mean(ts[1:])), 3)}

    sd_est = {}
    if full:
        log("statistical dimension estimate (Algorithm 5)")
        sd_est = {p: sd_estimate(p) for p in ("mixed", "plain")}
        log(f"  {sd_est}")

    def aab_solve(precision, reps=3):
        """The same solve with AAb_Solver (Algorithm 6) as the inner solver (it
        streams SA on every step; no Gram matrix)."""
        SA = mihs.mihs_sketch(A, w.sketch, w.m, w.sketch_seed, precision=precision, m2=w.m2)
        ws = mihs.SolveWorkspace(w.n, w.d, w.m, precision, dev)
        ts, info, x = [], None, None
        for _ in range(reps):
            e0, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(2))
            torch.cuda.synchronize()
            e0.record(stream)
            x, info = mihs.mihs_solve(A, b, lam, SA, alpha, beta, eps_sub=w.eps_sub, tol=args.tol,
                                      max_outer=300, max_inner=2000, precision=precision,
                                      workspace=ws, sync=False, inner="aab")
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        inf = mihs.info_to_dict(info)[0]
        err = float(np.linalg.norm(x.cpu().numpy() - x_ref) / np.linalg.norm(x_ref))
        return {"solve_ms": round(float(np.mean(ts[1:])), 3), "outer_iters": inf["outer_iters"],
                "inner_iters": inf["inner_iters_total"], "rel_err": err}

    aab = {}
    if full:
        log("AAb_Solver as the inner solver (Algorithm 6)")
        aab = {p: aab_solve(p) for p in ("mixed", "plain")}
        log(f"  {aab}")

    mx, pl = out["mixed"], out["plain"]
    info = mx["infos"][-1]
    s_a = 8 if w.a_dtype == "f64" else 4
    apass_bytes = w.n * w.d * s_a + w.n * 8
    # one CG step streams the operator once: the Gram matrix (d x d) when the
    # sketch has at least d rows, else SA; FP32 in the mixed path
    cg_bytes = min(w.m_out, w.d) * w.d * 4
    outer = info["outer_iters"]
    inner = info["inner_iters_total"]
    solve_bytes = outer * apass_bytes + inner * cg_bytes
    kernel_ms = mx["solve_ms"] - mx["overhead_ms"]
    achieved = solve_bytes / (kernel_ms * 1e-3) / 1e9
    traffic = MEASURED_TRAFFIC.get((w.name, "mixed"))
    result = {
        "metric": f"time-to-1e-10 rel.err per ridge solve (M-IHS, mixed precision; {w.sketch} sketch + solve)",
        "value": round(mx["ms"], 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
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
        "aab_inner": aab,
        "sd_estimate": {"sd_true": w.sd_target, "m": w.m_out,
                        "mixed_solve_ms_per_outer_iter": round(mx["solve_ms"] / max(1, outer), 3),
                        **{p: v for p, v in sd_est.items()}},
        "roofline": {"bound": "hbm", "kernel": "solve_kernel (mixed)",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": solve_bytes,
                     "kernel_ms": round(kernel_ms, 3),
                     "launch_overhead_ms": round(mx["overhead_ms"], 3)},
        "row_weights": list(mihs.row_weights()),
        "accuracy_ok": max(mx["errs"]) <= 1e-10 and max(pl["errs"]) <= 1e-10,
    }
    if full and not args.no_cpu_baseline:
        log("cpu baseline (the oracle on the host cores)")
        rows = args.cpu_sample_rows if args.cpu_sample_rows > 0 else w.n
        result["cpu_baseline"] = cpu_baseline(w, lam, A, b, rows)
    del A, b
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return result




def ridge_summary(r):
    """The keys of a ridge result that another workload's line carries."""
    keep = ("value", "unit", "ms_per_step", "steps", "warmup", "config", "plain_fp64_ms",
            "mixed_speedup_vs_plain", "mixed", "plain", "roofline", "row_weights",
            "accuracy_ok")
    return {k: r[k] for k in keep if k in r}


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.tol is None:
        args.tol = DEFAULT_TOL.get(args.workload, 5e-11)
    if args.workload in ("batched_lambda_path", "diff_2p18x1024", "small_gauss",
                         "dual_4096x2p16", "pd_16384x4096"):
        if args.gpus != 1:
            print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1"}))
            sys.exit(2)
        import paper_1912_03514_amd as mihs
        mihs.load_library()
        fn = {"batched_lambda_path": run_batched, "diff_2p18x1024": run_diff,
              "small_gauss": run_small, "dual_4096x2p16": run_dual,
              "pd_16384x4096": run_pd}[args.workload]
        out = fn(args)
        mihs.release_all()
        print(json.dumps(out), flush=True)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1912_03514_amd as mihs
    import workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    mihs.load_library()
    dev = torch.device("cuda", 0)
    # the sd estimate, the AAb_Solver solve and the oracle's CPU timing are
    # reported for the headline workload only (on the ill-conditioned one they
    # would take minutes)
    result = run_ridge(args, args.workload, args.steps, args.warmup,
                       full=args.workload == "srht_2p18x2048")
    if args.workload == "srht_2p18x2048" and not args.no_large:
        # the largest single-GPU ridge configuration, a few steps (each takes
        # seconds), reported beside the headline
        if args.tol_large is not None:
            args.tol = args.tol_large
        else:
            args.tol = DEFAULT_TOL["count_2p20x4096"]
        result["count_2p20x4096"] = ridge_summary(
            run_ridge(args, "count_2p20x4096", args.large_steps, 1, full=False))
    mihs.release_all()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
