"""GPU parity: the persistent M-IHS solve against the oracle (sketch taken from
the oracle so that only the solve is under test)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import sketches, solver as O
from gpu_common import announce, dev, rel, requires_gpu, to_dev, torch

pytestmark = [pytest.mark.gpu, requires_gpu]


def _mihs():
    import paper_1912_03514_amd as mihs
    return mihs


def _problem(n, d, sd, seed, rate=6.0, a_dtype=np.float64):
    sig = W.sigma_profile("exp", d, rate)
    return W.make_problem(n, d, sig, sd, seed, a_dtype)


def test_small_workload_plain_reaches_1e_10():
    """The small Gaussian workload (4096 x 256, m = 256, eps_sub = 1e-8)."""
    mihs = _mihs()
    w = W.workload("small_gauss")
    P = w.draw()
    SA = sketches.gaussian_sketch(P.A, w.m, w.sketch_seed)
    a, b = O.momentum_cor4(w.sd_target, w.m_out)
    xs = O.ridge_lstsq(P.A, P.b, P.lam)
    ref = O.mihs(P.A, P.b, P.lam, SA, a, b, inner="cg", eps_sub=w.eps_sub, tol=1e-10)
    announce("small_gauss plain solve, oracle SA")
    x, info = mihs.mihs_solve(to_dev(P.A), to_dev(P.b), P.lam, to_dev(SA), a, b,
                              eps_sub=w.eps_sub, tol=1e-10, max_outer=200, max_inner=2000)
    x = x.cpu().numpy()
    assert info["status"] == 0, info
    assert rel(x, xs) <= 1e-10
    assert abs(info["outer_iters"] - ref.outer) <= 2
    assert abs(info["inner_iters_total"] - sum(ref.inner)) <= max(4, 0.05 * sum(ref.inner))


def test_fixed_iterations_follow_oracle_trajectory():
    """N outer steps with a tight inner tolerance: the GPU iterate equals the
    oracle's iterate up to rounding (several row tiles and a ragged last tile)."""
    mihs = _mihs()
    P = _problem(3001, 130, 30.0, seed=21)
    SA = sketches.gaussian_sketch(P.A, 160, 4)
    a, b = O.momentum_cor4(30.0, 160)
    for N in (1, 2, 7):
        ref = O.mihs(P.A, P.b, P.lam, SA, a, b, inner="cg", eps_sub=1e-13, n_iter=N,
                     max_inner=5000)
        announce(f"trajectory n=3001 d=130 N={N}")
        x, info = mihs.mihs_solve(to_dev(P.A), to_dev(P.b), P.lam, to_dev(SA), a, b,
                                  eps_sub=1e-13, tol=0.0, max_outer=N, max_inner=5000)
        assert info["outer_iters"] == N
        assert rel(x.cpu().numpy(), ref.x) <= 1e-11, N


@pytest.mark.parametrize("n,d", [(700, 1), (900, 63), (1000, 64), (1500, 65), (2500, 257),
                                 (5000, 1000), (6000, 2048), (5200, 3001)])
def test_shapes_plain(n, d):
    """Ragged d over every register layout (d up to 64 * 64)."""
    mihs = _mihs()
    sd = max(0.5, d / 5)
    P = _problem(n, d, sd, seed=n + d)
    m = min(n, max(4 * int(math.ceil(sd)), d // 2 + 1))
    SA = sketches.countsketch(P.A, m, 3)
    a, b = O.momentum_cor4(sd, m)
    xs = O.ridge_lstsq(P.A, P.b, P.lam)
    announce(f"shape plain n={n} d={d} m={m}")
    x, info = mihs.mihs_solve(to_dev(P.A), to_dev(P.b), P.lam, to_dev(SA), a, b, eps_sub=1e-3,
                              tol=1e-11, max_outer=400, max_inner=4000)
    assert info["status"] == 0, info
    assert rel(x.cpu().numpy(), xs) <= 1e-10


def test_operator_paths_with_rows_wider_than_2048():
    """d in (2048, 4096]: the gradient pass splits rows into quarters and the inner
    CG works on 64 entries of a row per lane, through the Gram matrix (m >= d:
    FP64 H, or FP32 H in mixed precision; 12 rows of H per CG workgroup) or by
    streaming SA (m < d, FP64 or FP32 rows, and AAb_Solver); ragged d.  Every
    form reaches the closed form to 1e-10."""
    mihs = _mihs()
    n, d = 8000, 3001
    sd = d / 5
    P = _problem(n, d, sd, seed=77)
    xs = O.ridge_lstsq(P.A, P.b, P.lam)
    for m in (3200, 2400):
        SA = sketches.countsketch(P.A, m, 5)
        a, b = O.momentum_cor4(sd, m)
        for prec, sa, eps in (("plain", SA, 1e-3), ("mixed", SA.astype(np.float32), 1e-2)):
            announce(f"wide rows n={n} d={d} m={m} {prec}")
            x, info = mihs.mihs_solve(to_dev(P.A), to_dev(P.b), P.lam, to_dev(sa), a, b,
                                      eps_sub=eps, tol=1e-11, max_outer=400, max_inner=4000,
                                      precision=prec)
            assert info["status"] == 0, (m, prec, info)
            assert rel(x.cpu().numpy(), xs) <= 1e-10, (m, prec)
    # AAb_Solver as the inner solver on the same rows (the paper's eps_sub = 0.1)
    announce(f"wide rows n={n} d={d} m=2400 aab")
    x, info = mihs.mihs_solve(to_dev(P.A), to_dev(P.b), P.lam, to_dev(SA), a, b, eps_sub=0.1,
                              tol=1e-11, max_outer=400, max_inner=4000, inner="aab")
    assert info["status"] == 0, info
    assert rel(x.cpu().numpy(), xs) <= 1e-10


def test_fp32_matrix_and_mixed_inner():
    """FP32 A (upcast exactly) with an FP32 sketch and FP32 inner CG: the FP64
    outer gradient still drives the error to 1e-10."""
    mihs = _mihs()
    P = _problem(8192, 300, 60.0, seed=5, a_dtype=np.float32)
    SA = sketches.gaussian_sketch(P.A, 256, 9)
    a, b = O.momentum_cor4(60.0, 256)
    xs = O.ridge_lstsq(P.A.astype(np.float64), P.b, P.lam)
    for prec, sa in (("plain", SA), ("mixed", SA.astype(np.float32))):
        announce(f"fp32 A, {prec}")
        x, info = mihs.mihs_solve(to_dev(P.A), to_dev(P.b), P.lam, to_dev(sa), a, b,
                                  eps_sub=1e-2, tol=1e-11, max_outer=300, max_inner=2000,
                                  precision=prec)
        assert info["status"] == 0, (prec, info)
        assert rel(x.cpu().numpy(), xs) <= 1e-10, prec


@pytest.mark.parametrize("m", [120, 128, 200])
@pytest.mark.parametrize("prec", ["plain", "mixed"])
def test_cg_operator_paths(m, prec):
    """The inner CG applies (SA)^T SA by streaming SA (m < d) or through the Gram
    matrix (m >= d): both follow the oracle's trajectory for N fixed steps."""
    mihs = _mihs()
    d = 128
    P = _problem(2600, d, 25.0, seed=33)
    SA = sketches.gaussian_sketch(P.A, m, 6)
    a, b = O.momentum_cor4(25.0, m)
    N = 5
    ref = O.mihs(P.A, P.b, P.lam, SA, a, b, inner="cg", eps_sub=1e-12 if prec == "plain" else 1e-4,
                 n_iter=N, max_inner=5000)
    sa = SA if prec == "plain" else SA.astype(np.float32)
    announce(f"cg operator path m={m} d={d} {prec}")
    x, info = mihs.mihs_solve(to_dev(P.A), to_dev(P.b), P.lam, to_dev(sa), a, b,
                              eps_sub=1e-12 if prec == "plain" else 1e-4, tol=0.0, max_outer=N,
                              max_inner=5000, precision=prec)
    assert info["outer_iters"] == N
    # FP32 CG: each inner solve is accurate to about its tolerance, not to rounding
    assert rel(x.cpu().numpy(), ref.x) <= (1e-11 if prec == "plain" else 1e-4)


@pytest.mark.parametrize("m", [120, 200])
def test_aab_inner_follows_oracle_trajectory(m):
    """AAb_Solver (Algorithm 6) as the inner solver: N fixed outer steps follow
    the oracle's AAb trajectory (step counts and iterates), m below and above d."""
    mihs = _mihs()
    d = 128
    P = _problem(2600, d, 25.0, seed=34)
    SA = sketches.gaussian_sketch(P.A, m, 7)
    a, b = O.momentum_cor4(25.0, m)
    N = 5
    for eps in (0.1, 1e-12):
        ref = O.mihs(P.A, P.b, P.lam, SA, a, b, inner="aab", eps_sub=eps, n_iter=N,
                     max_inner=5000)
        announce(f"aab inner m={m} d={d} eps={eps}")
        x, info = mihs.mihs_solve(to_dev(P.A), to_dev(P.b), P.lam, to_dev(SA), a, b,
                                  eps_sub=eps, tol=0.0, max_outer=N, max_inner=5000, inner="aab")
        assert info["outer_iters"] == N
        # at eps = 1e-12 the residual estimate ends within rounding of the
        # threshold, so a solve may take one step more or less (a change of
        # about eps in the step)
        slack = 0 if eps >= 1e-6 else N
        assert abs(info["inner_iters_total"] - sum(ref.inner)) <= slack, (info, ref.inner)
        assert rel(x.cpu().numpy(), ref.x) <= 1e-11, eps


@pytest.mark.parametrize("prec", ["plain", "mixed"])
def test_aab_inner_reaches_1e_10(prec):
    """The small workload's shape with AAb_Solver at the paper's forcing term 0.1:
    the FP64 outer loop drives the error to 1e-10 (FP32 AAb in the mixed path)."""
    mihs = _mihs()
    P = _problem(4096, 256, 64.0, seed=12)
    SA = sketches.gaussian_sketch(P.A, 256, 7)
    a, b = O.momentum_cor4(64.0, 256)
    xs = O.ridge_lstsq(P.A, P.b, P.lam)
    sa = SA if prec == "plain" else SA.astype(np.float32)
    announce(f"aab inner to 1e-10, {prec}")
    x, info = mihs.mihs_solve(to_dev(P.A), to_dev(P.b), P.lam, to_dev(sa), a, b, eps_sub=0.1,
                              tol=1e-11, max_outer=300, max_inner=2000, precision=prec,
                              inner="aab")
    assert info["status"] == 0, info
    assert rel(x.cpu().numpy(), xs) <= 1e-10


def test_warm_start_and_momentum_state():
    """Two half-length solves chained through X and X_prev equal one long solve."""
    mihs = _mihs()
    P = _problem(4000, 96, 20.0, seed=8)
    SA = sketches.gaussian_sketch(P.A, 96, 2)
    a, b = O.momentum_cor4(20.0, 96)
    announce("warm start chain")
    full, _ = mihs.mihs_solve(to_dev(P.A), to_dev(P.b), P.lam, to_dev(SA), a, b, eps_sub=1e-12,
                              tol=0.0, max_outer=12, max_inner=3000)
    xprev = torch.zeros(96, dtype=torch.float64, device=dev())
    x1, _ = mihs.mihs_solve(to_dev(P.A), to_dev(P.b), P.lam, to_dev(SA), a, b, eps_sub=1e-12,
                            tol=0.0, max_outer=6, max_inner=3000, x_prev=xprev)
    x2, _ = mihs.mihs_solve(to_dev(P.A), to_dev(P.b), P.lam, to_dev(SA), a, b, eps_sub=1e-12,
                            tol=0.0, max_outer=6, max_inner=3000, x0=x1, x_prev=xprev)
    assert rel(x2.cpu().numpy(), full.cpu().numpy()) <= 1e-12


def test_zero_rhs_and_zero_iterations():
    mihs = _mihs()
    P = _problem(1024, 32, 8.0, seed=1)
    SA = sketches.gaussian_sketch(P.A, 64, 2)
    a, b = O.momentum_cor4(8.0, 64)
    announce("degenerate: b = 0 and max_outer = 0")
    x, info = mihs.mihs_solve(to_dev(P.A), to_dev(np.zeros(1024)), P.lam, to_dev(SA), a, b,
                              tol=1e-10, max_outer=50)
    assert info["status"] == 0 and info["outer_iters"] == 0
    assert np.all(x.cpu().numpy() == 0)
    x, info = mihs.mihs_solve(to_dev(P.A), to_dev(P.b), P.lam, to_dev(SA), a, b, tol=1e-10,
                              max_outer=0)
    assert info["outer_iters"] == 0 and np.all(x.cpu().numpy() == 0)


def test_invalid_arguments_are_rejected():
    mihs = _mihs()
    P = _problem(256, 16, 4.0, seed=2)
    SA = sketches.gaussian_sketch(P.A, 32, 2)
    A, b, S = to_dev(P.A), to_dev(P.b), to_dev(SA)
    with pytest.raises(mihs.MihsError):
        mihs.mihs_solve(A, b, -1.0, S, 0.5, 0.2)          # lambda <= 0
    with pytest.raises(mihs.MihsError):
        mihs.mihs_solve(A, b, P.lam, S, 0.5, 1.5)          # beta >= 1
    with pytest.raises(mihs.MihsError):
        mihs.mihs_solve(A[:8], b[:8], P.lam, S, 0.5, 0.2)  # n < d (b length checked first)
