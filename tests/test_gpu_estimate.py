"""GPU parity: the inexact Hutchinson estimate of the statistical dimension
(Algorithm 5) against the oracle, probe by probe."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import sketches, solver as O
from gpu_common import announce, rel, requires_gpu, to_dev, torch

pytestmark = [pytest.mark.gpu, requires_gpu]


def _mihs():
    import paper_1912_03514_amd as mihs
    return mihs


def _sketch(m, d, sd, seed, rate=6.0):
    """A sketch-shaped input: Gaussian sketch of a problem with an exponential
    spectrum (the estimator only sees SA)."""
    sig = W.sigma_profile("exp", d, rate)
    P = W.make_problem(max(4 * d, 1024), d, sig, sd, seed)
    return sketches.gaussian_sketch(P.A, m, seed + 1), P.lam


def _inner_ref(inner):
    return O.aab_solver if inner == "aab" else O.inner_cg


@pytest.mark.parametrize("inner", ["aab", "cg"])
@pytest.mark.parametrize("m,d", [(96, 1), (160, 63), (200, 130), (120, 128), (700, 1000),
                                 (1500, 2048), (2100, 3001)])
def test_probes_follow_oracle(m, d, inner):
    """eps_tr = 0.5, T = 3: every probe's inner solve (AAb_Solver or CG) takes
    the oracle's number of steps and its z matches the oracle's to rounding; so
    does the estimate (ragged d, m below and above d)."""
    mihs = _mihs()
    sd = max(0.5, d / 4)
    SA, lam = _sketch(m, d, sd, seed=d + m)
    T, seed = 3, 1234 + d
    V = sketches.rademacher_probes(d, T, seed)
    refs = [_inner_ref(inner)(SA, V[:, l], lam, 0.5) for l in range(T)]
    ref_sd = d - lam * sum(float(V[:, l] @ refs[l][0]) for l in range(T)) / T
    assert abs(ref_sd - O.hutchinson_sd(SA, lam, V, inner=inner, eps_tr=0.5)) <= 1e-12 * d
    announce(f"estimate_sd m={m} d={d} T={T} eps_tr=0.5 {inner}")
    est, Z, infos = mihs.mihs_estimate_sd(to_dev(SA), lam, T=T, seed=seed, eps_tr=0.5,
                                          want_z=True, inner=inner)
    Z = Z.cpu().numpy()
    if inner == "aab" and d == 1:
        # one column: the Krylov space ends after the first step, and the next
        # bidiagonalisation vector is rounding noise on either side, so compare
        # with the exact solve instead of step by step
        M = SA.T @ SA + lam
        for l in range(T):
            assert infos[l]["status"] == 0, infos[l]
            assert rel(Z[l], V[:, l] / M[0, 0]) <= 1e-12, l
        return
    for l in range(T):
        assert infos[l]["status"] == 0, infos[l]
        assert infos[l]["inner_iters_total"] == refs[l][1], (l, infos[l], refs[l][1])
        assert rel(Z[l], refs[l][0]) <= 1e-12, l
    assert abs(est - ref_sd) <= 1e-12 * max(1.0, abs(ref_sd))


@pytest.mark.parametrize("inner", ["aab", "cg"])
def test_tight_inner_tolerance_gives_exact_probe_trace(inner):
    """eps_tr = 1e-13: the estimate equals d - lambda/T sum v^T M^{-1} v with M
    factored exactly (oracle Cholesky)."""
    mihs = _mihs()
    m, d = 400, 256
    SA, lam = _sketch(m, d, 40.0, seed=3)
    T, seed = 8, 77
    V = sketches.rademacher_probes(d, T, seed)
    ref = O.hutchinson_sd(SA, lam, V, inner="exact")
    announce(f"estimate_sd tight inner tolerance {inner}")
    est, infos = mihs.mihs_estimate_sd(to_dev(SA), lam, T=T, seed=seed, eps_tr=1e-13,
                                       max_inner=5000, inner=inner)
    assert all(i["status"] == 0 for i in infos)
    assert abs(est - ref) <= 1e-10 * ref


def test_mixed_precision_sketch():
    """FP32 SA with the inner solve in FP32: each z is accurate to about the
    inner tolerance, so the estimate agrees with the FP64 probe trace of the
    same (upcast) SA."""
    mihs = _mihs()
    m, d = 600, 300
    SA, lam = _sketch(m, d, 60.0, seed=9)
    SA32 = SA.astype(np.float32)
    T, seed = 4, 5
    V = sketches.rademacher_probes(d, T, seed)
    ref = O.hutchinson_sd(SA32.astype(np.float64), lam, V, inner="exact")
    for inner in ("aab", "cg"):
        announce(f"estimate_sd mixed {inner}")
        est, infos = mihs.mihs_estimate_sd(to_dev(SA32), lam, T=T, seed=seed, eps_tr=1e-5,
                                           max_inner=5000, inner=inner)
        assert all(i["status"] == 0 for i in infos)
        assert abs(est - ref) <= 1e-4 * ref, inner


def test_headline_shape_estimate():
    """At the headline solve's sketch shape (m = d = 2048) with the paper's
    T = 2, eps_tr = 0.5 and AAb_Solver, FP64 and FP32: parity with the oracle's
    probes; the estimate lands within the Hutchinson spread of the sketched sd."""
    mihs = _mihs()
    w = W.workload("srht_2p18x2048")
    d = w.d
    SA, lam = _sketch(w.m, d, w.sd_target, seed=2048, rate=8.0)
    T, seed = 2, 99
    V = sketches.rademacher_probes(d, T, seed)
    refs = [O.aab_solver(SA, V[:, l], lam, 0.5) for l in range(T)]
    ref_sd = d - lam * sum(float(V[:, l] @ refs[l][0]) for l in range(T)) / T
    announce("estimate_sd 2048 x 2048 T=2 plain")
    est, infos = mihs.mihs_estimate_sd(to_dev(SA), lam, T=T, seed=seed, eps_tr=0.5)
    assert [i["inner_iters_total"] for i in infos] == [r[1] for r in refs]
    assert abs(est - ref_sd) <= 1e-12 * ref_sd
    exact = O.sketched_sd_exact(SA, lam)
    # variance of a Rademacher probe's quadratic form <= 2 ||M||_F^2 with M the
    # lambda-weighted inverse, ||M||_F^2 <= d; a relative residual of 0.5
    # adds at most d / 2
    assert abs(est - exact) <= 0.5 * d + 4 * math.sqrt(2 * d / T)
    announce("estimate_sd 2048 x 2048 T=2 mixed")
    est32, infos32 = mihs.mihs_estimate_sd(to_dev(SA.astype(np.float32)), lam, T=T, seed=seed,
                                           eps_tr=0.5)
    assert all(i["status"] == 0 for i in infos32)
    assert abs(est32 - ref_sd) <= 1e-3 * ref_sd


def test_invalid_arguments_are_rejected():
    mihs = _mihs()
    SA, lam = _sketch(64, 16, 4.0, seed=1)
    S = to_dev(SA)
    with pytest.raises(mihs.MihsError):
        mihs.mihs_estimate_sd(S, -1.0)
    with pytest.raises(mihs.MihsError):
        mihs.mihs_estimate_sd(S, lam, T=0)
    with pytest.raises(mihs.MihsError):
        mihs.mihs_estimate_sd(S, lam, eps_tr=-0.5)
    wide = torch.zeros((8, 5000), dtype=torch.float64, device="cuda")
    with pytest.raises(mihs.MihsError):
        mihs.mihs_estimate_sd(wide, lam)
