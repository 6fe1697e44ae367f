"""Pins of the oracle's solver against closed forms, invariants and the paper's
printed numbers."""
import math

import numpy as np
import pytest
import scipy.optimize

import workloads as W
from conftest import read_golden
from oracle import sketches, solver as O


def _small(n=600, d=40, sd=12.0, seed=11, rate=6.0):
    sig = W.sigma_profile("exp", d, rate)
    return W.make_problem(n, d, sig, sd, seed)


def test_closed_forms_agree_with_svd_filter_form():
    P = _small()
    xc = O.ridge_cholesky(P.A, P.b, P.lam)
    xq = O.ridge_lstsq(P.A, P.b, P.lam)
    # Tikhonov filter-factor form of the same solution (proof of Corollary 4)
    U, s, Vt = np.linalg.svd(P.A, full_matrices=False)
    xf = Vt.T @ ((s * s / (s * s + P.lam)) * (U.T @ P.b) / s)
    for x in (xc, xq):
        assert np.linalg.norm(x - xf) <= 1e-12 * np.linalg.norm(xf)
    # optimality: gradient of the ridge objective vanishes
    g = O.gradient(P.A, P.b, P.lam, xf)
    assert np.linalg.norm(g) <= 1e-12 * np.linalg.norm(P.A.T @ P.b)


def test_statistical_dimension_definition():
    P = _small()
    H = P.A.T @ P.A + P.lam * np.eye(P.A.shape[1])
    tr = np.trace(P.A @ np.linalg.solve(H, P.A.T))
    assert abs(O.statistical_dimension(P.A, P.lam) - tr) < 1e-9


def test_one_step_with_identity_sketch():
    """S = I (m = n), exact inner solve, alpha = 1, beta = 0: the first M-IHS
    step is a Newton step on a quadratic and lands on x*."""
    P = _small()
    xs = O.ridge_lstsq(P.A, P.b, P.lam)
    r = O.mihs(P.A, P.b, P.lam, P.A, 1.0, 0.0, inner="exact", n_iter=1)
    assert np.linalg.norm(r.x - xs) <= 1e-12 * np.linalg.norm(xs)


def test_theorem1_momentum_identities():
    for eps in (0.05, 0.3, 0.5, 0.9):
        a, b = O.momentum_thm1(eps)
        assert math.isclose(a, 4 * (1 - eps**2) / (math.sqrt(1 + eps) + math.sqrt(1 - eps)) ** 2,
                            rel_tol=1e-12)
        # sqrt(beta*) minimises over alpha the worse of the two extreme root moduli
        f = lambda al: max(1 - math.sqrt(al) / math.sqrt(1 + eps),
                           math.sqrt(al) / math.sqrt(1 - eps) - 1)
        res = scipy.optimize.minimize_scalar(f, bounds=(1e-6, 4.0), method="bounded",
                                             options={"xatol": 1e-12})
        assert math.isclose(res.fun, math.sqrt(b), rel_tol=1e-6, abs_tol=1e-9)
        assert math.isclose(res.x, a, rel_tol=1e-4)
        # every mu in [1/(1+eps), 1/(1-eps)] is under-damped: root modulus sqrt(beta)
        mus = np.linspace(1 / (1 + eps), 1 / (1 - eps), 7)
        assert O.heavy_ball_rate(mus, a, b) <= math.sqrt(b) * (1 + 1e-6)


def test_cor4_matches_paper_worked_number():
    """Figure 2's caption: kappa(A) (1/sqrt 2)^100 = 9e-8 with sd = 2000, m = 4000."""
    for name, sd, m, N, C, printed in read_golden("paper_worked_numbers.txt"):
        a, b = O.momentum_cor4(float(sd), int(m))
        bound = float(C) * math.sqrt(b) ** int(N)
        assert abs(bound - float(printed)) / float(printed) < 0.02
        assert math.isclose(a, (1 - b) ** 2)


def test_rate_matches_characteristic_polynomial():
    """With an exact inner solve the error contracts at the spectral radius given
    by eq. (characteristic) over the eigenvalues of H_s^{-1} H, close to sqrt(beta)."""
    w = W.workload("small_gauss")
    P = w.draw()
    SA = sketches.gaussian_sketch(P.A, w.m, w.sketch_seed)
    a, b = O.momentum_cor4(w.sd_target, w.m_out)
    xs = O.ridge_lstsq(P.A, P.b, P.lam)
    r = O.mihs(P.A, P.b, P.lam, SA, a, b, inner="exact", n_iter=40, keep_history=True)
    errs = np.array([np.linalg.norm(x - xs) for x in r.history])
    emp = (errs[35] / errs[15]) ** (1 / 20)
    H = P.A.T @ P.A + P.lam * np.eye(P.A.shape[1])
    Hs = SA.T @ SA + P.lam * np.eye(P.A.shape[1])
    mu = np.linalg.eigvals(np.linalg.solve(Hs, H)).real
    pred = O.heavy_ball_rate(mu, a, b)
    assert abs(emp - pred) < 0.03
    assert abs(emp - math.sqrt(b)) < 0.05
    # Corollary 4 iteration bound is not exceeded by much at this size
    assert np.argmax(errs / errs[0] < 1e-10) <= O.iterations_cor4(1e-10, b) + 5


def test_inner_solvers_agree_with_exact():
    P = _small(d=60, sd=20.0)
    SA = sketches.gaussian_sketch(P.A, 120, 3)
    g = O.gradient(P.A, P.b, P.lam, np.zeros(60))
    ex, _ = O.inner_exact_factory(SA, P.lam)(g)
    Hs = SA.T @ SA + P.lam * np.eye(60)
    for fn in (O.inner_cg, O.aab_solver):
        z, k = fn(SA, g, P.lam, 1e-12)
        assert np.linalg.norm(z - ex) <= 1e-9 * np.linalg.norm(ex)
        z, k = fn(SA, g, P.lam, 1e-2)
        assert k > 0
        # relative residual respected (AAb's test lags one iterate, so it is conservative)
        assert np.linalg.norm(Hs @ z - g) <= 1e-2 * np.linalg.norm(g) * 1.0001


def test_aab_residual_identity():
    """Section 3.5: ||(M^T M + lambda I) x^k - b|| = |phi_k thetabar_{k+1}|, so the
    stopping quantity t after a step is the true relative residual of the iterate
    before that step."""
    rng = np.random.default_rng(8)
    M = rng.standard_normal((50, 20))
    bvec = rng.standard_normal(20)
    lam = 0.3
    H = M.T @ M + lam * np.eye(20)
    tr = []
    O.aab_solver(M, bvec, lam, 0.0, max_iter=10, trace=tr)
    for j in range(1, len(tr)):
        xprev = tr[j - 1][0]
        res = np.linalg.norm(H @ xprev - bvec) / np.linalg.norm(bvec)
        assert math.isclose(res, tr[j][1], rel_tol=1e-7)


@pytest.mark.parametrize("inner", ["exact", "cg", "aab"])
def test_mihs_small_workload_reaches_1e_10(inner):
    w = W.workload("small_gauss")
    P = w.draw()
    SA = sketches.gaussian_sketch(P.A, w.m, w.sketch_seed)
    a, b = O.momentum_cor4(w.sd_target, w.m_out)
    xs = O.ridge_lstsq(P.A, P.b, P.lam)
    r = O.mihs(P.A, P.b, P.lam, SA, a, b, inner=inner, eps_sub=w.eps_sub, tol=1e-10)
    assert r.converged
    assert np.linalg.norm(r.x - xs) <= 1e-10 * np.linalg.norm(xs)
    assert r.outer <= O.iterations_cor4(1e-10, b) + 8


def test_sketch_independence():
    """x* does not depend on S: different sketch families reach the same point."""
    P = _small(n=1024, d=48, sd=16.0)
    xs = O.ridge_lstsq(P.A, P.b, P.lam)
    for kind, m in (("gaussian", 96), ("srht", 128), ("countsketch", 256)):
        SA = sketches.sketch(P.A, kind, m, 5)
        a, b = O.momentum_cor4(16.0, m)
        r = O.mihs(P.A, P.b, P.lam, SA, a, b, inner="cg", eps_sub=1e-3, tol=1e-12, max_outer=400)
        assert np.linalg.norm(r.x - xs) <= 1e-11 * np.linalg.norm(xs), kind


def test_adjoint_mode_solves_hessian_system():
    P = _small()
    rng = np.random.default_rng(1)
    gbar = rng.standard_normal(P.A.shape[1])
    SA = sketches.gaussian_sketch(P.A, 80, 2)
    a, b = O.momentum_cor4(12.0, 80)
    r = O.mihs(P.A, gbar, P.lam, SA, a, b, inner="cg", eps_sub=1e-6, tol=1e-12, rhs_mode=True)
    H = P.A.T @ P.A + P.lam * np.eye(P.A.shape[1])
    w = np.linalg.solve(H, gbar)
    assert np.linalg.norm(r.x - w) <= 1e-10 * np.linalg.norm(w)


def test_backward_matches_finite_differences():
    """dL/dB and dL/dlog(lambda) of L = sum_j ||C x*_j - y_j||^2 against central
    differences of dense forward solves (L is quadratic in B, so the B-difference
    is exact up to rounding)."""
    rng = np.random.default_rng(6)
    n, d, k = 200, 12, 3
    A = rng.standard_normal((n, d))
    B = rng.standard_normal((n, k))
    C = rng.standard_normal((5, d))
    Y = rng.standard_normal((5, k))
    loglam = math.log(0.7)

    def loss(Bm, ll):
        X = O.ridge_cholesky(A, Bm, math.exp(ll))
        return float(np.sum((C @ X - Y) ** 2))

    lam = math.exp(loglam)
    X = O.ridge_cholesky(A, B, lam)
    gbar = 2 * C.T @ (C @ X - Y)
    W_, dB, dlam = O.ridge_backward_dense(A, lam, X, gbar)
    h = 1e-6
    for _ in range(3):
        V = rng.standard_normal((n, k))
        fd = (loss(B + h * V, loglam) - loss(B - h * V, loglam)) / (2 * h)
        assert abs(fd - np.sum(dB * V)) <= 1e-6 * max(1.0, abs(fd))
    fd = (loss(B, loglam + h) - loss(B, loglam - h)) / (2 * h)
    assert abs(fd - lam * dlam) <= 1e-6 * max(1.0, abs(fd))


def test_planted_mistakes_are_caught(monkeypatch):
    """A wrong sign in the gradient or a swapped momentum pair must break the
    closed-form pin: shows the pins are not vacuous."""
    P = _small()
    xs = O.ridge_lstsq(P.A, P.b, P.lam)
    SA = sketches.gaussian_sketch(P.A, 80, 2)
    a, b = O.momentum_cor4(12.0, 80)
    good = O.mihs(P.A, P.b, P.lam, SA, a, b, inner="exact", n_iter=60)
    assert np.linalg.norm(good.x - xs) <= 1e-10 * np.linalg.norm(xs)
    orig = O.gradient
    monkeypatch.setattr(O, "gradient", lambda A, bb, lam, x: orig(A, bb, -lam, x))
    bad = O.mihs(P.A, P.b, P.lam, SA, a, b, inner="exact", n_iter=60)
    assert np.linalg.norm(bad.x - xs) > 1e-6 * np.linalg.norm(xs)
    monkeypatch.setattr(O, "gradient", orig)
    bad2 = O.mihs(P.A, P.b, P.lam, SA, b, a, inner="exact", n_iter=60)  # alpha <-> beta
    e2 = np.linalg.norm(bad2.x - xs) / np.linalg.norm(xs)
    assert e2 > 1e-8 or not np.isfinite(e2)


def _wide(n=60, d=400, seed=3):
    """An under-determined instance: A^T drawn by the same recipe as a tall A."""
    sig = W.sigma_profile("exp", n, 6.0)
    P = W.make_problem(d, n, sig, 15.0, seed)   # P.A is d x n (tall): A = P.A^T
    A = P.A.T.copy()
    rng = np.random.default_rng(seed + 1)
    b = A @ (rng.standard_normal(d) / math.sqrt(d)) + 1e-3 * rng.standard_normal(n)
    return A, b, P.lam


def test_dual_mihs_reaches_primal_closed_form():
    """Dual M-IHS (Algorithm 2) with CG or exact inner solves converges to the
    primal ridge solution, computed independently by least squares of
    [A; sqrt(lambda) I] (the problem has n < d)."""
    A, b, lam = _wide()
    xs = O.ridge_lstsq(A, b, lam)
    SAt = sketches.gaussian_sketch(A.T, 120, 4)   # S A^T, m x n
    a, bt = O.momentum_cor4(15.0, 120)
    for inner in ("exact", "cg"):
        r = O.dual_mihs(A, b, lam, SAt, a, bt, inner=inner, eps_sub=1e-10, tol=1e-13)
        assert r.converged
        assert np.linalg.norm(r.x - xs) <= 1e-10 * np.linalg.norm(xs), inner
        # eq. (dual_relation): nu* = (b - A x*) / lambda
        nu_ref = (b - A @ xs) / lam
        assert np.linalg.norm(r.nu - nu_ref) <= 1e-9 * np.linalg.norm(nu_ref), inner


def test_dual_one_step_with_identity_sketch():
    """S = I (the sketch of A^T is A^T itself), exact inner solve, alpha = 1,
    beta = 0: the sub-problem Hessian is A A^T + lambda I, so one step reaches nu*."""
    A, b, lam = _wide(n=30, d=90, seed=9)
    r = O.dual_mihs(A, b, lam, A.T.copy(), 1.0, 0.0, inner="exact", n_iter=1)
    nu_star = np.linalg.solve(A @ A.T + lam * np.eye(A.shape[0]), b)
    assert np.linalg.norm(r.nu - nu_star) <= 1e-12 * np.linalg.norm(nu_star)


def test_dual_planted_mistake_is_caught(monkeypatch):
    """Dropping the lambda nu term from the dual gradient breaks the pin."""
    A, b, lam = _wide()
    xs = O.ridge_lstsq(A, b, lam)
    SAt = sketches.gaussian_sketch(A.T, 120, 4)
    a, bt = O.momentum_cor4(15.0, 120)
    monkeypatch.setattr(O, "dual_gradient", lambda A_, b_, l_, nu: b_ - A_ @ (A_.T @ nu))
    r = O.dual_mihs(A, b, lam, SAt, a, bt, inner="exact", n_iter=80)
    assert np.linalg.norm(r.x - xs) > 1e-6 * np.linalg.norm(xs)


def test_hutchinson_exact_with_hadamard_probes():
    """Hadamard columns as probes (T = d, H H^T = d I): sum_l h_l^T M h_l = d tr(M),
    so Algorithm 5 with exact inner solves returns d - lambda tr(M^{-1}) exactly.
    With S = I that is sd(A) = sum sigma^2 / (sigma^2 + lambda) (Section 3.4)."""
    from scipy.linalg import hadamard
    P = _small(d=64)
    d = P.A.shape[1]
    assert d & (d - 1) == 0
    H = hadamard(d).astype(np.float64)
    SA = sketches.gaussian_sketch(P.A, 96, 3)
    est = O.hutchinson_sd(SA, P.lam, H, inner="exact")
    assert abs(est - O.sketched_sd_exact(SA, P.lam)) <= 1e-9 * d
    est_a = O.hutchinson_sd(P.A, P.lam, H, inner="exact")
    assert abs(est_a - O.statistical_dimension(P.A, P.lam)) <= 1e-9 * d


def test_hutchinson_random_probes_are_unbiased():
    """Rademacher probes from the counter-based rule: +-1 entries, and the mean
    of many single-probe estimates lies within 4 standard errors of the exact
    sketched quantity."""
    P = _small()
    d = P.A.shape[1]
    V = sketches.rademacher_probes(d, 400, 11)
    assert set(np.unique(V)) == {-1.0, 1.0}
    assert abs(V.mean()) < 0.02
    SA = sketches.gaussian_sketch(P.A, 96, 3)
    ests = np.array([O.hutchinson_sd(SA, P.lam, V[:, l:l + 1], inner="exact") for l in range(400)])
    se = ests.std(ddof=1) / math.sqrt(len(ests))
    assert abs(ests.mean() - O.sketched_sd_exact(SA, P.lam)) <= 4 * se


def test_hutchinson_inexact_inner_solvers_agree():
    """eps_tr small: AAb_Solver, CG and the exact solve give the same estimate."""
    P = _small()
    V = sketches.rademacher_probes(P.A.shape[1], 3, 5)
    SA = sketches.gaussian_sketch(P.A, 96, 3)
    ex = O.hutchinson_sd(SA, P.lam, V, inner="exact")
    for inner in ("aab", "cg"):
        assert abs(O.hutchinson_sd(SA, P.lam, V, inner=inner, eps_tr=1e-12) - ex) <= 1e-8 * abs(ex)


def _pd_problem(n=1500, d=160, sd=8.0, seed=21, rate=10.0):
    sig = W.sigma_profile("exp", min(n, d), rate)
    return W.make_problem(n, d, sig, sd, seed)


def test_pd_inner_reaches_dual_subproblem_solution():
    """Many dual M-IHS steps (exact inner solves) reach
    z* = (SA SA^T + lambda I)^{-1} SA c, and the recovered step
    (c - SA^T z*)/lambda is (SA^T SA + lambda I)^{-1} c (push-through identity),
    both from library solves."""
    P = _pd_problem()
    d = P.A.shape[1]
    SA = sketches.gaussian_sketch(P.A, 40, 5)
    WSAt = sketches.gaussian_sketch(SA.T.copy(), 40, 6)
    c = np.random.default_rng(0).standard_normal(d)
    a2, b2 = O.momentum_cor4(8.0, 40)
    z, _, _ = O._pd_inner(SA, WSAt, c, np.zeros(40), np.zeros(40), P.lam, a2, b2, 300, "exact",
                          0.0, None)
    zs = np.linalg.solve(SA @ SA.T + P.lam * np.eye(40), SA @ c)
    assert np.linalg.norm(z - zs) <= 1e-10 * np.linalg.norm(zs)
    dx = (c - SA.T @ z) / P.lam
    dxs = np.linalg.solve(SA.T @ SA + P.lam * np.eye(d), c)
    assert np.linalg.norm(dx - dxs) <= 1e-9 * np.linalg.norm(dxs)


def test_pd_one_step_with_identity_sketches():
    """S = I and W = I (the second sketch of A^T is A^T), exact inner solve,
    M = 1, unit step, no momentum: one outer step from x = 0 reaches x*."""
    P = _small(n=60, d=20, sd=6.0, seed=4)
    xs = O.ridge_lstsq(P.A, P.b, P.lam)
    r = O.primal_dual_mihs(P.A, P.b, P.lam, P.A, P.A.T.copy(), 1.0, 0.0, 1.0, 0.0, M=1,
                           inner="exact", n_iter=1)
    assert np.linalg.norm(r.x - xs) <= 1e-10 * np.linalg.norm(xs)


@pytest.mark.parametrize("inner", ["aab", "cg"])
def test_pd_reaches_closed_form_tall_and_wide(inner):
    """Algorithms 4 (n >= d) and 3 (n <= d) with m1 = m2 = 5 sd, M = 10 dual
    steps of eps_sub = 0.1 each: the iterate converges to the ridge solution
    from least squares of [A; sqrt(lambda) I]."""
    P = _pd_problem()
    xs = O.ridge_lstsq(P.A, P.b, P.lam)
    m = 40
    SA = sketches.gaussian_sketch(P.A, m, 5)
    WSAt = sketches.gaussian_sketch(SA.T.copy(), m, 6)
    a, b = O.momentum_cor4(8.0, m)
    r = O.primal_dual_mihs(P.A, P.b, P.lam, SA, WSAt, a, b, a, b, M=10, inner=inner,
                           n_iter=80)
    assert np.linalg.norm(r.x - xs) <= 1e-9 * np.linalg.norm(xs)
    # the wide problem A^T (d x n with d < n): Algorithm 3 on it
    Aw = P.A.T.copy()
    bw = np.random.default_rng(1).standard_normal(Aw.shape[0])
    xw = O.ridge_lstsq(Aw, bw, P.lam)
    SAt = sketches.gaussian_sketch(Aw.T.copy(), m, 7)
    WASt = sketches.gaussian_sketch(SAt.T.copy(), m, 8)
    rw = O.primal_dual_mihs_wide(Aw, bw, P.lam, SAt, WASt, a, b, a, b, M=10, inner=inner,
                                 n_iter=80)
    assert np.linalg.norm(rw.x - xw) <= 1e-9 * np.linalg.norm(xw)


def test_pd_planted_mistake_is_caught(monkeypatch):
    """Dropping the lambda z term of the dual gradient breaks the sub-problem pin."""
    P = _pd_problem()
    d = P.A.shape[1]
    SA = sketches.gaussian_sketch(P.A, 40, 5)
    WSAt = sketches.gaussian_sketch(SA.T.copy(), 40, 6)
    c = np.random.default_rng(0).standard_normal(d)
    a2, b2 = O.momentum_cor4(8.0, 40)
    monkeypatch.setattr(O, "pd_dual_gradient", lambda SM, cc, lam, z: SM @ (cc - SM.T @ z))
    z, _, _ = O._pd_inner(SA, WSAt, c, np.zeros(40), np.zeros(40), P.lam, a2, b2, 300, "exact",
                          0.0, None)
    zs = np.linalg.solve(SA @ SA.T + P.lam * np.eye(40), SA @ c)
    assert not (np.linalg.norm(z - zs) <= 1e-6 * np.linalg.norm(zs))


@pytest.mark.parametrize("beta", [0.04, 0.25, 0.5, 0.81])
def test_stop_threshold_is_exact_for_geometric_convergence(beta):
    """The relative-step rule (Corollary 4's rate rho = sqrt(beta)): for an iterate
    sequence x_k = x* + rho^k v converging at exactly that rate,
    ||x_{k+1} - x*|| = rho / (1 - rho) ||x_{k+1} - x_k||, so the rule stops at the
    first k whose true relative error is <= tol, never earlier and never later."""
    rng = np.random.default_rng(7)
    xs = rng.standard_normal(50)
    v = rng.standard_normal(50)
    rho = math.sqrt(beta)
    tol = 1e-10
    thr = O.stop_threshold(tol, beta)
    stop_k, first_ok = None, None
    for k in range(1, 400):
        x = xs + rho ** k * v
        # the differences in closed form (no cancellation against x*)
        step = np.linalg.norm(rho ** (k - 1) * (rho - 1.0) * v) / np.linalg.norm(x)
        err = np.linalg.norm(rho ** k * v) / np.linalg.norm(x)
        # the identity behind the rule
        assert math.isclose(err, step * rho / (1.0 - rho), rel_tol=1e-9)
        if stop_k is None and step <= thr:
            stop_k = k
        if first_ok is None and err <= tol * (1.0 + 1e-9):
            first_ok = k
        if stop_k is not None and first_ok is not None:
            break
    assert stop_k == first_ok, (stop_k, first_ok)
    # a planted mistake (threshold tol * rho, the rate's place swapped) stops
    # at another iterate whenever rho / (1 - rho) != 1 / rho
    wrong = tol * rho
    if abs(rho / (1.0 - rho) - 1.0 / rho) > 0.05:
        stop_w = next(k for k in range(1, 400)
                      if np.linalg.norm(rho ** (k - 1) * (rho - 1.0) * v)
                      / np.linalg.norm(xs + rho ** k * v) <= wrong)
        assert stop_w != first_ok
