"""Oracle: M-IHS for ridge regression, step by step, in float64 on the CPU.

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's CPU
baseline call this module; the GPU library shares no code with it.

Problem (Section 1, eq. (intro)):  x* = argmin 1/2 ||Ax - b||^2 + lambda/2 ||x||^2,
whose plain definition is x* = (A^T A + lambda I)^{-1} A^T b.

M-IHS (Section 3, eq. (mihs1) and Algorithm 1), with one sketch S for all
iterations:
    g^i      = A^T (b - A x^i) - lambda x^i
    dx^i     = argmin ||S A z||^2 + lambda ||z||^2 - 2 <g^i, z>
             = ((SA)^T SA + lambda I)^{-1} g^i            (solved inexactly)
    x^{i+1}  = x^i + alpha dx^i + beta (x^i - x^{i-1}),   x^0 = x^1.
(eq. (mihs1) writes the linear term with grad f = -g; the minimiser above is
the same step.)  Momentum: Corollary 4 (beta = sd/m, alpha = (1-beta)^2) or
Theorem 1 (beta*, alpha* from the embedding accuracy epsilon).

Inner solvers: exact (Cholesky of the d x d sketched Hessian), conjugate
gradients stopped on the relative residual eps_sub (Section 3.1's constant
forcing term), and AAb_Solver (Algorithm 6, Section 3.5).

Dual M-IHS (Section 2, eqs. (intro_dual), (dual_mihs1); Algorithm 2) for
n <= d iterates on the dual variable nu in R^n with a sketch of A^T and
recovers x* = A^T nu* (eq. (dual_relation)).

The statistical dimension that sets beta can be estimated from the sketch by
the inexact Hutchinson trace estimator (Algorithm 5, Section 3.4).

Primal-Dual M-IHS (Section 2, two-stage sketching, eq. (pd_mihs1); Algorithms 3
and 4) solves each sub-problem through its dual, approximately, by M-IHS steps
with a second sketch W (SA)^T of the dual's Hessian.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Tuple

import numpy as np
import scipy.linalg as sla


# ----------------------------------------------------------------------------
# Closed forms
# ----------------------------------------------------------------------------
def ridge_cholesky(A: np.ndarray, b: np.ndarray, lam: float) -> np.ndarray:
    """x* = (A^T A + lambda I)^{-1} A^T b by a dense Cholesky factorisation."""
    A64 = A.astype(np.float64, copy=False)
    H = A64.T @ A64 + lam * np.eye(A.shape[1])
    c = sla.cho_factor(H, lower=True)
    return sla.cho_solve(c, A64.T @ b)


def ridge_lstsq(A: np.ndarray, b: np.ndarray, lam: float) -> np.ndarray:
    """x* as the least-squares solution of [A; sqrt(lambda) I] x = [b; 0]
    (Householder QR via LAPACK; avoids squaring the condition number)."""
    n, d = A.shape
    M = np.vstack([A.astype(np.float64), math.sqrt(lam) * np.eye(d)])
    rhs = np.concatenate([b, np.zeros((d,) + b.shape[1:])])
    return np.linalg.lstsq(M, rhs, rcond=None)[0]


def statistical_dimension(A: np.ndarray, lam: float) -> float:
    """sd_lambda(A) = tr(A (A^T A + lambda I)^{-1} A^T) = sum sigma_i^2/(sigma_i^2+lambda) (Section 1)."""
    s = np.linalg.svd(A.astype(np.float64), compute_uv=False)
    return float(np.sum(s * s / (s * s + lam)))


# ----------------------------------------------------------------------------
# Momentum parameters
# ----------------------------------------------------------------------------
def momentum_cor4(sd: float, m: int) -> Tuple[float, float]:
    """Corollary 4: beta = sd/m, alpha = (1 - beta)^2; rate sqrt(beta)."""
    beta = sd / m
    if not 0.0 < beta < 1.0:
        raise ValueError("need 0 < sd < m")
    return (1.0 - beta) ** 2, beta


def momentum_thm1(eps: float) -> Tuple[float, float]:
    """Theorem 1: beta* = (eps / (1 + sqrt(1-eps^2)))^2, alpha* = (1 - beta*) sqrt(1 - eps^2)."""
    if not 0.0 < eps < 1.0:
        raise ValueError("need 0 < eps < 1")
    beta = (eps / (1.0 + math.sqrt(1.0 - eps * eps))) ** 2
    return (1.0 - beta) * math.sqrt(1.0 - eps * eps), beta


def heavy_ball_rate(mu: np.ndarray, alpha: float, beta: float) -> float:
    """Spectral radius of the two-term recursion for eigenvalues mu of
    (sketched Hessian)^{-1} (Hessian): largest root modulus of
    u^2 - (1 + beta - alpha mu) u + beta = 0 (eq. (characteristic))."""
    worst = 0.0
    for m_ in np.atleast_1d(mu):
        roots = np.roots([1.0, -(1.0 + beta - alpha * m_), beta])
        worst = max(worst, float(np.max(np.abs(roots))))
    return worst


def iterations_cor4(eta: float, beta: float) -> int:
    """Corollary 4: at most log(eta) / log(sqrt(beta)) iterations."""
    return int(math.ceil(math.log(eta) / math.log(math.sqrt(beta))))


# ----------------------------------------------------------------------------
# Gradient (Algorithm 1, the per-iteration pass over A)
# ----------------------------------------------------------------------------
def gradient(A: np.ndarray, b: np.ndarray, lam: float, x: np.ndarray) -> np.ndarray:
    """g = A^T (b - A x) - lambda x, FP32 A upcast exactly to FP64."""
    A64 = A.astype(np.float64, copy=False)
    return A64.T @ (b - A64 @ x) - lam * x


def gradient_rhs(A: np.ndarray, rhs: np.ndarray, lam: float, w: np.ndarray) -> np.ndarray:
    """Gradient of the adjoint system (A^T A + lambda I) w = rhs: rhs - A^T A w - lambda w."""
    A64 = A.astype(np.float64, copy=False)
    return rhs - A64.T @ (A64 @ w) - lam * w


# ----------------------------------------------------------------------------
# Inner solvers for ((SA)^T SA + lambda I) z = g
# ----------------------------------------------------------------------------
def inner_exact_factory(SA: np.ndarray, lam: float) -> Callable[[np.ndarray], Tuple[np.ndarray, int]]:
    SA64 = SA.astype(np.float64, copy=False)
    c = sla.cho_factor(SA64.T @ SA64 + lam * np.eye(SA.shape[1]), lower=True)
    return lambda g: (sla.cho_solve(c, g), 0)


def inner_cg(SA: np.ndarray, g: np.ndarray, lam: float, eps: float,
             max_iter: Optional[int] = None) -> Tuple[np.ndarray, int]:
    """Conjugate gradients from z = 0 on (SA^T SA + lambda I) z = g, the operator
    applied as SA^T (SA p) + lambda p; stops once ||r|| <= eps ||g||."""
    SA64 = SA.astype(np.float64, copy=False)
    d = g.shape[0]
    max_iter = max_iter if max_iter is not None else 10 * d
    z = np.zeros_like(g)
    r = g.copy()
    p = r.copy()
    rr = float(r @ r)
    stop = (eps * eps) * rr
    k = 0
    while rr > stop and k < max_iter:
        q = SA64.T @ (SA64 @ p) + lam * p
        a = rr / float(p @ q)
        z += a * p
        r -= a * q
        rr_new = float(r @ r)
        p = r + (rr_new / rr) * p
        rr = rr_new
        k += 1
    return z, k


def aab_solver(M: np.ndarray, b: np.ndarray, lam: float, eps: float,
               max_iter: Optional[int] = None, trace: Optional[list] = None) -> Tuple[np.ndarray, int]:
    """AAb_Solver (Algorithm 6) for (M^T M + lambda I) x = b.

    Upper bidiagonalisation started from theta_1 v = b; the sqrt(lambda) block is
    folded in by Givens rotations (Section 3.5): c = rho/rhobar,
    s = lambdabar/rhobar, thetabar = c theta, lambdabar^2 = lambda + (s theta)^2,
    rhobar = sqrt(rho^2 + lambdabar^2), starting from lambdabar_1 = sqrt(lambda).
    The first-step sine is therefore sqrt(lambda)/rhobar (the listing's
    sqrt(lambda/rhobar) contradicts the recurrence it implements; the text's
    recurrence is followed).  Stops on |phi rhobar| / theta_1 < eps, the
    relative residual norm of the previous iterate.  If `trace` is a list, it
    receives (x, t) after every step (the initial iterate with t = inf first).
    """
    M64 = M.astype(np.float64, copy=False)
    max_iter = max_iter if max_iter is not None else 10 * M.shape[1]
    theta1 = float(np.linalg.norm(b))
    if theta1 == 0.0:
        return np.zeros_like(b), 0
    v = b / theta1
    pv = M64 @ v
    rho = float(np.linalg.norm(pv))
    p = pv / rho
    rhobar = math.sqrt(rho * rho + lam)
    c = rho / rhobar
    s = math.sqrt(lam) / rhobar
    phi = theta1 / rhobar
    dvec = v / rhobar
    x = phi * dvec
    t = math.inf
    k = 0
    if trace is not None:
        trace.append((x.copy(), t))
    while t >= eps and k < max_iter:
        w = M64.T @ p - rho * v
        theta = float(np.linalg.norm(w))
        v = w / theta
        w2 = M64 @ v - theta * p
        rho = float(np.linalg.norm(w2))
        p = w2 / rho
        lbar = math.sqrt(lam + (s * theta) ** 2)
        thetabar = c * theta
        rhobar = math.sqrt(rho * rho + lbar * lbar)
        c = rho / rhobar
        s = lbar / rhobar
        dvec = (v - thetabar * dvec) / rhobar
        phi = -phi * thetabar / rhobar
        x = x + phi * dvec
        t = abs(phi * rhobar) / theta1
        k += 1
        if trace is not None:
            trace.append((x.copy(), t))
    return x, k


# ----------------------------------------------------------------------------
# M-IHS outer loop
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class MihsResult:
    x: np.ndarray
    outer: int
    inner: List[int]
    steps: List[float]
    converged: bool
    history: Optional[List[np.ndarray]] = None


def stop_threshold(tol: float, beta: float) -> float:
    """Relative-step threshold for the stop test: with contraction rate
    rho = sqrt(beta), ||x^{i+1} - x*|| <= rho/(1-rho) ||x^{i+1} - x^i||, so the
    iteration stops when ||x^{i+1}-x^i|| / ||x^{i+1}|| <= tol (1-rho)/rho."""
    rho = math.sqrt(beta)
    return tol * (1.0 - rho) / rho


def mihs(A: np.ndarray, b: np.ndarray, lam: float, SA: np.ndarray, alpha: float, beta: float,
         *, inner: str = "cg", eps_sub: float = 1e-2, max_inner: Optional[int] = None,
         n_iter: Optional[int] = None, tol: Optional[float] = None, max_outer: int = 500,
         x1: Optional[np.ndarray] = None, keep_history: bool = False,
         rhs_mode: bool = False) -> MihsResult:
    """M-IHS (Algorithm 1).  Runs exactly `n_iter` iterations if given, else
    stops on the relative-step rule with target `tol` (or at `max_outer`).

    rhs_mode=True solves (A^T A + lambda I) x = b for a d-vector b (the adjoint
    system of the backward pass): the gradient becomes b - A^T A x - lambda x.
    """
    d = A.shape[1]
    x = np.zeros(d) if x1 is None else np.array(x1, dtype=np.float64)
    x_prev = x.copy()
    exact = inner_exact_factory(SA, lam) if inner == "exact" else None
    inner_counts: List[int] = []
    steps: List[float] = []
    hist = [x.copy()] if keep_history else None
    thr = stop_threshold(tol, beta) if tol is not None else None
    limit = n_iter if n_iter is not None else max_outer
    converged = False
    it = 0
    for it in range(1, limit + 1):
        g = gradient_rhs(A, b, lam, x) if rhs_mode else gradient(A, b, lam, x)
        if inner == "exact":
            dx, k = exact(g)
        elif inner == "cg":
            dx, k = inner_cg(SA, g, lam, eps_sub, max_inner)
        elif inner == "aab":
            dx, k = aab_solver(SA, g, lam, eps_sub, max_inner)
        else:
            raise ValueError(inner)
        inner_counts.append(k)
        x_new = x + alpha * dx + beta * (x - x_prev)
        nrm = float(np.linalg.norm(x_new))
        step = float(np.linalg.norm(x_new - x)) / nrm if nrm > 0 else 0.0
        steps.append(step)
        x_prev, x = x, x_new
        if keep_history:
            hist.append(x.copy())
        if thr is not None and n_iter is None and step <= thr:
            converged = True
            break
    return MihsResult(x=x, outer=it, inner=inner_counts, steps=steps, converged=converged,
                      history=hist)


# ----------------------------------------------------------------------------
# Statistical dimension estimate (Algorithm 5)
# ----------------------------------------------------------------------------
def sketched_sd_exact(SA: np.ndarray, lam: float) -> float:
    """The quantity Algorithm 5 estimates, d - lambda tr(((SA)^T SA + lambda I)^{-1})
    = sum_i mu_i / (mu_i + lambda) over the eigenvalues mu_i of (SA)^T SA."""
    mu = np.linalg.eigvalsh(SA.astype(np.float64).T @ SA.astype(np.float64))
    return float(np.sum(mu / (mu + lam)))


def hutchinson_sd(SA: np.ndarray, lam: float, V: np.ndarray, *, inner: str = "aab",
                  eps_tr: float = 0.5, max_inner: Optional[int] = None) -> float:
    """Inexact Hutchinson estimate of sd (Algorithm 5): for each probe column v^l
    of V (d x T), z^l solves ((SA)^T SA + lambda I) z = v^l to relative residual
    eps_tr (AAb_Solver in the paper; CG or exact here as well); tau accumulates
    lambda <v^l, z^l>; the estimate is d - tau / T."""
    d, T = V.shape
    exact = inner_exact_factory(SA, lam) if inner == "exact" else None
    tau = 0.0
    for l in range(T):
        v = V[:, l]
        if inner == "exact":
            z, _ = exact(v)
        elif inner == "cg":
            z, _ = inner_cg(SA, v, lam, eps_tr, max_inner)
        elif inner == "aab":
            z, _ = aab_solver(SA, v, lam, eps_tr, max_inner)
        else:
            raise ValueError(inner)
        tau += lam * float(v @ z)
    return d - tau / T


# ----------------------------------------------------------------------------
# Dual M-IHS (n <= d)
# ----------------------------------------------------------------------------
def dual_gradient(A: np.ndarray, b: np.ndarray, lam: float, nu: np.ndarray) -> np.ndarray:
    """The descent direction of the dual objective g(nu) = 1/2 ||A^T nu||^2 +
    lambda/2 ||nu||^2 - <b, nu> (eq. (intro_dual)): b - A A^T nu - lambda nu
    (Algorithm 2's gradient line; it is -grad g)."""
    A64 = A.astype(np.float64, copy=False)
    return b - A64 @ (A64.T @ nu) - lam * nu


@dataclasses.dataclass
class DualMihsResult:
    x: np.ndarray     # primal solution A^T nu
    nu: np.ndarray    # dual iterate
    outer: int
    inner: List[int]
    steps: List[float]
    converged: bool


def dual_mihs(A: np.ndarray, b: np.ndarray, lam: float, SAt: np.ndarray, alpha: float,
              beta: float, *, inner: str = "cg", eps_sub: float = 1e-2,
              max_inner: Optional[int] = None, n_iter: Optional[int] = None,
              tol: Optional[float] = None, max_outer: int = 500) -> DualMihsResult:
    """Dual M-IHS (Algorithm 2) for A n x d with n <= d and SAt = S A^T (m x n).

    nu^1 = 0; per iteration
        g^i       = b - A A^T nu^i - lambda nu^i
        dnu^i     = ((S A^T)^T S A^T + lambda I)^{-1} g^i     (the sub-problem
                    of eq. (dual_mihs1), solved by the chosen inner solver)
        nu^{i+1}  = nu^i + alpha dnu^i + beta (nu^i - nu^{i-1}),  nu^0 = nu^1,
    and finally x = A^T nu (eq. (dual_relation)).  Runs `n_iter` iterations if
    given, else stops on the relative-step rule for nu with target `tol`."""
    n = A.shape[0]
    nu = np.zeros(n)
    nu_prev = nu.copy()
    exact = inner_exact_factory(SAt, lam) if inner == "exact" else None
    inner_counts: List[int] = []
    steps: List[float] = []
    thr = stop_threshold(tol, beta) if tol is not None else None
    limit = n_iter if n_iter is not None else max_outer
    converged = False
    it = 0
    for it in range(1, limit + 1):
        g = dual_gradient(A, b, lam, nu)
        if inner == "exact":
            dnu, k = exact(g)
        elif inner == "cg":
            dnu, k = inner_cg(SAt, g, lam, eps_sub, max_inner)
        elif inner == "aab":
            dnu, k = aab_solver(SAt, g, lam, eps_sub, max_inner)
        else:
            raise ValueError(inner)
        inner_counts.append(k)
        nu_new = nu + alpha * dnu + beta * (nu - nu_prev)
        nrm = float(np.linalg.norm(nu_new))
        step = float(np.linalg.norm(nu_new - nu)) / nrm if nrm > 0 else 0.0
        steps.append(step)
        nu_prev, nu = nu, nu_new
        if thr is not None and n_iter is None and step <= thr:
            converged = True
            break
    x = A.astype(np.float64, copy=False).T @ nu
    return DualMihsResult(x=x, nu=nu, outer=it, inner=inner_counts, steps=steps,
                          converged=converged)


# ----------------------------------------------------------------------------
# Primal-Dual M-IHS (two-stage sketching; Section 2, eq. (pd_mihs1); Algorithms 3, 4)
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class PrimalDualResult:
    x: np.ndarray
    outer: int
    inner: List[int]       # inner-solver steps summed over the M dual steps of each outer step
    steps: List[float]
    converged: bool
    nu: Optional[np.ndarray] = None


def pd_dual_gradient(SM: np.ndarray, c: np.ndarray, lam: float, z: np.ndarray) -> np.ndarray:
    """Gradient of the sub-problem's dual (Algorithms 3, 4): SM (c - SM^T z) - lambda z."""
    return SM @ (c - SM.T @ z) - lam * z


def _pd_inner(SM: np.ndarray, WSMt: np.ndarray, c: np.ndarray, z: np.ndarray,
              z_prev: np.ndarray, lam: float, alpha2: float, beta2: float, M: int,
              inner: str, eps_sub: float, max_inner: Optional[int]):
    """M M-IHS steps on the dual of the sketched sub-problem,
        min_z 1/2 ||SM^T z - c||^2 + lambda/2 ||z||^2      (z in R^{m1}),
    whose Hessian SM SM^T + lambda I is sketched again by WSMt = W SM^T (m2 x m1):
        g      = SM (c - SM^T z) - lambda z
        dz     = ((WSMt)^T WSMt + lambda I)^{-1} g          (inner solver)
        z_next = z + alpha2 dz + beta2 (z - z_prev)."""
    SM64 = SM.astype(np.float64, copy=False)
    exact = inner_exact_factory(WSMt, lam) if inner == "exact" else None
    total = 0
    for _ in range(M):
        g = pd_dual_gradient(SM64, c, lam, z)
        if inner == "exact":
            dz, k = exact(g)
        elif inner == "cg":
            dz, k = inner_cg(WSMt, g, lam, eps_sub, max_inner)
        elif inner == "aab":
            dz, k = aab_solver(WSMt, g, lam, eps_sub, max_inner)
        else:
            raise ValueError(inner)
        total += k
        z, z_prev = z + alpha2 * dz + beta2 * (z - z_prev), z
    return z, z_prev, total


def primal_dual_mihs(A: np.ndarray, b: np.ndarray, lam: float, SA: np.ndarray,
                     WSAt: np.ndarray, alpha1: float, beta1: float, alpha2: float,
                     beta2: float, *, M: int, inner: str = "aab", eps_sub: float = 0.1,
                     max_inner: Optional[int] = None, n_iter: Optional[int] = None,
                     tol: Optional[float] = None, max_outer: int = 500) -> PrimalDualResult:
    """Primal Dual M-IHS for n >= d (Algorithm 4).  SA = S A is m1 x d and
    WSAt = W (SA)^T is m2 x m1.  x^1 = 0, z^{1,1} = z^{1,0} = 0; per outer step
        b^i      = A^T (b - A x^i) - lambda x^i
        z        <- M dual M-IHS steps on min 1/2 ||(SA)^T z - b^i||^2 + lambda/2 ||z||^2
        dx^i     = (b^i - (SA)^T z) / lambda                  (eq. (dual_relation))
        x^{i+1}  = x^i + alpha1 dx^i + beta1 (x^i - x^{i-1}),  x^0 = x^1.
    The dual iterate and its momentum state carry over from one outer step to
    the next (z^{i+1,1} = z^{i,M+1}, and z^{i+1,0} = z^{i,M}).  Runs `n_iter`
    outer steps if given, else stops on the relative-step rule for x."""
    A64 = A.astype(np.float64, copy=False)
    SA64 = SA.astype(np.float64, copy=False)
    d = A.shape[1]
    m1 = SA.shape[0]
    x = np.zeros(d)
    x_prev = x.copy()
    z = np.zeros(m1)
    z_prev = z.copy()
    inner_counts: List[int] = []
    steps: List[float] = []
    thr = stop_threshold(tol, beta1) if tol is not None else None
    limit = n_iter if n_iter is not None else max_outer
    converged = False
    it = 0
    for it in range(1, limit + 1):
        bi = gradient(A64, b, lam, x)
        z, z_prev, k = _pd_inner(SA64, WSAt, bi, z, z_prev, lam, alpha2, beta2, M, inner,
                                 eps_sub, max_inner)
        inner_counts.append(k)
        dx = (bi - SA64.T @ z) / lam
        x_new = x + alpha1 * dx + beta1 * (x - x_prev)
        nrm = float(np.linalg.norm(x_new))
        step = float(np.linalg.norm(x_new - x)) / nrm if nrm > 0 else 0.0
        steps.append(step)
        x_prev, x = x, x_new
        if thr is not None and n_iter is None and step <= thr:
            converged = True
            break
    return PrimalDualResult(x=x, outer=it, inner=inner_counts, steps=steps,
                            converged=converged)


def primal_dual_mihs_wide(A: np.ndarray, b: np.ndarray, lam: float, SAt: np.ndarray,
                          WASt: np.ndarray, alpha1: float, beta1: float, alpha2: float,
                          beta2: float, *, M: int, inner: str = "aab", eps_sub: float = 0.1,
                          max_inner: Optional[int] = None, n_iter: Optional[int] = None,
                          tol: Optional[float] = None, max_outer: int = 500) -> PrimalDualResult:
    """Primal Dual M-IHS for n <= d (Algorithm 3).  SAt = S A^T is m1 x n and
    WASt = W (S A^T)^T is m2 x m1.  nu^1 = 0, z^{1,1} = z^{1,0} = 0; per outer step
        b^i       = b - A A^T nu^i - lambda nu^i
        z         <- M dual M-IHS steps on min 1/2 ||(S A^T)^T z - b^i||^2 + lambda/2 ||z||^2
        dnu^i     = (b^i - (S A^T)^T z) / lambda
        nu^{i+1}  = nu^i + alpha1 dnu^i + beta1 (nu^i - nu^{i-1}),
    and finally x = A^T nu.  z carries over as in Algorithm 4."""
    A64 = A.astype(np.float64, copy=False)
    SAt64 = SAt.astype(np.float64, copy=False)
    n = A.shape[0]
    m1 = SAt.shape[0]
    nu = np.zeros(n)
    nu_prev = nu.copy()
    z = np.zeros(m1)
    z_prev = z.copy()
    inner_counts: List[int] = []
    steps: List[float] = []
    thr = stop_threshold(tol, beta1) if tol is not None else None
    limit = n_iter if n_iter is not None else max_outer
    converged = False
    it = 0
    for it in range(1, limit + 1):
        bi = dual_gradient(A64, b, lam, nu)
        z, z_prev, k = _pd_inner(SAt64, WASt, bi, z, z_prev, lam, alpha2, beta2, M, inner,
                                 eps_sub, max_inner)
        inner_counts.append(k)
        dnu = (bi - SAt64.T @ z) / lam
        nu_new = nu + alpha1 * dnu + beta1 * (nu - nu_prev)
        nrm = float(np.linalg.norm(nu_new))
        step = float(np.linalg.norm(nu_new - nu)) / nrm if nrm > 0 else 0.0
        steps.append(step)
        nu_prev, nu = nu, nu_new
        if thr is not None and n_iter is None and step <= thr:
            converged = True
            break
    return PrimalDualResult(x=A64.T @ nu, outer=it, inner=inner_counts, steps=steps,
                            converged=converged, nu=nu)


# ----------------------------------------------------------------------------
# Backward of the ridge solution (differentiation workload)
# ----------------------------------------------------------------------------
def ridge_backward_dense(A: np.ndarray, lam: float, xstar: np.ndarray, gbar: np.ndarray):
    """For L(x*(B, lambda)) with dL/dx* = gbar (d x k):
    W = (A^T A + lambda I)^{-1} gbar, dL/dB = A W, dL/dlambda = -sum_j x*_j^T w_j."""
    A64 = A.astype(np.float64, copy=False)
    H = A64.T @ A64 + lam * np.eye(A.shape[1])
    c = sla.cho_factor(H, lower=True)
    W = sla.cho_solve(c, gbar)
    return W, A64 @ W, -float(np.sum(xstar * W))
