"""Seeded synthetic ridge-regression workloads.

This module only draws inputs: the matrix A, the right-hand side b, the
regularisation weight lambda and the sizes of each workload.  It holds none of
the solver's arithmetic, and both the CPU oracle and the GPU path take their
inputs from here.

Workload recipe (the paper's data model, eq. (setup): A x0 + w = b):

* A = G diag(sigma) Q with G iid N(0,1)/sqrt(n) (n x d) and Q Haar-orthogonal
  (QR of a seeded d x d Gaussian, columns sign-fixed by sign(diag R));
* x0 ~ N(0, 1/d) per entry;
* b = A x0 + w with w ~ N(0, 1e-4 * ||A x0||^2 / n) per entry (1% noise, as in
  the paper's noisy experiments, Section 4.4);
* lambda is chosen so that the statistical dimension of the *nominal* spectrum,
  sum_i sigma_i^2 / (sigma_i^2 + lambda) (Section 1), equals a target value.
  The realised statistical dimension of the drawn A differs slightly because G
  is not exactly orthonormal; over-estimating it is safe (Remark after
  Corollary 4).

The paper's own test matrices (RegTools profiles, Section 4.1) are not
available; these seeded matrices with exponential or polynomial singular-value
decay stand in for them.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

__all__ = [
    "sigma_profile", "lambda_for_sd", "nominal_sd", "Problem", "make_problem",
    "WORKLOADS", "Workload", "workload", "batched_specs", "BatchedSpec",
]


def sigma_profile(kind: str, d: int, rate: float = 0.0) -> np.ndarray:
    """Nominal singular values sigma_i, i = 1..d (index origin 1)."""
    i = np.arange(1, d + 1, dtype=np.float64)
    if kind == "exp":
        return np.exp(-rate * i / d)
    if kind == "poly":
        return i ** (-rate)
    raise ValueError(f"unknown sigma profile {kind!r}")


def nominal_sd(sigma: np.ndarray, lam: float) -> float:
    s2 = sigma.astype(np.float64) ** 2
    return float(np.sum(s2 / (s2 + lam)))


def lambda_for_sd(sigma: np.ndarray, target: float) -> float:
    """Bisection in log(lambda) so that the nominal statistical dimension hits `target`."""
    if not (0.0 < target < len(sigma)):
        raise ValueError("target statistical dimension must lie in (0, d)")
    lo, hi = 1e-30, 1e10
    for _ in range(300):
        mid = math.sqrt(lo * hi)
        if nominal_sd(sigma, mid) > target:
            lo = mid
        else:
            hi = mid
    return math.sqrt(lo * hi)


@dataclasses.dataclass
class Problem:
    A: np.ndarray          # n x d, row-major, float64 or float32
    b: np.ndarray          # n, float64
    x0: np.ndarray         # d, float64 (the planted signal)
    lam: float
    sigma: np.ndarray      # nominal singular values
    sd_target: float


def _haar_q(rng: np.random.Generator, d: int) -> np.ndarray:
    Z = rng.standard_normal((d, d))
    Q, R = np.linalg.qr(Z)
    return Q * np.sign(np.diag(R))[None, :]


def make_problem(n: int, d: int, sigma: np.ndarray, sd_target: float, seed: int,
                 a_dtype=np.float64, nrhs: int = 1) -> Problem:
    """Draw one dense problem on the host (numpy PCG64 stream `seed`)."""
    if len(sigma) != d:
        raise ValueError("sigma must have d entries")
    rng = np.random.default_rng(seed)
    Q = _haar_q(rng, d)
    G = rng.standard_normal((n, d)) / math.sqrt(n)
    A = (G * sigma[None, :]) @ Q
    del G
    if a_dtype == np.float32:
        A = A.astype(np.float32)
    A = np.ascontiguousarray(A)
    A64 = A.astype(np.float64, copy=False)
    shape = (d,) if nrhs == 1 else (d, nrhs)
    x0 = rng.standard_normal(shape) / math.sqrt(d)
    Ax0 = A64 @ x0
    noise_var = 1e-4 * float(np.sum(Ax0 * Ax0)) / (n * (1 if nrhs == 1 else nrhs))
    b = Ax0 + rng.standard_normal(Ax0.shape) * math.sqrt(noise_var)
    lam = lambda_for_sd(sigma, sd_target)
    return Problem(A=A, b=np.ascontiguousarray(b), x0=x0, lam=lam, sigma=sigma,
                   sd_target=sd_target)


def make_problem_torch(n: int, d: int, sigma: np.ndarray, sd_target: float, seed: int,
                       device, a_dtype: str = "f64", nrhs: int = 1):
    """Same recipe drawn on a device with torch's generator (for sizes where the
    host draw is too slow).  Returns (A, b, x0, lam) as torch tensors on `device`."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    sig = torch.as_tensor(sigma, dtype=torch.float64, device=device)
    Z = torch.randn(d, d, generator=g, dtype=torch.float64, device=device)
    Q, R = torch.linalg.qr(Z)
    Q = Q * torch.sign(torch.diagonal(R))[None, :]
    dt = torch.float64 if a_dtype == "f64" else torch.float32
    A = torch.empty(n, d, dtype=dt, device=device)
    blk = max(1, (1 << 27) // d)
    for r0 in range(0, n, blk):
        r1 = min(n, r0 + blk)
        G = torch.randn(r1 - r0, d, generator=g, dtype=torch.float64, device=device)
        G.mul_(sig[None, :] / math.sqrt(n))
        A[r0:r1] = (G @ Q).to(dt)
        del G
    shape = (d,) if nrhs == 1 else (d, nrhs)
    x0 = torch.randn(*shape, generator=g, dtype=torch.float64, device=device) / math.sqrt(d)
    Ax0 = torch.empty((n,) if nrhs == 1 else (n, nrhs), dtype=torch.float64, device=device)
    for r0 in range(0, n, blk):
        r1 = min(n, r0 + blk)
        Ax0[r0:r1] = A[r0:r1].to(torch.float64) @ x0
    noise_var = 1e-4 * float((Ax0 * Ax0).sum()) / (n * (1 if nrhs == 1 else nrhs))
    b = Ax0 + torch.randn(Ax0.shape, generator=g, dtype=torch.float64, device=device) * math.sqrt(noise_var)
    lam = lambda_for_sd(sigma, sd_target)
    return A, b.contiguous(), x0, lam


def make_dual_problem(n: int, d: int, sigma: np.ndarray, sd_target: float, seed: int,
                      a_dtype=np.float64):
    """Under-determined instance (n <= d) for Dual M-IHS: A^T = G diag(sigma) Q with
    G iid N(0,1)/sqrt(d) (d x n) and Q Haar (n x n) -- the tall recipe with the
    roles of n and d swapped -- x0 ~ N(0, 1/d), b = A x0 + 1% noise.
    Returns (At, b, lam) with At = A^T (d x n, row-major)."""
    P = make_problem(d, n, sigma, sd_target, seed, a_dtype)
    At = P.A
    rng = np.random.default_rng(seed + 7919)
    x0 = rng.standard_normal(d) / math.sqrt(d)
    Ax0 = At.astype(np.float64).T @ x0
    noise_var = 1e-4 * float(Ax0 @ Ax0) / n
    b = Ax0 + rng.standard_normal(n) * math.sqrt(noise_var)
    return At, b, P.lam


def make_dual_problem_torch(n: int, d: int, sigma: np.ndarray, sd_target: float, seed: int,
                            device, a_dtype: str = "f64"):
    """The same recipe drawn on a device (sizes where the host draw is slow).
    Returns (At, b, lam) as torch tensors on `device` (lam a float)."""
    import torch
    At, _, _, lam = make_problem_torch(d, n, sigma, sd_target, seed, device, a_dtype)
    g = torch.Generator(device=device)
    g.manual_seed(seed + 7919)
    x0 = torch.randn(d, generator=g, dtype=torch.float64, device=device) / math.sqrt(d)
    Ax0 = At.to(torch.float64).T @ x0
    noise_var = 1e-4 * float((Ax0 * Ax0).sum()) / n
    b = Ax0 + torch.randn(n, generator=g, dtype=torch.float64, device=device) * math.sqrt(noise_var)
    return At, b.contiguous(), lam


@dataclasses.dataclass
class Workload:
    name: str
    n: int
    d: int
    a_dtype: str            # "f64" or "f32"
    sigma_kind: str
    sigma_rate: float
    sd_target: float
    sketch: str             # "gaussian", "srht", "countsketch", "count_gauss"
    m: int
    m2: int = 0
    eps_sub: float = 1e-2
    data_seed: int = 0
    sketch_seed: int = 7
    nrhs: int = 1
    dual: bool = False      # under-determined (n <= d): Dual M-IHS on A^T

    @property
    def sigma(self) -> np.ndarray:
        return sigma_profile(self.sigma_kind, min(self.n, self.d), self.sigma_rate)

    @property
    def lam(self) -> float:
        return lambda_for_sd(self.sigma, self.sd_target)

    @property
    def m_out(self) -> int:
        """Rows of the sketch the solver sees (the second stage's, when there is one)."""
        return self.m2 if self.m2 else self.m

    def draw(self, n: Optional[int] = None) -> Problem:
        return make_problem(n or self.n, self.d, self.sigma, self.sd_target, self.data_seed,
                            np.float64 if self.a_dtype == "f64" else np.float32, self.nrhs)


# The workloads: a small one that the oracle finishes in seconds, the headline
# SRHT one, a CountSketch->Gaussian two-stage one with FP32 A, a batched
# lambda-path one (see batched_specs), a multi-RHS differentiation one and an
# under-determined one for Dual M-IHS.
WORKLOADS = {
    "small_gauss": Workload("small_gauss", 4096, 256, "f64", "exp", 6.0, 64.0, "gaussian", 256,
                            eps_sub=1e-8, data_seed=0, sketch_seed=7),
    # eps_sub = 0.1 is the paper's forcing term (Section 3.1); on this workload it keeps
    # the outer iteration count of eps_sub = 1e-2 with half the inner iterations.
    "srht_2p18x2048": Workload("srht_2p18x2048", 1 << 18, 2048, "f64", "exp", 8.0, 512.0, "srht",
                               2048, eps_sub=1e-1, data_seed=1000, sketch_seed=8),
    "count_2p20x4096": Workload("count_2p20x4096", 1 << 20, 4096, "f32", "poly", 1.5, 1024.0,
                                "count_gauss", 8192, m2=4096, eps_sub=1e-2, data_seed=2000,
                                sketch_seed=9),
    "diff_2p18x1024": Workload("diff_2p18x1024", 1 << 18, 1024, "f32", "exp", 8.0, 256.0, "srht",
                               1024, eps_sub=1e-2, data_seed=4000, sketch_seed=11, nrhs=64),
    # square-like, shaped like Figure 5's (max/min = 5e4/1e4, sd/min ~ 0.07, m1 = m2 = 8 sd)
    # within the 4096-column limit: Primal-Dual M-IHS (Algorithm 4), M = 25 dual steps
    "pd_16384x4096": Workload("pd_16384x4096", 1 << 14, 4096, "f64", "exp", 8.0, 256.0, "srht",
                              2048, m2=2048, eps_sub=1e-1, data_seed=6000, sketch_seed=13),
    # under-determined, shaped like Figure 4's (n, d, m, sd) = (4000, 2^16, 4000, 462)
    "dual_4096x2p16": Workload("dual_4096x2p16", 4096, 1 << 16, "f64", "exp", 8.0, 462.0, "srht",
                               4096, eps_sub=1e-1, data_seed=5000, sketch_seed=12, dual=True),
}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


@dataclasses.dataclass
class BatchedSpec:
    n: int
    d: int
    seed: int
    lambdas: np.ndarray     # 16 values, log grid over [1e-6, 1e-1] * sigma_1^2
    m: int                  # ceil(4 * sd(lambda_min)), nominal spectrum


def batched_specs(nprob: int = 256, nlam: int = 16, n_range=(4096, 65536),
                  d_range=(64, 512), size_seed: int = 3, base_seed: int = 3000) -> List[BatchedSpec]:
    """Sizes and lambda grids of the batched lambda-path workload: n_k and d_k
    integer-uniform (inclusive), sigma_i = exp(-6 i / d_k)."""
    rng = np.random.default_rng(size_seed)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=nprob)
    ds = rng.integers(d_range[0], d_range[1] + 1, size=nprob)
    out = []
    for k in range(nprob):
        d = int(ds[k])
        sig = sigma_profile("exp", d, 6.0)
        s1 = float(sig[0]) ** 2
        lams = s1 * 10.0 ** (-6.0 + 5.0 * np.arange(nlam) / (nlam - 1))
        m = int(math.ceil(4.0 * nominal_sd(sig, float(lams[0]))))
        out.append(BatchedSpec(n=int(ns[k]), d=d, seed=base_seed + k, lambdas=lams, m=m))
    return out
