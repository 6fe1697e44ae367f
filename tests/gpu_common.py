"""Shared helpers for the GPU parity tests (inputs come from `workloads`,
expected values from `oracle`)."""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

requires_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")


def dev():
    return torch.device("cuda", 0)


def to_dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev())


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def announce(msg):
    """Name the case before any GPU work, flushed, so a fault is attributable."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def closed_form_refined(A, b, lam, refine=2, chunk=1 << 16):
    """x* = (A^T A + lam I)^{-1} A^T b for device tensors too large for the host
    oracle: FP64 Gram matrix and Cholesky with torch (rocBLAS/rocSOLVER, not the
    library under test), then `refine` steps of iterative refinement whose
    gradients A^T (b - A x) - lam x are accumulated on the host in long double.
    Returns a host FP64 vector."""
    n, d = A.shape
    H = torch.zeros(d, d, dtype=torch.float64, device=A.device)
    Atb = torch.zeros(d, dtype=torch.float64, device=A.device)
    for r0 in range(0, n, chunk):
        Ac = A[r0:r0 + chunk].double()
        H += Ac.T @ Ac
        Atb += Ac.T @ b[r0:r0 + chunk]
        del Ac
    H += lam * torch.eye(d, dtype=torch.float64, device=A.device)
    L = torch.linalg.cholesky(H)
    del H
    x = torch.cholesky_solve(Atb[:, None], L)[:, 0]
    rows = 1 << 14
    for _ in range(refine):
        r = torch.empty(n, dtype=torch.float64, device=A.device)
        for r0 in range(0, n, chunk):
            r[r0:r0 + chunk] = b[r0:r0 + chunk] - A[r0:r0 + chunk].double() @ x
        rh = r.cpu().numpy().astype(np.longdouble)
        atr = np.zeros(d, dtype=np.longdouble)
        for r0 in range(0, n, rows):
            Ac = A[r0:r0 + rows].cpu().numpy().astype(np.longdouble)
            atr += Ac.T @ rh[r0:r0 + rows]
        g = atr - np.longdouble(lam) * x.cpu().numpy().astype(np.longdouble)
        x = x + torch.cholesky_solve(torch.from_numpy(g.astype(np.float64)).to(A.device)[:, None],
                                     L)[:, 0]
    return x.cpu().numpy()


def ridge_path_closed_form(A, b, lams):
    """x*_j = argmin ||A x - b||^2 + lam_j ||x||^2 for every lam_j, on the device
    with torch (rocSOLVER Householder QR, not the library under test): A = Q R,
    then for each lambda the small stacked problem [R; sqrt(lam_j) I] x ~ [Q^T b; 0]
    by a second QR and a triangular solve.  Backward stable: the error is about
    u kappa([A; sqrt(lam) I]) (plus u kappa^2 times the relative residual), far
    below the 1e-10 checked, where normal equations would give u kappa(A^T A).
    Returns a host d x len(lams) FP64 array."""
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
    y = Q2.transpose(1, 2).contiguous() @ rhs
    x = torch.linalg.solve_triangular(R2, y, upper=True)
    return x[:, :, 0].transpose(0, 1).contiguous().cpu().numpy()
