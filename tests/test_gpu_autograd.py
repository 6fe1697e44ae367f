"""GPU parity: the multi-RHS forward and the autograd backward (adjoint M-IHS)
against the dense oracle and central finite differences."""
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


def _setup(n=3000, d=100, k=20, adt=np.float64, seed=13):
    sig = W.sigma_profile("exp", d, 8.0)
    P = W.make_problem(n, d, sig, 25.0, seed, adt)
    A64 = P.A.astype(np.float64)
    m = 4 * 25
    m = max(m, 128)
    SA = sketches.gaussian_sketch(A64, m, 5)
    a, b = O.momentum_cor4(25.0, m)
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((n, k))
    return P, A64, SA, a, b, B, m


@pytest.mark.parametrize("adt,k", [(np.float64, 20), (np.float32, 16), (np.float64, 1)])
def test_multi_rhs_forward(adt, k):
    mihs = _mihs()
    P, A64, SA, a, b, B, m = _setup(adt=adt, k=k)
    ref = O.ridge_cholesky(A64, B, P.lam)
    announce(f"multi-rhs forward k={k} {adt.__name__}")
    X, infos = mihs.mihs_solve_multi(to_dev(P.A), to_dev(B), P.lam, to_dev(SA), a, b,
                                     eps_sub=1e-3, tol=1e-13, max_outer=500)
    assert all(i["status"] == 0 for i in infos)
    assert rel(X.cpu().numpy(), ref) <= 1e-10


def test_autograd_matches_dense_and_finite_differences():
    mihs = _mihs()
    P, A64, SA, a, b, B, m = _setup(n=2000, d=64, k=16)
    rng = np.random.default_rng(2)
    C = rng.standard_normal((32, 64))
    Y = rng.standard_normal((32, 16))
    kw = dict(eps_sub=1e-6, tol=1e-15, max_outer=800)
    Ad, SAd, Ct, Yt = to_dev(P.A), to_dev(SA), to_dev(C), to_dev(Y)

    def loss(Bt, ll):
        X = mihs.MIHSRidge.apply(Bt, ll, Ad, SAd, a, b, kw)
        return ((Ct @ X - Yt) ** 2).sum()

    Bt = to_dev(B).requires_grad_(True)
    ll = torch.tensor(math.log(P.lam), dtype=torch.float64, device="cuda", requires_grad=True)
    announce("autograd backward")
    L = loss(Bt, ll)
    L.backward()
    dB = Bt.grad.cpu().numpy()
    dll = float(ll.grad.cpu())
    # dense FP64 gradient
    Xs = O.ridge_cholesky(A64, B, P.lam)
    gbar = 2 * C.T @ (C @ Xs - Y)
    _, dBref, dlref = O.ridge_backward_dense(A64, P.lam, Xs, gbar)
    assert rel(dB, dBref) <= 1e-8
    assert abs(dll - P.lam * dlref) <= 1e-8 * abs(P.lam * dlref)
    # central finite differences of the GPU forward, h = 1e-6 (L is quadratic in B)
    h = 1e-6
    with torch.no_grad():
        for t in range(2):
            V = to_dev(rng.standard_normal(B.shape))
            fd = (float(loss(to_dev(B) + h * V, ll)) - float(loss(to_dev(B) - h * V, ll))) / (2 * h)
            an = float((to_dev(dB) * V).sum())
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (t, fd, an)
        fd = (float(loss(to_dev(B), ll + h)) - float(loss(to_dev(B), ll - h))) / (2 * h)
        assert abs(fd - dll) <= 1e-6 * max(1.0, abs(dll))
