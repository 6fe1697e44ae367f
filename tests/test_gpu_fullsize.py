"""GPU parity at the benchmark's full sizes, in the launch configuration that
bench.py times: the same seeded inputs (drawn on the device), the same sketch
and solve calls and parameters.  Expected values: the oracle's closed forms on
the host where they finish in seconds, else the refined closed form of
gpu_common (torch FP64 + long-double refinement, independent of the library)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import solver as O
from gpu_common import (announce, closed_form_refined, dev, rel, requires_gpu,
                        ridge_path_closed_form, torch)

pytestmark = [pytest.mark.gpu, requires_gpu]


def _mihs():
    import paper_1912_03514_amd as mihs
    return mihs


@pytest.fixture(scope="module")
def srht_problem():
    w = W.workload("srht_2p18x2048")
    announce("full-size SRHT workload: draw + host closed form")
    A, b, _, lam = W.make_problem_torch(w.n, w.d, w.sigma, w.sd_target, w.data_seed, dev(),
                                        w.a_dtype)
    xs = O.ridge_cholesky(A.cpu().numpy(), b.cpu().numpy(), lam)
    yield w, A, b, lam, xs
    del A, b
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["mixed", "plain"])
def test_fullsize_srht_solve(srht_problem, prec):
    """2^18 x 2048 FP64, SRHT m = 2048, eps_sub = 0.1, stop tol 5e-11."""
    mihs = _mihs()
    w, A, b, lam, xs = srht_problem
    alpha, beta = mihs.momentum(w.sd_target, w.m_out)
    announce(f"full-size SRHT solve ({prec})")
    SA = mihs.mihs_sketch(A, w.sketch, w.m, w.sketch_seed, precision=prec)
    x, info = mihs.mihs_solve(A, b, lam, SA, alpha, beta, eps_sub=w.eps_sub, tol=5e-11,
                              max_outer=300, max_inner=2000, precision=prec)
    assert info["status"] == 0, info
    assert rel(x.cpu().numpy(), xs) <= 1e-10


@pytest.fixture(scope="module")
def count_problem():
    w = W.workload("count_2p20x4096")
    announce("full-size CountSketch workload: draw + refined closed form")
    A, b, _, lam = W.make_problem_torch(w.n, w.d, w.sigma, w.sd_target, w.data_seed, dev(),
                                        w.a_dtype)
    xs = closed_form_refined(A, b, lam)
    torch.cuda.empty_cache()
    yield w, A, b, lam, xs
    del A, b
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", ["plain", "mixed"])
def test_fullsize_countsketch_solve(count_problem, prec):
    """2^20 x 4096 FP32 A (kappa ~ 6e8), CountSketch 8192 -> Gaussian 4096; the
    reference is refined in extended precision (FP64 normal equations alone are
    off by ~1e-8 here)."""
    mihs = _mihs()
    w, A, b, lam, xs = count_problem
    alpha, beta = mihs.momentum(w.sd_target, w.m_out)
    announce(f"full-size CountSketch solve ({prec})")
    SA = mihs.mihs_sketch(A, w.sketch, w.m, w.sketch_seed, precision=prec, m2=w.m2)
    x, info = mihs.mihs_solve(A, b, lam, SA, alpha, beta, eps_sub=w.eps_sub, tol=2e-12,
                              max_outer=400, max_inner=2000, precision=prec)
    assert info["status"] == 0, info
    assert rel(x.cpu().numpy(), xs) <= 1e-10


def _batched_full_set(precision="mixed"):
    """The benchmark's batched workload: 256 problems x 16 lambdas, one Gaussian
    sketch per problem, Corollary 4 momentum per lambda."""
    mihs = _mihs()
    specs = W.batched_specs()
    probs, lam_rows, al_rows, be_rows = [], [], [], []
    for i, s in enumerate(specs):
        sig = W.sigma_profile("exp", s.d, 6.0)
        A, b, _, _ = W.make_problem_torch(s.n, s.d, sig, s.d / 2, s.seed, dev(), "f64")
        SA = mihs.mihs_sketch(A, "gaussian", s.m, 10 + i, precision=precision)
        probs.append((A, b, SA))
        sds = np.array([W.nominal_sd(sig, float(l)) for l in s.lambdas])
        be = np.minimum(sds / s.m, 0.95)
        lam_rows.append(s.lambdas)
        al_rows.append((1.0 - be) ** 2)
        be_rows.append(be)
    return probs, lam_rows, al_rows, be_rows


def _check_every_result(probs, lam_rows, xs, infos, refs, what):
    """Every (problem, lambda) result against its closed form: status converged
    and relative error <= 1e-10, all 4096 of them."""
    errs, bad_status = [], []
    for i, (A, b, _) in enumerate(probs):
        X = xs[i].cpu().numpy()
        for j in range(len(lam_rows[i])):
            if infos[i][j]["status"] != 0:
                bad_status.append((i, j, infos[i][j]["status"]))
            errs.append((rel(X[:, j], refs[i][:, j]), i, j))
    errs.sort(reverse=True)
    over = [e for e in errs if e[0] > 1e-10]
    print(f"{what}: worst relative errors over all {len(errs)} results {errs[:3]}; "
          f"{len(over)} above 1e-10; status != 0: {bad_status[:5]}", flush=True)
    assert not bad_status, bad_status[:5]
    assert not over, over[:5]


@pytest.fixture(scope="module")
def batched_full():
    announce("full-size batched: draw 256 problems + mixed sketches")
    probs, lam_rows, al_rows, be_rows = _batched_full_set("mixed")
    announce("full-size batched: QR closed forms of all 4096 (problem, lambda) pairs")
    refs = [ridge_path_closed_form(A, b, lam_rows[i]) for i, (A, b, _) in enumerate(probs)]
    yield probs, lam_rows, al_rows, be_rows, refs
    del probs
    torch.cuda.empty_cache()


def test_fullsize_batched_lambda_paths(batched_full):
    """256 problems x 16 lambdas (n in [4096, 65536], d in [64, 512]) with mixed
    Gaussian sketches in one launch, with the default shape and with the
    autotuned plan the benchmark times (inexact inner CG, teams sized from
    measured costs): every one of the 4096 results against its QR closed form."""
    mihs = _mihs()
    probs, lam_rows, al_rows, be_rows, refs = batched_full
    T = lambda a: torch.as_tensor(np.array(a), device=dev())
    announce("full-size batched: solve (default shape)")
    xs, infos = mihs.mihs_solve_batched(probs, T(lam_rows), T(al_rows), T(be_rows),
                                        eps_sub=0.1, tol=3e-12, max_outer=400, max_inner=2000)
    _check_every_result(probs, lam_rows, xs, infos, refs, "default shape")
    announce("full-size batched: autotuned plan (inexact CG)")
    s = mihs.BatchedSolver(probs, T(lam_rows), T(al_rows), T(be_rows), eps_sub=0.1, tol=3e-12,
                           max_outer=400, max_inner=2000)
    tuned = s.tune(trial_outer=8)
    print(f"full-size batched tuning: {tuned['best']}")
    assert tuned["best"]["exact"] == 0
    s.run()
    torch.cuda.synchronize()
    _check_every_result(probs, lam_rows, s.xs, s.infos(), refs, "tuned CG plan")
    s.close()


def test_fullsize_batched_exact_subsolves(batched_full):
    """The same workload with exact sub-solves allowed (Exact M-IHS, Table 2):
    the tuner's choice, every result against its QR closed form."""
    mihs = _mihs()
    probs, lam_rows, al_rows, be_rows, refs = batched_full
    T = lambda a: torch.as_tensor(np.array(a), device=dev())
    announce("full-size batched: autotuned plan (exact allowed)")
    s = mihs.BatchedSolver(probs, T(lam_rows), T(al_rows), T(be_rows), eps_sub=0.1, tol=3e-12,
                           max_outer=400, max_inner=2000)
    tuned = s.tune(trial_outer=8, allow_exact=True)
    print(f"full-size batched tuning (exact allowed): {tuned['best']}")
    s.run()
    torch.cuda.synchronize()
    _check_every_result(probs, lam_rows, s.xs, s.infos(), refs, "tuned plan, exact allowed")
    s.close()


def test_fullsize_differentiation():
    """2^18 x 1024 FP32 A, 64 right-hand sides: forward and adjoint backward of
    L = sum ||C x*_j - y_j||^2 against the oracle's dense FP64 gradient."""
    mihs = _mihs()
    w = W.workload("diff_2p18x1024")
    announce("full-size differentiation: draw")
    A, B, _, lam = W.make_problem_torch(w.n, w.d, w.sigma, w.sd_target, w.data_seed, dev(),
                                        w.a_dtype, nrhs=w.nrhs)
    g = torch.Generator(device=dev()).manual_seed(w.data_seed + 1)
    C = torch.randn(128, w.d, generator=g, dtype=torch.float64, device=dev())
    Y = torch.randn(128, w.nrhs, generator=g, dtype=torch.float64, device=dev())
    alpha, beta = mihs.momentum(w.sd_target, w.m_out)
    kw = dict(eps_sub=w.eps_sub, tol=1e-12, max_outer=300)
    announce("full-size differentiation: forward + backward")
    SA = mihs.mihs_sketch(A, "srht", w.m, w.sketch_seed)
    Bt = B.clone().requires_grad_(True)
    ll = torch.tensor(math.log(lam), dtype=torch.float64, device=dev(), requires_grad=True)
    X = mihs.MIHSRidge.apply(Bt, ll, A, SA, alpha, beta, kw)
    L = ((C @ X - Y) ** 2).sum()
    L.backward()
    A64 = A.double().cpu().numpy()
    Xs = O.ridge_cholesky(A64, B.cpu().numpy(), lam)
    gbar = 2 * C.cpu().numpy().T @ (C.cpu().numpy() @ Xs - Y.cpu().numpy())
    _, dBref, dlref = O.ridge_backward_dense(A64, lam, Xs, gbar)
    assert rel(X.detach().cpu().numpy(), Xs) <= 1e-10
    assert rel(Bt.grad.cpu().numpy(), dBref) <= 1e-10
    assert abs(float(ll.grad) - lam * dlref) <= 1e-10 * abs(lam * dlref)

    # central differences with h = 1e-6 in FP64 at the full size, on dense
    # forward solves (torch Gram matrix + Cholesky on the device, not the
    # library): along three random directions V of B, and in log(lambda).  L is
    # quadratic in B, so the B differences are exact up to rounding; in
    # log(lambda) the truncation error is O(h^2).  The difference of the two
    # losses is formed as sum (r+ - r-)(r+ + r-) over the residuals
    # r = C X - Y of the two solves (the same number as L(+) - L(-), without
    # the cancellation that would leave u L / h ~ 1e-6 of rounding noise).
    announce("full-size differentiation: central differences")
    Ad = A.double()
    Hg = Ad.T @ Ad
    eye = torch.eye(w.d, dtype=torch.float64, device=dev())

    def residual(Bm, lam_):
        Lc = torch.linalg.cholesky(Hg + lam_ * eye)
        return C @ torch.cholesky_solve(Ad.T @ Bm, Lc) - Y

    def central(rp, rm):
        return float(((rp - rm) * (rp + rm)).sum()) / (2 * h)

    # Directions: the reference gradient weighted entrywise by random factors in
    # [0.5, 1.5), three draws.  Along a plain random direction <dL/dB, V> is a sum
    # with heavy cancellation (~2 against terms of ~1e3 here), and no FP64
    # difference quotient resolves it to 1e-6; these directions keep the
    # directional derivative of the size of its terms.
    h = 1e-6
    gv = torch.Generator(device=dev()).manual_seed(77)
    dBref_d = torch.as_tensor(dBref, device=dev())
    for t in range(3):
        wts = 0.5 + torch.rand(B.shape, generator=gv, dtype=torch.float64, device=dev())
        V = dBref_d * wts
        V = V * (B.norm() / V.norm())
        fd = central(residual(B + h * V, lam), residual(B - h * V, lam))
        an = float((Bt.grad * V).sum())
        ref = float((dBref_d * V).sum())
        print(f"FD direction {t}: analytic {an:.12e}, dense {ref:.12e}, central difference "
              f"{fd:.12e}", flush=True)
        assert abs(an - fd) <= 1e-6 * abs(fd), (t, an, fd)
    ll0 = math.log(lam)
    fd = central(residual(B, math.exp(ll0 + h)), residual(B, math.exp(ll0 - h)))
    print(f"FD log(lambda): analytic {float(ll.grad):.12e}, central difference {fd:.12e}",
          flush=True)
    assert abs(float(ll.grad) - fd) <= 1e-6 * abs(fd)
