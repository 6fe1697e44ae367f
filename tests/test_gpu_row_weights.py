"""Per-XCD row weights of the gradient pass on the GPU: the calibration sets
weights in [32, 64]; a solve with skewed weights reaches the same closed form as
with equal ones (only the grouping of the partial sums differs); the same
weights repeat the result bit for bit."""
import numpy as np
import pytest

import workloads as W
from oracle import sketches, solver as O
from gpu_common import announce, rel, requires_gpu, to_dev, torch

pytestmark = [pytest.mark.gpu, requires_gpu]


def test_calibrated_weights_are_in_range():
    import paper_1912_03514_amd as mihs
    announce("row weights: calibration")
    w = mihs.calibrate_rows()
    assert len(w) == 8 and max(w) == 64 and min(w) >= 32 and all(v % 4 == 0 for v in w), w
    assert mihs.row_weights() == w


@pytest.mark.parametrize("precision", ["plain", "mixed"])
def test_skewed_weights_reach_the_same_solution(precision):
    import paper_1912_03514_amd as mihs
    n, d, sd, m, seed = 1 << 15, 256, 64.0, 512, 71
    sig = W.sigma_profile("exp", d, 6.0)
    P = W.make_problem(n, d, sig, sd, seed)
    SA = sketches.gaussian_sketch(P.A, m, seed + 1)
    xs = O.ridge_lstsq(P.A, P.b, P.lam)
    A, b = to_dev(P.A), to_dev(P.b)
    SAd = to_dev(SA) if precision == "plain" else to_dev(SA.astype(np.float32))
    alpha, beta = mihs.momentum(sd, m)
    kw = dict(eps_sub=0.1, tol=1e-11, max_outer=300, max_inner=2000, precision=precision)
    saved = mihs.row_weights()
    try:
        res = {}
        for name, w in (("equal", None), ("skewed", [64, 32, 48, 63, 40, 64, 33, 50])):
            mihs.set_row_weights(w)
            announce(f"row weights {name}, {precision}: n={n} d={d} m={m}")
            x1, i1 = mihs.mihs_solve(A, b, P.lam, SAd, alpha, beta, **kw)
            x2, i2 = mihs.mihs_solve(A, b, P.lam, SAd, alpha, beta, **kw)
            assert i1["status"] == 0 and i2["status"] == 0, (i1, i2)
            assert torch.equal(x1, x2)
            res[name] = (x1.cpu().numpy(), i1)
        for name, (x, info) in res.items():
            assert rel(x, xs) <= 1e-10, (name, rel(x, xs))
        assert abs(res["equal"][1]["outer_iters"] - res["skewed"][1]["outer_iters"]) <= 1
        assert rel(res["skewed"][0], res["equal"][0]) <= 1e-10
    finally:
        mihs.set_row_weights(list(saved))
