"""GPU: the batched solve as a plan + launch (graph capture, repeated runs) and the
launch-shape autotuner, against the oracle's closed form."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import sketches, solver as O
from gpu_common import announce, rel, requires_gpu, to_dev, torch

pytestmark = [pytest.mark.gpu, requires_gpu]

# ragged d across every padded width (64 ... 512) and a ragged last row tile
SHAPES = [(1500, 70), (3001, 130), (2500, 17), (4000, 300), (5000, 200), (2100, 500)]
NLAM = 16


def _mihs():
    import paper_1912_03514_amd as mihs
    return mihs


@pytest.fixture(scope="module")
def problem_set():
    problems, refs, L, Al, Be = [], [], [], [], []
    for i, (n, d) in enumerate(SHAPES):
        sig = W.sigma_profile("exp", d, 6.0)
        P = W.make_problem(n, d, sig, d / 4, 700 + i)
        m = min(n, 4 * d)
        SA = sketches.gaussian_sketch(P.A, m, 60 + i)
        s1 = float(sig[0]) ** 2
        lams = s1 * 10.0 ** (-6.0 + 5.0 * np.arange(NLAM) / (NLAM - 1))
        sds = np.array([W.nominal_sd(sig, float(l)) for l in lams])
        betas = np.minimum(sds / m, 0.95)
        problems.append((P.A, P.b, SA))
        refs.append([O.ridge_lstsq(P.A, P.b, float(l)) for l in lams])
        L.append(lams)
        Al.append((1.0 - betas) ** 2)
        Be.append(betas)
    return problems, refs, np.array(L), np.array(Al), np.array(Be)


def _device_set(problem_set):
    problems, refs, L, Al, Be = problem_set
    dp = [(to_dev(A), to_dev(b), to_dev(SA)) for A, b, SA in problems]
    return dp, refs, to_dev(L), to_dev(Al), to_dev(Be)


def _check_closed_form(xs, infos, refs, tol=1e-10):
    for i, X in enumerate(xs):
        Xh = X.cpu().numpy()
        for j in range(NLAM):
            assert infos[i][j]["status"] == 0, (i, j, infos[i][j])
            assert rel(Xh[:, j], refs[i][j]) <= tol, (i, j, rel(Xh[:, j], refs[i][j]))


@pytest.mark.parametrize("tuning", [
    {"cg_cols": 32, "a_dma": 1, "inner_weight": 100.0},
    {"cg_cols": 16, "a_dma": 0, "inner_weight": 25.0},
    {"cg_cols": 64, "a_dma": 1, "inner_weight": 400.0},
    {"cg_cols": 32, "a_dma": 0, "inner_weight": 400.0},
    {"cg_cols": 512, "a_dma": 1, "inner_weight": 6.25},
    {"cg_cols": 32, "a_dma": 1, "inner_weight": 25.0, "exact": 1},
    {"cg_cols": 32, "a_dma": 0, "inner_weight": 6.25, "exact": 1},
])
def test_every_launch_shape_reaches_the_closed_form(problem_set, tuning):
    """Each candidate shape of the autotuner (CG sub-team width, the A pass
    through registers or direct-to-LDS, team sizing, inexact CG or exact
    Cholesky sub-solves) solves every (problem, lambda) to 1e-10."""
    mihs = _mihs()
    dp, refs, L, Al, Be = _device_set(problem_set)
    announce(f"batched plan shape {tuning}")
    s = mihs.BatchedSolver(dp, L, Al, Be, eps_sub=1e-2, tol=1e-12, max_outer=800,
                           max_inner=2000, tuning=tuning)
    s.run()
    torch.cuda.synchronize()
    infos = s.infos()
    _check_closed_form(s.xs, infos, refs)
    assert all(r["elapsed_us"] > 0 for inf in infos for r in inf)
    if tuning.get("exact"):
        # one exact sub-solve per outer step
        assert all(1 <= r["inner_iters_total"] <= r["outer_iters"] for inf in infos for r in inf)
        assert all(r["inner_iters_max"] == 1 for inf in infos for r in inf)


@pytest.mark.parametrize("cg_cols,exact", [(32, 0), (512, 0), (32, 1)])
def test_graph_replays_match_the_eager_run(problem_set, cg_cols, exact):
    """The launch captured in a HIP graph (with the Cholesky factor kernel when
    the sub-solves are exact), replayed three times with other eager work (and
    garbage in X) between the replays, gives bit-identical results to the eager
    launch of the same plan: the team CG (32 columns per workgroup, R and Z
    handed between workgroups at every step), the one-workgroup CG (512) and
    the exact sub-solves."""
    mihs = _mihs()
    dp, refs, L, Al, Be = _device_set(problem_set)
    s = mihs.BatchedSolver(dp, L, Al, Be, eps_sub=1e-2, tol=1e-12, max_outer=800,
                           max_inner=2000,
                           tuning={"cg_cols": cg_cols, "a_dma": 1, "inner_weight": 100.0,
                                   "exact": exact})
    announce("batched plan eager run")
    s.run()
    torch.cuda.synchronize()
    X_eager = s.X_all.clone()
    it_eager = [[r["outer_iters"] for r in inf] for inf in s.infos()]
    _check_closed_form(s.xs, s.infos(), refs)
    announce("batched plan graph capture")
    g = s.capture()
    for rep in range(3):
        s.X_all.fill_(float("nan"))
        s.info_all.fill_(0)
        junk = torch.randn(1 << 20, device=s.dev, dtype=torch.float64).sum()
        torch.cuda.synchronize()
        announce(f"batched plan graph replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(s.X_all, X_eager), rep
        assert [[r["outer_iters"] for r in inf] for inf in s.infos()] == it_eager, rep
        assert bool(torch.isfinite(junk))


def test_autotuner_picks_a_candidate_and_the_handle_keeps_it(problem_set):
    """mihs_tune_batched with exact sub-solves allowed times ten candidate
    shapes by coordinate descent, full runs of the best inexact and the best
    exact shape, and a schedule sized from the faster one's per-problem costs
    (an inexact one also with 64 columns per CG member), then up to three
    times more from the costs measured under the best of those while that
    gains, and keeps the best for this problem set: the plain batched call afterwards
    (which looks the shape up) still reaches the closed form, and so does a plan
    that asks for the measured schedule explicitly."""
    mihs = _mihs()
    dp, refs, L, Al, Be = _device_set(problem_set)
    s = mihs.BatchedSolver(dp, L, Al, Be, eps_sub=1e-2, tol=1e-12, max_outer=800,
                           max_inner=2000)
    announce("batched autotuner")
    res = s.tune(trial_outer=3, allow_exact=True)
    best = res["best"]
    assert 13 <= len(res["trial_ms"]) <= 16
    assert all(t > 0 for t in res["trial_ms"])
    assert best["cg_cols"] in (16, 32, 64, 128, 512) and best["a_dma"] in (0, 1)
    assert best["inner_weight"] in (6.25, 25.0, 100.0, 400.0)
    assert best["measured"] in (0, 1) and best["exact"] in (0, 1)
    s.run()
    torch.cuda.synchronize()
    _check_closed_form(s.xs, s.infos(), refs)
    announce("batched call after tuning")
    xs, infos = mihs.mihs_solve_batched(dp, L, Al, Be, eps_sub=1e-2, tol=1e-12, max_outer=800,
                                        max_inner=2000)
    _check_closed_form(xs, infos, refs)
    announce("batched plan on the measured schedule")
    m = mihs.BatchedSolver(dp, L, Al, Be, eps_sub=1e-2, tol=1e-12, max_outer=800, max_inner=2000,
                           tuning=dict(best, measured=1))
    m.run()
    torch.cuda.synchronize()
    _check_closed_form(m.xs, m.infos(), refs)


def test_plan_rejects_bad_tuning(problem_set):
    mihs = _mihs()
    dp, refs, L, Al, Be = _device_set(problem_set)
    with pytest.raises(mihs.MihsError):
        mihs.BatchedSolver(dp, L, Al, Be, tuning={"cg_cols": 48, "a_dma": 1,
                                                  "inner_weight": 100.0})


def test_measured_schedule_with_more_entries_than_workgroups():
    """600 entries (300 small problems x 20 lambdas, i.e. two column groups each)
    on the GPU's workgroups: the tuner's measured schedule packs many entries per
    bin; after tuning, a graph replay of the plan reaches the closed form on a
    sample of problems and lambdas."""
    mihs = _mihs()
    rng = np.random.default_rng(11)
    nlam = 20
    problems, L, Al, Be, refs = [], [], [], [], {}
    for i in range(300):
        d = int(rng.integers(8, 96))
        n = int(rng.integers(max(d, 200), 900))
        sig = W.sigma_profile("exp", d, 6.0)
        P = W.make_problem(n, d, sig, max(1.0, d / 4), 900 + i)
        m = min(n, 4 * d)
        SA = sketches.gaussian_sketch(P.A, m, 40 + i)
        s1 = float(sig[0]) ** 2
        lams = s1 * 10.0 ** (-6.0 + 5.0 * np.arange(nlam) / (nlam - 1))
        sds = np.array([W.nominal_sd(sig, float(l)) for l in lams])
        betas = np.minimum(sds / m, 0.95)
        problems.append((to_dev(P.A), to_dev(P.b), to_dev(SA)))
        L.append(lams)
        Al.append((1.0 - betas) ** 2)
        Be.append(betas)
        if i % 37 == 0:
            refs[i] = (P, lams)
    s = mihs.BatchedSolver(problems, to_dev(np.array(L)), to_dev(np.array(Al)),
                           to_dev(np.array(Be)), eps_sub=1e-2, tol=1e-12, max_outer=800,
                           max_inner=2000)
    announce("batched 300 problems: tuner with measured schedule")
    res = s.tune(trial_outer=3)
    # inexact shapes only (the default): eight short trials, one full run of
    # the best, runs of the measured schedule (with the best shape's CG width,
    # with 64 columns per CG member unless that is the same, and up to three
    # times re-sized from the costs measured under the best); exact sub-solves
    # never chosen
    assert 10 <= len(res["trial_ms"]) <= 14
    assert res["best"]["exact"] == 0
    g = s.capture()
    s.X_all.fill_(float("nan"))
    torch.cuda.synchronize()
    announce("batched 300 problems: graph replay")
    g.replay()
    torch.cuda.synchronize()
    infos = s.infos()
    for i, (P, lams) in refs.items():
        X = s.xs[i].cpu().numpy()
        for j in (0, 9, 19):
            assert infos[i][j]["status"] == 0, (i, j, infos[i][j])
            assert rel(X[:, j], O.ridge_lstsq(P.A, P.b, float(lams[j]))) <= 1e-10, (i, j)


@pytest.mark.parametrize("k", [1, 3])
def test_exact_subsolves_follow_the_oracle_trajectory(problem_set, k):
    """Exact sub-solves (Exact M-IHS): after k outer steps from x = 0 every
    column equals the oracle's M-IHS with a Cholesky sub-solve after k steps.
    The bound allows for the conditioning of the sub-problems (kappa up to 1e6
    at lambda = 1e-6 sigma_1^2, where two FP64 Cholesky solves may differ by
    up to kappa d u in the worst direction; measured differences are ~3e-11),
    far below the O(1) change of one step."""
    mihs = _mihs()
    problems, refs, L, Al, Be = problem_set
    dp, _, Ld, Ald, Bed = _device_set(problem_set)
    s = mihs.BatchedSolver(dp, Ld, Ald, Bed, eps_sub=1e-2, tol=0.0, max_outer=k, max_inner=2000,
                           tuning={"cg_cols": 32, "a_dma": 1, "inner_weight": 25.0, "exact": 1})
    announce(f"batched exact sub-solves, {k} outer steps")
    s.run()
    torch.cuda.synchronize()
    infos = s.infos()
    worst = 0.0
    for i, (A, b, SA) in enumerate(problems):
        X = s.xs[i].cpu().numpy()
        for j in range(0, NLAM, 5):
            assert infos[i][j]["outer_iters"] == k, (i, j, infos[i][j])
            ref = O.mihs(A, b, float(L[i, j]), SA, float(Al[i, j]), float(Be[i, j]),
                         inner="exact", n_iter=k).x
            e = rel(X[:, j], ref)
            worst = max(worst, e)
            assert e <= 1e-9, (i, j, e)
    print(f"exact trajectory after {k} steps: worst relative difference {worst:.2e}")


def test_exact_falls_back_to_the_cg_when_a_factorization_fails():
    """A Gram matrix whose FP32 rounding outweighs lambda (A of rank d - 8, an FP32
    sketch, lambda ~ 1e-12 ||H||: the near-null eigenvalues of the rounded H are
    ~1e-4 of either sign against lambda ~ 1e-9) meets a non-positive Cholesky
    pivot; such a problem runs the inexact CG instead.  With teams of one
    workgroup (300 problems) both plans then run the same one-workgroup CG, so
    the exact plan must equal the inexact one bit for bit, with CG step counts."""
    mihs = _mihs()
    rng = np.random.default_rng(5)
    nlam, problems, lams = 4, [], []
    for i in range(300):
        n, d = 600, 48
        Bm = rng.standard_normal((n, d - 8))
        A = np.hstack([Bm, Bm[:, :8] @ rng.standard_normal((8, 8))])
        b = rng.standard_normal(n)
        SA = sketches.gaussian_sketch(A, 2 * d, 100 + i).astype(np.float32)
        hn = float(np.linalg.norm(SA.astype(np.float64).T @ SA.astype(np.float64), 2))
        problems.append((to_dev(A), to_dev(b), torch.as_tensor(SA, device="cuda")))
        lams.append(hn * 1e-12 * (1.0 + np.arange(nlam)))
    L = to_dev(np.array(lams))
    Al = to_dev(np.full((300, nlam), 0.5))
    Be = to_dev(np.full((300, nlam), 0.2))
    runs = {}
    for exact in (0, 1):
        s = mihs.BatchedSolver(problems, L, Al, Be, eps_sub=1e-2, tol=0.0, max_outer=4,
                               max_inner=200, tuning={"cg_cols": 512, "a_dma": 1,
                                                      "inner_weight": 6.25, "exact": exact})
        announce(f"batched rank-deficient set, exact={exact}")
        s.run()
        torch.cuda.synchronize()
        runs[exact] = (s.X_all.clone(), s.infos())
    assert torch.equal(torch.nan_to_num(runs[0][0], nan=7.0), torch.nan_to_num(runs[1][0], nan=7.0))
    assert [[r["inner_iters_total"] for r in inf] for inf in runs[0][1]] == \
        [[r["inner_iters_total"] for r in inf] for inf in runs[1][1]]
    assert max(r["inner_iters_max"] for inf in runs[1][1] for r in inf) > 1


@pytest.mark.parametrize("sa_f32", [False, True])
def test_exact_subsolves_at_the_widest_padding(sa_f32):
    """Exact sub-solves with d above 512 (the 1024-wide layout: factors of up to
    1024 x 1024, the widest LDS panel) and 20 lambdas (entries of 16 and of 4
    columns), FP64 and FP32 Gram matrices: every (problem, lambda) reaches the
    closed form, one sub-solve per outer step."""
    mihs = _mihs()
    nlam = 20
    problems, refs, L, Al, Be = [], [], [], [], []
    for i, (n, d) in enumerate([(3000, 700), (2600, 1000)]):
        sig = W.sigma_profile("exp", d, 5.0)
        P = W.make_problem(n, d, sig, d / 4, 1300 + i)
        m = min(n, 2 * d)
        SA = sketches.gaussian_sketch(P.A, m, 70 + i)
        s1 = float(sig[0]) ** 2
        lams = s1 * 10.0 ** (-5.0 + 4.0 * np.arange(nlam) / (nlam - 1))
        sds = np.array([W.nominal_sd(sig, float(l)) for l in lams])
        betas = np.minimum(sds / m, 0.95)
        SAd = torch.as_tensor(SA.astype(np.float32), device="cuda") if sa_f32 else to_dev(SA)
        problems.append((to_dev(P.A), to_dev(P.b), SAd))
        refs.append((P, lams))
        L.append(lams)
        Al.append((1.0 - betas) ** 2)
        Be.append(betas)
    s = mihs.BatchedSolver(problems, to_dev(np.array(L)), to_dev(np.array(Al)),
                           to_dev(np.array(Be)), eps_sub=1e-2, tol=1e-12, max_outer=800,
                           max_inner=2000,
                           tuning={"cg_cols": 32, "a_dma": 1, "inner_weight": 25.0, "exact": 1})
    announce(f"batched exact sub-solves, d = 700 and 1000, sa_f32={sa_f32}")
    s.run()
    torch.cuda.synchronize()
    infos = s.infos()
    for i, (P, lams) in enumerate(refs):
        X = s.xs[i].cpu().numpy()
        for j in range(nlam):
            assert infos[i][j]["status"] == 0, (i, j, infos[i][j])
            assert infos[i][j]["inner_iters_max"] == 1, (i, j, infos[i][j])
            assert rel(X[:, j], O.ridge_lstsq(P.A, P.b, float(lams[j]))) <= 1e-10, (i, j)


def test_tuning_cache_file_skips_the_second_tuning(problem_set, tmp_path):
    """tune(cache=path) writes the chosen shape to a tuning-cache file; a new
    solver on an equal problem set reads it back (no trials) and still reaches
    the closed form."""
    mihs = _mihs()
    dp, refs, L, Al, Be = _device_set(problem_set)
    path = str(tmp_path / "tuning.json")
    s = mihs.BatchedSolver(dp, L, Al, Be, eps_sub=1e-2, tol=1e-12, max_outer=800,
                           max_inner=2000)
    announce("batched tuning with a cache file")
    first = s.tune(trial_outer=2, measure=False, cache=path)
    assert first["trial_ms"] and not first.get("from_cache")
    assert os.path.exists(path)
    assert mihs.tuning_cache_load(path) >= 1
    s2 = mihs.BatchedSolver(dp, L, Al, Be, eps_sub=1e-2, tol=1e-12, max_outer=800,
                            max_inner=2000)
    second = s2.tune(trial_outer=2, measure=False, cache=path)
    assert second.get("from_cache") and second["best"] == first["best"]
    announce("batched run with the cached shape")
    s2.run()
    torch.cuda.synchronize()
    _check_closed_form(s2.xs, s2.infos(), refs)
