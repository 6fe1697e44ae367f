"""Host logic of the batched launch: the schedule of problems over workgroups
(teams for heavy entries, single-workgroup bins for the rest), from the cost
model and from measured per-entry costs.  No GPU calls."""
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1912_03514_amd", "libmihs.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libmihs.so not built")


def _mihs():
    import paper_1912_03514_amd as mihs
    return mihs


def _check_layout(sched, d, G, cg_cols, singles_on_teams=False):
    """Every entry has a valid place; teams are disjoint ranges of their own;
    bins (team size 1) only share workgroups with other bin entries (the
    measured schedule may also put them on a team's workgroups, after the team
    entry); the CG sub-team is at most the team and about d / cg_cols
    workgroups."""
    t0, ts, tc = (np.array(sched[k]) for k in ("team0", "tsize", "tcg"))
    assert (ts >= 1).all() and (t0 >= 0).all() and (t0 + ts <= G).all()
    assert (tc >= 1).all() and (tc <= ts).all()
    for e in range(len(t0)):
        assert tc[e] == max(1, min(ts[e], -(-d[e] // cg_cols)))
    owner = {}
    for e in np.flatnonzero(ts > 1):
        for g in range(t0[e], t0[e] + ts[e]):
            assert g not in owner, "teams overlap"
            owner[g] = e
    if not singles_on_teams:
        for e in np.flatnonzero(ts == 1):
            assert t0[e] not in owner, "a bin entry sits on a team workgroup"
    return t0, ts


def _loads(t0, ts, cost, G):
    load = np.zeros(G)
    for e in range(len(t0)):
        load[t0[e]:t0[e] + ts[e]] += cost[e] / ts[e]
    return load


def test_model_schedule_of_the_batched_workload():
    """256 problems with n in [4096, 65536], d in [64, 512], 16 lambdas, 256
    workgroups: a valid layout whose heaviest entries (by n d + w d^2) get the
    largest teams."""
    mihs = _mihs()
    import workloads as W
    specs = W.batched_specs()
    shapes = [(s.n, s.d) for s in specs]
    tn = {"cg_cols": 32, "a_dma": 1, "inner_weight": 100.0}
    sched = mihs.batched_schedule(shapes, 16, 256, tn)
    d = np.array([s.d for s in specs])
    t0, ts = _check_layout(sched, d, 256, 32)
    w = np.array([s.n * s.d + 100.0 * s.d * s.d for s in specs])
    heavy = np.argmax(w)
    assert ts[heavy] == ts.max()


def test_more_entries_than_workgroups_share_bins():
    mihs = _mihs()
    rng = np.random.default_rng(1)
    shapes = [(int(rng.integers(500, 5000)), int(rng.integers(8, 300))) for _ in range(100)]
    shapes = [(max(n, d), d) for n, d in shapes]
    sched = mihs.batched_schedule(shapes, 40, 32, {"cg_cols": 16, "a_dma": 0,
                                                   "inner_weight": 25.0})
    d = np.repeat([s[1] for s in shapes], 3)  # 40 lambdas = 3 entries per problem
    t0, ts = _check_layout(sched, d, 32, 16)
    assert len(t0) == 300


def test_one_problem_takes_every_workgroup():
    mihs = _mihs()
    sched = mihs.batched_schedule([(100000, 300)], 16, 64, {"cg_cols": 64, "a_dma": 1,
                                                            "inner_weight": 100.0})
    assert sched["team0"] == [0] and sched["tsize"] == [64] and sched["tcg"] == [5]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_measured_schedule_bounds_the_makespan(seed):
    """Teams of ceil(c / L) for entries above the makespan L, first-fit bins of
    capacity L for the rest (team members' remaining capacity included): every
    workgroup's load is at most L, which is within a factor 2 of the lower
    bound max(sum c / G, max c / G), and no worse than the model schedule's
    load under the same costs."""
    mihs = _mihs()
    rng = np.random.default_rng(seed)
    G = 256
    shapes = [(int(rng.integers(4096, 65536)), int(rng.integers(64, 513))) for _ in range(256)]
    cost = rng.lognormal(mean=0.0, sigma=0.6, size=256) * 1000.0
    cost[rng.integers(0, 256, size=3)] *= 20.0  # a few entries far above the rest
    tn = {"cg_cols": 32, "a_dma": 1, "inner_weight": 25.0, "measured": 1}
    sched = mihs.batched_schedule(shapes, 16, G, tn, cost=list(cost))
    d = np.array([s[1] for s in shapes])
    t0, ts = _check_layout(sched, d, G, 32, singles_on_teams=True)
    load = _loads(t0, ts, cost, G)
    lb = max(cost.sum() / G, cost.max() / G)
    assert load.max() <= 2.0 * lb * (1 + 1e-9) + np.sort(cost)[len(cost) // 2]
    model = mihs.batched_schedule(shapes, 16, G, dict(tn, measured=0))
    mt0, mts = _check_layout(model, d, G, 32)
    assert load.max() <= _loads(mt0, mts, cost, G).max() * (1 + 1e-9)
    # the heavy entries got teams
    for e in np.argsort(-cost)[:3]:
        assert ts[e] > 1


def test_measured_flag_without_costs_uses_the_model():
    mihs = _mihs()
    shapes = [(20000, 200), (4096, 64), (65536, 512)]
    a = mihs.batched_schedule(shapes, 16, 16, {"cg_cols": 32, "a_dma": 1, "inner_weight": 25.0,
                                               "measured": 1})
    b = mihs.batched_schedule(shapes, 16, 16, {"cg_cols": 32, "a_dma": 1, "inner_weight": 25.0})
    assert a == b


def test_schedule_rejects_bad_arguments():
    mihs = _mihs()
    with pytest.raises(mihs.MihsError):
        mihs.batched_schedule([(10, 20)], 16, 8)  # n < d
    with pytest.raises(mihs.MihsError):
        mihs.batched_schedule([(100, 20)], 16, 8, {"cg_cols": 48, "a_dma": 1,
                                                   "inner_weight": 25.0})


def test_exact_sub_solves_use_the_whole_team_up_to_sixteen():
    """With exact sub-solves the columns split over the team: the sub-team is the
    team, capped at one member per column."""
    import paper_1912_03514_amd as mihs
    shapes = [(60000, 500), (50000, 480), (8000, 100), (6000, 90)]
    for cols in (32, 512):
        tn = {"cg_cols": cols, "a_dma": 1, "inner_weight": 25.0, "exact": 1}
        sched = mihs.batched_schedule(shapes, 16, 40, tuning=tn)
        assert max(sched["tsize"]) > 1
        for ts, tc in zip(sched["tsize"], sched["tcg"]):
            assert tc == min(ts, 16), (ts, tc)


def test_measured_schedule_fills_team_workgroups():
    """One entry of cost 1.6 and eleven of 0.2 on four workgroups: the large one
    gets a team of two (0.8 each).  With the small ones only on the other two
    workgroups the makespan is 1.2 (six of them on one); filling the team
    members' remaining capacity after their team entry brings it to 1.0."""
    mihs = _mihs()
    G = 4
    cost = np.array([1.6] + [0.2] * 11)
    shapes = [(40000, 300)] * len(cost)
    tn = {"cg_cols": 32, "a_dma": 1, "inner_weight": 25.0, "measured": 1}
    sched = mihs.batched_schedule(shapes, 16, G, tn, cost=list(cost * 1000.0))
    d = np.array([s[1] for s in shapes])
    t0, ts = _check_layout(sched, d, G, 32, singles_on_teams=True)
    load = _loads(t0, ts, cost, G)
    assert ts[0] == 2
    team = set(range(t0[0], t0[0] + 2))
    assert any(t0[e] in team for e in range(1, len(cost))), sched
    assert load.max() <= 1.0 + 1e-3, load
