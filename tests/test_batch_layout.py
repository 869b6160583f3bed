"""Host logic of the batched planner: the team layout derived from
per-instance costs (no GPU needed; the library's host-only entry point)."""
import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def pk():
    import paper_0907_4631_amd as pk
    pk.lib()
    return pk


def check_layout(L, cost, G, max_team, alpha):
    ts, tc, order, qbeg = L["team_size"], L["team_class"], L["order"], L["qbeg"]
    count = len(cost)
    assert ts.sum() == G
    assert np.all(ts >= 1) and np.all((ts & (ts - 1)) == 0)
    lim = 1
    while lim * 2 <= min(max_team, G):
        lim *= 2
    assert ts.max() <= lim
    starts = np.concatenate([[0], np.cumsum(ts)[:-1]])
    assert np.all(starts % ts == 0), "teams must start at a multiple of their size"
    assert np.all(np.diff(tc) >= 0), "classes are laid out in order"
    ncls = len(qbeg) - 1
    assert sorted(order.tolist()) == list(range(count))
    assert qbeg[0] == 0 and qbeg[-1] == count and np.all(np.diff(qbeg) >= 0)
    share = cost.sum() / G if cost.sum() > 0 else 1.0 / G
    main = []
    for c in range(ncls):
        sizes = ts[tc == c]
        assert len(sizes) >= 1, "every class has a team"
        s = int(sizes.max())
        main.append(s)
        # only the last class may carry single-workgroup extras
        if c < ncls - 1:
            assert np.all(sizes == s)
        q = order[qbeg[c]:qbeg[c + 1]]
        assert np.all(np.diff(cost[q]) <= 0), "queues run in descending cost"
        smax = int(ts.max())   # the planner may lower its cap when the grid is small
        for i in q:
            if s < smax:
                assert cost[i] <= alpha * share * s * (1 + 1e-12)
            if s > 1:
                assert cost[i] > alpha * share * s / 2
    assert all(a > b for a, b in zip(main, main[1:])), "class sizes strictly decrease"


@pytest.mark.parametrize("G,max_team,alpha", [(256, 16, 1.0), (256, 32, 0.5), (256, 4, 2.0),
                                              (256, 1, 1.0), (100, 64, 1.0), (3, 2, 0.5),
                                              (1, 8, 1.0)])
def test_layout_properties_config4_costs(pk, G, max_team, alpha):
    specs = W.config4_specs()
    g = np.random.default_rng(0)
    # cost shaped like the planner's model: rows times sqrt(t ||A||)
    cost = np.array([s.N ** 2 * (10 + 13 * np.sqrt(s.t * 8 * (s.N + 1) ** 2)) for s in specs])
    cost *= g.uniform(0.8, 1.2, cost.size)
    L = pk.batch_layout(cost, G, max_team, alpha)
    check_layout(L, cost, G, max_team, alpha)


@pytest.mark.parametrize("cost", [[1.0], [0.0, 0.0, 0.0], [5.0, 1.0, 1.0, 1.0, 1.0, 1e6],
                                  list(np.arange(1, 40, dtype=float))])
@pytest.mark.parametrize("G", [1, 7, 64])
def test_layout_small_cases(pk, cost, G):
    cost = np.asarray(cost, dtype=float)
    for max_team in (1, 2, 8, 64):
        L = pk.batch_layout(cost, G, max_team, 1.0)
        check_layout(L, cost, G, max_team, 1.0)


def test_heaviest_instance_gets_the_largest_team(pk):
    cost = np.ones(300)
    cost[17] = 400.0
    L = pk.batch_layout(cost, 256, 16, 1.0)
    assert L["order"][0] == 17 and L["team_size"][0] == 16


def test_layout_rejects_bad_arguments(pk):
    for args in [([1.0], 0, 4, 1.0), ([1.0], 4, 3, 1.0), ([1.0], 4, 4, 0.0),
                 ([-1.0], 4, 4, 1.0), ([np.nan], 4, 4, 1.0), ([1.0], 2000, 4, 1.0)]:
        with pytest.raises(pk.PhipmError) as e:
            pk.batch_layout(*args)
        assert e.value.status == pk.EINVAL
