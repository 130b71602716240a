"""Properties of the seeded synthetic workloads (they hold no power-flow arithmetic)."""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph

import synth


def _connected(n, f, t):
    g = sp.coo_matrix((np.ones(len(f)), (f, t)), shape=(n, n))
    return csgraph.connected_components(g, directed=False)[0] == 1


def test_config0_shape_and_determinism():
    a = synth.config0(0)
    b = synth.config0(0)
    g = a["grid"]
    assert g.n_bus == 14 and g.n_branch == 20 and g.n_pv == 4 and g.n_pq == 9
    assert (g.bus_type == 2).sum() == 1 and g.va[g.slack] == 0.0
    assert _connected(g.n_bus, g.f, g.t)
    assert np.array_equal(g.f, b["grid"].f) and np.array_equal(g.vm, b["grid"].vm)
    assert np.all((g.r >= 0.01) & (g.r <= 0.1) & (g.x >= 0.05) & (g.x <= 0.3) & (g.b >= 0) & (g.b <= 0.05))
    key = set(zip(np.minimum(g.f, g.t), np.maximum(g.f, g.t)))
    assert len(key) == g.n_branch  # no parallel branches


def test_meshed_grid_counts_and_smooth_planting():
    cfg = synth.config1(B=4)
    g = cfg["grid"]
    assert (g.n_bus, g.n_branch, g.n_pv) == (1354, 1991, 260)
    assert _connected(g.n_bus, g.f, g.t)
    assert abs(np.abs(g.va).max() - 0.2) < 1e-12 and g.va[g.slack] == 0.0
    assert g.vm.min() >= 0.95 - 1e-12 and g.vm.max() <= 1.05 + 1e-12
    # per-case draws: PQ loads scaled within [0.9, 1.1], PV setpoints near planted
    pq = g.bus_type == 0
    pv = g.bus_type == 1
    assert np.all((cfg["load_scale"][:, pq] >= 0.9) & (cfg["load_scale"][:, pq] <= 1.1))
    assert np.all(cfg["load_scale"][:, ~pq] == 1.0)
    rel = cfg["vm0"][:, pv] / g.vm[pv] - 1.0
    assert np.abs(rel).max() <= 0.01 + 1e-12
    assert np.all(cfg["vm0"][:, pq] == 1.0) and np.all(cfg["va0"] == 0.0)


def test_non_bridge_branches_brute_force():
    g = synth.config0(5)["grid"]
    nb = set(synth.non_bridge_branches(g.n_bus, g.f, g.t).tolist())
    for e in range(g.n_branch):
        keep = np.arange(g.n_branch) != e
        assert (e in nb) == _connected(g.n_bus, g.f[keep], g.t[keep])


def test_config2_outages_are_distinct_non_bridges():
    cfg = synth.config2(B=64, n_bus=600, n_branch=880, n_pv=90)
    g = cfg["grid"]
    out = cfg["outage"]
    assert len(set(out.tolist())) == 64
    for e in out[:8]:
        keep = np.arange(g.n_branch) != e
        assert _connected(g.n_bus, g.f[keep], g.t[keep])


def test_config3_time_series_recipe():
    cfg = synth.config3(n_bus=500, n_branch=730, n_pv=80)
    g = cfg["grid"]
    pq = g.bus_type == 0
    ls = cfg["load_scale"]
    assert ls.shape == (96, g.n_bus) and np.all(ls[:, ~pq] == 1.0)
    assert np.abs(ls[:, pq] - 1.0).max() < 0.15 + 6 * 0.02
    sp_ = cfg["solar_p"]
    assert np.all(sp_[:25] == 0.0) and np.all(sp_ >= 0) and sp_.max() <= 0.3
    assert (sp_.max(axis=0) > 0).sum() <= int(round(0.2 * pq.sum()))


def test_config4_sizes():
    cfg = synth.config4(n_grids=6, lo=100, hi=2000, big=3000)
    sizes = [gg.n_bus for gg in cfg["grids"]]
    assert len(sizes) == 7 and sizes[-1] == 3000
    assert all(100 <= s <= 2000 for s in sizes[:-1])
    for gg in cfg["grids"]:
        assert gg.n_branch == int(round(1.4 * gg.n_bus))
        assert (gg.bus_type == 2).sum() == 1
