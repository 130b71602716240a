"""Seeded synthetic grids and workloads.

The paper's experiments use the IEEE-118, case1354pegase and case9241pegase
grids and the LIPS dataset (Sec. 6.1). None of them is available here, so
these generators stand in for them with random grids of the same bus and
branch counts.  Every draw is seeded; configuration k uses seed 1000*k and
per-case draws use child streams of that seed.

Conventions shared with every consumer:
  * buses are numbered 0..n_bus-1, branches 0..n_branch-1;
  * bus types: PQ = 0, PV = 1, SLACK = 2 (exactly one slack per grid);
  * branches are pi-models with series r + jx and total charging b;
  * planted voltages (vm, va) are an exact solution by construction: the
    consumer computes the injections S = V * conj(Y V) from them itself.

Only numpy / scipy graph and random routines are used here.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph
import scipy.sparse.linalg as spla
from scipy.spatial import cKDTree

PQ, PV, SLACK = 0, 1, 2

# branch parameter ranges in per unit (identical for every configuration)
R_RANGE = (0.01, 0.1)
X_RANGE = (0.05, 0.3)
B_RANGE = (0.0, 0.05)
VM_RANGE = (0.95, 1.05)
VA_MAX = 0.2
PV_REPLANT = 0.01  # relative re-planting of PV setpoints per case


@dataclass
class Grid:
    n_bus: int
    f: np.ndarray  # int32 [n_branch] from-bus
    t: np.ndarray  # int32 [n_branch] to-bus
    r: np.ndarray  # float64 [n_branch]
    x: np.ndarray  # float64 [n_branch]
    b: np.ndarray  # float64 [n_branch] total line charging
    bus_type: np.ndarray  # int8 [n_bus]
    vm: np.ndarray  # float64 [n_bus] planted |V|
    va: np.ndarray  # float64 [n_bus] planted angle (rad), 0 at the slack
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_branch(self) -> int:
        return int(self.f.shape[0])

    @property
    def slack(self) -> int:
        return int(np.flatnonzero(self.bus_type == SLACK)[0])

    @property
    def n_pv(self) -> int:
        return int(np.count_nonzero(self.bus_type == PV))

    @property
    def n_pq(self) -> int:
        return int(np.count_nonzero(self.bus_type == PQ))


# ---------------------------------------------------------------- topology


def tree_chord_grid(rng: np.random.Generator, n_bus: int, n_branch: int):
    """Random recursive tree plus uniform random chords.

    Bus k (k >= 1) attaches to a uniformly chosen earlier bus; then distinct
    non-tree bus pairs are drawn uniformly until n_branch branches exist.
    Returns (f, t) int32 arrays without parallel branches.
    """
    if n_branch < n_bus - 1:
        raise ValueError("a connected grid needs at least n_bus-1 branches")
    max_edges = n_bus * (n_bus - 1) // 2
    if n_branch > max_edges:
        raise ValueError("too many branches for a simple graph")
    edges = []
    seen = set()
    for k in range(1, n_bus):
        p = int(rng.integers(0, k))
        edges.append((p, k))
        seen.add((p, k))
    while len(edges) < n_branch:
        a, c = (int(v) for v in rng.integers(0, n_bus, size=2))
        if a == c:
            continue
        key = (min(a, c), max(a, c))
        if key in seen:
            continue
        seen.add(key)
        edges.append(key)
    e = np.asarray(edges, dtype=np.int32)
    return e[:, 0].copy(), e[:, 1].copy()


def geometric_grid(rng: np.random.Generator, n_bus: int, n_branch: int, knn: int = 8):
    """Random geometric spanning tree plus nearest-neighbour chords.

    Buses are points drawn uniformly in the unit square.  The Euclidean
    minimum spanning tree of the k-nearest-neighbour graph gives the tree;
    the shortest k-NN edges not in the tree are added as chords until
    n_branch branches exist.  Returns (f, t, pos).
    """
    if n_branch < n_bus - 1:
        raise ValueError("a connected grid needs at least n_bus-1 branches")
    pos = rng.random((n_bus, 2))
    k = min(knn, n_bus - 1)
    while True:
        tree = cKDTree(pos)
        dist, idx = tree.query(pos, k=k + 1)
        rows = np.repeat(np.arange(n_bus), k)
        cols = idx[:, 1:].reshape(-1)
        d = dist[:, 1:].reshape(-1)
        a = np.minimum(rows, cols)
        c = np.maximum(rows, cols)
        key = a.astype(np.int64) * n_bus + c
        key, first = np.unique(key, return_index=True)
        a, c, d = a[first], c[first], d[first]
        g = sp.coo_matrix((d, (a, c)), shape=(n_bus, n_bus)).tocsr()
        ncomp, _ = csgraph.connected_components(g, directed=False)
        if ncomp == 1 and len(a) >= n_branch:
            break
        k = min(2 * k, n_bus - 1)
    mst = csgraph.minimum_spanning_tree(g).tocoo()
    tf = np.minimum(mst.row, mst.col)
    tt = np.maximum(mst.row, mst.col)
    tkey = set((tf.astype(np.int64) * n_bus + tt).tolist())
    order = np.argsort(d, kind="stable")
    chords = []
    need = n_branch - (n_bus - 1)
    for i in order:
        if len(chords) >= need:
            break
        kk = int(key[i])
        if kk in tkey:
            continue
        chords.append((int(a[i]), int(c[i])))
    if len(chords) < need:
        raise ValueError("k-NN graph too sparse for the requested branch count")
    f = np.concatenate([tf, np.asarray([p[0] for p in chords], dtype=np.int64)])
    t = np.concatenate([tt, np.asarray([p[1] for p in chords], dtype=np.int64)])
    perm = rng.permutation(n_branch)
    return f[perm].astype(np.int32), t[perm].astype(np.int32), pos


def branch_params(rng: np.random.Generator, n_branch: int):
    r = rng.uniform(*R_RANGE, size=n_branch)
    x = rng.uniform(*X_RANGE, size=n_branch)
    b = rng.uniform(*B_RANGE, size=n_branch)
    return r, x, b


def bus_types(rng: np.random.Generator, n_bus: int, n_pv: int) -> np.ndarray:
    """One uniformly chosen slack and n_pv uniformly chosen PV buses."""
    perm = rng.permutation(n_bus)
    bt = np.zeros(n_bus, dtype=np.int8)
    bt[perm[0]] = SLACK
    bt[perm[1 : 1 + n_pv]] = PV
    return bt


def non_bridge_branches(n_bus: int, f: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Indices of branches whose removal keeps the grid connected.

    Iterative Tarjan low-link search over the undirected multigraph (a
    branch with a parallel twin is never a bridge).
    """
    n_br = len(f)
    adj_ptr = np.zeros(n_bus + 1, dtype=np.int64)
    np.add.at(adj_ptr, f + 1, 1)
    np.add.at(adj_ptr, t + 1, 1)
    adj_ptr = np.cumsum(adj_ptr)
    adj_nb = np.empty(2 * n_br, dtype=np.int64)
    adj_e = np.empty(2 * n_br, dtype=np.int64)
    fill = adj_ptr[:-1].copy()
    for e in range(n_br):
        for u, v in ((f[e], t[e]), (t[e], f[e])):
            adj_nb[fill[u]] = v
            adj_e[fill[u]] = e
            fill[u] += 1
    disc = np.full(n_bus, -1, dtype=np.int64)
    low = np.zeros(n_bus, dtype=np.int64)
    is_bridge = np.zeros(n_br, dtype=bool)
    timer = 0
    for root in range(n_bus):
        if disc[root] >= 0:
            continue
        disc[root] = low[root] = timer
        timer += 1
        stack = [(root, -1, adj_ptr[root])]
        while stack:
            u, pe, it = stack[-1]
            if it < adj_ptr[u + 1]:
                stack[-1] = (u, pe, it + 1)
                v, e = adj_nb[it], adj_e[it]
                if e == pe:
                    continue
                if disc[v] < 0:
                    disc[v] = low[v] = timer
                    timer += 1
                    stack.append((v, e, adj_ptr[v]))
                else:
                    low[u] = min(low[u], disc[v])
            else:
                stack.pop()
                if stack:
                    p = stack[-1][0]
                    low[p] = min(low[p], low[u])
                    if low[u] > disc[p]:
                        is_bridge[pe] = True
    return np.flatnonzero(~is_bridge).astype(np.int32)


# ---------------------------------------------------------------- planting


def plant_iid(rng: np.random.Generator, n_bus: int, bus_type: np.ndarray):
    """|V| ~ U(0.95, 1.05) and angle ~ U(-0.2, 0.2) per bus, slack angle 0."""
    vm = rng.uniform(*VM_RANGE, size=n_bus)
    va = rng.uniform(-VA_MAX, VA_MAX, size=n_bus)
    va[bus_type == SLACK] = 0.0
    return vm, va


def _laplacian(n_bus, f, t, w):
    return sp.coo_matrix(
        (np.concatenate([w, w, -w, -w]),
         (np.concatenate([f, t, f, t]), np.concatenate([f, t, t, f]))),
        shape=(n_bus, n_bus)).tocsc()


def plant_smooth(rng: np.random.Generator, n_bus, f, t, x, bus_type):
    """Smooth planted voltage profile for meshed grids.

    Angles: zero-mean random nodal injections spread over the graph through
    the branch-susceptance Laplacian (weights 1/x) grounded at the slack,
    rescaled so that max|angle| = 0.2 rad.  Magnitudes: a second random
    injection pattern spread the same way (Laplacian + 1e-3 I), mapped affinely
    onto [0.95, 1.05].  This is input synthesis (a smooth, physically plausible
    profile whose injections stay well inside the loadability limit), not a
    power-flow solve of the workload.
    """
    lap = _laplacian(n_bus, f, t, 1.0 / x)
    s = int(np.flatnonzero(bus_type == SLACK)[0])
    keep = np.flatnonzero(np.arange(n_bus) != s)
    p = rng.standard_normal(n_bus)
    p -= p.mean()
    va = np.zeros(n_bus)
    va[keep] = spla.spsolve(lap[keep][:, keep].tocsc(), p[keep])
    va *= VA_MAX / np.max(np.abs(va))
    va[s] = 0.0
    q = rng.standard_normal(n_bus)
    q -= q.mean()
    fld = spla.spsolve((lap + 1e-3 * sp.identity(n_bus, format="csc")).tocsc(), q)
    span = fld.max() - fld.min()
    fld = (fld - fld.min()) / span if span > 0 else np.full(n_bus, 0.5)
    vm = VM_RANGE[0] + (VM_RANGE[1] - VM_RANGE[0]) * fld
    return vm, va


def _make_grid(rng, n_bus, n_branch, n_pv, *, geometric, smooth, name):
    if geometric:
        f, t, pos = geometric_grid(rng, n_bus, n_branch)
    else:
        f, t = tree_chord_grid(rng, n_bus, n_branch)
        pos = None
    r, x, b = branch_params(rng, len(f))
    bt = bus_types(rng, n_bus, n_pv)
    if smooth:
        vm, va = plant_smooth(rng, n_bus, f, t, x, bt)
    else:
        vm, va = plant_iid(rng, n_bus, bt)
    meta = {"pos": pos}
    return Grid(n_bus, f, t, r, x, b, bt, vm, va, name=name, meta=meta)


def flat_start(grid: Grid, vm_set=None):
    """Flat start: |V| = 1 at PQ buses, setpoint at PV and slack, angle 0.

    vm_set overrides the PV/slack setpoints (shape [n_bus] or [B, n_bus]).
    Returns (vm0, va0) with the broadcast shape of vm_set.
    """
    base = grid.vm if vm_set is None else np.asarray(vm_set, dtype=np.float64)
    vm0 = np.where(grid.bus_type == PQ, 1.0, base)
    va0 = np.zeros_like(vm0)
    return vm0, va0


# ---------------------------------------------------------------- configs


def config0(seed: int = 0) -> dict:
    """14 buses (1 slack, 4 PV, 9 PQ), 20 branches, one case, flat start."""
    rng = np.random.default_rng(seed)
    g = _make_grid(rng, 14, 20, 4, geometric=False, smooth=False, name="synthetic-14")
    vm0, va0 = flat_start(g)
    return {"name": "cfg0", "grid": g, "B": 1, "vm0": vm0[None], "va0": va0[None],
            "load_scale": np.ones((1, g.n_bus)), "seed": seed}


def config1(seed: int = 1000, B: int = 64, n_bus: int = 1354, n_branch: int = 1991,
            n_pv: int = 260) -> dict:
    """B cases on one meshed grid; per case PQ loads x U(0.9, 1.1) per bus and
    PV setpoints re-planted as the planted |V| x (1 + U(-0.01, 0.01)); flat start."""
    rng = np.random.default_rng(seed)
    g = _make_grid(rng, n_bus, n_branch, n_pv, geometric=True, smooth=True,
                   name=f"synthetic-{n_bus}")
    load_scale = np.ones((B, n_bus))
    vm_set = np.tile(g.vm, (B, 1))
    pq = g.bus_type == PQ
    pv = g.bus_type == PV
    for c, child in enumerate(np.random.SeedSequence(seed).spawn(B)):
        cr = np.random.default_rng(child)
        load_scale[c, pq] = cr.uniform(0.9, 1.1, size=int(pq.sum()))
        vm_set[c, pv] = g.vm[pv] * (1.0 + cr.uniform(-PV_REPLANT, PV_REPLANT, size=int(pv.sum())))
    vm0, va0 = flat_start(g, vm_set)
    return {"name": "cfg1", "grid": g, "B": B, "vm0": vm0, "va0": va0,
            "load_scale": load_scale, "seed": seed}


def _pegase_like(seed: int, n_bus=9241, n_branch=16049, n_pv=1445) -> Grid:
    rng = np.random.default_rng(seed)
    return _make_grid(rng, n_bus, n_branch, n_pv, geometric=True, smooth=True,
                      name=f"synthetic-{n_bus}")


def config2(seed: int = 2000, B: int = 1024, n_bus: int = 9241, n_branch: int = 16049,
            n_pv: int = 1445) -> dict:
    """N-1 batch: B distinct non-bridge outages sharing the base injections,
    every case warm-started from the planted (base-case) voltages."""
    g = _pegase_like(seed, n_bus, n_branch, n_pv)
    cand = non_bridge_branches(g.n_bus, g.f, g.t)
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    if B > len(cand):
        raise ValueError("not enough non-bridge branches")
    outage = np.sort(rng.choice(cand, size=B, replace=False)).astype(np.int32)
    vm0 = np.tile(g.vm, (B, 1))
    va0 = np.tile(g.va, (B, 1))
    return {"name": "cfg2", "grid": g, "B": B, "vm0": vm0, "va0": va0,
            "outage": outage, "load_scale": np.ones((1, g.n_bus)), "seed": seed}


def config3(seed: int = 3000, T: int = 96, n_bus: int = 9241, n_branch: int = 16049,
            n_pv: int = 1445, window: int = 16, grid_seed: int = 2000) -> dict:
    """Time series: per-bus load factor 1 + 0.15 sin(2 pi t/96 + phi) + N(0, 0.02)
    on PQ buses, plus solar active injection peak * max(0, sin(pi (t-24)/48))
    at 20% of the PQ buses (peak ~ U(0, 0.3) pu).  The grid is the N-1 batch's
    (grid_seed, as config2 draws it); the loads and the solar buses come from
    `seed`."""
    g = _pegase_like(grid_seed, n_bus, n_branch, n_pv)
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(1)[0])
    pq = np.flatnonzero(g.bus_type == PQ)
    phi = rng.uniform(0.0, 2 * np.pi, size=g.n_bus)
    noise = rng.normal(0.0, 0.02, size=(T, g.n_bus))
    tt = np.arange(T)[:, None]
    load_scale = np.ones((T, g.n_bus))
    fac = 1.0 + 0.15 * np.sin(2 * np.pi * tt / 96.0 + phi[None, :]) + noise
    load_scale[:, pq] = fac[:, pq]
    solar_bus = np.sort(rng.choice(pq, size=int(round(0.2 * len(pq))), replace=False))
    peak = np.zeros(g.n_bus)
    peak[solar_bus] = rng.uniform(0.0, 0.3, size=len(solar_bus))
    shape = np.maximum(0.0, np.sin(np.pi * (np.arange(T) - 24) / 48.0))
    solar_p = shape[:, None] * peak[None, :]
    return {"name": "cfg3", "grid": g, "T": T, "window": window,
            "load_scale": load_scale, "solar_p": solar_p, "seed": seed}


def config4(seed: int = 4000, n_grids: int = 128, lo: int = 100, hi: int = 80000,
            big: int = 80000, branches_per_bus: float = 1.4) -> dict:
    """Uneven batch: n_grids geometric grids with log-uniform sizes in
    [lo, hi] plus one grid of `big` buses; PV fraction 1445/9241."""
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(lo), np.log(hi), size=n_grids)).astype(np.int64)
    sizes = np.concatenate([sizes, [big]]) if big else sizes
    grids = []
    for k, children in enumerate(np.random.SeedSequence(seed).spawn(len(sizes))):
        n = int(sizes[k])
        nb = int(round(branches_per_bus * n))
        npv = int(round(n * 1445 / 9241))
        grids.append(_make_grid(np.random.default_rng(children), n, nb, npv,
                                geometric=True, smooth=True, name=f"synthetic-{n}"))
    return {"name": "cfg4", "grids": grids, "seed": seed}
