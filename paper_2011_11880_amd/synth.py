"""Seeded synthetic power-network generators.

This module draws topologies, device parameters, states, scenario factors and
contingency picks.  It holds none of the power-flow arithmetic: no branch
flows, no injections, no derivatives.  Both the HIP path (through the
binding) and the CPU oracle (through the tests) take their inputs from here.

Workload shapes follow the paper's case studies (Section IV): a 70,000-bus
synthetic grid with 88,207 branches and transformers, plus 2k/10k/25k grids.
The paper's datasets are not available, so these generators stand in for them.

Parameter distributions (all in per-unit, angles in radians except the
transformer phase shift, which is given in degrees like common network data):

* series resistance r ~ U(0.001, 0.05), reactance x ~ U(0.01, 0.3),
  total line charging b ~ U(0, 0.05);
* 15% of branches are transformers: tap ~ U(0.95, 1.05),
  phase shift ~ U(-5, 5) degrees; the others have tap 1 and shift 0;
* PQ loads P ~ U(0, 1), Q = 0.3 P;
* PV setpoints V ~ U(0.98, 1.05) and
  P = (sum of load P / (N_pv + 1)) * U(0.8, 1.2);
* shunts g ~ U(0, 0.01), b ~ U(0, 0.3);
* states: |V| ~ U(0.95, 1.05), theta ~ N(0, 0.1), Q_g ~ U(-1, 1) and the
  slack active power equal to total load minus total PV setpoint.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Network",
    "tiny_grid",
    "geometric_grid",
    "grid_70k",
    "grid_10k",
    "random_states",
    "batch_scenarios",
    "non_bridge_branches",
    "contingencies",
    "uneven_grids",
    "with_parallel_branches",
]


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


@dataclass
class Network:
    """Host structure-of-arrays description of one network.

    Index arrays are 0-based int32, numeric arrays float64.  Generators are
    listed PV first (input order) and then slack; a bus carries at most one
    generator.  ``br_status`` is 1 for an in-service branch.
    """

    n_bus: int
    br_from: np.ndarray
    br_to: np.ndarray
    br_r: np.ndarray
    br_x: np.ndarray
    br_b: np.ndarray
    br_tap: np.ndarray
    br_shift_deg: np.ndarray
    br_status: np.ndarray
    load_bus: np.ndarray
    load_p: np.ndarray
    load_q: np.ndarray
    pv_bus: np.ndarray
    pv_p: np.ndarray
    pv_v: np.ndarray
    slack_bus: np.ndarray
    slack_v: np.ndarray
    slack_theta: np.ndarray
    shunt_bus: np.ndarray
    shunt_g: np.ndarray
    shunt_b: np.ndarray
    coords: np.ndarray | None = field(default=None, repr=False)

    def __post_init__(self):
        for name in ("br_from", "br_to", "br_status", "load_bus", "pv_bus",
                     "slack_bus", "shunt_bus"):
            setattr(self, name, _i32(getattr(self, name)))
        for name in ("br_r", "br_x", "br_b", "br_tap", "br_shift_deg",
                     "load_p", "load_q", "pv_p", "pv_v", "slack_v",
                     "slack_theta", "shunt_g", "shunt_b"):
            setattr(self, name, _f64(getattr(self, name)))

    # sizes -----------------------------------------------------------------
    @property
    def n_branch(self) -> int:
        return int(self.br_from.shape[0])

    @property
    def n_load(self) -> int:
        return int(self.load_bus.shape[0])

    @property
    def n_pv(self) -> int:
        return int(self.pv_bus.shape[0])

    @property
    def n_slack(self) -> int:
        return int(self.slack_bus.shape[0])

    @property
    def n_gen(self) -> int:
        return self.n_pv + self.n_slack

    @property
    def n_shunt(self) -> int:
        return int(self.shunt_bus.shape[0])

    @property
    def n_var(self) -> int:
        """Length of the state vector [theta, V, Q_g, P_s] (eq. 3)."""
        return 2 * self.n_bus + self.n_gen + self.n_slack

    def copy(self) -> "Network":
        kw = {}
        for k, v in self.__dict__.items():
            kw[k] = v.copy() if isinstance(v, np.ndarray) else v
        return Network(**kw)

    def without_branch(self, e: int) -> "Network":
        """The same network with branch ``e`` taken out of service."""
        net = self.copy()
        net.br_status = net.br_status.copy()
        net.br_status[e] = 0
        return net


# ---------------------------------------------------------------------------
# building blocks
# ---------------------------------------------------------------------------

def _branch_params(rng: np.random.Generator, n_branch: int, xfmr_frac=0.15):
    r = rng.uniform(0.001, 0.05, n_branch)
    x = rng.uniform(0.01, 0.3, n_branch)
    b = rng.uniform(0.0, 0.05, n_branch)
    tap = np.ones(n_branch)
    shift = np.zeros(n_branch)
    n_x = int(round(xfmr_frac * n_branch))
    idx = rng.choice(n_branch, size=n_x, replace=False)
    tap[idx] = rng.uniform(0.95, 1.05, n_x)
    shift[idx] = rng.uniform(-5.0, 5.0, n_x)
    return r, x, b, tap, shift


def _prufer_tree(rng: np.random.Generator, n: int):
    """Uniform random labelled tree on n nodes, decoded from a Pruefer sequence."""
    if n == 1:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    if n == 2:
        return np.array([0]), np.array([1])
    seq = rng.integers(0, n, n - 2)
    degree = np.ones(n, dtype=np.int64)
    np.add.at(degree, seq, 1)
    import heapq
    leaves = [i for i in range(n) if degree[i] == 1]
    heapq.heapify(leaves)
    us, vs = [], []
    for s in seq:
        leaf = heapq.heappop(leaves)
        us.append(leaf)
        vs.append(int(s))
        degree[s] -= 1
        if degree[s] == 1:
            heapq.heappush(leaves, int(s))
    a = heapq.heappop(leaves)
    b = heapq.heappop(leaves)
    us.append(a)
    vs.append(b)
    return np.array(us), np.array(vs)


def _extra_edges(rng, n, existing: set, count: int):
    us, vs = [], []
    while len(us) < count:
        u, v = (int(z) for z in rng.integers(0, n, 2))
        if u == v:
            continue
        key = (min(u, v), max(u, v))
        if key in existing:
            continue
        existing.add(key)
        us.append(u)
        vs.append(v)
    return np.array(us, dtype=np.int64), np.array(vs, dtype=np.int64)


def _pv_setpoints(rng, load_p_total: float, n_pv: int):
    return (load_p_total / (n_pv + 1)) * rng.uniform(0.8, 1.2, n_pv)


# ---------------------------------------------------------------------------
# configurations
# ---------------------------------------------------------------------------

def tiny_grid(seed: int = 0, n_bus: int = 200, n_branch: int = 280,
              n_pv: int = 40, n_shunt: int = 0) -> Network:
    """Plain-method tiny grid: a random spanning tree plus extra random edges.

    200 buses and 280 branches by default (the tree's 199 edges plus 81
    uniform non-duplicate extra pairs, no self-loops).  Bus 0 is the slack,
    ``n_pv`` uniformly chosen buses are PV, every other bus carries a PQ load.
    """
    rng = np.random.default_rng(seed)
    fu, fv = _prufer_tree(rng, n_bus)
    existing = {(min(a, b), max(a, b)) for a, b in zip(fu.tolist(), fv.tolist())}
    n_extra = n_branch - (n_bus - 1)
    if n_extra < 0:
        raise ValueError("n_branch must be at least n_bus - 1")
    eu, ev = _extra_edges(rng, n_bus, existing, n_extra)
    u = np.concatenate([fu, eu])
    v = np.concatenate([fv, ev])
    flip = rng.random(u.shape[0]) < 0.5
    frm = np.where(flip, v, u)
    to = np.where(flip, u, v)
    r, x, b, tap, shift = _branch_params(rng, n_branch)

    slack = np.array([0])
    pv = np.sort(rng.choice(np.arange(1, n_bus), size=n_pv, replace=False))
    is_gen = np.zeros(n_bus, bool)
    is_gen[pv] = True
    is_gen[slack] = True
    loads = np.nonzero(~is_gen)[0]
    lp = rng.uniform(0.0, 1.0, loads.shape[0])
    lq = 0.3 * lp
    pv_v = rng.uniform(0.98, 1.05, n_pv)
    pv_p = _pv_setpoints(rng, lp.sum(), n_pv)
    slack_v = rng.uniform(0.98, 1.05, 1)
    sh_bus = np.sort(rng.choice(n_bus, size=n_shunt, replace=False))
    sh_g = rng.uniform(0.0, 0.01, n_shunt)
    sh_b = rng.uniform(0.0, 0.3, n_shunt)
    return Network(
        n_bus=n_bus, br_from=frm, br_to=to, br_r=r, br_x=x, br_b=b,
        br_tap=tap, br_shift_deg=shift, br_status=np.ones(n_branch),
        load_bus=loads, load_p=lp, load_q=lq,
        pv_bus=pv, pv_p=pv_p, pv_v=pv_v,
        slack_bus=slack, slack_v=slack_v, slack_theta=np.zeros(1),
        shunt_bus=sh_bus, shunt_g=sh_g, shunt_b=sh_b)


def geometric_grid(n_bus: int, n_branch: int, n_pv: int, n_load: int,
                   n_shunt: int, seed: int, xfmr_frac: float = 0.15) -> Network:
    """Random geometric grid with a connected backbone.

    Buses are uniform points in the unit square.  Branches are the Delaunay
    edges of the Euclidean minimum spanning tree (which makes the grid
    connected) followed by the shortest remaining Delaunay edges until
    ``n_branch`` edges exist.  Bus ids are then randomly permuted and each
    branch gets a random orientation.  One slack, ``n_pv`` PV buses,
    ``n_load`` load buses (disjoint from generator buses) and ``n_shunt``
    shunt buses are drawn uniformly.
    """
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import minimum_spanning_tree
    from scipy.spatial import Delaunay

    if n_pv + 1 + n_load > n_bus:
        raise ValueError("too many generators and loads for the bus count")
    rng = np.random.default_rng(seed)
    pts = rng.random((n_bus, 2))
    tri = Delaunay(pts)
    s = tri.simplices
    e = np.concatenate([s[:, [0, 1]], s[:, [1, 2]], s[:, [0, 2]]])
    e.sort(axis=1)
    e = np.unique(e, axis=0)
    length = np.hypot(*(pts[e[:, 0]] - pts[e[:, 1]]).T)
    g = coo_matrix((length, (e[:, 0], e[:, 1])), shape=(n_bus, n_bus)).tocsr()
    mst = minimum_spanning_tree(g).tocoo()
    tree = np.stack([np.minimum(mst.row, mst.col), np.maximum(mst.row, mst.col)], 1)
    if tree.shape[0] != n_bus - 1:
        raise RuntimeError("backbone is not spanning")
    key = e[:, 0].astype(np.int64) * n_bus + e[:, 1]
    tkey = tree[:, 0].astype(np.int64) * n_bus + tree[:, 1]
    rest = ~np.isin(key, tkey)
    order = np.argsort(length[rest], kind="stable")
    n_extra = n_branch - (n_bus - 1)
    if n_extra > order.shape[0]:
        raise ValueError("not enough Delaunay edges for the branch count")
    extra = e[rest][order[:n_extra]]
    edges = np.concatenate([tree, extra])
    perm = rng.permutation(n_bus)
    u = perm[edges[:, 0]]
    v = perm[edges[:, 1]]
    flip = rng.random(u.shape[0]) < 0.5
    frm = np.where(flip, v, u)
    to = np.where(flip, u, v)
    coords = np.empty_like(pts)
    coords[perm] = pts
    r, x, b, tap, shift = _branch_params(rng, n_branch, xfmr_frac)

    buses = rng.permutation(n_bus)
    slack = buses[:1]
    pv = np.sort(buses[1:1 + n_pv])
    loads = np.sort(buses[1 + n_pv:1 + n_pv + n_load])
    lp = rng.uniform(0.0, 1.0, n_load)
    lq = 0.3 * lp
    pv_v = rng.uniform(0.98, 1.05, n_pv)
    pv_p = _pv_setpoints(rng, lp.sum(), n_pv)
    slack_v = rng.uniform(0.98, 1.05, 1)
    sh_bus = np.sort(rng.choice(n_bus, size=n_shunt, replace=False))
    sh_g = rng.uniform(0.0, 0.01, n_shunt)
    sh_b = rng.uniform(0.0, 0.3, n_shunt)
    return Network(
        n_bus=n_bus, br_from=frm, br_to=to, br_r=r, br_x=x, br_b=b,
        br_tap=tap, br_shift_deg=shift, br_status=np.ones(n_branch),
        load_bus=loads, load_p=lp, load_q=lq,
        pv_bus=pv, pv_p=pv_p, pv_v=pv_v,
        slack_bus=slack, slack_v=slack_v, slack_theta=np.zeros(1),
        shunt_bus=sh_bus, shunt_g=sh_g, shunt_b=sh_b, coords=coords)


def _fractions(n_bus: int):
    """PV, load and shunt counts in the proportions of the 70,000-bus case
    (10,000 PV, 40,000 loads, 5% shunts)."""
    n_pv = int(round(n_bus / 7))
    n_load = int(round(4 * n_bus / 7))
    n_sh = int(round(0.05 * n_bus))
    return n_pv, n_load, n_sh


def grid_70k(seed: int = 1000) -> Network:
    """Paper-scale grid: 70,000 buses and 88,207 branches (Section IV-A)."""
    return geometric_grid(70000, 88207, 10000, 40000, 3500, seed)


def grid_10k(seed: int = 2000) -> Network:
    """10,000 buses, 12,500 branches, same proportions as the 70,000-bus grid."""
    n_pv, n_load, n_sh = _fractions(10000)
    return geometric_grid(10000, 12500, n_pv, n_load, n_sh, seed)


def random_states(net: Network, n_states: int | None = None, seed: int = 0):
    """Random states x = [theta, V, Q_g, P_s].

    Returns shape (n_var,) when ``n_states`` is None, else (n_states, n_var).
    """
    rng = np.random.default_rng(seed)
    s = 1 if n_states is None else n_states
    N, NG, NS = net.n_bus, net.n_gen, net.n_slack
    X = np.empty((s, net.n_var))
    X[:, :N] = rng.normal(0.0, 0.1, (s, N))
    X[:, N:2 * N] = rng.uniform(0.95, 1.05, (s, N))
    X[:, 2 * N:2 * N + NG] = rng.uniform(-1.0, 1.0, (s, NG))
    ps = net.load_p.sum() - net.pv_p.sum()
    X[:, 2 * N + NG:] = ps / max(NS, 1)
    return X[0] if n_states is None else X


def batch_scenarios(net: Network, n_scen: int, seed: int):
    """Load/renewable scenarios: per load a lognormal factor exp(0.1 z),
    z ~ N(0, 1), applied to both P and Q; per PV unit a factor U(0.5, 1.2)
    on its active-power setpoint.  Shapes (n_scen, n_load), (n_scen, n_pv)."""
    rng = np.random.default_rng(seed)
    load_scale = np.exp(0.1 * rng.standard_normal((n_scen, net.n_load)))
    pv_scale = rng.uniform(0.5, 1.2, (n_scen, net.n_pv))
    return load_scale, pv_scale


def non_bridge_branches(net: Network) -> np.ndarray:
    """In-service branches whose removal keeps the network connected.

    Iterative Tarjan bridge search on the multigraph (parallel branches are
    never bridges)."""
    N = net.n_bus
    live = np.nonzero(net.br_status != 0)[0]
    adj = [[] for _ in range(N)]
    for e in live.tolist():
        u, v = int(net.br_from[e]), int(net.br_to[e])
        adj[u].append((v, e))
        adj[v].append((u, e))
    disc = [-1] * N
    low = [0] * N
    is_bridge = np.zeros(net.n_branch, bool)
    t = 0
    for root in range(N):
        if disc[root] >= 0:
            continue
        disc[root] = low[root] = t
        t += 1
        stack = [(root, -1, iter(adj[root]))]
        while stack:
            u, pe, it = stack[-1]
            advanced = False
            for v, e in it:
                if e == pe:
                    continue
                if disc[v] < 0:
                    disc[v] = low[v] = t
                    t += 1
                    stack.append((v, e, iter(adj[v])))
                    advanced = True
                    break
                low[u] = min(low[u], disc[v])
            if advanced:
                continue
            stack.pop()
            if stack:
                p = stack[-1][0]
                low[p] = min(low[p], low[u])
                if low[u] > disc[p]:
                    is_bridge[pe] = True
    mask = np.zeros(net.n_branch, bool)
    mask[live] = True
    return np.nonzero(mask & ~is_bridge)[0].astype(np.int32)


def contingencies(net: Network, n: int, seed: int) -> np.ndarray:
    """``n`` distinct N-1 outages drawn without replacement from non-bridges."""
    rng = np.random.default_rng(seed)
    cand = non_bridge_branches(net)
    if n > cand.shape[0]:
        raise ValueError("not enough non-bridge branches")
    return np.sort(rng.choice(cand, size=n, replace=False)).astype(np.int32)


def uneven_grids(n_grids: int = 256, seed: int = 3000, lo: int = 500,
                 hi: int = 20000) -> list[Network]:
    """Independent grids with bus counts log-uniform in [lo, hi], 1.25
    branches per bus and the proportions of the 70,000-bus grid."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), n_grids))).astype(int)
    grids = []
    for k, nb in enumerate(sizes.tolist()):
        n_pv, n_load, n_sh = _fractions(nb)
        grids.append(geometric_grid(nb, int(round(1.25 * nb)), n_pv, n_load,
                                    n_sh, seed * 1000 + k))
    return grids


def with_parallel_branches(net: Network, n_par: int, seed: int) -> Network:
    """Copy of ``net`` with ``n_par`` extra branches parallel to existing ones
    (fresh parameters, sometimes reversed orientation)."""
    rng = np.random.default_rng(seed)
    pick = rng.choice(net.n_branch, size=n_par, replace=False)
    flip = rng.random(n_par) < 0.5
    f = np.where(flip, net.br_to[pick], net.br_from[pick])
    t = np.where(flip, net.br_from[pick], net.br_to[pick])
    r, x, b, tap, shift = _branch_params(rng, n_par, 0.5)
    cat = np.concatenate
    out = net.copy()
    out.br_from = _i32(cat([net.br_from, f]))
    out.br_to = _i32(cat([net.br_to, t]))
    out.br_r = cat([net.br_r, r])
    out.br_x = cat([net.br_x, x])
    out.br_b = cat([net.br_b, b])
    out.br_tap = cat([net.br_tap, tap])
    out.br_shift_deg = cat([net.br_shift_deg, shift])
    out.br_status = _i32(cat([net.br_status, np.ones(n_par)]))
    return out


def fill_zero_injection_buses(net: Network) -> Network:
    """Copy of ``net`` with a zero load added at every bus that has neither a
    load nor a generator, so that every bus row has an injection that a
    manufactured solution can set."""
    busy = np.zeros(net.n_bus, bool)
    busy[net.load_bus] = True
    busy[net.pv_bus] = True
    busy[net.slack_bus] = True
    add = np.nonzero(~busy)[0]
    out = net.copy()
    out.load_bus = _i32(np.concatenate([net.load_bus, add]))
    out.load_p = np.concatenate([net.load_p, np.zeros(add.size)])
    out.load_q = np.concatenate([net.load_q, np.zeros(add.size)])
    return out


def grid_meshed(n_bus: int, seed: int, mesh: float = 2.5, rx=(0.05, 0.3)) -> Network:
    """A well-meshed, transmission-like variant of the geometric grid for
    the fast decoupled method: ``mesh * n_bus`` branches (the MST plus the
    shortest remaining Delaunay edges, so no long thin corridors remain) and
    resistances r = x * U(rx) (R/X well below 1, where decoupling holds);
    other data as :func:`geometric_grid` with the 70k proportions."""
    n_pv, n_load, n_sh = _fractions(n_bus)
    net = geometric_grid(n_bus, int(round(mesh * n_bus)), n_pv, n_load, n_sh, seed)
    rng = np.random.default_rng(seed + 1)
    net.br_r = net.br_x * rng.uniform(rx[0], rx[1], net.n_branch)
    return net
