"""Seeded synthetic graphs and walk requests.

This module only builds inputs: sorted CSR graphs (offsets uint64[n+1],
destinations int32[m], optional weights uint32[m]) and request lists.  It holds
none of the walk arithmetic.  Both the CPU oracle and the GPU library take
what it returns, so a test hands the same arrays to each side.

Workload shapes stand in for the paper's real graphs (power-law degree
distributions with hubs, one walk of about 80-100 steps from every node); the
paper's datasets are not used.
"""
from __future__ import annotations

import math

import numpy as np


# --------------------------------------------------------------------------
# CSR construction
# --------------------------------------------------------------------------
def csr_from_edges(n: int, src, dst, w=None, symmetric: bool = False, dedup: bool = True):
    """Build a sorted CSR from an edge list.

    symmetric: add the reverse of every edge (same weight).
    dedup: drop repeated (src, dst) pairs, keeping the first weight.
    Returns (offsets uint64[n+1], dst int32[m], weights uint32[m] or None)."""
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    ww = None if w is None else np.asarray(w, dtype=np.uint32)
    if symmetric:
        src, dst = np.concatenate([src, dst]), np.concatenate([dst, src])
        if ww is not None:
            ww = np.concatenate([ww, ww])
    key = src * np.int64(n) + dst
    order = np.argsort(key, kind="stable")
    key = key[order]
    if dedup and key.size:
        keep = np.ones(key.size, dtype=bool)
        keep[1:] = key[1:] != key[:-1]
        order = order[keep]
        key = key[keep]
    s = (key // n).astype(np.int64)
    d = (key % n).astype(np.int32)
    counts = np.bincount(s, minlength=n).astype(np.uint64)
    O = np.zeros(n + 1, dtype=np.uint64)
    np.cumsum(counts, out=O[1:])
    W = None if ww is None else np.ascontiguousarray(ww[order])
    return O, np.ascontiguousarray(d), W


def degrees(O):
    O = np.asarray(O, dtype=np.uint64)
    return (O[1:] - O[:-1]).astype(np.int64)


def degree_stats(O) -> dict:
    d = degrees(O).astype(np.float64)
    s1 = float(d.sum())
    return {
        "n": int(d.size),
        "m": int(s1),
        "max_deg": int(d.max()) if d.size else 0,
        "isolated": int((d == 0).sum()),
        "sum_d2_over_sum_d": float((d * d).sum() / s1) if s1 else 0.0,
    }


# --------------------------------------------------------------------------
# Tiny graphs with known closed forms
# --------------------------------------------------------------------------
def _und(n, edges, w=None):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    return csr_from_edges(n, e[:, 0], e[:, 1], w, symmetric=True)


def star(k: int):
    """Centre 0 with leaves 1..k."""
    return _und(k + 1, [(0, i) for i in range(1, k + 1)])


def path(n: int):
    return _und(n, [(i, i + 1) for i in range(n - 1)])


def cycle(n: int):
    return _und(n, [(i, (i + 1) % n) for i in range(n)])


def complete(n: int):
    return _und(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


def triangle_with_tail():
    """Triangle 0-1-2 plus tail 2-3-4."""
    return _und(5, [(0, 1), (1, 2), (0, 2), (2, 3), (3, 4)])


def two_triangles():
    """Triangles 0-1-2 and 1-2-3 sharing edge 1-2, plus pendant 3-4."""
    return _und(5, [(0, 1), (0, 2), (1, 2), (1, 3), (2, 3), (3, 4)])


def weighted_diamond():
    """A weighted undirected graph with return, common and far candidates."""
    edges = [(0, 1), (0, 2), (1, 2), (1, 3), (2, 3), (3, 4), (2, 5), (4, 5)]
    w = [3, 1, 7, 2, 5, 4, 6, 1]
    return _und(6, edges, w)


def directed_dag():
    """Directed graph with sinks (3 and 5) and a node (4) only reachable."""
    src = [0, 0, 1, 1, 2, 4]
    dst = [1, 2, 2, 3, 3, 5]
    return csr_from_edges(6, src, dst)


def self_loop_graph():
    """Undirected triangle 0-1-2 with a self-loop on 1 and a pendant 2-3."""
    # both directions listed by hand; the self-loop is stored once
    src = [0, 1, 1, 2, 0, 2, 2, 3, 1]
    dst = [1, 0, 2, 1, 2, 0, 3, 2, 1]
    return csr_from_edges(4, src, dst)


def zero_weight_graph():
    """Weighted undirected graph with zero-weight edges; node 4's only edge has
    weight zero, so a walk that reaches it stops (total weight zero)."""
    edges = [(0, 1), (1, 2), (0, 2), (2, 3), (3, 4)]
    w = [5, 0, 2, 3, 0]
    return _und(5, edges, w)


TINY = {
    "star5": lambda: star(5),
    "path6": lambda: path(6),
    "cycle7": lambda: cycle(7),
    "k5": lambda: complete(5),
    "tri_tail": triangle_with_tail,
    "two_tri": two_triangles,
    "wdiamond": weighted_diamond,
    "dag": directed_dag,
    "selfloop": self_loop_graph,
    "zerow": zero_weight_graph,
}


# --------------------------------------------------------------------------
# Random small graphs (fuzzing)
# --------------------------------------------------------------------------
def random_small(rng: np.random.Generator, n_max: int = 12, directed: bool | None = None,
                 weighted: bool | None = None, self_loops: bool = True, zero_weights: bool = True):
    n = int(rng.integers(1, n_max + 1))
    if directed is None:
        directed = bool(rng.integers(0, 2))
    if weighted is None:
        weighted = bool(rng.integers(0, 2))
    dens = float(rng.uniform(0.05, 0.8))
    pairs = [(i, j) for i in range(n) for j in range(n) if (self_loops or i != j)]
    if not directed:
        pairs = [(i, j) for (i, j) in pairs if i <= j]
    pick = [pr for pr in pairs if rng.random() < dens]
    if not pick:
        return csr_from_edges(n, [], [], [] if weighted else None)
    e = np.asarray(pick, dtype=np.int64)
    w = None
    if weighted:
        w = rng.integers(0 if zero_weights else 1, 10, size=e.shape[0]).astype(np.uint32)
    if directed:
        return csr_from_edges(n, e[:, 0], e[:, 1], w)
    # undirected: self-loops stored once
    loops = e[:, 0] == e[:, 1]
    src = np.concatenate([e[:, 0], e[~loops, 1]])
    dst = np.concatenate([e[:, 1], e[~loops, 0]])
    ww = None if w is None else np.concatenate([w, w[~loops]])
    return csr_from_edges(n, src, dst, ww)


# --------------------------------------------------------------------------
# Barabasi-Albert preferential attachment
# --------------------------------------------------------------------------
def barabasi_albert(n: int, m: int, seed: int):
    """Undirected BA graph: start from a star on m+1 nodes (centre 0), then each
    new node attaches to m distinct existing nodes chosen with probability
    proportional to their degree.  Connected; no self-loops or multi-edges."""
    rng = np.random.default_rng(seed)
    src = [0] * m
    dst = list(range(1, m + 1))
    repeated = [0] * m + list(range(1, m + 1))  # each endpoint once per incident edge
    rep = np.empty(2 * m * n + 2 * m, dtype=np.int64)
    rep[: len(repeated)] = repeated
    nrep = len(repeated)
    for v in range(m + 1, n):
        chosen = set()
        while len(chosen) < m:
            k = int(rng.integers(0, nrep))
            chosen.add(int(rep[k]))
        for u in sorted(chosen):
            src.append(v)
            dst.append(u)
            rep[nrep] = v
            rep[nrep + 1] = u
            nrep += 2
    return csr_from_edges(n, src, dst, symmetric=True)


# --------------------------------------------------------------------------
# Chung-Lu power-law graphs
# --------------------------------------------------------------------------
def chung_lu_weights(n: int, gamma: float, mean_deg: float, w_max: float) -> np.ndarray:
    """Expected-degree sequence w_i = c (i + i0)^(-1/(gamma-1)) with w_0 = w_max
    and mean(w) = mean_deg (i0 found by bisection)."""
    beta = 1.0 / (gamma - 1.0)
    i = np.arange(n, dtype=np.float64)

    def mean_for(i0):
        c = w_max * i0 ** beta
        return float((c * (i + i0) ** (-beta)).mean())

    lo, hi = 1e-9, float(n) * 10
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if mean_for(mid) > mean_deg:
            hi = mid  # larger i0 flattens the sequence and lowers the mean
        else:
            lo = mid
        if hi / lo < 1 + 1e-12:
            break
    i0 = math.sqrt(lo * hi)
    c = w_max * i0 ** beta
    return c * (i + i0) ** (-beta)


def chung_lu(n: int, n_edges: int, gamma: float, mean_deg: float, w_max: float,
             wrange=(1, 100), seed: int = 0, relabel: bool = True, weighted: bool = True):
    """Undirected Chung-Lu graph: n_edges endpoint pairs sampled proportionally to
    the expected-degree sequence, self-loops and duplicates dropped, stored
    symmetrically with one uniform integer weight per undirected edge.
    Node ids are randomly relabelled (seeded)."""
    rng = np.random.default_rng(seed)
    w = chung_lu_weights(n, gamma, mean_deg, w_max)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    chunk = 1 << 23
    keys = []
    for off in range(0, n_edges, chunk):
        k = min(chunk, n_edges - off)
        a = np.searchsorted(cdf, rng.random(k), side="right")
        b = np.searchsorted(cdf, rng.random(k), side="right")
        np.minimum(a, n - 1, out=a)
        np.minimum(b, n - 1, out=b)
        lo = np.minimum(a, b).astype(np.uint64)
        hi = np.maximum(a, b).astype(np.uint64)
        keep = lo != hi
        keys.append((lo[keep] << np.uint64(32)) | hi[keep])
    key = np.unique(np.concatenate(keys))
    del keys
    lo = (key >> np.uint64(32)).astype(np.int64)
    hi = (key & np.uint64(0xFFFFFFFF)).astype(np.int64)
    del key
    ew = None
    if weighted:
        ew = rng.integers(wrange[0], wrange[1] + 1, size=lo.size).astype(np.uint32)
    if relabel:
        perm = rng.permutation(n).astype(np.int64)
        lo, hi = perm[lo], perm[hi]
    return csr_from_edges(n, lo, hi, ew, symmetric=True, dedup=False)


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------
def ba_10k():
    """10,000-node Barabasi-Albert graph, m = 5, generator seed 42, unweighted."""
    return barabasi_albert(10_000, 5, 42)


def chung_lu_1m():
    """1M nodes, 10M undirected edge samples, degree exponent 2.2, mean degree 20,
    max expected degree 5e4, weights uniform in [1, 100], seed 2."""
    return chung_lu(1_000_000, 10_000_000, 2.2, 20.0, 5.0e4, (1, 100), seed=2)


# --------------------------------------------------------------------------
# Many-graph, many-request workloads (batched and served forms)
# --------------------------------------------------------------------------
def many_graph_params(n_graphs: int = 64):
    """Graph g: n log-uniform in [1e3, 1e6], mean degree uniform in [8, 32],
    degree exponent 2.2, max expected degree sqrt(n * mean), weights U[1, 100],
    seed 100 + g."""
    out = []
    for g in range(n_graphs):
        rng = np.random.default_rng(100 + g)
        n = int(round(math.exp(rng.uniform(math.log(1e3), math.log(1e6)))))
        dbar = float(rng.uniform(8.0, 32.0))
        out.append(dict(n=n, n_edges=int(n * dbar / 2), mean_deg=dbar, w_max=math.sqrt(n * dbar), seed=100 + g))
    return out


def many_graph(params: dict):
    return chung_lu(params["n"], params["n_edges"], 2.2, params["mean_deg"], params["w_max"], (1, 100),
                    seed=params["seed"])


def many_graphs(n_graphs: int = 64, threads: int = 16):
    """Every graph of many_graph_params(), generated on host threads (numpy
    releases the GIL in its sorts and random fills), largest first.  Returns
    (params, [(O, D, W)] in graph order)."""
    import concurrent.futures as cf
    ps = many_graph_params(n_graphs)
    order = sorted(range(len(ps)), key=lambda g: -ps[g]["n"])
    with cf.ThreadPoolExecutor(max(1, threads)) as ex:
        got = dict(zip(order, ex.map(lambda g: many_graph(ps[g]), order)))
    return ps, [got[g] for g in range(len(ps))]


def many_requests(graph_nodes, n_requests: int = 4096, seed: int = 7, max_starts: int = 10_000):
    """Request k: graph uniform, 1..max_starts start nodes drawn uniformly with
    replacement, walk length uniform in [10, 200], (p, q) uniform over
    {0.25, 1, 4}^2, one walk per start, Philox seed 1000 + k."""
    rng = np.random.default_rng(seed)
    grid = [0.25, 1.0, 4.0]
    reqs = []
    for k in range(n_requests):
        g = int(rng.integers(0, len(graph_nodes)))
        ns = int(rng.integers(1, max_starts + 1))
        starts = rng.integers(0, graph_nodes[g], size=ns).astype(np.int32)
        reqs.append(dict(graph=g, starts=starts, walk_len=int(rng.integers(10, 201)),
                         p=grid[int(rng.integers(0, 3))], q=grid[int(rng.integers(0, 3))], seed=1000 + k))
    return reqs


def poisson_arrivals(n: int, rate: float, seed: int = 11) -> np.ndarray:
    """Open-loop arrival times (seconds from 0) of a Poisson process."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, size=n))


def chung_lu_device(n: int, n_edges: int, gamma: float, mean_deg: float, w_max: float, wrange=(1, 255),
                    seed: int = 0, device="cuda", chunk: int = 1 << 27, log=None):
    """The Chung-Lu construction of chung_lu(), run with torch on a GPU for
    graphs too large for host-side sorting (e.g. 1e9 edge samples).  Same
    recipe; the random stream is torch's (seeded), so the graph differs from
    the numpy version with the same seed.  Returns device tensors
    (offsets int64[n+1], dst int32[m], weights int32[m] holding uint32 values)."""
    import torch
    dev = torch.device(device)
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    if log:
        log("expected-degree sequence")
    w = torch.from_numpy(chung_lu_weights(n, gamma, mean_deg, w_max)).to(dev)
    cdf = torch.cumsum(w, 0)
    cdf /= cdf[-1].clone()
    del w
    keys = []
    for off in range(0, n_edges, chunk):
        k = min(chunk, n_edges - off)
        a = torch.searchsorted(cdf, torch.rand(k, generator=gen, device=dev, dtype=torch.float64), right=True)
        b = torch.searchsorted(cdf, torch.rand(k, generator=gen, device=dev, dtype=torch.float64), right=True)
        a.clamp_(max=n - 1)
        b.clamp_(max=n - 1)
        lo = torch.minimum(a, b)
        hi = torch.maximum(a, b)
        del a, b
        keep = lo != hi
        keys.append(((lo << 32) | hi)[keep])
        del lo, hi, keep
        if log:
            log(f"edge samples {off + k}")
    del cdf
    key = torch.unique(torch.cat(keys))  # sorted, duplicates dropped
    del keys
    if log:
        log(f"unique undirected edges {key.numel()}")
    lo = key >> 32
    hi = key & 0xFFFFFFFF
    del key
    ew = torch.randint(wrange[0], wrange[1] + 1, (lo.numel(),), generator=gen, device=dev, dtype=torch.int32)
    perm = torch.randperm(n, generator=gen, device=dev)
    lo = perm[lo]
    hi = perm[hi]
    del perm
    src = torch.cat([lo, hi])
    dst = torch.cat([hi, lo])
    del lo, hi
    ew = torch.cat([ew, ew])
    skey = (src << 32) | dst
    del dst
    skey, order = torch.sort(skey)
    if log:
        log("entries sorted")
    ew = ew[order]
    del order
    src = skey >> 32
    D = (skey & 0xFFFFFFFF).to(torch.int32)
    del skey
    counts = torch.bincount(src, minlength=n)
    del src
    O = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    torch.cumsum(counts, 0, out=O[1:])
    return O, D, ew
