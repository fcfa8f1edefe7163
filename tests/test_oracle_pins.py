"""Pins of the CPU oracle against what the paper and mathematics fix.

* Exact transition tables: the oracle's biased weights, normalised, equal the
  node2vec transition probability of Eq. (1) computed from the graph distance
  d(t, x) (breadth-first search from t), for every ordered pair (t, v).
* Closed forms on stars, complete graphs, cycles and paths.
* Chi-square of sampled conditional frequencies against the exact tables, and
  of whole short walks against brute-force enumeration of all walks.
* The stationary law of first-order weighted walks (proportional to the
  weighted degree).
* Invariants: every step follows an edge, dead ends stop a walk, lengths,
  padding, determinism, walk-id chunking, scale invariance of the weights, and
  node2vec(p = q = 1) == first order.
"""
from collections import Counter, deque
from fractions import Fraction

import numpy as np
import pytest
from scipy.stats import chisquare

import oracle
import synth

DYADIC = [0.25, 0.5, 1.0, 2.0, 4.0]


def bfs_dist(O, D, t):
    """Directed breadth-first distances from t (out-edges)."""
    dist = {t: 0}
    dq = deque([t])
    while dq:
        u = dq.popleft()
        for e in range(int(O[u]), int(O[u + 1])):
            x = int(D[e])
            if x not in dist:
                dist[x] = dist[u] + 1
                dq.append(x)
    return dist


def exact_table(O, D, W, t, v, p, q):
    """pi(x | t, v) from Eq. (1): alpha = 1/p (d=0), 1 (d=1), 1/q (d=2)."""
    dist = bfs_dist(O, D, t)
    pf, qf = Fraction(p), Fraction(q)
    vals = []
    for e in range(int(O[v]), int(O[v + 1])):
        x = int(D[e])
        w = 1 if W is None else int(W[e])
        dd = dist[x]
        assert dd <= 2  # x is reached through v
        alpha = 1 / pf if dd == 0 else (Fraction(1) if dd == 1 else 1 / qf)
        vals.append(alpha * w)
    s = sum(vals)
    return [x / s for x in vals] if s else None


def oracle_table(O, D, W, t, v, p, q):
    b = oracle.step_weights(O, D, W, t, v, True, oracle.q16(p), oracle.q16(q))
    s = int(sum(int(x) for x in b))
    return [Fraction(int(x), s) for x in b] if s else None


def edges(O, D):
    for t in range(len(O) - 1):
        for e in range(int(O[t]), int(O[t + 1])):
            yield t, int(D[e])


@pytest.mark.parametrize("name", sorted(synth.TINY))
def test_exact_transition_tables(name):
    O, D, W = synth.TINY[name]()
    for p in DYADIC:
        for q in DYADIC:
            for t, v in edges(O, D):
                assert oracle_table(O, D, W, t, v, p, q) == exact_table(O, D, W, t, v, p, q), (t, v, p, q)


def test_exact_tables_fuzz():
    rng = np.random.default_rng(11)
    for _ in range(150):
        O, D, W = synth.random_small(rng, n_max=9)
        p = float(rng.choice(DYADIC))
        q = float(rng.choice(DYADIC))
        for t, v in edges(O, D):
            assert oracle_table(O, D, W, t, v, p, q) == exact_table(O, D, W, t, v, p, q)


def test_non_dyadic_parameters_within_q16_bound():
    """For p, q that Q16 cannot hold exactly, alpha is off by at most 2^-17
    absolute; the normalised probabilities stay within the matching bound."""
    O, D, W = synth.weighted_diamond()
    for p, q in [(3.0, 0.3), (0.7, 1.9), (10.0, 0.1)]:
        P16, Q16 = oracle.q16(p), oracle.q16(q)
        assert abs(Fraction(P16, 65536) - 1 / Fraction(p)) <= Fraction(1, 2**17)
        assert abs(Fraction(Q16, 65536) - 1 / Fraction(q)) <= Fraction(1, 2**17)
        for t, v in edges(O, D):
            a = oracle_table(O, D, W, t, v, p, q)
            e = exact_table(O, D, W, t, v, p, q)
            for x, y in zip(a, e):
                assert abs(float(x - y)) < 1e-4


def test_q16_conversion():
    assert [oracle.q16(x) for x in DYADIC] == [262144, 131072, 65536, 32768, 16384]
    assert oracle.q16(3.0) == 21845  # 21845.33 rounds down
    assert oracle.q16(65536.0) == 1
    assert oracle.q16(65536.0 / 4294967295.0) == 4294967295
    for bad in [0.0, -1.0, float("nan"), float("inf"), 131072.0, 1e-6]:
        with pytest.raises(oracle.OracleError):
            oracle.q16(bad)


# --------------------------------------------------------------------------
# Closed forms (unweighted): probability of returning to t
# --------------------------------------------------------------------------
def p_return(O, D, t, v, p, q):
    tab = oracle_table(O, D, None, t, v, p, q)
    row = [int(D[e]) for e in range(int(O[v]), int(O[v + 1]))]
    return tab[row.index(t)]


@pytest.mark.parametrize("p", DYADIC)
@pytest.mark.parametrize("q", DYADIC)
def test_closed_forms(p, q):
    P, Q = Fraction(p), Fraction(q)
    k = 6
    O, D, _ = synth.star(k)  # leaf 1 -> centre 0 -> x: k-1 far leaves
    assert p_return(O, D, 1, 0, p, q) == (1 / P) / (1 / P + (k - 1) / Q)
    n = 6
    O, D, _ = synth.complete(n)  # every other neighbour is common
    assert p_return(O, D, 0, 1, p, q) == (1 / P) / (1 / P + (n - 2))
    O, D, _ = synth.cycle(7)  # one return, one far
    assert p_return(O, D, 0, 1, p, q) == (1 / P) / (1 / P + 1 / Q)
    O, D, _ = synth.path(6)
    assert p_return(O, D, 1, 2, p, q) == (1 / P) / (1 / P + 1 / Q)
    assert p_return(O, D, 4, 5, p, q) == 1  # leaf: forced return


# --------------------------------------------------------------------------
# Sampled frequencies vs exact tables (chi-square, threshold fixed at 1e-6)
# --------------------------------------------------------------------------
def _chi2(counts: Counter, probs: dict, n: int):
    keys = sorted(probs)
    obs = np.array([counts.get(k, 0) for k in keys], dtype=np.float64)
    exp = np.array([float(probs[k]) * n for k in keys])
    assert sum(counts.values()) == n
    assert all(k in probs for k in counts)  # nothing sampled with probability 0
    keep = exp > 0
    if keep.sum() <= 1:
        return 1.0
    return chisquare(obs[keep], exp[keep]).pvalue


@pytest.mark.parametrize("name,start,p,q", [
    ("two_tri", 0, 0.25, 4.0), ("wdiamond", 1, 2.0, 0.5), ("wdiamond", 3, 0.5, 2.0),
    ("tri_tail", 2, 4.0, 0.25), ("selfloop", 1, 0.5, 4.0), ("k5", 0, 2.0, 0.5),
])
def test_second_step_frequencies(name, start, p, q):
    O, D, W = synth.TINY[name]()
    nw = 200_000
    Y, lens = oracle.walks(O, D, W, [start], nw, 3, oracle.NODE2VEC, p, q, seed=99)
    assert np.all(lens == 3)
    # first step: first-order weighted from the start
    row = [int(D[e]) for e in range(int(O[start]), int(O[start + 1]))]
    wts = [1 if W is None else int(W[e]) for e in range(int(O[start]), int(O[start + 1]))]
    p1 = {x: Fraction(w, sum(wts)) for x, w in zip(row, wts)}
    assert _chi2(Counter(Y[:, 1].tolist()), p1, nw) > 1e-6
    # second step, conditional on the first
    for v in row:
        sel = Y[:, 1] == v
        tab = exact_table(O, D, W, start, v, p, q)
        nb = [int(D[e]) for e in range(int(O[v]), int(O[v + 1]))]
        probs = dict(zip(nb, tab))
        assert _chi2(Counter(Y[sel, 2].tolist()), probs, int(sel.sum())) > 1e-6


def _enumerate_walks(O, D, W, start, L, p, q):
    """All walks of L slots from start with exact probabilities; the first step
    is first-order (weights only), later steps follow Eq. (1)."""
    out = {}

    def rec(seq, prob):
        if len(seq) == L:
            out[tuple(seq)] = out.get(tuple(seq), 0) + prob
            return
        v = seq[-1]
        lo, hi = int(O[v]), int(O[v + 1])
        if len(seq) == 1:
            w = [1 if W is None else int(W[e]) for e in range(lo, hi)]
            s = sum(w)
            probs = [Fraction(x, s) for x in w] if s else None
        else:
            probs = exact_table(O, D, W, seq[-2], v, p, q)
        if hi == lo or probs is None:
            out[tuple(seq)] = out.get(tuple(seq), 0) + prob  # stopped early
            return
        for e, pr in zip(range(lo, hi), probs):
            if pr:
                rec(seq + [int(D[e])], prob * pr)

    rec([start], Fraction(1))
    return out


@pytest.mark.parametrize("name,start,p,q,L", [
    ("two_tri", 4, 0.5, 2.0, 5), ("wdiamond", 0, 0.25, 4.0, 5), ("dag", 0, 2.0, 0.5, 4),
    ("zerow", 0, 4.0, 0.25, 5), ("selfloop", 3, 1.0, 2.0, 5),
])
def test_whole_walks_brute_force(name, start, p, q, L):
    O, D, W = synth.TINY[name]()
    probs = _enumerate_walks(O, D, W, start, L, p, q)
    assert sum(probs.values()) == 1
    nw = 200_000
    Y, lens = oracle.walks(O, D, W, [start], nw, L, oracle.NODE2VEC, p, q, seed=3)
    seqs = Counter(tuple(int(x) for x in r[:ln]) for r, ln in zip(Y, lens))
    assert _chi2(seqs, probs, nw) > 1e-6


def test_stationary_first_order_weighted():
    """Long first-order weighted walks on a connected non-bipartite graph visit
    v with frequency S_v / sum(S) (S_v = weighted degree)."""
    O, D, W = synth.weighted_diamond()
    n = len(O) - 1
    S = np.array([int(W[int(O[v]):int(O[v + 1])].sum()) for v in range(n)], dtype=np.float64)
    Y, _ = oracle.walks(O, D, W, list(range(n)), 2000, 120, oracle.FIRST_ORDER, seed=8)
    visits = np.bincount(Y[:, 40:].ravel(), minlength=n)
    freq = visits / visits.sum()
    assert np.allclose(freq, S / S.sum(), rtol=0.02)


# --------------------------------------------------------------------------
# Invariants
# --------------------------------------------------------------------------
def _check_invariants(O, D, W, starts, Y, lens, L):
    n = len(O) - 1
    adj = {v: set(int(x) for x in D[int(O[v]):int(O[v + 1])]) for v in range(n)}
    wmap = {}
    for v in range(n):
        for e in range(int(O[v]), int(O[v + 1])):
            wmap[(v, int(D[e]))] = 1 if W is None else int(W[e])
    ns = len(starts)
    for w in range(Y.shape[0]):
        st = int(starts[w % ns])
        ln = int(lens[w])
        if st < 0 or st >= n:
            assert ln == 0 and np.all(Y[w] == -1)
            continue
        assert 1 <= ln <= L and Y[w, 0] == st
        assert np.all(Y[w, ln:] == -1)
        for s in range(1, ln):
            a, b = int(Y[w, s - 1]), int(Y[w, s])
            assert b in adj[a] and wmap[(a, b)] > 0
        if ln < L:
            last = int(Y[w, ln - 1])
            row_w = [wmap[(last, x)] for x in adj[last]]
            assert sum(row_w) == 0  # only a dead end (or all-zero row) stops a walk


@pytest.mark.parametrize("kind", [oracle.FIRST_ORDER, oracle.NODE2VEC])
def test_invariants_fuzz(kind):
    rng = np.random.default_rng(21 + kind)
    for it in range(60):
        O, D, W = synth.random_small(rng, n_max=10)
        n = len(O) - 1
        starts = rng.integers(-2, n + 2, size=int(rng.integers(1, 6)))
        L = int(rng.integers(1, 13))
        reps = int(rng.integers(1, 4))
        p, q = float(rng.choice(DYADIC + [3.0])), float(rng.choice(DYADIC + [0.3]))
        Y, lens = oracle.walks(O, D, W, starts, reps, L, kind, p, q, seed=it)
        assert Y.shape == (len(starts) * reps, L)
        _check_invariants(O, D, W, starts, Y, lens, L)
        # determinism
        Y2, l2 = oracle.walks(O, D, W, starts, reps, L, kind, p, q, seed=it)
        assert np.array_equal(Y, Y2) and np.array_equal(lens, l2)


def test_walk_id_chunking_and_subsets():
    O, D, W = synth.weighted_diamond()
    starts = [0, 1, 2, 3, 4, 5, 2]
    Y, lens = oracle.walks(O, D, W, starts, 3, 9, oracle.NODE2VEC, 0.5, 2.0, seed=4, walk_id_base=100)
    # row w uses walk id base + w: rows [7..21) equal a run over the same
    # start list rotated... simplest check: subset rows reproduce the full run
    rows = [20, 0, 7, 13]
    Ys, ls = oracle.walks(O, D, W, starts, 3, 9, oracle.NODE2VEC, 0.5, 2.0, seed=4, walk_id_base=100, rows=rows)
    assert np.array_equal(Ys, Y[rows]) and np.array_equal(ls, lens[rows])
    # reps 1..2 with base 100 + 7 equal rows 7..21 of the base-100 run
    Yb, lb = oracle.walks(O, D, W, starts, 2, 9, oracle.NODE2VEC, 0.5, 2.0, seed=4, walk_id_base=107)
    assert np.array_equal(Yb, Y[7:]) and np.array_equal(lb, lens[7:])
    # a different seed or base changes the walks
    Yc, _ = oracle.walks(O, D, W, starts, 3, 9, oracle.NODE2VEC, 0.5, 2.0, seed=5, walk_id_base=100)
    assert not np.array_equal(Yc, Y)


def test_scale_invariance():
    """Unweighted == all-ones weights; weights * c == weights; node2vec with
    p = q = 1 == first order.  Bit-exact, because for integers B,
    B c > floor(r c S / 2^64) iff B > floor(r S / 2^64)."""
    rng = np.random.default_rng(31)
    for it in range(40):
        O, D, W = synth.random_small(rng, n_max=10, weighted=True, zero_weights=(it % 2 == 0))
        n = len(O) - 1
        starts = np.arange(n)
        L = 10
        base = oracle.walks(O, D, W, starts, 2, L, oracle.NODE2VEC, 2.0, 0.5, seed=it)
        c = int(rng.integers(2, 1000))
        scaled = oracle.walks(O, D, W * np.uint32(c), starts, 2, L, oracle.NODE2VEC, 2.0, 0.5, seed=it)
        assert np.array_equal(base[0], scaled[0])
        fo = oracle.walks(O, D, W, starts, 2, L, oracle.FIRST_ORDER, seed=it)
        n11 = oracle.walks(O, D, W, starts, 2, L, oracle.NODE2VEC, 1.0, 1.0, seed=it)
        assert np.array_equal(fo[0], n11[0]) and np.array_equal(fo[1], n11[1])
        ones = np.ones_like(W)
        uw = oracle.walks(O, D, None, starts, 2, L, oracle.NODE2VEC, 4.0, 0.25, seed=it)
        ow = oracle.walks(O, D, ones, starts, 2, L, oracle.NODE2VEC, 4.0, 0.25, seed=it)
        assert np.array_equal(uw[0], ow[0])


def test_dead_ends_and_edge_cases():
    O, D, W = synth.directed_dag()
    Y, lens = oracle.walks(O, D, W, [0, 3, 5, 6, -1], 1, 6, oracle.NODE2VEC, 2.0, 0.5, seed=1)
    assert lens[1] == 1 and Y[1, 0] == 3 and np.all(Y[1, 1:] == -1)  # sink start
    assert lens[3] == 0 and np.all(Y[3] == -1)  # start out of range
    assert lens[4] == 0
    assert lens[0] in (3, 4) and int(Y[0, lens[0] - 1]) in (3, 5)
    # L = 1: only the start
    Y, lens = oracle.walks(O, D, W, [0, 1], 1, 1, oracle.FIRST_ORDER, seed=1)
    assert Y.tolist() == [[0], [1]] and lens.tolist() == [1, 1]
    # zero-weight row stops the walk: node 4 of zerow has a single zero edge
    O, D, W = synth.zero_weight_graph()
    Y, lens = oracle.walks(O, D, W, [4], 3, 5, oracle.FIRST_ORDER, seed=2)
    assert lens.tolist() == [1, 1, 1]
    # empty request
    Y, lens = oracle.walks(O, D, W, [], 1, 5, oracle.FIRST_ORDER, seed=2)
    assert Y.shape == (0, 5)


def test_validation_and_overflow():
    O, D, _ = synth.cycle(5)
    assert oracle.validate(O, D) == oracle.OK
    D2 = D.copy()
    D2[0], D2[1] = D2[1], D2[0]
    assert oracle.validate(O, D2) == oracle.ERR_UNSORTED
    D3 = D.copy()
    D3[3] = 5
    assert oracle.validate(O, D3) == oracle.ERR_UNSORTED
    O4 = O.copy()
    O4[2] = O4[1] - 1
    assert oracle.validate(O4, D) == oracle.ERR_UNSORTED
    O5 = O.copy()
    O5[-1] += 1
    assert oracle.validate(O5, D) == oracle.ERR_UNSORTED
    # duplicate entry in a row (multi-edge) is rejected
    O6, D6, _ = synth.csr_from_edges(3, [0, 0, 1], [1, 1, 2], dedup=False)
    assert oracle.validate(O6, D6) == oracle.ERR_UNSORTED
    # overflow precondition: row sum * max(P16, C16, Q16) must fit in 64 bits
    O, D, _ = synth.star(3)
    W = np.full(D.size, 2**32 - 1, dtype=np.uint32)
    oracle.walks(O, D, W, [0], 1, 4, oracle.NODE2VEC, 1.0, 1.0)  # 3 * 2^32 * 2^16 fits
    with pytest.raises(oracle.OracleError) as e:
        O7, D7, _ = synth.star(70000)
        W7 = np.full(D7.size, 2**32 - 1, dtype=np.uint32)
        oracle.walks(O7, D7, W7, [0], 1, 4, oracle.NODE2VEC, 1.0 / 65536.0 * 2, 1.0)
    assert e.value.code == oracle.ERR_OVERFLOW
