"""Pins of the oracle's approximated walks (Methods, "Approximated RWs"):
Sorted Unique Sub-Sampling of k neighbours when the degree exceeds k.

* structure: k sorted, unique positions, one per bucket of length floor(d/k),
  the last bucket taking the remainder;
* uniformity: the paper's experiment (1e7 sampled integers over a range of
  1e4), here as a chi-square of every position's count against its exact
  inclusion probability 1 / (its bucket's length);
* k >= degree: identical to the exact walk;
* exact transition tables of the approximated step, by enumerating every
  sub-sample (each bucket uniform and independent) on small rows, against
  sampled frequencies.
"""
from collections import Counter
from fractions import Fraction
from itertools import product

import numpy as np
import pytest
from scipy.stats import chisquare

import oracle
import synth
from tests.test_oracle_pins import exact_table


@pytest.mark.parametrize("d,k", [(10, 3), (7, 2), (100, 7), (65, 64), (10_000, 100), (5, 4)])
def test_suss_structure(d, k):
    b = d // k
    for s in range(40):
        pos = oracle.suss(11, s, 1000 + s, d, k).astype(np.int64)
        assert pos.size == k and np.all(np.diff(pos) > 0)
        for i, x in enumerate(pos):
            lo = i * b
            hi = (i + 1) * b if i + 1 < k else d
            assert lo <= x < hi


def test_suss_uniform_like_the_papers_experiment():
    """1e7 integers over [0, 1e4): 1e5 sub-samples of k = 100."""
    d, k, reps = 10_000, 100, 100_000
    counts = np.zeros(d, dtype=np.int64)
    for r in range(reps):
        counts[oracle.suss(7, 1 + r % 1000, r, d, k)] += 1
    assert counts.sum() == d // (d // k) * reps
    expected = np.full(d, reps / (d // k), dtype=np.float64)  # every bucket has length 100
    assert chisquare(counts, expected).pvalue > 1e-6


def test_suss_remainder_bucket():
    d, k, reps = 23, 4, 40_000  # buckets of 5, 5, 5 and 8
    counts = np.zeros(d, dtype=np.int64)
    for r in range(reps):
        counts[oracle.suss(3, 5, r, d, k)] += 1
    lens = [5] * 15 + [8] * 8
    expected = np.array([reps / l for l in lens])
    assert chisquare(counts, expected).pvalue > 1e-6


@pytest.mark.parametrize("name", sorted(synth.TINY))
def test_k_at_least_degree_is_exact(name):
    O, D, W = synth.TINY[name]()
    n = len(O) - 1
    kmax = int((O[1:] - O[:-1]).max()) if n else 1
    starts = list(range(n))
    for kind, p, q in [(oracle.FIRST_ORDER, 1.0, 1.0), (oracle.NODE2VEC, 0.25, 4.0), (oracle.NODE2VEC, 2.0, 1.0)]:
        ex = oracle.walks(O, D, W, starts, 3, 9, kind, p, q, seed=5)
        ap = oracle.walks(O, D, W, starts, 3, 9, kind, p, q, seed=5, k_approx=max(kmax, 1))
        assert np.array_equal(ex[0], ap[0]) and np.array_equal(ex[1], ap[1])


def approx_table(O, D, W, t, v, p, q, k):
    """Exact distribution of the approximated step from v (previous t)."""
    d = int(O[v + 1] - O[v])
    if d <= k:
        return exact_table(O, D, W, t, v, p, q)
    full = exact_table(O, D, W, t, v, p, q)  # proportional weights, normalised over N(v)
    b = d // k
    buckets = [range(i * b, (i + 1) * b if i + 1 < k else d) for i in range(k)]
    out = [Fraction(0)] * d
    combos = list(product(*buckets))
    for combo in combos:
        tot = sum(full[j] for j in combo)
        if tot == 0:
            continue
        for j in combo:
            out[j] += full[j] / tot / len(combos)
    return out


@pytest.mark.parametrize("k", [2, 3])
def test_approximated_step_frequencies(k):
    O, D, W = synth.star(7)  # centre 0 has degree 7
    # first step from leaf 1 goes to 0; second step from 0 is approximated
    nw, p, q = 120_000, 0.5, 2.0
    Y, lens = oracle.walks(O, D, W, [1], nw, 3, oracle.NODE2VEC, p, q, seed=21, k_approx=k)
    assert np.all(Y[:, 1] == 0)
    tab = approx_table(O, D, W, 1, 0, p, q, k)
    assert sum(tab) == 1
    row = [int(x) for x in D[int(O[0]):int(O[1])]]
    probs = dict(zip(row, tab))
    c = Counter(Y[:, 2].tolist())
    obs = np.array([c.get(x, 0) for x in row], dtype=np.float64)
    exp = np.array([float(probs[x]) * nw for x in row])
    assert chisquare(obs, exp).pvalue > 1e-6


def test_approximated_weighted_frequencies():
    O, D, W = synth.weighted_diamond()  # node 2 has degree 4, node 1 degree 3
    nw, p, q, k = 120_000, 0.25, 4.0, 2
    Y, lens = oracle.walks(O, D, W, [0], nw, 3, oracle.NODE2VEC, p, q, seed=4, k_approx=k)
    for v in (1, 2):
        sel = Y[:, 1] == v
        tab = approx_table(O, D, W, 0, v, p, q, k)
        row = [int(x) for x in D[int(O[v]):int(O[v + 1])]]
        c = Counter(Y[sel, 2].tolist())
        obs = np.array([c.get(x, 0) for x in row], dtype=np.float64)
        exp = np.array([float(pr) * int(sel.sum()) for pr in tab])
        keep = exp > 0
        assert all(c.get(x, 0) == 0 for x, e in zip(row, exp) if e == 0)
        assert chisquare(obs[keep], exp[keep]).pvalue > 1e-6


def test_approximated_invariants():
    rng = np.random.default_rng(3)
    for it in range(30):
        O, D, W = synth.random_small(rng, n_max=12)
        n = len(O) - 1
        starts = rng.integers(0, n, size=4)
        k = int(rng.integers(1, 5))
        Y, lens = oracle.walks(O, D, W, starts, 2, 10, oracle.NODE2VEC, 2.0, 0.5, seed=it, k_approx=k)
        for w in range(Y.shape[0]):
            for s in range(1, int(lens[w])):
                a, b = int(Y[w, s - 1]), int(Y[w, s])
                assert b in set(int(x) for x in D[int(O[a]):int(O[a + 1])])


def test_suss_buckets_independent():
    """Offsets within adjacent buckets are independent (every bucket has its own
    64-bit draw): chi-square of the joint offsets of buckets (0,1) and (1,2)."""
    d, k, reps = 40, 8, 60_000  # buckets of 5
    j01 = np.zeros((5, 5), dtype=np.int64)
    j12 = np.zeros((5, 5), dtype=np.int64)
    for r in range(reps):
        pos = oracle.suss(9, 3, r, d, k).astype(np.int64)
        off = pos - np.arange(k) * 5
        j01[off[0], off[1]] += 1
        j12[off[1], off[2]] += 1
    for j in (j01, j12):
        assert chisquare(j.ravel(), np.full(25, reps / 25)).pvalue > 1e-6
