"""Pins of the oracle's training contexts and scale-free negatives.

* SkipGram contexts: the pair multiset of a walk is symmetric, has
  sum_i min(i, w) + min(len-1-i, w) pairs, and equals an independent
  enumeration of all position pairs at distance <= w.
* Walklets of scale k (stride k) equal window-1 SkipGram pairs on the k
  subsequences y[r::k] of each walk (the corpus construction of the cited
  Walklets method).
* Negatives: node v is chosen by exactly ceil(O[v+1] 2^64/m) - ceil(O[v] 2^64/m)
  of the 2^64 draws (probability d_v / m); isolated nodes never; chi-square of
  frequencies against d_v / m.
"""
from collections import Counter

import numpy as np
from scipy.stats import chisquare

import oracle
import synth


def _walks():
    O, D, W = synth.weighted_diamond()
    Y, lens = oracle.walks(O, D, W, [0, 1, 2, 3, 4, 5, -1, 2], 2, 13, oracle.NODE2VEC, 0.5, 2.0, seed=3)
    return O, Y, lens


def test_skipgram_pairs_match_enumeration():
    O, Y, lens = _walks()
    for w in (1, 2, 5):
        C = oracle.contexts(Y, w)
        for r in range(Y.shape[0]):
            ln = int(lens[r])
            got = Counter()
            for i in range(Y.shape[1]):
                for c in C[r, i]:
                    if c >= 0:
                        got[(int(Y[r, i]), int(c))] += 1
            exp = Counter()
            for i in range(ln):
                for j in range(ln):
                    if i != j and abs(i - j) <= w:
                        exp[(int(Y[r, i]), int(Y[r, j]))] += 1
            assert got == exp
            assert sum(got.values()) == sum(min(i, w) + min(ln - 1 - i, w) for i in range(ln))
            assert got == Counter({(b, a): k for (a, b), k in got.items()})


def test_walklets_equal_skipgram_on_subsequences():
    O, Y, lens = _walks()
    for k in (2, 3, 4):
        C = oracle.contexts(Y, 1, stride=k)
        for r in range(Y.shape[0]):
            ln = int(lens[r])
            got = Counter()
            for i in range(ln):
                for c in C[r, i]:
                    if c >= 0:
                        got[(int(Y[r, i]), int(c))] += 1
            exp = Counter()
            for s0 in range(k):
                seq = [int(x) for x in Y[r, s0:ln:k]]
                sub = oracle.contexts(np.array([seq], dtype=np.int32), 1) if seq else np.empty((1, 0, 2), np.int32)
                for i, x in enumerate(seq):
                    for c in sub[0, i]:
                        if c >= 0:
                            exp[(x, int(c))] += 1
            assert got == exp


def test_negatives_interval_counts_and_frequencies():
    O, D, W = synth.star(6)  # degrees 6,1,1,1,1,1,1 ; m = 12
    O2 = np.concatenate([O, [O[-1]]]).astype(np.uint64)  # plus an isolated node 7
    m = int(O2[-1])
    for v in range(len(O2) - 1):
        lo, hi = int(O2[v]), int(O2[v + 1])
        count = -(-(hi << 64) // m) - (-(-(lo << 64) // m))
        # count the draws that land in v with the oracle's own scaling
        assert (count == 0) == (hi == lo)
    Y = np.zeros((4000, 25), dtype=np.int32)  # every position a valid centre
    N = oracle.negatives(O2, Y, 4, seed=9)
    c = np.bincount(N.ravel(), minlength=len(O2) - 1)
    assert c[-1] == 0  # the isolated node is never drawn
    deg = np.diff(O2.astype(np.int64))
    keep = deg > 0
    assert chisquare(c[keep], deg[keep] / m * N.size).pvalue > 1e-6


def test_negatives_exact_selection():
    O = np.array([0, 3, 3, 10, 11, 20], dtype=np.uint64)  # node 1 isolated
    m = 20
    Y = np.zeros((1, 400), dtype=np.int32)
    N = oracle.negatives(O, Y, 6, seed=5, walk_id_base=77)
    for i in range(400):
        for j in range(6):
            ctr = [i, 77, 0, 0x80000000 + j // 2]
            o = oracle.philox4x32_10(ctr, [5, 0])
            r64 = int(o[2 * (j % 2)]) | (int(o[2 * (j % 2) + 1]) << 32)
            T = (r64 * m) >> 64
            v = int(np.searchsorted(O, T, side="right")) - 1
            assert N[0, i, j] == v


def test_invalid_centres_are_padding():
    O, Y, lens = _walks()
    C = oracle.contexts(Y, 3)
    N = oracle.negatives(O, Y, 3, seed=1)
    inval = Y < 0
    assert np.all(C[inval] == -1) and np.all(N[inval] == -1)
