"""Pins of the oracle's Elias-Fano store and edge codes.

* A list worked out by hand from the definitions (tests/golden/ef_example.txt):
  every bit of H and L, the quantum indexes and ranks.
* select(i) is the i-th input value and rank(x) counts the values strictly
  below x (the paper's modified rank), against numpy on random lists.
* l = floor(log2(u / n)) and the total H + L bits stay within the paper's bound
  2n + n ceil(log2(u / n)).
* The quantum indexes point at the (j q)-th one / zero, counted with numpy.
* Edge codes of a graph: decoding select(i) gives back the CSR source and
  destination of entry i; the paper's degree formula
  d(a) = rank(phi(a+1, 0)) - rank(phi(a, 0)) and neighbour formula
  N(a) = {select(i) & (2^k - 1)} reproduce the CSR rows.
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "ef_example.txt")


def _bits(words, nbits):
    w = np.asarray(words, dtype=np.uint64)
    b = ((w[:, None] >> np.arange(64, dtype=np.uint64)) & np.uint64(1)).astype(np.uint8).reshape(-1)
    return b[:nbits]


def _golden():
    g = {}
    for line in open(GOLDEN):
        if line.startswith("#") or ":" not in line:
            continue
        k, v = line.split(":", 1)
        g[k.strip()] = v.strip()
    return g


def test_hand_worked_example():
    g = _golden()
    vals = [int(x) for x in g["values"].split()]
    ef = oracle.ef_encode(vals, int(g["u"]), q=int(g["q"]))
    assert ef["l"] == int(g["l"]) and ef["n_zeros"] == int(g["n_zeros"]) and ef["h_bits"] == int(g["h_bits"])
    assert "".join(map(str, _bits(ef["H"], ef["h_bits"]))) == g["H"]
    assert "".join(map(str, _bits(ef["L"], len(vals) * ef["l"]))) == g["L"]
    assert list(ef["S1"]) == [int(x) for x in g["S1"].split()]
    assert list(ef["S0"]) == [int(x) for x in g["S0"].split()]
    for kv in g["rank"].split():
        x, r = kv.split(":")
        assert oracle.ef_rank(ef, int(x)) == int(r)
    assert [oracle.ef_select(ef, i) for i in range(len(vals))] == vals


@pytest.mark.parametrize("seed", range(6))
def test_select_rank_random_lists(seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(1, 300))
    u = int(rng.choice([m, m + 1, 2 * m, 1000, 2**20, 2**40 + 3, 2**62]))
    y = np.sort(rng.integers(0, u, size=m, dtype=np.uint64))
    if seed == 0:
        y[:5] = y[0]  # repeated values are allowed in a non-decreasing list
        y.sort()
    q = int(rng.choice([1, 2, 3, 64]))
    ef = oracle.ef_encode(y, u, q=q)
    assert [oracle.ef_select(ef, i) for i in range(m)] == [int(v) for v in y]
    xs = set(int(v) for v in y) | set(int(v) + 1 for v in y) | {0, u} | set(
        int(v) for v in rng.integers(0, u, size=50, dtype=np.uint64))
    for x in xs:
        assert oracle.ef_rank(ef, x) == int(np.searchsorted(y, np.uint64(x), side="left")), x


@pytest.mark.parametrize("m,u", [(1, 1), (7, 25), (5, 5), (3, 1000), (1000, 2**40), (64, 2**62), (100, 640),
                                 (100, 641), (100, 1279)])
def test_low_bits_and_size_bound(m, u):
    y = np.sort(np.random.default_rng(m).integers(0, u, size=m, dtype=np.uint64))
    ef = oracle.ef_encode(y, u)
    assert ef["l"] == math.floor(math.log2(u / m)) if u >= m * 2 else ef["l"] == 0
    assert ef["l"] == max(0, int(math.floor(math.log2(u / m) + 1e-12)))
    total = ef["h_bits"] + m * ef["l"]
    assert total <= 2 * m + m * math.ceil(math.log2(u / m)) if u > m else total <= 2 * m + 1
    assert int(_bits(ef["H"], ef["h_bits"]).sum()) == m


@pytest.mark.parametrize("q", [1, 2, 5, 64, 1024])
def test_quantum_indexes(q):
    rng = np.random.default_rng(q)
    u = 5000
    y = np.sort(rng.integers(0, u, size=1500, dtype=np.uint64))
    ef = oracle.ef_encode(y, u, q=q)
    bits = _bits(ef["H"], ef["h_bits"]).astype(np.int64)
    ones_before = np.concatenate([[0], np.cumsum(bits)])
    zeros_before = np.arange(bits.size + 1) - ones_before
    assert len(ef["S1"]) == -(-1500 // q) and len(ef["S0"]) == -(-ef["n_zeros"] // q)
    for j, p in enumerate(ef["S1"]):
        assert bits[p] == 1 and ones_before[p] == j * q
    for j, p in enumerate(ef["S0"]):
        assert bits[p] == 0 and zeros_before[p] == j * q


def _graph_checks(O, D, q):
    n = len(O) - 1
    ef = oracle.ef_encode_graph(O, D, q=q)
    k = ef["k"]
    assert (1 << k) >= n and (k == 0 or (1 << (k - 1)) < n)
    src = np.repeat(np.arange(n), np.diff(O.astype(np.int64)))
    codes = [oracle.ef_select(ef, i) for i in range(len(D))]
    assert [c >> k for c in codes] == list(src)
    assert [c & ((1 << k) - 1) for c in codes] == list(D)
    assert all(a < b for a, b in zip(codes, codes[1:]))  # distinct edges give a strictly increasing list
    for a in range(n):
        lo, hi = oracle.ef_rank(ef, a << k), oracle.ef_rank(ef, (a + 1) << k)
        assert hi - lo == O[a + 1] - O[a]
        assert [oracle.ef_select(ef, i) & ((1 << k) - 1) for i in range(lo, hi)] == list(D[O[a]:O[a + 1]])
    return ef


@pytest.mark.parametrize("name", sorted(synth.TINY))
def test_edge_codes_tiny_catalogue(name):
    O, D, W = synth.TINY[name]()
    _graph_checks(O, D, 2)


def test_edge_codes_random_graphs():
    rng = np.random.default_rng(3)
    for _ in range(25):
        O, D, W = synth.random_small(rng, n_max=40)
        _graph_checks(O, D, int(rng.choice([1, 4, 1024])))


def test_edge_codes_single_node_and_empty():
    ef = _graph_checks(np.array([0, 1], dtype=np.uint64), np.array([0], dtype=np.int32), 4)
    assert ef["k"] == 0 and ef["u"] == 1 and ef["l"] == 0
    ef = oracle.ef_encode_graph(np.zeros(4, dtype=np.uint64), np.zeros(0, dtype=np.int32))
    assert ef["m"] == 0 and oracle.ef_rank(ef, 3 << ef["k"]) == 0
