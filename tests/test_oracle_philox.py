"""Pins for the oracle's random-number source and sampling primitives.

Philox4x32-10 (Salmon et al., SC'11) is cross-checked against an independent
implementation (rocRAND's open-source philox4x32_10 engine, compiled and run
as a black box on the host), plus statistical smoke tests.  The uniform-value
scaling and the first-index-exceeding selection of the sampler (Methods,
"Efficient sampling for Node2Vec RWs", steps 3-4) are pinned by exact
interval counting over all 2^64 draws.
"""
import os
import shutil
import subprocess
from fractions import Fraction

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def rocrand_prog(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("hipcc / rocRAND headers not available")
    out = tmp_path_factory.mktemp("philox") / "philox_check"
    subprocess.check_call([hipcc, "-O1", "-o", str(out), os.path.join(HERE, "philox_rocrand_check.cpp")],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    return str(out)


def test_philox_matches_rocrand(rocrand_prog):
    rng = np.random.default_rng(1234)
    cases = []
    for i in range(200):
        seed = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        if i < 4:
            seed = [0, 42, 2**64 - 1, 0x243F6A8885A308D3][i]
        step = int(rng.integers(0, 2**32))
        wid_lo = int(rng.integers(0, 2**30))
        wid_hi = int(rng.integers(0, 2**32))
        if i % 3 == 0:
            step, wid_lo, wid_hi = int(rng.integers(0, 300)), int(rng.integers(0, 10**6)), 0
        cases.append((seed, step, wid_lo, wid_hi))
    # counter (step, wid_lo, wid_hi, 0) == engine position: subsequence wid_hi,
    # offset 4 * (step + wid_lo * 2^32)
    inp = "".join(f"{s} {wh} {4 * (st + (wl << 32))}\n" for (s, st, wl, wh) in cases)
    res = subprocess.run([rocrand_prog], input=inp, capture_output=True, text=True, check=True)
    lines = res.stdout.strip().splitlines()
    assert len(lines) == len(cases)
    for (seed, step, wl, wh), line in zip(cases, lines):
        ref = [int(x) for x in line.split()]
        got = oracle.philox4x32_10([step, wl, wh, 0], [seed & 0xFFFFFFFF, seed >> 32])
        assert [int(x) for x in got] == ref, (seed, step, wl, wh)
        r64 = oracle.draw64(seed, step, (wh << 32) | wl)
        assert r64 == ref[0] | (ref[1] << 32)


def test_philox_statistics():
    # bit balance and top-byte uniformity over 2^16 consecutive counters
    n = 1 << 16
    vals = np.array([oracle.draw64(7, s % 97, s) for s in range(n)], dtype=np.uint64)
    bits = np.unpackbits(vals.view(np.uint8)).reshape(n, 64).mean(axis=0)
    assert np.all(np.abs(bits - 0.5) < 0.02)
    from scipy.stats import chisquare
    top = (vals >> np.uint64(56)).astype(np.int64)
    assert chisquare(np.bincount(top, minlength=256)).pvalue > 1e-6
    assert np.unique(vals).size == n


def test_scale_is_floor_of_product():
    rng = np.random.default_rng(5)
    for _ in range(2000):
        r = int(rng.integers(0, 2**63)) * 2 + int(rng.integers(0, 2))
        tot = int(rng.integers(1, 2**63)) * 2 + int(rng.integers(0, 2))
        assert oracle.scale(r, tot) == (r * tot) >> 64
    assert oracle.scale(2**64 - 1, 2**64 - 1) == 2**64 - 2
    assert oracle.scale(0, 12345) == 0


def _first_r_with_index_at_least(b, total, j):
    """Smallest r64 whose draw selects an index >= j (bisection over 2^64)."""
    lo, hi = 0, 2**64
    while lo < hi:
        mid = (lo + hi) // 2
        if oracle.select(b, oracle.scale(mid, total)) >= j:
            hi = mid
        else:
            lo = mid + 1
    return lo


@pytest.mark.parametrize("seed", range(12))
def test_selection_interval_counts_exact(seed):
    """Each index j is chosen by exactly ceil(B_j 2^64/S) - ceil(B_{j-1} 2^64/S)
    of the 2^64 draws, i.e. with probability b_j/S up to 2^-64: half-open
    intervals [B_{j-1}, B_j) of the cumulative sum."""
    rng = np.random.default_rng(seed)
    d = int(rng.integers(1, 9))
    if seed % 3 == 0:
        b = rng.integers(0, 2**40, size=d, dtype=np.uint64)
    else:
        b = rng.integers(0, 6, size=d).astype(np.uint64)
    if seed == 1:
        b = np.array([0, 2**63, 0, 2**62, 1], dtype=np.uint64)
    d = b.size
    total = int(sum(int(x) for x in b))
    if total == 0:
        b[0] = 1
        total = 1
    B = []
    acc = 0
    for x in b:
        acc += int(x)
        B.append(acc)
    prev = 0
    for j in range(d):
        start = _first_r_with_index_at_least(b, total, j + 1)
        count = start - prev
        expect = -(-(B[j] << 64) // total) - (-(-((B[j - 1] if j else 0) << 64) // total))
        assert count == expect, (j, count, expect)
        assert abs(Fraction(count, 2**64) - Fraction(int(b[j]), total)) < Fraction(1, 2**64)
        if int(b[j]) == 0:
            assert count == 0  # zero weight is never selected
        prev = start
    assert prev == 2**64
