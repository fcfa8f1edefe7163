"""Approximated walks (Sorted Unique Sub-Sampling of k neighbours per step)
on the GPU vs the oracle, bit for bit."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2110_06196_amd as n2v  # noqa: E402
from tests._devutil import run, upload  # noqa: E402

FO, NV = n2v.N2V_FIRST_ORDER, n2v.N2V_NODE2VEC


@pytest.fixture(autouse=True)
def _reset_tuning():
    n2v.n2v_set_tuning(reset=True)
    yield
    n2v.n2v_set_tuning(reset=True)


def run_approx(g, starts, reps, L, kind, p, q, k, seed, base=0):
    S = torch.from_numpy(np.ascontiguousarray(starts, dtype=np.int32)).cuda()
    Y, lens = n2v.n2v_walks_approximated(g, kind, S, reps, L, p, q, k, seed, base)
    torch.cuda.synchronize()
    return Y.cpu().numpy(), lens.cpu().numpy()


def check(O, D, W, g, starts, reps, L, kind, p, q, k, seed, base=0, rows=None):
    Y, lens = run_approx(g, starts, reps, L, kind, p, q, k, seed, base)
    Yo, lo = oracle.walks(O, D, W, starts, reps, L, kind, p, q, seed, base, rows=rows, k_approx=k)
    if rows is not None:
        Y, lens = Y[rows], lens[rows]
    bad = np.nonzero((Y != Yo).any(axis=1) | (lens != lo))[0]
    assert bad.size == 0, f"{bad.size} rows differ (k={k}, p={p}, q={q})"
    return Y, lens


@pytest.mark.parametrize("name", sorted(synth.TINY))
def test_tiny_catalogue(name):
    O, D, W = synth.TINY[name]()
    n = len(O) - 1
    g, keep = upload(O, D, W)
    starts = list(range(n)) + [-1, n]
    for k in (1, 2, 3):
        for kind, p, q in [(FO, 1.0, 1.0), (NV, 0.25, 4.0), (NV, 2.0, 1.0), (NV, 1.0, 1.0)]:
            check(O, D, W, g, starts, 3, 10, kind, p, q, k, seed=5, base=3)
    n2v.n2v_graph_release(g)


def test_fuzz():
    rng = np.random.default_rng(77)
    for it in range(60):
        O, D, W = synth.random_small(rng, n_max=14)
        n = len(O) - 1
        g, keep = upload(O, D, W)
        starts = rng.integers(-1, n + 1, size=int(rng.integers(1, 8)))
        k = int(rng.integers(1, 6))
        kind = NV if it % 3 else FO
        p, q = [(0.25, 4.0), (2.0, 0.5), (3.0, 0.3), (1.0, 1.0)][it % 4]
        check(O, D, W, g, starts, int(rng.integers(1, 3)), int(rng.integers(1, 16)), kind, p, q, k, seed=it)
        n2v.n2v_graph_release(g)


def test_hub_graph_every_shape():
    O, D, W = synth.chung_lu(20000, 200000, 2.0, 20.0, 15000.0, (1, 1000), seed=12)
    n = len(O) - 1
    g, keep = upload(O, D, W)
    starts = np.arange(n)
    rows = np.arange(0, n, 53)
    for k in (10, 100, 700):
        for kind, p, q in [(NV, 0.25, 4.0), (FO, 1.0, 1.0), (NV, 2.0, 1.0)]:
            ref = check(O, D, W, g, starts, 1, 20, kind, p, q, k, seed=9, rows=rows)
            for lanes in (4, 16, 64):
                n2v.n2v_set_tuning(lanes_per_walker=lanes)
                Y, lens = run_approx(g, starts, 1, 20, kind, p, q, k, seed=9)
                assert np.array_equal(Y[rows], ref[0]) and np.array_equal(lens[rows], ref[1]), (k, lanes)
            n2v.n2v_set_tuning(reset=True)
    # k at least the max degree: exactly the exact walks
    kmax = int((O[1:] - O[:-1]).max())
    for kind, p, q in [(NV, 0.25, 4.0), (FO, 1.0, 1.0)]:
        ex = run(g, starts, 1, 20, kind, p, q, 9)
        ap = run_approx(g, starts, 1, 20, kind, p, q, kmax, 9)
        assert np.array_equal(ex[0], ap[0]) and np.array_equal(ex[1], ap[1])
    n2v.n2v_graph_release(g)


def test_batched_approx_requests():
    O, D, W = synth.chung_lu(5000, 50000, 2.1, 20.0, 3000.0, (1, 100), seed=2)
    g, keep = upload(O, D, W)
    rng = np.random.default_rng(5)
    descs, bufs, reqs = [], [], []
    for k in range(40):
        starts = rng.integers(0, len(O) - 1, size=int(rng.integers(1, 300))).astype(np.int32)
        r = dict(starts=starts, L=int(rng.integers(2, 40)), kind=NV if k % 4 else FO, p=[0.25, 1.0, 4.0][k % 3],
                 q=[4.0, 1.0, 0.25][k % 3], k=[0, 5, 50][k % 3], seed=100 + k)
        S = torch.from_numpy(starts).cuda()
        Y = torch.empty((starts.size, r["L"]), dtype=torch.int32, device="cuda")
        lens = torch.empty(starts.size, dtype=torch.int32, device="cuda")
        descs.append(n2v.make_request(g, r["kind"], S, 1, r["L"], r["p"], r["q"], r["seed"], 0, Y, lens, r["k"]))
        bufs.append((S, Y, lens))
        reqs.append(r)
    n2v.n2v_walks_batched(descs)
    torch.cuda.synchronize()
    for r, (S, Y, lens) in zip(reqs, bufs):
        Yo, lo = oracle.walks(O, D, W, r["starts"], 1, r["L"], r["kind"], r["p"], r["q"], r["seed"], 0,
                              k_approx=r["k"])
        assert np.array_equal(Y.cpu().numpy(), Yo) and np.array_equal(lens.cpu().numpy(), lo)
    n2v.n2v_graph_release(g)
