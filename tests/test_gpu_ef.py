"""Elias-Fano graphs on the GPU: the store's bits equal the oracle's encoding,
select and rank equal the oracle's, and every walk kind and the negatives are
those of the CSR handle of the same graph and of the oracle, bit for bit."""
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
RUNS = [(FO, 1.0, 1.0), (NV, 1.0, 1.0), (NV, 2.0, 1.0), (NV, 0.25, 1.0), (NV, 0.25, 4.0), (NV, 4.0, 0.5),
        (NV, 1.0, 2.0)]


def upload_ef(O, D, W, q=0):
    Ot = torch.from_numpy(np.ascontiguousarray(O, dtype=np.uint64).view(np.int64)).cuda()
    Dt = torch.from_numpy(np.ascontiguousarray(D, dtype=np.int32)).cuda()
    Wt = None if W is None else torch.from_numpy(np.ascontiguousarray(W, dtype=np.uint32).view(np.int32)).cuda()
    g = n2v.n2v_graph_upload_ef(Ot, Dt, Wt, q)
    del Ot, Dt, Wt  # the handle owns everything it reads
    return g


def codes_of(O, D, k):
    src = np.repeat(np.arange(len(O) - 1, dtype=np.uint64), np.diff(O.astype(np.int64)))
    return (src << np.uint64(k)) | D.astype(np.uint64)


def check_layout(O, D, W, q):
    g = upload_ef(O, D, W, q)
    info = n2v.n2v_ef_info(g)
    ref = oracle.ef_encode_graph(O, D, q=q)
    for f in ("k", "l", "u", "n_zeros", "h_bits"):
        assert info[f] == ref[f], f
    assert info["n_codes"] == ref["m"] and info["quantum"] == q
    arr = n2v.ef_arrays(g)
    for name in ("H", "L", "S1", "S0"):
        got = arr[name].cpu().numpy().view(np.uint64)
        exp = ref[name][:got.size] if got.size else ref[name][:0]
        assert got.size == (info[{"H": "h_words", "L": "l_words", "S1": "s1_len", "S0": "s0_len"}[name]])
        assert np.array_equal(got, exp), name
    gi = n2v.n2v_graph_info(g)
    assert gi["storage"] == n2v.N2V_STORAGE_EF and gi["ef_quantum"] == q
    return g, ref


@pytest.mark.parametrize("name", sorted(synth.TINY))
@pytest.mark.parametrize("q", [8, 64, 1024])
def test_layout_tiny_catalogue(name, q):
    O, D, W = synth.TINY[name]()
    g, ref = check_layout(O, D, W, q)
    n2v.n2v_graph_release(g)


def test_layout_random_and_powerlaw():
    rng = np.random.default_rng(11)
    for it in range(20):
        O, D, W = synth.random_small(rng, n_max=60)
        g, _ = check_layout(O, D, W, int(rng.choice([8, 16, 256])))
        n2v.n2v_graph_release(g)
    O, D, W = synth.chung_lu(3000, 30000, 2.1, 15.0, 1500.0, (1, 9), seed=5)
    g, _ = check_layout(O, D, W, 8)
    n2v.n2v_graph_release(g)


def test_select_and_rank():
    O, D, W = synth.chung_lu(20000, 150000, 2.1, 12.0, 8000.0, (1, 50), seed=4)
    n = len(O) - 1
    for q in (8, 256, 4096):
        g = upload_ef(O, D, W, q)
        info = n2v.n2v_ef_info(g)
        codes = codes_of(O, D, info["k"])
        idx = torch.arange(codes.size + 3, dtype=torch.int64, device="cuda")
        sel = n2v.n2v_ef_select(g, idx).cpu().numpy().view(np.uint64)
        assert np.array_equal(sel[:codes.size], codes)
        assert (sel[codes.size:] == np.uint64(2**64 - 1)).all()
        rng = np.random.default_rng(q)
        xs = np.concatenate([codes, codes + np.uint64(1), np.arange(n + 1, dtype=np.uint64) << np.uint64(info["k"]),
                             rng.integers(0, info["u"], size=20000, dtype=np.uint64),
                             np.array([0, info["u"], info["u"] + 5], dtype=np.uint64)])
        rk = n2v.n2v_ef_rank(g, torch.from_numpy(xs.view(np.int64)).cuda()).cpu().numpy()
        assert np.array_equal(rk, np.searchsorted(codes, xs, side="left"))
        n2v.n2v_graph_release(g)
    # the oracle's own scans on a small graph
    O, D, W = synth.TINY["wdiamond"]()
    g = upload_ef(O, D, W, 8)
    ref = oracle.ef_encode_graph(O, D, q=8)
    xs = np.arange(ref["u"] + 2, dtype=np.uint64)
    rk = n2v.n2v_ef_rank(g, torch.from_numpy(xs.view(np.int64)).cuda()).cpu().numpy()
    assert list(rk) == [oracle.ef_rank(ref, int(x)) for x in xs]
    sel = n2v.n2v_ef_select(g, torch.arange(len(D), dtype=torch.int64, device="cuda")).cpu().numpy()
    assert list(sel) == [oracle.ef_select(ref, i) for i in range(len(D))]
    n2v.n2v_graph_release(g)


def _walk_pair(O, D, W, starts, reps, L, seed, q, oracle_rows=None):
    gc, keep = upload(O, D, W)
    ge = upload_ef(O, D, W, q)
    for kind, p, qq in RUNS:
        Yc, lc = run(gc, starts, reps, L, kind, p, qq, seed)
        Ye, le = run(ge, starts, reps, L, kind, p, qq, seed)
        assert np.array_equal(Yc, Ye) and np.array_equal(lc, le), (kind, p, qq)
        if oracle_rows is not None:
            Yo, lo = oracle.walks(O, D, W, starts, reps, L, kind, p, qq, seed, 0, rows=oracle_rows)
            rows = np.arange(len(Yc)) if oracle_rows is None else oracle_rows
            assert np.array_equal(Ye[rows], Yo) and np.array_equal(le[rows], lo), (kind, p, qq)
    n2v.n2v_graph_release(gc)
    n2v.n2v_graph_release(ge)


@pytest.mark.parametrize("name", sorted(synth.TINY))
def test_walks_tiny_catalogue(name):
    O, D, W = synth.TINY[name]()
    n = len(O) - 1
    _walk_pair(O, D, W, list(range(n)) + [-1, n], 3, 12, 7, 8, oracle_rows=np.arange(3 * (n + 2)))


def test_walks_fuzz():
    rng = np.random.default_rng(21)
    for it in range(30):
        O, D, W = synth.random_small(rng, n_max=16)
        n = len(O) - 1
        starts = rng.integers(-1, n + 1, size=int(rng.integers(1, 8)))
        reps = int(rng.integers(1, 3))
        _walk_pair(O, D, W, starts, reps, int(rng.integers(1, 20)), it, int(rng.choice([8, 64])),
                   oracle_rows=np.arange(reps * starts.size))


def test_walks_powerlaw_and_ba():
    O, D, W = synth.chung_lu(20000, 150000, 2.1, 12.0, 8000.0, (1, 50), seed=4)
    n = len(O) - 1
    _walk_pair(O, D, W, np.arange(n), 1, 20, 3, 256, oracle_rows=np.arange(0, n, 97))
    O, D, W = synth.ba_10k()
    n = len(O) - 1
    _walk_pair(O, D, W, np.arange(n), 1, 30, 9, 1024, oracle_rows=np.arange(0, n, 31))


def test_walks_dense_rows():
    """Rows spanning 2^(k - l) >= 64 buckets of high parts (a complete graph,
    128 buckets, and mean degree about 47, 64 buckets: the walks take the
    one-lane selects) and 32 buckets (mean degree about 25: the wavefront
    keeps the rows' bucket boundaries in its lanes) give the CSR walks and the
    oracle's."""
    O, D, _ = synth.complete(80)
    W = np.random.default_rng(3).integers(1, 60, size=len(D)).astype(np.uint32)
    _walk_pair(O, D, W, np.arange(80), 4, 25, 5, 64, oracle_rows=np.arange(0, 320, 7))
    for args in ((3000, 75000, 2.3, 50.0, 900.0), (3000, 40000, 2.3, 25.0, 600.0)):
        O, D, W = synth.chung_lu(*args, (1, 100), seed=8)
        n = len(O) - 1
        _walk_pair(O, D, W, np.arange(n), 1, 25, 6, 256, oracle_rows=np.arange(0, n, 29))


def test_negatives_and_handles_own_their_memory():
    O, D, W = synth.chung_lu(5000, 40000, 2.1, 12.0, 2000.0, (1, 100), seed=6)
    n = len(O) - 1
    g = upload_ef(O, D, W, 64)
    filler = [torch.full((D.size + 64,), -7, dtype=torch.int32, device="cuda") for _ in range(4)]
    S = torch.arange(n, dtype=torch.int32, device="cuda")
    Y, lens = n2v.n2v_walks_node2vec(g, S, 2, 30, 0.5, 2.0, 4)
    torch.cuda.synchronize()
    Yo, lo = oracle.walks(O, D, W, np.arange(n), 2, 30, oracle.NODE2VEC, 0.5, 2.0, 4, 0)
    assert np.array_equal(Y.cpu().numpy(), Yo)
    N = n2v.n2v_negative_samples(g, Y, 5, seed=3, walk_id_base=11)
    torch.cuda.synchronize()
    assert np.array_equal(N.cpu().numpy(), oracle.negatives(O, Y.cpu().numpy(), 5, 3, 11))
    del filler
    n2v.n2v_graph_release(g)


def test_ef_rejections_and_sizes():
    O, D, W = synth.chung_lu(200000, 2000000, 2.2, 20.0, 20000.0, (1, 100), seed=7)
    g = upload_ef(O, D, None, 256)
    gi = n2v.n2v_graph_info(g)
    csr_bytes = 8 * len(O) + 4 * len(D)
    assert gi["device_bytes"] < 0.7 * csr_bytes, (gi["device_bytes"], csr_bytes)
    S = torch.arange(10, dtype=torch.int32, device="cuda")
    with pytest.raises(n2v.N2VError):
        n2v.n2v_walks_approximated(g, NV, S, 1, 5, 1.0, 2.0, 4, 1)
    Y = torch.empty((10, 5), dtype=torch.int32, device="cuda")
    lens = torch.empty(10, dtype=torch.int32, device="cuda")
    with pytest.raises(n2v.N2VError):
        n2v.n2v_walks_batched([n2v.make_request(g, NV, S, 1, 5, 1.0, 2.0, 1, 0, Y, lens)])
    n2v.n2v_graph_release(g)
