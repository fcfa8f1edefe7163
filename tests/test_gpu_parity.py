"""GPU walks vs the CPU oracle, bit for bit, through the C ABI.

Covers the tiny-graph catalogue (every kind and bias class), random small
graphs (directed, weighted, zero weights, self-loops, dead ends, bad starts),
the 10k-node Barabasi-Albert workload in full, and the invariance of the
output under every tuning point and under the first-order / return-only
specialisations (all must equal the generic path and the oracle exactly).
"""
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
PQ = [(1.0, 1.0), (2.0, 0.5), (0.25, 4.0), (4.0, 1.0), (0.5, 1.0), (1.0, 2.0), (3.0, 0.3)]


@pytest.fixture(autouse=True)
def _reset_tuning():
    n2v.n2v_set_tuning(reset=True)
    yield
    n2v.n2v_set_tuning(reset=True)


def check(O, D, W, starts, reps, L, kind, p=1.0, q=1.0, seed=0, base=0, g=None, rows=None):
    keep = None
    if g is None:
        g, keep = upload(O, D, W)
    Y, lens = run(g, starts, reps, L, kind, p, q, seed, base)
    Yo, lo = oracle.walks(O, D, W, starts, reps, L, kind, p, q, seed, base, rows=rows)
    if rows is not None:
        Y, lens = Y[rows], lens[rows]
    bad = np.nonzero((Y != Yo).any(axis=1) | (lens != lo))[0]
    assert bad.size == 0, f"{bad.size} rows differ; first {bad[:5]}: gpu {Y[bad[0]][:12]} oracle {Yo[bad[0]][:12]}"
    del keep
    return Y, lens


@pytest.mark.parametrize("name", sorted(synth.TINY))
def test_tiny_catalogue(name):
    O, D, W = synth.TINY[name]()
    n = len(O) - 1
    g, keep = upload(O, D, W)
    starts = list(range(n)) + [-1, n, 2**31 - 1]
    for kind in (FO, NV):
        for p, q in (PQ if kind == NV else [(1.0, 1.0)]):
            for L in (1, 2, 11):
                check(O, D, W, starts, 3, L, kind, p, q, seed=17, base=5, g=g)
    n2v.n2v_graph_release(g)


def test_fuzz_small_graphs():
    rng = np.random.default_rng(2024)
    for it in range(120):
        O, D, W = synth.random_small(rng, n_max=14)
        n = len(O) - 1
        starts = rng.integers(-1, n + 1, size=int(rng.integers(1, 9)))
        L = int(rng.integers(1, 22))
        kind = NV if it % 4 else FO
        p, q = PQ[int(rng.integers(0, len(PQ)))]
        check(O, D, W, starts, int(rng.integers(1, 4)), L, kind, p, q, seed=it, base=int(rng.integers(0, 2**40)))


def _tuning_sweep(O, D, W, rows, L, cases, grid):
    n = len(O) - 1
    starts = np.arange(n)
    g, keep = upload(O, D, W)
    for kind, p, q in cases:
        ref = check(O, D, W, starts, 1, L, kind, p, q, seed=3, g=g, rows=rows)
        for lanes, tile, cap, route, flags in grid:
            n2v.n2v_set_tuning(lanes_per_walker=lanes, lds_tile=tile, list_cap=cap, route=route, flags=flags)
            Y, lens = run(g, starts, 1, L, kind, p, q, seed=3)
            assert np.array_equal(Y[rows], ref[0]) and np.array_equal(lens[rows], ref[1]), \
                (kind, p, q, lanes, tile, cap, route, flags)
        n2v.n2v_set_tuning(reset=True)
    n2v.n2v_graph_release(g)


def test_tuning_points_and_specialisations_identical():
    """Every lanes-per-walker / LDS tile / list capacity / route setting and the
    generic-only route give the oracle's walks (tile 1 forces N(t) lookups in
    global memory, list capacity 1 forces the two-pass fallback)."""
    O, D, W = synth.chung_lu(3000, 40000, 2.2, 20.0, 1500.0, (1, 100), seed=9)
    rows = np.arange(0, len(O) - 1, 7)
    cases = [(NV, 0.25, 4.0), (NV, 2.0, 1.0), (NV, 1.0, 1.0), (FO, 1.0, 1.0), (NV, 0.5, 2.0)]
    grid = [(lanes, tile, cap, route, flags)
            for lanes in (4, 8, 16, 32, 64) for tile in (1, 2048) for cap in (1, 512)
            for route in (0, 1, 2, 3, 4) for flags in (0, n2v.N2V_TUNE_GENERIC_ONLY)]
    for ww in (W, None):
        _tuning_sweep(O, D, ww, rows, 30, cases, grid)


def test_walk_counters_streams_and_threads():
    """node2vec launches hand out walks from a per-stream counter that a kernel
    zeroes before each launch: back-to-back launches on one stream, launches on
    several streams at once and four host threads launching onto one stream
    all give the oracle's walks."""
    import threading
    O, D, W = synth.chung_lu(5000, 60000, 2.2, 20.0, 2000.0, (1, 100), seed=31)
    n = len(O) - 1
    g, keep = upload(O, D, W)
    S = torch.arange(n, dtype=torch.int32, device="cuda")
    args = (g, S, 2, 30, 0.25, 4.0, 5)
    ref, rlens = n2v.n2v_walks_node2vec(*args)
    torch.cuda.synchronize()
    rows = np.arange(0, 2 * n, 13)
    Yo, lo = oracle.walks(O, D, W, np.arange(n), 2, 30, NV, 0.25, 4.0, 5, 0, rows=rows)
    assert np.array_equal(ref.cpu().numpy()[rows], Yo) and np.array_equal(rlens.cpu().numpy()[rows], lo)
    outs = [n2v.n2v_walks_node2vec(*args) for _ in range(3)]
    streams = [torch.cuda.Stream() for _ in range(3)]
    for st in streams:
        with torch.cuda.stream(st):
            outs.append(n2v.n2v_walks_node2vec(*args, stream=st))
    shared = torch.cuda.Stream()
    res = [None] * 4

    def worker(i):
        with torch.cuda.stream(shared):
            res[i] = n2v.n2v_walks_node2vec(*args, stream=shared)

    threads = [threading.Thread(target=worker, args=(i,)) for i in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    torch.cuda.synchronize()
    for i, (Y, L) in enumerate(outs + res):
        assert torch.equal(Y, ref) and torch.equal(L, rlens), i
    n2v.n2v_graph_release(g)
    del keep


def test_hub_rows_all_routes():
    """Hubs of degree ~1e4: many chunks per block in the two-pass route, long
    probe and stream lists, G-ary searches over long segments."""
    O, D, W = synth.chung_lu(20000, 200000, 2.0, 20.0, 15000.0, (1, 1000), seed=12)
    assert int((O[1:] - O[:-1]).max()) > 4096  # > 64 chunks of 64: several chunks per block
    rows = np.arange(0, len(O) - 1, 41)
    cases = [(NV, 0.25, 4.0), (NV, 4.0, 0.25), (NV, 2.0, 1.0)]
    grid = [(lanes, tile, cap, route, 0)
            for lanes in (4, 64) for tile in (1, 4096) for cap in (1, 4096) for route in (1, 2, 3, 4)]
    _tuning_sweep(O, D, W, rows, 24, cases, grid)


def test_giant_hub_rows_head_search():
    """Hubs adjacent to ~80% of 150,000 nodes: a 64-splitter slice of such a row
    holds ~1900 entries, so bisections go through the destination heads
    (every 32nd entry) and one 32-entry block.  Auto, probe and stream routes."""
    rng = np.random.default_rng(77)
    n = 150000
    hubs = rng.choice(n, size=6, replace=False)
    src, dst = [], []
    for h in hubs:
        nb = np.nonzero(rng.random(n) < 0.8)[0]
        src.append(np.full(nb.size, h))
        dst.append(nb)
    src.append(rng.integers(0, n, 300000))
    dst.append(rng.integers(0, n, 300000))
    src, dst = np.concatenate(src), np.concatenate(dst)
    keep = src != dst
    src, dst = src[keep], dst[keep]
    O, D, W = synth.csr_from_edges(n, src, dst, rng.integers(1, 1001, src.size), symmetric=True)
    deg = (O[1:] - O[:-1]).astype(np.int64)
    assert deg.max() > 1024 * 64  # splitter slices above 1024 entries
    starts = np.concatenate([hubs, rng.integers(0, n, 400)])
    g, keep_t = upload(O, D, W)
    # without stored lists every step takes a route: one walk per wavefront,
    # with the destination heads of the long rows
    Ot, Dt, Wt = keep_t
    g0 = n2v.n2v_graph_upload(Ot, Dt, Wt, flags=n2v.N2V_UPLOAD_NO_PAIR_LISTS)
    for h in (g, g0):
        for route in (0, 2, 3):
            n2v.n2v_set_tuning(route=route)
            for p, q in ((0.25, 4.0), (1.0, 2.0)):
                check(O, D, W, starts, 1, 8, NV, p, q, seed=5, g=h)
    n2v.n2v_set_tuning(reset=True)
    n2v.n2v_graph_release(g0)
    n2v.n2v_graph_release(g)


def test_hub_pair_lists_identical():
    """Stored common-neighbour lists of hub edges (built at upload) change no
    walk: a handle with them and one without give the same walks, equal to the
    oracle, for return / in-out biases on both sides of 1."""
    O, D, W = synth.chung_lu(20000, 300000, 2.1, 30.0, 8000.0, (1, 1000), seed=21)
    n = len(O) - 1
    g1, k1 = upload(O, D, W)
    Ot, Dt, Wt = k1
    g0 = n2v.n2v_graph_upload(Ot, Dt, Wt, flags=n2v.N2V_UPLOAD_NO_PAIR_LISTS)
    i1, i0 = n2v.n2v_graph_info(g1), n2v.n2v_graph_info(g0)
    assert i1["pair_lists"] > 1000 and i1["pair_entries"] > 0
    assert i0["pair_lists"] == 0 and i0["pair_entries"] == 0
    starts = np.arange(n)
    # on this graph the lists of only part of the edges fit the budget, so the
    # walks take one wavefront each and use the routes where no list is kept
    # (test_automatic_four_lane_lists_only covers the graphs whose edges all
    # keep one)
    assert i1["pair_lists"] < len(D)
    rows = np.arange(0, 2 * n, 57)
    for p, q in ((0.25, 4.0), (2.0, 0.5), (1.0, 2.0), (4.0, 0.25)):
        Y1, L1 = run(g1, starts, 2, 40, NV, p, q, seed=8)
        Y0, L0 = run(g0, starts, 2, 40, NV, p, q, seed=8)
        assert np.array_equal(Y1, Y0) and np.array_equal(L1, L0), (p, q)
        Yo, lo = oracle.walks(O, D, W, starts, 2, 40, NV, p, q, 8, 0, rows=rows)
        assert np.array_equal(Y1[rows], Yo) and np.array_equal(L1[rows], lo), (p, q)
    n2v.n2v_graph_release(g0)
    n2v.n2v_graph_release(g1)


def test_automatic_four_lane_lists_only():
    """Every edge keeps its stored list and the launch has at least 96 walks per
    CU: the automatic shape is then 4-lane groups of the lists-only variant.
    Its walks equal those of a handle without lists (the list-building routes)
    and the oracle's, for in-out biases on both sides of 1."""
    O, D, W = synth.chung_lu(20000, 200000, 2.2, 20.0, 2000.0, (1, 100), seed=31)
    n = len(O) - 1
    g1, k1 = upload(O, D, W)
    Ot, Dt, Wt = k1
    g0 = n2v.n2v_graph_upload(Ot, Dt, Wt, flags=n2v.N2V_UPLOAD_NO_PAIR_LISTS)
    assert n2v.n2v_graph_info(g1)["pair_lists"] == len(D)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    reps = -(-96 * cus // n)  # walks per node for at least 96 walks per CU
    starts = np.arange(n)
    rows = np.arange(0, reps * n, 97)
    for p, q in ((0.25, 4.0), (2.0, 0.5), (1.0, 2.0)):
        Y1, L1 = run(g1, starts, reps, 40, NV, p, q, seed=12)
        Y0, L0 = run(g0, starts, reps, 40, NV, p, q, seed=12)
        assert np.array_equal(Y1, Y0) and np.array_equal(L1, L0), (p, q)
        Yo, lo = oracle.walks(O, D, W, starts, reps, 40, NV, p, q, 12, 0, rows=rows)
        assert np.array_equal(Y1[rows], Yo) and np.array_equal(L1[rows], lo), (p, q)
    n2v.n2v_graph_release(g0)
    n2v.n2v_graph_release(g1)
    del k1


@pytest.mark.parametrize("off", [1, 6, 15])
def test_output_rows_at_any_alignment(off):
    """Walk rows leave in whole 64-byte lines chosen by address: an output array
    that starts `off` words into a line shifts every row's phase.  The walks
    equal those written to an aligned array, and nothing before or after the
    array is written (lane kernels, 4-, 16- and 64-lane groups, dead ends)."""
    O, D, W = synth.chung_lu(3000, 30000, 2.2, 12.0, 400.0, (1, 100), seed=13)
    n = len(O) - 1
    assert (np.diff(O) == 0).any()  # some starts are dead ends: their rows are padding
    g, keep = upload(O, D, W)
    S = torch.arange(n, dtype=torch.int32, device="cuda")
    L, reps = 37, 2
    nw = n * reps
    for lanes in (0, 4, 16, 64):
        n2v.n2v_set_tuning(reset=True) if lanes == 0 else n2v.n2v_set_tuning(lanes_per_walker=lanes)
        for kind, p, q in ((FO, 1.0, 1.0), (NV, 4.0, 1.0), (NV, 0.25, 4.0), (NV, 2.0, 0.5)):
            flat = torch.full((nw * L + off + 16,), -7, dtype=torch.int32, device="cuda")
            Y = flat[off:off + nw * L].view(nw, L)
            lens = torch.empty(nw, dtype=torch.int32, device="cuda")
            if kind == FO:
                ref, rl = n2v.n2v_walks_first_order(g, S, reps, L, 23)
                n2v.n2v_walks_first_order(g, S, reps, L, 23, walks=Y, lens=lens)
            else:
                ref, rl = n2v.n2v_walks_node2vec(g, S, reps, L, p, q, 23)
                n2v.n2v_walks_node2vec(g, S, reps, L, p, q, 23, walks=Y, lens=lens)
            torch.cuda.synchronize()
            assert torch.equal(Y, ref) and torch.equal(lens, rl), (lanes, kind, p, q)
            assert bool((flat[:off] == -7).all()) and bool((flat[off + nw * L:] == -7).all()), (lanes, kind, p, q)
    n2v.n2v_set_tuning(reset=True)
    n2v.n2v_graph_release(g)
    del keep


def test_edge_lists_over_budget():
    """A complete graph has n - 2 common neighbours on every edge, more than the
    lists' budget of 16 entries per graph entry: only part of the edges keep a
    list, the others use the routes, and the walks still equal the oracle's."""
    O, D, _ = synth.complete(40)
    rng = np.random.default_rng(5)
    W = rng.integers(1, 50, size=len(D)).astype(np.uint32)
    g, keep = upload(O, D, W)
    info = n2v.n2v_graph_info(g)
    assert 0 < info["pair_lists"] < len(D)
    for p, q in ((0.25, 4.0), (3.0, 0.3)):
        check(O, D, W, np.arange(40), 20, 30, NV, p, q, seed=13, g=g)
    n2v.n2v_graph_release(g)
    del keep


def test_ba_10k_full():
    """Barabasi-Albert, 10,000 nodes, m = 5, node2vec p = 2, q = 0.5, one walk of
    80 slots per node, seed 42: every walk."""
    O, D, W = synth.ba_10k()
    n = len(O) - 1
    Y, lens = check(O, D, W, np.arange(n), 1, 80, NV, 2.0, 0.5, seed=42)
    assert np.all(lens == 80)


def test_walk_id_base_chunking():
    O, D, W = synth.chung_lu(2000, 20000, 2.2, 16.0, 800.0, (1, 50), seed=4)
    g, keep = upload(O, D, W)
    starts = np.arange(len(O) - 1)
    full = run(g, starts, 2, 25, NV, 0.5, 2.0, seed=8, base=1000)
    part = run(g, starts[700:], 1, 25, NV, 0.5, 2.0, seed=8, base=1700)
    assert np.array_equal(full[0][700:2000], part[0])


def test_errors():
    O, D, W = synth.cycle(6)
    D2 = D.copy()
    D2[0], D2[1] = D2[1], D2[0]
    with pytest.raises(n2v.N2VError) as e:
        upload(O, D2, W)
    assert e.value.code == n2v.N2V_ERR_UNSORTED
    D3 = D.copy()
    D3[4] = 99
    with pytest.raises(n2v.N2VError) as e:
        upload(O, D3, W)
    assert e.value.code == n2v.N2V_ERR_UNSORTED
    O4 = O.copy()
    O4[-1] = O4[-1] - 1
    with pytest.raises(n2v.N2VError) as e:
        upload(O4, D, W)
    assert e.value.code == n2v.N2V_ERR_UNSORTED
    g, keep = upload(O, D, W)
    info = n2v.n2v_graph_info(g)
    assert info["n_nodes"] == 6 and info["n_entries"] == 12 and info["max_degree"] == 2
    for bad in (0.0, -1.0, float("nan"), float("inf"), 1e9):
        with pytest.raises(n2v.N2VError) as e:
            run(g, [0], 1, 5, NV, bad, 1.0)
        assert e.value.code == n2v.N2V_ERR_INVALID_ARG
    with pytest.raises(n2v.N2VError):
        run(g, [0], 1, 0, FO)
    # walk_len above 2^30 is refused before any device work (no output is touched)
    S1 = torch.zeros(1, dtype=torch.int32, device="cuda")
    Y1 = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert n2v.lib().n2v_walks_first_order(g, S1.data_ptr(), 1, 1, 2**30 + 1, 0, 0, Y1.data_ptr(), None,
                                           None) == n2v.N2V_ERR_INVALID_ARG
    assert n2v.lib().n2v_walks_node2vec(g, S1.data_ptr(), 1, 1, 2**30 + 1, 1.0, 2.0, 0, 0, Y1.data_ptr(), None,
                                        None) == n2v.N2V_ERR_INVALID_ARG
    # overflow precondition
    O5, D5, _ = synth.star(70000)
    W5 = np.full(D5.size, 2**30, dtype=np.uint32)
    g5, keep5 = upload(O5, D5, W5)
    assert n2v.n2v_graph_info(g5)["prefix_bytes"] == 8
    with pytest.raises(n2v.N2VError) as e:
        run(g5, [0], 1, 4, NV, 2.0 / 65536.0, 1.0)
    assert e.value.code == n2v.N2V_ERR_OVERFLOW
    # 64-bit prefix path is exact too
    check(O5, D5, W5, np.arange(0, 70001, 97), 1, 6, NV, 0.5, 1.0, seed=5, g=g5)
    check(O5, D5, W5, np.arange(0, 70001, 97), 1, 6, FO, seed=5, g=g5)
    n2v.n2v_graph_release(g)
    with pytest.raises(n2v.N2VError) as e:
        run(g, [0], 1, 5, FO)
    assert e.value.code == n2v.N2V_ERR_BAD_HANDLE


def _skewed_graph(kinds, seed):
    rng = np.random.default_rng(seed)
    n = 6000
    src, dst, wts = [], [], []
    for h, kind in enumerate(kinds):
        nb = np.arange(10, 10 + 4000)
        w = np.ones(nb.size, dtype=np.int64)
        if kind == "front":
            w[0] = 2**30
        elif kind == "middle":
            w[nb.size // 2] = 2**30
        elif kind == "back":
            w[-1] = 2**30
        elif kind == "geometric":
            w = np.minimum(2 ** (np.arange(nb.size) // 150), 2**30).astype(np.int64)
        else:
            w = np.where(rng.random(nb.size) < 0.9, 0, rng.integers(1, 100, nb.size))
            w[-1] = 5
        src += [h] * nb.size
        dst += list(nb)
        wts += list(w)
    # every hub's neighbours point back to every hub, so walks keep returning
    for x in range(10, 4010):
        for h in range(len(kinds)):
            src.append(x)
            dst.append(h)
            wts.append(int(rng.integers(1, 50)))
    return synth.csr_from_edges(n, np.array(src), np.array(dst), np.array(wts, dtype=np.uint32)), len(kinds)


@pytest.mark.parametrize("kinds", [("front", "middle", "back", "zeros"), ("geometric", "front")])
def test_first_order_skewed_prefixes(kinds):
    # Row prefixes far from linear drive the interpolated prefix search through
    # every bracket case: one dominant weight at the start, middle or end of a
    # long row, geometric weights (64-bit prefix), runs of zero weights.
    (O, D, W), nh = _skewed_graph(kinds, 31)
    g, keep = upload(O, D, W)
    starts = np.concatenate([np.arange(nh), np.arange(10, 4010, 7)])
    Y, lens = run(g, starts, 20, 30, FO, seed=4)
    Yo, lo = oracle.walks(O, D, W, starts, 20, 30, FO, seed=4)
    assert np.array_equal(Y, Yo) and np.array_equal(lens, lo)
    n2v.n2v_graph_release(g)


@pytest.mark.parametrize("weighted", [True, False])
def test_hub_sets_identical(weighted):
    """Membership sets of the long rows (built at upload: one bit per node and a
    running count per 480 ids) change no walk: set lookups of N(t) into v's set
    (positions from the counts) and of N(v) into t's set, forced whenever a
    side has a set or weighed by the automatic estimate, give the walks of a
    handle without sets and the oracle's."""
    O, D, W = synth.chung_lu(20000, 200000, 2.0, 20.0, 15000.0, (1, 1000), seed=12)
    if not weighted:
        W = None
    n = len(O) - 1
    g, keep = upload(O, D, W)
    Ot, Dt, Wt = keep
    gs = n2v.n2v_graph_upload(Ot, Dt, Wt, flags=n2v.N2V_UPLOAD_NO_PAIR_LISTS | n2v.N2V_UPLOAD_HUB_MIN_DEGREE_LOG2(6))
    g0 = n2v.n2v_graph_upload(Ot, Dt, Wt, flags=n2v.N2V_UPLOAD_NO_PAIR_LISTS | n2v.N2V_UPLOAD_NO_HUB_SETS)
    deg = (O[1:] - O[:-1]).astype(np.int64)
    info = n2v.n2v_graph_info(gs)
    assert info["hub_sets"] == int((deg >= 64).sum()) and info["hub_min_degree"] == 64
    assert n2v.n2v_graph_info(g0)["hub_sets"] == 0
    starts = np.arange(0, n, 7)
    rows = np.arange(0, starts.size, 29)
    for lanes, tile, route in ((64, 64, n2v.N2V_ROUTE_HUB_SETS), (64, 1, n2v.N2V_ROUTE_HUB_SETS),
                               (64, 4096, n2v.N2V_ROUTE_AUTO), (64, 64, n2v.N2V_ROUTE_AUTO)):
        n2v.n2v_set_tuning(lanes_per_walker=lanes, lds_tile=tile, list_cap=256, route=route)
        for p, q in ((0.25, 4.0), (1.0, 2.0), (4.0, 0.25), (2.0, 0.5)):
            Ys, Ls = run(gs, starts, 1, 24, NV, p, q, seed=31)
            Y0, L0 = run(g0, starts, 1, 24, NV, p, q, seed=31)
            assert np.array_equal(Ys, Y0) and np.array_equal(Ls, L0), (lanes, tile, route, p, q)
            Yo, lo = oracle.walks(O, D, W, starts, 1, 24, NV, p, q, 31, 0, rows=rows)
            assert np.array_equal(Ys[rows], Yo) and np.array_equal(Ls[rows], lo), (lanes, tile, route, p, q)
    n2v.n2v_set_tuning(reset=True)
    for h in (gs, g0, g):
        n2v.n2v_graph_release(h)
    del keep


def test_hub_sets_directed_self_loops():
    """Sets of out-rows of a directed graph with self-loops: a self-loop at t
    puts t in N(t) (a return, not a common neighbour), and membership follows
    the out-rows; walks equal the oracle's with the sets forced."""
    rng = np.random.default_rng(3)
    n = 3000
    hubs = rng.integers(0, n, 8)
    src = np.concatenate([rng.integers(0, n, 40000), np.repeat(hubs, 600), hubs])
    dst = np.concatenate([rng.integers(0, n, 40000), rng.integers(0, n, 4800), hubs])  # self-loops at the hubs
    O, D, W = synth.csr_from_edges(n, src, dst, rng.integers(1, 60, src.size), symmetric=False)
    g, keep = upload(O, D, W)
    Ot, Dt, Wt = keep
    gs = n2v.n2v_graph_upload(Ot, Dt, Wt, flags=n2v.N2V_UPLOAD_NO_PAIR_LISTS | n2v.N2V_UPLOAD_HUB_MIN_DEGREE_LOG2(4))
    assert n2v.n2v_graph_info(gs)["hub_sets"] > 0
    n2v.n2v_set_tuning(lanes_per_walker=64, route=n2v.N2V_ROUTE_HUB_SETS)
    for p, q in ((0.5, 2.0), (2.0, 0.25)):
        check(O, D, W, np.arange(n), 1, 20, NV, p, q, seed=4, g=gs)
    n2v.n2v_set_tuning(reset=True)
    n2v.n2v_graph_release(gs)
    n2v.n2v_graph_release(g)
    del keep
