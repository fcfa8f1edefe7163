"""Batched and served forms: every request's walks equal the plain entry
point's (and the oracle's on samples), whatever its company, arrival time or
admission order."""
import time

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

NV, FO = n2v.N2V_NODE2VEC, n2v.N2V_FIRST_ORDER
PQ = [0.25, 1.0, 4.0]


@pytest.fixture(scope="module")
def graphs():
    gs = []
    for k in range(6):
        n = [300, 2000, 5000, 800, 12000, 3000][k]
        O, D, W = synth.chung_lu(n, n * 8, 2.2, 16.0, (n * 16.0) ** 0.5 * 3, (1, 100), seed=50 + k)
        if k == 3:
            W = None
        g, keep = upload(O, D, W)
        gs.append((g, (O, D, W), keep))
    yield gs
    for g, _, _ in gs:
        n2v.n2v_graph_release(g)


def make_requests(graphs, n_req, seed, approx=False):
    """Random requests over the module's graphs; approx=True makes every fourth
    request an approximated one (k in {1, 3, 8}, below the hubs' degrees)."""
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(n_req):
        gi = int(rng.integers(0, len(graphs)))
        g, (O, D, W), _ = graphs[gi]
        n = len(O) - 1
        ns = int(rng.integers(1, 400)) if k % 7 else 0 if k % 14 == 0 else 1
        starts = rng.integers(-1, n, size=ns).astype(np.int32)
        L = int(rng.integers(1, 60))
        kind = FO if k % 5 == 0 else NV
        p, q = float(rng.choice(PQ)), float(rng.choice(PQ))
        ka = int(rng.choice([1, 3, 8])) if approx and k % 4 == 1 else 0
        reqs.append(dict(gi=gi, g=g, starts=starts, reps=int(rng.integers(1, 3)), L=L, kind=kind, p=p, q=q,
                         seed=1000 + k, base=int(rng.integers(0, 2**40)), k_approx=ka))
    return reqs


def plain(r):
    if r.get("k_approx", 0):
        S = torch.from_numpy(np.ascontiguousarray(r["starts"], dtype=np.int32)).cuda()
        Y, lens = n2v.n2v_walks_approximated(r["g"], r["kind"], S, r["reps"], r["L"], r["p"], r["q"], r["k_approx"],
                                             r["seed"], r["base"])
        torch.cuda.synchronize()
        return Y.cpu().numpy(), lens.cpu().numpy()
    return run(r["g"], r["starts"], r["reps"], r["L"], r["kind"], r["p"], r["q"], r["seed"], r["base"])


def oracle_rows(graphs, r, rows=None):
    """The oracle's walks of request r (all rows, or the given row indices)."""
    O, D, W = graphs[r["gi"]][1]
    return oracle.walks(O, D, W, r["starts"], r["reps"], r["L"], r["kind"], r["p"], r["q"], r["seed"], r["base"],
                        rows, k_approx=r.get("k_approx", 0))


def check_against_oracle(graphs, r, Y, lens, small=64, sample=8):
    """Every row of a request of at most `small` walks, else `sample` evenly
    spaced rows (first and last included), equal the oracle's."""
    nw = Y.shape[0]
    if nw == 0:
        return
    if nw <= small:
        Yo, lo = oracle_rows(graphs, r)
        assert np.array_equal(Y, Yo) and np.array_equal(lens, lo)
        return
    rows = np.unique(np.linspace(0, nw - 1, sample).astype(np.int64))
    Yo, lo = oracle_rows(graphs, r, rows)
    assert np.array_equal(Y[rows], Yo) and np.array_equal(lens[rows], lo)


def device_descs(reqs):
    descs, bufs = [], []
    for r in reqs:
        S = torch.from_numpy(r["starts"]).cuda()
        nw = r["starts"].size * r["reps"]
        Y = torch.full((nw, r["L"]), -7, dtype=torch.int32, device="cuda")
        lens = torch.full((nw,), -7, dtype=torch.int32, device="cuda")
        descs.append(n2v.make_request(r["g"], r["kind"], S, r["reps"], r["L"], r["p"], r["q"], r["seed"],
                                      r["base"], Y, lens))
        bufs.append((S, Y, lens))
    return descs, bufs


def test_batched_equals_plain_and_oracle(graphs):
    reqs = make_requests(graphs, 160, seed=1)
    descs, bufs = device_descs(reqs)
    n2v.n2v_walks_batched(descs)
    torch.cuda.synchronize()
    for i, r in enumerate(reqs):
        Yp, lp = plain(r)
        Yb, lb = bufs[i][1].cpu().numpy(), bufs[i][2].cpu().numpy()
        assert np.array_equal(Yb, Yp) and np.array_equal(lb, lp), i
        if i % 16 == 0:
            O, D, W = graphs[r["gi"]][1]
            Yo, lo = oracle.walks(O, D, W, r["starts"], r["reps"], r["L"], r["kind"], r["p"], r["q"], r["seed"],
                                  r["base"])
            assert np.array_equal(Yb, Yo) and np.array_equal(lb, lo), i


def test_batched_four_lane_groups(graphs):
    """The queue kernel with 4-lane groups (16 walks per wavefront, the shape
    of graphs whose edges all keep a stored list) gives the plain walks and the
    oracle's."""
    reqs = make_requests(graphs, 60, seed=3)
    descs, bufs = device_descs(reqs)
    n2v.n2v_set_tuning(lanes_per_walker=4, lds_tile=16, list_cap=32)
    try:
        b = n2v.n2v_batch_create(descs, autotune=False)
        assert n2v.n2v_batch_info(b)["lanes_per_walker"] == 4
        n2v.n2v_batch_launch(b)
        torch.cuda.synchronize()
        n2v.n2v_batch_destroy(b)
    finally:
        n2v.n2v_set_tuning(reset=True)
    for i, r in enumerate(reqs):
        Yp, lp = plain(r)
        Yb, lb = bufs[i][1].cpu().numpy(), bufs[i][2].cpu().numpy()
        assert np.array_equal(Yb, Yp) and np.array_equal(lb, lp), i
        if i % 10 == 0:
            O, D, W = graphs[r["gi"]][1]
            Yo, lo = oracle.walks(O, D, W, r["starts"], r["reps"], r["L"], r["kind"], r["p"], r["q"], r["seed"],
                                  r["base"])
            assert np.array_equal(Yb, Yo) and np.array_equal(lb, lo), i


def test_batch_plan_graph_replays(graphs):
    """The captured hipGraph is replayed several times with eager work and
    synchronisations in between; every replay reproduces the eager walks."""
    reqs = make_requests(graphs, 90, seed=2)
    descs, bufs = device_descs(reqs)
    ref = [plain(r) for r in reqs]
    for autotune in (True, False):
        b = n2v.n2v_batch_create(descs, autotune=autotune)
        info = n2v.n2v_batch_info(b)
        assert info["n_requests"] == len(reqs) and info["lanes_per_walker"] in (4, 16, 32, 64)
        for rep in range(3):
            for _, Y, lens in bufs:
                Y.fill_(-9)
                lens.fill_(-9)
            x = torch.randn(1000, device="cuda").sum()  # unrelated eager work
            n2v.n2v_batch_launch(b)
            torch.cuda.synchronize()
            assert torch.isfinite(x)
            for i in range(len(reqs)):
                assert np.array_equal(bufs[i][1].cpu().numpy(), ref[i][0]), (autotune, rep, i)
                assert np.array_equal(bufs[i][2].cpu().numpy(), ref[i][1]), (autotune, rep, i)
        n2v.n2v_batch_destroy(b)


def _drain(srv, ids, on_done, timeout=60.0):
    """Poll until every request is done; on_done(k, result) consumes (and
    releases) each result as it finishes, which frees its memory budget."""
    pending = dict(ids)
    t0 = time.time()
    while pending:
        for k in list(pending):
            res = n2v.n2v_request_poll(srv, pending[k])
            if res is not None:
                on_done(k, res)
                del pending[k]
        assert time.time() - t0 < timeout, f"server did not finish ({len(pending)} pending)"
        time.sleep(0.0005)


def _fetch(res, L):
    Y, lens = n2v.result_tensors(res, L)
    return Y.cpu().numpy(), lens.cpu().numpy()


def serve_all(graphs, reqs, budget_bytes, slots, tuning=None, pause_seed=9):
    """Submit every request to a new server (some while others run), drain it
    and return {k: ((walks, lens), steps, (t_arrival, t_admit, t_start, t_done))}."""
    srv = n2v.n2v_server_create(budget_bytes, slots, tuning)
    for g, _, _ in graphs:
        n2v.n2v_server_add_graph(srv, g)
    ids, keep = {}, []
    rng = np.random.default_rng(pause_seed)
    for k, r in enumerate(reqs):
        d, arr = n2v.host_request(r["g"], r["kind"], r["starts"], r["reps"], r["L"], r["p"], r["q"], r["seed"],
                                  r["base"], r.get("k_approx", 0))
        keep.append(arr)
        ids[k] = n2v.n2v_request_submit(srv, d, time.monotonic_ns())
        if rng.random() < 0.3:
            time.sleep(0.0005)
    got = {}

    def on_done(k, res):
        got[k] = (_fetch(res, reqs[k]["L"]), int(res.steps),
                  (res.t_arrival_ns, res.t_admit_ns, res.t_start_ns, res.t_done_ns))
        n2v.n2v_request_release(srv, ids[k])

    _drain(srv, ids, on_done)
    n2v.n2v_server_destroy(srv)
    return got


@pytest.mark.parametrize("budget_mb,slots", [(4096, 64), (2, 3)])
def test_server_mix_equals_alone(graphs, budget_mb, slots):
    """Requests submitted while others run (continuous batching) produce the
    walks of their plain, alone runs and the oracle's (every row of requests of
    up to 64 walks, 8 sampled rows of larger ones), approximated requests
    included; a squeezed budget forces queueing."""
    reqs = make_requests(graphs, 120, seed=3, approx=True)
    assert any(r["k_approx"] for r in reqs)
    got = serve_all(graphs, reqs, budget_mb << 20, slots)
    for k, r in enumerate(reqs):
        (Y, lens), steps, (ta, tad, ts, td) = got[k]
        Yp, lp = plain(r)
        assert np.array_equal(Y, Yp) and np.array_equal(lens, lp), k
        check_against_oracle(graphs, r, Y, lens)
        assert steps == int(np.maximum(lp.astype(np.int64) - 1, 0).sum())
        assert ta <= tad <= ts <= td


def test_server_fixed_tuning_equals_automatic(graphs):
    """A server created with a fixed launch shape (through the tuning argument
    of n2v_server_create) returns the walks of a server with the automatic
    shape (NULL), and the oracle's."""
    reqs = make_requests(graphs, 60, seed=11, approx=True)
    auto = serve_all(graphs, reqs, 4096 << 20, 32, None)
    for shape in (dict(lanes_per_walker=4, lds_tile=16, list_cap=32), dict(lanes_per_walker=32, lds_tile=64,
                                                                         list_cap=256, route=n2v.N2V_ROUTE_MERGE)):
        fixed = serve_all(graphs, reqs, 4096 << 20, 32, shape)
        for k, r in enumerate(reqs):
            (Ya, la), sa, _ = auto[k]
            (Yf, lf), sf, _ = fixed[k]
            assert np.array_equal(Ya, Yf) and np.array_equal(la, lf) and sa == sf, (shape, k)
    for k, r in enumerate(reqs):
        (Y, lens), _, _ = auto[k]
        check_against_oracle(graphs, r, Y, lens)


def test_server_rejects_and_errors(graphs):
    srv = n2v.n2v_server_create(1 << 16, 4)
    g = graphs[0][0]
    n2v.n2v_server_add_graph(srv, g)
    big = np.zeros(5000, dtype=np.int32)
    d, arr = n2v.host_request(g, NV, big, 1, 50, 1.0, 2.0, 1)
    with pytest.raises(n2v.N2VError) as e:
        n2v.n2v_request_submit(srv, d, 0)
    assert e.value.code == n2v.N2V_ERR_REJECTED
    d, arr = n2v.host_request(g, NV, big[:10], 1, 5, -1.0, 2.0, 1)
    with pytest.raises(n2v.N2VError) as e:
        n2v.n2v_request_submit(srv, d, 0)
    assert e.value.code == n2v.N2V_ERR_INVALID_ARG
    other = graphs[1][0]
    d, arr = n2v.host_request(other, NV, big[:10], 1, 5, 1.0, 2.0, 1)
    with pytest.raises(n2v.N2VError) as e:
        n2v.n2v_request_submit(srv, d, 0)
    assert e.value.code == n2v.N2V_ERR_BAD_HANDLE
    with pytest.raises(n2v.N2VError):
        n2v.n2v_request_poll(srv, 12345)
    n2v.n2v_server_destroy(srv)
    with pytest.raises(n2v.N2VError):
        n2v.n2v_server_destroy(srv)
