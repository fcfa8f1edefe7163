"""The batched and served workloads at their stated size, checked against the
oracle.

64 Chung-Lu graphs (n log-uniform in [1e3, 1e6], mean degree U[8, 32], degree
exponent 2.2, max expected degree sqrt(n * mean), weights U[1, 100], seeds
100 + g; 13.3M nodes, 265M entries) and 4096 node2vec requests (seed 7: graph
uniform, 1..1e4 starts drawn with replacement, length U[10, 200], (p, q) uniform
over {0.25, 1, 4}^2, Philox seed 1000 + k; 2.06e7 walks).  The batched form runs
them in one replay of the captured persistent launch (autotuned shape); the
served form takes them under open-loop Poisson arrivals at 1000 req/s.  For
every request, 4 evenly spaced walks, and every walk of the 64 smallest
requests, equal the oracle's; the served walks equal the batched ones on the
same rows.
"""
import concurrent.futures as cf
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

NV = n2v.N2V_NODE2VEC
THREADS = 16


@pytest.fixture(scope="module")
def workload():
    t0 = time.time()
    ps, host = synth.many_graphs(threads=THREADS)
    print(f"[c4] 64 graphs generated in {time.time() - t0:.1f} s", flush=True)
    graphs, keep = [], []
    for (O, D, W) in host:
        Ot = torch.from_numpy(O.view(np.int64)).cuda()
        Dt = torch.from_numpy(D).cuda()
        Wt = torch.from_numpy(W.view(np.int32)).cuda()
        graphs.append(n2v.n2v_graph_upload(Ot, Dt, Wt))
        keep.append((Ot, Dt, Wt))
    torch.cuda.synchronize()
    reqs = synth.many_requests([p["n"] for p in ps])
    assert len(reqs) == 4096
    # rows checked against the oracle: 4 evenly spaced walks of every request,
    # every walk of the 64 smallest
    small = set(np.argsort([r["starts"].size for r in reqs], kind="stable")[:64].tolist())
    rows = []
    for k, r in enumerate(reqs):
        nw = r["starts"].size
        rows.append(np.arange(nw, dtype=np.int64) if k in small
                    else np.unique(np.linspace(0, nw - 1, min(4, nw)).astype(np.int64)))
    t0 = time.time()

    def one(k):
        r = reqs[k]
        O, D, W = host[r["graph"]]
        return oracle.walks(O, D, W, r["starts"], 1, r["walk_len"], NV, r["p"], r["q"], r["seed"], 0, rows[k])

    with cf.ThreadPoolExecutor(THREADS) as ex:
        expect = list(ex.map(one, range(len(reqs))))
    print(f"[c4] oracle on {sum(x.size for x in rows)} walks in {time.time() - t0:.1f} s", flush=True)
    yield dict(graphs=graphs, reqs=reqs, rows=rows, expect=expect)
    torch.cuda.synchronize()
    for g in graphs:
        n2v.n2v_graph_release(g)


@pytest.mark.timeout(600)
def test_c4_batched_full_size(workload):
    graphs, reqs, rows, expect = workload["graphs"], workload["reqs"], workload["rows"], workload["expect"]
    bufs, descs = [], []
    for r in reqs:
        S = torch.from_numpy(r["starts"]).cuda()
        nw = r["starts"].size
        Y = torch.full((nw, r["walk_len"]), -7, dtype=torch.int32, device="cuda")
        lens = torch.full((nw,), -7, dtype=torch.int32, device="cuda")
        bufs.append((S, Y, lens))
        descs.append(n2v.make_request(graphs[r["graph"]], NV, S, 1, r["walk_len"], r["p"], r["q"], r["seed"], 0,
                                      Y, lens))
    plan = n2v.n2v_batch_create(descs, autotune=True)
    info = n2v.n2v_batch_info(plan)
    assert info["n_requests"] == 4096 and info["n_walks"] == sum(r["starts"].size for r in reqs)
    n2v.n2v_batch_launch(plan)
    torch.cuda.synchronize()
    print(f"[c4] batched shape {info['lanes_per_walker']} lanes, {info['n_chunks']} chunks", flush=True)
    bad = []
    for k, r in enumerate(reqs):
        idx = torch.from_numpy(rows[k]).cuda()
        Yg = bufs[k][1].index_select(0, idx).cpu().numpy()
        lg = bufs[k][2].index_select(0, idx).cpu().numpy()
        Yo, lo = expect[k]
        if not (np.array_equal(Yg, Yo) and np.array_equal(lg, lo)):
            bad.append(k)
    n2v.n2v_batch_destroy(plan)
    workload["batched"] = [(bufs[k][1].index_select(0, torch.from_numpy(rows[k]).cuda()).cpu().numpy())
                           for k in range(len(reqs))]
    del bufs
    assert not bad, f"requests differing from the oracle: {bad[:20]}"


@pytest.mark.timeout(600)
def test_c5_served_full_size(workload):
    """Open-loop Poisson arrivals (seed 11) at 1000 req/s, 200 GB budget."""
    graphs, reqs, rows, expect = workload["graphs"], workload["reqs"], workload["rows"], workload["expect"]
    srv = n2v.n2v_server_create(200 << 30, 4096)
    for g in graphs:
        n2v.n2v_server_add_graph(srv, g)
    hdesc = [n2v.host_request(graphs[r["graph"]], NV, r["starts"], 1, r["walk_len"], r["p"], r["q"], r["seed"])
             for r in reqs]
    arr = synth.poisson_arrivals(len(reqs), 1000.0)
    ids = [0] * len(reqs)
    got = [None] * len(reqs)
    lat = np.zeros(len(reqs))
    t0 = time.monotonic_ns() + 10_000_000
    nxt = 0
    pending = set()
    deadline = time.time() + 300
    while nxt < len(reqs) or pending:
        now = time.monotonic_ns()
        while nxt < len(reqs) and t0 + int(arr[nxt] * 1e9) <= now:
            ids[nxt] = n2v.n2v_request_submit(srv, hdesc[nxt][0], t0 + int(arr[nxt] * 1e9))
            pending.add(nxt)
            nxt += 1
        for k in list(pending):
            res = n2v.n2v_request_poll(srv, ids[k])
            if res is None:
                continue
            Y, lens = n2v.result_tensors(res, reqs[k]["walk_len"])
            idx = torch.from_numpy(rows[k]).cuda()
            got[k] = (Y.index_select(0, idx).cpu().numpy(), lens.index_select(0, idx).cpu().numpy(),
                      int(res.steps), int(lens.to(torch.int64).sub(1).clamp(min=0).sum().item()))
            lat[k] = (res.t_done_ns - res.t_arrival_ns) / 1e6
            n2v.n2v_request_release(srv, ids[k])
            pending.discard(k)
        assert time.time() < deadline, f"server did not finish ({len(pending)} pending)"
        time.sleep(0.0002)
    n2v.n2v_server_destroy(srv)
    print(f"[c5] 1000 req/s: p50 {np.percentile(lat, 50):.1f} ms, p99 {np.percentile(lat, 99):.1f} ms", flush=True)
    bad = []
    for k in range(len(reqs)):
        Yg, lg, steps, steps_full = got[k]
        Yo, lo = expect[k]
        ok = np.array_equal(Yg, Yo) and np.array_equal(lg, lo) and steps == steps_full
        if "batched" in workload:
            ok = ok and np.array_equal(Yg, workload["batched"][k])
        if not ok:
            bad.append(k)
    assert not bad, f"served requests differing from the oracle: {bad[:20]}"
