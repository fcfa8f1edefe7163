"""The allocation-free batched entry point (tables in the library's fixed
device array) gives the same walks as n2v_walks_batched, bit for bit, on two
calls in a row (the second smaller, so stale table entries from the first
would show), called through the C ABI."""
import ctypes

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2110_06196_amd as n2v  # noqa: E402
from tests._devutil import upload  # noqa: E402

NV, FO = n2v.N2V_NODE2VEC, n2v.N2V_FIRST_ORDER
PQ = [0.25, 1.0, 4.0]


@pytest.fixture(scope="module")
def graphs():
    gs = []
    for k in range(4):
        n = [3000, 20000, 800, 6000][k]
        O, D, W = synth.chung_lu(n, n * 8, 2.2, 16.0, (n * 16.0) ** 0.5 * 3, (1, 100), seed=70 + k)
        if k == 2:
            W = None
        g, keep = upload(O, D, W)
        gs.append((g, (O, D, W), keep))
    yield gs
    for g, _, _ in gs:
        n2v.n2v_graph_release(g)


def requests(graphs, n_req, max_starts, max_len, seed):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_req):
        gi = int(rng.integers(0, len(graphs)))
        g, (O, D, W), _ = graphs[gi]
        n = len(O) - 1
        ns = int(rng.integers(1, max_starts + 1)) if k % 9 else 0
        starts = rng.integers(-1, n, size=ns).astype(np.int32)
        out.append(dict(gi=gi, g=g, starts=starts, reps=int(rng.integers(1, 3)), L=int(rng.integers(1, max_len + 1)),
                        kind=FO if k % 5 == 0 else NV, p=float(rng.choice(PQ)), q=float(rng.choice(PQ)),
                        seed=500 + k, base=int(rng.integers(0, 2**40)), k_approx=3 if k % 11 == 4 else 0))
    return out


def descs_and_bufs(reqs, fill):
    descs, bufs = [], []
    for r in reqs:
        S = torch.from_numpy(r["starts"]).cuda()
        nw = r["starts"].size * r["reps"]
        Y = torch.full((nw, r["L"]), fill, dtype=torch.int32, device="cuda")
        lens = torch.full((nw,), fill, dtype=torch.int32, device="cuda")
        descs.append(n2v.make_request(r["g"], r["kind"], S, r["reps"], r["L"], r["p"], r["q"], r["seed"], r["base"],
                                      Y, lens, k_approx=r["k_approx"]))
        bufs.append((S, Y, lens))
    return descs, bufs


def call_noalloc(descs):
    """Through the C ABI directly (ctypes), on torch's current stream."""
    L = n2v.lib()
    arr = (n2v.RequestDesc * len(descs))(*descs)
    rc = L.n2v_walks_batched_noalloc(arr, len(descs), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == n2v.N2V_OK, L.n2v_last_error()


def check_equal(graphs, reqs, ref, got):
    for i, r in enumerate(reqs):
        a, b = ref[i], got[i]
        assert torch.equal(a[1], b[1]) and torch.equal(a[2], b[2]), (i, r["kind"], r["p"], r["q"], r["k_approx"])
    # a few rows of the first requests against the oracle as well
    for i, r in enumerate(reqs[:6]):
        nw = r["starts"].size * r["reps"]
        if nw == 0:
            continue
        rows = np.unique(np.linspace(0, nw - 1, 3).astype(np.int64))
        O, D, W = graphs[r["gi"]][1]
        Yo, lo = oracle.walks(O, D, W, r["starts"], r["reps"], r["L"], r["kind"], r["p"], r["q"], r["seed"],
                              r["base"], rows, k_approx=r["k_approx"])
        assert np.array_equal(got[i][1].cpu().numpy()[rows], Yo) and np.array_equal(got[i][2].cpu().numpy()[rows], lo)


def test_noalloc_equals_batched_two_calls(graphs):
    # call 1: about 1.75e6 walks with 4-lane groups (a queue of tens of
    # thousands of chunks in the fixed array)
    big = requests(graphs, 64, 40000, 8, seed=1)
    print(f"[no_alloc] call 1: {len(big)} requests, {sum(r['starts'].size * r['reps'] for r in big)} walks", flush=True)
    d_ref, b_ref = descs_and_bufs(big, -7)
    d_new, b_new = descs_and_bufs(big, -9)
    n2v.n2v_set_tuning(lanes_per_walker=4, lds_tile=16, list_cap=32)
    try:
        n2v.n2v_walks_batched(d_ref)
        call_noalloc(d_new)
        torch.cuda.synchronize()
    finally:
        n2v.n2v_set_tuning(reset=True)
    check_equal(graphs, big, b_ref, b_new)
    del b_ref, b_new
    # call 2: a smaller batch with the automatic shape
    small = requests(graphs, 40, 300, 60, seed=2)
    print(f"[no_alloc] call 2: {len(small)} requests", flush=True)
    d_ref, b_ref = descs_and_bufs(small, -7)
    d_new, b_new = descs_and_bufs(small, -9)
    n2v.n2v_walks_batched(d_ref)
    call_noalloc(d_new)
    torch.cuda.synchronize()
    check_equal(graphs, small, b_ref, b_new)


def test_noalloc_rejects_over_limit():
    L = n2v.lib()
    arr = (n2v.RequestDesc * 4097)()
    assert L.n2v_walks_batched_noalloc(arr, 4097, None) == n2v.N2V_ERR_INVALID_ARG
    assert b"4096" in L.n2v_last_error()
