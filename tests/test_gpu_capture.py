"""Plain walk launches captured in a HIP graph: under capture the kernels take
fixed walk shares instead of the per-stream counter, and every replay (with
eager work and synchronisations between replays) gives the eager walks."""
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


@pytest.mark.parametrize("kind,p,q", [(n2v.N2V_NODE2VEC, 0.25, 4.0), (n2v.N2V_NODE2VEC, 2.0, 1.0),
                                      (n2v.N2V_FIRST_ORDER, 1.0, 1.0)])
def test_captured_walks_replay_equal_eager(kind, p, q):
    O, D, W = synth.chung_lu(4000, 50000, 2.2, 20.0, 1800.0, (1, 100), seed=41)
    n = len(O) - 1
    g, keep = upload(O, D, W)
    S = torch.arange(n, dtype=torch.int32, device="cuda")

    def launch(Y, L):
        if kind == n2v.N2V_FIRST_ORDER:
            n2v.n2v_walks_first_order(g, S, 2, 24, 9, 0, Y, L)
        else:
            n2v.n2v_walks_node2vec(g, S, 2, 24, p, q, 9, 0, Y, L)

    ref_Y = torch.empty((2 * n, 24), dtype=torch.int32, device="cuda")
    ref_L = torch.empty(2 * n, dtype=torch.int32, device="cuda")
    launch(ref_Y, ref_L)  # eager (also warms the launch-shape caches)
    torch.cuda.synchronize()
    rows = np.arange(0, 2 * n, 17)
    Yo, lo = oracle.walks(O, D, W, np.arange(n), 2, 24, kind, p, q, 9, 0, rows=rows)
    assert np.array_equal(ref_Y.cpu().numpy()[rows], Yo) and np.array_equal(ref_L.cpu().numpy()[rows], lo)

    Y = torch.full((2 * n, 24), -7, dtype=torch.int32, device="cuda")
    L = torch.full((2 * n,), -7, dtype=torch.int32, device="cuda")
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        launch(Y, L)
    for _ in range(3):
        Y.fill_(-7)
        L.fill_(-7)
        other_Y = torch.empty_like(ref_Y)
        other_L = torch.empty_like(ref_L)
        launch(other_Y, other_L)  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(Y, ref_Y) and torch.equal(L, ref_L)
        assert torch.equal(other_Y, ref_Y) and torch.equal(other_L, ref_L)
    del graph
    n2v.n2v_graph_release(g)
    del keep
