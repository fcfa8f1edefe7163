"""Training corpora on the GPU vs the oracle, element by element: context
slots (SkipGram / CBOW windows, Walklets strides) and scale-free negatives,
on walks the GPU generated (so padding and ragged rows are the real ones)."""
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

NV = n2v.N2V_NODE2VEC


def _walks(g, n, reps, L, seed, extra_starts=()):
    starts = np.concatenate([np.arange(n), np.asarray(extra_starts, dtype=np.int64)]).astype(np.int32)
    S = torch.from_numpy(starts).cuda()
    Y, lens = n2v.n2v_walks_node2vec(g, S, reps, L, 0.5, 2.0, seed)
    torch.cuda.synchronize()
    return Y


def _check_contexts(Y, window, stride):
    C = n2v.n2v_walk_contexts(Y, window, stride)
    torch.cuda.synchronize()
    Co = oracle.contexts(Y.cpu().numpy(), window, stride)
    assert np.array_equal(C.cpu().numpy(), Co), (window, stride)


def _check_negatives(g, O, Y, n_neg, seed, base):
    N = n2v.n2v_negative_samples(g, Y, n_neg, seed, base)
    torch.cuda.synchronize()
    No = oracle.negatives(O, Y.cpu().numpy(), n_neg, seed, base)
    assert np.array_equal(N.cpu().numpy(), No), (n_neg, seed, base)


@pytest.mark.parametrize("name", sorted(synth.TINY))
def test_tiny_catalogue(name):
    O, D, W = synth.TINY[name]()
    n = len(O) - 1
    g, keep = upload(O, D, W)
    for L in (1, 2, 7, 300):
        Y = _walks(g, n, 3, L, seed=L, extra_starts=(-1, n))
        for window, stride in [(1, 1), (2, 1), (5, 1), (1, 2), (1, 3), (3, 2), (129, 1), (200, 3)]:
            _check_contexts(Y, window, stride)
        for n_neg in (1, 2, 5, 8):
            _check_negatives(g, O, Y, n_neg, seed=11 + n_neg, base=5)
    n2v.n2v_graph_release(g)


def test_fuzz():
    rng = np.random.default_rng(4)
    for it in range(40):
        O, D, W = synth.random_small(rng, n_max=20)
        n = len(O) - 1
        g, keep = upload(O, D, W)
        Y = _walks(g, n, int(rng.integers(1, 4)), int(rng.integers(1, 40)), seed=it, extra_starts=(-1,))
        _check_contexts(Y, int(rng.integers(1, 12)), int(rng.integers(1, 5)))
        _check_negatives(g, O, Y, int(rng.integers(1, 12)), seed=int(rng.integers(0, 2**63)),
                         base=int(rng.integers(0, 2**40)))
        n2v.n2v_graph_release(g)


def test_power_law_graph_with_isolated_nodes():
    # hubs, many degree-1 nodes and isolated nodes (empty offset intervals the
    # degree-proportional search must step over)
    O, D, W = synth.chung_lu(30000, 120000, 2.0, 8.0, 20000.0, (1, 50), seed=3)
    deg = O[1:] - O[:-1]
    assert (deg == 0).sum() > 1000 and deg.max() > 2000
    n = len(O) - 1
    g, keep = upload(O, D, W)
    Y = _walks(g, n, 1, 40, seed=1)
    for window, stride in [(5, 1), (10, 1), (1, 4)]:
        _check_contexts(Y, window, stride)
    for n_neg in (5, 6):
        _check_negatives(g, O, Y, n_neg, seed=99, base=2**33 + 7)
    # the guide table is reused: a second graph handle gets its own
    g2, keep2 = upload(O, D, W)
    _check_negatives(g2, O, Y, 3, seed=1, base=0)
    n2v.n2v_graph_release(g2)
    n2v.n2v_graph_release(g)


def test_negatives_follow_degrees():
    # large-sample frequency check of the GPU draws themselves
    O, D, W = synth.chung_lu(2000, 20000, 2.2, 10.0, 500.0, (1, 5), seed=8)
    n = len(O) - 1
    g, keep = upload(O, D, W)
    Y = torch.zeros((20000, 50), dtype=torch.int32, device="cuda")
    N = n2v.n2v_negative_samples(g, Y, 10, seed=5)
    counts = torch.bincount(N.flatten().long(), minlength=n).cpu().numpy().astype(np.float64)
    deg = (O[1:] - O[:-1]).astype(np.float64)
    exp = deg / deg.sum() * counts.sum()
    assert counts[deg == 0].sum() == 0
    sel = exp > 50
    z = (counts[sel] - exp[sel]) / np.sqrt(exp[sel])
    assert np.abs(z).max() < 6.0 and abs(z.mean()) < 0.2
    n2v.n2v_graph_release(g)


def test_empty_and_degenerate():
    # no edges at all: every slot -1
    O = np.zeros(6, dtype=np.uint64)
    D = np.zeros(0, dtype=np.int32)
    g, keep = upload(O, D, None)
    Y = torch.tensor([[0, 1, -1], [4, -1, -1]], dtype=torch.int32, device="cuda")
    N = n2v.n2v_negative_samples(g, Y, 4, seed=1)
    torch.cuda.synchronize()
    assert (N.cpu().numpy() == -1).all()
    # zero walks: nothing written, no error
    Y0 = torch.empty((0, 5), dtype=torch.int32, device="cuda")
    assert n2v.n2v_negative_samples(g, Y0, 3, seed=1).shape == (0, 5, 3)
    assert n2v.n2v_walk_contexts(Y0, 2).shape == (0, 5, 4)
    n2v.n2v_graph_release(g)
    # one node with a self loop
    O = np.array([0, 1], dtype=np.uint64)
    D = np.array([0], dtype=np.int32)
    g, keep = upload(O, D, None)
    Y = torch.tensor([[0, 0, 0]], dtype=torch.int32, device="cuda")
    _check_negatives(g, O, Y, 5, seed=3, base=0)
    _check_contexts(Y, 4, 1)
    n2v.n2v_graph_release(g)


def test_invalid_arguments():
    O, D, W = synth.TINY["k5"]()
    g, keep = upload(O, D, W)
    Y = torch.zeros((2, 3), dtype=torch.int32, device="cuda")
    C = torch.empty((2, 3, 2), dtype=torch.int32, device="cuda")
    lib = n2v.lib()
    assert lib.n2v_walk_contexts(Y.data_ptr(), 2, 3, 0, 1, C.data_ptr(), None) == n2v.N2V_ERR_INVALID_ARG
    assert lib.n2v_walk_contexts(Y.data_ptr(), 2, 3, 1, 0, C.data_ptr(), None) == n2v.N2V_ERR_INVALID_ARG
    assert lib.n2v_walk_contexts(Y.data_ptr(), 2, 0, 1, 1, C.data_ptr(), None) == n2v.N2V_ERR_INVALID_ARG
    assert lib.n2v_walk_contexts(Y.data_ptr(), 2, 3, (1 << 16) + 1, 1, C.data_ptr(), None) == n2v.N2V_ERR_INVALID_ARG
    assert lib.n2v_walk_contexts(None, 2, 3, 1, 1, C.data_ptr(), None) == n2v.N2V_ERR_INVALID_ARG
    assert lib.n2v_negative_samples(g, Y.data_ptr(), 2, 3, 0, 1, 0, C.data_ptr(), None) == n2v.N2V_ERR_INVALID_ARG
    assert lib.n2v_negative_samples(g + 999, Y.data_ptr(), 2, 3, 1, 1, 0, C.data_ptr(), None) == n2v.N2V_ERR_BAD_HANDLE
    n2v.n2v_graph_release(g)


def test_binding_holds_uploaded_tensors():
    # Tensors handed to n2v_graph_upload as temporaries stay alive until
    # release: new allocations cannot take their memory.
    O, D, W = synth.chung_lu(5000, 40000, 2.1, 12.0, 2000.0, (1, 100), seed=6)
    n = len(O) - 1
    g = n2v.n2v_graph_upload(torch.from_numpy(O.view(np.int64)).cuda(), torch.from_numpy(D).cuda(),
                             torch.from_numpy(W.view(np.int32)).cuda())
    filler = [torch.full((D.size + 64,), -7, dtype=torch.int32, device="cuda") for _ in range(4)]
    Y = _walks(g, n, 2, 30, seed=4)
    Yo, lo = oracle.walks(O, D, W, np.arange(n), 2, 30, oracle.NODE2VEC, 0.5, 2.0, 4, 0)
    assert np.array_equal(Y.cpu().numpy(), Yo)
    _check_negatives(g, O, Y, 4, seed=2, base=0)
    del filler
    n2v.n2v_graph_release(g)
    assert g not in n2v._borrowed


def test_long_walks_wide_reach():
    # reach window * stride beyond what the LDS tile holds: the global-gather
    # form; and strides far beyond the walk length
    O, D, W = synth.TINY["wdiamond"]()
    n = len(O) - 1
    g, keep = upload(O, D, W)
    Y = _walks(g, n, 1, 9000, seed=2, extra_starts=(-1,))
    for window, stride in [(8, 1000), (3, 4000), (2, 2**31 + 5), (1, 2**32 - 1), (4, 1)]:
        _check_contexts(Y, window, stride)
    _check_negatives(g, O, Y, 3, seed=8, base=2**32 - 2)
    n2v.n2v_graph_release(g)
