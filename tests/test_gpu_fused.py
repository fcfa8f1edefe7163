"""Fused walk -> context generation (no walk array): the context slots of
every position, emitted while the walk is taken, equal the contexts of the
materialised walks (GPU and oracle) element by element, for first-order and
node2vec walks, ragged lengths (dead ends, bad starts), SkipGram windows and
Walklets strides, on every walker-group width."""
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

FO, NV = n2v.N2V_FIRST_ORDER, n2v.N2V_NODE2VEC


@pytest.fixture(autouse=True)
def _reset_tuning():
    n2v.n2v_set_tuning(reset=True)
    yield
    n2v.n2v_set_tuning(reset=True)


def _check(g, O, D, W, starts, reps, L, kind, p, q, seed, base, window, stride):
    S = torch.from_numpy(np.ascontiguousarray(starts, dtype=np.int32)).cuda()
    C, lens = n2v.n2v_walks_contexts(g, kind, S, reps, L, p, q, seed, base, window, stride)
    if kind == FO:
        Y, lens_p = n2v.n2v_walks_first_order(g, S, reps, L, seed, base)
    else:
        Y, lens_p = n2v.n2v_walks_node2vec(g, S, reps, L, p, q, seed, base)
    Cu = n2v.n2v_walk_contexts(Y, window, stride)
    torch.cuda.synchronize()
    assert torch.equal(lens, lens_p)
    assert torch.equal(C, Cu), (L, kind, p, q, window, stride)
    Yo, lo = oracle.walks(O, D, W, starts, reps, L, kind, p, q, seed, base)
    assert np.array_equal(lens.cpu().numpy(), lo)
    assert np.array_equal(C.cpu().numpy(), oracle.contexts(Yo, window, stride))


@pytest.mark.parametrize("name", sorted(synth.TINY))
def test_tiny_catalogue(name):
    O, D, W = synth.TINY[name]()
    n = len(O) - 1
    g, keep = upload(O, D, W)
    starts = np.concatenate([np.arange(n), [-1, n]]).astype(np.int32)
    for L in (1, 2, 7, 40):
        for kind, p, q in ((FO, 1.0, 1.0), (NV, 0.25, 4.0), (NV, 2.0, 1.0)):
            for window, stride in ((1, 1), (2, 1), (5, 1), (1, 3), (3, 2)):
                _check(g, O, D, W, starts, 2, L, kind, p, q, 7, 3, window, stride)
    n2v.n2v_graph_release(g)
    del keep


@pytest.mark.parametrize("lanes", [4, 16, 64])
def test_power_law_all_group_widths(lanes):
    O, D, W = synth.chung_lu(5000, 40000, 2.2, 16.0, 600.0, (1, 100), seed=9)
    n = len(O) - 1
    g, keep = upload(O, D, W)
    n2v.n2v_set_tuning(lanes_per_walker=lanes)
    starts = np.arange(n, dtype=np.int32)
    for kind, p, q in ((NV, 0.25, 4.0), (NV, 1.0, 2.0), (FO, 1.0, 1.0)):
        for window, stride, L in ((5, 1, 80), (1, 4, 30), (20, 1, 60), (2, 3, 9)):
            _check(g, O, D, W, starts, 1, L, kind, p, q, 11, 0, window, stride)
    n2v.n2v_graph_release(g)
    del keep


def test_automatic_four_lane_lists_only():
    """Every edge keeps its stored list and the launch has at least 96 walks per
    CU: the fused kernel's automatic shape is 4-lane groups of the lists-only
    variant; its contexts equal those of the materialised walks and the
    oracle's."""
    O, D, W = synth.chung_lu(20000, 200000, 2.2, 20.0, 2000.0, (1, 100), seed=31)
    n = len(O) - 1
    g, keep = upload(O, D, W)
    assert n2v.n2v_graph_info(g)["pair_lists"] == len(D)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    reps = -(-96 * cus // n)
    starts = np.arange(n, dtype=np.int32)
    for kind, p, q in ((NV, 0.25, 4.0), (NV, 2.0, 1.0), (FO, 1.0, 1.0)):
        _check(g, O, D, W, starts, reps, 20, kind, p, q, 19, 0, 5, 1)
    n2v.n2v_graph_release(g)
    del keep


def test_errors():
    O, D, W = synth.TINY["tri_tail"]()
    g, keep = upload(O, D, W)
    S = torch.zeros(3, dtype=torch.int32, device="cuda")
    with pytest.raises(n2v.N2VError):
        n2v.n2v_walks_contexts(g, NV, S, 1, 10, 1.0, 1.0, 0, 0, 0, 1)  # window 0
    with pytest.raises(n2v.N2VError):
        n2v.n2v_walks_contexts(g, NV, S, 1, 10, 1.0, 1.0, 0, 0, 1, 0)  # stride 0
    with pytest.raises(n2v.N2VError):
        n2v.n2v_walks_contexts(g, NV, S, 1, 5000, 1.0, 1.0, 0, 0, 2000, 1)  # halo beyond the fused limit
    n2v.n2v_graph_release(g)
    del keep
