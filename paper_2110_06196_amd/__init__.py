"""Exact DeepWalk / node2vec walk generation on AMD Instinct MI355X.

Thin ctypes binding over the C ABI in ``include/n2vwalk.h`` (library
``libn2vwalk.so``, built by ``paper_2110_06196_amd.build``).  The functions
keep the C names; they take torch tensors for device memory and torch streams,
marshal pointers and sizes, and raise ``N2VError`` on a non-zero status.
Every step of the walk runs in the library's HIP kernels: there is no CPU or
PyTorch fallback, and importing this module without the built library raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch  # loaded first so the library binds to the same HIP runtime

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libn2vwalk.so")

N2V_OK, N2V_PENDING = 0, 1
N2V_ERR_INVALID_ARG, N2V_ERR_UNSORTED, N2V_ERR_OVERFLOW = -1, -2, -3
N2V_ERR_NOMEM, N2V_ERR_HIP, N2V_ERR_BAD_HANDLE, N2V_ERR_REJECTED = -4, -5, -6, -7
N2V_STORAGE_CSR, N2V_STORAGE_EF = 0, 1
N2V_FIRST_ORDER, N2V_NODE2VEC = 0, 1
N2V_TUNE_GENERIC_ONLY = 1
N2V_UPLOAD_NO_PAIR_LISTS = 1
N2V_UPLOAD_NO_HUB_SETS = 2
N2V_ROUTE_AUTO, N2V_ROUTE_TWO_PASS, N2V_ROUTE_PROBE, N2V_ROUTE_STREAM, N2V_ROUTE_MERGE = 0, 1, 2, 3, 4
N2V_ROUTE_HUB_SETS = 5


def N2V_UPLOAD_HUB_MIN_DEGREE_LOG2(k: int) -> int:
    return (k & 31) << 8
N2V_BATCH_AUTOTUNE = 1

_STATUS = {
    0: "OK", 1: "PENDING", -1: "INVALID_ARG", -2: "UNSORTED", -3: "OVERFLOW", -4: "NOMEM",
    -5: "HIP", -6: "BAD_HANDLE", -7: "REJECTED",
}


class N2VError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class GraphInfo(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_uint64), ("n_entries", ctypes.c_uint64),
                ("max_degree", ctypes.c_uint64), ("max_row_wsum", ctypes.c_uint64),
                ("sum_deg_sq", ctypes.c_uint64), ("weighted", ctypes.c_uint32),
                ("prefix_bytes", ctypes.c_uint32), ("device_bytes", ctypes.c_uint64),
                ("storage", ctypes.c_uint32), ("ef_quantum", ctypes.c_uint32),
                ("pair_lists", ctypes.c_uint64), ("pair_entries", ctypes.c_uint64),
                ("hub_sets", ctypes.c_uint64), ("hub_min_degree", ctypes.c_uint64)]


class EFInfo(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("l", ctypes.c_uint32), ("quantum", ctypes.c_uint32),
                ("pad", ctypes.c_uint32), ("u", ctypes.c_uint64), ("n_codes", ctypes.c_uint64),
                ("n_zeros", ctypes.c_uint64), ("h_bits", ctypes.c_uint64), ("h_words", ctypes.c_uint64),
                ("l_words", ctypes.c_uint64), ("s1_len", ctypes.c_uint64), ("s0_len", ctypes.c_uint64),
                ("d_H", ctypes.c_void_p), ("d_L", ctypes.c_void_p), ("d_S1", ctypes.c_void_p),
                ("d_S0", ctypes.c_void_p)]


class Tuning(ctypes.Structure):
    _fields_ = [("lanes_per_walker", ctypes.c_uint32), ("lds_tile", ctypes.c_uint32),
                ("list_cap", ctypes.c_uint32), ("route", ctypes.c_uint32), ("flags", ctypes.c_uint32)]


class RequestDesc(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_uint64), ("kind", ctypes.c_uint32),
                ("walks_per_start", ctypes.c_uint32), ("walk_len", ctypes.c_uint32),
                ("k_approx", ctypes.c_uint32), ("p", ctypes.c_double), ("q", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("walk_id_base", ctypes.c_uint64),
                ("d_starts", ctypes.c_void_p), ("n_starts", ctypes.c_uint64),
                ("d_walks", ctypes.c_void_p), ("d_lens", ctypes.c_void_p)]


class BatchInfo(ctypes.Structure):
    _fields_ = [("n_requests", ctypes.c_uint32), ("n_chunks", ctypes.c_uint32),
                ("lanes_per_walker", ctypes.c_uint32), ("lds_tile", ctypes.c_uint32),
                ("list_cap", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("n_walks", ctypes.c_uint64), ("est_cost", ctypes.c_double)]


class Result(ctypes.Structure):
    _fields_ = [("d_walks", ctypes.c_void_p), ("d_lens", ctypes.c_void_p),
                ("n_walks", ctypes.c_uint64), ("steps", ctypes.c_uint64),
                ("t_arrival_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64),
                ("t_start_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64)]


# Every exported symbol with its ctypes signature (also checked by the tests).
_U64, _U32, _I32, _VP, _D = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p, ctypes.c_double
SIGNATURES = {
    "n2v_graph_upload": [_VP, _U64, _VP, _U64, _VP, _U32, _VP, ctypes.POINTER(_U64)],
    "n2v_graph_info": [_U64, ctypes.POINTER(GraphInfo)],
    "n2v_graph_release": [_U64],
    "n2v_walks_first_order": [_U64, _VP, _U64, _U32, _U32, _U64, _U64, _VP, _VP, _VP],
    "n2v_walks_node2vec": [_U64, _VP, _U64, _U32, _U32, _D, _D, _U64, _U64, _VP, _VP, _VP],
    "n2v_walks_approximated": [_U64, _U32, _VP, _U64, _U32, _U32, _D, _D, _U32, _U64, _U64, _VP, _VP, _VP],
    "n2v_graph_upload_ef": [_VP, _U64, _VP, _U64, _VP, _U32, _VP, ctypes.POINTER(ctypes.c_uint64)],
    "n2v_ef_info": [_U64, ctypes.POINTER(EFInfo)],
    "n2v_ef_select": [_U64, _VP, _U64, _VP, _VP],
    "n2v_ef_rank": [_U64, _VP, _U64, _VP, _VP],
    "n2v_walk_contexts": [_VP, _U64, _U32, _U32, _U32, _VP, _VP],
    "n2v_walks_contexts": [_U64, _U32, _VP, _U64, _U32, _U32, _D, _D, _U64, _U64, _U32, _U32, _VP, _VP, _VP],
    "n2v_negative_samples": [_U64, _VP, _U64, _U32, _U32, _U64, _U64, _VP, _VP],
    "n2v_set_tuning": [ctypes.POINTER(Tuning)],
    "n2v_walks_batched": [ctypes.POINTER(RequestDesc), _U32, _VP],
    "n2v_walks_batched_noalloc": [ctypes.POINTER(RequestDesc), _U32, _VP],
    "n2v_batch_create": [ctypes.POINTER(RequestDesc), _U32, _U32, ctypes.POINTER(_U64)],
    "n2v_batch_launch": [_U64, _VP],
    "n2v_batch_info": [_U64, ctypes.POINTER(BatchInfo)],
    "n2v_batch_destroy": [_U64],
    "n2v_server_create": [_U64, _U32, ctypes.POINTER(Tuning), ctypes.POINTER(_U64)],
    "n2v_server_add_graph": [_U64, _U64],
    "n2v_request_submit": [_U64, ctypes.POINTER(RequestDesc), _U64, ctypes.POINTER(_U64)],
    "n2v_request_poll": [_U64, _U64, ctypes.POINTER(Result)],
    "n2v_request_release": [_U64, _U64],
    "n2v_server_destroy": [_U64],
    "n2v_last_error": [],
}

_lib = None
_borrowed: dict = {}  # graph handle -> the device tensors the library reads
_lock = threading.Lock()


def lib():
    """Load libn2vwalk.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing: build it with "
                                  "`python -m paper_2110_06196_amd.build` (HIP for gfx950)")
            L = ctypes.CDLL(LIB_PATH)
            for name, args in SIGNATURES.items():
                f = getattr(L, name)
                f.argtypes = args
                f.restype = ctypes.c_char_p if name == "n2v_last_error" else ctypes.c_int
            _lib = L
    return _lib


def _check(rc: int) -> int:
    if rc < 0:
        raise N2VError(rc, lib().n2v_last_error().decode(errors="replace"))
    return rc


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t, dtype, name):
    if t is None:
        return None
    if not t.is_cuda or t.dtype != dtype or not t.is_contiguous():
        raise N2VError(N2V_ERR_INVALID_ARG, f"{name} must be a contiguous CUDA {dtype} tensor")
    return t


# ---------------------------------------------------------------------------
# Graphs
# ---------------------------------------------------------------------------
def n2v_graph_upload(offsets, dst, weights=None, stream=None, flags: int = 0) -> int:
    """Register a CSR graph held in device tensors (uint64 / int64 offsets,
    int32 destinations, optional int32/uint32 weights viewed as uint32).
    The tensors are borrowed: keep them alive until n2v_graph_release.
    flags: 0 or any of N2V_UPLOAD_NO_PAIR_LISTS, N2V_UPLOAD_NO_HUB_SETS and
    N2V_UPLOAD_HUB_MIN_DEGREE_LOG2(k)."""
    if offsets.dtype == torch.int64:
        offsets = offsets.view(torch.uint64) if hasattr(torch, "uint64") else offsets
    _dev(dst, torch.int32, "dst")
    if weights is not None and weights.dtype not in (torch.int32, getattr(torch, "uint32", torch.int32)):
        raise N2VError(N2V_ERR_INVALID_ARG, "weights must be uint32 (or int32 bit pattern)")
    h = ctypes.c_uint64(0)
    _check(lib().n2v_graph_upload(_ptr(offsets), offsets.numel() - 1, _ptr(dst), dst.numel(),
                                  _ptr(weights), flags, _stream(stream), ctypes.byref(h)))
    # The library reads these arrays until release: hold them so that the
    # caching allocator cannot hand their memory to another tensor meanwhile.
    _borrowed[h.value] = (offsets, dst, weights)
    return h.value


def n2v_graph_info(g: int) -> dict:
    info = GraphInfo()
    _check(lib().n2v_graph_info(g, ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in GraphInfo._fields_}


def n2v_graph_upload_ef(offsets, dst, weights=None, quantum: int = 0, stream=None) -> int:
    """Build an Elias-Fano graph from CSR device tensors (same layout as
    n2v_graph_upload).  The tensors are not referenced after the call."""
    if offsets.dtype == torch.int64:
        offsets = offsets.view(torch.uint64) if hasattr(torch, "uint64") else offsets
    _dev(dst, torch.int32, "dst")
    if weights is not None and weights.dtype not in (torch.int32, getattr(torch, "uint32", torch.int32)):
        raise N2VError(N2V_ERR_INVALID_ARG, "weights must be uint32 (or int32 bit pattern)")
    h = ctypes.c_uint64(0)
    _check(lib().n2v_graph_upload_ef(_ptr(offsets), offsets.numel() - 1, _ptr(dst), dst.numel(), _ptr(weights),
                                     quantum, _stream(stream), ctypes.byref(h)))
    return h.value


def n2v_ef_info(g: int) -> dict:
    """Shape of an Elias-Fano graph and the device addresses of its arrays (d_H, d_L, d_S1, d_S0)."""
    info = EFInfo()
    _check(lib().n2v_ef_info(g, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in EFInfo._fields_ if f != "pad"}


def ef_arrays(g: int) -> dict:
    """Copies of the Elias-Fano arrays H, L, S1, S0 of graph g as device int64 tensors."""
    info = n2v_ef_info(g)
    out = {}
    for name, n in (("H", info["h_words"]), ("L", info["l_words"]), ("S1", info["s1_len"]), ("S0", info["s0_len"])):
        t = torch.empty(max(int(n), 1), dtype=torch.int64, device="cuda")
        if n:
            torch.cuda.synchronize()
            rc = _hip().hipMemcpy(t.data_ptr(), info["d_" + name], int(n) * 8, 3)  # device to device
            if rc != 0:
                raise N2VError(N2V_ERR_HIP, f"hipMemcpy failed ({rc})")
        out[name] = t[:int(n)]
    return out


def n2v_ef_select(g: int, idx, out=None, stream=None):
    _dev(idx, torch.int64, "idx")
    if out is None:
        out = torch.empty_like(idx)
    _check(lib().n2v_ef_select(g, _ptr(idx), idx.numel(), _ptr(out), _stream(stream)))
    return out


def n2v_ef_rank(g: int, x, out=None, stream=None):
    _dev(x, torch.int64, "x")
    if out is None:
        out = torch.empty_like(x)
    _check(lib().n2v_ef_rank(g, _ptr(x), x.numel(), _ptr(out), _stream(stream)))
    return out


def n2v_graph_release(g: int) -> None:
    _check(lib().n2v_graph_release(g))
    _borrowed.pop(g, None)


def n2v_set_tuning(lanes_per_walker=0, lds_tile=0, list_cap=0, route=0, flags=0, reset=False) -> None:
    """Process-wide launch tuning (zero = automatic); reset=True restores automatic."""
    if reset:
        _check(lib().n2v_set_tuning(None))
        return
    t = Tuning(lanes_per_walker, lds_tile, list_cap, route, flags)
    _check(lib().n2v_set_tuning(ctypes.byref(t)))


# ---------------------------------------------------------------------------
# Plain walks
# ---------------------------------------------------------------------------
def _alloc_out(starts, walks_per_start, walk_len, walks, lens):
    nw = starts.numel() * walks_per_start
    if walks is None:
        walks = torch.empty((nw, walk_len), dtype=torch.int32, device=starts.device)
    if lens is None:
        lens = torch.empty(nw, dtype=torch.int32, device=starts.device)
    _dev(walks, torch.int32, "walks")
    _dev(lens, torch.int32, "lens")
    if walks.numel() != nw * walk_len or lens.numel() != nw:
        raise N2VError(N2V_ERR_INVALID_ARG, "walks / lens have the wrong size")
    return walks, lens


def n2v_walks_first_order(g: int, starts, walks_per_start: int, walk_len: int, seed: int,
                          walk_id_base: int = 0, walks=None, lens=None, stream=None):
    """Enqueue first-order walks; returns (walks int32[n][walk_len], lens int32[n])."""
    _dev(starts, torch.int32, "starts")
    walks, lens = _alloc_out(starts, walks_per_start, walk_len, walks, lens)
    _check(lib().n2v_walks_first_order(g, _ptr(starts), starts.numel(), walks_per_start, walk_len,
                                       seed, walk_id_base, _ptr(walks), _ptr(lens), _stream(stream)))
    return walks, lens


def n2v_walks_node2vec(g: int, starts, walks_per_start: int, walk_len: int, p: float, q: float,
                       seed: int, walk_id_base: int = 0, walks=None, lens=None, stream=None):
    """Enqueue node2vec walks; returns (walks int32[n][walk_len], lens int32[n])."""
    _dev(starts, torch.int32, "starts")
    walks, lens = _alloc_out(starts, walks_per_start, walk_len, walks, lens)
    _check(lib().n2v_walks_node2vec(g, _ptr(starts), starts.numel(), walks_per_start, walk_len,
                                    float(p), float(q), seed, walk_id_base, _ptr(walks), _ptr(lens),
                                    _stream(stream)))
    return walks, lens


def n2v_walks_approximated(g: int, kind: int, starts, walks_per_start: int, walk_len: int, p: float, q: float,
                           k: int, seed: int, walk_id_base: int = 0, walks=None, lens=None, stream=None):
    """Enqueue approximated walks (k sub-sampled neighbours per step from rows longer than k)."""
    _dev(starts, torch.int32, "starts")
    walks, lens = _alloc_out(starts, walks_per_start, walk_len, walks, lens)
    _check(lib().n2v_walks_approximated(g, kind, _ptr(starts), starts.numel(), walks_per_start, walk_len,
                                        float(p), float(q), k, seed, walk_id_base, _ptr(walks), _ptr(lens),
                                        _stream(stream)))
    return walks, lens


def n2v_walk_contexts(walks, window: int, stride: int = 1, contexts=None, stream=None):
    """Context slots int32[n_walks][walk_len][2 window] of every walk position."""
    _dev(walks, torch.int32, "walks")
    nw, L = walks.shape
    if contexts is None:
        contexts = torch.empty((nw, L, 2 * window), dtype=torch.int32, device=walks.device)
    _dev(contexts, torch.int32, "contexts")
    _check(lib().n2v_walk_contexts(_ptr(walks), nw, L, window, stride, _ptr(contexts), _stream(stream)))
    return contexts


def n2v_walks_contexts(g: int, kind: int, starts, walks_per_start: int, walk_len: int, p: float, q: float,
                       seed: int, walk_id_base: int, window: int, stride: int = 1, contexts=None, lens=None,
                       stream=None):
    """Fused walk -> contexts: the context slots [n_walks][walk_len][2 window]
    of the walks, without the walk array; returns (contexts, lens)."""
    _dev(starts, torch.int32, "starts")
    nw = starts.numel() * walks_per_start
    if contexts is None:
        contexts = torch.empty((nw, walk_len, 2 * window), dtype=torch.int32, device=starts.device)
    if lens is None:
        lens = torch.empty(nw, dtype=torch.int32, device=starts.device)
    _dev(contexts, torch.int32, "contexts")
    _dev(lens, torch.int32, "lens")
    if contexts.numel() != nw * walk_len * 2 * window or lens.numel() != nw:
        raise N2VError(N2V_ERR_INVALID_ARG, "contexts / lens have the wrong size")
    _check(lib().n2v_walks_contexts(g, kind, _ptr(starts), starts.numel(), walks_per_start, walk_len, float(p),
                                    float(q), seed, walk_id_base, window, stride, _ptr(contexts), _ptr(lens),
                                    _stream(stream)))
    return contexts, lens


def n2v_negative_samples(g: int, walks, n_neg: int, seed: int, walk_id_base: int = 0, negatives=None, stream=None):
    """Degree-proportional negatives int32[n_walks][walk_len][n_neg] for every walk position."""
    _dev(walks, torch.int32, "walks")
    nw, L = walks.shape
    if negatives is None:
        negatives = torch.empty((nw, L, n_neg), dtype=torch.int32, device=walks.device)
    _dev(negatives, torch.int32, "negatives")
    _check(lib().n2v_negative_samples(g, _ptr(walks), nw, L, n_neg, seed, walk_id_base, _ptr(negatives),
                                      _stream(stream)))
    return negatives


def make_request(graph: int, kind: int, starts, walks_per_start: int, walk_len: int, p=1.0, q=1.0,
                 seed=0, walk_id_base=0, walks=None, lens=None, k_approx: int = 0) -> RequestDesc:
    return RequestDesc(graph, kind, walks_per_start, walk_len, k_approx, float(p), float(q), seed,
                       walk_id_base, starts.data_ptr() if starts is not None else None,
                       starts.numel() if starts is not None else 0,
                       walks.data_ptr() if walks is not None else None,
                       lens.data_ptr() if lens is not None else None)


def n2v_walks_batched(reqs, stream=None) -> None:
    """reqs: list of RequestDesc (device pointers inside); one launch."""
    arr = (RequestDesc * len(reqs))(*reqs)
    _check(lib().n2v_walks_batched(arr, len(reqs), _stream(stream)))


def n2v_walks_batched_noalloc(reqs, stream=None) -> None:
    """As n2v_walks_batched, with the tables in the library's fixed device
    array (no device allocation; at most 4096 requests)."""
    arr = (RequestDesc * len(reqs))(*reqs)
    _check(lib().n2v_walks_batched_noalloc(arr, len(reqs), _stream(stream)))


def n2v_batch_create(reqs, autotune: bool = True) -> int:
    """Upload the request/chunk tables, pick the launch shape, capture a hipGraph."""
    arr = (RequestDesc * len(reqs))(*reqs)
    h = ctypes.c_uint64(0)
    _check(lib().n2v_batch_create(arr, len(reqs), N2V_BATCH_AUTOTUNE if autotune else 0, ctypes.byref(h)))
    return h.value


def n2v_batch_launch(b: int, stream=None) -> None:
    _check(lib().n2v_batch_launch(b, _stream(stream)))


def n2v_batch_info(b: int) -> dict:
    info = BatchInfo()
    _check(lib().n2v_batch_info(b, ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in BatchInfo._fields_}


def n2v_batch_destroy(b: int) -> None:
    _check(lib().n2v_batch_destroy(b))


# ---------------------------------------------------------------------------
# Serving
# ---------------------------------------------------------------------------
def n2v_server_create(hbm_budget_bytes: int, max_slots: int, tuning: dict | None = None) -> int:
    """tuning: None (automatic launch shape) or a dict of n2v_tuning_t fields
    (lanes_per_walker, lds_tile, list_cap, route, flags) fixing the shape."""
    h = ctypes.c_uint64(0)
    t = None
    if tuning is not None:
        t = ctypes.byref(Tuning(*(int(tuning.get(k, 0)) for k, _ in Tuning._fields_)))
    _check(lib().n2v_server_create(hbm_budget_bytes, max_slots, t, ctypes.byref(h)))
    return h.value


def n2v_server_add_graph(s: int, g: int) -> None:
    _check(lib().n2v_server_add_graph(s, g))


def host_request(graph: int, kind: int, starts_np, walks_per_start: int, walk_len: int, p=1.0, q=1.0,
                 seed=0, walk_id_base=0, k_approx: int = 0):
    """A RequestDesc whose starts point at host memory (for n2v_request_submit).
    Returns (desc, keepalive): keep the second item alive until submit returns."""
    import numpy as np
    arr = np.ascontiguousarray(starts_np, dtype=np.int32)
    d = RequestDesc(graph, kind, walks_per_start, walk_len, k_approx, float(p), float(q), seed, walk_id_base,
                    arr.ctypes.data if arr.size else None, arr.size, None, None)
    return d, arr


def n2v_request_submit(s: int, desc: RequestDesc, arrival_ns: int) -> int:
    h = ctypes.c_uint64(0)
    _check(lib().n2v_request_submit(s, ctypes.byref(desc), arrival_ns, ctypes.byref(h)))
    return h.value


def n2v_request_poll(s: int, r: int):
    """Returns None while pending, else a Result."""
    res = Result()
    rc = _check(lib().n2v_request_poll(s, r, ctypes.byref(res)))
    return None if rc == N2V_PENDING else res


_hip_rt = None


def _hip():
    """The HIP runtime already loaded by torch (same soname, same instance)."""
    global _hip_rt
    if _hip_rt is None:
        rt = ctypes.CDLL("libamdhip64.so.7")
        rt.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        rt.hipMemcpy.restype = ctypes.c_int
        _hip_rt = rt
    return _hip_rt


def result_tensors(res: Result, walk_len: int):
    """Copy a finished request's server-owned walks / lens into new torch tensors."""
    nw = int(res.n_walks)
    Y = torch.empty((nw, walk_len), dtype=torch.int32, device="cuda")
    lens = torch.empty(nw, dtype=torch.int32, device="cuda")
    if nw:
        torch.cuda.synchronize()
        for dst, src, nbytes in ((Y.data_ptr(), res.d_walks, nw * walk_len * 4), (lens.data_ptr(), res.d_lens, nw * 4)):
            rc = _hip().hipMemcpy(dst, src, nbytes, 3)  # device to device
            if rc != 0:
                raise N2VError(N2V_ERR_HIP, f"hipMemcpy failed ({rc})")
    return Y, lens


def n2v_request_release(s: int, r: int) -> None:
    _check(lib().n2v_request_release(s, r))


def n2v_server_destroy(s: int) -> None:
    _check(lib().n2v_server_destroy(s))
