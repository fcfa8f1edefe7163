"""Plain CPU oracle for exact DeepWalk / node2vec walk generation.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The GPU library
(``paper_2110_06196_amd``) never imports it and shares no code with it.

The arithmetic lives in ``n2v_oracle.c`` (single-threaded, plain loops); this
module only compiles it with gcc and marshals numpy arrays through ctypes.
Each C function cites the passage of the paper it follows (Methods, "First and
second-order RW-based embedding methods", Eq. 1-3 and the four sampling steps
of "Efficient sampling for Node2Vec RWs").
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "n2v_oracle.c")
_LIB = os.path.join(_HERE, "libn2v_oracle.so")

OK, ERR_INVALID_ARG, ERR_UNSORTED, ERR_OVERFLOW = 0, -1, -2, -3
FIRST_ORDER, NODE2VEC = 0, 1

_lock = threading.Lock()
_lib = None


def build() -> str:
    """Compile the oracle with gcc (plain -O2, no vectorisation tricks needed)."""
    tmp = _LIB + f".tmp{os.getpid()}"
    subprocess.check_call(
        ["gcc", "-O2", "-std=gnu11", "-Wall", "-Wextra", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"]
    )
    os.replace(tmp, _LIB)
    return _LIB


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t)) if a is not None else None


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build()
            L = ctypes.CDLL(_LIB)
            u64p = ctypes.POINTER(ctypes.c_uint64)
            u32p = ctypes.POINTER(ctypes.c_uint32)
            i32p = ctypes.POINTER(ctypes.c_int32)
            i64p = ctypes.POINTER(ctypes.c_int64)
            L.n2vo_q16.argtypes = [ctypes.c_double, u32p]
            L.n2vo_q16.restype = ctypes.c_int
            L.n2vo_philox4x32_10.argtypes = [u32p, u32p, u32p]
            L.n2vo_philox4x32_10.restype = None
            L.n2vo_draw64.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64]
            L.n2vo_draw64.restype = ctypes.c_uint64
            L.n2vo_scale.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
            L.n2vo_scale.restype = ctypes.c_uint64
            L.n2vo_validate.argtypes = [u64p, ctypes.c_int64, i32p, ctypes.c_uint64]
            L.n2vo_validate.restype = ctypes.c_int
            L.n2vo_stats.argtypes = [u64p, ctypes.c_int64, u32p, u64p, u64p]
            L.n2vo_stats.restype = None
            L.n2vo_step_weights.argtypes = [u64p, i32p, u32p, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int, ctypes.c_uint32, ctypes.c_uint32, u64p]
            L.n2vo_step_weights.restype = ctypes.c_int64
            L.n2vo_select.argtypes = [u64p, ctypes.c_int64, ctypes.c_uint64]
            L.n2vo_select.restype = ctypes.c_int64
            common = [u64p, ctypes.c_int64, i32p, ctypes.c_uint64, u32p, i32p, ctypes.c_int64,
                      ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, ctypes.c_double,
                      ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64]
            L.n2vo_walks_subset.argtypes = common + [i64p, ctypes.c_int64, i32p, i32p]
            L.n2vo_walks_subset.restype = ctypes.c_int
            L.n2vo_walks.argtypes = common + [i32p, i32p]
            L.n2vo_walks.restype = ctypes.c_int
            L.n2vo_suss.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint32,
                                    ctypes.c_uint32, u32p]
            L.n2vo_suss.restype = None
            L.n2vo_walks_approx_subset.argtypes = (common[:12] + [ctypes.c_uint32] + common[12:] +
                                                   [i64p, ctypes.c_int64, i32p, i32p])
            L.n2vo_walks_approx_subset.restype = ctypes.c_int
            L.n2vo_contexts.argtypes = [i32p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                        i32p]
            L.n2vo_contexts.restype = None
            L.n2vo_negatives.argtypes = [u64p, ctypes.c_int64, i32p, ctypes.c_int64, ctypes.c_uint32,
                                         ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, i32p]
            L.n2vo_negatives.restype = None
            shp = ctypes.POINTER(EFShape)
            L.n2vo_ef_shape_of.argtypes = [ctypes.c_uint64, ctypes.c_uint64, shp]
            L.n2vo_ef_shape_of.restype = None
            L.n2vo_ef_graph_shape.argtypes = [ctypes.c_int64, ctypes.c_uint64, shp]
            L.n2vo_ef_graph_shape.restype = ctypes.c_int
            L.n2vo_ef_words.argtypes = [shp, ctypes.c_uint32, u64p, u64p, u64p, u64p]
            L.n2vo_ef_words.restype = None
            L.n2vo_ef_encode.argtypes = [u64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32, u64p, u64p, u64p,
                                         u64p]
            L.n2vo_ef_encode.restype = ctypes.c_int
            L.n2vo_ef_encode_graph.argtypes = [u64p, ctypes.c_int64, i32p, ctypes.c_uint64, ctypes.c_uint32, u64p,
                                               u64p, u64p, u64p]
            L.n2vo_ef_encode_graph.restype = ctypes.c_int
            L.n2vo_ef_select.argtypes = [shp, u64p, u64p, ctypes.c_uint64]
            L.n2vo_ef_select.restype = ctypes.c_uint64
            L.n2vo_ef_rank.argtypes = [shp, u64p, u64p, ctypes.c_uint64]
            L.n2vo_ef_rank.restype = ctypes.c_uint64
            _lib = L
    return _lib


class EFShape(ctypes.Structure):
    """n2vo_ef_shape: k, l, u, m, n_zeros, h_bits."""
    _fields_ = [("k", ctypes.c_uint32), ("l", ctypes.c_uint32), ("u", ctypes.c_uint64), ("m", ctypes.c_uint64),
                ("n_zeros", ctypes.c_uint64), ("h_bits", ctypes.c_uint64)]


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle status {code}")
        self.code = code


def _csr(offsets, dst, weights):
    O = np.ascontiguousarray(offsets, dtype=np.uint64)
    D = np.ascontiguousarray(dst, dtype=np.int32)
    W = None if weights is None else np.ascontiguousarray(weights, dtype=np.uint32)
    return O, D, W


def q16(x: float) -> int:
    out = ctypes.c_uint32(0)
    rc = lib().n2vo_q16(float(x), ctypes.byref(out))
    if rc != OK:
        raise OracleError(rc)
    return int(out.value)


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().n2vo_philox4x32_10(_p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32), _p(o, ctypes.c_uint32))
    return o


def draw64(seed: int, step: int, wid: int) -> int:
    return int(lib().n2vo_draw64(seed, step, wid))


def scale(r64: int, total: int) -> int:
    return int(lib().n2vo_scale(r64, total))


def validate(offsets, dst) -> int:
    O, D, _ = _csr(offsets, dst, None)
    n = O.size - 1
    return int(lib().n2vo_validate(_p(O, ctypes.c_uint64), n, _p(D, ctypes.c_int32), D.size))


def stats(offsets, weights=None):
    O = np.ascontiguousarray(offsets, dtype=np.uint64)
    W = None if weights is None else np.ascontiguousarray(weights, dtype=np.uint32)
    md, ms = ctypes.c_uint64(0), ctypes.c_uint64(0)
    lib().n2vo_stats(_p(O, ctypes.c_uint64), O.size - 1, _p(W, ctypes.c_uint32),
                     ctypes.byref(md), ctypes.byref(ms))
    return int(md.value), int(ms.value)


def step_weights(offsets, dst, weights, t: int, v: int, second_order: bool, P16: int, Q16: int):
    O, D, W = _csr(offsets, dst, weights)
    d = int(O[v + 1] - O[v])
    b = np.zeros(max(d, 1), dtype=np.uint64)
    got = lib().n2vo_step_weights(_p(O, ctypes.c_uint64), _p(D, ctypes.c_int32), _p(W, ctypes.c_uint32),
                                  t, v, int(second_order), P16, Q16, _p(b, ctypes.c_uint64))
    assert got == d
    return b[:d]


def select(b, T: int) -> int:
    bb = np.ascontiguousarray(b, dtype=np.uint64)
    return int(lib().n2vo_select(_p(bb, ctypes.c_uint64), bb.size, T))


def suss(seed: int, step: int, wid: int, d: int, k: int):
    """Sorted Unique Sub-Sampling: k positions in [0, d) (d > k)."""
    out = np.zeros(k, dtype=np.uint32)
    lib().n2vo_suss(seed, step, wid, d, k, _p(out, ctypes.c_uint32))
    return out


def walks(offsets, dst, weights, starts, walks_per_start: int, walk_len: int, kind: int,
          p: float = 1.0, q: float = 1.0, seed: int = 0, walk_id_base: int = 0, rows=None, k_approx: int = 0):
    """Run the oracle.  rows: None for all walks, else the walk-row indices to produce.
    k_approx > 0: approximated walks (SUSS sub-sample of k_approx neighbours per step).

    Returns (Y int32[nrows][walk_len], lens int32[nrows])."""
    O, D, W = _csr(offsets, dst, weights)
    S = np.ascontiguousarray(starts, dtype=np.int32)
    n = O.size - 1
    args = (_p(O, ctypes.c_uint64), n, _p(D, ctypes.c_int32), D.size, _p(W, ctypes.c_uint32),
            _p(S, ctypes.c_int32), S.size, walks_per_start, walk_len, kind, float(p), float(q),
            seed, walk_id_base)
    if k_approx:
        if rows is None:
            rows = np.arange(S.size * walks_per_start, dtype=np.int64)
        idx = np.ascontiguousarray(rows, dtype=np.int64)
        Y = np.empty((idx.size, walk_len), dtype=np.int32)
        lens = np.empty(idx.size, dtype=np.int32)
        rc = lib().n2vo_walks_approx_subset(*args[:12], k_approx, *args[12:], _p(idx, ctypes.c_int64), idx.size,
                                            _p(Y, ctypes.c_int32), _p(lens, ctypes.c_int32))
    elif rows is None:
        nw = S.size * walks_per_start
        Y = np.empty((nw, walk_len), dtype=np.int32)
        lens = np.empty(nw, dtype=np.int32)
        rc = lib().n2vo_walks(*args, _p(Y, ctypes.c_int32), _p(lens, ctypes.c_int32))
    else:
        idx = np.ascontiguousarray(rows, dtype=np.int64)
        Y = np.empty((idx.size, walk_len), dtype=np.int32)
        lens = np.empty(idx.size, dtype=np.int32)
        rc = lib().n2vo_walks_subset(*args, _p(idx, ctypes.c_int64), idx.size,
                                     _p(Y, ctypes.c_int32), _p(lens, ctypes.c_int32))
    if rc != OK:
        raise OracleError(rc)
    return Y, lens


def walks_threaded(offsets, dst, weights, starts, walks_per_start, walk_len, kind, p=1.0, q=1.0,
                   seed=0, walk_id_base=0, rows=None, threads=1, k_approx=0):
    """Same as walks(), with disjoint slices of `rows` handed to `threads` OS threads.

    ctypes releases the GIL during each call, so the slices run concurrently;
    the arithmetic is still the single-threaded C routine per slice."""
    if rows is None:
        rows = np.arange(len(starts) * walks_per_start, dtype=np.int64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    threads = max(1, min(int(threads), rows.size or 1))
    parts = np.array_split(rows, threads)
    out = [None] * threads

    def run(i):
        out[i] = walks(offsets, dst, weights, starts, walks_per_start, walk_len, kind, p, q, seed,
                       walk_id_base, parts[i], k_approx)

    ts = [threading.Thread(target=run, args=(i,)) for i in range(threads)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    Y = np.concatenate([o[0] for o in out]) if out else np.empty((0, walk_len), np.int32)
    lens = np.concatenate([o[1] for o in out]) if out else np.empty(0, np.int32)
    return Y, lens


def contexts(Y, window: int, stride: int = 1):
    """Context slots [nw][L][2 window] of every walk position (see n2v_oracle.h)."""
    Yc = np.ascontiguousarray(Y, dtype=np.int32)
    nw, L = Yc.shape
    C = np.empty((nw, L, 2 * window), dtype=np.int32)
    lib().n2vo_contexts(_p(Yc, ctypes.c_int32), nw, L, window, stride, _p(C, ctypes.c_int32))
    return C


def negatives(offsets, Y, n_neg: int, seed: int, walk_id_base: int = 0):
    """Scale-free negatives [nw][L][n_neg] (see n2v_oracle.h)."""
    O = np.ascontiguousarray(offsets, dtype=np.uint64)
    Yc = np.ascontiguousarray(Y, dtype=np.int32)
    nw, L = Yc.shape
    N = np.empty((nw, L, n_neg), dtype=np.int32)
    lib().n2vo_negatives(_p(O, ctypes.c_uint64), O.size - 1, _p(Yc, ctypes.c_int32), nw, L, n_neg, seed,
                         walk_id_base, _p(N, ctypes.c_int32))
    return N


def _ef_arrays(shape, q):
    u64 = ctypes.c_uint64
    hw, lw, n1, n0 = u64(), u64(), u64(), u64()
    lib().n2vo_ef_words(ctypes.byref(shape), q, ctypes.byref(hw), ctypes.byref(lw), ctypes.byref(n1),
                        ctypes.byref(n0))
    mk = lambda k: np.zeros(max(1, k.value), dtype=np.uint64)
    return mk(hw), mk(lw), mk(n1), mk(n0)


def ef_encode(values, u: int, q: int = 1024) -> dict:
    """Elias-Fano list of non-decreasing values below u (see n2v_oracle.h):
    dict with the shape fields and the arrays H, L, S1, S0 (uint64)."""
    y = np.ascontiguousarray(values, dtype=np.uint64)
    shape = EFShape()
    lib().n2vo_ef_shape_of(y.size, u, ctypes.byref(shape))
    H, L, S1, S0 = _ef_arrays(shape, q)
    rc = lib().n2vo_ef_encode(_p(y, ctypes.c_uint64), y.size, u, q, _p(H, ctypes.c_uint64),
                              _p(L, ctypes.c_uint64), _p(S1, ctypes.c_uint64), _p(S0, ctypes.c_uint64))
    if rc != OK:
        raise OracleError(rc)
    return _ef_dict(shape, q, H, L, S1, S0)


def ef_encode_graph(offsets, dst, q: int = 1024) -> dict:
    """Elias-Fano list of the edge codes phi_k(a, b) = a 2^k + b of a sorted CSR graph."""
    O = np.ascontiguousarray(offsets, dtype=np.uint64)
    D = np.ascontiguousarray(dst, dtype=np.int32)
    n = O.size - 1
    shape = EFShape()
    if lib().n2vo_ef_graph_shape(n, D.size, ctypes.byref(shape)) != OK:
        raise OracleError(ERR_INVALID_ARG)
    H, L, S1, S0 = _ef_arrays(shape, q)
    rc = lib().n2vo_ef_encode_graph(_p(O, ctypes.c_uint64), n, _p(D, ctypes.c_int32), D.size, q,
                                    _p(H, ctypes.c_uint64), _p(L, ctypes.c_uint64), _p(S1, ctypes.c_uint64),
                                    _p(S0, ctypes.c_uint64))
    if rc != OK:
        raise OracleError(rc)
    return _ef_dict(shape, q, H, L, S1, S0)


def _ef_dict(shape, q, H, L, S1, S0):
    return {"k": shape.k, "l": shape.l, "u": shape.u, "m": shape.m, "n_zeros": shape.n_zeros,
            "h_bits": shape.h_bits, "q": q, "H": H, "L": L, "S1": S1, "S0": S0, "_shape": shape}


def ef_select(ef: dict, i: int) -> int:
    """The i-th smallest element (plain scan of H)."""
    return int(lib().n2vo_ef_select(ctypes.byref(ef["_shape"]), _p(ef["H"], ctypes.c_uint64),
                                    _p(ef["L"], ctypes.c_uint64), i))


def ef_rank(ef: dict, x: int) -> int:
    """The number of elements strictly below x (plain scan of H)."""
    return int(lib().n2vo_ef_rank(ctypes.byref(ef["_shape"]), _p(ef["H"], ctypes.c_uint64),
                                  _p(ef["L"], ctypes.c_uint64), x))
