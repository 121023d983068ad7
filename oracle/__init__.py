"""Plain CPU oracle of the SLASH hot path.

TEST INFRASTRUCTURE: only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package.  The product library
never loads it.  The C source ``oracle/slash_oracle.c`` is the definition;
this module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, asdict

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None
EMPTY = 0xFFFFFFFF


def build_lib() -> str:
    """Compile the oracle (plain C, -O2) in-tree; always recompiles."""
    src = os.path.join(_HERE, "slash_oracle.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-o", tmp, src, "-lm"])
    os.replace(tmp, _SO)
    return _SO


class _P(C.Structure):
    _fields_ = [(n, C.c_uint32) for n in ("dim", "K", "L", "log2_buckets", "R", "cm_rows",
                                          "log2_cm_width", "hash_mode")] + [("seed", C.c_uint64)]


@dataclass
class Params:
    dim: int = 1 << 20
    K: int = 4
    L: int = 16
    log2_buckets: int = 16
    R: int = 32
    cm_rows: int = 4
    log2_cm_width: int = 10
    hash_mode: int = 0
    seed: int = 0

    def c(self) -> _P:
        d = asdict(self)
        return _P(**{k: (v & (2**64 - 1) if k == "seed" else v) for k, v in d.items()})

    @property
    def M(self) -> int:
        return self.K * self.L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            raise RuntimeError("oracle/liboracle.so is not built; run __graft_entry__.build()")
        L = C.CDLL(_SO)
        vp, P = C.c_void_p, C.POINTER(_P)
        L.oracle_constants_size.restype = C.c_uint64
        L.oracle_constants_size.argtypes = [P]
        L.oracle_constants.argtypes = [P, vp]
        L.oracle_splitmix64.restype = C.c_uint64
        L.oracle_splitmix64.argtypes = [vp]
        L.oracle_hash_rows.argtypes = [P, vp, vp, vp, C.c_uint64, C.c_uint64, vp, vp]
        L.oracle_priority.restype = C.c_uint32
        L.oracle_priority.argtypes = [P, vp, C.c_uint32, C.c_uint32]
        L.oracle_priorities.argtypes = [P, vp, C.c_uint32, vp, C.c_uint64, vp]
        L.oracle_build.argtypes = [P, vp, vp, vp, C.c_uint64, vp, vp]
        L.oracle_insert.argtypes = [P, vp, vp, vp, C.c_uint32, vp, vp, C.c_uint64]
        L.oracle_query.argtypes = [P, vp, vp, vp, vp, vp, C.c_uint64, vp, C.c_uint32, C.c_uint32,
                                   vp, vp, C.c_int]
        L.oracle_aggregate.argtypes = [P, vp, vp, C.c_uint64, C.c_uint32, C.c_uint32, vp, vp, C.c_int]
        L.oracle_tk_sketch.argtypes = [P, vp, vp, C.c_uint64, vp]
        L.oracle_tk_merge.argtypes = [P, vp, vp]
        L.oracle_tk_build.argtypes = [P, vp, vp, vp, C.c_uint64, vp, vp]
        L.oracle_tk_insert.argtypes = [P, vp, vp, vp, C.c_uint32, vp, vp, C.c_uint64]
        L.oracle_tk_report.argtypes = [P, vp, C.c_uint32, C.c_uint32, vp, vp]
        L.oracle_jaccard_knn.argtypes = [vp, vp, C.c_uint64, vp, vp, C.c_uint64, C.c_uint32, vp, vp, vp]
        L.oracle_mean_cosine.argtypes = [vp, vp, C.c_uint64, vp, vp, C.c_uint64, vp, C.c_uint32, C.c_uint32, vp, vp]
        L.oracle_tk_query.argtypes = [P, vp, vp, vp, vp, C.c_uint64, vp, C.c_uint32, C.c_uint32, vp, vp]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _csr(indptr, indices):
    return (np.ascontiguousarray(indptr, dtype=np.int64),
            np.ascontiguousarray(indices, dtype=np.int32))


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what} failed with status {code}")
        self.code = code


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError(rc, what)


def layout(p: Params) -> dict:
    """Offsets of each constant group in the flat table (same order as the C code)."""
    n_h = p.M if p.hash_mode == 2 else (p.L if p.hash_mode else 1)
    o = {"a_h": 0}
    o["b_h"] = n_h
    o["dir"] = 2 * n_h
    o["a_tj"] = o["dir"] + p.M
    o["b_t"] = o["a_tj"] + p.M
    o["key_t"] = o["b_t"] + p.L
    o["m1_t"] = o["key_t"] + p.L
    o["m2_t"] = o["m1_t"] + p.L
    o["a_r"] = o["m2_t"] + p.L
    o["b_r"] = o["a_r"] + p.cm_rows
    o["total"] = o["b_r"] + p.cm_rows
    return o


def constants(p: Params) -> np.ndarray:
    pc = p.c()
    n = lib().oracle_constants_size(C.byref(pc))
    out = np.zeros(n, dtype=np.uint64)
    _check(lib().oracle_constants(C.byref(pc), _p(out)), "oracle_constants")
    return out


def splitmix64_stream(seed: int, n: int) -> np.ndarray:
    s = np.array([seed & (2**64 - 1)], dtype=np.uint64)
    return np.array([lib().oracle_splitmix64(_p(s)) for _ in range(n)], dtype=np.uint64)


def hash_rows(p: Params, cs, indptr, indices, row_begin=0, row_end=None, with_h=False):
    indptr, indices = _csr(indptr, indices)
    n = len(indptr) - 1
    row_end = n if row_end is None else row_end
    m = row_end - row_begin
    bk = np.zeros((m, p.L), dtype=np.uint32)
    hv = np.zeros((m, p.M), dtype=np.uint32) if with_h else None
    _check(lib().oracle_hash_rows(C.byref(p.c()), _p(cs), _p(indptr), _p(indices), row_begin,
                                  row_end, _p(bk), _p(hv) if with_h else None), "oracle_hash_rows")
    return (bk, hv) if with_h else bk


def priorities(p: Params, cs, t: int, ids) -> np.ndarray:
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    out = np.zeros(len(ids), dtype=np.uint32)
    lib().oracle_priorities(C.byref(p.c()), _p(cs), t, _p(ids), len(ids), _p(out))
    return out


def build(p: Params, cs, indptr, indices):
    """Tables after pre-processing: ids [L, 2^B, R] and seen [L, 2^B]."""
    indptr, indices = _csr(indptr, indices)
    nb = 1 << p.log2_buckets
    ids = np.zeros((p.L, nb, p.R), dtype=np.uint32)
    seen = np.zeros((p.L, nb), dtype=np.uint32)
    _check(lib().oracle_build(C.byref(p.c()), _p(cs), _p(indptr), _p(indices), len(indptr) - 1,
                              _p(ids), _p(seen)), "oracle_build")
    return ids, seen


def insert(p: Params, cs, ids, seen, first_id: int, indptr, indices):
    """In-place streaming insert of new rows with ids first_id, first_id+1, ..."""
    indptr, indices = _csr(indptr, indices)
    assert ids.flags.c_contiguous and seen.flags.c_contiguous
    _check(lib().oracle_insert(C.byref(p.c()), _p(cs), _p(ids), _p(seen), first_id, _p(indptr),
                               _p(indices), len(indptr) - 1), "oracle_insert")


def query(p: Params, cs, ids, seen, qindptr, qindices, k: int, k_max: int | None = None,
          kq=None, exact: bool = False):
    """Top-k (ids, scores) per query, rows of stride k_max, padded (EMPTY, 0)."""
    qindptr, qindices = _csr(qindptr, qindices)
    k_max = k if k_max is None else k_max
    nq = len(qindptr) - 1
    oi = np.zeros((nq, k_max), dtype=np.uint32)
    osc = np.zeros((nq, k_max), dtype=np.uint32)
    kqa = None if kq is None else np.ascontiguousarray(kq, dtype=np.uint32)
    _check(lib().oracle_query(C.byref(p.c()), _p(cs), _p(ids), _p(seen), _p(qindptr),
                              _p(qindices), nq, _p(kqa) if kqa is not None else None, k, k_max,
                              _p(oi), _p(osc), 1 if exact else 0), "oracle_query")
    return oi, osc


def aggregate(p: Params, cs, cand, k: int, k_max: int | None = None, exact: bool = False):
    """Top-k (ids, scores) of one candidate multiset (row of stride k_max)."""
    k_max = k if k_max is None else k_max
    c = np.ascontiguousarray(cand, dtype=np.uint32)
    oi = np.zeros(k_max, dtype=np.uint32)
    osc = np.zeros(k_max, dtype=np.uint32)
    _check(lib().oracle_aggregate(C.byref(p.c()), _p(cs), _p(c) if len(c) else None, len(c), k, k_max, _p(oi),
                                  _p(osc), 1 if exact else 0), "oracle_aggregate")
    return oi, osc


# ------------------------------------------------------------ Topkapi buckets
# A sketch is an array [W, C, 2] of uint32 (heavy hitter, count) with
# W = cm_rows and C = 2^log2_cm_width; empty cells are (EMPTY, 0).


def tk_shape(p: Params) -> tuple:
    return (p.cm_rows, 1 << p.log2_cm_width, 2)


def tk_sketch(p: Params, cs, ids) -> np.ndarray:
    """Sketch of the stream ids, inserted in the given order."""
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    sk = np.zeros(tk_shape(p), dtype=np.uint32)
    _check(lib().oracle_tk_sketch(C.byref(p.c()), _p(cs), _p(ids) if len(ids) else None, len(ids), _p(sk)),
           "oracle_tk_sketch")
    return sk


def tk_merge(p: Params, a, b) -> np.ndarray:
    """Merge(a, b) of two sketches (a new array)."""
    out = np.ascontiguousarray(a, dtype=np.uint32).copy()
    b = np.ascontiguousarray(b, dtype=np.uint32)
    _check(lib().oracle_tk_merge(C.byref(p.c()), _p(out), _p(b)), "oracle_tk_merge")
    return out


def tk_build(p: Params, cs, indptr, indices):
    """Topkapi tables after pre-processing: cells [L, 2^B, W, C, 2], seen [L, 2^B]."""
    indptr, indices = _csr(indptr, indices)
    nb = 1 << p.log2_buckets
    cells = np.zeros((p.L, nb) + tk_shape(p), dtype=np.uint32)
    seen = np.zeros((p.L, nb), dtype=np.uint32)
    _check(lib().oracle_tk_build(C.byref(p.c()), _p(cs), _p(indptr), _p(indices), len(indptr) - 1,
                                 _p(cells), _p(seen)), "oracle_tk_build")
    return cells, seen


def tk_insert(p: Params, cs, cells, seen, first_id: int, indptr, indices):
    """In-place streaming insert into Topkapi tables."""
    indptr, indices = _csr(indptr, indices)
    assert cells.flags.c_contiguous and seen.flags.c_contiguous
    _check(lib().oracle_tk_insert(C.byref(p.c()), _p(cs), _p(cells), _p(seen), first_id, _p(indptr),
                                  _p(indices), len(indptr) - 1), "oracle_tk_insert")


def tk_report(p: Params, sk, k: int, k_max: int | None = None):
    """Top-k (ids, counts) of one sketch, padded (EMPTY, 0)."""
    k_max = k if k_max is None else k_max
    sk = np.ascontiguousarray(sk, dtype=np.uint32)
    oi = np.zeros(k_max, dtype=np.uint32)
    osc = np.zeros(k_max, dtype=np.uint32)
    _check(lib().oracle_tk_report(C.byref(p.c()), _p(sk), k, k_max, _p(oi), _p(osc)), "oracle_tk_report")
    return oi, osc


def tk_query(p: Params, cs, cells, qindptr, qindices, k: int, k_max: int | None = None, kq=None):
    """Top-k (ids, counts) per query from Topkapi tables, rows of stride k_max."""
    qindptr, qindices = _csr(qindptr, qindices)
    k_max = k if k_max is None else k_max
    nq = len(qindptr) - 1
    oi = np.zeros((nq, k_max), dtype=np.uint32)
    osc = np.zeros((nq, k_max), dtype=np.uint32)
    kqa = None if kq is None else np.ascontiguousarray(kq, dtype=np.uint32)
    cells = np.ascontiguousarray(cells, dtype=np.uint32)
    _check(lib().oracle_tk_query(C.byref(p.c()), _p(cs), _p(cells), _p(qindptr), _p(qindices), nq,
                                 _p(kqa) if kqa is not None else None, k, k_max, _p(oi), _p(osc)),
           "oracle_tk_query")
    return oi, osc


# ------------------------------------------------------- quality references


def jaccard_knn(indptr, indices, qindptr, qindices, k: int):
    """Brute-force Jaccard k nearest rows per query, ties by ascending id:
    (ids [nq, k], intersection sizes [nq, k], union sizes [nq, k]); slots past
    the data size hold (EMPTY, 0, 0)."""
    indptr, indices = _csr(indptr, indices)
    qindptr, qindices = _csr(qindptr, qindices)
    n, nq = len(indptr) - 1, len(qindptr) - 1
    oi = np.zeros((nq, k), dtype=np.uint32)
    on = np.zeros((nq, k), dtype=np.uint32)
    ou = np.zeros((nq, k), dtype=np.uint32)
    _check(lib().oracle_jaccard_knn(_p(indptr), _p(indices) if len(indices) else None, n, _p(qindptr),
                                    _p(qindices) if len(qindices) else None, nq, k, _p(oi), _p(on), _p(ou)),
           "oracle_jaccard_knn")
    return oi, on, ou


def mean_cosine(indptr, indices, qindptr, qindices, ids, k: int):
    """Per query: mean cosine similarity of the first k non-EMPTY ids of its
    row of `ids` (0 when there are none), and how many there were."""
    indptr, indices = _csr(indptr, indices)
    qindptr, qindices = _csr(qindptr, qindices)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    nq = len(qindptr) - 1
    assert ids.shape[0] == nq and ids.ndim == 2
    mean = np.zeros(nq, dtype=np.float64)
    cnt = np.zeros(nq, dtype=np.uint32)
    _check(lib().oracle_mean_cosine(_p(indptr), _p(indices) if len(indices) else None, len(indptr) - 1,
                                    _p(qindptr), _p(qindices) if len(qindices) else None, nq, _p(ids),
                                    ids.shape[1], k, _p(mean), _p(cnt)), "oracle_mean_cosine")
    return mean, cnt
