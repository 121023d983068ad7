"""ctypes binding of libslash.so (include/slash.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  Device buffers are torch tensors on the current HIP device
(uint32 data travels in int32 tensors, bit-identical); streams are torch
streams.  Functions keep the C names.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
SO_PATH = os.path.join(_HERE, "libslash.so")
_lib = None

SLASH_OK, E_INVAL, E_NOMEM, E_DEVICE, E_CAPACITY, E_BUSY, E_CLOSED, E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6, -7
FLAG_TRUSTED = 1
FLAG_EXACT = 2
EMPTY = 0xFFFFFFFF
_NAMES = {0: "OK", -1: "E_INVAL", -2: "E_NOMEM", -3: "E_DEVICE", -4: "E_CAPACITY", -5: "E_BUSY",
          -6: "E_CLOSED", -7: "E_UNSUPPORTED"}


class SlashError(RuntimeError):
    def __init__(self, code: int, what: str, msg: str):
        super().__init__(f"{what}: {_NAMES.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [(n, C.c_uint32) for n in ("dim", "K", "L", "log2_buckets", "R", "cm_rows", "log2_cm_width",
                                          "k_max", "hash_mode", "bucket")] + [("seed", C.c_uint64)]

    @classmethod
    def of(cls, **kw) -> "Params":
        p = cls()
        for k, v in kw.items():
            setattr(p, k, (int(v) & (2**64 - 1)) if k == "seed" else int(v))
        return p


class CSR(C.Structure):
    _fields_ = [("indptr", C.c_void_p), ("indices", C.c_void_p), ("n_rows", C.c_uint64)]


class IndexInfo(C.Structure):
    _fields_ = [("params", Params), ("n_items", C.c_uint64), ("table_bytes", C.c_uint64),
                ("n_buckets", C.c_uint32), ("reserved", C.c_uint32)]


class PhaseStat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_uint32), ("reserved", C.c_uint32),
                ("total_ms", C.c_double), ("alg_bytes", C.c_double)]


SERVE_MAX_K = 128


class ServeConfig(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_uint64), ("max_batch", C.c_uint32), ("max_inflight", C.c_uint32),
                ("queue_capacity", C.c_uint32), ("max_wait_us", C.c_uint32), ("max_query_nnz", C.c_uint32),
                ("max_insert_nnz", C.c_uint32), ("insert_fusion", C.c_uint32), ("reserved", C.c_uint32)]


class Completion(C.Structure):
    _fields_ = [("ticket", C.c_uint64), ("epoch", C.c_uint64), ("status", C.c_int32), ("kind", C.c_uint32),
                ("k", C.c_uint32), ("n_ids", C.c_uint32), ("first_id", C.c_uint32), ("reserved", C.c_uint32),
                ("ids", C.c_uint32 * SERVE_MAX_K), ("scores", C.c_uint32 * SERVE_MAX_K),
                ("t_submit_s", C.c_double), ("t_done_s", C.c_double)]


class ServeStats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("queries_done", "inserts_done", "rows_inserted", "batches",
                                          "rejected_busy", "rejected_nomem", "peak_inflight", "peak_hbm_bytes")] + \
               [("busy_s", C.c_double), ("launch_s", C.c_double), ("wait_s", C.c_double), ("pack_s", C.c_double),
                ("fused_commits", C.c_uint64), ("split_batches", C.c_uint64)]


class Schedule(C.Structure):
    _fields_ = [("waves_per_query", C.c_uint32), ("queries_per_ticket", C.c_uint32),
                ("groups_per_cu", C.c_uint32), ("reserved", C.c_uint32)]


def lib() -> C.CDLL:
    """The loaded library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(SO_PATH):
            raise RuntimeError(f"{SO_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(SO_PATH)
        vp, u32, u64, st = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int
        P = C.POINTER
        sig = {
            "slash_build": ([P(Params), CSR, vp, P(vp)], st),
            "slash_insert": ([vp, CSR, u32, vp, vp], st),
            "slash_query": ([vp, CSR, vp, u32, u32, vp, vp, vp], st),
            "slash_query_batched": ([vp, CSR, vp, u32, u32, vp, vp, P(Schedule), vp], st),
            "slash_query_batched_static": ([vp, CSR, vp, u32, u32, vp, vp, P(Schedule), vp], st),
            "slash_autotune": ([vp, CSR, u32, P(Schedule), vp], st),
            "slash_hash": ([vp, CSR, u32, vp, vp], st),
            "slash_export_tables": ([vp, vp, vp, vp], st),
            "slash_import_tables": ([P(Params), vp, vp, u64, vp, P(vp)], st),
            "slash_index_info_get": ([vp, P(IndexInfo)], st),
            "slash_save": ([vp, C.c_char_p, vp], st),
            "slash_load": ([C.c_char_p, vp, P(vp)], st),
            "slash_build_profile": ([vp, vp, u32, P(u32)], st),
            "slash_free": ([vp], None),
            "slash_last_error": ([], C.c_char_p),
            "slash_set_allocator": ([vp, vp, vp], st),
            "slash_release_cache": ([], None),
            "slash_serve_start": ([vp, P(ServeConfig), P(vp)], st),
            "slash_serve_submit_query": ([vp, vp, u32, u32, P(u64)], st),
            "slash_serve_submit_insert": ([vp, vp, vp, u32, P(u64)], st),
            "slash_serve_poll": ([vp, P(Completion), u32, P(u32)], st),
            "slash_serve_stop": ([vp, P(ServeStats)], st),
            "slash_serve_replay": ([vp, u64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, u32], st),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def slash_last_error() -> str:
    return lib().slash_last_error().decode()


def _check(rc: int, what: str):
    if rc != SLASH_OK:
        raise SlashError(rc, what, slash_last_error())


def _stream(stream) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_i32(t: torch.Tensor) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    return t.contiguous()


def csr(indptr: torch.Tensor, indices: torch.Tensor) -> tuple[CSR, tuple]:
    """CSR struct over device tensors (int64 indptr, int32 indices); returns
    (struct, tensors to keep alive)."""
    ip = _dev_i32(indptr)
    ix = _dev_i32(indices)
    if ip.dtype != torch.int64 or ix.dtype != torch.int32:
        raise TypeError("indptr must be int64 and indices int32")
    n = ip.numel() - 1
    c = CSR(ip.data_ptr() if n >= 0 else 0, ix.data_ptr() if ix.numel() else ip.data_ptr(), max(n, 0))
    return c, (ip, ix)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


# ---------------------------------------------------------------- calls


def slash_build(params: Params, indptr: torch.Tensor, indices: torch.Tensor, stream=None) -> C.c_void_p:
    c, keep = csr(indptr, indices)
    out = C.c_void_p()
    _check(lib().slash_build(C.byref(params), c, _stream(stream), C.byref(out)), "slash_build")
    return out


def slash_insert(index, indptr, indices, flags: int = 0, new_ids: torch.Tensor | None = None, stream=None):
    c, keep = csr(indptr, indices)
    _check(lib().slash_insert(index, c, flags, _ptr(new_ids), _stream(stream)), "slash_insert")


def _outputs(index, n, out_ids, out_scores):
    if out_ids is None or out_scores is None:
        km = slash_index_info_get(index)["k_max"]
        dev = torch.device("cuda", torch.cuda.current_device())
        if out_ids is None:
            out_ids = torch.empty((n, km), dtype=torch.int32, device=dev)
        if out_scores is None:
            out_scores = torch.empty((n, km), dtype=torch.int32, device=dev)
    return out_ids, out_scores


def slash_query(index, indptr, indices, k: int, k_per_query: torch.Tensor | None = None, flags: int = 0,
                out_ids=None, out_scores=None, stream=None):
    """Top-k (ids, scores) as int32 tensors [n, k_max] holding uint32 bits."""
    c, keep = csr(indptr, indices)
    oi, osc = _outputs(index, c.n_rows, out_ids, out_scores)
    _check(lib().slash_query(index, c, _ptr(k_per_query), k, flags, _ptr(oi), _ptr(osc), _stream(stream)),
           "slash_query")
    return oi, osc


def slash_query_batched(index, indptr, indices, k: int, k_per_query=None, flags: int = 0, schedule=None,
                        out_ids=None, out_scores=None, stream=None):
    c, keep = csr(indptr, indices)
    oi, osc = _outputs(index, c.n_rows, out_ids, out_scores)
    sch = None
    if schedule is not None:
        sch = C.byref(Schedule(*[int(schedule.get(f, 0)) for f, _ in Schedule._fields_]))
    _check(lib().slash_query_batched(index, c, _ptr(k_per_query), k, flags, _ptr(oi), _ptr(osc), sch,
                                     _stream(stream)), "slash_query_batched")
    return oi, osc


def slash_query_batched_static(index, indptr, indices, k: int, k_per_query=None, flags: int = 0, schedule=None,
                               out_ids=None, out_scores=None, stream=None):
    """slash_query_batched without any device allocation by the library
    (its scratch is a static device array; see include/slash.h)."""
    c, keep = csr(indptr, indices)
    oi, osc = _outputs(index, c.n_rows, out_ids, out_scores)
    sch = None
    if schedule is not None:
        sch = C.byref(Schedule(*[int(schedule.get(f, 0)) for f, _ in Schedule._fields_]))
    _check(lib().slash_query_batched_static(index, c, _ptr(k_per_query), k, flags, _ptr(oi), _ptr(osc), sch,
                                            _stream(stream)), "slash_query_batched_static")
    return oi, osc


def slash_autotune(index, indptr, indices, k: int, stream=None) -> dict:
    c, keep = csr(indptr, indices)
    best = Schedule()
    _check(lib().slash_autotune(index, c, k, C.byref(best), _stream(stream)), "slash_autotune")
    return {f: int(getattr(best, f)) for f, _ in Schedule._fields_}


def slash_hash(index, indptr, indices, flags: int = 0, stream=None) -> torch.Tensor:
    c, keep = csr(indptr, indices)
    L = slash_index_info_get(index)["L"]
    out = torch.empty((c.n_rows, L), dtype=torch.int32, device=indptr.device)
    _check(lib().slash_hash(index, c, flags, _ptr(out), _stream(stream)), "slash_hash")
    return out


def slash_export_tables(index, stream=None):
    info = slash_index_info_get(index)
    dev = torch.device("cuda", torch.cuda.current_device())
    if info["bucket"]:
        # Topkapi cells: (heavy hitter, count) per cell of cm_rows x 2^log2_cm_width
        shape = (info["L"], info["n_buckets"], info["cm_rows"], 1 << info["log2_cm_width"], 2)
    else:
        shape = (info["L"], info["n_buckets"], info["R"])
    ids = torch.empty(shape, dtype=torch.int32, device=dev)
    seen = torch.empty((info["L"], info["n_buckets"]), dtype=torch.int32, device=dev)
    _check(lib().slash_export_tables(index, _ptr(ids), _ptr(seen), _stream(stream)), "slash_export_tables")
    return ids, seen


def slash_import_tables(params: Params, ids: torch.Tensor, seen: torch.Tensor, n_items: int, stream=None) -> C.c_void_p:
    """New index over exported tables (ids [L][2^B][R] or Topkapi cells
    [L][2^B][cm_rows][2^log2_cm_width][2], seen [L][2^B] device tensors)."""
    out = C.c_void_p()
    _check(lib().slash_import_tables(C.byref(params), _ptr(ids.contiguous()), _ptr(seen.contiguous()), n_items,
                                     _stream(stream), C.byref(out)), "slash_import_tables")
    return out


def slash_save(index, path: str, stream=None):
    _check(lib().slash_save(index, os.fsencode(path), _stream(stream)), "slash_save")


def slash_load(path: str, stream=None) -> C.c_void_p:
    out = C.c_void_p()
    _check(lib().slash_load(os.fsencode(path), _stream(stream), C.byref(out)), "slash_load")
    return out


def slash_index_info_get(index) -> dict:
    info = IndexInfo()
    _check(lib().slash_index_info_get(index, C.byref(info)), "slash_index_info_get")
    d = {f: int(getattr(info.params, f)) for f, _ in Params._fields_}
    d.update(n_items=int(info.n_items), table_bytes=int(info.table_bytes), n_buckets=int(info.n_buckets))
    return d


def slash_build_profile(index) -> dict:
    """Per-phase build timing (HIP events on the build stream):
    {phase: {launches, total_ms, alg_bytes}}."""
    arr = (PhaseStat * 16)()
    n = C.c_uint32()
    _check(lib().slash_build_profile(index, arr, 16, C.byref(n)), "slash_build_profile")
    return {arr[i].name.decode(): {"launches": int(arr[i].launches), "total_ms": float(arr[i].total_ms),
                                   "alg_bytes": float(arr[i].alg_bytes)} for i in range(n.value)}


def slash_free(index):
    if index:
        lib().slash_free(index)


def slash_release_cache():
    """Return the device blocks the library keeps for reuse to the device."""
    lib().slash_release_cache()


# ------------------------------------------------------------- serving


def _np(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(C.c_void_p)


def slash_serve_start(index, hbm_budget_bytes=1 << 30, max_batch=1024, max_inflight=4, queue_capacity=1 << 20,
                      max_wait_us=0, max_query_nnz=4096, max_insert_nnz=0, insert_fusion=0) -> C.c_void_p:
    cfg = ServeConfig(hbm_budget_bytes, max_batch, max_inflight, queue_capacity, max_wait_us, max_query_nnz,
                      max_insert_nnz, insert_fusion, 0)
    out = C.c_void_p()
    _check(lib().slash_serve_start(index, C.byref(cfg), C.byref(out)), "slash_serve_start")
    return out


def slash_serve_submit_query(srv, indices, k: int) -> int:
    a, p = _np(indices, np.int32)
    t = C.c_uint64()
    _check(lib().slash_serve_submit_query(srv, p, len(a), k, C.byref(t)), "slash_serve_submit_query")
    return int(t.value)


def slash_serve_submit_insert(srv, indptr, indices) -> int:
    ip, pp = _np(indptr, np.int64)
    ix, px = _np(indices, np.int32)
    t = C.c_uint64()
    _check(lib().slash_serve_submit_insert(srv, pp, px, len(ip) - 1, C.byref(t)), "slash_serve_submit_insert")
    return int(t.value)


def slash_serve_poll(srv, max_n: int = 1024) -> list:
    buf = (Completion * max_n)()
    n = C.c_uint32()
    _check(lib().slash_serve_poll(srv, buf, max_n, C.byref(n)), "slash_serve_poll")
    out = []
    for i in range(n.value):
        c = buf[i]
        out.append({"ticket": int(c.ticket), "epoch": int(c.epoch), "status": int(c.status), "kind": int(c.kind),
                    "k": int(c.k), "n_ids": int(c.n_ids), "first_id": int(c.first_id),
                    "ids": np.array(c.ids[:c.k], dtype=np.uint32), "scores": np.array(c.scores[:c.k], dtype=np.uint32),
                    "t_submit_s": float(c.t_submit_s), "t_done_s": float(c.t_done_s)})
    return out


def slash_serve_stop(srv) -> dict:
    st = ServeStats()
    _check(lib().slash_serve_stop(srv, C.byref(st)), "slash_serve_stop")
    return {f: (float(getattr(st, f)) if f.endswith("_s") else int(getattr(st, f))) for f, _ in ServeStats._fields_}


def slash_serve_replay(srv, t_arrival, is_insert, ins_rows, q_indptr, q_indices, q_k, ins_indptr, ins_indices,
                       out_stride: int = 0):
    """Open-loop replay; returns (latency_s float64[n], ids uint32[n, out_stride] or None)."""
    n = len(t_arrival)
    ta, pta = _np(t_arrival, np.float64)
    ii, pii = _np(np.asarray(is_insert).astype(np.uint8), np.uint8)
    ir, pir = _np(ins_rows, np.uint32)
    qp, pqp = _np(q_indptr, np.int64)
    qx, pqx = _np(q_indices, np.int32)
    qk, pqk = _np(q_k, np.uint32)
    ip_, pip = _np(ins_indptr, np.int64)
    ix, pix = _np(ins_indices, np.int32)
    lat = np.zeros(n, dtype=np.float64)
    ids = np.full((n, max(out_stride, 1)), EMPTY, dtype=np.uint32) if out_stride else None
    _check(lib().slash_serve_replay(srv, n, pta, pii, pir, pqp, pqx, pqk, pip, pix, lat.ctypes.data_as(C.c_void_p),
                                    ids.ctypes.data_as(C.c_void_p) if ids is not None else None, out_stride),
           "slash_serve_replay")
    return lat, ids


def as_u32(t: torch.Tensor) -> np.ndarray:
    """Host numpy uint32 view of an int32 device tensor."""
    return t.detach().cpu().numpy().view(np.uint32)


class Index:
    """Owning wrapper around a slash_index handle."""

    def __init__(self, params: Params, indptr, indices, stream=None):
        self.params = params
        self.handle = slash_build(params, indptr, indices, stream) if indptr is not None else None

    @classmethod
    def from_tables(cls, params: Params, ids, seen, n_items: int, stream=None):
        """Index restored from exported tables (see tables())."""
        self = cls(params, None, None)
        self.handle = slash_import_tables(params, ids, seen, n_items, stream)
        return self

    @classmethod
    def load(cls, path: str, stream=None):
        """Index loaded from a file written by save()."""
        self = cls(None, None, None)
        self.handle = slash_load(path, stream)
        info = slash_index_info_get(self.handle)
        self.params = Params.of(**{f: info[f] for f, _ in Params._fields_})
        return self

    def save(self, path: str, stream=None):
        slash_save(self.handle, path, stream)

    def close(self):
        if getattr(self, "handle", None):
            slash_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def insert(self, indptr, indices, flags=0, new_ids=None, stream=None):
        slash_insert(self.handle, indptr, indices, flags, new_ids, stream)

    def query(self, indptr, indices, k, **kw):
        return slash_query(self.handle, indptr, indices, k, **kw)

    def query_batched(self, indptr, indices, k, **kw):
        return slash_query_batched(self.handle, indptr, indices, k, **kw)

    def autotune(self, indptr, indices, k, stream=None):
        return slash_autotune(self.handle, indptr, indices, k, stream)

    def hash(self, indptr, indices, flags=0, stream=None):
        return slash_hash(self.handle, indptr, indices, flags, stream)

    def tables(self, stream=None):
        return slash_export_tables(self.handle, stream)

    def info(self):
        return slash_index_info_get(self.handle)
