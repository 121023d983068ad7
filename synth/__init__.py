"""Seeded synthetic workload generator (inputs only; none of the method's arithmetic).

Rows, queries and request traces are counter-based (Philox4x32-10), so any row
or query can be regenerated alone and results do not depend on thread count.
The C source is ``synth/synth.c``; ``build_lib()`` compiles it into
``synth/libsynth.so``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_lib = None


_SO_GPU = os.path.join(_HERE, "libsynth_gpu.so")
_lib_gpu = None


def build_lib() -> str:
    """Compile the generator libraries in-tree (always recompiles): the host
    library (gcc) and its device build (hipcc, gfx950)."""
    src = os.path.join(_HERE, "synth.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-pthread", "-o", tmp, src, "-lm"])
    os.replace(tmp, _SO)
    tmp = _SO_GPU + ".tmp"
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-O3", "-fPIC", "-shared", "-std=c++17",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                           "-o", tmp, os.path.join(_HERE, "synth_gpu.hip")],
                          stderr=subprocess.DEVNULL)
    os.replace(tmp, _SO_GPU)
    return _SO


class RowsSpec(C.Structure):
    _fields_ = [
        ("key", C.c_uint64), ("dim", C.c_uint32), ("index_kind", C.c_uint32),
        ("zipf_s", C.c_double), ("nnz_kind", C.c_uint32), ("nnz_a", C.c_double),
        ("nnz_b", C.c_double), ("nnz_lo", C.c_uint32), ("nnz_hi", C.c_uint32),
    ]


class QuerySpec(C.Structure):
    _fields_ = [
        ("key", C.c_uint64), ("n_data", C.c_uint64), ("nnz_mode", C.c_uint32),
        ("median", C.c_double), ("sigma", C.c_double), ("lo", C.c_uint32), ("hi", C.c_uint32),
        ("f_lo", C.c_double), ("f_hi", C.c_double), ("n_kmix", C.c_uint32),
        ("kmix", C.c_uint32 * 8),
    ]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            raise RuntimeError("synth/libsynth.so is not built; run __graft_entry__.build()")
        L = C.CDLL(_SO)
        L.synth_derive.restype = C.c_uint64
        L.synth_derive.argtypes = [C.c_uint64, C.c_uint32]
        L.synth_ctx_new.restype = C.c_void_p
        L.synth_ctx_new.argtypes = [C.POINTER(RowsSpec)]
        L.synth_ctx_free.argtypes = [C.c_void_p]
        L.synth_rows_nnz.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.c_void_p, C.c_int]
        L.synth_rows_fill.argtypes = [C.c_void_p, C.c_uint64, C.c_uint64, C.c_void_p, C.c_void_p, C.c_int]
        L.synth_queries_nnz.argtypes = [C.c_void_p, C.POINTER(QuerySpec), C.c_uint64, C.c_uint64,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
        L.synth_queries_fill.argtypes = [C.c_void_p, C.POINTER(QuerySpec), C.c_uint64, C.c_uint64,
                                         C.c_void_p, C.c_void_p, C.c_int]
        L.synth_arrivals.argtypes = [C.c_uint64, C.c_uint64, C.c_double, C.c_double, C.c_uint32,
                                     C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p]
        L.synth_philox.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        L.synth_ctx_tables.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(RowsSpec)]
        _lib = L
    return _lib


def lib_gpu():
    global _lib_gpu
    if _lib_gpu is None:
        if not os.path.exists(_SO_GPU):
            raise RuntimeError("synth/libsynth_gpu.so is not built; run __graft_entry__.build()")
        L = C.CDLL(_SO_GPU)
        u64, u32, vp = C.c_uint64, C.c_uint32, C.c_void_p
        L.synth_gpu_rows_nnz.argtypes = [u64, u64, u64, vp, u32, u32, u32, vp, vp]
        L.synth_gpu_rows_fill.argtypes = [u64, u64, u64, u32, C.c_int, vp, vp, vp, vp]
        _lib_gpu = L
    return _lib_gpu


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def default_threads() -> int:
    n = os.cpu_count() or 1
    return max(1, min(16, n))


def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    lib().synth_philox(_ptr(c), _ptr(k), _ptr(o))
    return o


# stream tags for derive()
STREAM_DATA, STREAM_QUERY, STREAM_INDEX, STREAM_ARRIVAL, STREAM_INSERT = 1, 2, 3, 4, 5


def derive(master: int, tag: int) -> int:
    return int(lib().synth_derive(master & (2**64 - 1), tag))


class RowLaw:
    """Distribution of binary sparse rows: nnz law + feature-index law."""

    def __init__(self, key: int, dim: int, index: str = "zipf", zipf_s: float = 1.1,
                 nnz: str = "poisson", nnz_a: float = 40.0, nnz_b: float = 0.0,
                 nnz_lo: int = 1, nnz_hi: int = 2**31 - 1):
        self.spec = RowsSpec(key & (2**64 - 1), dim, 0 if index == "zipf" else 1, zipf_s,
                             0 if nnz == "poisson" else 1, nnz_a, nnz_b, max(1, nnz_lo), nnz_hi)
        self._ctx = lib().synth_ctx_new(C.byref(self.spec))
        # held so that the destructor still works while the interpreter tears
        # down module globals
        self._free = lib().synth_ctx_free
        if not self._ctx:
            raise ValueError("invalid row law")

    def __del__(self):
        if getattr(self, "_ctx", None):
            self._free(self._ctx)
            self._ctx = None

    @property
    def dim(self) -> int:
        return int(self.spec.dim)

    def rows(self, row0: int, n: int, threads: int | None = None):
        """CSR (indptr int64[n+1], indices int32[nnz]) of rows [row0, row0+n)."""
        th = threads or default_threads()
        nnz = np.empty(n, dtype=np.uint32)
        lib().synth_rows_nnz(self._ctx, row0, n, _ptr(nnz), th)
        indptr = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(nnz, out=indptr[1:])
        indices = np.empty(int(indptr[-1]), dtype=np.int32)
        lib().synth_rows_fill(self._ctx, row0, n, _ptr(indptr), _ptr(indices), th)
        return indptr, indices

    def gpu_rows(self, row0: int, n: int, stream=None):
        """Rows [row0, row0+n) generated on the current HIP device, bit-identical
        to rows(); returns (indptr int64, indices int32) device tensors."""
        import torch
        g = lib_gpu()
        tab_p, pcdf_p, pn, spec = C.c_void_p(), C.c_void_p(), C.c_uint32(), RowsSpec()
        lib().synth_ctx_tables(self._ctx, C.byref(tab_p), C.byref(pcdf_p), C.byref(pn), C.byref(spec))
        if spec.nnz_kind != 0:
            raise NotImplementedError("device generation supports Poisson row sizes only")
        dev = torch.device("cuda", torch.cuda.current_device())
        if getattr(self, "_dev_tabs", None) is None:
            pcdf = np.ctypeslib.as_array(C.cast(pcdf_p, C.POINTER(C.c_double)), shape=(pn.value,)).copy()
            tab = None
            if spec.index_kind == 0:
                tab = np.ctypeslib.as_array(C.cast(tab_p, C.POINTER(C.c_uint64)), shape=(spec.dim,)).copy()
                tab = torch.from_numpy(tab.view(np.int64)).to(dev)
            self._dev_tabs = (torch.from_numpy(pcdf).to(dev), tab)
        pcdf_t, tab_t = self._dev_tabs
        st = C.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)
        nnz = torch.empty(n, dtype=torch.int32, device=dev)
        rc = g.synth_gpu_rows_nnz(spec.key, row0, n, C.c_void_p(pcdf_t.data_ptr()), pn.value, spec.nnz_lo,
                                  spec.nnz_hi, C.c_void_p(nnz.data_ptr()), st)
        if rc:
            raise RuntimeError("synth_gpu_rows_nnz failed")
        indptr = torch.zeros(n + 1, dtype=torch.int64, device=dev)
        torch.cumsum(nnz, 0, out=indptr[1:])
        del nnz
        total = int(indptr[-1].item())
        indices = torch.empty(max(total, 1), dtype=torch.int32, device=dev)
        rc = g.synth_gpu_rows_fill(spec.key, row0, n, spec.dim, 1 if spec.index_kind == 0 else 0,
                                   C.c_void_p(tab_t.data_ptr()) if tab_t is not None else None,
                                   C.c_void_p(indptr.data_ptr()), C.c_void_p(indices.data_ptr()), st)
        if rc:
            raise RuntimeError("synth_gpu_rows_fill failed")
        return indptr, indices[:total]

    def device_rows(self, row0: int, n: int, chunk: int = 1 << 20, threads: int | None = None):
        """Rows [row0, row0+n) as one CSR on the current HIP device, the same
        rows as rows(): generated on the device for Poisson row sizes, else on
        the host chunk by chunk (bounded host memory) and copied over."""
        if self.spec.nnz_kind == 0:
            return self.gpu_rows(row0, n)
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        th = threads or default_threads()
        nnz = np.empty(n, dtype=np.uint32)
        lib().synth_rows_nnz(self._ctx, row0, n, _ptr(nnz), th)
        indptr = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(nnz, out=indptr[1:])
        total = int(indptr[-1])
        indices = torch.empty(max(total, 1), dtype=torch.int32, device=dev)
        for a in range(0, n, chunk):
            b = min(n, a + chunk)
            sub = np.ascontiguousarray(indptr[a:b + 1])
            part = np.empty(int(sub[-1] - sub[0]), dtype=np.int32)
            lib().synth_rows_fill(self._ctx, row0 + a, b - a, _ptr(sub), _ptr(part), th)
            indices[int(sub[0]):int(sub[-1])].copy_(torch.from_numpy(part))
        return torch.from_numpy(indptr).to(dev), indices[:total]

    def queries(self, key: int, n_data: int, q0: int, n: int, nnz_mode: str = "same",
                median: float = 40.0, sigma: float = 1.0, lo: int = 5, hi: int = 2000,
                f: tuple = (0.2, 0.2), kmix=(10,), threads: int | None = None):
        """Perturbed dataset points with a known planted source.

        Returns (indptr, indices, src int64[n], k uint32[n])."""
        th = threads or default_threads()
        km = (C.c_uint32 * 8)(*list(kmix)[:8])
        q = QuerySpec(key & (2**64 - 1), n_data, 0 if nnz_mode == "same" else 1, median, sigma,
                      lo, hi, f[0], f[1], len(kmix), km)
        src = np.empty(n, dtype=np.uint64)
        nnz = np.empty(n, dtype=np.uint32)
        kq = np.empty(n, dtype=np.uint32)
        lib().synth_queries_nnz(self._ctx, C.byref(q), q0, n, _ptr(src), _ptr(nnz), _ptr(kq), th)
        indptr = np.zeros(n + 1, dtype=np.int64)
        np.cumsum(nnz, out=indptr[1:])
        indices = np.empty(int(indptr[-1]), dtype=np.int32)
        rc = lib().synth_queries_fill(self._ctx, C.byref(q), q0, n, _ptr(indptr), _ptr(indices), th)
        if rc != 0:
            raise RuntimeError(f"query generation failed ({rc})")
        return indptr, indices, src.astype(np.int64), kq


def arrivals(key: int, n: int, rate: float, insert_frac: float = 0.1, ins_lo: int = 1,
             ins_hi: int = 4096):
    """Open-loop Poisson request trace: (t_arrival s, is_insert bool, insert_size)."""
    t = np.empty(n, dtype=np.float64)
    ins = np.empty(n, dtype=np.uint8)
    sz = np.empty(n, dtype=np.uint32)
    rc = lib().synth_arrivals(key & (2**64 - 1), n, rate, insert_frac, ins_lo, ins_hi,
                              _ptr(t), _ptr(ins), _ptr(sz))
    if rc != 0:
        raise ValueError("invalid arrival spec")
    return t, ins.astype(bool), sz
