"""Host-side checks that need no GPU: the bench contract's refusal of more
than one GPU, and host-visible errors of the C ABI that are raised before any
device work (NULL arguments, invalid parameters)."""
import ctypes
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def _lib():
    so = os.path.join(ROOT, "paper_2008_03260_amd", "libslash.so")
    if not os.path.exists(so):
        from paper_2008_03260_amd import build
        build.build()
    return ctypes.CDLL(so)


def test_null_and_invalid_arguments_fail_before_device_work():
    sys.path.insert(0, ROOT)
    from paper_2008_03260_amd import api
    L = _lib()
    L.slash_last_error.restype = ctypes.c_char_p
    out = ctypes.c_void_p()
    # NULL out pointer and NULL params are rejected on the host
    assert L.slash_build(None, api.CSR(None, None, 0), None, None) == api.E_INVAL
    assert L.slash_build(None, api.CSR(None, None, 0), None, ctypes.byref(out)) == api.E_INVAL
    assert b"NULL" in L.slash_last_error()
    # parameters outside what the kernels implement
    bad = api.Params.of(dim=1 << 20, K=64, L=128, log2_buckets=10, R=8, cm_rows=2, log2_cm_width=8, k_max=10)
    assert L.slash_build(ctypes.byref(bad), api.CSR(None, None, 0), None, ctypes.byref(out)) == api.E_UNSUPPORTED
    bad = api.Params.of(dim=1 << 20, K=4, L=8, log2_buckets=10, R=300, cm_rows=2, log2_cm_width=8, k_max=10)
    assert L.slash_build(ctypes.byref(bad), api.CSR(None, None, 0), None, ctypes.byref(out)) == api.E_INVAL
    assert b"R must be" in L.slash_last_error()
    # shapes no query kernel can answer are refused at build: more slots per
    # query than 16 waves hold (16 per thread), a sketch larger than LDS
    for kw in (dict(L=128, R=256, cm_rows=4, log2_cm_width=12), dict(L=32, R=64, cm_rows=16, log2_cm_width=16)):
        bad = api.Params.of(dim=1 << 20, K=4, log2_buckets=10, k_max=10, **kw)
        assert L.slash_build(ctypes.byref(bad), api.CSR(None, None, 0), None, ctypes.byref(out)) == api.E_UNSUPPORTED
        assert b"no query form fits" in L.slash_last_error()
    # calls on a NULL index
    L.slash_free(None)  # a NULL index is ignored
    assert L.slash_query(None, api.CSR(None, None, 0), None, 1, 0, None, None, None) == api.E_INVAL
    assert L.slash_import_tables(None, None, None, 0, None, ctypes.byref(out)) == api.E_INVAL
