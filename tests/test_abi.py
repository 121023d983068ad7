"""Host-side checks of the C ABI library (no GPU needed)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SO = os.path.join(ROOT, "paper_2008_03260_amd", "libslash.so")
HDR = os.path.join(ROOT, "include", "slash.h")


def _declared():
    txt = open(HDR).read()
    return sorted(set(re.findall(r"^SLASH_API\s+[\w\s\*]+?\b(slash_\w+)\s*\(", txt, flags=re.M)))


def _ensure_built():
    if not os.path.exists(SO):
        from paper_2008_03260_amd import build
        build.build()


def test_header_declares_core_calls():
    names = _declared()
    for n in ("slash_build", "slash_insert", "slash_query", "slash_query_batched", "slash_free",
              "slash_last_error", "slash_serve_start", "slash_serve_submit_query", "slash_serve_poll",
              "slash_serve_stop"):
        assert n in names


def test_library_exports_every_declared_symbol():
    _ensure_built()
    lib = ctypes.CDLL(SO)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_library_exports_nothing_else():
    _ensure_built()
    import subprocess
    out = subprocess.check_output(["nm", "-D", "--defined-only", SO]).decode()
    exported = sorted({l.split()[-1] for l in out.splitlines() if " T " in l})
    assert exported == _declared(), set(exported) ^ set(_declared())
