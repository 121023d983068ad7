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


def test_binding_struct_layouts_match_header(tmp_path):
    """Every struct the binding passes across the ABI has the header's size and field offsets."""
    import subprocess
    import sys
    sys.path.insert(0, ROOT)
    from paper_2008_03260_amd import api
    checks = {
        "slash_params": (api.Params, ["dim", "k_max", "hash_mode", "seed"]),
        "slash_csr": (api.CSR, ["indptr", "indices", "n_rows"]),
        "slash_index_info": (api.IndexInfo, ["params", "n_items", "table_bytes", "n_buckets"]),
        "slash_schedule": (api.Schedule, ["waves_per_query", "groups_per_cu"]),
        "slash_phase_stat": (api.PhaseStat, ["name", "launches", "total_ms", "alg_bytes"]),
        "slash_serve_config": (api.ServeConfig, ["hbm_budget_bytes", "max_batch", "max_query_nnz", "max_insert_nnz",
                                                 "insert_fusion"]),
        "slash_completion": (api.Completion, ["ticket", "status", "ids", "scores", "t_submit_s", "t_done_s"]),
        "slash_serve_stats": (api.ServeStats, ["queries_done", "peak_hbm_bytes", "busy_s", "wait_s", "pack_s",
                                               "fused_commits", "split_batches"]),
    }
    src = ['#include <stdio.h>', '#include <stddef.h>', '#include "slash.h"', "int main(void) {"]
    for cname, (_, fields) in checks.items():
        src.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for f in fields:
            src.append(f'  printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    src.append("  return 0;\n}")
    c = tmp_path / "layout.c"
    c.write_text("\n".join(src))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(c)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)]).decode().splitlines())
    for cname, (cls, fields) in checks.items():
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for f in fields:
            assert int(got[f"{cname}.{f}"]) == getattr(cls, f).offset, (cname, f)
