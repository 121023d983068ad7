"""Helpers shared by the oracle tests (test-side only)."""
import json
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def h(x):
    return int(x, 16) if isinstance(x, str) else int(x)


def params_from(d):
    return oracle.Params(**{k: int(v) for k, v in d.items()})


def constants_with(p, **groups):
    """Real constants for p, with the named groups replaced."""
    cs = oracle.constants(p)
    lay = oracle.layout(p)
    for g, vals in groups.items():
        for i, v in enumerate(vals):
            cs[lay[g] + i] = np.uint64(h(v))
    return cs


def csr(rows):
    indptr = np.zeros(len(rows) + 1, dtype=np.int64)
    for i, r in enumerate(rows):
        indptr[i + 1] = indptr[i] + len(r)
    indices = np.array([v for r in rows for v in r], dtype=np.int32)
    return indptr, indices
