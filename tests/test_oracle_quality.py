"""Pins of the oracle's quality references (brute-force Jaccard k nearest
neighbours, S@k cosine terms) against hand-worked values, an independent
brute force written with Python sets and exact fractions, and identities of
the two similarity measures."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle_util import csr, load_golden

EMPTY = oracle.EMPTY


def test_jaccard_knn_hand_worked():
    g = load_golden("quality_hand.json")
    ip, ix = csr(g["data"])
    qi, qx = csr(g["queries"])
    ids, inter, uni = oracle.jaccard_knn(ip, ix, qi, qx, g["k"])
    for q, want in enumerate(g["knn"]):
        assert ids[q].tolist() == want["ids"]
        assert inter[q].tolist() == want["inter"]
        assert uni[q].tolist() == want["union"]


def test_mean_cosine_hand_worked():
    g = load_golden("quality_hand.json")
    ip, ix = csr(g["data"])
    qi, qx = csr(g["queries"])
    c = g["cosine"]
    mean, cnt = oracle.mean_cosine(ip, ix, qi, qx, np.array(c["ids"], dtype=np.uint32), c["k"])
    assert cnt.tolist() == c["count"]
    assert np.allclose(mean, c["mean"], rtol=0, atol=1e-12)


def _py_knn(data, queries, k):
    # independent brute force: Python sets, exact fractions, a full sort
    out = []
    sets = [set(r) for r in data]
    for q in queries:
        qs = set(q)
        sc = [(-Fraction(len(qs & s), len(qs | s)), i, len(qs & s), len(qs | s)) for i, s in enumerate(sets)]
        sc.sort()
        out.append([(i, a, b) for _, i, a, b in sc[:k]])
    return out


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_jaccard_knn_matches_python_sets(seed):
    rng = np.random.default_rng(seed)
    # a small universe so that overlaps and exact ties are common
    data = [rng.integers(0, 40, size=rng.integers(1, 12)).tolist() for _ in range(300)]
    queries = [rng.integers(0, 40, size=rng.integers(1, 12)).tolist() for _ in range(25)]
    k = 17
    ids, inter, uni = oracle.jaccard_knn(*csr(data), *csr(queries), k)
    want = _py_knn(data, queries, k)
    for q in range(len(queries)):
        assert list(zip(ids[q].tolist(), inter[q].tolist(), uni[q].tolist())) == want[q]


def test_jaccard_knn_self_and_bounds():
    # a dataset row as query is its own nearest neighbour at similarity 1
    # (unless an identical set has a smaller id); every similarity is in
    # [0, 1] and never above the cosine of the same pair
    law = synth.RowLaw(synth.derive(5, synth.STREAM_DATA), 1 << 12)
    ip, ix = law.rows(0, 400)
    rows = [ix[ip[i]:ip[i + 1]] for i in range(400)]
    qrows = [rows[i] for i in (0, 17, 399)]
    ids, inter, uni = oracle.jaccard_knn(ip, ix, *csr(qrows), 400)
    for q, src in enumerate((0, 17, 399)):
        exact = ids[q][inter[q] == uni[q]]  # rows holding the same set
        assert src in exact.tolist() and ids[q, 0] == exact.min()
        assert (inter[q] <= uni[q]).all()
        jac = inter[q] / uni[q]
        assert (np.diff(jac) <= 1e-15).all()
    mean, cnt = oracle.mean_cosine(ip, ix, *csr(qrows), ids, 400)
    assert (cnt == 400).all()
    # mean cosine over all rows >= mean Jaccard over all rows (J <= cos pairwise)
    for q in range(3):
        assert mean[q] >= float(np.mean(inter[q] / uni[q])) - 1e-12


def test_mean_cosine_ignores_order_and_repeats():
    data = [[1, 2, 3, 4], [4, 3, 2, 1, 1, 1]]
    mean, cnt = oracle.mean_cosine(*csr(data), *csr([[2, 1, 2]]), np.array([[0, 1]], dtype=np.uint32), 2)
    assert cnt[0] == 2 and math.isclose(mean[0], 2 / math.sqrt(8), rel_tol=0, abs_tol=1e-15)


def test_mean_cosine_rejects_unknown_ids():
    with pytest.raises(oracle.OracleError):
        oracle.mean_cosine(*csr([[1]]), *csr([[1]]), np.array([[5]], dtype=np.uint32), 1)
