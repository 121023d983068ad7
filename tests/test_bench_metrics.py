"""bench.py's quality measurements (S@k and the brute-force Jaccard top-k of
the set recall) agree with the oracle's pinned references."""
import numpy as np

import bench
import oracle
import synth


def _data(n, nq, seed):
    law = synth.RowLaw(synth.derive(seed, synth.STREAM_DATA), 1 << 12)
    ip, ix = law.rows(0, n)
    qi, qx, _, _ = law.queries(synth.derive(seed, synth.STREAM_QUERY), n, 0, nq)
    return ip, ix, qi, qx


def test_jaccard_top_matches_oracle():
    ip, ix, qi, qx = _data(3000, 40, 1)
    got = bench.jaccard_top(ip, ix, qi, qx, 10)
    want, _, _ = oracle.jaccard_knn(ip, ix, qi, qx, 10)
    assert (got == want.astype(np.int64)).all()


def test_s_at_k_matches_oracle():
    ip, ix, qi, qx = _data(2000, 30, 2)
    rng = np.random.default_rng(0)
    ids = rng.integers(0, 2000, size=(30, 64)).astype(np.uint32)
    ids[rng.random(ids.shape) < 0.2] = oracle.EMPTY
    ids[3] = oracle.EMPTY  # a query with nothing returned counts 0
    for k in (1, 64):
        mean, _ = oracle.mean_cosine(ip, ix, qi, qx, ids, k)
        assert abs(bench.s_at_k(bench.host_fetch(ip, ix), qi, qx, ids, k) - float(np.mean(mean))) < 1e-12


def test_set_recall():
    truth = np.array([[1, 2, 3], [4, 5, 6]])
    got = np.array([[3, 2, 9], [7, 8, 9]])
    assert abs(bench.set_recall(got, truth) - (2 / 3 + 0) / 2) < 1e-15
