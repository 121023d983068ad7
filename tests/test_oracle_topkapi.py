"""Pins of the oracle's Topkapi buckets (Section 3.1, Appendix 2) against
things other than itself: hand-worked examples, the majority-vote theorem for
a one-cell sketch, the closed form of a sketch of distinct ids, merge
identities, the lower-bound invariant against brute-force counts, and
batch independence of streaming insertion."""
import numpy as np
import pytest

import oracle
import synth
from oracle_util import constants_with, csr, h, load_golden, params_from

EMPTY = oracle.EMPTY


def _row_hash(p, cs, r, c):
    # count-min row hash written from its definition with Python integers
    lay = oracle.layout(p)
    if p.log2_cm_width == 0:
        return 0
    a, b = int(cs[lay["a_r"] + r]), int(cs[lay["b_r"] + r])
    return ((a * c + b) % 2**64) >> (64 - p.log2_cm_width)


def _hand_params(lw, rows):
    d = load_golden("doph_hand.json")
    p = params_from(d["params"])
    p.log2_cm_width = lw
    p.cm_rows = rows
    return p, d


def test_single_cell_hand_worked():
    g = load_golden("topkapi_hand.json")["single_cell"]
    p, _ = _hand_params(0, 1)
    cs = oracle.constants(p)
    for stream, cell in zip(g["streams"], g["cells"]):
        sk = oracle.tk_sketch(p, cs, stream)
        assert sk.reshape(-1).tolist() == cell


def test_two_row_sketch_and_report_hand_worked():
    g = load_golden("topkapi_hand.json")["two_rows"]
    p, _ = _hand_params(g["log2_cm_width"], len(g["a_r"]))
    cs = constants_with(p, a_r=g["a_r"], b_r=g["b_r"])
    sk = oracle.tk_sketch(p, cs, g["stream"])
    assert sk.tolist() == g["sketch"]
    oi, osc = oracle.tk_report(p, sk, g["k"], g["k_max"])
    assert oi.tolist() == g["ids"] and osc.tolist() == g["scores"]


def test_merge_cells_hand_worked():
    g = load_golden("topkapi_hand.json")["merge_cells"]
    p, _ = _hand_params(0, 1)
    for a, b, want in g["cases"]:
        got = oracle.tk_merge(p, np.array([[a]], dtype=np.uint32), np.array([[b]], dtype=np.uint32))
        assert got.reshape(-1).tolist() == want, (a, b)


def test_query_fold_hand_worked():
    t = load_golden("topkapi_hand.json")
    g, q = t["two_rows"], t["query_fold"]
    p, d = _hand_params(g["log2_cm_width"], len(g["a_r"]))
    qh = load_golden("query_hand.json")
    groups = dict(d["constants"])
    groups.update(dir=qh["dir"], a_r=g["a_r"], b_r=g["b_r"])
    cs = constants_with(p, **groups)
    nb = 1 << p.log2_buckets
    cells = np.zeros((p.L, nb) + oracle.tk_shape(p), dtype=np.uint32)
    cells[..., 0] = EMPTY
    cells[0, 21] = oracle.tk_sketch(p, cs, g["stream"])
    cells[1, 28] = oracle.tk_sketch(p, cs, q["s2_stream"])
    assert oracle.hash_rows(p, cs, *csr([qh["query_row"]]))[0].tolist() == [21, 28]
    oi, osc = oracle.tk_query(p, cs, cells, *csr([qh["query_row"]]), k=q["k"], k_max=q["k_max"])
    assert oi[0].tolist() == q["ids"] and osc[0].tolist() == q["scores"]


def test_one_cell_sketch_finds_a_strict_majority():
    # Boyer and Moore's majority vote: an element occurring more than n/2
    # times is the survivor, whatever the order
    p = oracle.Params(L=1, cm_rows=1, log2_cm_width=0, seed=3)
    cs = oracle.constants(p)
    rng = np.random.default_rng(5)
    for _ in range(300):
        n = int(rng.integers(1, 60))
        maj = int(rng.integers(0, 1000))
        m = n // 2 + 1
        others = rng.integers(0, 1000, size=n - m)
        others[others == maj] += 1000
        stream = np.concatenate([np.full(m, maj), others])
        rng.shuffle(stream)
        sk = oracle.tk_sketch(p, cs, stream)
        assert int(sk[0, 0, 0]) == maj and int(sk[0, 0, 1]) >= 1


@pytest.mark.parametrize("rows,lw", [(1, 0), (1, 3), (4, 4), (3, 6)])
def test_distinct_stream_closed_form(rows, lw):
    # With distinct ids the count of a cell alternates 1, 0, 1, ...: after n
    # ids a cell holds its last id with count 1 when n is odd, and its
    # second-to-last id with count 0 when n is even (none: EMPTY, 0).
    p = oracle.Params(L=1, cm_rows=rows, log2_cm_width=lw, seed=11)
    cs = oracle.constants(p)
    rng = np.random.default_rng(rows * 100 + lw)
    for _ in range(20):
        ids = rng.choice(1 << 30, size=int(rng.integers(0, 400)), replace=False)
        sk = oracle.tk_sketch(p, cs, ids)
        C = 1 << lw
        for r in range(rows):
            per = [[] for _ in range(C)]
            for x in ids.tolist():
                per[_row_hash(p, cs, r, x)].append(x)
            for c in range(C):
                s = per[c]
                want = (EMPTY, 0) if not s else ((s[-1], 1) if len(s) % 2 else (s[-2], 0))
                assert tuple(sk[r, c].tolist()) == want


def test_merge_identities():
    p = oracle.Params(L=1, cm_rows=3, log2_cm_width=3, seed=17)
    cs = oracle.constants(p)
    rng = np.random.default_rng(7)
    empty = oracle.tk_sketch(p, cs, [])
    for _ in range(50):
        a = oracle.tk_sketch(p, cs, rng.integers(0, 40, size=int(rng.integers(0, 80))))
        b = oracle.tk_sketch(p, cs, rng.integers(0, 40, size=int(rng.integers(0, 80))))
        assert (oracle.tk_merge(p, a, empty) == a).all()
        assert (oracle.tk_merge(p, empty, a) == a).all()
        assert (oracle.tk_merge(p, a, b) == oracle.tk_merge(p, b, a)).all()


@pytest.fixture(scope="module")
def small_tk():
    p = oracle.Params(dim=1 << 20, K=4, L=8, log2_buckets=6, R=1, cm_rows=2, log2_cm_width=3, seed=23)
    cs = oracle.constants(p)
    law = synth.RowLaw(synth.derive(29, synth.STREAM_DATA), 1 << 20)
    ip, ix = law.rows(0, 3000)
    return p, cs, law, ip, ix


def test_build_is_the_sketch_of_each_bucket_in_id_order(small_tk):
    p, cs, law, ip, ix = small_tk
    cells, seen = oracle.tk_build(p, cs, ip, ix)
    bk = oracle.hash_rows(p, cs, ip, ix)
    for t in range(p.L):
        for b in range(1 << p.log2_buckets):
            members = np.nonzero(bk[:, t] == b)[0]
            assert seen[t, b] == len(members)
            assert (cells[t, b] == oracle.tk_sketch(p, cs, members)).all()


def test_insert_in_batches_equals_bulk_build(small_tk):
    p, cs, law, ip, ix = small_tk
    want = oracle.tk_build(p, cs, ip, ix)
    n0 = 1000
    cells, seen = oracle.tk_build(p, cs, ip[: n0 + 1], ix[: ip[n0]])
    cur = n0
    for m in (1, 7, 500, 1492):
        oracle.tk_insert(p, cs, cells, seen, cur, ip[cur: cur + m + 1] - ip[cur], ix[ip[cur]: ip[cur + m]])
        cur += m
    assert cur == 3000
    assert (cells == want[0]).all() and (seen == want[1]).all()


def test_scores_never_exceed_exact_counts(small_tk):
    # a merged count only adds counts of the same id (each at most 1 per
    # bucket of distinct ids) or shrinks, so it is at most the id's number of
    # occurrences among the probed buckets' full member lists
    p, cs, law, ip, ix = small_tk
    cells, _ = oracle.tk_build(p, cs, ip, ix)
    bk = oracle.hash_rows(p, cs, ip, ix)
    qi, qx, src, _ = law.queries(synth.derive(29, synth.STREAM_QUERY), 3000, 0, 40)
    qb = oracle.hash_rows(p, cs, qi, qx)
    big = p.L * (p.cm_rows << p.log2_cm_width)
    oi, osc = oracle.tk_query(p, cs, cells, qi, qx, k=big, k_max=big)
    seen_any = False
    for q in range(len(qi) - 1):
        mult = {}
        for t in range(p.L):
            for x in np.nonzero(bk[:, t] == qb[q, t])[0].tolist():
                mult[x] = mult.get(x, 0) + 1
        for i, s in zip(oi[q].tolist(), osc[q].tolist()):
            if i == EMPTY:
                assert s == 0
                continue
            assert 1 <= s <= mult.get(i, 0)
            seen_any = True
        # output order: count desc, id asc, no repeated id
        live = [(s, i) for i, s in zip(oi[q].tolist(), osc[q].tolist()) if i != EMPTY]
        assert live == sorted(live, key=lambda v: (-v[0], v[1]))
        assert len({i for _, i in live}) == len(live)
    assert seen_any


def test_planted_duplicate_scores_all_tables_when_alone():
    # a bucket holding a single id keeps it with count 1; an exact copy of a
    # row whose buckets are all private then scores L
    p = oracle.Params(dim=1 << 20, K=4, L=6, log2_buckets=20, R=1, cm_rows=2, log2_cm_width=2, seed=31)
    cs = oracle.constants(p)
    law = synth.RowLaw(synth.derive(31, synth.STREAM_DATA), 1 << 20, index="uniform")
    ip, ix = law.rows(0, 200)
    cells, seen = oracle.tk_build(p, cs, ip, ix)
    bk = oracle.hash_rows(p, cs, ip, ix)
    hit = 0
    for r in range(200):
        if all(seen[t, bk[r, t]] == 1 for t in range(p.L)):
            oi, osc = oracle.tk_query(p, cs, cells, ip[r: r + 2] - ip[r], ix[ip[r]: ip[r + 1]], k=1)
            assert oi[0, 0] == r and osc[0, 0] == p.L
            hit += 1
    assert hit > 100
