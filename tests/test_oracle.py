"""Pins of the CPU oracle against things other than itself: hand-worked
examples, published generator outputs, closed forms, invariants, special cases
and brute force on tiny inputs."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle_util import constants_with, csr, h, load_golden, params_from

EMPTY = oracle.EMPTY


# ------------------------------------------------------------- constants


def test_splitmix64_published_outputs():
    # First outputs of SplitMix64 from state 0, as printed by the published
    # reference implementation (Steele, Lea, Flood 2014; Vigna's splitmix64.c).
    got = [int(x) for x in oracle.splitmix64_stream(0, 4)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F, 0xF88BB8A8724C81EC]


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_constant_draw_order(mode):
    # The whole table is one SplitMix64 stream consumed in the documented order.
    p = oracle.Params(dim=1000, K=3, L=5, log2_buckets=7, R=4, cm_rows=3, log2_cm_width=6,
                      hash_mode=mode, seed=987654321)
    cs = oracle.constants(p)
    lay = oracle.layout(p)
    st = [int(x) for x in oracle.splitmix64_stream(p.seed, lay["total"])]
    it = iter(st)
    n_h = p.M if mode == 2 else (p.L if mode else 1)
    for t in range(n_h):
        assert int(cs[lay["a_h"] + t]) == next(it) | 1
        assert int(cs[lay["b_h"] + t]) == next(it)
    for b in range(p.M):
        assert int(cs[lay["dir"] + b]) == next(it) >> 63
    for t in range(p.L):
        for j in range(p.K):
            assert int(cs[lay["a_tj"] + t * p.K + j]) == next(it) | 1
        assert int(cs[lay["b_t"] + t]) == next(it)
    for t in range(p.L):
        assert int(cs[lay["key_t"] + t]) == next(it) & 0xFFFFFFFF
        assert int(cs[lay["m1_t"] + t]) == (next(it) & 0xFFFFFFFF) | 1
        assert int(cs[lay["m2_t"] + t]) == (next(it) & 0xFFFFFFFF) | 1
    for r in range(p.cm_rows):
        assert int(cs[lay["a_r"] + r]) == next(it) | 1
        assert int(cs[lay["b_r"] + r]) == next(it)


def test_invalid_params_rejected():
    for bad in (dict(K=0), dict(L=0), dict(R=0), dict(log2_buckets=0), dict(log2_buckets=33),
                dict(cm_rows=0), dict(hash_mode=3), dict(dim=0)):
        p = oracle.Params(**bad)
        with pytest.raises(oracle.OracleError):
            oracle.constants(p)


# -------------------------------------------------------------- hashing


@pytest.mark.parametrize("case", range(4))
def test_doph_hand_worked(case):
    g = load_golden("doph_hand.json")
    p = params_from(g["params"])
    c = g["cases"][case]
    cs = constants_with(p, dir=c["dir"], **{k: v for k, v in g["constants"].items()})
    ip, ix = csr([c["row"]])
    bk, hv = oracle.hash_rows(p, cs, ip, ix, with_h=True)
    assert hv[0].tolist() == c["h"], c["name"]
    assert bk[0].tolist() == c["buckets"], c["name"]


def test_doph_hand_worked_per_table_mode():
    g = load_golden("doph_hand.json")
    p = params_from(g["params"])
    p.hash_mode = 1
    m1 = g["mode1"]
    groups = dict(g["constants"])
    groups.update(a_h=m1["a_h"], b_h=m1["b_h"], dir=m1["dir"])
    cs = constants_with(p, **groups)
    ip, ix = csr([m1["row"]])
    bk, hv = oracle.hash_rows(p, cs, ip, ix, with_h=True)
    assert hv[0].tolist() == m1["h"]
    assert bk[0].tolist() == m1["buckets"]


def test_classic_minhash_hand_worked():
    # hash_mode 2: M independent MinHash functions (Section 2.2 MinHash with
    # the L x K seeds of Section 4 "Initialization"), no bins, no
    # densification; the fixture derives every value by hand
    g = load_golden("doph_hand.json")
    p = params_from(g["params"])
    p.hash_mode = 2
    m2 = g["mode2"]
    groups = dict(g["constants"])
    groups.update(a_h=m2["a_h"], b_h=m2["b_h"], dir=m2["dir"])
    cs = constants_with(p, **groups)
    for c in m2["cases"]:
        ip, ix = csr([c["row"]])
        bk, hv = oracle.hash_rows(p, cs, ip, ix, with_h=True)
        assert hv[0].tolist() == c["h"], c["name"]
        assert bk[0].tolist() == c["buckets"], c["name"]


def test_classic_minhash_collision_rate_is_jaccard():
    # Section 2.2: Pr[min of x = min of y under a random permutation] is the
    # Jaccard similarity; every one of the M functions is such a MinHash.
    rng = np.random.default_rng(7)
    x, y = _jaccard_pairs(rng, 1 << 20, 24, 8)  # J = 24 / 40 = 0.6
    hits = tot = 0
    for seed in range(200):
        p = oracle.Params(dim=1 << 20, K=4, L=8, log2_buckets=16, hash_mode=2, seed=seed)
        _, hv = oracle.hash_rows(p, oracle.constants(p), *csr([x, y]), with_h=True)
        hits += int((hv[0] == hv[1]).sum())
        tot += p.M
    assert abs(hits / tot - 0.6) < 0.03, hits / tot


def test_classic_minhash_functions_are_row_minima():
    # each value is the minimum over the row of what the row's single
    # elements hash to under the same function
    p = oracle.Params(dim=5000, K=3, L=2, log2_buckets=20, hash_mode=2, seed=13)
    cs = oracle.constants(p)
    rng = np.random.default_rng(8)
    rows = _rand_rows(rng, 30, p.dim)
    singles = sorted({v for r in rows for v in r})
    _, hs = oracle.hash_rows(p, cs, *csr([[v] for v in singles]), with_h=True)
    u = {v: hs[i] for i, v in enumerate(singles)}
    _, hv = oracle.hash_rows(p, cs, *csr(rows), with_h=True)
    for r, vals in zip(rows, hv):
        assert vals.tolist() == np.min(np.stack([u[i] for i in r]), axis=0).tolist()


def test_classic_minhash_single_function_is_one_bin_doph():
    # with K = L = 1 both families hash with the same first constant pair and
    # keep the row minimum, so they agree
    rng = np.random.default_rng(9)
    rows = _rand_rows(rng, 50, 1 << 20)
    out = []
    for mode in (0, 2):
        p = oracle.Params(dim=1 << 20, K=1, L=1, log2_buckets=12, hash_mode=mode, seed=17)
        out.append(oracle.hash_rows(p, oracle.constants(p), *csr(rows)))
    assert (out[0] == out[1]).all()


def _rand_rows(rng, n, dim, lo=1, hi=60):
    return [rng.choice(dim, size=rng.integers(lo, hi + 1), replace=False).tolist() for _ in range(n)]


def test_single_bin_is_textbook_minhash():
    # M = 1: the one DOPH value of a row is min over its elements of u(i), and
    # u(i) is what a one-element row hashes to (Section 2.2, MinHash).
    p = oracle.Params(dim=5000, K=1, L=1, log2_buckets=20, R=4, seed=11)
    cs = oracle.constants(p)
    rng = np.random.default_rng(0)
    rows = _rand_rows(rng, 50, p.dim)
    singles = sorted({v for r in rows for v in r})
    ip, ix = csr([[v] for v in singles])
    _, hs = oracle.hash_rows(p, cs, ip, ix, with_h=True)
    u = dict(zip(singles, hs[:, 0].tolist()))
    ip, ix = csr(rows)
    _, hv = oracle.hash_rows(p, cs, ip, ix, with_h=True)
    for r, v in zip(rows, hv[:, 0].tolist()):
        assert v == min(u[i] for i in r)


def test_doph_is_min_over_elements_bin_by_bin():
    # Without empty bins (a row covering every bin) the DOPH value of each bin
    # is the minimum of the one-element values that land in that bin; a
    # one-element row puts its value in every bin, so its bin is found by
    # hashing it together with an element known to sit elsewhere.
    p = oracle.Params(dim=1 << 16, K=2, L=2, log2_buckets=20, R=4, seed=5)
    cs = oracle.constants(p)
    rng = np.random.default_rng(1)
    elems = rng.choice(p.dim, size=400, replace=False).tolist()
    ip, ix = csr([[v] for v in elems])
    _, hs = oracle.hash_rows(p, cs, ip, ix, with_h=True)
    u = {v: int(hs[i, 0]) for i, v in enumerate(elems)}
    # the bin of a value: M equal ranges of [0, 2^32)
    binof = {v: (u[v] * p.M) >> 32 for v in elems}
    row = elems
    ip, ix = csr([row])
    _, hv = oracle.hash_rows(p, cs, ip, ix, with_h=True)
    for b in range(p.M):
        members = [u[v] for v in row if binof[v] == b]
        assert members, "row must cover every bin"
        assert hv[0, b] == min(members)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_hash_invariant_to_order_and_duplicates(mode):
    p = oracle.Params(dim=1 << 20, K=4, L=8, log2_buckets=16, hash_mode=mode, seed=3)
    cs = oracle.constants(p)
    rng = np.random.default_rng(2)
    rows = _rand_rows(rng, 40, p.dim)
    perm = [list(rng.permutation(r)) + list(rng.choice(r, size=3)) for r in rows]
    a = oracle.hash_rows(p, cs, *csr(rows))
    b = oracle.hash_rows(p, cs, *csr(perm))
    assert (a == b).all()


@pytest.mark.parametrize("mode", [0, 1])
def test_single_nonzero_fills_all_bins(mode):
    p = oracle.Params(dim=1 << 20, K=4, L=8, log2_buckets=16, hash_mode=mode, seed=4)
    cs = oracle.constants(p)
    ip, ix = csr([[123456], [7]])
    _, hv = oracle.hash_rows(p, cs, ip, ix, with_h=True)
    if mode == 0:
        assert (hv[0] == hv[0, 0]).all() and (hv[1] == hv[1, 0]).all()
    else:
        for t in range(p.L):
            assert (hv[0, t * p.K:(t + 1) * p.K] == hv[0, t * p.K]).all()


def test_invalid_rows_rejected():
    p = oracle.Params(dim=100, K=2, L=2, log2_buckets=8, seed=1)
    cs = oracle.constants(p)
    for rows in ([[]], [[100]], [[-1]], [[3, 200]]):
        with pytest.raises(oracle.OracleError):
            oracle.hash_rows(p, cs, *csr(rows))


def _jaccard_pairs(rng, dim, n_inter, n_only):
    base = rng.choice(dim, size=n_inter + 2 * n_only, replace=False)
    x = base[: n_inter + n_only]
    y = np.concatenate([base[:n_inter], base[n_inter + n_only:]])
    return x.tolist(), y.tolist()


def test_doph_bin_collision_rate_is_jaccard():
    # Section 2.2 (MinHash collision probability = Jaccard similarity, the
    # formula read with |x| + |y| - x.y in the denominator); DOPH keeps this
    # per bin.  Averaged over seeds, within a binomial-scale tolerance.
    rng = np.random.default_rng(3)
    x, y = _jaccard_pairs(rng, 1 << 20, 24, 8)  # J = 24 / 40 = 0.6
    J = 24 / 40
    hits = tot = 0
    for seed in range(300):
        p = oracle.Params(dim=1 << 20, K=4, L=8, log2_buckets=16, seed=seed)
        cs = oracle.constants(p)
        _, hv = oracle.hash_rows(p, cs, *csr([x, y]), with_h=True)
        hits += int((hv[0] == hv[1]).sum())
        tot += p.M
    rate = hits / tot
    # bins of one seed are dependent; 300 independent seeds give sd <= ~0.03
    assert abs(rate - J) < 0.05, rate


def test_bucket_collision_bounds():
    # Per table, similar pairs collide far more often than dissimilar ones;
    # identical rows always collide; disjoint rows collide only by accident.
    rng = np.random.default_rng(4)
    near = _jaccard_pairs(rng, 1 << 20, 36, 4)   # J = 0.8
    far = _jaccard_pairs(rng, 1 << 20, 4, 36)    # J = 0.05
    dis = _jaccard_pairs(rng, 1 << 20, 0, 40)
    rates = {}
    for name, (x, y) in dict(near=near, far=far, dis=dis).items():
        hit = tot = 0
        for seed in range(100):
            p = oracle.Params(dim=1 << 20, K=4, L=16, log2_buckets=20, seed=seed)
            cs = oracle.constants(p)
            bk = oracle.hash_rows(p, cs, *csr([x, y, x]))
            assert (bk[0] == bk[2]).all()
            hit += int((bk[0] == bk[1]).sum())
            tot += p.L
        rates[name] = hit / tot
    assert rates["near"] >= 0.8 ** 4 - 0.05
    assert rates["far"] < 0.1
    assert rates["dis"] < 0.01


# ------------------------------------------------------------ priorities


def test_priority_hand_worked():
    g = load_golden("priority_hand.json")
    p = oracle.Params(L=1, seed=0)
    for c in g["cases"]:
        cs = constants_with(p, key_t=[c["key"]], m1_t=[c["m1"]], m2_t=[c["m2"]])
        assert oracle.priorities(p, cs, 0, [h(c["id"])])[0] == h(c["p"]), c["why"]


def _inverse_priority(p_vals, key, m1, m2):
    # invert x ^= x >> 15, x *= m2, x ^= x >> 16, x *= m1, x ^= key
    M = 1 << 32
    x = p_vals.astype(np.uint64)
    x = x ^ (x >> np.uint64(15)) ^ (x >> np.uint64(30))
    x = (x * np.uint64(pow(m2, -1, M))) % np.uint64(M)
    x = x ^ (x >> np.uint64(16))
    x = (x * np.uint64(pow(m1, -1, M))) % np.uint64(M)
    return (x ^ np.uint64(key)).astype(np.uint32)


def test_priority_is_a_bijection():
    p = oracle.Params(L=3, seed=77)
    cs = oracle.constants(p)
    lay = oracle.layout(p)
    rng = np.random.default_rng(5)
    ids = rng.integers(0, 2**32, size=200000, dtype=np.uint64).astype(np.uint32)
    for t in range(p.L):
        pv = oracle.priorities(p, cs, t, ids)
        back = _inverse_priority(pv, int(cs[lay["key_t"] + t]), int(cs[lay["m1_t"] + t]),
                                 int(cs[lay["m2_t"] + t]))
        assert (back == ids).all()
    dense = np.arange(1 << 22, dtype=np.uint32)
    assert len(np.unique(oracle.priorities(p, cs, 1, dense))) == len(dense)


# ----------------------------------------------------------------- build


def _data(n, seed=9, dim=1 << 20):
    law = synth.RowLaw(synth.derive(seed, synth.STREAM_DATA), dim)
    return law, law.rows(0, n)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_build_matches_brute_force(mode):
    p = oracle.Params(dim=1 << 20, K=2, L=4, log2_buckets=5, R=6, hash_mode=mode, seed=21)
    cs = oracle.constants(p)
    _, (ip, ix) = _data(700)
    ids, seen = oracle.build(p, cs, ip, ix)
    bk = oracle.hash_rows(p, cs, ip, ix)
    for t in range(p.L):
        assert seen[t].sum() == 700
        for b in range(1 << p.log2_buckets):
            members = np.nonzero(bk[:, t] == b)[0].astype(np.uint32)
            assert seen[t, b] == len(members)
            pri = oracle.priorities(p, cs, t, members)
            want = members[np.argsort(pri, kind="stable")][: p.R].tolist()
            got = ids[t, b]
            f = min(p.R, len(members))
            assert got[:f].tolist() == want
            assert (got[f:] == EMPTY).all()


def test_reservoir_keeps_everything_when_light():
    p = oracle.Params(dim=1 << 20, K=4, L=4, log2_buckets=12, R=64, seed=2)
    cs = oracle.constants(p)
    _, (ip, ix) = _data(2000)
    ids, seen = oracle.build(p, cs, ip, ix)
    bk = oracle.hash_rows(p, cs, ip, ix)
    for t in range(p.L):
        light = np.nonzero((seen[t] > 0) & (seen[t] <= p.R))[0]
        for b in light[:200]:
            assert sorted(ids[t, b, : seen[t, b]].tolist()) == np.nonzero(bk[:, t] == b)[0].tolist()


def test_insert_equals_bulk_build():
    # The kept set is the bottom-R by priority, so streaming insertion in any
    # batch split equals one bulk build on the union (Section 3.1 streaming
    # insert; Algorithm 1).
    p = oracle.Params(dim=1 << 20, K=4, L=6, log2_buckets=6, R=8, seed=31)
    cs = oracle.constants(p)
    _, (ip, ix) = _data(1500)
    full_ids, full_seen = oracle.build(p, cs, ip, ix)
    n0 = 600
    ids, seen = oracle.build(p, cs, ip[: n0 + 1], ix[: ip[n0]])
    rng = np.random.default_rng(6)
    cur = n0
    while cur < 1500:
        m = int(min(1500 - cur, rng.integers(1, 200)))
        sub_ip = ip[cur: cur + m + 1] - ip[cur]
        sub_ix = ix[ip[cur]: ip[cur + m]]
        oracle.insert(p, cs, ids, seen, cur, sub_ip, sub_ix)
        cur += m
    assert (ids == full_ids).all() and (seen == full_seen).all()


def test_insert_rejects_bad_rows_without_change():
    p = oracle.Params(dim=100, K=2, L=2, log2_buckets=4, R=3, seed=1)
    cs = oracle.constants(p)
    ip, ix = csr([[1, 2], [3, 4]])
    ids, seen = oracle.build(p, cs, ip, ix)
    before = ids.copy(), seen.copy()
    with pytest.raises(oracle.OracleError):
        oracle.insert(p, cs, ids, seen, 2, *csr([[5], [500]]))
    assert (ids == before[0]).all() and (seen == before[1]).all()


# ----------------------------------------------------------------- query


def _tables_from(g, p):
    nb = 1 << p.log2_buckets
    ids = np.full((p.L, nb, p.R), EMPTY, dtype=np.uint32)
    seen = np.zeros((p.L, nb), dtype=np.uint32)
    for e in g["tables"]["entries"]:
        ids[e["t"], e["b"]] = e["ids"]
        seen[e["t"], e["b"]] = e["seen"]
    return ids, seen


@pytest.mark.parametrize("variant", ["one_row", "two_rows", "exact"])
def test_query_hand_worked(variant):
    g = load_golden("query_hand.json")
    d = load_golden("doph_hand.json")
    p = params_from(d["params"])
    v = g[variant] if variant != "exact" else g["one_row"]
    p.cm_rows = len(v["a_r"])
    groups = dict(d["constants"])
    groups.update(dir=g["dir"], a_r=v["a_r"], b_r=v["b_r"])
    cs = constants_with(p, **groups)
    ids, seen = _tables_from(g, p)
    oi, osc = oracle.query(p, cs, ids, seen, *csr([g["query_row"]]), k=g["k"], k_max=g["k_max"],
                           exact=(variant == "exact"))
    want = g[variant]
    assert oi[0].tolist() == want["ids"] and osc[0].tolist() == want["scores"]


def _candidates(p, cs, ids, seen, row):
    bk = oracle.hash_rows(p, cs, *csr([row]))[0]
    c = []
    for t in range(p.L):
        f = min(p.R, int(seen[t, bk[t]]))
        c += ids[t, bk[t], :f].tolist()
    return c


@pytest.fixture(scope="module")
def small_index():
    p = oracle.Params(dim=1 << 20, K=4, L=16, log2_buckets=10, R=16, cm_rows=2,
                      log2_cm_width=6, seed=41)
    cs = oracle.constants(p)
    law, (ip, ix) = _data(20000, seed=13)
    ids, seen = oracle.build(p, cs, ip, ix)
    qi, qx, src, _ = law.queries(synth.derive(13, synth.STREAM_QUERY), 20000, 0, 60)
    return p, cs, ids, seen, qi, qx, src


def test_countmin_never_underestimates(small_index):
    p, cs, ids, seen, qi, qx, _ = small_index
    big = p.L * p.R
    oi, osc = oracle.query(p, cs, ids, seen, qi, qx, k=big, k_max=big)
    for q in range(len(qi) - 1):
        row = qx[qi[q]:qi[q + 1]].tolist()
        cnt = {}
        for c in _candidates(p, cs, ids, seen, row):
            cnt[c] = cnt.get(c, 0) + 1
        live = oi[q] != EMPTY
        assert sorted(oi[q][live].tolist()) == sorted(cnt)
        for i, s in zip(oi[q][live].tolist(), osc[q][live].tolist()):
            assert s >= cnt[i]
        # order: estimate desc, then id asc
        pairs = list(zip((-osc[q][live]).tolist(), oi[q][live].tolist()))
        assert pairs == sorted(pairs)


def test_exact_counting_brute_force(small_index):
    p, cs, ids, seen, qi, qx, _ = small_index
    oi, osc = oracle.query(p, cs, ids, seen, qi, qx, k=10, k_max=12, exact=True)
    for q in range(len(qi) - 1):
        cnt = {}
        for c in _candidates(p, cs, ids, seen, qx[qi[q]:qi[q + 1]].tolist()):
            cnt[c] = cnt.get(c, 0) + 1
        want = sorted(cnt.items(), key=lambda kv: (-kv[1], kv[0]))[:10]
        n = len(want)
        assert oi[q, :n].tolist() == [a for a, _ in want]
        assert osc[q, :n].tolist() == [b for _, b in want]
        assert (oi[q, n:] == EMPTY).all() and (osc[q, n:] == 0).all()


def test_identity_row_hash_gives_exact_counts(small_index):
    # Count-min with a collision-free row hash counts exactly: a = 2^(64-lw),
    # b = 0 gives g(c) = c mod w, injective when w exceeds every id.
    p0, cs0, ids, seen, qi, qx, _ = small_index
    p = oracle.Params(**{**p0.__dict__, "cm_rows": 1, "log2_cm_width": 16})
    cs = constants_with(p, a_r=[hex(1 << 48)], b_r=["0x0"])
    lay0, lay = oracle.layout(p0), oracle.layout(p)
    cs[: lay["a_r"]] = cs0[: lay0["a_r"]]
    a = oracle.query(p, cs, ids, seen, qi, qx, k=10)
    b = oracle.query(p, cs, ids, seen, qi, qx, k=10, exact=True)
    assert (a[0] == b[0]).all() and (a[1] == b[1]).all()


def test_one_counter_ranks_by_id(small_index):
    # d = 1, w = 1: every estimate equals |C|, so the top-k are the k smallest
    # distinct candidate ids.
    p0, cs0, ids, seen, qi, qx, _ = small_index
    p = oracle.Params(**{**p0.__dict__, "cm_rows": 1, "log2_cm_width": 0})
    cs = oracle.constants(p)
    lay0, lay = oracle.layout(p0), oracle.layout(p)
    cs[: lay["a_r"]] = cs0[: lay0["a_r"]]
    oi, osc = oracle.query(p, cs, ids, seen, qi, qx, k=5)
    for q in range(len(qi) - 1):
        c = _candidates(p, cs, ids, seen, qx[qi[q]:qi[q + 1]].tolist())
        want = sorted(set(c))[:5]
        assert oi[q, : len(want)].tolist() == want
        assert (osc[q, : len(want)] == len(c)).all()


def test_topk_prefix_and_per_query_k(small_index):
    p, cs, ids, seen, qi, qx, _ = small_index
    a, sa = oracle.query(p, cs, ids, seen, qi, qx, k=20)
    ks = np.array([1, 10, 20, 3] * 15, dtype=np.uint32)
    b, sb = oracle.query(p, cs, ids, seen, qi, qx, k=0, k_max=20, kq=ks)
    for q, k in enumerate(ks):
        assert (b[q, :k] == a[q, :k]).all() and (sb[q, :k] == sa[q, :k]).all()
        assert (b[q, k:] == EMPTY).all() and (sb[q, k:] == 0).all()
    with pytest.raises(oracle.OracleError):
        oracle.query(p, cs, ids, seen, qi, qx, k=30, k_max=20)


def test_planted_duplicate_found_at_rank_one():
    # Near-duplicate corollary (Section 5): with no sub-sampling (R >= N) and
    # exact counting, a dataset point queried as itself collides in all L
    # tables, so it ranks first with score L unless a smaller id shares all
    # L buckets.
    p = oracle.Params(dim=1 << 20, K=4, L=8, log2_buckets=12, R=512, seed=51)
    cs = oracle.constants(p)
    _, (ip, ix) = _data(500, seed=17)
    ids, seen = oracle.build(p, cs, ip, ix)
    bk = oracle.hash_rows(p, cs, ip, ix)
    oi, osc = oracle.query(p, cs, ids, seen, ip, ix, k=1, exact=True)
    for x in range(500):
        twins = np.nonzero((bk == bk[x]).all(axis=1))[0]
        assert oi[x, 0] == twins.min() and osc[x, 0] == p.L


def test_recall_at_10_on_tiny_config():
    # recall@10 of the planted neighbour on the tiny configuration (N = 1e5,
    # K=4, L=16, 2^16 buckets, R=32, count-min 4 x 1024, f = 0.2).
    p = oracle.Params(dim=1 << 20, K=4, L=16, log2_buckets=16, R=32, cm_rows=4,
                      log2_cm_width=10, seed=synth.derive(2020, synth.STREAM_INDEX))
    cs = oracle.constants(p)
    law = synth.RowLaw(synth.derive(2020, synth.STREAM_DATA), 1 << 20)
    ip, ix = law.rows(0, 100000)
    qi, qx, src, _ = law.queries(synth.derive(2020, synth.STREAM_QUERY), 100000, 0, 400)
    ids, seen = oracle.build(p, cs, ip, ix)
    oi, _ = oracle.query(p, cs, ids, seen, qi, qx, k=10)
    recall = np.mean([s in row for s, row in zip(src.tolist(), oi.tolist())])
    assert recall >= 0.9, recall


@pytest.mark.parametrize("variant", ["one_row", "two_rows", "exact"])
def test_aggregate_hand_worked(variant):
    # the aggregation step alone, on the hand fixture's candidate multiset
    g = load_golden("query_hand.json")
    d = load_golden("doph_hand.json")
    p = params_from(d["params"])
    v = g[variant] if variant != "exact" else g["one_row"]
    p.cm_rows = len(v["a_r"])
    cs = constants_with(p, a_r=v["a_r"], b_r=v["b_r"])
    oi, osc = oracle.aggregate(p, cs, [10, 11, 12, 11, 14], k=g["k"], k_max=g["k_max"],
                               exact=(variant == "exact"))
    want = g[variant]
    assert oi.tolist() == want["ids"] and osc.tolist() == want["scores"]
