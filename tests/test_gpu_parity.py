"""GPU parity: the HIP path through the C ABI against the CPU oracle, element
by element (bucket ids, every reservoir slot and seen count, every top-k id
and score).  All integer, so the bar is bit-exact."""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EMPTY = 0xFFFFFFFF


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2008_03260_amd import api as a
    a.lib()
    return a


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def u32(t):
    return t.detach().cpu().numpy().view(np.uint32)


def params_pair(api, k_max=10, **kw):
    base = dict(dim=1 << 20, K=4, L=8, log2_buckets=10, R=16, cm_rows=4, log2_cm_width=10, hash_mode=0, seed=99)
    base.update(kw)
    return api.Params.of(k_max=k_max, **base), oracle.Params(**base)


def rows_of(n, seed=1, dim=1 << 20, **law):
    lw = synth.RowLaw(synth.derive(seed, synth.STREAM_DATA), dim, **law)
    return lw, lw.rows(0, n)


def csr_from_lists(rows):
    ip = np.zeros(len(rows) + 1, dtype=np.int64)
    for i, r in enumerate(rows):
        ip[i + 1] = ip[i] + len(r)
    return ip, np.array([v for r in rows for v in r], dtype=np.int32)


# ------------------------------------------------------------------ hash


HASH_SHAPES = [
    dict(K=4, L=16, hash_mode=0),           # M = 64 (tiny configuration)
    dict(K=4, L=32, hash_mode=0),           # M = 128 (200M-point shard)
    dict(K=3, L=7, hash_mode=0),            # M = 21, not a power of two
    dict(K=8, L=128, log2_buckets=18),      # M = 1024 (wide configuration)
    dict(K=1, L=1, hash_mode=0),            # M = 1, textbook MinHash
    dict(K=4, L=16, hash_mode=1),           # per-table DOPH
    dict(K=5, L=3, hash_mode=1),
    dict(K=64, L=64, log2_buckets=12),      # M = 4096, the largest
    dict(K=4, L=16, hash_mode=2),           # classic MinHash, 64 functions
    dict(K=3, L=7, hash_mode=2),
    dict(K=16, L=64, log2_buckets=12, hash_mode=2),  # 1024 functions, constants in global memory
]


@pytest.mark.parametrize("shape", HASH_SHAPES, ids=lambda s: "-".join(f"{k}{v}" for k, v in s.items()))
def test_hash_parity(api, shape):
    gp, op = params_pair(api, **shape)
    _, (ip, ix) = rows_of(3000, seed=3)
    # edge rows: single nonzero, repeats, long rows, extreme indices
    extra = [[0], [(1 << 20) - 1], [5, 5, 5], list(range(0, 3000, 3)), [7, 1 << 19, 7, 3]]
    eip, eix = csr_from_lists(extra)
    ip = np.concatenate([ip, ip[-1] + eip[1:]])
    ix = np.concatenate([ix, eix])
    idx = api.Index(gp, dev(ip[:2]), dev(ix[: ip[1]]))
    got = u32(idx.hash(dev(ip), dev(ix)))
    cs = oracle.constants(op)
    want = oracle.hash_rows(op, cs, ip, ix)
    assert (got == want).all(), np.argwhere(got != want)[:5]


# ----------------------------------------------------------------- build


def check_tables(api, idx, op, cs, ip, ix):
    gi, gsn = idx.tables()
    wi, wsn = oracle.build(op, cs, ip, ix)
    gi, gsn = u32(gi), u32(gsn)
    assert (gsn == wsn).all(), np.argwhere(gsn != wsn)[:5]
    bad = np.argwhere(gi != wi)
    assert len(bad) == 0, bad[:5]


# bucket bits choose the sort's passes: 3 (one pass), 8 (one full pass), 10
# and 12 (two), 17 and 20 (three, the last of 1 and 4 bits); 22 bits take the
# general key-value sort and the separate scan for bucket runs
@pytest.mark.parametrize("shape", [dict(), dict(L=16, log2_buckets=12, R=32), dict(K=2, L=5, log2_buckets=3, R=7),
                                   dict(hash_mode=1, L=6), dict(hash_mode=2, L=6), dict(R=1),
                                   dict(R=130, log2_buckets=6), dict(L=4, log2_buckets=8),
                                   dict(L=3, log2_buckets=17, R=4), dict(L=4, log2_buckets=20, R=8),
                                   dict(L=2, log2_buckets=22, R=4)],
                         ids=["base", "wide", "tiny-buckets", "mode1", "mode2", "R1", "R130", "B8", "B17", "B20",
                              "B22-general-sort"])
def test_build_parity(api, shape):
    gp, op = params_pair(api, **shape)
    _, (ip, ix) = rows_of(20000, seed=5)
    idx = api.Index(gp, dev(ip), dev(ix))
    check_tables(api, idx, op, oracle.constants(op), ip, ix)
    assert idx.info()["n_items"] == 20000


def test_build_heavy_buckets(api):
    # identical rows pile into one bucket per table: 40000 > one wave's share,
    # so the chunked bottom-R reduction runs (two rounds)
    gp, op = params_pair(api, L=4, R=24)
    _, (ip0, ix0) = rows_of(3000, seed=6)
    dup = [[11, 22, 33, 44]] * 40000
    dip, dix = csr_from_lists(dup)
    ip = np.concatenate([ip0, ip0[-1] + dip[1:]])
    ix = np.concatenate([ix0, dix])
    idx = api.Index(gp, dev(ip), dev(ix))
    check_tables(api, idx, op, oracle.constants(op), ip, ix)


@pytest.mark.parametrize("R", [37, 64, 100])
def test_build_bucket_sizes_at_select_boundaries(api, R):
    # groups of identical rows fill one bucket per table with exactly n ids:
    # sizes on either side of every select path's limit (the register path
    # for 64, 128, 256 and 512 ids, the streaming list, the chunked heavy path above
    # 16384 ids), with random rows around them
    sizes = [1, 37, 63, 64, 65, 100, 127, 128, 129, 255, 256, 257, 511, 512, 513, 16384, 16385]
    gp, op = params_pair(api, L=4, log2_buckets=14, R=R)
    _, (ip0, ix0) = rows_of(2000, seed=12)
    groups = []
    for g, n in enumerate(sizes):
        groups += [[5000 + 16 * g + j for j in range(5)]] * n
    gip, gix = csr_from_lists(groups)
    ip = np.concatenate([ip0, ip0[-1] + gip[1:]])
    ix = np.concatenate([ix0, gix])
    idx = api.Index(gp, dev(ip), dev(ix))
    check_tables(api, idx, op, oracle.constants(op), ip, ix)


def test_build_ragged_and_tiny(api):
    for n in (1, 2, 63, 64, 65, 4097):
        gp, op = params_pair(api, L=3, log2_buckets=4, R=5)
        _, (ip, ix) = rows_of(n, seed=10 + n)
        idx = api.Index(gp, dev(ip), dev(ix))
        check_tables(api, idx, op, oracle.constants(op), ip, ix)


def test_build_empty_index(api):
    gp, op = params_pair(api, L=2, log2_buckets=3, R=2)
    idx = api.Index(gp, dev(np.zeros(1, dtype=np.int64)), dev(np.zeros(1, dtype=np.int32)))
    gi, gsn = idx.tables()
    assert (u32(gi) == EMPTY).all() and (u32(gsn) == 0).all()


def test_insert_equals_bulk_build(api):
    gp, op = params_pair(api, L=6, log2_buckets=8, R=8)
    _, (ip, ix) = rows_of(9000, seed=8)
    n0 = 3000
    idx = api.Index(gp, dev(ip[: n0 + 1]), dev(ix[: ip[n0]]))
    rng = np.random.default_rng(0)
    cur = n0
    while cur < 9000:
        m = int(min(9000 - cur, rng.integers(1, 1500)))
        sip = ip[cur: cur + m + 1] - ip[cur]
        six = ix[ip[cur]: ip[cur + m]]
        nid = torch.empty(m, dtype=torch.int32, device="cuda")
        idx.insert(dev(sip), dev(six), new_ids=nid)
        assert (u32(nid) == np.arange(cur, cur + m)).all()
        cur += m
    torch.cuda.synchronize()
    check_tables(api, idx, op, oracle.constants(op), ip, ix)
    assert idx.info()["n_items"] == 9000


@pytest.mark.parametrize("R", [1, 16, 24, 64, 100, 128, 256])
def test_insert_small_batches_by_reservoir_size(api, R):
    # batches of at most 4096 rows are grouped by bucket in LDS and merged by
    # sixteen lanes per bucket holding the reservoir in registers (1 to 16
    # entries per lane); one batch carries 2000 identical rows, so every table
    # gets a run of 2000 ids in one bucket
    gp, op = params_pair(api, L=3, log2_buckets=6, R=R)
    _, (ip0, ix0) = rows_of(9000, seed=21)
    dip, dix = csr_from_lists([[11, 22, 33, 44]] * 2000)
    n0 = 3000
    # rows: [0, 3000) base, then batches of 1, 4096 (with the 2000 duplicates
    # in the middle), 17 and 4096 - 2000 + ... rows
    parts = [(ip0[: n0 + 1], ix0[: ip0[n0]])]
    cur = n0
    for m in (1, 1000):
        parts.append((ip0[cur: cur + m + 1] - ip0[cur], ix0[ip0[cur]: ip0[cur + m]]))
        cur += m
    parts.append((dip, dix))
    for m in (1096, 17, 3886):
        parts.append((ip0[cur: cur + m + 1] - ip0[cur], ix0[ip0[cur]: ip0[cur + m]]))
        cur += m
    ips, ixs, off = [np.zeros(1, np.int64)], [], 0
    for pi, px in parts:
        ips.append(pi[1:] + off)
        ixs.append(px)
        off += int(pi[-1])
    ip, ix = np.concatenate(ips), np.concatenate(ixs)
    idx = api.Index(gp, dev(ip[: n0 + 1]), dev(ix[: ip[n0]]))
    # insert batches: 1 row, then 1000 + 2000 duplicates + 1096 = 4096 rows,
    # then 17, then 3886
    bounds = [n0, n0 + 1, n0 + 1 + 4096, n0 + 1 + 4096 + 17, len(ip) - 1]
    for a, b in zip(bounds[:-1], bounds[1:]):
        idx.insert(dev(ip[a: b + 1] - ip[a]), dev(ix[ip[a]: ip[b]]))
    torch.cuda.synchronize()
    check_tables(api, idx, op, oracle.constants(op), ip, ix)
    assert idx.info()["n_items"] == len(ip) - 1


def test_tables_export_import_roundtrip(api):
    # an index restored from its exported tables answers and grows exactly
    # like the original
    gp, op = params_pair(api, L=6, log2_buckets=8, R=12)
    law, (ip, ix) = rows_of(6000, seed=17)
    a = api.Index(gp, dev(ip[:5001]), dev(ix[: ip[5000]]))
    ids, seen = a.tables()
    b = api.Index.from_tables(gp, ids.clone(), seen.clone(), 5000)
    assert b.info()["n_items"] == 5000
    tail = (dev(ip[5000:] - ip[5000]), dev(ix[ip[5000]:]))
    a.insert(*tail)
    b.insert(*tail)
    torch.cuda.synchronize()
    for x, y in zip(a.tables(), b.tables()):
        assert torch.equal(x, y)
    check_tables(api, b, op, oracle.constants(op), ip, ix)
    qi, qx, _, _ = law.queries(synth.derive(17, synth.STREAM_QUERY), 6000, 0, 50)
    ra, rb = a.query(dev(qi), dev(qx), 10), b.query(dev(qi), dev(qx), 10)
    assert torch.equal(ra[0], rb[0]) and torch.equal(ra[1], rb[1])
    with pytest.raises(api.SlashError):
        api.Index.from_tables(gp, ids, seen, 2**32)


def test_invalid_rows_rejected(api):
    gp, op = params_pair(api, dim=1000, L=2, log2_buckets=4, R=3)
    for rows in ([[1, 2], []], [[1, 2], [1000]], [[-3]]):
        ip, ix = csr_from_lists(rows)
        with pytest.raises(api.SlashError) as e:
            api.Index(gp, dev(ip), dev(ix))
        assert e.value.code == api.E_INVAL
    ip, ix = csr_from_lists([[1, 2], [3]])
    idx = api.Index(gp, dev(ip), dev(ix))
    before = [u32(t).copy() for t in idx.tables()]
    bip, bix = csr_from_lists([[4], [5000]])
    with pytest.raises(api.SlashError):
        idx.insert(dev(bip), dev(bix))
    after = [u32(t) for t in idx.tables()]
    assert all((a == b).all() for a, b in zip(before, after))
    assert idx.info()["n_items"] == 2


def test_invalid_params_rejected(api):
    ip, ix = csr_from_lists([[1]])
    for bad in (dict(K=0), dict(L=0), dict(R=0), dict(log2_buckets=0), dict(log2_buckets=31), dict(k_max=0),
                dict(hash_mode=3), dict(cm_rows=0), dict(log2_cm_width=17)):
        gp, _ = params_pair(api, **bad)
        with pytest.raises(api.SlashError) as e:
            api.Index(gp, dev(ip), dev(ix))
        assert e.value.code in (api.E_INVAL, api.E_UNSUPPORTED)


# ----------------------------------------------------------------- query


@pytest.fixture(scope="module")
def qsetup(api):
    gp, op = params_pair(api, k_max=24, L=16, log2_buckets=12, R=16, cm_rows=3, log2_cm_width=8)
    law, (ip, ix) = rows_of(30000, seed=21)
    qi, qx, src, _ = law.queries(synth.derive(21, synth.STREAM_QUERY), 30000, 0, 300, nnz_mode="lognormal",
                                 median=40, sigma=1.0, lo=1, hi=2000, f=(0.1, 0.4))
    idx = api.Index(gp, dev(ip), dev(ix))
    cs = oracle.constants(op)
    oids, oseen = oracle.build(op, cs, ip, ix)
    return idx, op, cs, oids, oseen, qi, qx


@pytest.mark.parametrize("k", [1, 10, 24])
def test_query_parity(api, qsetup, k):
    idx, op, cs, oids, oseen, qi, qx = qsetup
    gi, gs = idx.query(dev(qi), dev(qx), k)
    wi, ws = oracle.query(op, cs, oids, oseen, qi, qx, k, k_max=24)
    assert (u32(gi) == wi).all() and (u32(gs) == ws).all()


@pytest.mark.parametrize("k", [1, 10, 24])
def test_query_exact_variant(api, qsetup, k):
    # ranking by exact multiplicity (the oracle's exact variant), plain and
    # batched, and the count-min estimate never below the exact count
    idx, op, cs, oids, oseen, qi, qx = qsetup
    gi, gs = idx.query(dev(qi), dev(qx), k, flags=api.FLAG_EXACT)
    wi, ws = oracle.query(op, cs, oids, oseen, qi, qx, k, k_max=24, exact=True)
    assert (u32(gi) == wi).all() and (u32(gs) == ws).all()
    bi, bs = idx.query_batched(dev(qi), dev(qx), k, flags=api.FLAG_EXACT)
    torch.cuda.synchronize()
    assert (u32(bi) == wi).all() and (u32(bs) == ws).all()
    assert int(ws.max()) <= op.L


@pytest.mark.parametrize("k", [10, 24])
def test_query_small_batches(api, qsetup, k):
    # batches too small to fill the GPU run each query with 16 waves; k = 24
    # (above 16) takes the radix select
    idx, op, cs, oids, oseen, qi, qx = qsetup
    wi, ws = oracle.query(op, cs, oids, oseen, qi, qx, k, k_max=24)
    for a, b in ((0, 1), (1, 4), (4, 37)):
        gi, gs = idx.query(dev(qi[a: b + 1] - qi[a]), dev(qx[qi[a]: qi[b]]), k)
        assert (u32(gi) == wi[a:b]).all() and (u32(gs) == ws[a:b]).all()


@pytest.mark.parametrize("waves", [8, 16])
def test_query_wide_groups_large_k(api, qsetup, waves):
    # 8- and 16-wave groups take their own forms of the radix select and of
    # the final ranking; per-query k from 0 to k_max against the oracle
    idx, op, cs, oids, oseen, qi, qx = qsetup
    kq = np.random.default_rng(5).choice([0, 1, 10, 17, 24], size=len(qi) - 1).astype(np.uint32)
    wi, ws = oracle.query(op, cs, oids, oseen, qi, qx, 0, k_max=24, kq=kq)
    gi, gs = idx.query_batched(dev(qi), dev(qx), 0, k_per_query=dev(kq.view(np.int32)),
                               schedule=dict(waves_per_query=waves, queries_per_ticket=0))
    torch.cuda.synchronize()
    assert (u32(gi) == wi).all() and (u32(gs) == ws).all()


def test_query_per_query_k(api, qsetup):
    idx, op, cs, oids, oseen, qi, qx = qsetup
    kq = np.random.default_rng(1).choice([0, 1, 10, 24], size=len(qi) - 1).astype(np.uint32)
    gi, gs = idx.query(dev(qi), dev(qx), 0, k_per_query=dev(kq.view(np.int32)))
    wi, ws = oracle.query(op, cs, oids, oseen, qi, qx, 0, k_max=24, kq=kq)
    assert (u32(gi) == wi).all() and (u32(gs) == ws).all()


def test_query_k_above_kmax_rejected(api, qsetup):
    idx, op, cs, oids, oseen, qi, qx = qsetup
    with pytest.raises(api.SlashError):
        idx.query(dev(qi), dev(qx), 25)
    kq = np.full(len(qi) - 1, 30, dtype=np.uint32)
    with pytest.raises(api.SlashError):
        idx.query(dev(qi), dev(qx), 0, k_per_query=dev(kq.view(np.int32)))


def test_query_exact_special_cases(api):
    # one counter (w = 1): every estimate is |C|, so ranking is by id
    gp, op = params_pair(api, k_max=7, L=8, log2_buckets=6, R=6, cm_rows=1, log2_cm_width=0)
    law, (ip, ix) = rows_of(3000, seed=31)
    idx = api.Index(gp, dev(ip), dev(ix))
    cs = oracle.constants(op)
    oids, oseen = oracle.build(op, cs, ip, ix)
    gi, gs = idx.query(dev(ip[:101]), dev(ix[: ip[100]]), 7)
    wi, ws = oracle.query(op, cs, oids, oseen, ip[:101], ix[: ip[100]], 7)
    assert (u32(gi) == wi).all() and (u32(gs) == ws).all()


@pytest.mark.parametrize("lw", [0, 1], ids=["w1", "w2"])
def test_query_counter_overflow_recount(api, lw):
    # 16 tables x 32 full slots = 512 occurrences over 1 or 2 counters per
    # row: counts pass 255, so the 8-bit sketch overflows and the query is
    # recounted with 16-bit counters
    gp, op = params_pair(api, k_max=12, L=16, log2_buckets=3, R=32, cm_rows=2, log2_cm_width=lw)
    law, (ip, ix) = rows_of(4000, seed=41)
    idx = api.Index(gp, dev(ip), dev(ix))
    cs = oracle.constants(op)
    oids, oseen = oracle.build(op, cs, ip, ix)
    assert int(oseen.min()) > op.R
    qi, qx = ip[:41], ix[: ip[40]]
    gi, gs = idx.query(dev(qi), dev(qx), 12)
    wi, ws = oracle.query(op, cs, oids, oseen, qi, qx, 12)
    assert int(ws.max()) > 255
    assert (u32(gi) == wi).all() and (u32(gs) == ws).all()


@pytest.mark.parametrize("waves", [8, 16])
@pytest.mark.parametrize("lw", [0, 1], ids=["w1", "w2"])
def test_query_wide_groups_estimates_above_255(api, waves, lw):
    # every estimate above 255 (1 or 2 counters per row over 512
    # occurrences) and k above the few-outputs bound: the radix select starts
    # at the estimate's second byte, in the 16-wave form after clearing the
    # histogram the distinct ids counted into
    gp, op = params_pair(api, k_max=24, L=16, log2_buckets=3, R=32, cm_rows=2, log2_cm_width=lw)
    law, (ip, ix) = rows_of(4000, seed=43)
    idx = api.Index(gp, dev(ip), dev(ix))
    cs = oracle.constants(op)
    oids, oseen = oracle.build(op, cs, ip, ix)
    qi, qx = ip[:33], ix[: ip[32]]
    kq = np.random.default_rng(7).choice([20, 24], size=32).astype(np.uint32)
    wi, ws = oracle.query(op, cs, oids, oseen, qi, qx, 0, k_max=24, kq=kq)
    assert int(ws[:, 0].min()) > 255
    gi, gs = idx.query_batched(dev(qi), dev(qx), 0, k_per_query=dev(kq.view(np.int32)),
                               schedule=dict(waves_per_query=waves, queries_per_ticket=0))
    torch.cuda.synchronize()
    assert (u32(gi) == wi).all() and (u32(gs) == ws).all()


@pytest.mark.parametrize("sched", [dict(waves_per_query=1, queries_per_ticket=1),
                                   dict(waves_per_query=2, queries_per_ticket=3),
                                   dict(waves_per_query=4, queries_per_ticket=8, groups_per_cu=1),
                                   dict(waves_per_query=8, queries_per_ticket=1),
                                   dict(waves_per_query=16, queries_per_ticket=2),
                                   dict(waves_per_query=4, queries_per_ticket=0),
                                   dict(waves_per_query=16, queries_per_ticket=0)])
def test_batched_equals_plain(api, qsetup, sched):
    idx, op, cs, oids, oseen, qi, qx = qsetup
    a = idx.query(dev(qi), dev(qx), 10)
    for _ in range(2):  # second call replays the recorded graph
        b = idx.query_batched(dev(qi), dev(qx), 10, schedule=sched)
        torch.cuda.synchronize()
        assert (u32(a[0]) == u32(b[0])).all() and (u32(a[1]) == u32(b[1])).all()


def test_batched_one_group_per_query_follows_batch_size(api, qsetup):
    # the one-group-per-query form updates its recorded grid to each batch
    idx, op, cs, oids, oseen, qi, qx = qsetup
    sched = dict(waves_per_query=4, queries_per_ticket=0)
    for n in (len(qi) - 1, 37, 1, len(qi) - 1):
        sip, six = qi[: n + 1], qx[: qi[n]]
        a = idx.query(dev(sip), dev(six), 10)
        b = idx.query_batched(dev(sip), dev(six), 10, schedule=sched)
        torch.cuda.synchronize()
        assert (u32(a[0]) == u32(b[0])).all() and (u32(a[1]) == u32(b[1])).all(), n


def test_autotune_and_batched_default(api, qsetup):
    idx, op, cs, oids, oseen, qi, qx = qsetup
    best = idx.autotune(dev(qi), dev(qx), 10)
    assert best["waves_per_query"] in (1, 2, 4, 8, 16)
    a = idx.query(dev(qi), dev(qx), 10)
    b = idx.query_batched(dev(qi), dev(qx), 10)
    assert (u32(a[0]) == u32(b[0])).all() and (u32(a[1]) == u32(b[1])).all()


def test_tiny_config_end_to_end(api):
    # tiny configuration: N = 1e5, K=4, L=16, 2^16 buckets, R=32, count-min
    # 4 x 1024, k = 10, 1000 planted-perturbation queries
    master = 2020
    gp, op = params_pair(api, k_max=10, L=16, log2_buckets=16, R=32, cm_rows=4, log2_cm_width=10,
                         seed=synth.derive(master, synth.STREAM_INDEX))
    law = synth.RowLaw(synth.derive(master, synth.STREAM_DATA), 1 << 20)
    ip, ix = law.rows(0, 100000)
    qi, qx, src, _ = law.queries(synth.derive(master, synth.STREAM_QUERY), 100000, 0, 1000)
    idx = api.Index(gp, dev(ip), dev(ix))
    cs = oracle.constants(op)
    check_tables(api, idx, op, cs, ip, ix)
    oids, oseen = oracle.build(op, cs, ip, ix)
    gi, gs = idx.query(dev(qi), dev(qx), 10)
    wi, ws = oracle.query(op, cs, oids, oseen, qi, qx, 10)
    assert (u32(gi) == wi).all() and (u32(gs) == ws).all()
    recall = np.mean([s in r for s, r in zip(src.tolist(), u32(gi).tolist())])
    assert recall >= 0.9


def test_insert_large_batch_path(api):
    # batches above 4096 rows take the sort-based insert path
    gp, op = params_pair(api, L=5, log2_buckets=7, R=9)
    _, (ip, ix) = rows_of(15000, seed=12)
    n0 = 2000
    idx = api.Index(gp, dev(ip[: n0 + 1]), dev(ix[: ip[n0]]))
    for a, b in ((n0, 8000), (8000, 8001), (8001, 15000)):
        idx.insert(dev(ip[a: b + 1] - ip[a]), dev(ix[ip[a]: ip[b]]))
    torch.cuda.synchronize()
    check_tables(api, idx, op, oracle.constants(op), ip, ix)


@pytest.mark.parametrize("log2_buckets", [12, 6], ids=["B12", "B6-full-reservoirs"])
def test_wide_config_end_to_end(api, log2_buckets):
    # wide configuration at 20000 rows: D = 2^24, nnz ~ lognormal(median 500,
    # sigma 0.8) clipped to [50, 20000], uniform indices; K=8, L=128, R=128,
    # count-min 8 x 16384 (counted one row per pass), k in {1, 10, 100}.  The
    # tables are kept at 2^12 buckets so the host copy stays small (2^18 is
    # covered by the hash test); with 2^6 buckets every reservoir is full and
    # a query aggregates 16384 slots.
    master = 2024
    gp, op = params_pair(api, k_max=100, dim=1 << 24, K=8, L=128, log2_buckets=log2_buckets, R=128, cm_rows=8,
                         log2_cm_width=14, seed=synth.derive(master, synth.STREAM_INDEX))
    law = synth.RowLaw(synth.derive(master, synth.STREAM_DATA), 1 << 24, index="uniform", nnz="lognormal",
                       nnz_a=500.0, nnz_b=0.8, nnz_lo=50, nnz_hi=20000)
    n = 20000
    ip, ix = law.rows(0, n)
    qi, qx, src, kq = law.queries(synth.derive(master, synth.STREAM_QUERY), n, 0, 48, nnz_mode="lognormal",
                                  median=500, sigma=0.8, lo=50, hi=20000, f=(0.1, 0.4), kmix=(1, 10, 100))
    idx = api.Index(gp, dev(ip[: 15001]), dev(ix[: ip[15000]]))
    idx.insert(dev(ip[15000:] - ip[15000]), dev(ix[ip[15000]:]))
    cs = oracle.constants(op)
    check_tables(api, idx, op, cs, ip, ix)
    oids, oseen = oracle.build(op, cs, ip, ix)
    wi, ws = oracle.query(op, cs, oids, oseen, qi, qx, 0, k_max=100, kq=kq)
    gi, gs = idx.query(dev(qi), dev(qx), 0, k_per_query=dev(kq.view(np.int32)))
    assert (u32(gi) == wi).all() and (u32(gs) == ws).all()
    bi, bs = idx.query_batched(dev(qi), dev(qx), 0, k_per_query=dev(kq.view(np.int32)))
    torch.cuda.synchronize()
    assert (u32(bi) == wi).all() and (u32(bs) == ws).all()
    ei, es = oracle.query(op, cs, oids, oseen, qi, qx, 0, k_max=100, kq=kq, exact=True)
    gi, gs = idx.query(dev(qi), dev(qx), 0, k_per_query=dev(kq.view(np.int32)), flags=api.FLAG_EXACT)
    assert (u32(gi) == ei).all() and (u32(gs) == es).all()
    if log2_buckets == 6:
        assert int(oseen.min()) > 128  # every reservoir full


# ------------------------------------------ the 200M-shard query instance


@pytest.fixture(scope="module")
def headline(api):
    # The query shape of the 200M-point shard (K=4, L=32, R=64, count-min
    # 4 x 4096, k_max = 100) on 200k rows with 2^10 buckets per table, so the
    # mean bucket load (195) matches the shard's (191) and most reservoirs
    # are full: a query aggregates about 2048 slots, 8 per thread of the
    # 4-wave kernels.  Queries follow the batched mix (lognormal nnz, 10-40%
    # replaced, k drawn from {1, 10, 100}).
    master = 2021
    gp, op = params_pair(api, k_max=100, K=4, L=32, log2_buckets=10, R=64, cm_rows=4, log2_cm_width=12,
                         seed=synth.derive(master, synth.STREAM_INDEX))
    law = synth.RowLaw(synth.derive(master, synth.STREAM_DATA), 1 << 20)
    n = 200_000
    ip, ix = law.rows(0, n)
    qi, qx, src, kq = law.queries(synth.derive(master, synth.STREAM_QUERY), n, 0, 400, nnz_mode="lognormal",
                                  median=40, sigma=1.0, lo=5, hi=2000, f=(0.1, 0.4), kmix=(1, 10, 100))
    idx = api.Index(gp, dev(ip), dev(ix))
    cs = oracle.constants(op)
    oids, oseen = oracle.build(op, cs, ip, ix)
    assert np.mean(np.minimum(oseen, op.R)) > 0.9 * op.R  # most reservoirs full
    wi, ws = oracle.query(op, cs, oids, oseen, qi, qx, 0, k_max=100, kq=kq)
    return idx, op, cs, oids, oseen, qi, qx, kq, wi, ws


def test_headline_shape_tables(api, headline):
    idx, op, cs, oids, oseen, *_ = headline
    gi, gsn = idx.tables()
    assert (u32(gsn) == oseen).all()
    assert (u32(gi) == oids).all()


@pytest.mark.parametrize("sched", [None, dict(waves_per_query=4, queries_per_ticket=0),
                                   dict(waves_per_query=4, queries_per_ticket=1),
                                   dict(waves_per_query=4, queries_per_ticket=8, groups_per_cu=2),
                                   dict(waves_per_query=16, queries_per_ticket=0)],
                         ids=["plain", "4w-grid", "4w-persistent", "4w-persistent-8", "16w-grid"])
def test_headline_shape_query_parity(api, headline, sched):
    # plain slash_query, and the batched path in the launch forms bench.py
    # uses, against the oracle element by element (k in {1, 10, 100})
    idx, op, cs, oids, oseen, qi, qx, kq, wi, ws = headline
    kd = dev(kq.view(np.int32))
    if sched is None:
        gi, gs = idx.query(dev(qi), dev(qx), 0, k_per_query=kd)
    else:
        for _ in range(2):  # the second call replays the recorded graph
            gi, gs = idx.query_batched(dev(qi), dev(qx), 0, k_per_query=kd, schedule=sched)
            torch.cuda.synchronize()
            assert (u32(gi) == wi).all() and (u32(gs) == ws).all()
    assert (u32(gi) == wi).all() and (u32(gs) == ws).all()


def test_headline_shape_autotuned(api, headline):
    idx, op, cs, oids, oseen, qi, qx, kq, wi, ws = headline
    best = idx.autotune(dev(qi), dev(qx), 100)
    gi, gs = idx.query_batched(dev(qi), dev(qx), 0, k_per_query=dev(kq.view(np.int32)))
    torch.cuda.synchronize()
    assert (u32(gi) == wi).all() and (u32(gs) == ws).all(), best
    # k = 10 for every query (the planted-query workload)
    w10, s10 = oracle.query(op, cs, oids, oseen, qi, qx, 10, k_max=100)
    gi, gs = idx.query_batched(dev(qi), dev(qx), 10, schedule=dict(waves_per_query=4, queries_per_ticket=0))
    torch.cuda.synchronize()
    assert (u32(gi) == w10).all() and (u32(gs) == s10).all()


def test_headline_shape_exact(api, headline):
    idx, op, cs, oids, oseen, qi, qx, kq, wi, ws = headline
    ei, es = oracle.query(op, cs, oids, oseen, qi, qx, 0, k_max=100, kq=kq, exact=True)
    gi, gs = idx.query_batched(dev(qi), dev(qx), 0, k_per_query=dev(kq.view(np.int32)), flags=api.FLAG_EXACT,
                               schedule=dict(waves_per_query=4, queries_per_ticket=0))
    torch.cuda.synchronize()
    assert (u32(gi) == ei).all() and (u32(gs) == es).all()
    # the count-min estimate is never below the exact count
    assert (ws[:, 0] >= es[:, 0]).all()


@pytest.mark.parametrize("k", [101, 500, 1024])
def test_query_large_k(api, k):
    # k above 100 up to the largest k_max: candidates from 16 tables of 64
    # slots (at most 1024 distinct ids), so a query can fill its whole row
    gp, op = params_pair(api, k_max=1024, L=16, log2_buckets=6, R=64, cm_rows=2, log2_cm_width=9)
    law, (ip, ix) = rows_of(20000, seed=51)
    idx = api.Index(gp, dev(ip), dev(ix))
    cs = oracle.constants(op)
    oids, oseen = oracle.build(op, cs, ip, ix)
    qi, qx = ip[:65], ix[: ip[64]]
    wi, ws = oracle.query(op, cs, oids, oseen, qi, qx, k, k_max=1024)
    assert (wi[:, min(k, 500) - 1] != EMPTY).any()  # rows well past 100 entries are filled
    gi, gs = idx.query(dev(qi), dev(qx), k)
    assert (u32(gi) == wi).all() and (u32(gs) == ws).all()
    bi, bs = idx.query_batched(dev(qi), dev(qx), k)
    torch.cuda.synchronize()
    assert (u32(bi) == wi).all() and (u32(bs) == ws).all()


def test_query_classic_minhash_mode(api):
    gp, op = params_pair(api, k_max=10, L=12, log2_buckets=9, R=16, hash_mode=2)
    law, (ip, ix) = rows_of(8000, seed=61)
    idx = api.Index(gp, dev(ip), dev(ix))
    cs = oracle.constants(op)
    check_tables(api, idx, op, cs, ip, ix)
    oids, oseen = oracle.build(op, cs, ip, ix)
    qi, qx, _, _ = law.queries(synth.derive(61, synth.STREAM_QUERY), 8000, 0, 100)
    wi, ws = oracle.query(op, cs, oids, oseen, qi, qx, 10)
    gi, gs = idx.query(dev(qi), dev(qx), 10)
    assert (u32(gi) == wi).all() and (u32(gs) == ws).all()


def test_import_rejects_data_past_fill(api):
    # a query reads a bucket's first min(R, seen) slots as the oracle does,
    # which holds for imported tables only if the slots past that are empty:
    # import checks it
    gp, op = params_pair(api, L=3, log2_buckets=5, R=8)
    _, (ip, ix) = rows_of(100, seed=71)
    a = api.Index(gp, dev(ip), dev(ix))
    ids, seen = a.tables()
    sn = u32(seen)
    t, b = np.argwhere(sn < op.R)[0]
    bad = ids.clone()
    bad[t, b, sn[t, b]] = 5
    with pytest.raises(api.SlashError) as e:
        api.Index.from_tables(gp, bad, seen, 100)
    assert e.value.code == api.E_INVAL
    ok = api.Index.from_tables(gp, ids, seen, 100)
    assert ok.info()["n_items"] == 100


@pytest.mark.parametrize("bucket", [0, 1], ids=["reservoir", "topkapi"])
def test_save_load_roundtrip(api, tmp_path, bucket):
    # an index saved to a file and loaded back answers and grows exactly like
    # the original; the header carries the parameters and sizes
    import struct
    kw = dict(L=6, log2_buckets=8, R=12) if bucket == 0 else dict(L=6, log2_buckets=8, R=1, cm_rows=2,
                                                                   log2_cm_width=3)
    gp, op = params_pair(api, k_max=16, hash_mode=2 if bucket == 0 else 0, **kw)
    gp.bucket = bucket
    law, (ip, ix) = rows_of(7000, seed=81)
    a = api.Index(gp, dev(ip[:5001]), dev(ix[: ip[5000]]))
    a.insert(dev(ip[5000:6001] - ip[5000]), dev(ix[ip[5000]: ip[6000]]))
    path = str(tmp_path / "index.slash")
    a.save(path)
    raw = open(path, "rb").read()
    magic, fmt, hb = struct.unpack_from("<8sII", raw, 0)
    fields = struct.unpack_from("<10I", raw, 16)
    seed, n_items, tb, sb = struct.unpack_from("<QQQQ", raw, 56)
    assert magic == b"SLASHIDX" and fmt == 1 and hb == 128
    assert fields == (gp.dim, gp.K, gp.L, gp.log2_buckets, gp.R, gp.cm_rows, gp.log2_cm_width, gp.k_max,
                      gp.hash_mode, gp.bucket)
    assert seed == gp.seed and n_items == 6000 and len(raw) == 128 + tb + sb
    b = api.Index.load(path)
    assert b.info()["n_items"] == 6000 and b.params.bucket == bucket
    for x, y in zip(a.tables(), b.tables()):
        assert torch.equal(x, y)
    tail = (dev(ip[6000:] - ip[6000]), dev(ix[ip[6000]:]))
    a.insert(*tail)
    b.insert(*tail)
    torch.cuda.synchronize()
    for x, y in zip(a.tables(), b.tables()):
        assert torch.equal(x, y)
    qi, qx, _, _ = law.queries(synth.derive(81, synth.STREAM_QUERY), 7000, 0, 40)
    ra, rb = a.query(dev(qi), dev(qx), 16), b.query(dev(qi), dev(qx), 16)
    assert torch.equal(ra[0], rb[0]) and torch.equal(ra[1], rb[1])
    if bucket == 0:
        check_tables(api, b, op, oracle.constants(op), ip, ix)
    # a damaged file is refused
    for name, data in (("flipped", raw[:200] + bytes([raw[200] ^ 1]) + raw[201:]), ("short", raw[:-4]),
                       ("magic", b"X" + raw[1:])):
        bad = str(tmp_path / name)
        open(bad, "wb").write(data)
        with pytest.raises(api.SlashError) as e:
            api.Index.load(bad)
        assert e.value.code == api.E_INVAL, name


def test_wide_config_full_bucket_count(api):
    # the wide configuration's own table shape (K=8, L=128, 2^18 buckets,
    # R=128: 17 GB of reservoirs) on 20000 of its rows: seen everywhere, the
    # fill of every bucket, the reservoir of every non-empty bucket, and 48
    # queries of the k mix (count-min 8 x 16384, 16384 slots per query)
    free, _ = torch.cuda.mem_get_info()
    if free < (64 << 30):
        pytest.skip("needs ~64 GB of free device memory")
    master = 2024
    gp, op = params_pair(api, k_max=100, dim=1 << 24, K=8, L=128, log2_buckets=18, R=128, cm_rows=8,
                         log2_cm_width=14, seed=synth.derive(master, synth.STREAM_INDEX))
    law = synth.RowLaw(synth.derive(master, synth.STREAM_DATA), 1 << 24, index="uniform", nnz="lognormal",
                       nnz_a=500.0, nnz_b=0.8, nnz_lo=50, nnz_hi=20000)
    n = 20000
    ip, ix = law.rows(0, n)
    qi, qx, src, kq = law.queries(synth.derive(master, synth.STREAM_QUERY), n, 0, 48, nnz_mode="lognormal",
                                  median=500, sigma=0.8, lo=50, hi=20000, f=(0.1, 0.4), kmix=(1, 10, 100))
    idx = api.Index(gp, dev(ip), dev(ix))
    cs = oracle.constants(op)
    oids, oseen = oracle.build(op, cs, ip, ix)
    gi, gsn = idx.tables()
    assert (u32(gsn) == oseen).all()
    for t in range(op.L):  # slots in use per bucket = min(R, seen), for every bucket
        live = (gi[t] != -1).sum(dim=1)
        assert torch.equal(live, torch.clamp(gsn[t].to(live.dtype), max=op.R))
    tt, bb = np.nonzero(oseen)
    got = u32(gi[torch.from_numpy(tt).cuda(), torch.from_numpy(bb).cuda()])
    assert (got == oids[tt, bb]).all()
    del gi, gsn
    wi, ws = oracle.query(op, cs, oids, oseen, qi, qx, 0, k_max=100, kq=kq)
    del oids
    kd = dev(kq.view(np.int32))
    gi, gs = idx.query(dev(qi), dev(qx), 0, k_per_query=kd)
    assert (u32(gi) == wi).all() and (u32(gs) == ws).all()
    bi, bs = idx.query_batched(dev(qi), dev(qx), 0, k_per_query=kd)
    torch.cuda.synchronize()
    assert (u32(bi) == wi).all() and (u32(bs) == ws).all()
    idx.close()
