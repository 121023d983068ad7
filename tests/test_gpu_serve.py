"""Serving loop (continuous batching with epoch-ordered inserts): every
served result equals the oracle's result on the index state of its epoch
(the rows inserted before it), and the standalone result of the same
library."""
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


@pytest.fixture(scope="module")
def setup(api):
    law = synth.RowLaw(synth.derive(31, synth.STREAM_DATA), 1 << 20)
    n0, n1 = 20000, 1500
    ip, ix = law.rows(0, n0 + n1)
    qi, qx, _, kq = law.queries(synth.derive(31, synth.STREAM_QUERY), n0, 0, 1200, nnz_mode="lognormal",
                                median=40, sigma=1.0, lo=5, hi=2000, f=(0.1, 0.4), kmix=(1, 10, 100))
    params = api.Params.of(dim=1 << 20, K=4, L=16, log2_buckets=12, R=16, cm_rows=4, log2_cm_width=10, k_max=100,
                           seed=synth.derive(31, synth.STREAM_INDEX))
    return law, params, ip, ix, n0, n1, qi, qx, kq


def oracle_params(params):
    return oracle.Params(**{f: int(getattr(params, f)) for f in ("dim", "K", "L", "log2_buckets", "R", "cm_rows",
                                                                 "log2_cm_width", "hash_mode", "seed")})


def oracle_answers(params, ip, ix, n_rows, qi, qx, kq):
    """(ids, scores) [nq, k_max] of the oracle on the first n_rows rows."""
    op = oracle_params(params)
    cs = oracle.constants(op)
    sip, six = ip[: n_rows + 1], ix[: ip[n_rows]]
    if params.bucket:
        cells, _ = oracle.tk_build(op, cs, sip, six)
        return oracle.tk_query(op, cs, cells, qi, qx, 0, k_max=params.k_max, kq=kq)
    oids, oseen = oracle.build(op, cs, sip, six)
    return oracle.query(op, cs, oids, oseen, qi, qx, 0, k_max=params.k_max, kq=kq)


def standalone(api, params, ip, ix, n_rows, qi, qx, kq):
    idx = api.Index(params, dev(ip[: n_rows + 1]), dev(ix[: ip[n_rows]]))
    gi, gs = idx.query(dev(qi), dev(qx), 0, k_per_query=dev(kq.view(np.int32)))
    torch.cuda.synchronize()
    out = u32(gi), u32(gs)
    idx.close()
    return out


def test_served_results_equal_standalone(api, setup):
    law, params, ip, ix, n0, n1, qi, qx, kq = setup
    ref_i, ref_s = standalone(api, params, ip, ix, n0, qi, qx, kq)
    idx = api.Index(params, dev(ip[: n0 + 1]), dev(ix[: ip[n0]]))
    srv = api.slash_serve_start(idx.handle, hbm_budget_bytes=64 << 20, max_batch=128, max_inflight=3)
    tickets = {}
    for q in range(len(qi) - 1):
        t = api.slash_serve_submit_query(srv, qx[qi[q]:qi[q + 1]], int(kq[q]))
        tickets[t] = q
    got = []
    while len(got) < len(tickets):
        got += api.slash_serve_poll(srv)
    stats = api.slash_serve_stop(srv)
    assert stats["queries_done"] == len(tickets) and stats["batches"] >= 1
    for c in got:
        q = tickets[c["ticket"]]
        k = int(kq[q])
        assert c["status"] == 0 and c["epoch"] == 0 and c["k"] == k
        assert (c["ids"] == ref_i[q, :k]).all() and (c["scores"] == ref_s[q, :k]).all()
    idx.close()


def test_served_results_equal_oracle(api, setup):
    # every completion against the oracle's build of the same rows, with
    # several batches in flight (small batches, four slots)
    law, params, ip, ix, n0, n1, qi, qx, kq = setup
    ref_i, ref_s = oracle_answers(params, ip, ix, n0, qi, qx, kq)
    idx = api.Index(params, dev(ip[: n0 + 1]), dev(ix[: ip[n0]]))
    srv = api.slash_serve_start(idx.handle, hbm_budget_bytes=64 << 20, max_batch=16, max_inflight=4)
    tickets = {api.slash_serve_submit_query(srv, qx[qi[q]:qi[q + 1]], int(kq[q])): q for q in range(len(qi) - 1)}
    got = []
    while len(got) < len(tickets):
        got += api.slash_serve_poll(srv)
    stats = api.slash_serve_stop(srv)
    assert stats["batches"] > 4
    for c in got:
        q = tickets[c["ticket"]]
        k = int(kq[q])
        assert c["status"] == 0 and c["epoch"] == 0 and c["k"] == k
        assert (c["ids"] == ref_i[q, :k]).all() and (c["scores"] == ref_s[q, :k]).all()
    idx.close()


def test_max_wait_holds_partial_batches(api, setup):
    # with a long max_wait the scheduler launches only full batches (and the
    # last one once its oldest query has waited); results are unchanged
    law, params, ip, ix, n0, n1, qi, qx, kq = setup
    ref_i, ref_s = standalone(api, params, ip, ix, n0, qi, qx, kq)
    idx = api.Index(params, dev(ip[: n0 + 1]), dev(ix[: ip[n0]]))
    srv = api.slash_serve_start(idx.handle, hbm_budget_bytes=64 << 20, max_batch=64, max_inflight=3,
                                max_wait_us=50_000)
    nq = len(qi) - 1
    tickets = {api.slash_serve_submit_query(srv, qx[qi[q]:qi[q + 1]], int(kq[q])): q for q in range(nq)}
    got = []
    while len(got) < nq:
        got += api.slash_serve_poll(srv)
    stats = api.slash_serve_stop(srv)
    assert stats["queries_done"] == nq and stats["batches"] <= -(-nq // 64) + 2
    assert stats["busy_s"] > 0
    for c in got:
        q = tickets[c["ticket"]]
        k = int(kq[q])
        assert c["status"] == 0 and (c["ids"] == ref_i[q, :k]).all() and (c["scores"] == ref_s[q, :k]).all()
    idx.close()


def test_inserts_close_epochs(api, setup):
    # queries submitted before an insert see the index without it; those
    # after see it (the inserted index equals a bulk build on the union)
    law, params, ip, ix, n0, n1, qi, qx, kq = setup
    check_epochs(api, setup, params)


def test_inserts_close_epochs_topkapi_buckets(api, setup):
    # the same with Topkapi buckets (4 x 16 cells per bucket)
    params = api.Params.of(dim=1 << 20, K=4, L=16, log2_buckets=12, R=1, cm_rows=4, log2_cm_width=4, k_max=100,
                           bucket=1, seed=synth.derive(31, synth.STREAM_INDEX))
    check_epochs(api, setup, params)


def check_epochs(api, setup, params):
    law, _, ip, ix, n0, n1, qi, qx, kq = setup
    before = oracle_answers(params, ip, ix, n0, qi, qx, kq)
    after = oracle_answers(params, ip, ix, n0 + n1, qi, qx, kq)
    # the library's own standalone answers agree with the oracle too
    for ref, n in ((before, n0), (after, n0 + n1)):
        gi, gs = standalone(api, params, ip, ix, n, qi, qx, kq)
        assert (gi == ref[0]).all() and (gs == ref[1]).all()
    idx = api.Index(params, dev(ip[: n0 + 1]), dev(ix[: ip[n0]]))
    srv = api.slash_serve_start(idx.handle, hbm_budget_bytes=64 << 20, max_batch=64, max_inflight=4)
    nq = len(qi) - 1
    tickets = {}
    for q in range(nq // 2):
        tickets[api.slash_serve_submit_query(srv, qx[qi[q]:qi[q + 1]], int(kq[q]))] = ("q", q, 0)
    sip = ip[n0: n0 + n1 + 1] - ip[n0]
    six = ix[ip[n0]: ip[n0 + n1]]
    tickets[api.slash_serve_submit_insert(srv, sip, six)] = ("i", None, 1)
    for q in range(nq // 2, nq):
        tickets[api.slash_serve_submit_query(srv, qx[qi[q]:qi[q + 1]], int(kq[q]))] = ("q", q, 1)
    got = []
    while len(got) < len(tickets):
        got += api.slash_serve_poll(srv)
    api.slash_serve_stop(srv)
    for c in got:
        kind, q, epoch = tickets[c["ticket"]]
        assert c["status"] == 0 and c["epoch"] == epoch
        if kind == "i":
            assert c["first_id"] == n0 and c["n_ids"] == n1
            continue
        ref_i, ref_s = before if epoch == 0 else after
        k = int(kq[q])
        assert (c["ids"] == ref_i[q, :k]).all() and (c["scores"] == ref_s[q, :k]).all()
    assert idx.info()["n_items"] == n0 + n1
    idx.close()


def test_stop_drains_and_rejects(api, setup):
    law, params, ip, ix, n0, n1, qi, qx, kq = setup
    idx = api.Index(params, dev(ip[: n0 + 1]), dev(ix[: ip[n0]]))
    with pytest.raises(api.SlashError) as e:
        api.slash_serve_start(idx.handle, hbm_budget_bytes=1 << 10)
    assert e.value.code == api.E_NOMEM
    srv = api.slash_serve_start(idx.handle, hbm_budget_bytes=64 << 20, max_batch=32, max_inflight=2,
                                max_query_nnz=2000)
    with pytest.raises(api.SlashError) as e:
        api.slash_serve_submit_query(srv, np.arange(2001), 10)
    assert e.value.code == api.E_INVAL
    with pytest.raises(api.SlashError) as e:
        api.slash_serve_submit_query(srv, np.array([1, 2, 1 << 21]), 10)
    assert e.value.code == api.E_INVAL
    with pytest.raises(api.SlashError) as e:
        api.slash_serve_submit_query(srv, np.array([1, 2]), 129)
    assert e.value.code == api.E_INVAL
    n = 0
    for q in range(len(qi) - 1):
        api.slash_serve_submit_query(srv, qx[qi[q]:qi[q + 1]], int(kq[q]))
        n += 1
    stats = api.slash_serve_stop(srv)  # returns only after every accepted request ran
    assert stats["queries_done"] == n
    idx.close()


def test_replay_open_loop(api, setup):
    # open-loop arrivals with about a hundred inserts interleaved among the
    # queries, several batches and inserts in flight at once: each query's
    # returned ids equal the oracle's top-k on the rows inserted before it
    # (submission order fixes its epoch: the inserts submitted before it)
    law, params, ip, ix, n0, n1, qi, qx, kq = setup
    idx = api.Index(params, dev(ip[: n0 + 1]), dev(ix[: ip[n0]]))
    srv = api.slash_serve_start(idx.handle, hbm_budget_bytes=128 << 20, max_batch=256, max_inflight=4)
    n = 1000
    t, ins, sz = synth.arrivals(synth.derive(31, synth.STREAM_ARRIVAL), n, 20000.0, 0.1, 1, 64)
    nq = int((~ins).sum())
    q_ptr = np.zeros(nq + 1, dtype=np.int64)
    reps = [(q % (len(qi) - 1)) for q in range(nq)]
    lens = np.array([qi[r + 1] - qi[r] for r in reps])
    q_ptr[1:] = np.cumsum(lens)
    q_idx = np.concatenate([qx[qi[r]:qi[r + 1]] for r in reps])
    q_k = np.array([kq[r] for r in reps], dtype=np.uint32)
    rows = int(sz[ins].sum())
    iip, iix = law.rows(n0, rows)
    lat, ids = api.slash_serve_replay(srv, t, ins, sz, q_ptr, q_idx, q_k, iip, iix, out_stride=100)
    stats = api.slash_serve_stop(srv)
    assert (lat >= 0).all() and stats["queries_done"] == nq and stats["inserts_done"] == int(ins.sum())
    assert stats["rows_inserted"] == rows
    assert int(ins.sum()) >= 50
    # the oracle replays the same sequence: inserts grow its tables, each run
    # of queries between two inserts is answered on the tables of that epoch
    op = oracle_params(params)
    cs = oracle.constants(op)
    oids, oseen = oracle.build(op, cs, ip[: n0 + 1], ix[: ip[n0]])
    next_id, next_row, qn, i = n0, 0, 0, 0
    while i < n:
        if ins[i]:
            m = int(sz[i])
            sip = iip[next_row: next_row + m + 1] - iip[next_row]
            six = iix[iip[next_row]: iip[next_row + m]]
            oracle.insert(op, cs, oids, oseen, next_id, sip, six)
            next_id += m
            next_row += m
            i += 1
            continue
        j = i
        while j < n and not ins[j]:
            j += 1
        m = j - i  # queries qn .. qn + m of this epoch
        sub_ip = q_ptr[qn: qn + m + 1] - q_ptr[qn]
        sub_ix = q_idx[q_ptr[qn]: q_ptr[qn + m]]
        wi, _ = oracle.query(op, cs, oids, oseen, sub_ip, sub_ix, 0, k_max=100, kq=q_k[qn: qn + m])
        for r in range(m):
            k = int(q_k[qn + r])
            assert (ids[i + r, :k] == wi[r, :k]).all(), (i + r, k)
            assert (ids[i + r, k:] == EMPTY).all()
        qn += m
        i = j
    idx.close()


@pytest.mark.parametrize("bucket,fusion,shape", [(0, 0, "small"), (0, 1, "small"), (0, 2, "small"), (1, 0, "small"),
                                                 (0, 0, "headline"), (0, 2, "headline")])
def test_burst_inserts_prepared_ahead(api, setup, bucket, fusion, shape):
    # every request submitted before the first poll, so the FIFO is long:
    # inserts are prepared ahead (at most eight insert slots at once, runs of
    # back-to-back inserts sharing a slot) while the query batches before
    # them run; each query equals the oracle on the rows inserted before it,
    # and the ids of the inserts follow submission order.  fusion 2 writes
    # every insert that follows a query batch in that batch's launch (the
    # queries must not see it), fusion 1 never does.  A batch whose insert
    # has more requests queued behind it is only gathered in the insert's
    # launch and ranked in the next one.  "headline": the 200M-point shard's
    # table shape (L = 32, R = 64, count-min 4 x 4096) on 20k rows
    law, params, ip, ix, n0, n1, qi, qx, kq = setup
    if shape == "headline":
        params = api.Params.of(dim=1 << 20, K=4, L=32, log2_buckets=10, R=64, cm_rows=4, log2_cm_width=12,
                               k_max=100, seed=synth.derive(31, synth.STREAM_INDEX))
    if bucket:
        params = api.Params.of(dim=1 << 20, K=4, L=16, log2_buckets=12, R=1, cm_rows=4, log2_cm_width=4, k_max=100,
                               bucket=1, seed=synth.derive(31, synth.STREAM_INDEX))
    rng = np.random.default_rng(7)
    plan = []  # ("q", query index) or ("i", rows)
    nq = len(qi) - 1
    q = 0
    for block in range(40):
        for _ in range(int(rng.integers(0, 6))):
            plan.append(("q", q % nq))
            q += 1
        for _ in range(block % 4):
            plan.append(("i", int(rng.integers(1, 40))))
    total_rows = sum(m for kind, m in plan if kind == "i")
    iip, iix = law.rows(n0, total_rows)
    idx = api.Index(params, dev(ip[: n0 + 1]), dev(ix[: ip[n0]]))
    srv = api.slash_serve_start(idx.handle, hbm_budget_bytes=256 << 20, max_batch=16, max_inflight=4,
                                insert_fusion=fusion)
    tickets = {}
    row = 0
    n_ins = 0
    for kind, v in plan:
        if kind == "q":
            tickets[api.slash_serve_submit_query(srv, qx[qi[v]:qi[v + 1]], int(kq[v]))] = ("q", v, n_ins)
        else:
            sip = iip[row: row + v + 1] - iip[row]
            six = iix[iip[row]: iip[row + v]]
            n_ins += 1
            tickets[api.slash_serve_submit_insert(srv, sip, six)] = ("i", (n0 + row, v), n_ins)
            row += v
    got = []
    while len(got) < len(tickets):
        got += api.slash_serve_poll(srv)
    stats = api.slash_serve_stop(srv)
    assert stats["inserts_done"] == n_ins and stats["rows_inserted"] == total_rows
    if fusion == 1 or bucket:
        assert stats["fused_commits"] == 0
    elif fusion == 2:
        # an insert queued right behind a query batch (there are dozens)
        assert stats["fused_commits"] >= 1, stats
        if shape == "headline":
            # with requests queued behind the insert, the batch is split
            assert stats["split_batches"] >= 1, stats
    # the oracle's tables after each insert, and its answers per epoch
    op = oracle_params(params)
    cs = oracle.constants(op)
    answers = {}
    queries_by_epoch = {}
    for kind, v, e in tickets.values():
        if kind == "q":
            queries_by_epoch.setdefault(e, []).append(v)
    epochs = sorted(queries_by_epoch)
    # rebuild from the union for each epoch that has queries (inserts equal a
    # bulk build on the union, for both bucket kinds)
    rows_before = [0]
    for kind, v in plan:
        if kind == "i":
            rows_before.append(rows_before[-1] + v)
    uip = np.concatenate([ip[: n0 + 1], ip[n0] + iip[1:]])
    uix = np.concatenate([ix[: ip[n0]], iix])
    for e in epochs:
        qs = sorted(set(queries_by_epoch[e]))
        n_rows = n0 + rows_before[e]
        sub_ip = np.concatenate([[0], np.cumsum([qi[v + 1] - qi[v] for v in qs])]).astype(np.int64)
        sub_ix = np.concatenate([qx[qi[v]:qi[v + 1]] for v in qs])
        sub_k = np.array([kq[v] for v in qs], dtype=np.uint32)
        wi, ws = oracle_answers(params, uip, uix, n_rows, sub_ip, sub_ix, sub_k)
        for r, v in enumerate(qs):
            answers[(e, v)] = (wi[r], ws[r])
    for c in got:
        kind, v, e = tickets[c["ticket"]]
        assert c["status"] == 0 and c["epoch"] == e
        if kind == "i":
            assert (c["first_id"], c["n_ids"]) == v
            continue
        k = int(kq[v])
        ref_i, ref_s = answers[(e, v)]
        assert (c["ids"] == ref_i[:k]).all() and (c["scores"] == ref_s[:k]).all(), (e, v)
    assert idx.info()["n_items"] == n0 + total_rows
    idx.close()
