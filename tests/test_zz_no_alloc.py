"""The allocation-free batched query (slash_query_batched_static) against the
allocating batched path, element by element, through the C ABI: two calls in
a row on the same static scratch, the second with a smaller batch, in both
launch forms; a batch beyond the static scratch is refused."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("sched", [dict(waves_per_query=4, queries_per_ticket=0),
                                   dict(waves_per_query=4, queries_per_ticket=2),
                                   None], ids=["grid", "persistent", "default"])
def test_static_equals_batched_two_calls(api, sched):
    law = synth.RowLaw(synth.derive(77, synth.STREAM_DATA), 1 << 20)
    ip, ix = law.rows(0, 60000)
    p = api.Params.of(dim=1 << 20, K=4, L=32, log2_buckets=8, R=64, cm_rows=4, log2_cm_width=12, k_max=100,
                      seed=synth.derive(77, synth.STREAM_INDEX))
    idx = api.Index(p, dev(ip), dev(ix))
    qi, qx, _, kq = law.queries(synth.derive(77, synth.STREAM_QUERY), 60000, 0, 3000, nnz_mode="lognormal",
                                median=40, sigma=1.0, lo=5, hi=2000, f=(0.1, 0.4), kmix=(1, 10, 100))
    for n in (3000, 700):  # the second call reuses the scratch with a smaller batch
        sip, six, skq = dev(qi[: n + 1]), dev(qx[: qi[n]]), dev(kq[:n].view(np.int32))
        ai, a_s = api.slash_query_batched(idx.handle, sip, six, 0, k_per_query=skq, schedule=sched)
        bi, b_s = api.slash_query_batched_static(idx.handle, sip, six, 0, k_per_query=skq, schedule=sched)
        torch.cuda.synchronize()
        assert (u32(ai) == u32(bi)).all() and (u32(a_s) == u32(b_s)).all(), n
    idx.close()


def test_static_refuses_oversized_batch(api):
    law = synth.RowLaw(synth.derive(78, synth.STREAM_DATA), 1 << 20)
    ip, ix = law.rows(0, 1000)
    p = api.Params.of(dim=1 << 20, K=1, L=1024, log2_buckets=4, R=1, cm_rows=1, log2_cm_width=4, k_max=4,
                      seed=5)
    idx = api.Index(p, dev(ip), dev(ix))
    # 4,194,240 / 1024 = 4095 queries fit; 4096 do not
    n = 4096
    qi = np.arange(n + 1, dtype=np.int64)
    qx = np.arange(n, dtype=np.int32)
    with pytest.raises(api.SlashError) as e:
        api.slash_query_batched_static(idx.handle, dev(qi), dev(qx), 4)
    assert e.value.code == api.E_INVAL
    a = api.slash_query_batched(idx.handle, dev(qi[:4096]), dev(qx[:4095]), 4)
    b = api.slash_query_batched_static(idx.handle, dev(qi[:4096]), dev(qx[:4095]), 4)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    idx.close()
