"""The C ABI's completion and error contract on the GPU: calls marked
[async] return before their work is done and report device-side checks
through vmo_sync; a call on another stream waits for the previous
asynchronous call's work; pool_bytes bounds the cached workspace."""
import numpy as np
import pytest
import torch

import oracle
import vmo_gen
from gpu_util import compare_order, dev_h, dev_x, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1105_4490_amd as Pk
    return Pk


def test_invalid_input_reported_by_sync(P):
    ctx = P.Context(0)
    m = 50
    mu = np.concatenate([np.arange(m, 2 * m), np.arange(m)]).astype(np.int32)
    rp0 = torch.full((m,), -7, dtype=torch.int32, device="cuda")
    # vmo_matched_perms with a vperm that is not a permutation: the call
    # returns VMO_OK, writes nothing, and vmo_sync returns VMO_E_INVALID
    import ctypes as C
    vperm = torch.zeros(2 * m, dtype=torch.int32, device="cuda")
    cp0 = torch.full((m,), -7, dtype=torch.int32, device="cuda")
    dmu = torch.as_tensor(mu).cuda()
    st = P.lib().vmo_matched_perms(ctx.h, C.c_int32(m), P._ptr(vperm), P._ptr(dmu), P._ptr(rp0), P._ptr(cp0),
                                   P._stream())
    assert st == P.VMO_OK
    with pytest.raises(P.VmoError) as e:
        ctx.sync()
    assert e.value.status == P.VMO_E_INVALID and "not a permutation" in str(e.value)
    assert (host(rp0) == -7).all() and (host(cp0) == -7).all()
    ctx.sync()                                     # cleared
    # a row without a partner column
    bad_mu = mu.copy()
    bad_mu[3] = 7                                  # a row, not a column
    ctx.matched_perms(m, torch.arange(2 * m, dtype=torch.int32, device="cuda"), torch.as_tensor(bad_mu).cuda())
    with pytest.raises(P.VmoError, match="partner column"):
        ctx.sync()
    # vmo_finegrain with a column outside [0, n)
    g = vmo_gen.grid2d(6)
    col = g.col.copy()
    col[5] = g.n + 3
    x = vmo_gen.random_points(g.m + g.n, 1)
    ctx.finegrain(g.m, g.n, torch.as_tensor(g.rowptr).cuda(), torch.as_tensor(col).cuda(), dev_x(x))
    with pytest.raises(P.VmoError, match="CSR arrays invalid"):
        ctx.sync()
    # valid input: no error, same result as before the change of contract
    got = ctx.finegrain(g.m, g.n, torch.as_tensor(g.rowptr).cuda(), torch.as_tensor(g.col).cuda(), dev_x(x))
    ctx.sync()
    assert np.array_equal(host(got), oracle.finegrain(g.m, g.n, g.rowptr, g.col, x))
    ctx.close()


def test_async_calls_on_two_streams(P):
    """Two orderings queued back to back on two streams of one context (the
    second call waits for the first's work before reusing its pool blocks),
    then a third on the first stream: every result equals the oracle's."""
    ctx = P.Context(0)
    cases = []
    for N, seed in ((14, 1), (11, 2), (12, 3)):
        g = vmo_gen.grid3d(N, seed=N)
        h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
        x = vmo_gen.random_points(h.k, seed, clusters=4)
        cases.append((h, x, oracle.order(h, x, 16, seed, mode=oracle.GRAPH_MODE, ord=oracle.BBD), seed))
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    outs = []
    for (h, x, _, seed), st in zip(cases, (sa, sb, sa)):
        with torch.cuda.stream(st):
            dh, dx = dev_h(h), dev_x(x)
            outs.append((ctx.order(dh, dx, 16, seed, mode=P.GRAPH, order=P.BBD), dh, dx))
    sa.synchronize()
    sb.synchronize()
    for (o, _, _), (h, _, ref, _) in zip(outs, cases):
        compare_order(o, ref, oracle.GRAPH_MODE, h.k, h.l)
    ctx.close()


def test_pool_bytes_bounds_the_cached_workspace(P):
    g = vmo_gen.grid3d(32, seed=2)
    h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    x = vmo_gen.random_points(h.k, 2, clusters=4)
    held = {}
    for cap in (0, 1 << 20):
        ctx = P.Context(0, pool_bytes=cap)
        dh, dx = dev_h(h), dev_x(x)
        o = ctx.order(dh, dx, 64, 1, mode=P.GRAPH, order=P.BBD)
        ctx.sync()                      # trims to the bound
        held[cap] = ctx.pool_bytes()
        c = ctx.cut(dh, o["part"], 64)  # a call that waits: trims as well
        assert ctx.pool_bytes() <= max(cap, 0) or cap == 0
        assert c["cut_net"] == oracle.cut(h, host(o["part"]), 64)["cut_net"]
        ctx.close()
    assert held[0] > (1 << 20) >= held[1 << 20]
