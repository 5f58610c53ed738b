"""The allocation-free cut (vmo_cut_noalloc, workspace in the library's
static device arena) against vmo_cut, through the C ABI: two calls in a row,
the second on a smaller input; nets above 64 pins (the sorted path),
non-integer weights and costs over several orders of magnitude, part ids
beyond nparts, part weights.  Integer results and part weights must be
identical, and the FP64 totals too (same kernels, same order); both are also
checked against the oracle.  Sizes beyond the limit are rejected before any
work."""
import numpy as np
import pytest
import torch

import oracle
import vmo_gen
from gpu_util import dev_h, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1105_4490_amd as P
    return P.Context(0)


def big_case(seed):
    g = vmo_gen.zipf_rect(20000, 400, seed, clip=400)     # column-net: nets of ~280 pins
    h = oracle.colnet(g.m, g.n, g.rowptr, g.col)
    r = vmo_gen.rng(seed, 31)
    h.w = (10.0 ** r.uniform(-3, 3, size=h.k)).astype(np.float32)
    h.c = (10.0 ** r.uniform(-2, 2, size=h.l)).astype(np.float32)
    nparts = 70
    part = r.integers(0, nparts + 8, size=h.k).astype(np.int32)   # some ids >= nparts (not weighed)
    return h, part, nparts


def small_case(seed):
    g = vmo_gen.grid2d(12)
    h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
    r = vmo_gen.rng(seed, 32)
    h.w = r.uniform(0.1, 3.0, size=h.k).astype(np.float32)
    nparts = 5
    part = r.integers(0, nparts, size=h.k).astype(np.int32)
    return h, part, nparts


def check_against_oracle(h, part, nparts, got):
    ref = oracle.cut(h, part, nparts)
    assert got["nets_cut"] == ref["nets_cut"]
    assert np.array_equal(host(got["part_weight"]), ref["part_weight"])
    # FP64 sums of non-negative terms in another order: within (l + 1) 2^-53 of the total
    for f in ("lambda_minus_one", "cut_net"):
        assert abs(got[f] - ref[f]) <= (h.l + 1) * 2.0 ** -53 * ref[f], f


def test_noalloc_cut_equals_cut_twice(ctx):
    for h, part, nparts in (big_case(1), small_case(2)):
        print("case k", h.k, "l", h.l, "nparts", nparts, flush=True)
        dh = dev_h(h)
        dp = torch.as_tensor(part).cuda()
        a = ctx.cut(dh, dp, nparts)
        b = ctx.cut(dh, dp, nparts, noalloc=True)
        for f in ("lambda_minus_one", "cut_net", "nets_cut"):
            assert a[f] == b[f], f
        assert torch.equal(a["part_weight"], b["part_weight"])
        check_against_oracle(h, part, nparts, b)
        # unit weights: part sizes
        h1 = oracle.Hypergraph(h.k, h.l, h.ptr, h.pins, None, h.c)
        dh1 = dev_h(h1)
        a1 = ctx.cut(dh1, dp, nparts)
        b1 = ctx.cut(dh1, dp, nparts, noalloc=True)
        assert torch.equal(a1["part_weight"], b1["part_weight"]) and a1["cut_net"] == b1["cut_net"]
        assert np.array_equal(host(b1["part_weight"]), np.bincount(part[part < nparts], minlength=nparts))


def test_noalloc_cut_rejects_sizes_beyond_the_limit(ctx):
    import paper_1105_4490_amd as P
    k = (1 << 20) + 1
    dh = P.DeviceHypergraph(k, 0, torch.zeros(1, dtype=torch.int64, device="cuda"),
                            torch.zeros(1, dtype=torch.int32, device="cuda"))
    part = torch.zeros(k, dtype=torch.int32, device="cuda")
    with pytest.raises(P.VmoError) as e:
        ctx.cut(dh, part, 1, noalloc=True)
    assert e.value.status == P.VMO_E_UNSUPPORTED
    # the context still works afterwards, with and without the arena
    h, part2, nparts = small_case(3)
    dh2 = dev_h(h)
    dp2 = torch.as_tensor(part2).cuda()
    assert ctx.cut(dh2, dp2, nparts, noalloc=True)["cut_net"] == ctx.cut(dh2, dp2, nparts)["cut_net"]
