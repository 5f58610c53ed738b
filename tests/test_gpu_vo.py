"""GPU parity of the whole V+O path (hypergraph model, multilevel layout of
Algorithms 2 and 3, recursive ordering of Algorithm 7 with emission, cut) at
sizes where every multi-kernel path runs: the tree built by sort and node
kernels above 4,096 points, the spread and unspread walks, the attraction
kernels above 16,384 points, the step applied by k_combine, coarsening over
many levels.  The layout is compared bit for bit with the oracle's strict
mode, the ordering and cut element by element.

The 64^3 benchmark input is compared with digests written by
tests/golden/make_vo_golden.py (oracle only); the smaller cases run the
oracle here."""
import hashlib
import json
import os

import numpy as np
import pytest
import torch

import oracle
import vmo_gen
from gpu_util import compare_order, dev_h, host

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx():
    import paper_1105_4490_amd as P
    return P.Context(0)


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


@pytest.mark.parametrize("case", ["grid3d20_bbd64", "grid3d32_bbd64", "zipf20k_sbd64"])
def test_vo_against_oracle(ctx, case):
    """Layout (bit for bit), then the recursive ordering with the layout
    inside (vmo_order with x = NULL), against oracle.layout + oracle.order."""
    import paper_1105_4490_amd as P
    if case.startswith("grid3d"):
        side = int(case[6:8])
        g = vmo_gen.grid3d(side, seed=1)
        h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
        mode, order, omode, oord = P.GRAPH, P.BBD, oracle.GRAPH_MODE, oracle.BBD
    else:
        g = vmo_gen.zipf_rect(20000, 10000, 2, clip=2000)
        h = oracle.colnet(g.m, g.n, g.rowptr, g.col)
        mode, order, omode, oord = P.NET, P.SBD, oracle.NET_MODE, oracle.SBD
    print("case", case, "k", h.k, "l", h.l, flush=True)
    x = oracle.layout(h, oracle.layout_params(seed=1))
    ref = oracle.order(h, x, 64, 1, mode=omode, ord=oord)
    dh = dev_h(h)
    gx = host(ctx.layout(dh, P.layout_params(seed=1)))
    assert np.array_equal(gx, x), "layout not bit-identical"
    o = ctx.order(dh, None, 64, 1, mode=mode, order=order, lp=P.layout_params(seed=1))
    compare_order(o, ref, omode, h.k, h.l)
    c = ctx.cut(dh, o["part"], 64)
    rc = oracle.cut(h, ref.part, 64)
    assert c["cut_net"] == rc["cut_net"] and c["lambda_minus_one"] == rc["lambda_minus_one"]


def test_vo_grid3d64_bbd64_against_golden(ctx):
    """The benchmark input (64^3, seed 1, 64 parts, BBD with separators):
    layout, ordering arrays, cut metrics and the layout's total walk
    interactions (the numerator of the walk's measured flop rate) equal the
    oracle's, as recorded in golden/vo_grid3d64_bbd64.json."""
    import paper_1105_4490_amd as P
    with open(os.path.join(GOLD, "vo_grid3d64_bbd64.json")) as f:
        gold = json.load(f)
    g = vmo_gen.grid3d(64, seed=1)
    rowptr = torch.as_tensor(g.rowptr).cuda()
    col = torch.as_tensor(g.col).cuda()
    h = ctx.model(P.SYMMETRIC, g.m, g.n, rowptr, col)
    assert (h.k, h.l) == (gold["k"], gold["l"])
    lp = P.layout_params(seed=1)
    ctx.profile(True, every=1)
    ctx.profile_reset()
    x = ctx.layout(h, lp)
    walk = ctx.profile_read("walk")
    ctx.profile(False)
    assert digest(host(x)) == gold["x_sha256"], "64^3 layout not bit-identical"
    assert int(walk["work"]) == gold["layout_interactions"]
    o = ctx.order(h, x, 64, 1, mode=P.GRAPH, order=P.BBD)
    n = int(host(o["n_nodes"])[0])
    assert n == gold["n_nodes"]
    assert digest(host(o["vperm"]).astype(np.int32)) == gold["vperm_sha256"]
    assert digest(host(o["part"]).astype(np.int32)) == gold["part_sha256"]
    assert digest(host(o["node_heap"])[:n].astype(np.int32)) == gold["node_heap_sha256"]
    assert digest(host(o["node_vptr"])[:n + 1].astype(np.int32)) == gold["node_vptr_sha256"]
    assert digest(host(o["split_cut"])[:n].astype(np.float64)) == gold["split_cut_sha256"]
    c = ctx.cut(h, o["part"], 64)
    assert c["cut_net"] == gold["cut_net"] and c["lambda_minus_one"] == gold["lambda_minus_one"]
    # the V+O call (layout inside) gives the same ordering
    o2 = ctx.order(h, None, 64, 1, mode=P.GRAPH, order=P.BBD, lp=lp)
    assert digest(host(o2["vperm"]).astype(np.int32)) == gold["vperm_sha256"]
