"""GPU parity of the recursive ordering of the border (Sec. 4.2: separator
blocks of a graph-mode ordering sorted by b two-bit words) against the CPU
oracle, through the C ABI: the hand-derived example, grid graphs of several
sizes and part counts in BBD and SBD form, the 64^3 benchmark graph, in-place
output and rejection of inconsistent ordering arrays.  Permutations are
compared bit for bit."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import vmo_gen
from gpu_util import dev_h, dev_x, host

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "border_words.json")


@pytest.fixture(scope="module")
def ctx():
    import paper_1105_4490_amd as P
    return P.Context(0)


def edge_graph(k, edges):
    ptr = np.arange(0, 2 * len(edges) + 1, 2, dtype=np.int64)
    pins = np.array([p for e in edges for p in sorted(e)], dtype=np.int32)
    return oracle.Hypergraph(k, len(edges), ptr, pins)


def dev_i32(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def grid_xyz(side, seed):
    perm = vmo_gen.rng(seed, 2).permutation(side ** 3)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(side ** 3)
    x = np.zeros((4, side ** 3), np.float32)
    x[0], x[1], x[2] = inv % side, (inv // side) % side, inv // (side * side)
    x += vmo_gen.rng(seed, 3).uniform(-0.2, 0.2, size=x.shape).astype(np.float32)
    return x


def test_border_golden_on_gpu(ctx):
    g = json.load(open(GOLDEN))
    h = edge_graph(g["k"], g["edges"])
    o = {"vperm": dev_i32(g["vperm"]), "part": dev_i32(g["part"]), "node_heap": dev_i32(g["node_heap"]),
         "node_vptr": dev_i32(g["node_vptr"]), "n_nodes": dev_i32([g["n_nodes"]])}
    for b in (0, 1, 2):
        got = ctx.order_border(dev_h(h), o, g["P"], b)
        assert host(got).tolist() == g[f"vperm_b{b}"], b


@pytest.mark.parametrize("side,P,seed,ord_,b", [(8, 8, 1, 1, 1), (10, 16, 2, 1, 2), (12, 32, 3, 1, 3),
                                               (11, 12, 4, 0, 2), (16, 64, 5, 1, 4)])
def test_border_parity(ctx, side, P, seed, ord_, b):
    g = vmo_gen.grid3d(side, seed=seed)
    h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    x = grid_xyz(side, seed)
    dh = dev_h(h)
    o = ctx.order(dh, dev_x(x), P, seed, mode=1, order=ord_)
    ref = oracle.order(h, x, P, seed, mode=oracle.GRAPH_MODE, ord=ord_)
    assert np.array_equal(host(o["vperm"]), ref.vperm)
    got = ctx.order_border(dh, o, P, b)
    want = oracle.border(h, ref.vperm, ref.part, ref.node_heap, ref.node_vptr, ref.n_nodes, P, b)
    assert np.array_equal(host(got), want)
    # in place gives the same
    same = ctx.order_border(dh, o, P, b, out=o["vperm"])
    assert np.array_equal(host(same), want)


def test_border_full_size(ctx):
    """The 64^3 7-point graph, symmetric model, 64 parts, BBD, b = 3: exact."""
    side, P, b = 64, 64, 3
    g = vmo_gen.grid3d(side, seed=1)
    h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    x = grid_xyz(side, 1)
    dh = dev_h(h)
    o = ctx.order(dh, dev_x(x), P, 1, mode=1, order=1)
    ref = oracle.order(h, x, P, 1, mode=oracle.GRAPH_MODE, ord=oracle.BBD)
    got = ctx.order_border(dh, o, P, b)
    want = oracle.border(h, ref.vperm, ref.part, ref.node_heap, ref.node_vptr, ref.n_nodes, P, b)
    assert np.array_equal(host(got), want)
    # the separator blocks did move
    assert not np.array_equal(want, ref.vperm)


def test_border_rejects_inconsistent_arrays(ctx):
    import paper_1105_4490_amd as Pk
    g = json.load(open(GOLDEN))
    h = edge_graph(g["k"], g["edges"])
    bad_perm = list(g["vperm"])
    bad_perm[1] = bad_perm[0]  # not a permutation
    o = {"vperm": dev_i32(bad_perm), "part": dev_i32(g["part"]), "node_heap": dev_i32(g["node_heap"]),
         "node_vptr": dev_i32(g["node_vptr"]), "n_nodes": dev_i32([g["n_nodes"]])}
    with pytest.raises(Pk.VmoError):
        ctx.order_border(dev_h(h), o, g["P"], 2)
    o["vperm"] = dev_i32(g["vperm"])
    o["node_heap"] = dev_i32([40] + g["node_heap"][1:])  # heap id beyond 4P
    with pytest.raises(Pk.VmoError):
        ctx.order_border(dev_h(h), o, g["P"], 2)
    o["node_heap"] = dev_i32(g["node_heap"])
    with pytest.raises(Pk.VmoError):
        ctx.order_border(dev_h(h), o, g["P"], 16)  # b out of range
    # a net with three pins is not an edge
    h3 = oracle.Hypergraph(g["k"], 1, np.array([0, 3], np.int64), np.array([0, 1, 2], np.int32))
    with pytest.raises(Pk.VmoError):
        ctx.order_border(dev_h(h3), o, g["P"], 1)
