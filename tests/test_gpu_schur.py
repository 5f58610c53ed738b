"""GPU parity of the Schur-complement recursion (Sec. 4.2: every separator
block of a graph-mode ordering reordered by the BBD ordering of its induced
graph) against the CPU oracle, through the C ABI: grid graphs of several sizes
and part counts (BBD and SBD outer orderings), the 64^3 benchmark graph,
in-place output, P3 = 1 and rejection of bad input.  Permutations are compared
bit for bit."""
import numpy as np
import pytest
import torch

import oracle
import vmo_gen
from gpu_util import dev_h, dev_x, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1105_4490_amd as P
    return P.Context(0)


def grid_case(side, seed):
    g = vmo_gen.grid3d(side, seed=seed)
    h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    perm = vmo_gen.rng(seed, 2).permutation(g.n)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(g.n)
    x = np.zeros((4, g.n), np.float32)
    x[0], x[1], x[2] = inv % side, (inv // side) % side, inv // (side * side)
    x += vmo_gen.rng(seed, 3).uniform(-0.3, 0.3, size=x.shape).astype(np.float32)
    return h, x


def run_case(ctx, side, P, P3, seed, ord_):
    h, x = grid_case(side, seed)
    dh, dx = dev_h(h), dev_x(x)
    o = ctx.order(dh, dx, P, seed, mode=1, order=ord_)
    ref = oracle.order(h, x, P, seed, mode=oracle.GRAPH_MODE, ord=ord_)
    assert np.array_equal(host(o["vperm"]), ref.vperm)
    got = ctx.order_schur(dh, dx, o, P, P3, seed)
    want = oracle.schur(h, x, ref.vperm, ref.part, ref.node_heap, ref.node_vptr, ref.n_nodes, P, P3, seed)
    return h, dh, dx, o, ref, got, want


@pytest.mark.parametrize("side,P,P3,seed,ord_", [(8, 8, 2, 1, 1), (10, 16, 4, 2, 1), (12, 32, 8, 3, 1),
                                                 (11, 12, 3, 4, 0), (16, 64, 16, 5, 1), (9, 5, 64, 6, 1)])
def test_schur_parity(ctx, side, P, P3, seed, ord_):
    h, dh, dx, o, ref, got, want = run_case(ctx, side, P, P3, seed, ord_)
    assert np.array_equal(host(got), want)
    assert not np.array_equal(want, ref.vperm)
    # in place gives the same
    same = ctx.order_schur(dh, dx, o, P, P3, seed, out=o["vperm"])
    assert np.array_equal(host(same), want)


def test_schur_one_part_is_a_copy(ctx):
    h, x = grid_case(8, 7)
    dh, dx = dev_h(h), dev_x(x)
    o = ctx.order(dh, dx, 8, 7, mode=1, order=1)
    got = ctx.order_schur(dh, dx, o, 8, 1, 7)
    assert np.array_equal(host(got), host(o["vperm"]))
    ref = oracle.order(h, x, 8, 7, mode=oracle.GRAPH_MODE, ord=oracle.BBD)
    want = oracle.schur(h, x, ref.vperm, ref.part, ref.node_heap, ref.node_vptr, ref.n_nodes, 8, 1, 7)
    assert np.array_equal(host(got), want)


def test_schur_full_size(ctx):
    """The 64^3 7-point graph, symmetric model, 64 parts, BBD; every
    separator block ordered into 8 parts: exact."""
    h, dh, dx, o, ref, got, want = run_case(ctx, 64, 64, 8, 1, 1)
    assert np.array_equal(host(got), want)
    assert not np.array_equal(want, ref.vperm)


def test_schur_rejects_bad_input(ctx):
    import paper_1105_4490_amd as Pk
    h, x = grid_case(8, 1)
    dh, dx = dev_h(h), dev_x(x)
    o = ctx.order(dh, dx, 8, 1, mode=1, order=1)
    with pytest.raises(Pk.VmoError):
        ctx.order_schur(dh, dx, o, 8, 0, 1)  # P3 < 1
    xb = x.copy()
    xb[2, 5] = np.nan
    with pytest.raises(Pk.VmoError):
        ctx.order_schur(dh, dev_x(xb), o, 8, 2, 1)
    bad = dict(o)
    vp = host(o["vperm"]).copy()
    vp[1] = vp[0]  # not a permutation
    bad["vperm"] = torch.as_tensor(vp).cuda()
    with pytest.raises(Pk.VmoError):
        ctx.order_schur(dh, dx, bad, 8, 2, 1)
    # a net with three pins is not an edge
    h3 = oracle.Hypergraph(h.k, 1, np.array([0, 3], np.int64), np.array([0, 1, 2], np.int32))
    with pytest.raises(Pk.VmoError):
        ctx.order_schur(dev_h(h3), dx, o, 8, 2, 1)
