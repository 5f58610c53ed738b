"""Pins for the oracle's recursive SBD/BBD ordering (Algorithm 7 applied
recursively, Sec. 4.1-4.2, Sec. 5): permutations are bijections, weights
add up, each net sits at the lowest common ancestor of its pins' leaves
(recomputed here from heap ids), graph-mode separators leave no edge
between the two sides of any split (caption of Algorithm 7), and the fill-in
example of Sec. 4 goes from 6 fill entries to 0."""
import json
import os

import numpy as np
import pytest

import oracle
import vmo_gen

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def blocks(o, k):
    """heap id -> list of vertices in its emitted block."""
    out = {}
    for r in range(o.n_nodes):
        out[int(o.node_heap[r])] = o.vperm[o.node_vptr[r]:o.node_vptr[r + 1]].tolist()
    return out


def leaf_of(o, k):
    lf = np.full(k, -1)
    for h, vs in blocks(o, k).items():
        lf[vs] = h
    return lf


def lca(a, b):
    while a != b:
        if a > b:
            a //= 2
        else:
            b //= 2
    return a


def check_common(h, o, P):
    k = h.k
    assert sorted(o.vperm.tolist()) == list(range(k))
    assert o.node_vptr[0] == 0 and o.node_vptr[o.n_nodes] == k
    assert (np.diff(o.node_vptr[:o.n_nodes + 1]) >= 0).all()
    heaps = o.node_heap[:o.n_nodes].tolist()
    assert len(set(heaps)) == len(heaps) and 1 in heaps
    for hh in heaps:                       # every node's parent exists
        assert hh == 1 or hh // 2 in heaps
    assert all(hh < 4 * P for hh in heaps)
    # parts: leaves get ids in [0, P), separators P + heap id
    for hh, vs in blocks(o, k).items():
        for v in vs:
            assert o.part[v] in (range(P) if 2 * hh not in heaps else [P + hh])


def emitted_order_ok(o, post):
    """in-order (SBD) or post-order (BBD) of the heap tree."""
    heaps = set(o.node_heap[:o.n_nodes].tolist())
    seq = []

    def walk(hh):
        if hh not in heaps:
            return
        internal = 2 * hh in heaps
        if not internal:
            seq.append(hh)
            return
        walk(2 * hh)
        if not post:
            seq.append(hh)
        walk(2 * hh + 1)
        if post:
            seq.append(hh)
    walk(1)
    return seq == o.node_heap[:o.n_nodes].tolist()


@pytest.mark.parametrize("seed,P,ord_", [(1, 16, oracle.SBD), (2, 13, oracle.BBD), (3, 5, oracle.SBD), (4, 1, oracle.BBD)])
def test_net_mode_invariants_and_lca(seed, P, ord_):
    g = vmo_gen.zipf_rect(300, 200, seed, clip=30)
    h = oracle.colnet(g.m, g.n, g.rowptr, g.col)
    x = vmo_gen.random_points(h.k, seed, clusters=6)
    o = oracle.order(h, x, P, seed, mode=oracle.NET_MODE, ord=ord_)
    check_common(h, o, P)
    assert emitted_order_ok(o, ord_ == oracle.BBD)
    assert sorted(o.nperm.tolist()) == list(range(h.l))
    lf = leaf_of(o, h.k)
    heaps = o.node_heap[:o.n_nodes].tolist()
    netnode = {}
    for r in range(o.n_nodes):
        for e in o.nperm[o.node_nptr[r]:o.node_nptr[r + 1]]:
            netnode[int(e)] = heaps[r]
    empty = set(o.nperm[o.node_nptr[o.n_nodes]:].tolist())
    for e, net in enumerate(h.nets()):
        if len(net) == 0:
            assert e in empty
            continue
        a = int(lf[net[0]])
        for v in net[1:]:
            a = lca(a, int(lf[v]))
        assert netnode[e] == a
    # within a block nets ascend; the cut at a node counts its nets
    for r in range(o.n_nodes):
        blk = o.nperm[o.node_nptr[r]:o.node_nptr[r + 1]]
        assert (np.diff(blk) > 0).all()
        internal = 2 * heaps[r] in heaps
        assert o.split_cut[r] == (len(blk) if internal else 0)
    cut = oracle.cut(h, o.part, P)
    assert o.split_cut.sum() == cut["cut_net"]
    assert cut["part_weight"].sum() == h.k


@pytest.mark.parametrize("seed,P,ord_", [(5, 8, oracle.BBD), (6, 6, oracle.SBD), (7, 64, oracle.BBD)])
def test_graph_mode_separators(seed, P, ord_):
    g = vmo_gen.grid3d(8, seed=seed)
    h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    # the true grid coordinates, un-permuted, as a given geometry
    perm = vmo_gen.rng(seed, 2).permutation(g.n)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(g.n)
    i = inv
    x = np.zeros((4, g.n), np.float32)
    x[0], x[1], x[2] = i % 8, (i // 8) % 8, i // 64
    o = oracle.order(h, x, P, seed, mode=oracle.GRAPH_MODE, ord=ord_)
    check_common(h, o, P)
    assert emitted_order_ok(o, ord_ == oracle.BBD)
    heaps = o.node_heap[:o.n_nodes].tolist()
    bl = blocks(o, h.k)
    sub = {}

    def collect(hh):
        if hh not in bl:
            return set()
        s = set(bl[hh]) | collect(2 * hh) | collect(2 * hh + 1)
        sub[hh] = s
        return s
    collect(1)
    nbr = [set() for _ in range(h.k)]
    for a, b in h.nets():
        nbr[a].add(b)
        nbr[b].add(a)
    for hh in heaps:
        if 2 * hh not in heaps:
            continue
        L, R = sub.get(2 * hh, set()), sub.get(2 * hh + 1, set())
        for v in L:
            assert not (nbr[v] & R)
        # the separator size is the split's cut
        assert o.split_cut[heaps.index(hh)] == len(bl[hh])
        # every separator vertex was put there for an edge across the plane:
        # it touches the node's own vertex set
        for v in bl[hh]:
            assert nbr[v] & (L | R | set(bl[hh]))


def symbolic_fill(A):
    """Fill entries of Gaussian elimination without pivoting (Algorithm 5
    without the pivot search) on a boolean pattern."""
    A = A.copy()
    n = A.shape[0]
    fill = 0
    for kk in range(n):
        for i in range(kk + 1, n):
            if not A[i, kk]:
                continue
            for j in range(kk + 1, n):
                if A[kk, j] and not A[i, j]:
                    A[i, j] = True
                    fill += 1
    return fill


def test_arrowhead_fill_example():
    gold = json.load(open(os.path.join(GOLD, "arrowhead_fill.json")))
    A = np.array(gold["pattern"], dtype=bool)
    assert symbolic_fill(A) == gold["fill_original_order"]
    h = oracle.hypergraph(4, [[0, 1], [0, 2], [0, 3]])
    x = np.zeros((4, 4), np.float32)
    x[0] = [0.0, -2.0, 2.0, 2.0]
    x[1] = [0.0, 0.0, 0.5, -0.5]
    for seed in range(4):
        o = oracle.order(h, x, 2, seed, mode=oracle.GRAPH_MODE, ord=oracle.BBD)
        assert o.vperm[-1] == 0                        # the hub is the separator, placed last
        B = A[np.ix_(o.vperm, o.vperm)]
        assert symbolic_fill(B) == gold["fill_hub_last"], gold["why"]


def test_sbd_and_bbd_share_blocks():
    g = vmo_gen.grid2d(16)
    h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
    x = vmo_gen.random_points(h.k, 3)
    a = oracle.order(h, x, 8, 2, ord=oracle.SBD)
    b = oracle.order(h, x, 8, 2, ord=oracle.BBD)
    ba, bb = blocks(a, h.k), blocks(b, h.k)
    assert ba == bb


def test_degenerate_orders():
    h = oracle.hypergraph(1, [[0], []])
    o = oracle.order(h, np.zeros((4, 1), np.float32), 4, 1)
    assert o.n_nodes == 1 and o.vperm.tolist() == [0] and o.nperm.tolist() == [0, 1]
    h = oracle.hypergraph(6, [[0, 1], [2, 3, 4, 5]])
    o = oracle.order(h, np.ones((4, 6), np.float32), 4, 1)   # coincident points: unsplittable
    assert o.n_nodes == 1 and o.part.tolist() == [0] * 6
    with pytest.raises(ValueError):
        oracle.order(oracle.hypergraph(3, [[0, 1, 2]]), np.zeros((4, 3), np.float32), 2, 1, mode=oracle.GRAPH_MODE)


def test_job_index_changes_seeding():
    x = vmo_gen.random_points(2000, 4)
    g = vmo_gen.random_hypergraph_csr(2000, 500, 1)
    h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
    a = oracle.order(h, x, 16, 3, job=0)
    b = oracle.order(h, x, 16, 3, job=0)
    c = oracle.order(h, x, 16, 3, job=1)
    assert np.array_equal(a.vperm, b.vperm)
    assert not np.array_equal(a.vperm, c.vperm)
