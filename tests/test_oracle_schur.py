"""Oracle pins for the Schur-complement recursion (Sec. 4.2: Algorithm 7
applied recursively to G3 = (V3, E'3), the graph of a separator and the edges
inside it).  The induced graphs, local ids, net order and composition are
rebuilt here from sets and compared with o_schur; the reordered blocks are
checked to be recursive BBD orderings of their own graphs (no edge between the
two halves of a split) and to keep their vertex sets, and leaf blocks do not
move."""
import numpy as np
import pytest

import oracle
import vmo_gen


def grid_order(side, P, seed):
    g = vmo_gen.grid3d(side, seed=seed)
    h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    perm = vmo_gen.rng(seed, 2).permutation(g.n)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(g.n)
    x = np.zeros((4, g.n), np.float32)
    x[0], x[1], x[2] = inv % side, (inv // side) % side, inv // (side * side)
    x += vmo_gen.rng(seed, 3).uniform(-0.3, 0.3, size=x.shape).astype(np.float32)
    return h, x, oracle.order(h, x, P, seed, mode=oracle.GRAPH_MODE, ord=oracle.BBD)


@pytest.mark.parametrize("side,P,P3,seed", [(8, 8, 2, 1), (10, 16, 4, 2), (12, 32, 8, 3)])
def test_schur_rebuilt_from_sets(side, P, P3, seed):
    h, x, o = grid_order(side, P, seed)
    out = oracle.schur(h, x, o.vperm, o.part, o.node_heap, o.node_vptr, o.n_nodes, P, P3, seed)
    edges = [tuple(e) for e in h.nets()]
    expect = o.vperm.copy()
    moved = 0
    for r in range(o.n_nodes):
        lo, hi = int(o.node_vptr[r]), int(o.node_vptr[r + 1])
        blk = [int(v) for v in o.vperm[lo:hi]]
        if len(blk) < 2 or o.part[blk[0]] < P:
            continue
        local = {v: i for i, v in enumerate(blk)}
        nets = [sorted((local[a], local[b])) for a, b in edges if a in local and b in local]
        sub = oracle.hypergraph(len(blk), nets)
        xs = x[:, blk]
        so = oracle.order(sub, xs, P3, seed, mode=oracle.GRAPH_MODE, ord=oracle.BBD, job=int(o.node_heap[r]))
        expect[lo:hi] = np.array(blk)[so.vperm]
        moved += int((expect[lo:hi] != o.vperm[lo:hi]).any())
        # the sub-ordering is a BBD of the block's graph: no edge joins the
        # vertex sets of the two subtrees of any internal node
        heaps = [int(t) for t in so.node_heap[:so.n_nodes]]
        blocks = {heaps[t]: set(so.vperm[so.node_vptr[t]:so.node_vptr[t + 1]].tolist()) for t in range(so.n_nodes)}

        def subtree(hh):
            if hh not in blocks:
                return set()
            return blocks[hh] | subtree(2 * hh) | subtree(2 * hh + 1)
        for hh in heaps:
            if 2 * hh in blocks:
                L, R = subtree(2 * hh), subtree(2 * hh + 1)
                assert not any((a in L and b in R) or (a in R and b in L) for a, b in nets)
    assert out.tolist() == expect.tolist()
    assert moved > 0
    assert sorted(out.tolist()) == list(range(h.k))
    for r in range(o.n_nodes):
        lo, hi = o.node_vptr[r], o.node_vptr[r + 1]
        assert set(out[lo:hi].tolist()) == set(o.vperm[lo:hi].tolist())
        if hi > lo and o.part[o.vperm[lo]] < P:
            assert np.array_equal(out[lo:hi], o.vperm[lo:hi])


def test_schur_one_part_keeps_order():
    """P3 = 1: every separator is a single leaf of its own ordering, which
    lists its vertices in ascending id: the blocks become sorted by id."""
    h, x, o = grid_order(8, 8, 4)
    out = oracle.schur(h, x, o.vperm, o.part, o.node_heap, o.node_vptr, o.n_nodes, 8, 1, 4)
    for r in range(o.n_nodes):
        lo, hi = o.node_vptr[r], o.node_vptr[r + 1]
        blk = o.vperm[lo:hi]
        if hi - lo >= 2 and o.part[blk[0]] >= 8:
            assert np.array_equal(out[lo:hi], np.sort(blk))
