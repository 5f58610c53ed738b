"""Oracle pins for the recursive ordering of the border (Sec. 4.2: the cut
rows and columns of a recursive BBD ordering brought into recursive BBD form
by b two-bit words per separator vertex): a hand-derived example
(tests/golden/border_words.json) and, on real graph-mode orderings, the words
recomputed from explicit vertex sets of the split tree instead of heap-id
arithmetic."""
import json
import os

import numpy as np
import pytest

import oracle
import vmo_gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "border_words.json")


def edge_graph(k, edges):
    ptr = np.arange(0, 2 * len(edges) + 1, 2, dtype=np.int64)
    pins = np.array([p for e in edges for p in sorted(e)], dtype=np.int32)
    return oracle.Hypergraph(k, len(edges), ptr, pins)


def test_border_golden():
    g = json.load(open(GOLDEN))
    h = edge_graph(g["k"], g["edges"])
    for b in (0, 1, 2):
        out = oracle.border(h, g["vperm"], g["part"], g["node_heap"], g["node_vptr"], g["n_nodes"], g["P"], b)
        assert out.tolist() == g[f"vperm_b{b}"], b


def test_border_rejects_bad_levels():
    g = json.load(open(GOLDEN))
    h = edge_graph(g["k"], g["edges"])
    with pytest.raises(ValueError):
        oracle.border(h, g["vperm"], g["part"], g["node_heap"], g["node_vptr"], g["n_nodes"], g["P"], 16)


def grid_order(side, P, seed, ord_):
    g = vmo_gen.grid3d(side, seed=seed)
    h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    perm = vmo_gen.rng(seed, 2).permutation(g.n)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(g.n)
    x = np.zeros((4, g.n), np.float32)
    x[0], x[1], x[2] = inv % side, (inv // side) % side, inv // (side * side)
    x += vmo_gen.rng(seed, 3).uniform(-0.2, 0.2, size=x.shape).astype(np.float32)
    return h, oracle.order(h, x, P, seed, mode=oracle.GRAPH_MODE, ord=ord_)


@pytest.mark.parametrize("side,P,seed,ord_,b", [(8, 8, 1, oracle.BBD, 1), (10, 16, 2, oracle.BBD, 2),
                                               (10, 32, 3, oracle.BBD, 3), (9, 12, 4, oracle.SBD, 2)])
def test_border_words_from_vertex_sets(side, P, seed, ord_, b):
    h, o = grid_order(side, P, seed, ord_)
    out = oracle.border(h, o.vperm, o.part, o.node_heap, o.node_vptr, o.n_nodes, P, b)
    heaps = [int(x) for x in o.node_heap[:o.n_nodes]]
    blocks = {heaps[r]: [int(v) for v in o.vperm[o.node_vptr[r]:o.node_vptr[r + 1]]] for r in range(o.n_nodes)}
    sub = {}

    def collect(hh):
        if hh not in blocks:
            return set()
        s = set(blocks[hh]) | collect(2 * hh) | collect(2 * hh + 1)
        sub[hh] = s
        return s
    collect(1)
    nbr = [set() for _ in range(h.k)]
    for a, c in h.nets():
        nbr[a].add(c)
        nbr[c].add(a)
    # the nodes of each depth below a node, as sets of heap ids
    expect = []
    for r in range(o.n_nodes):
        hh = heaps[r]
        blk = blocks[hh]
        if 2 * hh not in blocks:  # a leaf block stays as it is
            expect += blk
            continue
        level = [hh]
        words = {w: 0 for w in blk}
        for i in range(1, b + 1):
            level = [c for g in level for c in (2 * g, 2 * g + 1) if c in blocks]
            # the nodes at depth d + i that split: their first and second parts
            first = set().union(*[sub[2 * g] for g in level if 2 * g in sub])
            second = set().union(*[sub[2 * g + 1] for g in level if 2 * g + 1 in sub])
            for w in blk:
                bits = (1 if nbr[w] & first else 0) | (2 if nbr[w] & second else 0)
                words[w] |= bits << (2 * (b - i))
        expect += sorted(blk, key=lambda w: words[w])  # sorted() is stable
    assert out.tolist() == expect
    # a permutation with the same blocks
    assert sorted(out.tolist()) == list(range(h.k))
    for r in range(o.n_nodes):
        lo, hi = o.node_vptr[r], o.node_vptr[r + 1]
        assert set(out[lo:hi].tolist()) == set(o.vperm[lo:hi].tolist())
