"""Pins for the oracle's cut metrics: the hand-worked cuts of the Fig. 2
hypergraph and its dual, brute-force minimum bisections, and a set-based
recount on random weighted hypergraphs."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
import vmo_gen

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _f2():
    d = json.load(open(os.path.join(GOLD, "f2_hypergraph.json")))
    return d, oracle.hypergraph(d["k"], d["nets"])


def test_f2_hand_worked_cuts():
    d, h = _f2()
    for case in d["cuts"]:
        r = oracle.cut(h, np.array(case["part"]), 2)
        assert r["lambda_minus_one"] == case["lambda_minus_one"], case["why"]
        assert r["cut_net"] == case["cut_net"], case["why"]
        assert r["part_weight"].sum() == 5.0


def test_f2_brute_force_minimum_bisection():
    d, h = _f2()
    best = None
    arg = []
    for mask in range(1 << 5):
        part = np.array([(mask >> v) & 1 for v in range(5)])
        if part.sum() not in (2, 3):
            continue
        c = oracle.cut(h, part, 2)["lambda_minus_one"]
        if best is None or c < best:
            best, arg = c, []
        if c == best:
            arg.append(frozenset(np.nonzero(part == 0)[0]))
    assert best == d["min_bisection_lambda_minus_one_sizes_2_3"], d["min_bisection_why"]
    # the three splits listed with the example: {1,2}|{3,4,5}, {1,2,5}|{3,4}, {1,5}|{2,3,4}
    want = [{0, 1}, {0, 1, 4}, {0, 4}]
    got = {frozenset(s) for s in arg}
    for s in want:
        comp = frozenset(set(range(5)) - s)
        assert frozenset(s) in got or comp in got
    # unrestricted minimum: {5} alone gives 0
    assert oracle.cut(h, np.array([0, 0, 0, 0, 1]), 2)["lambda_minus_one"] == 0


def test_f2_dual_cut():
    d, h = _f2()
    du = oracle.dual(h)
    r = oracle.cut(du, np.array(d["dual_cut"]["part"]), 2)
    assert r["lambda_minus_one"] == d["dual_cut"]["lambda_minus_one"], d["dual_cut"]["why"]


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_cut_against_set_recount(seed):
    g = vmo_gen.random_hypergraph_csr(60, 80, seed, maxdeg=7, empty_frac=0.1)
    h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
    r = vmo_gen.rng(seed, 99)
    h.c = r.integers(1, 5, size=h.l).astype(np.float32)
    h.w = r.integers(1, 4, size=h.k).astype(np.float32)
    P = 5
    part = r.integers(0, P, size=h.k).astype(np.int32)
    got = oracle.cut(h, part, P)
    lm1 = cn = 0.0
    for e, net in enumerate(h.nets()):
        lam = len({int(part[v]) for v in net})
        lm1 += h.c[e] * max(lam - 1, 0)
        cn += h.c[e] * (lam > 1)
    assert got["lambda_minus_one"] == lm1
    assert got["cut_net"] == cn
    pw = np.zeros(P)
    for v in range(h.k):
        pw[part[v]] += h.w[v]
    assert np.array_equal(got["part_weight"], pw)
    assert got["part_weight"].sum() == h.w.sum()


def test_cut_minimum_over_bisections_small():
    """On a 6-vertex path of 2-pin nets the minimum balanced bisection cuts 1 net."""
    h = oracle.hypergraph(6, [[i, i + 1] for i in range(5)])
    best = min(oracle.cut(h, np.array(p), 2)["cut_net"]
               for p in itertools.product([0, 1], repeat=6) if sum(p) == 3)
    assert best == 1


def test_split_cuts_hand_worked():
    """Recursive bisection into P = 3 parts: the root holds parts [0, 3),
    child 2 the parts [0, 2), child 3 part 2; node 2's children 4 and 5 hold
    parts 0 and 1.  Nets {0,1} (parts 0,1) are cut at node 2, {1,2} (parts
    1,2) at the root, {0,3} (parts 0,0) nowhere, {3,4} (parts 0,1) at node 2;
    costs 1, 2, 4, 8 give split = {1: 2, 2: 1 + 8}."""
    h = oracle.hypergraph(5, [[0, 1], [1, 2], [0, 3], [3, 4]], c=[1, 2, 4, 8])
    part = np.array([0, 1, 2, 0, 1], dtype=np.int32)
    sp, graph = oracle.split_cuts(h, part, 3)
    assert not graph
    want = np.zeros(12)
    want[1], want[2] = 2, 9
    assert np.array_equal(sp, want)
    # with separator ids (P + h): the sizes of the separators
    part2 = np.array([0, 3 + 1, 2, 3 + 2, 3 + 1], dtype=np.int32)
    sp2, graph2 = oracle.split_cuts(h, part2, 3)
    assert graph2 and sp2[1] == 2 and sp2[2] == 1 and sp2.sum() == 3


@pytest.mark.parametrize("seed,mode,P", [(1, 0, 13), (2, 0, 64), (3, 1, 16), (4, 1, 7)])
def test_split_cuts_equal_the_orderings_own(seed, mode, P):
    """The per-split cut recovered from part ids alone equals the one the
    recursive ordering records while it splits (nets placed at the node that
    cuts them, separators at their node), node by node."""
    if mode == 0:
        g = vmo_gen.random_hypergraph_csr(600, 400, seed, maxdeg=5)
        h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
        h.c = vmo_gen.rng(seed, 12).integers(1, 5, size=h.l).astype(np.float32)
    else:
        g = vmo_gen.grid3d(9, seed=seed)
        h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    x = vmo_gen.random_points(h.k, seed, clusters=5)
    o = oracle.order(h, x, P, seed, mode=mode, ord=oracle.BBD)
    sp, graph = oracle.split_cuts(h, o.part, P)
    assert graph == (mode == 1 and (o.part >= P).any())
    rec = np.zeros(4 * P)
    for r in range(o.n_nodes):
        rec[o.node_heap[r]] = o.split_cut[r]
    assert np.array_equal(sp, rec)
