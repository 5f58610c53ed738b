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
