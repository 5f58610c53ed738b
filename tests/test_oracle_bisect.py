"""Pins for the oracle's quantized 2-means split (Algorithm 4 with m = 2 and
the plane of Algorithm 7): closed-form quantization, the global optimum of
eq. (11) by enumeration on small separated point sets, the Lloyd fixed-point
property in exact rational arithmetic, and the 8 x 4 grid's closed-form SSE."""
import itertools
import json
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import vmo_gen

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_quantize_closed_form():
    x = np.zeros((4, 3), dtype=np.float32)
    x[0] = [0.0, 5.0, 10.0]
    x[1] = [1.0, 2.0, 3.0]
    q, lo, s = oracle.quantize(x)
    assert lo.tolist() == [0.0, 1.0, 0.0, 0.0]
    assert s == (2 ** 20 - 1) / 10.0
    assert q[0].tolist() == [0, 524287, 2 ** 20 - 1]   # floor(5 * 1048575 / 10)
    assert q[1].tolist() == [0, 104857, 209715]        # floor(1 * s), floor(2 * s)
    assert (q[2] == 0).all() and (q[3] == 0).all()


def _sse(P, mask):
    tot = 0.0
    for m in (mask, ~mask):
        if m.any():
            c = P[m].mean(axis=0)
            tot += ((P[m] - c) ** 2).sum()
    return tot


@pytest.mark.parametrize("seed", range(6))
def test_two_means_equals_enumerated_optimum_on_separated_clusters(seed):
    g = vmo_gen.rng(seed, 1)
    n = 12
    a = g.standard_normal((n // 2, 4)) * 0.3
    b = g.standard_normal((n - n // 2, 4)) * 0.3 + np.array([6.0, -3.0, 2.0, 1.0])
    P = np.concatenate([a, b]).astype(np.float32)
    r = oracle.bisect(np.ascontiguousarray(P.T), seed=seed)
    assert r.split
    best = None
    for bits in range(1, 1 << (n - 1)):
        mask = np.array([(bits >> i) & 1 for i in range(n)], dtype=bool)
        s = _sse(P.astype(np.float64), mask)
        if best is None or s < best[0]:
            best = (s, mask)
    got = r.side == 1
    assert np.array_equal(got, best[1]) or np.array_equal(got, ~best[1])


@pytest.mark.parametrize("seed", range(5))
def test_lloyd_result_is_a_fixed_point(seed):
    x = vmo_gen.random_points(400, seed, clusters=3)
    r = oracle.bisect(x, seed=seed)
    assert r.split
    q, lo, s = oracle.quantize(x)
    Q = q.T.astype(np.int64)
    side = r.side
    means = []
    for a in (0, 1):
        sel = Q[side == a]
        assert sel.shape[0] > 0
        means.append([Fraction(int(v), sel.shape[0]) for v in sel.sum(axis=0)])
    # each point is on the side of its nearer centre (exactly), with the
    # tie rule "<= -> part 1"; points whose distance gap is within the FP64
    # rounding of the plane test are skipped
    for i in range(Q.shape[0]):
        d1 = sum((int(Q[i, d]) - means[0][d]) ** 2 for d in range(4))
        d2 = sum((int(Q[i, d]) - means[1][d]) ** 2 for d in range(4))
        if abs(d1 - d2) < Fraction(1, 1000) * (d1 + d2) * Fraction(1, 10 ** 6):
            continue
        assert (side[i] == 0) == (d1 <= d2)
    # reported centres = lo + mean / scale, rounded to FP32
    for a in (0, 1):
        for d in range(4):
            want = np.float32(float(lo[d]) + float(means[a][d]) / s)
            assert r.centres[a, d] == want


def test_grid_8x4_closed_form_and_rownet_root_cut():
    gold = json.load(open(os.path.join(GOLD, "grid8x4_sse.json")))
    cols, rows = 8, 4
    P = np.array([[c, r] for r in range(rows) for c in range(cols)], dtype=np.float64)
    left = P[:, 0] < 4
    assert _sse(P, np.ones(32, bool)) == gold["unsplit"]
    assert _sse(P, left) == gold["split_4_4_columns"]
    assert _sse(P, P[:, 0] < 5) == gold["split_5_3_columns"]
    assert _sse(P, P[:, 1] < 2) == gold["split_2_2_rows"]
    x = np.zeros((4, 32), dtype=np.float32)
    x[0], x[1] = P[:, 0], P[:, 1]
    g = vmo_gen.grid2d(cols, rows)
    h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
    hits = 0
    for seed in range(12):
        r = oracle.bisect(x, seed=seed)
        if not r.split:
            continue
        if _sse(P, r.side == 0) != gold["split_4_4_columns"]:
            continue
        hits += 1
        o = oracle.order(h, x, 2, seed)
        root = list(o.node_heap[:o.n_nodes]).index(1)
        assert o.split_cut[root] == gold["rownet_root_cut_for_4_4"], gold["rownet_why"]
    assert hits >= 3


def test_degenerate_inputs():
    x = np.ones((4, 10), dtype=np.float32)
    assert not oracle.bisect(x, 1).split          # all points coincide
    assert not oracle.bisect(np.zeros((4, 1), np.float32), 1).split
    x = vmo_gen.random_points(2, 3)
    r = oracle.bisect(x, 1)
    assert r.split and sorted(r.side.tolist()) == [0, 1]


def test_seed_determinism_and_dependence():
    x = vmo_gen.random_points(500, 9)
    a, b = oracle.bisect(x, 5), oracle.bisect(x, 5)
    assert np.array_equal(a.side, b.side) and np.array_equal(a.centres, b.centres)
    sides = {oracle.bisect(x, s).side.tobytes() for s in range(8)}
    assert len(sides) >= 2   # a uniform blob has several Lloyd fixed points


def test_d2_draw_index_hand_derived():
    """k-means++ (Algorithm 4, m = 2): golden/d2_draw.json is a case where t
    equals an inclusive prefix sum of the D^2 weights exactly, so the draw
    rule alone decides z2 (the strict rule takes the next point; '>=' or an
    exclusive prefix would take others).  With t_max = 0 the reported centres
    are the seeds themselves; the points sit on the 2^20 grid at scale 1, so
    the centres are the seed points exactly."""
    with open(os.path.join(GOLD, "d2_draw.json")) as f:
        g = json.load(f)
    seed = g["seed"]
    assert oracle.rng(seed, 16, 1, 0) == int(g["r0"]) and oracle.rng(seed, 16, 1, 1) == int(g["r1"])
    q = np.array(g["points_q"], dtype=np.int64)
    # the stored draw, re-derived from its stated definition
    n = g["n"]
    i1 = (int(g["r0"]) * n) >> 64
    d = [int(((q[i] - q[i1]) ** 2).sum()) for i in range(n)]
    T = sum(d)
    t = (int(g["r1"]) * T) >> 64
    assert (i1, [str(v) for v in d], str(T), str(t)) == (g["i1"], g["d"], g["T"], g["t"])
    x = np.ascontiguousarray(q.T.astype(np.float32))
    qq, lo, s = oracle.quantize(x)
    assert s == 1.0 and (lo == 0).all() and np.array_equal(qq, q.T.astype(np.uint32))
    r = oracle.bisect(x, seed=seed, t_max=0)
    assert r.split and r.iters == 0
    assert np.array_equal(r.centres[0], q[g["i1"]].astype(np.float32))
    assert np.array_equal(r.centres[1], q[g["i2"]].astype(np.float32))
    assert g["i2"] not in (g["i2_if_ge"], g["i2_if_exclusive_prefix"])
