"""GPU parity of the Kernighan-Lin refinement (Sec. 3; Kernighan and Lin
1970) against the CPU oracle, through the C ABI: the hand-derived pass
sequence, two cliques, random multigraphs with several bisections and
left-out vertices, 2-means bisections of grid graphs (labels and gains
exact); at the benchmark size (64 bisections of the 64^3 graph) the
properties that hold at any size: side sizes and membership kept, gains equal
to the recounted cut reductions, and after convergence no pair swap that
lowers a cut."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import vmo_gen
from gpu_util import dev_h, host

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "kl_path4.json")


@pytest.fixture(scope="module")
def ctx():
    import paper_1105_4490_amd as P
    return P.Context(0)


def edge_graph(k, edges):
    edges = [tuple(sorted(e)) for e in edges]
    ptr = np.arange(0, 2 * len(edges) + 1, 2, dtype=np.int64)
    pins = np.array([p for e in edges for p in e], dtype=np.int32)
    return oracle.Hypergraph(k, len(edges), ptr, pins)


def dlabel(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def run_both(ctx, h, label, passes):
    want, wgain = oracle.refine_kl(h, label, passes)
    got, ggain = ctx.refine_kl(dev_h(h), dlabel(label), passes)
    assert np.array_equal(host(got), want)
    assert np.array_equal(host(ggain), wgain)
    return want, wgain


def test_kl_golden(ctx):
    g = json.load(open(GOLDEN))
    h = edge_graph(g["k"], g["edges"])
    got, gain = ctx.refine_kl(dev_h(h), dlabel(g["label_in"]), 8)
    assert host(got).tolist() == g["label_out"] and host(gain).tolist() == g["gain"]


def test_kl_two_cliques(ctx):
    edges = [(a, b) for a in range(5) for b in range(a + 1, 5)]
    edges += [(a, b) for a in range(5, 10) for b in range(a + 1, 10)] + [(4, 5)]
    run_both(ctx, edge_graph(10, edges), [0, 0, 0, 1, 1, 1, 1, 1, 0, 0], 4)


def random_case(k, l, G, seed):
    r = vmo_gen.rng(seed, 9)
    a = r.integers(0, k, size=l)
    b = r.integers(0, k, size=l)
    keep = a != b
    edges = [(int(min(x, y)), int(max(x, y))) for x, y in zip(a[keep], b[keep])]   # parallel edges kept
    r2 = vmo_gen.rng(seed, 10)
    label = np.where(r2.random(k) < 0.1, -1, 2 * r2.integers(0, G, size=k) + r2.integers(0, 2, size=k))
    return edge_graph(k, edges), label.astype(np.int32)


@pytest.mark.parametrize("k,l,G,seed,passes", [(60, 150, 1, 1, 3), (200, 500, 3, 2, 50), (300, 700, 5, 3, 2),
                                               (120, 600, 2, 4, 50), (600, 1500, 1, 5, 4), (900, 2000, 7, 6, 50)])
def test_kl_random_parity(ctx, k, l, G, seed, passes):
    h, label = random_case(k, l, G, seed)
    run_both(ctx, h, label, passes)


@pytest.mark.parametrize("side,seed", [(24, 1), (30, 2)])
def test_kl_grid_bisection_parity(ctx, side, seed):
    """2-means bisection (the oracle's) of a 2-D grid at jittered points."""
    g = vmo_gen.grid2d(side)
    h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    ids = np.arange(g.m)
    x = np.zeros((4, g.m), np.float32)
    x[0], x[1] = ids % side, ids // side
    x += vmo_gen.rng(seed, 3).uniform(-0.45, 0.45, size=x.shape).astype(np.float32)
    b = oracle.bisect(x, seed)
    label = b.side.astype(np.int32)
    want, gain = run_both(ctx, h, label, 20)
    assert int(gain[0]) >= 0


def cut_of(edges, label, G):
    la, lb = label[edges[:, 0]], label[edges[:, 1]]
    inside = (la >= 0) & (lb >= 0) & ((la >> 1) == (lb >> 1))
    cutm = inside & (la != lb)
    return np.bincount(la[cutm] >> 1, minlength=G)


def no_improving_swap(edges, label, g):
    A = np.nonzero(label == 2 * g)[0]
    B = np.nonzero(label == 2 * g + 1)[0]
    inside = (label[edges[:, 0]] >> 1 == g) & (label[edges[:, 1]] >> 1 == g) & (label[edges[:, 0]] >= 0) & \
             (label[edges[:, 1]] >= 0)
    e = edges[inside]
    D = np.zeros(label.size, np.int64)
    diff = label[e[:, 0]] != label[e[:, 1]]
    np.add.at(D, e[:, 0], np.where(diff, 1, -1))
    np.add.at(D, e[:, 1], np.where(diff, 1, -1))
    top = D[A].max() + D[B].max()
    if top <= 0:
        return True
    mult = {}
    for a, b in e[diff].tolist():
        key = (a, b) if label[a] == 2 * g else (b, a)
        mult[key] = mult.get(key, 0) + 1
    ca = A[D[A] + D[B].max() > 0]
    cb = B[D[B] + D[A].max() > 0]
    for a in ca.tolist():
        for b in cb.tolist():
            if D[a] + D[b] - 2 * mult.get((a, b), 0) > 0:
                return False
    return True


def test_kl_full_size_properties(ctx):
    """The 64^3 7-point graph cut into 64 blocks of 16^3 grid points; each
    block bisected by a tilted plane through its middle (jittered); passes
    until convergence."""
    side = 64
    g = vmo_gen.grid3d(side, seed=1)
    h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    perm = vmo_gen.rng(1, 2).permutation(g.m)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(g.m)
    gx, gy, gz = inv % side, (inv // side) % side, inv // (side * side)
    block = (gx // 16) + 4 * (gy // 16) + 16 * (gz // 16)
    r = vmo_gen.rng(7, 1)
    lx, ly, lz = gx % 16, gy % 16, gz % 16
    t = lx + 0.5 * ly + 0.25 * lz + r.uniform(-2, 2, size=g.m)
    label = (2 * block + (t > np.median(t))).astype(np.int32)
    got, gain = ctx.refine_kl(dev_h(h), dlabel(label), 100)
    out, gain = host(got), host(gain)
    edges = h.pins.reshape(-1, 2).astype(np.int64)
    assert gain.shape == (64,)
    before, after = cut_of(edges, label, 64), cut_of(edges, out, 64)
    assert np.array_equal(gain, before - after) and (gain >= 0).all() and gain.sum() > 0
    for gg in range(64):
        assert np.array_equal(np.sort(label[label >> 1 == gg] & 1), np.sort(out[out >> 1 == gg] & 1))
    assert np.array_equal(label >> 1, out >> 1)
    for gg in (0, 21, 42, 63):
        assert no_improving_swap(edges, out, gg)


def test_kl_rejects(ctx):
    import paper_1105_4490_amd as Pk
    h = edge_graph(4, [(0, 1), (1, 2)])
    with pytest.raises(Pk.VmoError):
        ctx.refine_kl(dev_h(h), dlabel([0, 1, -2, 0]), 1)
    h3 = oracle.Hypergraph(4, 1, np.array([0, 3], np.int64), np.array([0, 1, 2], np.int32))
    with pytest.raises(Pk.VmoError):
        ctx.refine_kl(dev_h(h3), dlabel([0, 1, 0, 1]), 1)
    got, gain = ctx.refine_kl(dev_h(h), dlabel([-1, -1, -1, -1]), 3)
    assert host(got).tolist() == [-1] * 4 and host(gain).size == 0


def test_kl_large_bisection_in_device_memory(ctx):
    """A bisection above 9,216 vertices keeps its state in device memory
    instead of LDS: a 110 x 110 grid, random sides, two passes; side sizes
    kept and the gain equal to the recounted cut reduction."""
    side = 110
    g = vmo_gen.grid2d(side)
    h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    label = vmo_gen.rng(3, 4).integers(0, 2, size=g.m).astype(np.int32)
    got, gain = ctx.refine_kl(dev_h(h), dlabel(label), 2)
    out, gain = host(got), host(gain)
    edges = h.pins.reshape(-1, 2).astype(np.int64)
    assert int(gain[0]) == int(cut_of(edges, label, 1)[0] - cut_of(edges, out, 1)[0]) > 0
    assert int((out == 1).sum()) == int((label == 1).sum())
