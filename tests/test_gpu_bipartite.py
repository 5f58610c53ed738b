"""GPU parity of the strengthened diagonal (Sec. 4.2, Sec. 5) against the CPU
oracle, through the C ABI: the bipartite model (exact); the heavy edge
matching (exact: the greedy matching of a strict order is unique); the
augmentation (several maximum matchings are correct: the size is compared
with the oracle's Hopcroft-Karp and the GPU matching is checked to be a valid
matching of the pattern); Algorithm 7 with matched pairs on bipartite graphs
of grids up to the 64^3 benchmark matrix (exact, with the oracle's matching as
the input of both sides); the Schur-complement recursion with the matching;
row and column permutations; finegrain coordinates (exact)."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import oracle
import vmo_gen
from gpu_util import compare_order, dev_h, dev_x, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1105_4490_amd as P
    return P.Context(0)


def dev(a, dt=None):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=dt)).cuda()


def random_pattern(m, n, density, seed, diag=False):
    r = vmo_gen.rng(seed, 1)
    a = r.random((m, n)) < density
    if diag:
        a[np.arange(min(m, n)), np.arange(min(m, n))] = True
    A = sp.csr_matrix(a.astype(np.float32))
    A.sort_indices()
    return A.indptr.astype(np.int64), A.indices.astype(np.int32)


def pattern_case(name):
    if name.startswith("rand"):
        _, m, n, d, seed = name.split(":")
        m, n, seed = int(m), int(n), int(seed)
        rp, cc = random_pattern(m, n, float(d), seed)
        return m, n, rp, cc
    if name.startswith("grid3d"):
        side = int(name.split(":")[1])
        g = vmo_gen.grid3d(side, seed=1)
    else:
        g = vmo_gen.grid2d(int(name.split(":")[1]))
    return g.m, g.n, g.rowptr.astype(np.int64), g.col.astype(np.int32)


def check_valid(m, n, rp, cc, mrow, mcol):
    edges = set(zip(np.repeat(np.arange(m), np.diff(rp)).tolist(), cc.tolist()))
    for i in range(m):
        j = int(mrow[i])
        if j >= 0:
            assert (i, j) in edges and mcol[j] == i
    assert int((mrow >= 0).sum()) == int((mcol >= 0).sum())


@pytest.mark.parametrize("name", ["rand:7:5:0.4:1", "rand:40:90:0.05:2", "grid2d:20"])
def test_bipartite_model(ctx, name):
    import paper_1105_4490_amd as P
    m, n, rp, cc = pattern_case(name)
    h = oracle.bipartite(m, n, rp, cc)
    g = ctx.model(P.BIPARTITE, m, n, dev(rp), dev(cc))
    assert (g.k, g.l) == (h.k, h.l)
    assert np.array_equal(host(g.net_ptr), h.ptr)
    assert np.array_equal(host(g.pins), h.pins)


@pytest.mark.parametrize("name,weights,seed", [("rand:60:60:0.05:1", "none", 0), ("rand:300:250:0.01:2", "ties", 5),
                                               ("rand:200:200:0.02:3", "distinct", 9), ("grid2d:40", "none", 3),
                                               ("grid3d:24", "diag", 1), ("grid3d:64", "none", 2)])
def test_match_heavy_exact(ctx, name, weights, seed):
    m, n, rp, cc = pattern_case(name)
    nnz = int(rp[-1])
    r = vmo_gen.rng(seed, 8)
    a = None
    if weights == "ties":
        a = r.integers(-3, 4, size=nnz).astype(np.float32)          # zeros and equal magnitudes
    elif weights == "distinct":
        a = ((r.permutation(nnz) + 1) * np.where(r.random(nnz) < 0.5, -1, 1)).astype(np.float32)
    elif weights == "diag":
        rows = np.repeat(np.arange(m), np.diff(rp))
        a = np.where(rows == cc, 6.0, -1.0).astype(np.float32) + r.uniform(-0.1, 0.1, nnz).astype(np.float32)
    er, ec, es = oracle.match_heavy(m, n, rp, cc, a, seed=seed)
    g = ctx.match(m, n, dev(rp), dev(cc), None if a is None else dev(a, np.float32), seed=seed, augment=False)
    assert g["size"] == es
    assert np.array_equal(host(g["mrow"]), er)
    assert np.array_equal(host(g["mcol"]), ec)
    mu = host(g["mu"])
    assert np.array_equal(mu, oracle.mu_of(m, n, er, ec))
    if weights == "diag":
        assert es == m and np.array_equal(er, np.arange(m))


@pytest.mark.parametrize("name,seed", [("rand:60:60:0.04:1", 1), ("rand:80:70:0.03:2", 2), ("rand:400:400:0.004:3", 3),
                                       ("rand:500:300:0.006:4", 4), ("grid2d:40", 5), ("grid3d:20", 6),
                                       ("grid3d:64", 7)])
def test_match_augmented_is_maximum(ctx, name, seed):
    m, n, rp, cc = pattern_case(name)
    _, _, size = oracle.match(m, n, rp, cc, None, seed=seed)
    g = ctx.match(m, n, dev(rp), dev(cc), None, seed=seed, augment=True)
    mrow, mcol = host(g["mrow"]), host(g["mcol"])
    assert g["size"] == size
    if m * n <= 10 ** 6 or name.startswith("grid"):
        check_valid(m, n, rp, cc, mrow, mcol)
    # augmenting keeps every row the heavy matching matched
    hr, _, _ = oracle.match_heavy(m, n, rp, cc, None, seed=seed)
    assert (mrow[hr >= 0] >= 0).all()
    if name.startswith("grid"):
        assert size == m


def grid_case(kind, side, seed):
    g = vmo_gen.grid3d(side, seed=1) if kind == "3d" else vmo_gen.grid2d(side)
    m = g.m
    h = oracle.bipartite(m, m, g.rowptr, g.col)
    r = vmo_gen.rng(seed, 5)
    ids = np.arange(m)
    if kind == "3d":   # the pattern's ids are permuted: vertex v sits at grid index inv[v]
        perm = vmo_gen.rng(1, 2).permutation(m)
        ids = np.empty_like(perm)
        ids[perm] = np.arange(m)
        pos = np.stack([ids % side, (ids // side) % side, ids // (side * side)]).astype(np.float32)
    else:
        pos = np.stack([ids % side, ids // side, np.zeros(m)]).astype(np.float32)
    x = np.zeros((4, 2 * m), np.float32)
    x[:3, :m] = pos + r.uniform(-0.3, 0.3, size=(3, m))
    x[:3, m:] = pos + r.uniform(-0.3, 0.3, size=(3, m))
    x[3] = r.uniform(-0.1, 0.1, size=2 * m)
    mrow, mcol, size = oracle.match(m, m, g.rowptr, g.col, None, seed=seed)
    assert size == m
    return g, h, x, oracle.mu_of(m, m, mrow, mcol)


@pytest.mark.parametrize("kind,side,P,seed,ord_", [("2d", 12, 8, 1, 1), ("2d", 20, 16, 2, 0), ("3d", 8, 16, 3, 1),
                                                   ("3d", 12, 64, 4, 1), ("2d", 9, 3, 5, 1)])
def test_order_matched_parity(ctx, kind, side, P, seed, ord_):
    g, h, x, mu = grid_case(kind, side, seed)
    ref = oracle.order(h, x, P, seed, mode=oracle.GRAPH_MODE, ord=ord_, mu=mu)
    o = ctx.order_matched(dev_h(h), dev_x(x), dev(mu, np.int32), P, seed, order=ord_)
    compare_order(o, ref, oracle.GRAPH_MODE, h.k, h.l)
    # the rule changed the result: without the matching the separators differ
    plain = oracle.order(h, x, P, seed, mode=oracle.GRAPH_MODE, ord=ord_)
    assert not np.array_equal(plain.vperm, ref.vperm)
    # an all -1 matching gives the plain ordering
    none = ctx.order_matched(dev_h(h), dev_x(x), dev(np.full(h.k, -1), np.int32), P, seed, order=ord_)
    compare_order(none, plain, oracle.GRAPH_MODE, h.k, h.l)


def test_order_matched_full_size(ctx):
    """The bipartite graph of the 64^3 7-point matrix (524,288 vertices,
    1,810,432 edges), the oracle's perfect matching, 64 parts, BBD: exact."""
    g, h, x, mu = grid_case("3d", 64, 1)
    ref = oracle.order(h, x, 64, 1, mode=oracle.GRAPH_MODE, ord=oracle.BBD, mu=mu)
    dh, dx, dmu = dev_h(h), dev_x(x), dev(mu, np.int32)
    o = ctx.order_matched(dh, dx, dmu, 64, 1)
    compare_order(o, ref, oracle.GRAPH_MODE, h.k, h.l)
    rp, cp = ctx.matched_perms(g.m, o["vperm"], dmu)
    er, ec = oracle.matched_perms(g.m, ref.vperm, mu)
    assert np.array_equal(host(rp), er) and np.array_equal(host(cp), ec)
    s = ctx.order_schur(dh, dx, o, 64, 8, 1, mu=dmu)
    want = oracle.schur(h, x, ref.vperm, ref.part, ref.node_heap, ref.node_vptr, ref.n_nodes, 64, 8, 1, mu=mu)
    assert np.array_equal(host(s), want)


@pytest.mark.parametrize("kind,side,P,P3,seed", [("2d", 12, 8, 4, 1), ("3d", 10, 16, 8, 2)])
def test_schur_matched_parity(ctx, kind, side, P, P3, seed):
    g, h, x, mu = grid_case(kind, side, seed)
    ref = oracle.order(h, x, P, seed, mode=oracle.GRAPH_MODE, ord=oracle.BBD, mu=mu)
    dh, dx, dmu = dev_h(h), dev_x(x), dev(mu, np.int32)
    o = ctx.order_matched(dh, dx, dmu, P, seed)
    got = ctx.order_schur(dh, dx, o, P, P3, seed, mu=dmu)
    want = oracle.schur(h, x, ref.vperm, ref.part, ref.node_heap, ref.node_vptr, ref.n_nodes, P, P3, seed, mu=mu)
    assert np.array_equal(host(got), want)
    plain = oracle.schur(h, x, ref.vperm, ref.part, ref.node_heap, ref.node_vptr, ref.n_nodes, P, P3, seed)
    assert not np.array_equal(plain, want)


@pytest.mark.parametrize("kind,side,P,seed", [("2d", 10, 8, 1), ("3d", 9, 16, 2)])
def test_matched_perms_parity(ctx, kind, side, P, seed):
    g, h, x, mu = grid_case(kind, side, seed)
    ref = oracle.order(h, x, P, seed, mode=oracle.GRAPH_MODE, ord=oracle.BBD, mu=mu)
    rp, cp = ctx.matched_perms(g.m, dev(ref.vperm, np.int32), dev(mu, np.int32))
    er, ec = oracle.matched_perms(g.m, ref.vperm, mu)
    assert np.array_equal(host(rp), er) and np.array_equal(host(cp), ec)


def test_finegrain_parity(ctx):
    for m, n, d, seed in [(9, 7, 0.3, 1), (300, 200, 0.02, 2), (2000, 2000, 0.003, 3)]:
        rp, cc = random_pattern(m, n, d, seed)
        x = vmo_gen.random_points(m + n, seed, clusters=3)
        want = oracle.finegrain(m, n, rp, cc, x)
        got = ctx.finegrain(m, n, dev(rp), dev(cc), dev_x(x))
        assert np.array_equal(host(got), want)


def test_matched_rejects_bad_input(ctx):
    import paper_1105_4490_amd as Pk
    g, h, x, mu = grid_case("2d", 6, 1)
    dh, dx = dev_h(h), dev_x(x)
    k = h.k
    bad = mu.copy()
    bad[0] = 0                                    # a fixed point
    with pytest.raises(Pk.VmoError):
        ctx.order_matched(dh, dx, dev(bad, np.int32), 4, 1)
    bad = mu.copy()
    bad[0] = -1                                   # not an involution
    with pytest.raises(Pk.VmoError):
        ctx.order_matched(dh, dx, dev(bad, np.int32), 4, 1)
    # a pair that is not an edge: row 0 with the column of a far row
    m = g.m
    bad = np.full(k, -1, np.int32)
    bad[0], bad[m + m - 1] = m + m - 1, 0
    with pytest.raises(Pk.VmoError):
        ctx.order_matched(dh, dx, dev(bad, np.int32), 4, 1)
    # not a permutation: checked on the device, reported by the next sync
    ctx.matched_perms(m, dev(np.zeros(k), np.int32), dev(mu, np.int32))
    with pytest.raises(Pk.VmoError, match="not a permutation"):
        ctx.sync()
    ctx.sync()   # the word was cleared
    a = np.ones(int(g.rowptr[-1]), np.float32)
    a[3] = np.inf
    with pytest.raises(Pk.VmoError):
        ctx.match(m, m, dev(g.rowptr, np.int64), dev(g.col, np.int32), dev(a))
