"""Oracle pins for the strengthened diagonal (Sec. 4.2 and Sec. 5): the
bipartite model of Table 1 rebuilt from its definition; the heavy edge
matching against a plain greedy by weight (distinct weights) and against the
property that characterises the greedy matching of a strict edge order; the
Hopcroft-Karp augmentation against scipy's maximum bipartite matching;
Algorithm 7 with matched pairs (pairs never split, reduction to the plain
ordering without a matching, a hand-derived example); the row and column
permutations (matching on the diagonal, BBD blocks); finegrain coordinates
(exact half-integers); the Schur-complement recursion with the matching."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import maximum_bipartite_matching

import oracle
import vmo_gen


def random_pattern(m, n, density, seed, diag=False):
    r = vmo_gen.rng(seed, 1)
    a = r.random((m, n)) < density
    if diag:
        a[np.arange(min(m, n)), np.arange(min(m, n))] = True
    A = sp.csr_matrix(a.astype(np.float32))
    A.sort_indices()
    return A.indptr.astype(np.int64), A.indices.astype(np.int32), a


def test_bipartite_model_from_definition():
    rowptr, col, a = random_pattern(7, 5, 0.4, 1)
    h = oracle.bipartite(7, 5, rowptr, col)
    assert h.k == 12 and h.l == int(a.sum())
    edges = {tuple(e) for e in h.nets()}
    assert edges == {(i, 7 + j) for i in range(7) for j in range(5) if a[i, j]}
    assert all(len(e) == 2 and e[0] < e[1] for e in h.nets())
    # CSR order: nonzero e of row i is the e-th edge
    rows = np.repeat(np.arange(7), np.diff(rowptr))
    assert [tuple(e) for e in h.nets()] == [(int(i), 7 + int(j)) for i, j in zip(rows, col)]


def greedy_by_weight(m, n, rowptr, col, w):
    rows = np.repeat(np.arange(m), np.diff(rowptr))
    mrow, mcol = np.full(m, -1), np.full(n, -1)
    for e in np.argsort(-w, kind="stable"):
        i, j = rows[e], col[e]
        if mrow[i] < 0 and mcol[j] < 0:
            mrow[i], mcol[j] = j, i
    return mrow, mcol


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_heavy_matching_distinct_weights_is_greedy(seed):
    m, n = 40, 35
    rowptr, col, _ = random_pattern(m, n, 0.15, seed)
    nnz = int(rowptr[-1])
    w = vmo_gen.rng(seed, 2).permutation(nnz).astype(np.float32) + 1.0   # distinct
    a = w * np.where(vmo_gen.rng(seed, 3).random(nnz) < 0.5, -1, 1).astype(np.float32)
    mrow, mcol, size = oracle.match_heavy(m, n, rowptr, col, a, seed=7)
    er, ec = greedy_by_weight(m, n, rowptr, col, np.abs(a))
    assert np.array_equal(mrow, er) and np.array_equal(mcol, ec)
    assert size == int((er >= 0).sum())


@pytest.mark.parametrize("seed,weighted", [(1, False), (2, False), (3, True)])
def test_heavy_matching_is_dominated_greedy(seed, weighted):
    """A matching M is the greedy matching of a strict order iff it is a
    matching and every other edge meets an edge of M that precedes it."""
    m, n = 50, 60
    rowptr, col, _ = random_pattern(m, n, 0.08, seed)
    nnz = int(rowptr[-1])
    a = None
    if weighted:   # few distinct values: many ties broken by the scrambled index
        a = vmo_gen.rng(seed, 4).integers(1, 4, size=nnz).astype(np.float32)
    mrow, mcol, size = oracle.match_heavy(m, n, rowptr, col, a, seed=seed)
    keys = np.array([oracle.match_key(a, e, seed) for e in range(nnz)], dtype=np.uint64)
    assert len(set(keys.tolist())) == nnz                      # no ties
    rows = np.repeat(np.arange(m), np.diff(rowptr))
    key_of = {(int(rows[e]), int(col[e])): int(keys[e]) for e in range(nnz)}
    matched = [(i, int(mrow[i])) for i in range(m) if mrow[i] >= 0]
    assert size == len(matched)
    assert all(mcol[j] == i for i, j in matched)
    assert all(key_of.get((i, j)) is not None for i, j in matched)
    for e in range(nnz):
        i, j = int(rows[e]), int(col[e])
        if mrow[i] == j:
            continue
        dom = []
        if mrow[i] >= 0:
            dom.append(key_of[(i, int(mrow[i]))])
        if mcol[j] >= 0:
            dom.append(key_of[(int(mcol[j]), j)])
        assert dom and max(dom) > keys[e], (i, j)
    # weights dominate the index: with a heaviest entry per row and column on
    # the diagonal, the matching is the diagonal
    sq = 30
    rp, cc, _ = random_pattern(sq, sq, 0.2, seed, diag=True)
    rr = np.repeat(np.arange(sq), np.diff(rp))
    val = np.where(rr == cc, 10.0, 1.0).astype(np.float32)
    mr, _, s2 = oracle.match_heavy(sq, sq, rp, cc, val, seed=seed)
    assert s2 == sq and np.array_equal(mr, np.arange(sq))


@pytest.mark.parametrize("m,n,density,seed", [(60, 60, 0.04, 1), (80, 70, 0.03, 2), (100, 100, 0.025, 3),
                                              (200, 200, 0.01, 4)])
def test_augment_is_maximum(m, n, density, seed):
    rowptr, col, a = random_pattern(m, n, density, seed)
    hr, hc, hs = oracle.match_heavy(m, n, rowptr, col, None, seed=seed)
    mrow, mcol, size = oracle.match_augment(m, n, rowptr, col, hr, hc)
    ref = maximum_bipartite_matching(sp.csr_matrix(a.astype(np.float32)), perm_type="column")
    assert size == int((ref >= 0).sum()) >= hs
    for i in range(m):
        if mrow[i] >= 0:
            assert a[i, mrow[i]] and mcol[mrow[i]] == i
    assert int((mcol >= 0).sum()) == size
    assert all(mrow[i] >= 0 for i in range(m) if hr[i] >= 0)   # augmenting keeps matched rows matched


def test_augment_perfect_with_diagonal():
    m = 300
    rowptr, col, _ = random_pattern(m, m, 0.01, 9, diag=True)
    mrow, mcol, size = oracle.match(m, m, rowptr, col, None, seed=1)
    assert size == m and sorted(mrow.tolist()) == list(range(m))


def grid_bipartite(side, seed):
    g = vmo_gen.grid2d(side)
    m = g.m
    h = oracle.bipartite(m, m, g.rowptr, g.col)
    r = vmo_gen.rng(seed, 5)
    pos = np.stack([np.arange(m) % side, np.arange(m) // side]).astype(np.float32)
    x = np.zeros((4, 2 * m), np.float32)
    x[:2, :m] = pos + r.uniform(-0.3, 0.3, size=(2, m))
    x[:2, m:] = pos + r.uniform(-0.3, 0.3, size=(2, m))
    x[2:] = r.uniform(-0.1, 0.1, size=(2, 2 * m))
    return g, h, x


def subtree_sets(o):
    blocks = {int(o.node_heap[t]): set(o.vperm[o.node_vptr[t]:o.node_vptr[t + 1]].tolist())
              for t in range(o.n_nodes)}

    def sub(hh):
        return set() if hh not in blocks else blocks[hh] | sub(2 * hh) | sub(2 * hh + 1)
    return blocks, sub


@pytest.mark.parametrize("side,P,seed", [(8, 4, 1), (12, 16, 2), (16, 32, 3)])
def test_order_mu_keeps_pairs(side, P, seed):
    g, h, x = grid_bipartite(side, seed)
    m = g.m
    mrow, mcol, size = oracle.match(m, m, g.rowptr, g.col, None, seed=seed)
    assert size == m
    mu = oracle.mu_of(m, m, mrow, mcol)
    o = oracle.order(h, x, P, seed, mode=oracle.GRAPH_MODE, ord=oracle.BBD, mu=mu)
    assert np.array_equal(o.part, o.part[mu])                  # every pair in one block
    blocks, sub = subtree_sets(o)
    nets = [tuple(e) for e in h.nets()]
    for hh in blocks:
        if 2 * hh in blocks:
            L, R = sub(2 * hh), sub(2 * hh + 1)
            assert not any((a in L and b in R) or (a in R and b in L) for a, b in nets)
    for t in range(o.n_nodes):                                  # square diagonal blocks
        blk = o.vperm[o.node_vptr[t]:o.node_vptr[t + 1]]
        assert int((blk < m).sum()) == int((blk >= m).sum())
    plain = oracle.order(h, x, P, seed, mode=oracle.GRAPH_MODE, ord=oracle.BBD)
    none = oracle.order(h, x, P, seed, mode=oracle.GRAPH_MODE, ord=oracle.BBD, mu=np.full(2 * m, -1, np.int32))
    assert np.array_equal(none.vperm, plain.vperm) and np.array_equal(none.part, plain.part)
    assert int((o.part >= P).sum()) >= int((plain.part >= P).sum())


def test_order_mu_hand_example():
    """Two diagonal 2 x 2 blocks and the nonzero a_12 joining them; rows
    r0..r3 are vertices 0..3, columns c0..c3 are 4..7, the matching is the
    diagonal.  Points of r0, r1, c0, c1 lie near x = 0 and those of r2, r3,
    c2, c3 near x = 10, so the split separates the two groups and the only
    cut edge is {r1, c2}.  r1 (x = 0.4) is nearer the plane (x near 5.1) than
    c2 (x = 9.9), so r1 enters the separator, and with the matching c1 too."""
    rowptr = np.array([0, 2, 5, 7, 9], np.int64)
    col = np.array([0, 1, 0, 1, 2, 2, 3, 2, 3], np.int32)
    h = oracle.bipartite(4, 4, rowptr, col)
    x = np.zeros((4, 8), np.float32)
    x[0] = [0.0, 0.4, 10.0, 10.2, 0.1, 0.3, 9.9, 10.1]
    x[1] = [0.0, 0.1, 0.0, 0.1, 0.1, 0.0, 0.1, 0.0]
    mu = np.array([4, 5, 6, 7, 0, 1, 2, 3], np.int32)
    for use_mu, sep in [(True, {1, 5}), (False, {1})]:
        o = oracle.order(h, x, 2, 1, mode=oracle.GRAPH_MODE, ord=oracle.BBD, mu=mu if use_mu else None)
        assert o.n_nodes == 3 and o.node_heap[2] == 1
        assert set(o.vperm[o.node_vptr[2]:o.node_vptr[3]].tolist()) == sep
        leaves = [set(o.vperm[o.node_vptr[t]:o.node_vptr[t + 1]].tolist()) for t in (0, 1)]
        near0 = {0, 1, 4, 5} - sep
        assert sorted(map(sorted, leaves)) == sorted([sorted(near0), [2, 3, 6, 7]])


@pytest.mark.parametrize("side,P,seed", [(8, 4, 1), (10, 8, 2)])
def test_matched_perms(side, P, seed):
    g, h, x = grid_bipartite(side, seed)
    m = g.m
    mrow, mcol, _ = oracle.match(m, m, g.rowptr, g.col, None, seed=seed)
    mu = oracle.mu_of(m, m, mrow, mcol)
    o = oracle.order(h, x, P, seed, mode=oracle.GRAPH_MODE, ord=oracle.BBD, mu=mu)
    rp, cp = oracle.matched_perms(m, o.vperm, mu)
    assert sorted(rp.tolist()) == list(range(m)) and sorted(cp.tolist()) == list(range(m))
    A = np.zeros((m, m), bool)
    A[np.repeat(np.arange(m), np.diff(g.rowptr)), g.col] = True
    B = A[rp][:, cp]
    assert B.diagonal().all()
    # block b of the row order = rows of emission rank b; leaf blocks meet
    # no other leaf block
    rb = np.zeros(m, int)
    t = 0
    for r in range(o.n_nodes):
        for v in o.vperm[o.node_vptr[r]:o.node_vptr[r + 1]]:
            if v < m:
                rb[t] = r
                t += 1
    leaf = np.array([o.part[o.vperm[o.node_vptr[r]]] < P if o.node_vptr[r] < o.node_vptr[r + 1] else False
                     for r in range(o.n_nodes)])
    ii, jj = np.nonzero(B)
    bad = leaf[rb[ii]] & leaf[rb[jj]] & (rb[ii] != rb[jj])
    assert not bad.any()


def test_finegrain_half_integers():
    rowptr, col, a = random_pattern(9, 7, 0.3, 5)
    r = vmo_gen.rng(5, 6)
    x = r.integers(-50, 50, size=(4, 16)).astype(np.float32)
    xnz = oracle.finegrain(9, 7, rowptr, col, x)
    rows = np.repeat(np.arange(9), np.diff(rowptr))
    for e in range(int(rowptr[-1])):
        for d in range(4):
            num = int(x[d, rows[e]]) + int(x[d, 9 + col[e]])     # exact: x2 is an integer
            assert 2 * float(xnz[d, e]) == num


def test_schur_with_mu_rebuilt():
    g, h, x = grid_bipartite(12, 4)
    m = g.m
    mrow, mcol, _ = oracle.match(m, m, g.rowptr, g.col, None, seed=4)
    mu = oracle.mu_of(m, m, mrow, mcol)
    P, P3, seed = 8, 4, 4
    o = oracle.order(h, x, P, seed, mode=oracle.GRAPH_MODE, ord=oracle.BBD, mu=mu)
    out = oracle.schur(h, x, o.vperm, o.part, o.node_heap, o.node_vptr, o.n_nodes, P, P3, seed, mu=mu)
    edges = [tuple(e) for e in h.nets()]
    expect = o.vperm.copy()
    for r in range(o.n_nodes):
        lo, hi = int(o.node_vptr[r]), int(o.node_vptr[r + 1])
        blk = [int(v) for v in o.vperm[lo:hi]]
        if len(blk) < 2 or o.part[blk[0]] < P:
            continue
        local = {v: i for i, v in enumerate(blk)}
        nets = [sorted((local[a], local[b])) for a, b in edges if a in local and b in local]
        mu3 = np.array([local.get(int(mu[v]), -1) for v in blk], np.int32)
        assert (mu3 >= 0).all()                                   # pairs sit in one block
        so = oracle.order(oracle.hypergraph(len(blk), nets), x[:, blk], P3, seed, mode=oracle.GRAPH_MODE,
                          ord=oracle.BBD, job=int(o.node_heap[r]), mu=mu3)
        expect[lo:hi] = np.array(blk)[so.vperm]
        assert np.array_equal(so.part, so.part[mu3])
    assert out.tolist() == expect.tolist()
    assert not np.array_equal(out, o.vperm)
