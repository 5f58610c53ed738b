"""Pins for the oracle's layout (Sec. 2): the gradient against finite
differences of the energy eq. (6), against the direct sum of eq. (7) and the
general form eq. (5); exact scaling laws of its two terms (Sec. 2.1); the
tree's geometry against an independent Morton ordering; the coarsening
against the characterisation of the greedy matching; and end-to-end sanity
(the 2-D grid's optimal first cut, separated components)."""
import json
import os

import numpy as np
import pytest

import oracle
import vmo_gen

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def energy(h, x, w, c):
    """eq. (6) with d = 4, in FP64, direct O(k^2)."""
    x = x.astype(np.float64)
    f = 0.0
    for e, net in enumerate(h.nets()):
        if len(net) == 0:
            continue
        z = x[:, net].mean(axis=1, keepdims=True)
        f += 0.5 * c[e] * ((x[:, net] - z) ** 2).sum()
    d = x[:, :, None] - x[:, None, :]
    r2 = (d ** 2).sum(axis=0)
    np.fill_diagonal(r2, np.inf)
    f += 0.5 * (np.outer(w, w) / r2).sum()
    return f


def grad_eq7(h, x, w, c):
    """eq. (7) in FP64, direct."""
    x = x.astype(np.float64)
    k = h.k
    y = np.zeros((4, k))
    for e, net in enumerate(h.nets()):
        if len(net) == 0:
            continue
        z = x[:, net].mean(axis=1)
        for n in net:
            y[:, n] += c[e] * (x[:, n] - z)
    for n in range(k):
        d = x - x[:, n:n + 1]
        r2 = (d ** 2).sum(axis=0)
        r2[n] = np.inf
        y[:, n] += 2.0 * (w * w[n] / r2 ** 2 * d).sum(axis=1)
    return y


def grad_eq5(h, x, w, c, gamma=2.0):
    """eq. (5) with alpha = beta = 1, delta = 2, general gamma, FP64."""
    x = x.astype(np.float64)
    y = np.zeros_like(x)
    for e, net in enumerate(h.nets()):
        if len(net) == 0:
            continue
        z = x[:, net].mean(axis=1)
        nrm = np.linalg.norm(x[:, net] - z[:, None], axis=0)
        first = (nrm ** (gamma - 2) * (x[:, net] - z[:, None])).sum(axis=1)
        for n in net:
            y[:, n] += -gamma / 2 * c[e] / len(net) * first
            y[:, n] += gamma / 2 * c[e] * np.linalg.norm(x[:, n] - z) ** (gamma - 2) * (x[:, n] - z)
    for n in range(h.k):
        d = x - x[:, n:n + 1]
        r2 = (d ** 2).sum(axis=0)
        r2[n] = np.inf
        y[:, n] += 2.0 * (w * w[n] / r2 ** 2 * d).sum(axis=1)
    return y


def small_case(seed, k=30, l=25):
    g = vmo_gen.random_hypergraph_csr(k, l, seed, maxdeg=5)
    h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
    r = vmo_gen.rng(seed, 5)
    h.w = r.uniform(0.5, 2.0, size=k).astype(np.float32)
    h.c = r.uniform(0.5, 2.0, size=l).astype(np.float32)
    x = (r.standard_normal((4, k)) * 3).astype(np.float32)
    return h, x


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_gradient_theta0_equals_finite_differences_of_energy(seed):
    h, x = small_case(seed)
    y, _ = oracle.gradient(h, x, theta=0.0)
    xd = x.astype(np.float64)
    fd = np.zeros_like(xd)
    eps = 1e-5
    for d in range(4):
        for n in range(h.k):
            a = xd.copy(); a[d, n] += eps
            b = xd.copy(); b[d, n] -= eps
            fd[d, n] = (energy(h, a, h.w, h.c) - energy(h, b, h.w, h.c)) / (2 * eps)
    scale = np.abs(fd).max()
    assert np.abs(y - fd).max() <= 1e-4 * scale


@pytest.mark.parametrize("seed", [4, 5])
def test_gradient_theta0_equals_direct_eq7_and_eq5(seed):
    h, x = small_case(seed, k=60, l=40)
    y, _ = oracle.gradient(h, x, theta=0.0)
    y7 = grad_eq7(h, x, h.w, h.c)
    y5 = grad_eq5(h, x, h.w, h.c)
    assert np.allclose(y5, y7, rtol=1e-12, atol=1e-12 * np.abs(y7).max())   # gamma = 2 cancellation
    assert np.abs(y - y7).max() <= 2e-6 * np.abs(y7).max()


@pytest.mark.parametrize("seed", [6, 7])
def test_tree_approximation_is_close(seed):
    h, x = small_case(seed, k=600, l=300)
    x = vmo_gen.random_points(600, seed)
    y0, _ = oracle.gradient(h, x, theta=0.0)
    y1, _ = oracle.gradient(h, x, theta=0.5)
    err = np.linalg.norm(y1 - y0, axis=0) / np.linalg.norm(y0, axis=0)
    assert np.median(err) < 2e-2
    assert np.percentile(err, 95) < 1e-1


@pytest.mark.parametrize("theta", [0.0, 0.5])
def test_gradient_scaling_laws_exact(theta):
    """Sec. 2.1: the rubber-band term scales like theta^gamma, the charge term
    like theta^-delta; for the gradient, degree 1 and degree -3.  Scaling by 2
    is exact in binary floating point, so the identities hold bit for bit."""
    h, x = small_case(8, k=200, l=120)
    hc = oracle.Hypergraph(h.k, h.l, h.ptr, h.pins, h.w, np.zeros(h.l, np.float32))   # charges only
    hw = oracle.Hypergraph(h.k, h.l, h.ptr, h.pins, np.full(h.k, 1e-30, np.float32), h.c)  # bands only
    r1, _ = oracle.gradient(hc, x, theta=theta)
    r2, _ = oracle.gradient(hc, 2 * x, theta=theta)
    assert np.array_equal(r2, r1 / 8)
    a1, _ = oracle.gradient(hw, x, theta=theta)
    a2, _ = oracle.gradient(hw, 2 * x, theta=theta)
    assert np.array_equal(a2, 2 * a1)


def test_gradient_translation_and_rotation_invariance():
    h, x = small_case(9, k=80, l=50)
    y, _ = oracle.gradient(h, x, theta=0.0)
    t = np.array([[3.0], [-1.0], [0.5], [2.0]], dtype=np.float32)
    yt, _ = oracle.gradient(h, x + t, theta=0.0)
    assert np.abs(yt - y).max() <= 1e-4 * np.abs(y).max()
    R, _ = np.linalg.qr(vmo_gen.rng(9, 1).standard_normal((4, 4)))
    xr = (R @ x.astype(np.float64)).astype(np.float32)
    yr, _ = oracle.gradient(h, xr, theta=0.0)
    assert np.abs(yr - R @ y).max() <= 1e-4 * np.abs(y).max()


def morton(kq):
    key = np.zeros(kq.shape[1], dtype=np.uint64)
    for b in range(15, -1, -1):
        for d in range(4):
            key = (key << np.uint64(1)) | ((kq[d] >> b) & 1).astype(np.uint64)
    return key


@pytest.mark.parametrize("seed,cap", [(1, 8), (2, 1), (3, 4)])
def test_tree_geometry(seed, cap):
    k = 500
    x = vmo_gen.random_points(k, seed, clusters=4, spread=0.05)
    x[:, 10] = x[:, 11]            # a coincident pair
    w = vmo_gen.rng(seed, 3).uniform(0.5, 2, size=k).astype(np.float32)
    T = oracle.tree(x, w, leaf_cap=cap)
    lo = x.min(axis=1).astype(np.float64)
    ext = (x.max(axis=1).astype(np.float64) - lo).max()
    kq = np.minimum(np.floor((x - lo[:, None]) * (65536.0 / ext)), 65535).astype(np.uint32)
    key = morton(kq)
    assert np.array_equal(T.order, np.lexsort((np.arange(k), key)))
    for t in range(T.n):
        f, c_, dep = T.first[t], T.count[t], T.depth[t]
        pts = T.order[f:f + c_]
        side = 1 << (16 - dep)
        cell_lo = (T.cell2[t] - side) // 2
        assert ((kq[:, pts] >= cell_lo[:, None]) & (kq[:, pts] < cell_lo[:, None] + side)).all()
        assert bool(T.leaf[t]) == (c_ <= cap or dep == 16)
        # children tile the parent in order; next skips the subtree
        if not T.leaf[t]:
            ch, pos = t + 1, f
            while ch != T.next[t]:
                assert T.first[ch] == pos and T.depth[ch] == dep + 1
                pos += T.count[ch]
                ch = T.next[ch]
            assert pos == f + c_
        W = w[pts].astype(np.float64).sum()
        assert abs(T.W[t] - W) <= 1e-6 * W
        X = (w[pts] * x[:, pts].astype(np.float64)).sum(axis=1) / W
        assert np.allclose(T.X[t], X, rtol=1e-6, atol=1e-6 * ext)
    assert T.next[0] == T.n


def prio(seed, level, u, v, om):
    return (om, oracle.rng(seed, 3 | (level << 8), u, v), -u, -v)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_coarsening_is_the_greedy_matching(seed):
    g = vmo_gen.random_hypergraph_csr(120, 150, seed, maxdeg=4)
    h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
    h.c = vmo_gen.rng(seed, 4).integers(1, 4, size=h.l).astype(np.float32)
    h.w = np.ones(h.k, np.float32)
    pi, H = oracle.coarsen(h, seed, 0, 0)
    # candidate pairs and their priorities
    om = {}
    for e, net in enumerate(h.nets()):
        if 2 <= len(net) <= 64:
            for i in range(len(net)):
                for j in range(i + 1, len(net)):
                    p = (int(net[i]), int(net[j]))
                    om[p] = max(om.get(p, -1.0), float(h.c[e]) / (len(net) - 1))
    P = {p: prio(seed, 0, p[0], p[1], o) for p, o in om.items()}
    groups = {}
    for v in range(h.k):
        groups.setdefault(int(pi[v]), []).append(v)
    nbrs = [set() for _ in range(h.k)]
    for (u, v) in om:
        nbrs[u].add(v)
        nbrs[v].add(u)
    # recover the matching: pairs of a group that are candidates and both
    # have more than one neighbour or are the pair itself
    mate = {}
    for gid, mem in groups.items():
        core = [v for v in mem if not (len(nbrs[v]) == 1 and len(mem) > 2)] if len(mem) > 2 else mem
        if len(mem) >= 2:
            pairs = [(a, b) for a in mem for b in mem if a < b and (a, b) in P]
            # the matched pair is the one of highest priority in the group
            best = max(pairs, key=lambda p: P[p])
            mate[best[0]], mate[best[1]] = best[1], best[0]
    # greedy characterisation: every unmatched candidate pair has a matched
    # pair of higher priority at one of its ends; matching is maximal
    for (u, v), pr in P.items():
        if mate.get(u) == v:
            continue
        assert u in mate or v in mate
        higher = [P[tuple(sorted((a, mate[a])))] for a in (u, v) if a in mate]
        assert max(higher) > pr
    # single-neighbour rule and group numbering by smallest member
    for v in range(h.k):
        if v not in mate and len(nbrs[v]) == 1:
            u = next(iter(nbrs[v]))
            assert pi[v] == pi[u]
    mins = sorted(min(m) for m in groups.values())
    assert [int(pi[m]) for m in mins] == list(range(H.k))
    assert H.w.sum() == h.k
    # coarse nets: images of size >= 2, equal images merged, ordered by smallest net id
    img = {}
    for e, net in enumerate(h.nets()):
        s = tuple(sorted({int(pi[v]) for v in net}))
        if len(s) >= 2:
            if s in img:
                img[s][1] += float(h.c[e])
            else:
                img[s] = [e, float(h.c[e])]
    want = sorted((rep, s, cst) for s, (rep, cst) in img.items())
    assert H.l == len(want)
    for j, (rep, s, cst) in enumerate(want):
        assert tuple(H.pins[H.ptr[j]:H.ptr[j + 1]].tolist()) == s
        assert H.c[j] == np.float32(cst)


def test_star_collapses():
    """Single-neighbour vertices join their neighbour (Sec. 2.3): a star
    of 20 leaves coarsens to one vertex."""
    h = oracle.hypergraph(21, [[0, i] for i in range(1, 21)])
    pi, H = oracle.coarsen(h, 1)
    assert H.k == 1 and (pi == 0).all() and H.l == 0 and H.w[0] == 21


def test_init_and_prolong_ranges():
    x = oracle.layout_init(81, 5, 0, 3)
    a = 81 ** 0.25
    assert (x >= -0.5 * a).all() and (x < 0.5 * a).all()
    assert len(np.unique(x)) > 300
    pi = np.repeat(np.arange(81, dtype=np.int32), 2)[:150]
    xf = oracle.layout_prolong(pi, x, 5, 0, 2, jitter=1e-3)
    sig = np.float32((150 / 81) ** 0.25)
    eps = 1e-3 * float((x.max(axis=1).astype(np.float64) - x.min(axis=1)).max()) / 81 ** 0.25
    assert np.abs(xf - sig * x[:, pi]).max() <= eps * (1 + 1e-6)


def test_step_moves_each_vertex_alpha_along_its_gradient():
    g = vmo_gen.grid2d(10)
    h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
    x0 = oracle.layout_init(h.k, 3)
    p = oracle.layout_params()
    x1, y, alpha = oracle.layout_iter(h, x0, p, 0)
    lo, hi = x0.min(axis=1).astype(np.float64), x0.max(axis=1).astype(np.float64)
    assert abs(alpha - float(np.float32(0.1)) * np.prod(hi - lo) ** 0.25) <= 1e-14 * alpha
    step = (x1 - x0).astype(np.float64)
    nrm = np.linalg.norm(step, axis=0)
    assert np.allclose(nrm, alpha, rtol=1e-5)
    cos = (-(step * y).sum(axis=0)) / (nrm * np.linalg.norm(y, axis=0))
    assert (cos > 1 - 1e-6).all()
    x2, _, a2 = oracle.layout_iter(h, x1, p, 1, alpha)
    assert a2 == alpha * np.float64(np.float32(0.9))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_layout_grid_first_cut_is_optimal(seed):
    """A good visual representation of the 32 x 32 grid (Fig. 1-style) lets
    2-means find the straight first cut: 2 * 32 cut nets in the row-net model."""
    g = vmo_gen.grid2d(32)
    h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
    x = oracle.layout(h, oracle.layout_params(seed=seed))
    assert np.isfinite(x).all()
    o = oracle.order(h, x, 2, seed)
    assert o.split_cut[:o.n_nodes].max() == 64


def test_layout_disconnected_components_packed_apart():
    """Theorem on connectedness (Sec. 2.2): components are laid out alone and
    placed side by side; the first split then cuts nothing."""
    a = vmo_gen.grid2d(8)
    nets = [list(a.col[a.rowptr[i]:a.rowptr[i + 1]]) for i in range(a.m)]
    nets += [[v + 64 for v in n] for n in nets]
    h = oracle.hypergraph(128, nets)
    assert len(set(oracle.components(h).tolist())) == 2
    x = oracle.layout(h, oracle.layout_params(seed=2))
    e0 = (x[:, :64].max(axis=1).astype(np.float64) - x[:, :64].min(axis=1)).max()
    e1 = (x[:, 64:].max(axis=1).astype(np.float64) - x[:, 64:].min(axis=1)).max()
    gap = x[0, 64:].min() - (x[0, :64].min() + e0)
    assert abs(gap - 0.1 * max(e0, e1)) <= 1e-5 * max(e0, e1)
    assert (x.min(axis=1) == 0).all()
    # with a wide gap the first 2-means split separates the components
    x = oracle.layout(h, oracle.layout_params(seed=2, pack_gap=3.0))
    o = oracle.order(h, x, 2, 1)
    assert o.split_cut[:o.n_nodes].max() == 0


# ------------------------------------------------ plain evaluation of eq. (7) ----

@pytest.mark.parametrize("seed", [4, 5])
def test_plain_gradient_theta0_is_the_direct_sum(seed):
    """theta = 0 opens every node: the plain walk is then the direct O(k^2)
    sum of eq. (7), here recomputed with numpy in FP64; every walk meets the
    k - 1 other points."""
    h, x = small_case(seed, k=60, l=40)
    y, s, nint = oracle.gradient_plain(h, x, theta=0.0)
    y7 = grad_eq7(h, x, h.w.astype(np.float64), h.c.astype(np.float64))
    assert np.abs(y - y7).max() <= 1e-12 * np.abs(y7).max()
    assert (nint == h.k - 1).all()
    assert (s >= np.abs(y) * (1 - 1e-12)).all()


@pytest.mark.parametrize("seed,k", [(6, 600), (7, 3000)])
def test_strict_fp32_gradient_within_rounding_of_plain(seed, k):
    """The strict FP32 evaluation (the order the GPU reproduces) agrees with
    the plain FP64 one to 1e-5 of the rounding magnitudes s, element by
    element, and both walks make the same interactions."""
    g = vmo_gen.random_hypergraph_csr(k, k // 2, seed, maxdeg=5)
    h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
    h.w = vmo_gen.rng(seed, 5).uniform(0.5, 2.0, size=k).astype(np.float32)
    x = vmo_gen.random_points(k, seed, clusters=6)
    y32, _ = oracle.gradient(h, x, theta=0.5)
    y, s, nint = oracle.gradient_plain(h, x, theta=0.5)
    assert (np.abs(y32 - y) <= 1e-5 * s).all()
    _, cnt = oracle.gradient_sample(h, x, np.arange(k), theta=0.5)
    assert np.array_equal(nint, cnt)
    ys, ss, ns = oracle.gradient_plain(h, x, theta=0.5, ids=np.array([5, 0, k - 1], np.int32))
    assert np.array_equal(ys, y[:, [5, 0, k - 1]]) and np.array_equal(ns, nint[[5, 0, k - 1]])


def test_plain_step_two_points_by_hand():
    """Two points joined by one net, unit weights: x0 = 0, x1 = (1,1,1,1).
    Attraction: z = (1/2)(1,1,1,1), so y0 = -(1/2)(1,1,1,1); repulsion on
    point 0: 2 w w (x1 - x0) / |x1 - x0|^4 = 2 (1,1,1,1) / 16; hence
    y0 = -(3/8)(1,1,1,1) and y1 = -y0.  The box is the unit cube, V = 1,
    so alpha = step0_frac (0.1f); each point moves alpha along -y/|y|:
    x0 -> (alpha/2)(1,1,1,1), x1 -> (1 - alpha/2)(1,1,1,1)."""
    h = oracle.hypergraph(2, [[0, 1]])
    x = np.zeros((4, 2), np.float32)
    x[:, 1] = 1.0
    p = oracle.layout_params()
    xn, y, s, alpha = oracle.layout_iter_plain(h, x, p, 0)
    assert np.array_equal(y[:, 0], np.full(4, -0.375)) and np.array_equal(y[:, 1], np.full(4, 0.375))
    a = float(np.float32(0.1))
    assert alpha == a
    assert np.array_equal(xn[:, 0], np.full(4, np.float32(a / 2)))
    assert np.array_equal(xn[:, 1], np.full(4, np.float32(1 - a / 2)))
    # the strict step takes the same values here (every operation exact or
    # rounded once to the same float)
    xs, ys, a2 = oracle.layout_iter(h, x, p, 0)
    assert a2 == alpha and np.array_equal(ys, y.astype(np.float32))
    assert np.abs(xs - xn).max() <= 2 ** -24


def test_strict_step_two_points_flat_box_by_hand():
    """x0 = 0, x1 = (2,0,0,0), one net: y0 = (-1,0,0,0) + 2 (2,0,0,0)/16 =
    (-3/4,0,0,0).  The box is flat (V = 0), so its largest side, 2, replaces
    V^(1/4): alpha = 0.2 (from 0.1f); the points move to (alpha,0,0,0) and
    (2 - alpha,0,0,0) up to the FP32 roundings of the step, f = fl(alpha /
    |y|) then fl(f y), and the next step is 0.9f times as long."""
    h = oracle.hypergraph(2, [[0, 1]])
    x = np.zeros((4, 2), np.float32)
    x[0, 1] = 2.0
    p = oracle.layout_params()
    x1, y, alpha = oracle.layout_iter(h, x, p, 0)
    assert np.array_equal(y[:, 0], np.array([-0.75, 0, 0, 0], np.float32))
    assert alpha == 2.0 * float(np.float32(0.1))
    f = np.float32(alpha / 0.75)
    t = np.float32(f * np.float32(0.75))
    assert abs(float(t) - alpha) <= 2 ** -24 * 2
    assert np.array_equal(x1[:, 0], np.array([t, 0, 0, 0], np.float32))
    assert np.array_equal(x1[:, 1], np.array([np.float32(2.0) - t, 0, 0, 0], np.float32))
    _, _, a2 = oracle.layout_iter(h, x1, p, 1, alpha)
    assert a2 == alpha * float(np.float32(0.9))


def test_init_and_prolong_values_hand_derived():
    """Algorithm 2's random start and prolongation at one vertex, against
    exact values derived by hand from the random words
    (golden/init_prolong.json): k = 16 gives k^(1/4) = 2, so the start is
    (top 24 bits - 2^23) / 2^23; the prolongation 16 -> 256 has sigma = 2
    and eps = 2^-10 * 8 / 2, and its one rounding is that of the final sum."""
    with open(os.path.join(GOLD, "init_prolong.json")) as f:
        g = json.load(f)
    gi = g["init"]
    x = oracle.layout_init(gi["k"], g["seed"], g["comp"], gi["level"])
    for d, val in enumerate(gi["values"]):
        r = int(val["r"])
        assert oracle.rng(g["seed"], 1 | (gi["level"] << 8) | (g["comp"] << 32), gi["v"], d) == r
        assert val["top24"] == r >> 40
        assert x[d, gi["v"]] == np.float32(val["x"])
    gp = g["prolong"]
    xc = np.array(gp["xc"], np.float32)
    pi = np.array(gp["pi"], np.int32)
    xf = oracle.layout_prolong(pi, xc, g["seed"], g["comp"], gp["fine_level"], jitter=gp["jitter"])
    for d, val in enumerate(gp["values"]):
        assert oracle.rng(g["seed"], 2 | (gp["fine_level"] << 8) | (g["comp"] << 32), gp["v"], d) == int(val["r"])
        assert xf[d, gp["v"]] == np.float32(val["x"])
