"""GPU parity of the layout (Sec. 2) against the CPU oracle, through the C
ABI: the 2^d-tree (exact node arrays and charges), the gradient of eq. (7)
(net centres, attraction, tree walk), descent steps of Algorithm 3,
coarsening (Sec. 2.3), and the full multilevel layout.

Two references.  STRICT: the oracle's FP32 evaluation in the frozen order of
parts, which the GPU reproduces bit for bit (compared with array_equal).
PLAIN: eq. (7) evaluated in FP64 as one running sum per point over the
depth-first walk (oracle.gradient_plain), which shares no order with the
GPU; gradients are compared element by element at |dy| <= 1e-5 * s (s: the
magnitudes of the terms, the scale of FP32 rounding), coordinates at
|dx| <= 1e-5 * max(|x_ref|, bounding-box diagonal)."""
import numpy as np
import pytest
import torch

import oracle
import vmo_gen
from gpu_util import dev_h, dev_x, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1105_4490_amd as P
    return P.Context(0)


def tree_points(k, seed):
    x = vmo_gen.random_points(k, seed, clusters=4, spread=0.05)
    x[:, 10] = x[:, 11]
    x[:, 20:30] = x[:, 30:31]          # a clump of coincident points
    return x


# k <= 1,024: the one-workgroup build's bitonic sort; 1,025..4,096: its
# wavefront runs merged in LDS (three merges up to 2,048 points, four above);
# larger: the multi-kernel build
@pytest.mark.parametrize("k,seed,cap", [(1, 1, 8), (7, 2, 8), (500, 3, 8), (1024, 7, 8), (1025, 8, 4), (2048, 9, 8),
                                        (2049, 10, 1), (3001, 11, 8), (4096, 12, 8), (4097, 13, 8), (5000, 4, 1),
                                        (30011, 5, 4), (100000, 6, 8)])
def test_tree(ctx, k, seed, cap):
    x = tree_points(k, seed) if k > 40 else vmo_gen.random_points(k, seed)
    w = vmo_gen.rng(seed, 3).uniform(0.5, 2, size=k).astype(np.float32)
    T = oracle.tree(x, w, leaf_cap=cap)
    g = ctx.tree(dev_x(x), torch.as_tensor(w).cuda(), leaf_cap=cap)
    assert g["n"] == T.n
    ints = host(g["ints"])
    assert np.array_equal(host(g["order"]), T.order)
    assert np.array_equal(ints[:, 0], T.first)
    assert np.array_equal(ints[:, 1], T.count)
    assert np.array_equal(ints[:, 2], T.depth)
    assert np.array_equal(ints[:, 3], T.leaf)
    assert np.array_equal(ints[:, 4], T.next)
    assert np.array_equal(host(g["cell2"]), T.cell2)
    flt = host(g["flt"])
    assert np.array_equal(flt[:, 0], T.W)
    assert np.array_equal(flt[:, 1:], T.X)


def weighted_case(seed, k, l, maxdeg=5):
    g = vmo_gen.random_hypergraph_csr(k, l, seed, maxdeg=maxdeg)
    h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
    r = vmo_gen.rng(seed, 5)
    h.w = r.uniform(0.5, 2.0, size=k).astype(np.float32)
    h.c = r.uniform(0.5, 2.0, size=l).astype(np.float32)
    return h


@pytest.mark.parametrize("seed,k,l,theta", [(1, 300, 200, 0.0), (2, 3000, 2500, 0.5), (4, 4096, 3000, 0.5),
                                           (5, 4097, 3000, 0.5), (3, 40000, 30000, 0.5)])
def test_gradient(ctx, seed, k, l, theta):
    h = weighted_case(seed, k, l)
    x = vmo_gen.random_points(k, seed, clusters=6)
    y, z = oracle.gradient(h, x, theta=theta)
    gy, gz, nint = ctx.gradient(dev_h(h), dev_x(x), theta=theta)
    assert np.array_equal(host(gz), z)
    assert np.array_equal(host(gy), y)
    if k <= 3000:
        _, cnt = oracle.gradient_sample(h, x, np.arange(k), theta=theta)
        assert nint == int(cnt.sum())


def test_gradient_heavy_vertices(ctx):
    # k > 16384 with Zipf vertex degrees up to 2000: the attraction of the
    # vertices of more than 32 nets is summed by a wavefront each, the rest by
    # one thread each, both in net order
    g = vmo_gen.zipf_rect(20000, 10000, 6, clip=2000)
    h = oracle.colnet(g.m, g.n, g.rowptr, g.col)
    r = vmo_gen.rng(6, 5)
    h.w = r.uniform(0.5, 2.0, size=h.k).astype(np.float32)
    h.c = r.uniform(0.5, 2.0, size=h.l).astype(np.float32)
    assert np.diff(g.rowptr).max() > 500
    x = vmo_gen.random_points(h.k, 6, clusters=6)
    y, z = oracle.gradient(h, x, theta=0.5)
    gy, gz, _ = ctx.gradient(dev_h(h), dev_x(x), theta=0.5)
    assert np.array_equal(host(gz), z)
    assert np.array_equal(host(gy), y)


@pytest.mark.parametrize("k", [3000, 9000])
def test_gradient_coincident_points(ctx, k):
    """Many coincident points: leaves at depth 16 hold more than leaf_cap
    points (one-block tree build below 4097 points, multi-kernel above)."""
    h = weighted_case(11, k, k // 2)
    x = np.round(vmo_gen.random_points(k, 11, clusters=3)).astype(np.float32)
    y, z = oracle.gradient(h, x, theta=0.5)
    gy, gz, _ = ctx.gradient(dev_h(h), dev_x(x), theta=0.5)
    assert np.array_equal(host(gz), z)
    assert np.array_equal(host(gy), y)


@pytest.mark.parametrize("case", ["grid", "weighted"])
def test_descent_steps(ctx, case):
    if case == "grid":
        g = vmo_gen.grid2d(24)
        h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
    else:
        h = weighted_case(7, 2000, 1500)
    p = oracle.layout_params(seed=3)
    import paper_1105_4490_amd as P
    gp = P.layout_params(seed=3)
    x = oracle.layout_init(h.k, 3)
    xo, a = x.copy(), 0.0
    for it in range(12):
        xo, _, a = oracle.layout_iter(h, xo, p, it, a)
    gx = dev_x(x)
    ga = ctx.layout_steps(dev_h(h), gx, gp, 0, 12, 0.0)
    assert ga == a
    assert np.array_equal(host(gx), xo)


def test_profile_times_every_nth_walk(ctx):
    """Live timing with sampling: six descent steps (one walk each) time six
    walks with every = 1 and the first and fourth with every = 3; the sampled
    interaction counts are part of the full ones, and the steps' results do
    not depend on the timing."""
    import paper_1105_4490_amd as P
    h = weighted_case(7, 2000, 1500)
    gp = P.layout_params(seed=3)
    x0 = oracle.layout_init(h.k, 3)
    dh = dev_h(h)
    res = {}
    for every in (1, 3):
        ctx.profile(True, every=every)
        ctx.profile_reset()
        gx = dev_x(x0)
        ctx.layout_steps(dh, gx, gp, 0, 6, 0.0)
        res[every] = (ctx.profile_read("walk"), host(gx))
        ctx.profile(False)
    full, part = res[1][0], res[3][0]
    assert full["launches"] == 6 and part["launches"] == 2
    assert 0 < part["work"] < full["work"] and part["total_ms"] > 0
    assert np.array_equal(res[1][1], res[3][1])
    # uncounted timing: the same launches timed, no work counted, same steps
    ctx.profile(True, every=3, count=False)
    ctx.profile_reset()
    gx = dev_x(x0)
    ctx.layout_steps(dh, gx, gp, 0, 6, 0.0)
    unc = ctx.profile_read("walk")
    ctx.profile(False)
    assert unc["launches"] == 2 and unc["work"] == 0 and unc["total_ms"] > 0
    assert np.array_equal(host(gx), res[1][1])


@pytest.mark.parametrize("case", ["random", "grid3d", "star", "weighted", "pairs", "short_nets", "heavy", "hubs"])
def test_coarsen(ctx, case):
    if case == "hubs":
        # three hubs in 5,000, 4,097 and 2,049 nets of 2-4 pins (chunks of
        # 2,048 nets: 3, 3 and 2 of them), with costs that tie and differ
        r = vmo_gen.rng(9, 2)
        nets = []
        for hub, deg in ((0, 5000), (1, 4097), (2, 2049)):
            for i in range(deg):
                m = int(r.integers(1, 4))
                nets.append([hub] + sorted(int(v) for v in r.choice(np.arange(3, 6000), size=m, replace=False)))
        nets += [sorted(int(v) for v in r.choice(np.arange(3, 6000), size=3, replace=False)) for _ in range(3000)]
        h = oracle.hypergraph(6000, nets)
        h.c = r.integers(1, 3, size=h.l).astype(np.float32)
    elif case == "heavy":
        # column nets of Zipf rows: about 2% of the vertices lie in more than
        # 32 nets (up to 600), past the degree where a vertex's candidates are
        # scanned by a whole wavefront
        g = vmo_gen.zipf_rect(3000, 6000, 3, clip=600)
        h = oracle.colnet(g.m, g.n, g.rowptr, g.col)
        deg = np.diff(g.rowptr)
        assert (deg > 32).sum() > 20 and deg.max() > 200
    elif case == "random":
        g = vmo_gen.random_hypergraph_csr(3000, 2500, 1, maxdeg=6)
        h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
    elif case == "grid3d":
        g = vmo_gen.grid3d(12, seed=2)
        h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    elif case == "star":
        h = oracle.hypergraph(60, [[0, i] for i in range(1, 40)] + [[40, 41, 42], [41, 42, 43], [50, 51], [50, 51]])
    elif case == "pairs":
        # every net joins a matched pair (some twice): no net survives
        h = oracle.hypergraph(8, [[0, 1], [2, 3], [4, 5], [6, 7], [0, 1]])
    elif case == "short_nets":
        # empty and one-pin nets only: no image reaches two vertices
        h = oracle.hypergraph(8, [[], [3], [], [5]])
    else:
        h = weighted_case(4, 5000, 4000, maxdeg=80)
        h.c = vmo_gen.rng(4, 1).integers(1, 4, size=h.l).astype(np.float32)
    for level, comp in [(0, 0), (3, 17)]:
        pi, H = oracle.coarsen(h, 9, comp, level)
        gpi, gH = ctx.coarsen(dev_h(h), 9, comp, level)
        assert np.array_equal(host(gpi), pi)
        assert (gH.k, gH.l) == (H.k, H.l)
        assert np.array_equal(host(gH.net_ptr), H.ptr)
        assert np.array_equal(host(gH.pins)[:int(H.ptr[-1])], H.pins)
        assert np.array_equal(host(gH.w), H.w)
        assert np.array_equal(host(gH.c), H.c)


def compare_layout(gx, x):
    diag = float(np.linalg.norm(x.max(axis=1).astype(np.float64) - x.min(axis=1)))
    err = float(np.abs(gx.astype(np.float64) - x).max())
    assert err <= 1e-5 * diag, (err, diag)
    return err


@pytest.mark.parametrize("case", ["grid", "disconnected", "colnet"])
def test_full_layout(ctx, case):
    import paper_1105_4490_amd as P
    if case == "grid":
        g = vmo_gen.grid2d(32)
        h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
    elif case == "disconnected":
        a = vmo_gen.grid2d(12)
        nets = [list(a.col[a.rowptr[i]:a.rowptr[i + 1]]) for i in range(a.m)]
        nets += [[v + 144 for v in n] for n in nets] + [[290], []]
        h = oracle.hypergraph(300, nets)   # two grids, 1 net of one vertex, isolated vertices
    else:
        g = vmo_gen.zipf_rect(3000, 1500, 2, clip=50)
        h = oracle.colnet(g.m, g.n, g.rowptr, g.col)
    x = oracle.layout(h, oracle.layout_params(seed=5))
    gx = host(ctx.layout(dev_h(h), P.layout_params(seed=5)))
    compare_layout(gx, x)
    assert np.array_equal(gx, x), "layout not bit-identical"


def test_order_with_layout_inside(ctx):
    """vmo_order with x = NULL lays out first (the whole V+O path)."""
    import paper_1105_4490_amd as P
    g = vmo_gen.grid2d(32)
    h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
    o = ctx.order(dev_h(h), None, 16, 3, lp=P.layout_params(seed=5))
    x = oracle.layout(h, oracle.layout_params(seed=5))
    ref = oracle.order(h, x, 16, 3)
    from gpu_util import compare_order
    compare_order(o, ref, oracle.NET_MODE, h.k, h.l)


@pytest.mark.parametrize("side", [48, 64, 104])
def test_full_size_gradient_sampled(ctx, side):
    """The 7-point pattern of side^3 vertices, symmetric model (48: 110,592
    vertices, walk parts spread; 64: the benchmark size, and 104: 1,124,864
    vertices, both above the 200,000 points where the walk stops spreading),
    at clustered synthetic coordinates: the gradient checked at 2000 sampled
    vertices against the oracle."""
    g = vmo_gen.grid3d(side, seed=1)
    h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    dh = dev_h(h)
    x = vmo_gen.random_points(h.k, side, clusters=64, spread=0.3)
    gy, _, nint = ctx.gradient(dh, dev_x(x))
    ids = vmo_gen.rng(1, 77).choice(h.k, size=2000, replace=False).astype(np.int32)
    y, cnt = oracle.gradient_sample(h, x, ids)
    assert np.array_equal(host(gy)[:, ids], y)
    assert nint > 0


# --------------------------------------------- plain reference, tolerance ----

def check_plain_gradient(gy, y, s):
    gy = np.asarray(gy, np.float64)
    bad = np.abs(gy - y) > 1e-5 * s
    assert not bad.any(), (int(bad.sum()), float((np.abs(gy - y) / np.maximum(s, 1e-300)).max()))


@pytest.mark.parametrize("seed,k,l,theta", [(1, 300, 200, 0.0), (2, 3000, 2500, 0.5), (4, 4096, 3000, 0.5),
                                           (5, 4097, 3000, 0.5), (3, 40000, 30000, 0.5)])
def test_gradient_against_plain(ctx, seed, k, l, theta):
    """vmo_gradient against the plain FP64 evaluation of eq. (7), element by
    element; the kernel's interaction count equals the plain walks' total at
    every size."""
    h = weighted_case(seed, k, l)
    x = vmo_gen.random_points(k, seed, clusters=6)
    y, s, nint = oracle.gradient_plain(h, x, theta=theta)
    gy, _, gcount = ctx.gradient(dev_h(h), dev_x(x), theta=theta)
    check_plain_gradient(host(gy), y, s)
    assert gcount == int(nint.sum())


@pytest.mark.parametrize("k", [3000, 9000])
def test_gradient_coincident_points_against_plain(ctx, k):
    h = weighted_case(11, k, k // 2)
    x = np.round(vmo_gen.random_points(k, 11, clusters=3)).astype(np.float32)
    y, s, nint = oracle.gradient_plain(h, x, theta=0.5)
    gy, _, gcount = ctx.gradient(dev_h(h), dev_x(x), theta=0.5)
    check_plain_gradient(host(gy), y, s)
    assert gcount == int(nint.sum())


@pytest.mark.parametrize("side", [48, 64])
def test_full_size_gradient_against_plain(ctx, side):
    """The 7-point pattern of side^3 vertices (64: the benchmark size), at
    clustered coordinates: every vertex's gradient against the plain
    evaluation, and the walk's interaction count (the numerator of the
    measured flop rate) against the plain walks' total."""
    g = vmo_gen.grid3d(side, seed=1)
    h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    x = vmo_gen.random_points(h.k, side, clusters=64, spread=0.3)
    y, s, nint = oracle.gradient_plain(h, x)
    gy, _, gcount = ctx.gradient(dev_h(h), dev_x(x))
    check_plain_gradient(host(gy), y, s)
    assert gcount == int(nint.sum())


def check_plain_step(gx, xr):
    diag = float(np.linalg.norm(xr.max(axis=1).astype(np.float64) - xr.min(axis=1)))
    tol = 1e-5 * np.maximum(np.abs(xr.astype(np.float64)), diag)
    err = np.abs(gx.astype(np.float64) - xr)
    assert (err <= tol).all(), (int((err > tol).sum()), float(err.max()), diag)


@pytest.mark.parametrize("case", ["grid", "weighted", "grid3d"])
def test_descent_steps_against_plain(ctx, case):
    """Twelve descent steps of Algorithm 3, one call each: every GPU step,
    from the GPU's own state, against the plain FP64 step from the same FP32
    state (same tree decisions; only the rounding differs).  The step length
    is set from the same box in FP64 on both sides and must agree exactly."""
    import paper_1105_4490_amd as P
    if case == "grid":
        g = vmo_gen.grid2d(24)
        h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
    elif case == "weighted":
        h = weighted_case(7, 2000, 1500)
    else:
        g = vmo_gen.grid3d(34, seed=3)       # 39,304 vertices: the multi-kernel tree, spread walk
        h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    p = oracle.layout_params(seed=3)
    gp = P.layout_params(seed=3)
    dh = dev_h(h)
    gx = dev_x(oracle.layout_init(h.k, 3))
    ga = 0.0
    for it in range(12):
        x0 = host(gx).copy()
        xr, _, _, a = oracle.layout_iter_plain(h, x0, p, it, ga)
        ga = ctx.layout_steps(dh, gx, gp, it, 1, ga)
        assert ga == a
        check_plain_step(host(gx), xr)


def test_descent_steps_40k_strict(ctx):
    """Twelve strict descent steps at 39,304 points (the multi-kernel tree
    build, the spread walk, k_attract above 16,384 points, the step applied by
    k_combine), bit for bit against the oracle's strict steps."""
    import paper_1105_4490_amd as P
    g = vmo_gen.grid3d(34, seed=3)
    h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    p = oracle.layout_params(seed=3)
    gp = P.layout_params(seed=3)
    x = oracle.layout_init(h.k, 3)
    xo, a = x.copy(), 0.0
    for it in range(12):
        xo, _, a = oracle.layout_iter(h, xo, p, it, a)
    gx = dev_x(x)
    ga = ctx.layout_steps(dev_h(h), gx, gp, 0, 12, 0.0)
    assert ga == a
    assert np.array_equal(host(gx), xo)
