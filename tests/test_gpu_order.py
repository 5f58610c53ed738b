"""GPU parity of the ordering path against the CPU oracle, through the C ABI:
models and dual, components, cut, one 2-means split, recursive SBD/BBD in
net and graph mode, batched and plain forms.  Integer and index results are
compared bit for bit; the FP32 centres too (they are fixed by exact integer
sums and a specified FP64 evaluation)."""
import numpy as np
import pytest
import torch

import oracle
import vmo_gen
from gpu_util import compare_order, dev_h, dev_x, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1105_4490_amd as P
    return P.Context(0)


def csr_dev(g):
    return torch.as_tensor(g.rowptr).cuda(), torch.as_tensor(g.col).cuda()


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_models_and_dual(ctx, kind):
    g = vmo_gen.grid3d(6, seed=3) if kind == 2 else vmo_gen.zipf_rect(3000, 1700, 5, clip=60)
    rp, cl = csr_dev(g)
    h = ctx.model(kind, g.m, g.n, rp, cl)
    ref = oracle.model(kind, g.m, g.n, g.rowptr, g.col)
    assert (h.k, h.l) == (ref.k, ref.l)
    assert np.array_equal(host(h.net_ptr), ref.ptr)
    assert np.array_equal(host(h.pins)[:int(ref.ptr[-1])], ref.pins)
    d = ctx.dual(h)
    dref = oracle.dual(ref)
    assert np.array_equal(host(d.net_ptr), dref.ptr)
    assert np.array_equal(host(d.pins)[:int(dref.ptr[-1])], dref.pins)


@pytest.mark.parametrize("seed", [1, 2])
def test_components(ctx, seed):
    g = vmo_gen.random_hypergraph_csr(20000, 9000, seed, maxdeg=3, empty_frac=0.05)
    h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
    lab = ctx.components(dev_h(h))
    assert np.array_equal(host(lab), oracle.components(h))


def test_components_grid(ctx):
    """One component with long paths and randomly numbered vertices (the
    symmetric 3-D grid, rows permuted), and the same grid keeping every third
    edge (many components of all sizes)."""
    g = vmo_gen.grid3d(40, seed=5)
    h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    lab = host(ctx.components(dev_h(h)))
    assert np.array_equal(lab, oracle.components(h)) and not lab.any()
    keep = np.arange(h.l) % 3 == 0
    nets = [list(h.pins[h.ptr[e]:h.ptr[e + 1]]) for e in range(h.l) if keep[e]]
    h2 = oracle.hypergraph(h.k, nets)
    lab2 = host(ctx.components(dev_h(h2)))
    assert np.array_equal(lab2, oracle.components(h2))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_cut(ctx, seed):
    g = vmo_gen.random_hypergraph_csr(5000, 4000, seed, maxdeg=9)
    # a few large nets take the sort path
    rows = [list(g.col[g.rowptr[i]:g.rowptr[i + 1]]) for i in range(g.m)]
    r = vmo_gen.rng(seed, 11)
    rows += [sorted(r.choice(5000, size=300 + 100 * j, replace=False).tolist()) for j in range(5)]
    h = oracle.hypergraph(5000, rows)
    h.c = r.integers(1, 7, size=h.l).astype(np.float32)
    h.w = r.integers(1, 4, size=h.k).astype(np.float32)
    P = 37
    part = r.integers(0, P, size=h.k).astype(np.int32)
    got = ctx.cut(dev_h(h), torch.as_tensor(part).cuda(), P)
    ref = oracle.cut(h, part, P)
    assert got["lambda_minus_one"] == ref["lambda_minus_one"]
    assert got["cut_net"] == ref["cut_net"]
    assert got["nets_cut"] == ref["nets_cut"]
    assert np.array_equal(host(got["part_weight"]), ref["part_weight"])
    check_max_split(got, h, part, P)


def check_max_split(got, h, part, P):
    sp, graph = oracle.split_cuts(h, part, P)
    assert got["separators"] == graph
    assert got["max_split"] == sp.max()
    assert got["max_split_node"] == (int(np.argmax(sp)) if sp.max() > 0 else 0)


@pytest.mark.parametrize("seed", [4, 5])
def test_cut_non_integer_weights_and_costs(ctx, seed):
    """Weights and costs spread over several orders of magnitude: the part
    weights (added per part in ascending vertex id) and the per-split cut
    (per node in ascending net id) equal the oracle's bit for bit; the FP64
    totals, summed in another fixed order, agree within (l + 1) 2^-53 of the
    total, and are the same on a second run."""
    g = vmo_gen.random_hypergraph_csr(6000, 5000, seed, maxdeg=9)
    h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
    r = vmo_gen.rng(seed, 13)
    h.w = (10.0 ** r.uniform(-4, 4, size=h.k)).astype(np.float32)
    h.c = (10.0 ** r.uniform(-3, 3, size=h.l)).astype(np.float32)
    P = 29
    part = r.integers(0, P, size=h.k).astype(np.int32)
    dh, dp = dev_h(h), torch.as_tensor(part).cuda()
    got = ctx.cut(dh, dp, P)
    again = ctx.cut(dh, dp, P)
    ref = oracle.cut(h, part, P)
    assert np.array_equal(host(got["part_weight"]), ref["part_weight"])
    assert got["nets_cut"] == ref["nets_cut"]
    for f in ("lambda_minus_one", "cut_net"):
        assert abs(got[f] - ref[f]) <= (h.l + 1) * 2.0 ** -53 * ref[f], f
        assert got[f] == again[f]
    check_max_split(got, h, part, P)


@pytest.mark.parametrize("k,seed,clusters", [(2, 1, 0), (1000, 2, 3), (4099, 3, 0), (70001, 4, 5), (262144, 5, 0)])
def test_bisect(ctx, k, seed, clusters):
    x = vmo_gen.random_points(k, seed, clusters=clusters)
    got = ctx.bisect(dev_x(x), seed)
    ref = oracle.bisect(x, seed)
    assert got["split"] == ref.split
    assert np.array_equal(host(got["side"]), ref.side)
    assert np.array_equal(host(got["centres"]), ref.centres)
    assert got["iters"] == ref.iters


def test_bisect_d2_draw_hand_derived(ctx):
    """The k-means++ draw of golden/d2_draw.json (t on a prefix sum exactly):
    with t_max = 0 vmo_bisect reports the seed points as the centres."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "d2_draw.json")) as f:
        g = json.load(f)
    q = np.array(g["points_q"], dtype=np.int64)
    x = np.ascontiguousarray(q.T.astype(np.float32))
    got = ctx.bisect(dev_x(x), g["seed"], t_max=0)
    cen = host(got["centres"])
    assert got["split"] and got["iters"] == 0
    assert np.array_equal(cen[0], q[g["i1"]].astype(np.float32))
    assert np.array_equal(cen[1], q[g["i2"]].astype(np.float32))


def test_bisect_degenerate(ctx):
    for x in (np.ones((4, 50), np.float32), np.zeros((4, 1), np.float32)):
        got = ctx.bisect(dev_x(x), 1)
        assert not got["split"] and not host(got["side"]).any()


def grid_coords(N, seed, perm_seed):
    perm = vmo_gen.rng(perm_seed, 2).permutation(N ** 3)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(N ** 3)
    x = np.zeros((4, N ** 3), np.float32)
    x[0], x[1], x[2] = inv % N, (inv // N) % N, inv // (N * N)
    x += vmo_gen.rng(seed, 9).standard_normal(x.shape).astype(np.float32) * 0.1
    return x


@pytest.mark.parametrize("N,P,ordr", [(8, 8, 1), (16, 64, 1), (16, 13, 0), (20, 64, 1)])
def test_order_graph_mode(ctx, N, P, ordr):
    g = vmo_gen.grid3d(N, seed=N)
    h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    x = grid_coords(N, 1, N)
    dh = dev_h(h)
    got = ctx.order(dh, dev_x(x), P, 7, mode=1, order=ordr)
    ref = oracle.order(h, x, P, 7, mode=oracle.GRAPH_MODE, ord=ordr)
    compare_order(got, ref, oracle.GRAPH_MODE, h.k, h.l)
    # the cut call's maximum split cut (|S_h| here) is the ordering's own
    c = ctx.cut(dh, got["part"], P)
    assert c["separators"] and c["max_split"] == ref.split_cut[:ref.n_nodes].max()


@pytest.mark.parametrize("case", ["grid", "zipf", "tiny", "costs"])
@pytest.mark.parametrize("ordr", [0, 1])
def test_order_net_mode(ctx, case, ordr):
    if case == "grid":
        g = vmo_gen.grid2d(32)
        h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
        x = oracle.layout(h, oracle.layout_params(seed=3))
        P = 16
    elif case in ("zipf", "costs"):
        g = vmo_gen.zipf_rect(20000, 10000, 3)
        h = oracle.colnet(g.m, g.n, g.rowptr, g.col)
        x = vmo_gen.random_points(h.k, 3, clusters=20)
        P = 256
        if case == "costs":
            # non-integer costs over seven orders of magnitude: the split cuts
            # are FP64 sums whose value depends on their order
            r = vmo_gen.rng(3, 9)
            h.c = (r.uniform(0.1, 1.0, h.l) * 10.0 ** r.integers(-3, 4, h.l)).astype(np.float32)
    else:
        h = oracle.hypergraph(7, [[0, 1], [], [2, 3, 4], [5, 6], [0, 6], []])
        x = vmo_gen.random_points(7, 4)
        P = 5
    dh = dev_h(h)
    got = ctx.order(dh, dev_x(x), P, 11, mode=0, order=ordr)
    ref = oracle.order(h, x, P, 11, mode=oracle.NET_MODE, ord=ordr)
    compare_order(got, ref, oracle.NET_MODE, h.k, h.l)
    # the cut call's maximum split cut (nets cut at each node) is the ordering's own
    c = ctx.cut(dh, got["part"], P)
    assert not c["separators"] and c["max_split"] == ref.split_cut[:ref.n_nodes].max()


def test_order_degenerate(ctx):
    for h, x, P in [(oracle.hypergraph(1, [[0], []]), np.zeros((4, 1), np.float32), 4),
                    (oracle.hypergraph(6, [[0, 1], [2, 3, 4, 5]]), np.ones((4, 6), np.float32), 4),
                    (oracle.hypergraph(6, [[0, 1], [2, 3, 4, 5]]), vmo_gen.random_points(6, 1), 1)]:
        got = ctx.order(dev_h(h), dev_x(x), P, 3)
        ref = oracle.order(h, x, P, 3)
        compare_order(got, ref, oracle.NET_MODE, h.k, h.l)


def test_order_rejects_bad_input(ctx):
    import paper_1105_4490_amd as P
    h = oracle.hypergraph(3, [[0, 1, 2]])
    with pytest.raises(P.VmoError):
        ctx.order(dev_h(h), dev_x(np.zeros((4, 3), np.float32)), 2, 1, mode=1)
    bad = oracle.Hypergraph(3, 1, np.array([0, 2], np.int64), np.array([2, 1], np.int32))
    with pytest.raises(P.VmoError):
        ctx.order(dev_h(bad), dev_x(np.zeros((4, 3), np.float32)), 2, 1)
    x = np.zeros((4, 3), np.float32)
    x[0, 1] = np.nan
    with pytest.raises(P.VmoError):
        ctx.order(dev_h(h), dev_x(x), 2, 1)


def mixed_jobs(n_jobs, seed):
    r = vmo_gen.rng(seed, 21)
    jobs, refs = [], []
    for j in range(n_jobs):
        kind = j % 3
        if kind == 0:
            g = vmo_gen.banded(int(r.integers(500, 3000)), int(r.integers(5, 40)), seed * 100 + j)
            h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
            mode, ordr = 0, 0
        elif kind == 1:
            g = vmo_gen.grid3d(int(r.integers(5, 12)), seed=j)
            h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
            mode, ordr = 1, 1
        else:
            g = vmo_gen.zipf_rect(int(r.integers(500, 4000)), 700, seed * 100 + j)
            h = oracle.colnet(g.m, g.n, g.rowptr, g.col)
            mode, ordr = 0, 1
        x = vmo_gen.random_points(h.k, seed * 1000 + j, clusters=4)
        P = int(r.integers(8, 33))
        jobs.append({"h": dev_h(h), "x": dev_x(x), "P": P, "seed": 5, "mode": mode, "order": ordr, "job_index": j})
        refs.append((h, oracle.order(h, x, P, 5, mode=mode, ord=ordr, job=j), mode))
    return jobs, refs


@pytest.mark.parametrize("plain", [False, True])
def test_order_batch_equals_single(ctx, plain):
    jobs, refs = mixed_jobs(12, 4)
    outs = ctx.order_batch(jobs, plain=plain)
    for o, (h, ref, mode) in zip(outs, refs):
        compare_order(o, ref, mode, h.k, h.l)


def test_order_full_size_graph_mode(ctx):
    """The 64^3 7-point pattern, symmetric model, 64 parts, BBD: exact."""
    N = 64
    g = vmo_gen.grid3d(N, seed=1)
    h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    x = grid_coords(N, 2, 1)
    got = ctx.order(dev_h(h), dev_x(x), 64, 1, mode=1, order=1)
    ref = oracle.order(h, x, 64, 1, mode=oracle.GRAPH_MODE, ord=oracle.BBD)
    compare_order(got, ref, oracle.GRAPH_MODE, h.k, h.l)


def test_order_full_size_column_net(ctx):
    """200,000 x 100,000, Zipf(2) row degrees clipped to 2000, column-net, 256
    parts, SBD: ordering, permutations, split cuts and the cut metrics of the
    result exact at full size (clustered synthetic coordinates)."""
    g = vmo_gen.zipf_rect(200000, 100000, seed=3)
    h = oracle.colnet(g.m, g.n, g.rowptr, g.col)
    assert (h.k, h.l) == (200000, 100000)
    x = vmo_gen.random_points(h.k, 3, clusters=64, spread=0.3)
    dh = dev_h(h)
    got = ctx.order(dh, dev_x(x), 256, 3, mode=0, order=0)
    ref = oracle.order(h, x, 256, 3, mode=oracle.NET_MODE, ord=oracle.SBD)
    compare_order(got, ref, oracle.NET_MODE, h.k, h.l)
    c = ctx.cut(dh, got["part"], 256)
    cr = oracle.cut(h, ref.part, 256)
    assert c["lambda_minus_one"] == cr["lambda_minus_one"] and c["cut_net"] == cr["cut_net"]
    assert c["nets_cut"] == cr["nets_cut"]


def test_order_batch_full_count_sampled(ctx):
    """512 banded matrices of the batched mix (rows log-uniform in
    [1e3, 5e4], half bandwidth 5-40, 0.1 % off-band, 8-32 parts, row-net,
    SBD) ordered by one batched call; 32 jobs of at most 1e4 rows are
    checked against the oracle, every job's permutation is a bijection with
    parts in range."""
    mats = vmo_gen.batch_banded(512, seed=2)
    jobs = []
    for i, (g, parts) in enumerate(mats):
        rp, cl = csr_dev(g)
        dh = ctx.model(0, g.m, g.n, rp, cl)
        x = vmo_gen.random_points(g.m, 7000 + i, clusters=3)
        jobs.append({"h": dh, "x": dev_x(x), "P": parts, "seed": 4, "mode": 0, "order": 0, "job_index": i})
    outs = ctx.order_batch(jobs)
    for (g, parts), o in zip(mats, outs):
        vp = host(o["vperm"])
        assert np.array_equal(np.sort(vp), np.arange(g.m))
        pa = host(o["part"])
        assert pa.min() >= 0 and pa.max() < parts
    small = [i for i, (g, _) in enumerate(mats) if g.m <= 10000]
    sample = small[:: max(1, len(small) // 32)][:32]
    assert len(sample) >= 16
    for i in sample:
        g, parts = mats[i]
        h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
        x = vmo_gen.random_points(g.m, 7000 + i, clusters=3)
        ref = oracle.order(h, x, parts, 4, mode=oracle.NET_MODE, ord=oracle.SBD, job=i)
        compare_order(outs[i], ref, oracle.NET_MODE, h.k, h.l)


def test_order_batch_rejects_bad_job(ctx):
    """One invalid job (a pin out of range) fails the batch and is named."""
    import paper_1105_4490_amd as P
    jobs, _ = mixed_jobs(5, 8)
    bad = oracle.Hypergraph(3, 1, np.array([0, 2], np.int64), np.array([0, 7], np.int32))
    jobs[3] = {"h": dev_h(bad), "x": dev_x(np.zeros((4, 3), np.float32)), "P": 2, "seed": 1, "mode": 0, "order": 0,
               "job_index": 3}
    with pytest.raises(P.VmoError, match="job 3"):
        ctx.order_batch(jobs)
