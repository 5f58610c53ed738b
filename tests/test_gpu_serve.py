"""Serving with continuous batching (vmo_serve_*): each job's result equals
the oracle's ordering of that job alone, whatever else is resident; jobs that
do not fit the memory budget wait for room; jobs laid out at admission match
the whole-path ordering; impossible jobs are refused."""
import time

import numpy as np
import pytest

import oracle
import vmo_gen
from gpu_util import compare_order, dev_h, dev_x

pytestmark = pytest.mark.gpu


def job_set(n, seed, scale=1):
    r = vmo_gen.rng(seed, 31)
    out = []
    for j in range(n):
        kind = j % 3
        if kind == 0:
            g = vmo_gen.banded(int(r.integers(300, 2500)) * scale, int(r.integers(5, 30)), seed * 97 + j)
            h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
            mode, ordr = 0, 0
        elif kind == 1:
            g = vmo_gen.grid3d(int(r.integers(4, 11)), seed=j + 1)
            h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
            mode, ordr = 1, 1
        else:
            g = vmo_gen.zipf_rect(int(r.integers(300, 3000)) * scale, 600, seed * 97 + j)
            h = oracle.colnet(g.m, g.n, g.rowptr, g.col)
            mode, ordr = 0, 1
        x = vmo_gen.random_points(h.k, seed * 1000 + j, clusters=3)
        P = int(r.integers(2, 33))
        ref = oracle.order(h, x, P, 9, mode=mode, ord=ordr, job=100 + j)
        out.append(({"h": dev_h(h), "x": dev_x(x), "P": P, "seed": 9, "mode": mode, "order": ordr,
                     "job_index": 100 + j}, (h, ref, mode)))
    return out


def test_serve_mix_equals_alone_and_oracle():
    import paper_1105_4490_amd as P
    jobs = job_set(12, 3)
    srv = P.Server(budget_bytes=256 << 20, max_jobs=64)
    tickets = [srv.submit(j) for j, _ in jobs[:6]]
    time.sleep(0.01)
    tickets += [srv.submit(j) for j, _ in jobs[6:]]      # arrive while the first ones run
    for t, (_, (h, ref, mode)) in zip(tickets, jobs):
        o, lat = srv.wait(t)
        compare_order(o, ref, mode, h.k, h.l)
        assert lat > 0
    st = srv.stats()
    assert st["completed"] == 12 and st["ticks"] > 0
    # continuous batching: ticks ran the segments of several jobs together
    assert st["max_tick_jobs"] > 1 and st["tick_jobs"] > st["ticks"]
    srv.close()
    # the same job alone on a fresh server
    srv = P.Server(budget_bytes=64 << 20, max_jobs=4)
    j, (h, ref, mode) = jobs[4]
    o, _ = srv.wait(srv.submit(j))
    compare_order(o, ref, mode, h.k, h.l)
    srv.close()


def test_serve_admission_waits_for_room():
    """A budget that holds only a few jobs at a time: the rest queue and all finish right."""
    import paper_1105_4490_amd as P
    jobs = job_set(9, 5)
    srv = P.Server(budget_bytes=10 << 20, max_jobs=3)
    tickets = [srv.submit(j) for j, _ in jobs]
    for t, (_, (h, ref, mode)) in zip(tickets, jobs):
        o, _ = srv.wait(t)
        compare_order(o, ref, mode, h.k, h.l)
    srv.close()


def test_serve_refuses_jobs_larger_than_the_arena():
    import paper_1105_4490_amd as P
    srv = P.Server(budget_bytes=1 << 20, max_jobs=2)    # about 1.6k vertex slots
    g = vmo_gen.grid2d(128)
    h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
    with pytest.raises(P.VmoError):
        srv.submit({"h": dev_h(h), "x": dev_x(vmo_gen.random_points(h.k, 1)), "P": 4, "seed": 1})
    srv.close()


@pytest.mark.parametrize("threads", [0, 4])
def test_serve_with_layout_at_admission(threads):
    """Jobs without coordinates are laid out after admission (by the serving
    thread, or by layout threads running beside the ticks); every result
    equals the oracle's whole path (layout, then ordering)."""
    import paper_1105_4490_amd as P
    srv = P.Server(budget_bytes=64 << 20, max_jobs=8, layout_threads=threads)
    jobs = []
    for i, side in enumerate((24, 13, 18, 9, 21, 16)):
        g = vmo_gen.grid2d(side, side + i % 3)
        h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
        seed = 4 + i
        t = srv.submit({"h": dev_h(h), "x": None, "P": 8, "seed": 2, "job_index": i}, lp=P.layout_params(seed=seed))
        jobs.append((t, h, seed, i))
    for t, h, seed, i in jobs:
        o, _ = srv.wait(t)
        x = oracle.layout(h, oracle.layout_params(seed=seed))
        compare_order(o, oracle.order(h, x, 8, 2, job=i), oracle.NET_MODE, h.k, h.l)
    srv.close()


def test_layout_bytes_bounds_the_layout_workspace():
    """The footprint the server admits layouts by (vmo_layout_bytes) bounds
    what a layout's workspace takes: a fresh context's pool after one layout."""
    import paper_1105_4490_amd as P
    cases = []
    g = vmo_gen.grid3d(20, seed=1)
    cases.append(oracle.symmetric(g.m, g.n, g.rowptr, g.col))
    g = vmo_gen.zipf_rect(20000, 10000, 2)
    cases.append(oracle.colnet(g.m, g.n, g.rowptr, g.col))
    g = vmo_gen.grid2d(32)
    cases.append(oracle.rownet(g.m, g.n, g.rowptr, g.col))
    g = vmo_gen.grid3d(64, seed=1)
    cases.append(oracle.symmetric(g.m, g.n, g.rowptr, g.col))
    for h in cases:
        ctx = P.Context(0)
        dh = dev_h(h)
        ctx.layout(dh, P.layout_params(seed=1))
        ctx.sync()
        held = ctx.pool_bytes()
        bound = P.Context.layout_bytes(h.k, h.l, int(h.ptr[-1]))
        print("layout workspace k", h.k, "held", held, "bound", bound, flush=True)
        assert 0 < held <= bound, (h.k, held, bound)
        ctx.close()


def test_serve_layouts_admitted_by_footprint():
    """A layout share that holds one layout at a time: the layouts of the
    jobs wait for one another, the peak footprint in flight stays within the
    share, and every result equals the oracle's whole path."""
    import paper_1105_4490_amd as P
    jobs_h = []
    for i, side in enumerate((20, 14, 17, 11)):
        g = vmo_gen.grid2d(side, side + 1)
        jobs_h.append(oracle.rownet(g.m, g.n, g.rowptr, g.col))
    need = max(P.Context.layout_bytes(h.k, h.l, int(h.ptr[-1])) for h in jobs_h)
    budget = int(need / 0.6 * 2 * 1.2)          # half of the 60 % layout share holds one layout
    srv = P.Server(budget_bytes=max(budget, 2 << 20), max_jobs=8, layout_threads=4)
    tickets = []
    for i, h in enumerate(jobs_h):
        t = srv.submit({"h": dev_h(h), "x": None, "P": 8, "seed": 2, "job_index": i}, lp=P.layout_params(seed=3 + i))
        tickets.append(t)
    for i, (t, h) in enumerate(zip(tickets, jobs_h)):
        o, _ = srv.wait(t)
        x = oracle.layout(h, oracle.layout_params(seed=3 + i))
        compare_order(o, oracle.order(h, x, 8, 2, job=i), oracle.NET_MODE, h.k, h.l)
    st = srv.stats()
    assert 0 < st["layout_bytes_peak"] <= st["layout_budget_bytes"] // 2
    srv.close()
