"""Throughput of the geometric ordering path on one MI355X.

Workload: the 3-D 7-point Laplacian pattern on a 64^3 grid (262,144 rows,
1,810,432 nonzeros) with rows and columns permuted by one seeded
permutation, symmetric hypergraph model, 64 parts, recursive BBD order with
the vertex separators of Algorithm 7, FP32 coordinates from the multilevel
layout.  One step = the whole path on device-resident CSR input: hypergraph
model, layout (components, coarsening, descent with the tree walk,
prolongation, packing), recursive 2-means ordering with separators and
emission, and the cut metrics of the result.

Prints one JSON line (see the field list at the end of main()).

Two more workloads are measured by their own modes (one JSON line each):
  --mode batch   512 banded matrices (rows log-uniform in [1e3, 5e4], half
                 bandwidth 5-40, 0.1 % off-band entries, 8-32 parts each,
                 row-net, SBD), coordinates laid out beforehand: recursive
                 ordering of all of them by one segmented launch sequence per
                 level, against the same work done one subproblem at a time.
  --mode serve   a Poisson stream of ordering jobs (nnz log-uniform in
                 [1e3, 1e7], uniform over the three matrix shapes), submitted to
                 the continuous-batching server at their arrival times; p50/p99
                 latency and nnz/s.
"""
import argparse
import json
import math
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

P_PARTS = 64
N_SIDE = 64
SEED = 1
SCHUR_P3 = 8         # parts of each separator block in the Schur-complement recursion
# Algorithmic flops of one interaction (one term of the repulsion in eq. (7)),
# the count fixed for this measurement (the kernel executes about 26 VALU
# instructions per interaction: 4 sub, r^2 as 1 mul + 3 fma, 2 mul, the IEEE
# division's 11, 4 fma, and the zero-distance select).
FLOPS_PER_INTERACTION = 20
# HBM bytes per walk launch (average over the walk launches of one counting and
# one timed step of this workload), from two
# rocprofv3 --pmc passes (FETCH_SIZE x 2.000, WRITE_SIZE x 1.000: the factors a
# plain copy of known size gives); profiles/k_walk_grid3d64_traffic.md
WALK_TRAFFIC_BYTES = 111.16e6 + 29.28e6
PEAK_FP32_VALU_TFLOPS = 157.3        # 256 CUs x 128 FP32 lanes (packed) x 2 (fma) x 2.4 GHz
PEAK_FP32_UNPACKED_TFLOPS = 78.6     # the same without packed FP32 (this build disables it)
# live timing brackets every PROFILE_EVERY-th launch of a kernel with HIP
# events: an event pair costs about 13 us of stream time, 2.5 % of a step when
# every walk is timed.  3 is prime to the 700 walk launches of a step, so over
# the timed steps the timed launches cover every launch position of the step.
PROFILE_EVERY = 3
PEAK_HBM_GBS = 8000.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2,
                    help="untimed steps (the launch tuner settles during the first steps)")
    ap.add_argument("--side", type=int, default=N_SIDE, help="grid side of the workload (64 = the 64^3 case)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--path-only", action="store_true",
                    help="only the timed V+O steps (no order-only, border, Schur or LU-ordering fields)")
    ap.add_argument("--cpu-side", type=int, default=48, help="grid side of the oracle's all-cores V+O sample")
    ap.add_argument("--cpu-side1", type=int, default=28, help="grid side of the oracle's one-thread V+O sample")
    ap.add_argument("--cpu-threads", type=int, default=16,
                    help="host threads of the oracle's all-cores leg (capped at the cores this process may use)")
    ap.add_argument("--no-batch", action="store_true", help="path mode: leave out the batched-ordering field")
    ap.add_argument("--no-serve", action="store_true", help="path mode: leave out the serving field")
    ap.add_argument("--no-zipf", action="store_true",
                    help="path mode: leave out the rectangular Zipf V+O field (200,000 x 100,000, column-net)")
    ap.add_argument("--mode", choices=("path", "batch", "serve", "zipf", "copy"), default="path",
                    help="copy: a plain 256 MiB device copy, three times (calibrates the HBM byte counters); "
                         "zipf: only the rectangular Zipf V+O field")
    ap.add_argument("--jobs", type=int, default=512, help="batch mode: number of matrices")
    ap.add_argument("--layout-threads", type=int, default=4, help="batch mode: streams laying out the matrices")
    ap.add_argument("--no-plain", action="store_true", help="batch mode: skip the plain per-subproblem form")
    ap.add_argument("--requests", type=int, default=40, help="serve mode: number of requests")
    ap.add_argument("--rate", type=float, default=200.0, help="serve mode: arrivals per second")
    ap.add_argument("--nnz-max", type=float, default=1e7, help="serve mode: largest nnz of a request")
    ap.add_argument("--serve-budget-gib", type=int, default=64,
                    help="serve mode: device memory of the server (40 %% arenas, 60 %% layouts)")
    ap.add_argument("--serve-threads", type=int, default=4, help="serve mode: layout threads")
    ap.add_argument("--no-stable", action="store_true",
                    help="serve mode: skip the second stream at half the measured capacity")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU design is described, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.mode == "copy":
        return copy_calibration()

    import paper_1105_4490_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_1105_4490_amd import build as b
        b.build()
    import vmo_gen

    torch.cuda.set_device(0)
    ctx = P.Context(0)
    if args.mode == "batch":
        return bench_batch(args, ctx)
    if args.mode == "serve":
        return bench_serve(args, ctx)
    if args.mode == "zipf":
        print(json.dumps(bench_zipf(ctx, P.layout_params(seed=SEED), args.steps)))
        return None
    g = vmo_gen.grid3d(args.side, seed=SEED)
    nnz = g.nnz
    rowptr = torch.as_tensor(g.rowptr).cuda()
    col = torch.as_tensor(g.col).cuda()
    lp = P.layout_params(seed=SEED)

    def step():
        h = ctx.model(P.SYMMETRIC, g.m, g.n, rowptr, col)
        o = ctx.order(h, None, P_PARTS, SEED, mode=P.GRAPH, order=P.BBD, lp=lp)
        c = ctx.cut(h, o["part"], P_PARTS)
        return o, c

    for _ in range(args.warmup):
        o, c = step()
    torch.cuda.synchronize()
    # one untimed step with every walk counting its interactions (the same in
    # every step: the inputs and the arithmetic are fixed), then the timed
    # steps with every PROFILE_EVERY-th walk timed in its uncounted form
    ctx.profile(True, every=1)
    ctx.profile_reset()
    step()
    torch.cuda.synchronize()
    counted = ctx.profile_read("walk")
    ctx.profile(False)
    ctx.profile(True, every=PROFILE_EVERY, count=False)
    ctx.profile_reset()
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        o, c = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    walk = ctx.profile_read("walk")
    assign = ctx.profile_read("assign")
    ctx.profile(False)
    dt = t1 - t0
    value = nnz * args.steps / dt
    ms = 1e3 * dt / args.steps

    ipl = counted["work"] / max(counted["launches"], 1)  # interactions per walk launch
    avg_ms = walk["total_ms"] / max(walk["launches"], 1)
    w_tflops = FLOPS_PER_INTERACTION * ipl / (avg_ms * 1e-3) / 1e12 if avg_ms > 0 else 0.0
    roof = {"bound": "alu", "kernel": "k_walk", "achieved": round(w_tflops, 3), "peak": PEAK_FP32_VALU_TFLOPS,
            "unit": "TFLOP/s", "frac": round(w_tflops / PEAK_FP32_VALU_TFLOPS, 4),
            "flops_per_interaction": FLOPS_PER_INTERACTION,
            "frac_of_unpacked_peak": round(w_tflops / PEAK_FP32_UNPACKED_TFLOPS, 4),
            "traffic": WALK_TRAFFIC_BYTES if args.side == N_SIDE else None,
            "launches_timed": walk["launches"], "timed_every": PROFILE_EVERY,
            "avg_launch_ms": round(avg_ms, 4),
            "share_of_step": round(walk["total_ms"] * PROFILE_EVERY / (1e3 * dt), 4),
            "interactions_per_launch": ipl, "launches_counted": counted["launches"]}
    a_gbs = assign["work"] / (assign["total_ms"] * 1e-3) / 1e9 if assign["total_ms"] > 0 else 0.0

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_side, args.cpu_side1, args.cpu_threads)

    n_nodes = int(o["n_nodes"].item())
    sep = float(o["split_cut"][:n_nodes].sum().item())
    line = {
        "metric": "matrix nnz ordered/sec (full recursive SBD/BBD)",
        "value": value, "unit": "nnz/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"3-D 7-point Laplacian {args.side}^3 ({g.m} rows, {nnz} nnz), rows/cols permuted, "
                               f"symmetric hypergraph, {P_PARTS} parts, recursive BBD with separators, "
                               "layout + order (V+O) from device-resident CSR",
                   "parts": P_PARTS, "seed": SEED},
        "latency_ms": {"p50": 1e3 * statistics.median(lat), "p99": 1e3 * sorted(lat)[min(len(lat) - 1,
                                                                                          math.ceil(0.99 * len(lat)) - 1)]},
        "result": {"separator_vertices": sep, "max_split": float(o["split_cut"][:n_nodes].max().item()),
                   "cut_net": c["cut_net"], "lambda_minus_one": c["lambda_minus_one"], "tree_nodes": n_nodes},
        "roofline": roof,
        "lloyd_assign": {"bound": "hbm", "achieved": round(a_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": round(a_gbs / PEAK_HBM_GBS, 4), "launches_timed": assign["launches"],
                         "share_of_step": round(assign["total_ms"] * PROFILE_EVERY / (1e3 * dt), 4)},
        "cpu_baseline": cpu,
    }
    if not args.path_only:
        # the further rows of the method; a failure there is reported in the
        # line, which the step's measurement above does not depend on
        try:
            h = ctx.model(P.SYMMETRIC, g.m, g.n, rowptr, col)
            line.update(order_only_and_border(ctx, h, g, lp, o, args.steps))
            if not args.no_cpu_baseline:
                line["cpu_order_only"] = cpu_order_only(ctx, h, g, args.cpu_threads)
            line.update(bench_lu_pipeline(ctx, g, rowptr, col, lp, 2))
        except Exception as e:  # noqa: BLE001
            line["extras_error"] = f"{type(e).__name__}: {e}"
            print(f"bench: extra fields failed: {e}", file=sys.stderr, flush=True)
        if not args.no_zipf:
            try:
                line["zipf"] = bench_zipf(ctx, lp, 3)
            except Exception as e:  # noqa: BLE001
                line["zipf_error"] = f"{type(e).__name__}: {e}"
                print(f"bench: zipf field failed: {e}", file=sys.stderr, flush=True)
        if not args.no_batch:
            try:
                line["batch"] = bench_batch(args, ctx, field=True)
            except Exception as e:  # noqa: BLE001
                line["batch_error"] = f"{type(e).__name__}: {e}"
                print(f"bench: batch field failed: {e}", file=sys.stderr, flush=True)
        if not args.no_serve:
            try:
                line["serve"] = bench_serve(args, ctx, field=True)
            except Exception as e:  # noqa: BLE001
                line["serve_error"] = f"{type(e).__name__}: {e}"
                print(f"bench: serve field failed: {e}", file=sys.stderr, flush=True)
    print(json.dumps(line))


def order_only_and_border(ctx, h, g, lp, o, steps):
    """The O column (ordering from given coordinates: the layout of the same
    matrix, computed before the timed region), the recursive ordering of the
    border (b = 3 two-bit words) of the V+O result, the Schur-complement
    recursion of the O result and the Kernighan-Lin refinement of 2-means
    bisections of the leaf blocks, each timed over `steps` calls after one
    untimed call."""
    import torch
    x = ctx.layout(h, lp)
    ctx.order(h, x, P_PARTS, SEED, mode=1, order=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.order(h, x, P_PARTS, SEED, mode=1, order=1)
    torch.cuda.synchronize()
    dt_o = (time.perf_counter() - t0) / steps
    b = 3
    ctx.order_border(h, o, P_PARTS, b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.order_border(h, o, P_PARTS, b)
    torch.cuda.synchronize()
    dt_b = (time.perf_counter() - t0) / steps
    # Schur-complement recursion of the ordering from the same coordinates
    ox = ctx.order(h, x, P_PARTS, SEED, mode=1, order=1)
    ctx.order_schur(h, x, ox, P_PARTS, SCHUR_P3, SEED)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.order_schur(h, x, ox, P_PARTS, SCHUR_P3, SEED)
    torch.cuda.synchronize()
    dt_s = (time.perf_counter() - t0) / steps
    kl = bench_kl(ctx, h, x, o, steps)
    return {"kl": kl, "order_only": {"metric": "matrix nnz ordered/sec (recursive BBD from given coordinates)",
                           "value": g.nnz / dt_o, "unit": "nnz/s", "ms": 1e3 * dt_o},
            "border": {"b": b, "value": g.nnz / dt_b, "unit": "nnz/s", "ms": 1e3 * dt_b,
                       "what": "recursive ordering of the border of the V+O result (separator blocks sorted by "
                               "b two-bit words), one call per timing"},
            "schur": {"P3": SCHUR_P3, "value": g.nnz / dt_s, "unit": "nnz/s", "ms": 1e3 * dt_s,
                      "what": "Schur-complement recursion: every separator block of the ordering reordered by the "
                              "BBD ordering of its induced graph into P3 parts, all blocks in one batched pass"}}


def bench_zipf(ctx, lp, steps):
    """V+O of the rectangular Zipf matrix: 200,000 x 100,000, row degrees
    min(Zipf(2), 2000), column-net, 256 parts, SBD (net mode), from
    device-resident CSR; one untimed run, then `steps` timed runs, each split
    into its layout and its ordering."""
    import numpy as np
    import torch
    import paper_1105_4490_amd as P
    import vmo_gen
    g = vmo_gen.zipf_rect(200000, 100000, SEED)
    rowptr = torch.as_tensor(g.rowptr).cuda()
    col = torch.as_tensor(g.col).cuda()
    parts = 256

    def run():
        h = ctx.model(P.COLUMN_NET, g.m, g.n, rowptr, col)
        a = time.perf_counter()
        x = ctx.layout(h, lp)
        torch.cuda.synchronize()
        b = time.perf_counter()
        o = ctx.order(h, x, parts, SEED, mode=P.NET, order=P.SBD)
        c = ctx.cut(h, o["part"], parts)
        torch.cuda.synchronize()
        return b - a, time.perf_counter() - b, c

    run()
    lay, ordr = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        a, b, c = run()
        lay.append(a)
        ordr.append(b)
    dt = (time.perf_counter() - t0) / steps
    deg = np.diff(g.rowptr)
    return {"metric": "matrix nnz ordered/sec (V+O, recursive SBD)", "value": g.nnz / dt, "unit": "nnz/s",
            "ms": 1e3 * dt, "layout_ms": 1e3 * statistics.median(lay), "order_cut_ms": 1e3 * statistics.median(ordr),
            "steps": steps, "cut_net": c["cut_net"], "max_split": c["max_split"],
            "config": {"workload": f"rectangular Zipf {g.m} x {g.n} ({g.nnz} nnz), row degrees min(Zipf(2), 2000) "
                                   f"(largest {int(deg.max())}), column-net, {parts} parts, recursive SBD, "
                                   "layout + order from device-resident CSR", "seed": SEED}}


def bench_kl(ctx, h, x, o, steps, passes=4):
    """Kernighan-Lin refinement of 2-means bisections: every leaf block of
    the V+O result is split by one 2-means bisection of its layout points
    (untimed), and the 64 bisections are refined together (one workgroup
    each), `passes` passes, each timing from the same labels."""
    import torch
    part = o["part"].long()
    label = torch.full((h.k,), -1, dtype=torch.int32, device=part.device)
    sizes = []
    for p in range(P_PARTS):
        verts = torch.nonzero(part == p).flatten()
        if verts.numel() < 2:
            continue
        b = ctx.bisect(x[:, verts].contiguous(), SEED)
        label[verts] = (2 * p + b["side"].int()).int()
        sizes.append(int(verts.numel()))
    ctx.refine_kl(h, label, passes)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out, gain = ctx.refine_kl(h, label, passes)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    pins = h.pins.view(-1, 2).long()
    la, lb = label[pins[:, 0]], label[pins[:, 1]]
    same = (la >= 0) & (lb >= 0) & ((la >> 1) == (lb >> 1))
    cut0 = int((same & (la != lb)).sum().item())
    return {"ms": 1e3 * dt, "passes": passes, "bisections": len(sizes), "mean_vertices": sum(sizes) / max(len(sizes), 1),
            "cut_before": cut0, "cut_reduction": int(gain.sum().item()),
            "what": "Kernighan-Lin passes on the 2-means bisection of every leaf block of the V+O result, "
                    "all bisections in one launch"}


def bench_lu_pipeline(ctx, g, rowptr, col, lp, steps):
    """The ordering for LU of the same matrix with a strengthened diagonal:
    bipartite model, heavy edge matching on synthetic values with a dominant
    diagonal (|a_ii| about 6, off-diagonal about 1) augmented to a maximum
    matching, layout of the bipartite graph, BBD ordering that keeps matched
    pairs together, Schur-complement recursion with the matching, row and
    column permutations; timed as a whole over `steps` runs after one untimed
    run, with a per-phase split of one more run.  The pattern-only matching
    (ties broken by the scrambled index, so the augmentation has work to do)
    is timed on its own."""
    import numpy as np
    import torch
    import paper_1105_4490_amd as P
    import vmo_gen
    rows = np.repeat(np.arange(g.m), np.diff(g.rowptr))
    a = (np.where(rows == g.col, 6.0, -1.0) + vmo_gen.rng(SEED, 71).uniform(-0.1, 0.1, g.nnz)).astype(np.float32)
    da = torch.as_tensor(a).cuda()
    phases = {}

    def run(split=False):
        marks = [time.perf_counter()]

        def mark(name):
            if split:
                torch.cuda.synchronize()
                marks.append(time.perf_counter())
                phases[name] = 1e3 * (marks[-1] - marks[-2])
        hb = ctx.model(P.BIPARTITE, g.m, g.n, rowptr, col)
        mt = ctx.match(g.m, g.n, rowptr, col, da, seed=SEED)
        mark("model_match")
        x = ctx.layout(hb, lp)
        mark("layout")
        o = ctx.order_matched(hb, x, mt["mu"], P_PARTS, SEED)
        mark("order")
        s = ctx.order_schur(hb, x, o, P_PARTS, SCHUR_P3, SEED, mu=mt["mu"])
        rp, cp = ctx.matched_perms(g.m, s, mt["mu"])
        mark("schur_perms")
        return mt, o

    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        mt, o = run()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    run(split=True)
    n_nodes = int(o["n_nodes"].item())
    ctx.match(g.m, g.n, rowptr, col, None, seed=SEED)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        mp = ctx.match(g.m, g.n, rowptr, col, None, seed=SEED)
    torch.cuda.synchronize()
    dm = (time.perf_counter() - t0) / steps
    heavy = ctx.match(g.m, g.n, rowptr, col, None, seed=SEED, augment=False)
    return {"lu_ordering": {"value": g.nnz / dt, "unit": "nnz/s", "ms": 1e3 * dt, "steps": steps,
                            "phases_ms": {k: round(v, 3) for k, v in phases.items()},
                            "bipartite_vertices": g.m + g.n, "matching_size": mt["size"],
                            "separator_vertices": float(o["split_cut"][:n_nodes].sum().item()),
                            "what": "bipartite model + strengthened diagonal (heavy edge matching, augmented) + "
                                    "layout of the bipartite graph + BBD ordering keeping matched pairs together "
                                    f"+ Schur-complement recursion (P3 = {SCHUR_P3}) + row/column permutations"},
            "match_pattern_only": {"ms": 1e3 * dm, "size": mp["size"], "heavy_size": heavy["size"]}}


def _pct(v, q):
    v = sorted(v)
    return v[min(len(v) - 1, max(0, math.ceil(q * len(v)) - 1))]


def bench_batch(args, ctx, field=False):
    """Recursive ordering of many banded matrices: batched against plain.
    field: return the result as a dict (a field of the default line) instead
    of printing a line of its own."""
    import torch
    import paper_1105_4490_amd as P
    import vmo_gen
    t = time.perf_counter()
    mats = vmo_gen.batch_banded(args.jobs, seed=SEED)
    gen_s = time.perf_counter() - t
    print(f"bench: generated {len(mats)} matrices in {gen_s:.1f} s", file=sys.stderr, flush=True)
    t = time.perf_counter()
    hs = [ctx.model(P.ROW_NET, g.m, g.n, torch.as_tensor(g.rowptr).cuda(), torch.as_tensor(g.col).cuda())
          for g, _ in mats]
    torch.cuda.synchronize()
    # coordinates (untimed): layouts run on several streams at once, one context each
    import concurrent.futures
    xs = [None] * len(mats)
    nthr = max(1, args.layout_threads)

    def lay(w):
        c = P.Context(0)
        st = torch.cuda.Stream()
        with torch.cuda.stream(st):
            for i in range(w, len(mats), nthr):
                xs[i] = c.layout(hs[i], P.layout_params(seed=SEED + i))
                if (i + 1) % 64 == 0:
                    print(f"bench: laid out {i + 1} matrices", file=sys.stderr, flush=True)
        st.synchronize()
        c.close()

    with concurrent.futures.ThreadPoolExecutor(nthr) as ex:
        list(ex.map(lay, range(nthr)))
    torch.cuda.synchronize()
    jobs = [{"h": hs[i], "x": xs[i], "P": parts, "seed": SEED, "mode": P.NET, "order": P.SBD, "job_index": i}
            for i, (g, parts) in enumerate(mats)]
    lay_s = time.perf_counter() - t
    nnz = sum(g.nnz for g, _ in mats)
    rows = sum(g.m for g, _ in mats)

    def run(plain, steps):
        # the plain form is not timed per launch (its many small launches
        # would each carry an event pair)
        ctx.profile(not plain, every=4)
        ctx.profile_reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            outs = ctx.order_batch(jobs, plain=plain)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        a = ctx.profile_read("assign")
        ctx.profile(False)
        return outs, dt, a

    for _ in range(args.warmup):
        run(False, 1)
    outs, dt_b, a_b = run(False, args.steps)
    print(f"bench: batched {1e3 * dt_b:.1f} ms", file=sys.stderr, flush=True)
    if args.no_plain:
        outs_p, dt_p = outs, float("nan")
    else:
        outs_p, dt_p, _ = run(True, 1)
        print(f"bench: plain {1e3 * dt_p:.1f} ms", file=sys.stderr, flush=True)
    same = all(torch.equal(a["vperm"], b["vperm"]) and torch.equal(a["part"], b["part"])
               for a, b in zip(outs, outs_p))
    a_gbs = a_b["work"] / (a_b["total_ms"] * 1e-3) / 1e9 if a_b["total_ms"] > 0 else 0.0
    line = {
        "metric": "matrix nnz ordered/sec (batched recursive SBD, coordinates given)",
        "value": nnz / dt_b, "unit": "nnz/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * dt_b, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32 grid / f64 plane", "data": "synthetic",
        "config": {"workload": f"{len(mats)} banded matrices ({rows} rows, {nnz} nnz), rows log-uniform "
                               "1e3-5e4, half bandwidth 5-40, 0.1% off-band, 8-32 parts, row-net, recursive SBD; "
                               "coordinates from the layout, computed before the timed region",
                   "jobs": len(mats), "seed": SEED},
        "plain": {"value": nnz / dt_p, "unit": "nnz/s", "ms": 1e3 * dt_p,
                  "form": "one launch sequence per subproblem"},
        "batched_over_plain": dt_p / dt_b, "identical_results": same,
        "lloyd_assign": {"bound": "hbm", "achieved": round(a_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": round(a_gbs / PEAK_HBM_GBS, 4), "launches_timed": a_b["launches"],
                         "timed_every": 4,
                         "share_of_step": round(4 * a_b["total_ms"] / (1e3 * dt_b * args.steps), 4)},
        "untimed": {"generate_s": round(gen_s, 1), "layout_s": round(lay_s, 1)},
    }
    if field:
        return {k: line[k] for k in ("metric", "value", "unit", "ms_per_step", "config", "plain",
                                     "batched_over_plain", "identical_results", "lloyd_assign", "untimed")}
    print(json.dumps(line))


def _serve_matrix(spec):
    import vmo_gen
    if spec["kind"] == "grid2d":
        return vmo_gen.grid2d(spec["N"]), 0
    if spec["kind"] == "grid3d":
        return vmo_gen.grid3d(spec["N"], seed=spec["seed"]), 1
    return vmo_gen.zipf_rect(spec["m"], spec["n"], spec["seed"]), 2


def bench_serve(args, ctx, field=False):
    """A Poisson stream of whole-path ordering jobs through the server (the
    stream's length scaled down from 3,000 requests to --requests).  field:
    return the result as a dict instead of printing a line."""
    import numpy as np
    import torch
    import paper_1105_4490_amd as P
    import vmo_gen
    # model, parts and order of each shape: 2-D grid row-net 16 SBD; 3-D grid
    # symmetric 64 BBD with separators; rectangular column-net 256 SBD
    shapes = {0: (P.ROW_NET, 16, P.NET, P.SBD), 1: (P.SYMMETRIC, 64, P.GRAPH, P.BBD), 2: (P.COLUMN_NET, 256, P.NET, P.SBD)}
    reqs = vmo_gen.serve_stream(args.requests, seed=SEED, rate=args.rate, nnz_max=args.nnz_max)
    jobs = []
    t = time.perf_counter()
    for i, spec in enumerate(reqs):
        g, kind = _serve_matrix(spec)
        model, parts, mode, order = shapes[kind]
        h = ctx.model(model, g.m, g.n, torch.as_tensor(g.rowptr).cuda(), torch.as_tensor(g.col).cuda())
        jobs.append(({"h": h, "x": None, "P": parts, "seed": SEED, "mode": mode, "order": order, "job_index": i},
                     spec["arrival"], g.nnz))
    torch.cuda.synchronize()
    prep_s = time.perf_counter() - t
    print(f"bench: prepared {len(jobs)} requests ({sum(j[2] for j in jobs)} nnz) in {prep_s:.1f} s",
          file=sys.stderr, flush=True)
    lp = P.layout_params(seed=SEED)

    def stream(arrivals):
        """Submit the jobs at the given arrival times; (latencies ms, span s, stats)."""
        srv = P.Server(budget_bytes=args.serve_budget_gib << 30, max_jobs=256, layout_threads=args.serve_threads)
        tickets = []
        t0 = time.perf_counter()
        for (jb, _, nz), at in zip(jobs, arrivals):
            now = time.perf_counter() - t0
            if at > now:
                time.sleep(at - now)
            tickets.append(srv.submit(jb, lp))
        lat = []
        done_at = 0.0
        for i, tk in enumerate(tickets):
            o, ms = srv.wait(tk)
            lat.append(ms)
            done_at = max(done_at, time.perf_counter() - t0)
            if (i + 1) % 10 == 0:
                print(f"bench: {i + 1} requests done", file=sys.stderr, flush=True)
        st = srv.stats()
        srv.close()
        return lat, done_at, st

    total = sum(j[2] for j in jobs)
    lat, span, st = stream([j[1] for j in jobs])
    capacity = total / span
    line = {
        "metric": "matrix nnz ordered/sec (served, full recursive SBD/BBD) + p50/p99 latency",
        "value": capacity, "unit": "nnz/s", "n_gpus": 1, "steps": len(jobs), "warmup": 0,
        "ms_per_step": 1e3 * span / len(jobs), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"Poisson stream of {len(jobs)} requests at {args.rate}/s, nnz log-uniform "
                               f"[1e3, {args.nnz_max:.0e}], uniform over 2-D grid (row-net, 16, SBD), 3-D grid "
                               "(symmetric, 64, BBD), rectangular Zipf (column-net, 256, SBD); layout + order",
                   "seed": SEED},
        "latency_ms": {"p50": _pct(lat, 0.5), "p99": _pct(lat, 0.99), "max": max(lat)},
        "offered_nnz_per_s": total / max(jobs[-1][1], 1e-9),
        "busy_ms": st["busy_ms"], "ticks": st["ticks"], "max_tick_jobs": st["max_tick_jobs"],
        "mean_tick_jobs": st["tick_jobs"] / max(st["ticks"], 1), "layout_bytes_peak": st["layout_bytes_peak"],
    }
    # the same jobs one at a time through the plain call, back to back: the
    # rate serving is measured against
    torch.cuda.synchronize()
    t = time.perf_counter()
    for jb, _, _ in jobs:
        ctx.order(jb["h"], None, jb["P"], SEED, mode=jb["mode"], order=jb["order"], lp=lp)
    torch.cuda.synchronize()
    seq_s = time.perf_counter() - t
    line["sequential"] = {"nnz_per_s": total / seq_s, "s": seq_s,
                          "what": "the same jobs one at a time through the plain call (layout + order)"}
    line["served_over_sequential"] = capacity * seq_s / total
    if not args.no_stable and capacity < line["offered_nnz_per_s"]:
        # the same jobs again as a Poisson stream at half the measured capacity
        rate = 0.5 * capacity / (total / len(jobs))
        g = vmo_gen.rng(SEED, 61)
        arr = list(np.cumsum(g.exponential(1.0 / rate, size=len(jobs))))
        print(f"bench: stable run at {rate:.2f} requests/s", file=sys.stderr, flush=True)
        lat2, span2, _ = stream(arr)
        line["stable"] = {"rate_per_s": rate, "nnz_per_s": total / span2,
                          "latency_ms": {"p50": _pct(lat2, 0.5), "p99": _pct(lat2, 0.99), "max": max(lat2)}}
    if field:
        line["scaled"] = f"{len(jobs)} requests of the 3,000-request stream"
        return {k: line[k] for k in ("metric", "value", "unit", "config", "latency_ms", "offered_nnz_per_s",
                                     "busy_ms", "ticks", "max_tick_jobs", "mean_tick_jobs", "layout_bytes_peak",
                                     "sequential", "served_over_sequential", "scaled")
                + (("stable",) if "stable" in line else ())}
    print(json.dumps(line))


def copy_calibration():
    """A device copy of known size (256 MiB read and 256 MiB written per
    dispatch, three dispatches): what FETCH_SIZE and WRITE_SIZE read for it
    scales the counts taken on the walk."""
    import torch
    a = torch.ones(1 << 26, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"mode": "copy", "bytes_per_copy": a.numel() * 4, "copies": 3}))


def host_cpu():
    """Model name of the host CPU and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail, os.cpu_count() or avail


def _oracle_vo(side):
    import oracle
    import vmo_gen
    g = vmo_gen.grid3d(side, seed=SEED)
    t = time.perf_counter()
    h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    x = oracle.layout(h, oracle.layout_params(seed=SEED))
    o = oracle.order(h, x, P_PARTS, SEED, mode=oracle.GRAPH_MODE, ord=oracle.BBD)
    oracle.cut(h, o.part, P_PARTS)
    return g, time.perf_counter() - t


def cpu_baseline(side, side1, threads):
    """The oracle on the full V+O path of smaller instances of the same
    generator (the 64^3 instance takes it minutes): on all the host cores it
    may use (OpenMP over the independent per-vertex loops; the result does not
    depend on the thread count) for the side^3 instance, and on one thread for
    the side1^3 instance."""
    import oracle
    oracle.build()
    model, avail, nproc = host_cpu()
    nthr = max(1, min(threads, avail))
    oracle.set_threads(nthr)
    g, dt = _oracle_vo(side)
    oracle.set_threads(1)
    g1, dt1 = _oracle_vo(side1)
    oracle.set_threads(nthr)
    return {"value": g.nnz / dt, "unit": "nnz/s", "cores": nthr, "kind": "oracle",
            "sample": f"full V+O path (model, layout, {P_PARTS}-part BBD, cut) of the {side}^3 instance of the "
                      f"same generator ({g.m} rows, {g.nnz} nnz) in {dt:.1f} s on {nthr} threads",
            "single_thread": {"value": g1.nnz / dt1, "cores": 1, "seconds": round(dt1, 2),
                              "sample": f"the {side1}^3 instance ({g1.m} rows, {g1.nnz} nnz)"},
            "cpu_model": model, "nproc": nproc, "cores_available": avail}


def synthetic_grid_coords(n, seed):
    """Coordinates of the permuted n^3 grid's vertices: vertex v sits at the
    grid position of the original vertex the generator's permutation sent to
    v, plus a small seeded jitter."""
    import numpy as np
    import vmo_gen
    perm = vmo_gen.rng(seed, 2).permutation(n ** 3)   # the permutation vmo_gen.grid3d applies
    inv = np.empty_like(perm)
    inv[perm] = np.arange(n ** 3)
    x = np.zeros((4, n ** 3), np.float32)
    x[0], x[1], x[2] = inv % n, (inv // n) % n, inv // (n * n)
    x += vmo_gen.rng(seed, 9).standard_normal(x.shape).astype(np.float32) * 0.1
    return x


def cpu_order_only(ctx, h, g, threads):
    """The O column at full size: the oracle's recursive BBD of the 64^3
    matrix from given coordinates (its grid positions with a seeded jitter),
    timed on the host, beside the GPU ordering of the same input."""
    import torch
    import oracle
    x = synthetic_grid_coords(round(g.m ** (1 / 3)), SEED)
    hh = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    model, avail, nproc = host_cpu()
    t = time.perf_counter()
    oracle.order(hh, x, P_PARTS, SEED, mode=oracle.GRAPH_MODE, ord=oracle.BBD)
    dt = time.perf_counter() - t
    dx = torch.as_tensor(x).cuda().contiguous()
    ctx.order(h, dx, P_PARTS, SEED, mode=1, order=1)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(5):
        ctx.order(h, dx, P_PARTS, SEED, mode=1, order=1)
    torch.cuda.synchronize()
    dg = (time.perf_counter() - t) / 5
    return {"value": g.nnz / dt, "unit": "nnz/s", "cores": 1, "kind": "oracle",
            "sample": f"O column (recursive {P_PARTS}-part BBD from given coordinates) of the full {g.m}-row instance, "
                      f"{dt:.2f} s (the ordering's loops are sequential in the oracle)",
            "gpu_same_input": {"value": g.nnz / dg, "unit": "nnz/s", "ms": round(1e3 * dg, 3)},
            "cpu_model": model, "nproc": nproc}


if __name__ == "__main__":
    main()
