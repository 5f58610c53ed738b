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
FLOPS_PER_INTERACTION = 23   # 4 sub, 4 mul + 3 add (r^2), 2 mul (2 W w), 1 mul (r^4), 1 div, 4 mul + 4 add
PEAK_FP32_VALU_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--side", type=int, default=N_SIDE, help="grid side of the workload (64 = the 64^3 case)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-side", type=int, default=28, help="grid side of the oracle's timed sample")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU design is described, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1105_4490_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_1105_4490_amd import build as b
        b.build()
    import vmo_gen

    torch.cuda.set_device(0)
    ctx = P.Context(0)
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
    ctx.profile(True)
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

    flops = FLOPS_PER_INTERACTION * walk["work"]
    w_tflops = flops / (walk["total_ms"] * 1e-3) / 1e12 if walk["total_ms"] > 0 else 0.0
    roof = {"bound": "alu", "kernel": "k_walk", "achieved": round(w_tflops, 3), "peak": PEAK_FP32_VALU_TFLOPS,
            "unit": "TFLOP/s", "frac": round(w_tflops / PEAK_FP32_VALU_TFLOPS, 4), "traffic": None,
            "launches": walk["launches"], "avg_launch_ms": round(walk["total_ms"] / max(walk["launches"], 1), 4),
            "share_of_step": round(walk["total_ms"] / (1e3 * dt), 4),
            "interactions_per_step": walk["work"] / args.steps}
    a_gbs = assign["work"] / (assign["total_ms"] * 1e-3) / 1e9 if assign["total_ms"] > 0 else 0.0

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.cpu_side)

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
                         "frac": round(a_gbs / PEAK_HBM_GBS, 4), "launches": assign["launches"],
                         "share_of_step": round(assign["total_ms"] / (1e3 * dt), 4)},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


def cpu_baseline(side):
    """The oracle, single-threaded, on the full path of a smaller instance of
    the same generator (the 64^3 instance takes it many minutes)."""
    import oracle
    import vmo_gen
    oracle.build()
    g = vmo_gen.grid3d(side, seed=SEED)
    t = time.perf_counter()
    h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    x = oracle.layout(h, oracle.layout_params(seed=SEED))
    o = oracle.order(h, x, P_PARTS, SEED, mode=oracle.GRAPH_MODE, ord=oracle.BBD)
    oracle.cut(h, o.part, P_PARTS)
    dt = time.perf_counter() - t
    return {"value": g.nnz / dt, "unit": "nnz/s", "cores": 1, "kind": "oracle",
            "sample": f"full V+O path (model, layout, {P_PARTS}-part BBD, cut) of the {side}^3 instance of the "
                      f"same generator ({g.m} rows, {g.nnz} nnz) in {dt:.1f} s"}


if __name__ == "__main__":
    main()
