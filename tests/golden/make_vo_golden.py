"""Writes vo_<name>.json: the oracle's full V+O result (hypergraph model,
multilevel layout, recursive ordering, cut) for the workloads the GPU path is
measured and tested on at full size, as SHA-256 digests of its arrays plus its
cut metrics and the layout's total walk interactions.  Calls only oracle/ and
the seeded input generators (vmo_gen).  The GPU tests compare their own
results against these digests element for element (a digest match is
equality of every element).

Run: python tests/golden/make_vo_golden.py [name ...]   (default: all)
   grid3d64_bbd64   64^3 7-point pattern, one random symmetric permutation
                    (seed 1), symmetric model, layout seed 1, 64 parts, BBD,
                    graph mode, order seed 1, t_max 32 (the benchmark input)
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import oracle  # noqa: E402
import vmo_gen  # noqa: E402


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def grid3d64_bbd64():
    g = vmo_gen.grid3d(64, seed=1)
    h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    oracle.interactions_reset()
    x = oracle.layout(h, oracle.layout_params(seed=1))
    nint = oracle.interactions()
    o = oracle.order(h, x, 64, 1, mode=oracle.GRAPH_MODE, ord=oracle.BBD, t_max=32)
    c = oracle.cut(h, o.part, 64)
    return {
        "workload": "3-D 7-point pattern 64^3, rows/cols permuted by seed 1, symmetric model, layout seed 1, "
                    "64 parts, BBD with separators (graph mode), order seed 1, t_max 32",
        "k": h.k, "l": h.l, "nnz": int(g.nnz),
        "x_sha256": digest(x.astype(np.float32)),
        "vperm_sha256": digest(o.vperm.astype(np.int32)),
        "part_sha256": digest(o.part.astype(np.int32)),
        "node_heap_sha256": digest(o.node_heap[:o.n_nodes].astype(np.int32)),
        "node_vptr_sha256": digest(o.node_vptr[:o.n_nodes + 1].astype(np.int32)),
        "split_cut_sha256": digest(o.split_cut[:o.n_nodes].astype(np.float64)),
        "n_nodes": int(o.n_nodes),
        "separator_vertices": int((o.part >= 64).sum()),
        "max_split": float(o.split_cut[:o.n_nodes].max()),
        "cut_net": float(c["cut_net"]), "lambda_minus_one": float(c["lambda_minus_one"]),
        "nets_cut": int(c["nets_cut"]),
        "layout_interactions": int(nint),
    }


CASES = {"grid3d64_bbd64": grid3d64_bbd64}


def main(names):
    for name in names or list(CASES):
        t = time.time()
        out = CASES[name]()
        out["oracle_seconds"] = round(time.time() - t, 1)
        with open(os.path.join(HERE, "vo_%s.json" % name), "w") as f:
            json.dump(out, f, indent=1)
            f.write("\n")
        print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main(sys.argv[1:])
