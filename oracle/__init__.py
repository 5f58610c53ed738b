"""CPU oracle for the geometric matrix ordering method (arXiv 1105.4490).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package; the product path (the
HIP library and its binding) never does.  It shares no code with the product.

The hypergraph models of the paper's Table 1 are written here in numpy; the
rest (components, cut, quantized 2-means, recursive ordering, coarsening,
tree, gradient, multilevel layout) is plain sequential C in
``vmo_oracle.c``, compiled with ``-O2 -ffp-contract=off`` and called through
ctypes.  Each function cites the passage of the paper it follows.

Parity pins: every function here is checked by ``tests/test_oracle_*.py``
against values the paper prints, closed forms, brute force or independent
library routines; see the test files for the pin of each function.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vmo_oracle.c")
_LIB = os.path.join(_HERE, "_vmo_oracle.so")

ROW_NET, COLUMN_NET, SYMMETRIC = 0, 1, 2
NET_MODE, GRAPH_MODE = 0, 1
SBD, BBD = 0, 1


def build(force: bool = False) -> str:
    """Compile the C oracle (gcc, -O2, no FP contraction, OpenMP over
    independent per-vertex loops only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = C.CDLL(_LIB)
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


@dataclass
class Hypergraph:
    """Weighted hypergraph (Definition of a hypergraph, Sec. 1.1): nets as CSR
    (ptr int64 [l+1], pins int32 ascending within a net), w [k] and c [l]
    float32 or None (all ones)."""
    k: int
    l: int
    ptr: np.ndarray
    pins: np.ndarray
    w: np.ndarray | None = None
    c: np.ndarray | None = None

    def nets(self):
        for e in range(self.l):
            yield self.pins[self.ptr[e]:self.ptr[e + 1]]


def hypergraph(k, nets, w=None, c=None) -> Hypergraph:
    """Hypergraph from a Python list of nets (each an iterable of vertex ids)."""
    nets = [sorted(int(v) for v in e) for e in nets]
    ptr = np.zeros(len(nets) + 1, dtype=np.int64)
    ptr[1:] = np.cumsum([len(e) for e in nets])
    pins = np.array([v for e in nets for v in e], dtype=np.int32)
    return Hypergraph(int(k), len(nets), ptr, pins,
                      None if w is None else np.asarray(w, dtype=np.float32),
                      None if c is None else np.asarray(c, dtype=np.float32))


# ---------------------------------------------------------------- Table 1 ----

def rownet(m, n, rowptr, col) -> Hypergraph:
    """Row-net model (Table 1): vertices = columns, net i = columns of row i."""
    return Hypergraph(int(n), int(m), np.asarray(rowptr, np.int64).copy(), np.asarray(col, np.int32).copy())


def transpose(m, n, rowptr, col):
    """CSR of A^T (columns ascending within each row of A^T), by stable sort."""
    rowptr = np.asarray(rowptr, np.int64)
    col = np.asarray(col, np.int64)
    rows = np.repeat(np.arange(m, dtype=np.int64), np.diff(rowptr))
    order = np.lexsort((rows, col))
    tptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(col, minlength=n), out=tptr[1:])
    return tptr, rows[order].astype(np.int32)


def colnet(m, n, rowptr, col) -> Hypergraph:
    """Column-net model (Table 1): vertices = rows, net j = rows with a_ij != 0."""
    tptr, tcol = transpose(m, n, rowptr, col)
    return Hypergraph(int(m), int(n), tptr, tcol)


def symmetric(m, n, rowptr, col) -> Hypergraph:
    """Symmetric model (Table 1) of a square pattern: nets are the distinct
    pairs {i, j}, i < j, with a_ij != 0 or a_ji != 0, ordered by (i, j);
    diagonal entries are dropped (they would be one-vertex nets)."""
    assert m == n
    rowptr = np.asarray(rowptr, np.int64)
    rows = np.repeat(np.arange(m, dtype=np.int64), np.diff(rowptr))
    cols = np.asarray(col, np.int64)
    a = np.minimum(rows, cols)
    b = np.maximum(rows, cols)
    keep = a != b
    key = np.unique(a[keep] * n + b[keep])
    l = key.shape[0]
    pins = np.empty(2 * l, dtype=np.int32)
    pins[0::2] = key // n
    pins[1::2] = key % n
    return Hypergraph(int(n), int(l), np.arange(0, 2 * l + 1, 2, dtype=np.int64), pins)


def model(kind, m, n, rowptr, col) -> Hypergraph:
    return (rownet, colnet, symmetric)[kind](m, n, rowptr, col)


# ---------------------------------------------------------------- C parts ----

def dual(h: Hypergraph) -> Hypergraph:
    """Dual hypergraph (Definition of the dual, Sec. 1.1); weights and costs swap."""
    dptr = np.zeros(h.k + 1, dtype=np.int64)
    dp = np.zeros(max(int(h.ptr[-1]), 1), dtype=np.int32)
    rc = lib().o_dual(C.c_int32(h.k), C.c_int32(h.l), _p(h.ptr), _p(h.pins), _p(dptr), _p(dp))
    assert rc == 0
    return Hypergraph(h.l, h.k, dptr, dp[:int(h.ptr[-1])], h.c, h.w)


def components(h: Hypergraph) -> np.ndarray:
    """label(v) = smallest vertex id in v's connected component (Algorithm 1)."""
    lab = np.zeros(h.k, dtype=np.int32)
    rc = lib().o_components(C.c_int32(h.k), C.c_int32(h.l), _p(h.ptr), _p(h.pins), _p(lab))
    assert rc == 0
    return lab


def cut(h: Hypergraph, part, nparts: int):
    """(lambda-1) metric, cut-net metric, number of cut nets, part weights."""
    part = np.ascontiguousarray(part, dtype=np.int32)
    out = np.zeros(3, dtype=np.float64)
    pw = np.zeros(max(nparts, 1), dtype=np.float64)
    rc = lib().o_cut(C.c_int32(h.k), C.c_int32(h.l), _p(h.ptr), _p(h.pins), _p(h.c), _p(part), _p(h.w),
                     C.c_int32(nparts), _p(out), _p(pw))
    assert rc == 0
    return {"lambda_minus_one": out[0], "cut_net": out[1], "nets_cut": int(out[2]), "part_weight": pw[:nparts]}


def split_cuts(h: Hypergraph, part, P: int):
    """Per-split cut of a recursive bisection into P parts (o_split_cuts):
    (split [4P] by heap id, graph) -- the cost of the nets cut at each node
    (the deepest node whose part range holds all the net's parts), or, when
    separator ids P + h occur (graph mode), the size of each S_h."""
    part = np.ascontiguousarray(part, dtype=np.int32)
    sp = np.zeros(4 * P, dtype=np.float64)
    g = lib().o_split_cuts(C.c_int32(h.k), C.c_int32(h.l), _p(h.ptr), _p(h.pins), _p(h.c), _p(part), C.c_int32(P),
                           _p(sp))
    return sp, bool(g)


def quantize(x):
    x = np.ascontiguousarray(x, dtype=np.float32)
    k = x.shape[1]
    q = np.zeros((4, k), dtype=np.uint32)
    lo = np.zeros(4, dtype=np.float32)
    s = C.c_double(0)
    rc = lib().o_quantize(C.c_int32(k), _p(x), _p(q), _p(lo), C.byref(s))
    assert rc == 0
    return q, lo, s.value


def set_threads(n: int):
    """Host threads for the oracle's independent per-vertex loops (results do
    not depend on it)."""
    lib().o_set_threads(C.c_int(int(n)))


def max_threads() -> int:
    return int(lib().o_max_threads())


def splitmix64(seed, n):
    """n-th output of the SplitMix64 stream seeded with `seed`."""
    f = lib().o_splitmix64
    f.restype = C.c_uint64
    return int(f(C.c_uint64(seed), C.c_uint64(n)))


def rng(seed, a, b, c):
    f = lib().o_rng
    f.restype = C.c_uint64
    return int(f(C.c_uint64(seed), C.c_uint64(a), C.c_uint64(b), C.c_uint64(c)))


@dataclass
class BisectResult:
    split: bool
    side: np.ndarray
    centres: np.ndarray
    iters: int
    plane: np.ndarray


def bisect(x, seed: int, t_max: int = 32) -> BisectResult:
    """One 2-means split (Algorithm 4, m = 2; plane of Algorithm 7)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    k = x.shape[1]
    side = np.zeros(k, dtype=np.uint8)
    cen = np.zeros(8, dtype=np.float32)
    it = C.c_int32(0)
    plane = np.zeros(5, dtype=np.float64)
    rc = lib().o_bisect(C.c_int32(k), _p(x), C.c_uint64(seed), C.c_int32(t_max), _p(side), _p(cen),
                        C.byref(it), _p(plane))
    assert rc >= 0
    return BisectResult(rc == 0, side, cen.reshape(2, 4), it.value, plane)


@dataclass
class OrderResult:
    vperm: np.ndarray
    nperm: np.ndarray | None
    part: np.ndarray
    node_heap: np.ndarray
    node_vptr: np.ndarray
    node_nptr: np.ndarray | None
    split_cut: np.ndarray
    n_nodes: int


def order(h: Hypergraph, x, P: int, seed: int, mode: int = NET_MODE, ord: int = SBD, t_max: int = 32,
          job: int = 0, mu=None) -> OrderResult:
    """Recursive SBD/BBD ordering (Algorithm 7 applied recursively, Sec. 4.2);
    mu (graph mode): a strengthened diagonal, mu[v] = v's partner or -1
    (o_order_mu)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    mu = None if mu is None else np.ascontiguousarray(mu, dtype=np.int32)
    k, l = h.k, h.l
    vperm = np.zeros(k, dtype=np.int32)
    part = np.zeros(k, dtype=np.int32)
    nperm = np.zeros(max(l, 1), dtype=np.int32) if mode == NET_MODE else None
    heap = np.zeros(4 * P, dtype=np.int32)
    vptr = np.zeros(4 * P + 1, dtype=np.int32)
    nptr = np.zeros(4 * P + 2, dtype=np.int32) if mode == NET_MODE else None
    sc = np.zeros(4 * P, dtype=np.float64)
    nn = C.c_int32(0)
    rc = lib().o_order_mu(C.c_int32(k), C.c_int32(l), _p(h.ptr), _p(h.pins), _p(h.c), C.c_int(mode),
                          C.c_int(ord), _p(x), _p(mu), C.c_int32(P), C.c_uint64(seed), C.c_uint64(job),
                          C.c_int32(t_max), _p(vperm), _p(nperm), _p(part), _p(heap), _p(vptr), _p(nptr), _p(sc),
                          C.byref(nn))
    if rc != 0:
        raise ValueError("oracle order rejected its input")
    return OrderResult(vperm, None if nperm is None else nperm[:l], part, heap, vptr, nptr, sc, nn.value)


def border(h: Hypergraph, vperm, part, node_heap, node_vptr, n_nodes: int, P: int, b: int):
    """Recursive ordering of the border (Sec. 4.2, cut rows and columns into
    recursive BBD form): vperm of a graph-mode ordering with every separator
    block sorted, stably, by b two-bit words (o_border)."""
    out = np.zeros(h.k, dtype=np.int32)
    arr = [np.ascontiguousarray(a, dtype=np.int32) for a in (vperm, part, node_heap, node_vptr)]
    rc = lib().o_border(C.c_int32(h.k), C.c_int32(h.l), _p(h.ptr), _p(h.pins), _p(arr[0]), _p(arr[1]), _p(arr[2]),
                        _p(arr[3]), C.c_int32(n_nodes), C.c_int32(P), C.c_int32(b), _p(out))
    if rc != 0:
        raise ValueError("oracle border rejected its input")
    return out


def schur(h: Hypergraph, x, vperm, part, node_heap, node_vptr, n_nodes: int, P: int, P3: int, seed: int,
          t_max: int = 32, mu=None):
    """Schur-complement recursion (Sec. 4.2, Algorithm 7 applied to G3 = (V3,
    E'3)): vperm of a graph-mode ordering with every separator block of at
    least two vertices reordered by the recursive BBD ordering (P3 parts,
    draws keyed by the separator's heap id) of its own graph (o_schur)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.zeros(h.k, dtype=np.int32)
    arr = [np.ascontiguousarray(a, dtype=np.int32) for a in (vperm, part, node_heap, node_vptr)]
    mu = None if mu is None else np.ascontiguousarray(mu, dtype=np.int32)
    rc = lib().o_schur(C.c_int32(h.k), C.c_int32(h.l), _p(h.ptr), _p(h.pins), _p(x), _p(mu), _p(arr[0]), _p(arr[1]),
                       _p(arr[2]), _p(arr[3]), C.c_int32(n_nodes), C.c_int32(P), C.c_int32(P3), C.c_uint64(seed),
                       C.c_int32(t_max), _p(out))
    if rc != 0:
        raise ValueError("oracle schur rejected its input")
    return out


# ------------------------------------------------- strengthened diagonal ----

def bipartite(m, n, rowptr, col) -> Hypergraph:
    """Bipartite model (Table 1): vertices r_0..r_{m-1} (ids 0..m-1) and
    c_0..c_{n-1} (ids m..m+n-1); one edge {r_i, c_j} per nonzero, in CSR
    order."""
    rowptr = np.asarray(rowptr, np.int64)
    col = np.asarray(col, np.int64)
    nnz = int(rowptr[-1])
    rows = np.repeat(np.arange(m, dtype=np.int64), np.diff(rowptr))
    pins = np.empty(2 * nnz, np.int32)
    pins[0::2] = rows
    pins[1::2] = m + col
    return Hypergraph(int(m) + int(n), nnz, np.arange(0, 2 * nnz + 1, 2, dtype=np.int64), pins)


def match_key(a, e: int, seed: int) -> int:
    """Priority of nonzero e in the heavy edge matching (o_match_key)."""
    a = None if a is None else np.ascontiguousarray(a, dtype=np.float32)
    lib().o_match_key.restype = C.c_uint64
    return int(lib().o_match_key(_p(a), C.c_int64(e), C.c_uint32(seed)))


def match_heavy(m, n, rowptr, col, a=None, seed: int = 0):
    """Heavy edge matching (o_match_heavy): (mrow, mcol, size)."""
    rowptr = np.ascontiguousarray(rowptr, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    a = None if a is None else np.ascontiguousarray(a, dtype=np.float32)
    mrow = np.zeros(max(m, 1), np.int32)
    mcol = np.zeros(max(n, 1), np.int32)
    lib().o_match_heavy.restype = C.c_int64
    size = lib().o_match_heavy(C.c_int32(m), C.c_int32(n), _p(rowptr), _p(col), _p(a), C.c_uint32(seed), _p(mrow),
                               _p(mcol))
    if size < 0:
        raise ValueError("oracle match rejected its input")
    return mrow[:m], mcol[:n], int(size)


def match_augment(m, n, rowptr, col, mrow, mcol):
    """Hopcroft-Karp augmentation (o_match_augment) of copies of mrow/mcol."""
    rowptr = np.ascontiguousarray(rowptr, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    mrow = np.array(mrow, np.int32, copy=True)
    mcol = np.array(mcol, np.int32, copy=True)
    lib().o_match_augment.restype = C.c_int64
    size = lib().o_match_augment(C.c_int32(m), C.c_int32(n), _p(rowptr), _p(col), _p(mrow), _p(mcol))
    return mrow, mcol, int(size)


def match(m, n, rowptr, col, a=None, seed: int = 0, augment: bool = True):
    """Strengthened diagonal: heavy edge matching, then (augment) Hopcroft-Karp."""
    mrow, mcol, size = match_heavy(m, n, rowptr, col, a, seed)
    if augment:
        mrow, mcol, size = match_augment(m, n, rowptr, col, mrow, mcol)
    return mrow, mcol, size


def mu_of(m, n, mrow, mcol):
    """mu on the bipartite graph's vertices: partner id or -1."""
    mu = np.full(m + n, -1, np.int32)
    mr = np.asarray(mrow)
    mc = np.asarray(mcol)
    mu[:m] = np.where(mr >= 0, mr + m, -1)
    mu[m:] = np.where(mc >= 0, mc, -1)
    return mu


def matched_perms(m, vperm, mu):
    """Row and column permutations with the matching on the diagonal."""
    vperm = np.ascontiguousarray(vperm, np.int32)
    mu = np.ascontiguousarray(mu, np.int32)
    rp = np.zeros(max(m, 1), np.int32)
    cp = np.zeros(max(m, 1), np.int32)
    if lib().o_matched_perms(C.c_int32(m), _p(vperm), _p(mu), _p(rp), _p(cp)) != 0:
        raise ValueError("oracle matched_perms: a row has no partner column")
    return rp[:m], cp[:m]


def finegrain(m, n, rowptr, col, x):
    """Nonzero coordinates [4][nnz] from bipartite coordinates [4][m+n]."""
    rowptr = np.ascontiguousarray(rowptr, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    x = np.ascontiguousarray(x, np.float32)
    out = np.zeros((4, int(rowptr[-1])), np.float32)
    lib().o_finegrain(C.c_int32(m), C.c_int32(n), _p(rowptr), _p(col), _p(x), _p(out))
    return out


def refine_kl(h: Hypergraph, label, passes: int):
    """Kernighan-Lin passes on the bisections of a graph (o_refine_kl):
    label[v] = 2 g + side, or -1; returns (new labels, cut reduction per
    bisection)."""
    label = np.array(label, dtype=np.int32, copy=True)
    G = max(int(label.max()) // 2 + 1, 1) if label.size else 1
    gain = np.zeros(G, np.int64)
    rc = lib().o_refine_kl(C.c_int32(h.k), C.c_int32(h.l), _p(h.ptr), _p(h.pins), _p(label), C.c_int32(passes),
                           _p(gain))
    if rc != 0:
        raise ValueError("oracle refine_kl rejected its input")
    return label, gain


# ---------------------------------------------------------------- layout ----

class LayoutParams(C.Structure):
    _fields_ = [("seed", C.c_uint64), ("coarsest_iters", C.c_int32), ("level_iters", C.c_int32),
                ("min_coarse", C.c_int32), ("max_levels", C.c_int32), ("leaf_cap", C.c_int32),
                ("match_max_net", C.c_int32), ("theta", C.c_float), ("step0_frac", C.c_float),
                ("decay", C.c_float), ("jitter", C.c_float), ("stall", C.c_float), ("pack_gap", C.c_float)]


def layout_params(seed=1, coarsest_iters=100, level_iters=30, min_coarse=64, max_levels=40, leaf_cap=8,
                  match_max_net=64, theta=0.5, step0_frac=0.1, decay=0.9, jitter=1e-3, stall=0.95,
                  pack_gap=0.1) -> LayoutParams:
    return LayoutParams(seed, coarsest_iters, level_iters, min_coarse, max_levels, leaf_cap, match_max_net,
                        theta, step0_frac, decay, jitter, stall, pack_gap)


def _wc(h: Hypergraph):
    w = h.w if h.w is not None else np.ones(h.k, dtype=np.float32)
    c = h.c if h.c is not None else np.ones(max(h.l, 1), dtype=np.float32)
    return np.ascontiguousarray(w, np.float32), np.ascontiguousarray(c, np.float32)


def coarsen(h: Hypergraph, seed: int, comp: int = 0, level: int = 0, match_max: int = 64):
    """One coarsening step (Sec. 2.3).  Returns (pi, coarse hypergraph)."""
    w, c = _wc(h)
    pi = np.zeros(h.k, dtype=np.int32)
    cptr = np.zeros(h.l + 1, dtype=np.int64)
    cpins = np.zeros(max(int(h.ptr[-1]), 1), dtype=np.int32)
    cw = np.zeros(h.k, dtype=np.float32)
    cc = np.zeros(max(h.l, 1), dtype=np.float32)
    kc, lc = C.c_int32(0), C.c_int32(0)
    rc = lib().o_coarsen(C.c_int32(h.k), C.c_int32(h.l), _p(h.ptr), _p(h.pins), _p(w), _p(c), C.c_uint64(seed),
                         C.c_uint64(comp), C.c_int32(level), C.c_int32(match_max), _p(pi), C.byref(kc), C.byref(lc),
                         _p(cptr), _p(cpins), _p(cw), _p(cc))
    assert rc == 0
    kc, lc = kc.value, lc.value
    return pi, Hypergraph(kc, lc, cptr[:lc + 1].copy(), cpins[:int(cptr[lc])].copy(), cw[:kc].copy(), cc[:lc].copy())


@dataclass
class Tree:
    n: int
    first: np.ndarray
    count: np.ndarray
    depth: np.ndarray
    leaf: np.ndarray
    next: np.ndarray
    cell2: np.ndarray
    W: np.ndarray
    X: np.ndarray
    order: np.ndarray


def tree(x, w=None, leaf_cap: int = 8) -> Tree:
    """2^d-tree with cluster charges (Sec. 2.1, Algorithm 3)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    k = x.shape[1]
    w = np.ones(k, np.float32) if w is None else np.ascontiguousarray(w, np.float32)
    cap = 17 * k + 64
    ints = np.zeros((cap, 8), dtype=np.int32)
    cell2 = np.zeros((cap, 4), dtype=np.int32)
    flt = np.zeros((cap, 5), dtype=np.float32)
    order_ = np.zeros(k, dtype=np.int32)
    n = lib().o_tree(C.c_int32(k), _p(x), _p(w), C.c_int32(leaf_cap), _p(ints), _p(cell2), _p(flt), _p(order_),
                     C.c_int32(cap))
    assert n > 0
    return Tree(n, ints[:n, 0].copy(), ints[:n, 1].copy(), ints[:n, 2].copy(), ints[:n, 3].copy(),
                ints[:n, 4].copy(), cell2[:n].copy(), flt[:n, 0].copy(), flt[:n, 1:].copy(), order_)


def gradient(h: Hypergraph, x, theta=0.5, leaf_cap=8):
    """Gradient of eq. (6) as eq. (7): attraction + tree-walk repulsion. Returns (y, z)."""
    w, c = _wc(h)
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.zeros((4, h.k), dtype=np.float32)
    z = np.zeros((4, max(h.l, 1)), dtype=np.float32)
    rc = lib().o_gradient(C.c_int32(h.k), C.c_int32(h.l), _p(h.ptr), _p(h.pins), _p(w), _p(c), _p(x),
                          C.c_float(theta), C.c_int32(leaf_cap), _p(y), _p(z))
    assert rc == 0
    return y, z[:, :h.l]


def gradient_sample(h: Hypergraph, x, ids, theta=0.5, leaf_cap=8):
    """Gradient at sampled vertices, and each one's interaction count."""
    w, c = _wc(h)
    x = np.ascontiguousarray(x, dtype=np.float32)
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    y = np.zeros((4, ids.shape[0]), dtype=np.float32)
    nint = np.zeros(ids.shape[0], dtype=np.int64)
    rc = lib().o_gradient_sample(C.c_int32(h.k), C.c_int32(h.l), _p(h.ptr), _p(h.pins), _p(w), _p(c), _p(x),
                                 C.c_float(theta), C.c_int32(leaf_cap), C.c_int32(ids.shape[0]), _p(ids), _p(y),
                                 _p(nint))
    assert rc == 0
    return y, nint


def gradient_plain(h: Hypergraph, x, theta=0.5, leaf_cap=8, ids=None):
    """Plain evaluation of eq. (7) (o_gradient_plain): FP64, one running sum
    per point over the depth-first walk from the root.  Returns (y, s, nint):
    y [4][n] FP64, s [4][n] the magnitudes that bound an FP32 evaluation's
    rounding, nint [n] interactions per walk; n = k, or len(ids)."""
    w, c = _wc(h)
    x = np.ascontiguousarray(x, dtype=np.float32)
    if ids is not None:
        ids = np.ascontiguousarray(ids, dtype=np.int32)
    n = h.k if ids is None else ids.shape[0]
    y = np.zeros((4, n), dtype=np.float64)
    s = np.zeros((4, n), dtype=np.float64)
    nint = np.zeros(max(n, 1), dtype=np.int64)
    rc = lib().o_gradient_plain(C.c_int32(h.k), C.c_int32(h.l), _p(h.ptr), _p(h.pins), _p(w), _p(c), _p(x),
                                C.c_float(theta), C.c_int32(leaf_cap), C.c_int32(n), _p(ids), _p(y), _p(s),
                                _p(nint))
    assert rc == 0
    return y, s, nint[:n]


def layout_iter_plain(h: Hypergraph, x, params: LayoutParams, it: int, alpha: float = 0.0):
    """One descent step with the plain gradient (o_layout_iter_plain).
    Returns (x_new FP32, y FP64, s FP64, alpha)."""
    w, c = _wc(h)
    x = np.ascontiguousarray(x, dtype=np.float32).copy()
    y = np.zeros((4, h.k), dtype=np.float64)
    s = np.zeros((4, h.k), dtype=np.float64)
    a = C.c_double(alpha)
    rc = lib().o_layout_iter_plain(C.c_int32(h.k), C.c_int32(h.l), _p(h.ptr), _p(h.pins), _p(w), _p(c), _p(x),
                                   C.byref(params), C.c_int32(it), C.byref(a), _p(y), _p(s))
    assert rc == 0
    return x, y, s, a.value


def interactions_reset():
    """Clears the count of walk interactions kept across strict gradients."""
    lib().o_interactions_reset()


def interactions() -> int:
    """Walk interactions of every strict gradient since the last reset (e.g.
    all levels and steps of one layout)."""
    lib().o_interactions.restype = C.c_int64
    return int(lib().o_interactions())


def layout_iter(h: Hypergraph, x, params: LayoutParams, it: int, alpha: float = 0.0):
    """One steepest-descent step (Algorithm 3).  Returns (x_new, y, alpha)."""
    w, c = _wc(h)
    x = np.ascontiguousarray(x, dtype=np.float32).copy()
    y = np.zeros((4, h.k), dtype=np.float32)
    a = C.c_double(alpha)
    rc = lib().o_layout_iter(C.c_int32(h.k), C.c_int32(h.l), _p(h.ptr), _p(h.pins), _p(w), _p(c), _p(x),
                             C.byref(params), C.c_int32(it), C.byref(a), _p(y))
    assert rc == 0
    return x, y, a.value


def layout_init(k: int, seed: int, comp: int = 0, level: int = 0):
    x = np.zeros((4, k), dtype=np.float32)
    lib().o_layout_init(C.c_int32(k), C.c_uint64(seed), C.c_uint64(comp), C.c_int32(level), _p(x))
    return x


def layout_prolong(pi, xc, seed: int, comp: int, flevel: int, jitter: float = 1e-3):
    pi = np.ascontiguousarray(pi, np.int32)
    xc = np.ascontiguousarray(xc, np.float32)
    kf, kc = pi.shape[0], xc.shape[1]
    xf = np.zeros((4, kf), dtype=np.float32)
    lib().o_layout_prolong(C.c_int32(kf), C.c_int32(kc), _p(pi), _p(xc), C.c_uint64(seed), C.c_uint64(comp),
                           C.c_int32(flevel), C.c_float(jitter), _p(xf))
    return xf


def layout(h: Hypergraph, params: LayoutParams | None = None):
    """Multilevel layout of every component, packed (Algorithm 2)."""
    params = params or layout_params()
    w, c = _wc(h)
    x = np.zeros((4, h.k), dtype=np.float32)
    rc = lib().o_layout(C.c_int32(h.k), C.c_int32(h.l), _p(h.ptr), _p(h.pins), _p(w), _p(c), C.byref(params), _p(x))
    assert rc == 0
    return x
