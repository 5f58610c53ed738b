"""Pins for the oracle's hypergraph models, dual, components and RNG.

Each test pins the oracle to something other than itself: the worked example
of Fig. 2, the identities the paper states (the dual of the dual, row-net and
column-net are duals), brute force on dense patterns, scipy's independent
connected-components routine, and SplitMix64's published output stream.
"""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import oracle
import vmo_gen

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _f2():
    d = json.load(open(os.path.join(GOLD, "f2_hypergraph.json")))
    return d, oracle.hypergraph(d["k"], d["nets"])


def _nets(h):
    return [list(map(int, e)) for e in h.nets()]


def test_f2_dual_and_double_dual():
    d, h = _f2()
    du = oracle.dual(h)
    assert du.k == len(d["nets"]) and du.l == d["k"]
    assert _nets(du) == d["dual_nets"]
    dd = oracle.dual(du)
    assert _nets(dd) == d["nets"]


def test_f2_components():
    d, h = _f2()
    assert oracle.components(h).tolist() == d["components"]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_double_dual_is_identity_with_empty_and_duplicate_nets(seed):
    g = vmo_gen.random_hypergraph_csr(40, 60, seed, maxdeg=5, empty_frac=0.2)
    # duplicate some nets on purpose: the nets form a multiset
    rows = [list(g.col[g.rowptr[i]:g.rowptr[i + 1]]) for i in range(g.m)]
    rows += rows[:7]
    h = oracle.hypergraph(40, rows)
    dd = oracle.dual(oracle.dual(h))
    assert dd.k == h.k and dd.l == h.l
    assert np.array_equal(dd.ptr, h.ptr) and np.array_equal(dd.pins, h.pins)


def _dense(csr):
    A = np.zeros((csr.m, csr.n), dtype=bool)
    for i in range(csr.m):
        A[i, csr.col[csr.rowptr[i]:csr.rowptr[i + 1]]] = True
    return A


@pytest.mark.parametrize("seed", [4, 5])
def test_models_against_dense_brute_force(seed):
    g = vmo_gen.zipf_rect(30, 17, seed, clip=9)
    A = _dense(g)
    rn = oracle.rownet(g.m, g.n, g.rowptr, g.col)
    cn = oracle.colnet(g.m, g.n, g.rowptr, g.col)
    assert rn.k == 17 and rn.l == 30
    assert _nets(rn) == [list(np.nonzero(A[i])[0]) for i in range(30)]
    assert cn.k == 30 and cn.l == 17
    assert _nets(cn) == [list(np.nonzero(A[:, j])[0]) for j in range(17)]


@pytest.mark.parametrize("seed", [6, 7])
def test_rownet_and_colnet_are_duals(seed):
    """Observation 4 after Table 1: the column-net and row-net models are each other's dual."""
    g = vmo_gen.zipf_rect(50, 33, seed, clip=12)
    rn = oracle.rownet(g.m, g.n, g.rowptr, g.col)
    cn = oracle.colnet(g.m, g.n, g.rowptr, g.col)
    d = oracle.dual(rn)
    assert d.k == cn.k and d.l == cn.l
    assert np.array_equal(d.ptr, cn.ptr) and np.array_equal(d.pins, cn.pins)


def test_symmetric_model_brute_force():
    g = vmo_gen.grid3d(3, seed=11)
    A = _dense(g)
    assert (A == A.T).all()
    h = oracle.symmetric(g.m, g.n, g.rowptr, g.col)
    want = [[i, j] for i in range(g.n) for j in range(i + 1, g.n) if A[i, j]]
    assert _nets(h) == want
    # 7-point stencil on 3^3: 3 * 2 * 3 * 3 = 54 undirected edges
    assert h.l == 54


def test_grid3d_nnz_closed_form():
    for N in (2, 3, 5):
        g = vmo_gen.grid3d(N, seed=1)
        assert g.nnz == 7 * N ** 3 - 6 * N ** 2


@pytest.mark.parametrize("seed", [8, 9, 10])
def test_components_against_scipy(seed):
    g = vmo_gen.random_hypergraph_csr(300, 120, seed, maxdeg=3, empty_frac=0.1)
    h = oracle.rownet(g.m, g.n, g.rowptr, g.col)
    lab = oracle.components(h)
    # vertex-vertex graph through nets, via the incidence matrix B: B^T B
    B = sp.csr_matrix((np.ones(g.nnz), g.col, g.rowptr), shape=(g.m, g.n))
    ncomp, sc = csg.connected_components(B.T @ B, directed=False)
    # min-id label per scipy component
    mins = np.full(ncomp, h.k)
    for v in range(h.k):
        mins[sc[v]] = min(mins[sc[v]], v)
    assert np.array_equal(lab, mins[sc])


def test_splitmix64_published_stream():
    """SplitMix64 (Steele, Lea, Flood 2014) seeded with 1234567."""
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    assert [oracle.splitmix64(1234567, i) for i in range(1, 6)] == want


def test_rng_chains_the_stream():
    """rng(seed, a, b, c) = the (c+1)-th output of the stream seeded by the
    (b+1)-th output of the stream seeded by the (a+1)-th output of seed."""
    s0 = oracle.splitmix64(99, 3 + 1)
    s1 = oracle.splitmix64(s0, 5 + 1)
    assert oracle.rng(99, 3, 5, 7) == oracle.splitmix64(s1, 7 + 1)
