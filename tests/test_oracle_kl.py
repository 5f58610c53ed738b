"""Oracle pins for the Kernighan-Lin refinement (Sec. 3: partitionings of
Algorithm 4 improved by a few Kernighan-Lin iterations; Kernighan and Lin
1970): a hand-derived pass sequence, two cliques joined by one edge (the
optimal cut is found), and on random graphs with several bisections the
invariants (side sizes kept, other vertices untouched, the reported gain equal
to the recounted cut reduction) and, after convergence, that no single pair
swap lowers the cut (brute force)."""
import json
import os

import numpy as np
import pytest

import oracle
import vmo_gen

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "kl_path4.json")


def edge_graph(k, edges):
    edges = [tuple(sorted(e)) for e in edges]
    ptr = np.arange(0, 2 * len(edges) + 1, 2, dtype=np.int64)
    pins = np.array([p for e in edges for p in e], dtype=np.int32)
    return oracle.Hypergraph(k, len(edges), ptr, pins)


def group_cut(edges, label, g):
    c = 0
    for a, b in edges:
        if label[a] >= 0 and label[b] >= 0 and label[a] // 2 == g and label[b] // 2 == g:
            c += label[a] % 2 != label[b] % 2
    return c


def random_graph(k, l, seed):
    r = vmo_gen.rng(seed, 9)
    a = r.integers(0, k, size=l)
    b = r.integers(0, k, size=l)
    keep = a != b
    return [(int(min(x, y)), int(max(x, y))) for x, y in zip(a[keep], b[keep])]


def test_kl_hand_derived():
    g = json.load(open(GOLDEN))
    h = edge_graph(g["k"], g["edges"])
    out, gain = oracle.refine_kl(h, g["label_in"], 8)
    assert out.tolist() == g["label_out"] and gain.tolist() == g["gain"]
    one, gain1 = oracle.refine_kl(h, g["label_in"], 1)   # the first pass alone
    assert one.tolist() == g["label_out"] and gain1.tolist() == g["gain"]
    zero, gain0 = oracle.refine_kl(h, g["label_in"], 0)
    assert zero.tolist() == g["label_in"] and gain0.tolist() == [0]


def test_kl_two_cliques():
    edges = [(a, b) for a in range(5) for b in range(a + 1, 5)]
    edges += [(a, b) for a in range(5, 10) for b in range(a + 1, 10)] + [(4, 5)]
    h = edge_graph(10, edges)
    label = [0, 0, 0, 1, 1, 1, 1, 1, 0, 0]                # two vertices of each clique misplaced
    out, gain = oracle.refine_kl(h, label, 4)
    assert group_cut(edges, out, 0) == 1                  # the single joining edge
    assert int(gain[0]) == group_cut(edges, label, 0) - 1
    assert len(set(out[:5].tolist())) == 1 and len(set(out[5:].tolist())) == 1


@pytest.mark.parametrize("k,l,G,seed", [(60, 150, 1, 1), (200, 500, 3, 2), (300, 700, 5, 3), (120, 600, 2, 4)])
def test_kl_invariants_and_local_optimum(k, l, G, seed):
    edges = random_graph(k, l, seed)
    h = edge_graph(k, edges)
    r = vmo_gen.rng(seed, 10)
    label = np.where(r.random(k) < 0.1, -1, 2 * r.integers(0, G, size=k) + r.integers(0, 2, size=k)).astype(np.int32)
    out, gain = oracle.refine_kl(h, label, 50)
    assert np.array_equal(out < 0, label < 0)
    for g in range(G):
        before = label[label // 2 == g]
        after = out[(out // 2 == g) & (out >= 0)]
        assert np.array_equal(np.sort(before[before >= 0] % 2), np.sort(after % 2))   # side sizes kept
        assert np.array_equal(np.nonzero((label >= 0) & (label // 2 == g))[0],
                              np.nonzero((out >= 0) & (out // 2 == g))[0])         # membership kept
        assert int(gain[g]) == group_cut(edges, label, g) - group_cut(edges, out, g) >= 0
        # converged: no pair swap inside the bisection lowers its cut
        A = [v for v in range(k) if out[v] == 2 * g]
        B = [v for v in range(k) if out[v] == 2 * g + 1]
        c0 = group_cut(edges, out, g)
        for a in A:
            for b in B:
                t = out.copy()
                t[a], t[b] = t[b], t[a]
                assert group_cut(edges, t, g) >= c0, (a, b)
