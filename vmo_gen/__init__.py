"""Seeded synthetic sparse-matrix generators.

These build the input matrices only (CSR pattern: ``rowptr`` int64 [m+1],
``col`` int32, columns strictly ascending within a row).  They hold none of
the ordering method's arithmetic: no hypergraph model, no layout, no
bisection.  Both the CPU oracle tests and the GPU path draw their inputs from
here, so the two sides always see byte-identical matrices.

The shapes stand in for the sparse test matrices of the paper's experiments
(Section 5, Tables 3 and 4: 3.5k to 3M rows, 67k to 37M nonzeros), which are
not available here:

* ``grid2d``   2-D 5-point Laplacian pattern on an N x N grid.
* ``grid3d``   3-D 7-point Laplacian pattern on an N^3 grid, rows and columns
               permuted by one seeded Fisher-Yates permutation (P A P^T), so
               the pattern stays structurally symmetric.
* ``zipf_rect`` rectangular m x n matrix, row degrees Zipf(alpha) clipped,
               distinct uniform column indices per row.
* ``banded``   square block-banded pattern of half-bandwidth h plus a small
               fraction of uniform off-band entries.
* ``batch_banded`` / ``serve_stream`` the batched and streamed mixes.

All randomness comes from numpy's PCG64 keyed by ``(seed, tag)`` through
``numpy.random.SeedSequence``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Csr", "rng", "grid2d", "grid3d", "zipf_rect", "banded", "batch_banded",
    "serve_stream", "random_points", "random_hypergraph_csr", "csr_from_pairs",
]


@dataclass
class Csr:
    m: int
    n: int
    rowptr: np.ndarray  # int64 [m+1]
    col: np.ndarray     # int32 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])


def rng(seed: int, *tag: int) -> np.random.Generator:
    """Independent PCG64 stream for (seed, tag...)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF, *[int(t) for t in tag]])))


def csr_from_pairs(m: int, n: int, r: np.ndarray, c: np.ndarray) -> Csr:
    """CSR of the pattern {(r_i, c_i)}; duplicates removed, columns sorted."""
    r = np.asarray(r, dtype=np.int64)
    c = np.asarray(c, dtype=np.int64)
    key = np.unique(r * n + c)
    rr = key // n
    cc = (key % n).astype(np.int32)
    counts = np.bincount(rr, minlength=m).astype(np.int64)
    rowptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return Csr(m, n, rowptr, cc)


def grid2d(N: int, M: int | None = None) -> Csr:
    """5-point pattern on an M-row by N-column grid (M = N by default): row
    r*N+c couples to itself and its in-grid neighbours."""
    M = N if M is None else M
    idx = np.arange(N * M, dtype=np.int64)
    r, c = idx // N, idx % N
    rows = [idx]
    cols = [idx]
    for dr, dc in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        ok = (r + dr >= 0) & (r + dr < M) & (c + dc >= 0) & (c + dc < N)
        rows.append(idx[ok])
        cols.append((r[ok] + dr) * N + (c[ok] + dc))
    return csr_from_pairs(N * M, N * M, np.concatenate(rows), np.concatenate(cols))


def grid3d(N: int, seed: int | None = None) -> Csr:
    """7-point pattern on N^3, then one symmetric permutation P A P^T (if seed)."""
    n = N ** 3
    idx = np.arange(n, dtype=np.int64)
    x, y, z = idx % N, (idx // N) % N, idx // (N * N)
    rows = [idx]
    cols = [idx]
    for d, (ax, stride) in enumerate(((x, 1), (y, N), (z, N * N))):
        for s in (-1, 1):
            ok = (ax + s >= 0) & (ax + s < N)
            rows.append(idx[ok])
            cols.append(idx[ok] + s * stride)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    if seed is not None:
        perm = rng(seed, 2).permutation(n).astype(np.int64)  # Fisher-Yates inside numpy
        r, c = perm[r], perm[c]
    return csr_from_pairs(n, n, r, c)


def _distinct_uniform(g: np.random.Generator, deg: np.ndarray, n: int) -> tuple[np.ndarray, np.ndarray]:
    """For row i draw deg[i] distinct uniform values in [0, n) (rejection of repeats)."""
    m = deg.shape[0]
    have = np.zeros(m, dtype=np.int64)
    keys = np.zeros(0, dtype=np.int64)
    need = deg.astype(np.int64).copy()
    while need.sum() > 0:
        rows = np.repeat(np.arange(m, dtype=np.int64), need)
        vals = g.integers(0, n, size=rows.shape[0], dtype=np.int64)
        # keep draw order: first occurrence of a new value wins, none beyond need
        keys = np.concatenate([keys, rows * n + vals])
        keys = np.unique(keys)
        have = np.bincount(keys // n, minlength=m).astype(np.int64)
        need = deg - have
    return keys // n, keys % n


def zipf_rect(m: int, n: int, seed: int, alpha: float = 2.0, clip: int = 2000) -> Csr:
    """Row degrees min(Zipf(alpha), clip, n); distinct uniform columns per row."""
    g = rng(seed, 3)
    deg = np.minimum(g.zipf(alpha, size=m), min(clip, n)).astype(np.int64)
    r, c = _distinct_uniform(g, deg, n)
    return csr_from_pairs(m, n, r, c)


def banded(n: int, h: int, seed: int, frac: float = 0.001) -> Csr:
    """|i-j| <= h band plus round(frac * nnz_band) distinct uniform off-band entries."""
    i = np.arange(n, dtype=np.int64)
    rows, cols = [], []
    for s in range(-h, h + 1):
        ok = (i + s >= 0) & (i + s < n)
        rows.append(i[ok])
        cols.append(i[ok] + s)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    extra = int(round(frac * r.shape[0]))
    g = rng(seed, 4)
    er = np.zeros(0, dtype=np.int64)
    ec = np.zeros(0, dtype=np.int64)
    keys = np.zeros(0, dtype=np.int64)
    while keys.shape[0] < extra:
        a = g.integers(0, n, size=2 * (extra - keys.shape[0]) + 8, dtype=np.int64)
        b = g.integers(0, n, size=a.shape[0], dtype=np.int64)
        ok = np.abs(a - b) > h
        k2 = a[ok] * n + b[ok]
        _, first = np.unique(np.concatenate([keys, k2]), return_index=True)
        merged = np.concatenate([keys, k2])
        keys = merged[np.sort(first)][:extra]
    er, ec = keys // n, keys % n
    return csr_from_pairs(n, n, np.concatenate([r, er]), np.concatenate([c, ec]))


def batch_banded(count: int, seed: int, nmin: int = 1000, nmax: int = 50000,
                 hmin: int = 5, hmax: int = 40, pmin: int = 8, pmax: int = 32) -> list[tuple[Csr, int]]:
    """The batched mix: log-uniform sizes, uniform half-bandwidth and part counts."""
    g = rng(seed, 5)
    out = []
    for j in range(count):
        nn = int(round(math.exp(g.uniform(math.log(nmin), math.log(nmax)))))
        h = int(g.integers(hmin, hmax + 1))
        P = int(g.integers(pmin, pmax + 1))
        out.append((banded(nn, h, seed * 100003 + j), P))
    return out


def serve_stream(count: int, seed: int, rate: float = 200.0, nnz_min: float = 1e3,
                 nnz_max: float = 1e7) -> list[dict]:
    """Poisson arrivals; nnz* log-uniform; generator uniform over the three shapes."""
    g = rng(seed, 6)
    t = 0.0
    out = []
    for j in range(count):
        t += g.exponential(1.0 / rate)
        nz = math.exp(g.uniform(math.log(nnz_min), math.log(nnz_max)))
        kind = int(g.integers(0, 3))
        if kind == 0:
            side = max(2, int(round(math.sqrt(nz / 5.0))))
            spec = {"kind": "grid2d", "N": side}
        elif kind == 1:
            side = max(2, int(round((nz / 7.0) ** (1.0 / 3.0))))
            spec = {"kind": "grid3d", "N": side, "seed": seed * 7919 + j}
        else:
            rows = max(2, int(round(nz / 5.58)))
            spec = {"kind": "zipf", "m": rows, "n": max(1, rows // 2), "seed": seed * 7919 + j}
        spec["arrival"] = t
        out.append(spec)
    return out


def random_points(k: int, seed: int, clusters: int = 0, spread: float = 1.0) -> np.ndarray:
    """FP32 SoA coordinates [4, k]; optional Gaussian clusters."""
    g = rng(seed, 7)
    if clusters <= 0:
        x = g.standard_normal((4, k))
    else:
        centres = g.standard_normal((clusters, 4)) * 10.0
        lab = g.integers(0, clusters, size=k)
        x = (centres[lab] + g.standard_normal((k, 4)) * spread).T
    return np.ascontiguousarray(x.astype(np.float32))


def random_hypergraph_csr(k: int, l: int, seed: int, maxdeg: int = 6, empty_frac: float = 0.0) -> Csr:
    """Random hypergraph given as the CSR of its nets (rows = nets, cols = vertices)."""
    g = rng(seed, 8)
    deg = g.integers(1, maxdeg + 1, size=l).astype(np.int64)
    if empty_frac > 0:
        deg[g.random(l) < empty_frac] = 0
    deg = np.minimum(deg, k)
    r, c = _distinct_uniform(g, deg, k)
    return csr_from_pairs(l, k, r, c)
