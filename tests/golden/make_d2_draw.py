"""Writes d2_draw.json: a hand-checkable case of the k-means++ D^2 draw
(Algorithm 4, m = 2) in which the random point t falls exactly on a prefix
sum of the D^2 weights, so that the draw rule decides which point is taken.

The only call into the oracle is oracle.rng (SplitMix64 chained by key
words, pinned by its published output stream); everything else is exact
integer arithmetic written out here:
  i1 = floor(r0 * n / 2^64),  d_i = |q_i - q_i1|^2,  T = sum d_i,
  t  = floor(r1 * T / 2^64),  i2 = min{ i : d_0 + ... + d_i > t }.
The points are integers on the 2^20 grid with lo = 0 and largest side
2^20 - 1 in every run, so quantization maps them to themselves (scale 1).
Run: python tests/golden/make_d2_draw.py
"""
import itertools
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import oracle  # noqa: E402

TAG_KMEANS = 16
QMAX = 2 ** 20 - 1
N = 6
MID = 2 ** 19


def four_squares(m, cap):
    """Some (a, b, c, e) with a^2 + b^2 + c^2 + e^2 = m, all <= cap."""
    a = min(math.isqrt(m), cap)
    while a >= 0:
        r = m - a * a
        b = min(math.isqrt(r), cap)
        while b >= 0 and b >= math.isqrt(max(r - b * b, 0)) // 2:
            r2 = r - b * b
            c = min(math.isqrt(r2), cap)
            while c >= 0:
                e2 = r2 - c * c
                e = math.isqrt(e2)
                if e * e == e2 and e <= cap:
                    return a, b, c, e
                c -= 1
                if c < math.isqrt(e2) - 2:
                    break
            b -= 1
        a -= 1
    return None


def design(seed):
    r0 = oracle.rng(seed, TAG_KMEANS, 1, 0)
    r1 = oracle.rng(seed, TAG_KMEANS, 1, 1)
    i1 = (r0 * N) >> 64
    phi = r1 / 2 ** 64
    # fixed points besides z1 = (MID, 0, 0, 0): the two ends of the box in
    # dimension 0 and two near points; one more near point u is tuned
    fixed = {"A": (0, 3, 0, 0), "B": (QMAX, 0, 5, 0), "P": (MID + 7, 11, 0, 2), "Q": (MID - 40, 0, 0, 13)}
    slots = [i for i in range(N) if i != i1]
    for perm in itertools.permutations(list(fixed) + ["U"]):
        at = dict(zip(slots, perm))
        for j in slots:
            if j + 1 >= N or j + 2 >= N:
                continue
            if at.get(j + 1) is None or at.get(j + 2) is None:
                continue   # j+1 or j+2 is z1
            # u must lie at or before j so that it moves the prefix and T
            u = [i for i in slots if at[i] == "U"][0]
            if u > j:
                continue
            dist = {nm: sum((a - b) ** 2 for a, b in zip(p, (MID, 0, 0, 0))) for nm, p in fixed.items()}
            X = sum(dist[at[i]] for i in slots if i <= j and at[i] != "U")
            Y = sum(dist[at[i]] for i in slots if i > j)
            est = (phi * (X + Y) - X) / (1 - phi)
            if est < 1:
                continue
            for du in range(max(int(est) - 3, 1), int(est) + 4):
                T = X + du + Y
                t = (r1 * T) >> 64
                if t != X + du:
                    continue
                sq = four_squares(du, MID - 100)
                if sq is None:
                    continue
                pts = [None] * N
                pts[i1] = (MID, 0, 0, 0)
                for i in slots:
                    pts[i] = fixed[at[i]] if at[i] != "U" else (MID + sq[0], sq[1], sq[2], sq[3])
                return r0, r1, i1, j, pts
    return None


def main():
    for seed in range(1, 2000):
        got = design(seed)
        if got:
            break
    r0, r1, i1, j, pts = got
    d = [sum((a - b) ** 2 for a, b in zip(p, pts[i1])) for p in pts]
    T = sum(d)
    t = (r1 * T) >> 64
    pre = list(itertools.accumulate(d))
    i2 = min(i for i in range(N) if pre[i] > t)
    i2_ge = min(i for i in range(N) if pre[i] >= t)
    i2_excl = min(i for i in range(N) if pre[i] - d[i] > t)
    assert pre[j] == t and i2 == j + 1 and len({i2, i2_ge, i2_excl}) == 3
    for dim in range(4):
        assert min(p[dim] for p in pts) == 0
    assert max(max(p[dim] for p in pts) for dim in range(4)) == QMAX
    out = {
        "source": "Algorithm 4 (k-means++ with m = 2): z1 uniform, z2 drawn with probability d_i / T; "
                  "exact integer draw i2 = min{i : prefix_incl(i) > t}, t = floor(r1 T / 2^64)",
        "seed": seed, "job": 0, "node": 1, "n": N,
        "points_q": [list(p) for p in pts],
        "r0": str(r0), "r1": str(r1),
        "i1": i1, "d": [str(v) for v in d], "T": str(T), "t": str(t),
        "prefix_incl": [str(v) for v in pre],
        "i2": i2,
        "i2_if_ge": i2_ge, "i2_if_exclusive_prefix": i2_excl,
        "why": "t equals the inclusive prefix at index %d exactly, so the strict rule (>) takes the next point "
               "%d; a >= rule would take %d and an exclusive prefix %d" % (j, i2, i2_ge, i2_excl),
    }
    with open(os.path.join(HERE, "d2_draw.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
