"""Writes init_prolong.json: exact values of the random coarsest start and
of one prolongation (Algorithm 2) for one vertex, derived by hand from the
random words.

The only call into the oracle is oracle.rng (SplitMix64 chained by key
words, pinned by its published output stream).  The arithmetic is written
out in exact rationals:
  start:  u = (r >> 40) / 2^24,  x = (u - 1/2) k^(1/4);  k = 16 makes
          k^(1/4) = 2, so x = ((r >> 40) - 2^23) / 2^23 exactly;
  prolongation: x_f(v) = sigma x_c(pi(v)) + eps u,  u = (r >> 40) / 2^23 - 1,
          sigma = (k_f / k_c)^(1/4) = 2 for k_f = 256, k_c = 16,
          eps = jitter (largest side of x_c) / k_c^(1/4) = 2^-10 * 8 / 2;
          sigma x_c and eps u are exact in FP32, their sum is rounded once
          to the nearest FP32 value (ties to even).
Key words: start (1 | level << 8 | comp << 32, v, d); prolongation
(2 | fine level << 8 | comp << 32, v, d).
Run: python tests/golden/make_init_prolong.py
"""
import json
import os
import sys
from fractions import Fraction

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import oracle  # noqa: E402

SEED, COMP = 7, 3


def f32(q: Fraction) -> float:
    """Nearest FP32 value of an exact rational that a double holds exactly."""
    d = float(q)
    assert Fraction(d) == q
    return float(np.float32(d))


def main():
    # coarsest start, k = 16, level 2, vertex 5
    k, level, v = 16, 2, 5
    init = []
    for d in range(4):
        r = oracle.rng(SEED, 1 | (level << 8) | (COMP << 32), v, d)
        top = r >> 40
        x = Fraction(top - 2 ** 23, 2 ** 23)
        init.append({"r": str(r), "top24": top, "x": float(x)})
    # prolongation 16 -> 256, fine level 4, coarse points on a dyadic grid
    kc, kf, flevel = 16, 256, 4
    xc = np.zeros((4, kc), np.float32)
    for i in range(kc):
        xc[0, i] = (i % 5) * 2.0          # 0..8: the largest side, 8
        xc[1, i] = (i % 3) * 0.75
        xc[2, i] = -((i % 4) * 0.5)
        xc[3, i] = (i % 2) * 1.25
    pi = (np.arange(kf) * 7 + 3) % kc
    fv = 201
    jitter = 2.0 ** -10
    eps = Fraction(2 ** -10) * 8 / 2
    pro = []
    for d in range(4):
        r = oracle.rng(SEED, 2 | (flevel << 8) | (COMP << 32), fv, d)
        top = r >> 40
        u = Fraction(top, 2 ** 23) - 1
        a = 2 * Fraction(float(xc[d, pi[fv]]))
        b = eps * u
        pro.append({"r": str(r), "top24": top, "sigma_xc": float(a), "eps_u": float(b), "x": f32(a + b)})
    out = {
        "source": "Algorithm 2: random coarsest start and prolongation with scale and small random displacement "
                  "(readings: x = (u - 1/2) k^(1/4); sigma = (k_f/k_c)^(1/4), eps = jitter * side / k_c^(1/4))",
        "seed": SEED, "comp": COMP,
        "init": {"k": k, "level": level, "v": v, "values": init},
        "prolong": {"kc": kc, "kf": kf, "fine_level": flevel, "v": fv, "jitter": jitter,
                    "xc": xc.tolist(), "pi": pi.tolist(), "values": pro},
    }
    with open(os.path.join(HERE, "init_prolong.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps({"init": init, "prolong": pro}, indent=1))


if __name__ == "__main__":
    main()
