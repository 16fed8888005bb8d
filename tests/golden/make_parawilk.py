"""Write parawilk_table1.json: scaled residuals (eqn (9)) of the oracle's
emulated LU solve of randomized ParaWilk_256(d=4, b=15, alpha=1/2) for 3..9
slices and native FP64, block size 64, several seeds.

The setting is the paper's Table 1 (numerical-properties section); the right-hand side
is HPL's U(-1/2, 1/2) (the paper does not state it).  Every value comes
from oracle/ on inputs from matgen/; run from the repository root:

    python tests/golden/make_parawilk.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import matgen  # noqa: E402
import oracle as O  # noqa: E402

N, D, BLK, ALPHA, NB = 256, 4, 15, 0.5, 64
SEEDS = list(range(6))
SLICES = list(range(3, 10))


def case(seed):
    A = matgen.parawilk_random(N, D, BLK, ALPHA, seed=seed)
    b = matgen.hpl_uniform(N, seed=seed, substream=1)[:, :1]
    return A, b


def main():
    out = {"n": N, "d": D, "b": BLK, "alpha": ALPHA, "nb": NB, "rhs": "U(-1/2,1/2)",
           "seeds": {}}
    for seed in SEEDS:
        A, b = case(seed)
        row = {}
        for s in SLICES + [None]:
            LU, piv, info = O.getrf(A, nb=NB, s=s)
            x = O.getrs(LU, piv, b)
            row["native" if s is None else str(s)] = O.scaled_residual(A, x, b)
        out["seeds"][str(seed)] = row
    with open(os.path.join(HERE, "parawilk_table1.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
