"""Write learned_ceiling.json: what per-tile slice counts can gain once FP64
refinement is part of the solve, on the oracle alone.

For each phi-matrix (n = 1024, nb = 256, seed 61, right-hand side U(-1,1)
seed 62): the smallest constant slice count whose LU reaches a backward
error of 1e-15 within two refinement steps, and the ideal per-tile maps: on
the s = 9 factorization's path, each update tile's label (the smallest s whose
tile update is within tau of the s = 9 update) for three tau, the LU with
those maps, and the refinement steps it then needs.  Every value comes from
oracle/ on inputs from matgen/; run from the repository root:

    python tests/golden/make_learned_ceiling.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import matgen  # noqa: E402
import oracle as O  # noqa: E402
from oracle import learned as OL  # noqa: E402

N, NB, TOL = 1024, 256, 1e-15


def best_constant(A, b, max_steps=2):
    for s in range(3, 10):
        _, io = O.gesv_ir(A, b, nb=NB, s=s, tol=TOL, maxiter=max_steps, s_max=s)
        if io["converged"]:
            return s, io["iters"]
    return None, None


def ideal_map(A, b, tau):
    LU, piv, _ = O.getrf(A, nb=NB, s=9)
    steps = []
    for j1 in range(NB, N, NB):
        j0 = j1 - NB
        steps.append(OL.tile_labels(np.asfortranarray(LU[j1:, j0:j1]),
                                    np.asfortranarray(LU[j0:j1, j1:]), tau=tau))
    Lm, pv, _ = OL.getrf_tiles(A, NB, steps)
    x = O.getrs(Lm, pv, b)
    it = 0
    while O.backward_error(A, x, b) > TOL and it < 10:
        x = x + O.getrs(Lm, pv, b - A @ x)
        it += 1
    labels = np.concatenate(steps)
    return {"products_per_tile": float(np.mean(labels * (labels + 1) / 2)),
            "label_counts_s3_to_s9": np.bincount(labels, minlength=10)[3:].tolist(),
            "refinement_steps": it}


def main():
    out = {"n": N, "nb": NB, "tol": TOL, "max_steps_constant": 2, "full_count_products": 45,
           "rows": []}
    for phi in (0.0, 1.0, 4.0, 8.0, 12.0):
        A = matgen.phi_matrix(N, N, phi, seed=61)
        b = matgen.uniform(N, 1, seed=62)
        s, it = best_constant(A, b)
        row = {"phi": phi, "best_constant_s": s, "best_constant_steps": it,
               "best_constant_products": s * (s + 1) // 2, "ideal": {}}
        for te in (26, 30, 40):
            row["ideal"][f"tau=2^-{te}"] = ideal_map(A, b, 2.0 ** -te)
        out["rows"].append(row)
        print(row, flush=True)
    with open(os.path.join(HERE, "learned_ceiling.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
