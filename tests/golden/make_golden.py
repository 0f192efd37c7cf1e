"""Writes tests/golden/oracle_large.json: FP64 oracle values at lattice sizes
whose oracle cost is too high to recompute inside a test run (16x16 and
24x24, C = 32, n = 8).  Calls only the oracle and the shared input
generators.

    python tests/golden/make_golden.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as R  # noqa: E402
from vqmc_inputs import init_theta, uniform_sz0  # noqa: E402

CASES = [
    # (L, C, n, n_samples): uniform Sz = 0 configurations (seed 1), theta seed 0
    (16, 32, 8, 2),
    (24, 32, 8, 2),
]
O_INDEX_SEED = 5
O_INDEX_COUNT = 96


def main():
    out = {"note": "FP64 oracle values; theta = init_theta(C, n, seed=0), spins = "
                   "uniform_sz0(L, B, seed=1)[:n_samples]; J1 = 1, J2 = 0.5, Marshall sign on",
           "cases": []}
    for L, C, n, ns in CASES:
        t0 = time.time()
        m = R.RefModel(L, C, n, 1.0, 0.5, 1)
        th = init_theta(C, n, seed=0)
        s = uniform_sz0(L, ns, seed=1)
        la, sg = R.log_psi(m, th, s)
        el = R.local_energy(m, th, s)
        O = R.log_derivs(m, th, s)
        idx = np.sort(np.random.default_rng(O_INDEX_SEED).choice(O.shape[1], O_INDEX_COUNT,
                                                                  replace=False))
        out["cases"].append(dict(L=L, C=C, n=n, n_samples=ns, log_psi=la.tolist(),
                                 sign=sg.astype(int).tolist(), e_loc=el.tolist(),
                                 o_index=idx.tolist(), o_values=O[:, idx].tolist(),
                                 o_row_norm=np.linalg.norm(O, axis=1).tolist()))
        print("L=%d done in %.1f s" % (L, time.time() - t0), flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_large.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
