"""Writes the stored FP64 oracle values that are too costly to recompute
inside a test run.  Calls only the oracle and the shared input generators.

    python tests/golden/make_golden.py [large] [subsets] [10x10]

* oracle_large.json   -- 16x16 and 24x24 (C = 32, n = 8): log psi, E_loc and
                         96 sampled columns of O for the first two uniform
                         Sz = 0 configurations;
* oracle_subsets.json -- 16x16 and 24x24: log psi and E_loc of the first 256
                         configurations of the full batch (the error subset of
                         the 24x24 workload), and log psi, E_loc and sampled O
                         columns of configurations at later positions of the
                         full batch (the ones a kernel reaches only after its
                         grid has gone round once);
* oracle_10x10.json   -- 10x10 (C = 16, n = 6): E_loc of the full batch of
                         4096 uniform configurations, and 32 Metropolis chains
                         run by the oracle's sampler from the Neel state, with
                         their final configurations, log psi and E_loc.
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as R  # noqa: E402
from vqmc_inputs import init_theta, neel, uniform_sz0  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
NOTE = ("FP64 oracle values; theta = init_theta(C, n, seed=0), spins = uniform_sz0(L, B, seed=1) "
        "(the first rows of any larger batch are the same); J1 = 1, J2 = 0.5, Marshall sign on")

LARGE_CASES = [(16, 32, 8, 2), (24, 32, 8, 2)]  # (L, C, n, n_samples)
O_INDEX_SEED = 5
O_INDEX_COUNT = 96

# full batch sizes of the two large workloads, and positions in them that lie
# beyond one pass of any grid the library launches there (256 light-cone
# workgroups at 24x24, at most 2048 log-derivative workgroups), with the
# first and last rows of a few later rounds
SUBSET = 256
STRIDE_INDEX = {
    16: [256, 257, 511, 1000, 2048, 2049, 4095, 6000, 8191],
    24: [256, 257, 511, 1000, 2048, 2049, 4095, 8191, 12289, 16383],
}
FULL_B = {16: 8192, 24: 16384}

B10 = 4096
METRO_CHAINS, METRO_SWEEPS, METRO_SEED = 32, 500, 2


def _o_columns(O):
    idx = np.sort(np.random.default_rng(O_INDEX_SEED).choice(O.shape[1], O_INDEX_COUNT, replace=False))
    return idx, O[:, idx]


def large():
    out = {"note": NOTE, "cases": []}
    for L, C, n, ns in LARGE_CASES:
        t0 = time.time()
        m = R.RefModel(L, C, n, 1.0, 0.5, 1)
        th = init_theta(C, n, seed=0)
        s = uniform_sz0(L, ns, seed=1)
        la, sg = R.log_psi(m, th, s)
        el = R.local_energy(m, th, s)
        O = R.log_derivs(m, th, s)
        idx, ov = _o_columns(O)
        out["cases"].append(dict(L=L, C=C, n=n, n_samples=ns, log_psi=la.tolist(),
                                 sign=sg.astype(int).tolist(), e_loc=el.tolist(),
                                 o_index=idx.tolist(), o_values=ov.tolist(),
                                 o_row_norm=np.linalg.norm(O, axis=1).tolist()))
        print("large L=%d done in %.1f s" % (L, time.time() - t0), flush=True)
    _write("oracle_large.json", out)


def subsets():
    out = {"note": NOTE, "cases": []}
    for L in (16, 24):
        C, n, B = 32, 8, FULL_B[L]
        m = R.RefModel(L, C, n, 1.0, 0.5, 1)
        th = init_theta(C, n, seed=0)
        s_all = uniform_sz0(L, B, seed=1)
        t0 = time.time()
        pos = np.array(STRIDE_INDEX[L])
        s = s_all[pos]
        la, sg = R.log_psi(m, th, s)
        el = R.local_energy(m, th, s)
        O = R.log_derivs(m, th, s)
        idx, ov = _o_columns(O)
        stride = dict(index=pos.tolist(), log_psi=la.tolist(), sign=sg.astype(int).tolist(),
                      e_loc=el.tolist(), o_index=idx.tolist(), o_values=ov.tolist(),
                      o_row_norm=np.linalg.norm(O, axis=1).tolist())
        print("subsets L=%d: %d later rows in %.1f s" % (L, len(pos), time.time() - t0), flush=True)
        t0 = time.time()
        s = s_all[:SUBSET]
        la, sg = R.log_psi(m, th, s)
        el = R.local_energy(m, th, s)
        print("subsets L=%d: first %d rows in %.1f s" % (L, SUBSET, time.time() - t0), flush=True)
        out["cases"].append(dict(L=L, C=C, n=n, B=B, stride=stride,
                                 subset=dict(n_samples=SUBSET, log_psi=la.tolist(),
                                             sign=sg.astype(int).tolist(), e_loc=el.tolist())))
        _write("oracle_subsets.json", out)


def tenbyten():
    L, C, n = 10, 16, 6
    m = R.RefModel(L, C, n, 1.0, 0.5, 1)
    th = init_theta(C, n, seed=0)
    t0 = time.time()
    el = R.local_energy(m, th, uniform_sz0(L, B10, seed=1))
    print("10x10: E_loc of %d uniform configurations in %.1f s" % (B10, time.time() - t0), flush=True)
    t0 = time.time()
    s, la, na, mm = R.sample(m, th, neel(L, METRO_CHAINS), METRO_SWEEPS, METRO_SEED)
    em = R.local_energy(m, th, s)
    print("10x10: %d chains x %d sweeps in %.1f s, acceptance %.3f" % (
        METRO_CHAINS, METRO_SWEEPS, time.time() - t0, na.sum() / (METRO_CHAINS * METRO_SWEEPS * L * L)),
        flush=True)
    out = {"note": NOTE.replace("spins = uniform_sz0(L, B, seed=1)", "uniform: spins = uniform_sz0(10, 4096, "
                                "seed=1)"),
           "L": L, "C": C, "n": n,
           "uniform": dict(B=B10, e_loc=el.tolist()),
           "metropolis": dict(chains=METRO_CHAINS, sweeps=METRO_SWEEPS, seed=METRO_SEED, proposal=0,
                              start="neel", counter_base=0,
                              spins=["".join("u" if v > 0 else "d" for v in row) for row in s],
                              log_psi=la.tolist(), e_loc=em.tolist(), n_accepted=na.tolist())}
    _write("oracle_10x10.json", out)


def _write(name, obj):
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(obj, f, indent=1)


def main(argv):
    parts = argv or ["large", "subsets", "10x10"]
    for p in parts:
        {"large": large, "subsets": subsets, "10x10": tenbyten}[p]()


if __name__ == "__main__":
    main(sys.argv[1:])
