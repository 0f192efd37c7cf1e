"""Parity of the whole hot path at the 16x16 and 24x24 workload sizes, in the
launch configuration bench.py times (the full batch in one call per entry
point), against stored FP64 oracle values (tests/golden/oracle_subsets.json,
written by tests/golden/make_golden.py) and live oracle calls:

* rows that the kernels reach only after their grid has gone round once
  (the light-cone local energy runs at most 256 workgroups at 24x24, the
  log-derivatives at most 2048): E_loc and sampled O columns per row;
* the error subset, the first 256 configurations of the batch: E_loc (Eq.
  Es-Os-G) per precision, O_k, and the SR step (Eq. delta) solved by the
  library on its own E and O against the oracle's exact solve on the
  oracle's E and O -- the errors of E/N, O_k and delta that the precision
  forms are held to (|dE/N| <= 1e-4 relative, O_k and delta <= 1e-3)."""
import json
import os

import numpy as np
import pytest
import torch

from gpu_common import R, V, models, to_dev, host, announce
from vqmc_inputs import init_theta, uniform_sz0

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "oracle_subsets.json")
PREC = {"fp32": V.PREC_FP32, "bf16x3": V.PREC_BF16X3, "bf16": V.PREC_BF16}
# per-row relative E_loc error (max over rows) and |dE/N| of the mean
E_BAR = {"fp32": (1e-4, 5e-5), "bf16x3": (1e-3, 1e-4), "bf16": (1e-1, 1e-2)}


def _case(L):
    return {c["L"]: c for c in json.load(open(GOLD))["cases"]}[L]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("L", [16, 24])
def test_full_batch_pipeline_against_oracle(L):
    g = _case(L)
    C, n, B = g["C"], g["n"], g["B"]
    st, sub = g["stride"], g["subset"]
    ns = sub["n_samples"]
    pos = np.array(st["index"])
    th_np = init_theta(C, n, seed=0)
    s_np = uniform_sz0(L, B, seed=1)
    th, s = to_dev(th_np), to_dev(s_np)
    gm, rm = models(L, C, n)
    assert V.local_energy_method(gm) == V.ELOC_LIGHTCONE
    e_sub = {}
    for name, prec in PREC.items():
        announce("%dx%d full batch B=%d local energy" % (L, L, B), name)
        flags = torch.full((B,), -1, dtype=torch.int32, device="cuda")
        el = host(V.vqmc_local_energy(gm.with_prec(prec), th, s, flags=flags))
        assert (host(flags) == 0).all() and np.isfinite(el).all()
        # per-row errors relative to |E_loc| or, where a row's terms nearly
        # cancel, to the batch's root-mean-square local energy
        ref = np.array(sub["e_loc"])
        scale = np.sqrt((ref ** 2).mean())
        rs = np.abs(el[pos] - st["e_loc"]) / np.maximum(np.abs(st["e_loc"]), scale)
        rb = np.abs(el[:ns] - ref) / np.maximum(np.abs(ref), scale)
        de = abs(el[:ns].mean() - ref.mean()) / abs(ref.mean())
        print("%dx%d %s E_loc: later rows max rel %.2e, first %d rows max rel %.2e, |dE/N| rel %.2e"
              % (L, L, name, rs.max(), ns, rb.max(), de), flush=True)
        bar, mbar = E_BAR[name]
        assert rs.max() <= bar and rb.max() <= bar
        assert de <= mbar
        e_sub[name] = el[:ns].copy()
    announce("%dx%d full batch log-derivatives" % (L, L))
    O = V.vqmc_log_derivs(gm, th, s)
    Op = host(O[torch.from_numpy(pos).cuda()])
    idx = np.array(st["o_index"])
    ov = np.take_along_axis(Op, np.repeat(idx[None, :], len(pos), 0), axis=1)
    ref = np.array(st["o_values"])
    err = np.abs(ov - ref).max() / np.abs(ref).max()
    print("%dx%d O later rows: sampled columns max rel %.2e" % (L, L, err), flush=True)
    assert err <= 1e-5
    np.testing.assert_allclose(np.linalg.norm(Op, axis=1), st["o_row_norm"], rtol=1e-5)
    # the error subset: O_k and the SR step against the oracle's
    O_sub = O[:ns].contiguous()
    del O
    O_ref = R.log_derivs(rm, th_np, s_np[:ns])
    Og = host(O_sub).astype(np.float64)
    o_err = _rel(Og, O_ref)
    o_row = (np.linalg.norm(Og - O_ref, axis=1) / np.linalg.norm(O_ref, axis=1)).max()
    print("%dx%d O first %d rows: Frobenius rel %.2e, worst row %.2e" % (L, L, ns, o_err, o_row), flush=True)
    assert o_err <= 1e-5 and o_row <= 1e-5
    d_ref = R.sr_solve(O_ref, np.array(sub["e_loc"]), 1e-4)["delta"]
    for name in ("fp32", "bf16x3", "bf16"):
        d, _, info = V.vqmc_sr_solve(O_sub, to_dev(e_sub[name]), V.SrOpts(method=V.SR_DUAL, eps=1e-4))
        d_err = _rel(host(d), d_ref)
        print("%dx%d delta (sample-space Cholesky) with %s energies: rel %.2e" % (L, L, name, d_err), flush=True)
        if name != "bf16":
            assert d_err <= 1e-3
