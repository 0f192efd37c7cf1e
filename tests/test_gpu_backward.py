"""GPU parity of the per-sample log-derivatives O_k and of the autograd
wrapper, through the C ABI, against the FP64 oracle and central finite
differences."""
import json
import os

import numpy as np
import pytest
import torch

from gpu_common import R, V, models, to_dev, host, announce
from vqmc_inputs import init_theta, neel, uniform_sz0

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "oracle_large.json")


def _rel_fro(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("L,C,n,B", [(4, 4, 2, 37), (6, 8, 3, 19), (10, 16, 6, 12), (16, 32, 8, 3)])
def test_log_derivs_parity(L, C, n, B):
    gm, rm = models(L, C, n)
    th = init_theta(C, n, seed=0)
    s = uniform_sz0(L, B, seed=1)
    ref = R.log_derivs(rm, th, s)
    announce("log_derivs", L, C, n, B)
    O = host(V.vqmc_log_derivs(gm, to_dev(th), to_dev(s)))
    rel = _rel_fro(O, ref)
    worst = max(_rel_fro(O[b], ref[b]) for b in range(B))
    print("O L=%d rel fro %.3e worst sample %.3e" % (L, rel, worst))
    assert rel <= 1e-5 and worst <= 1e-5


def test_log_derivs_24x24_against_stored_oracle():
    g = {c["L"]: c for c in json.load(open(GOLD))["cases"]}[24]
    gm, _ = models(24, g["C"], g["n"])
    s = uniform_sz0(24, g["n_samples"], seed=1)
    announce("log_derivs 24x24")
    O = host(V.vqmc_log_derivs(gm, to_dev(init_theta(g["C"], g["n"], seed=0)), to_dev(s)))
    idx = np.array(g["o_index"])
    ref = np.array(g["o_values"])
    np.testing.assert_allclose(O[:, idx], ref, rtol=1e-4, atol=1e-5 * np.abs(ref).max())
    np.testing.assert_allclose(np.linalg.norm(O, axis=1), g["o_row_norm"], rtol=1e-5)


def test_log_derivs_central_fd_10x10():
    """64 samples x 32 random parameters against central finite differences
    of the FP64 log|psi| with h = 1e-6."""
    gm, rm = models(10, 16, 6)
    th = init_theta(16, 6, seed=0)
    s = uniform_sz0(10, 64, seed=2)
    O = host(V.vqmc_log_derivs(gm, to_dev(th), to_dev(s)))
    rng = np.random.default_rng(31)
    idx = rng.choice(th.size, 32, replace=False)
    h = 1e-6
    th64 = th.astype(np.float64)
    errs = []
    for k in idx:
        tp, tm = th64.copy(), th64.copy()
        tp[k] += h
        tm[k] -= h
        fd = (R.log_psi(rm, tp, s)[0] - R.log_psi(rm, tm, s)[0]) / (2 * h)
        # per parameter: relative to the column's largest |dlog psi / dtheta_k|
        errs.append(np.abs(O[:, k] - fd).max() / np.abs(fd).max())
    errs = np.array(errs)
    print("FD max rel err %.3e" % errs.max())
    assert errs.max() <= 1e-5


def test_log_derivs_padded_rows_and_determinism():
    gm, rm = models(6, 8, 2)
    th = to_dev(init_theta(8, 2, seed=3))
    s = to_dev(uniform_sz0(6, 9, seed=4))
    P = V.num_params(gm)
    big = torch.full((9, P + 13), 7.0, dtype=torch.float32, device="cuda")
    V.vqmc_log_derivs(gm, th, s, O=big)
    O1 = V.vqmc_log_derivs(gm, th, s)
    assert torch.equal(big[:, :P], O1)
    assert bool((big[:, P:] == 7.0).all())
    O2 = V.vqmc_log_derivs(gm, th, s)
    assert torch.equal(O1, O2)
    ws = V.log_derivs_workspace(gm, 9)
    with pytest.raises(V.VqmcError):
        V.vqmc_log_derivs(gm, th, s, workspace=torch.empty(max(ws // 2, 1), dtype=torch.uint8,
                                                              device="cuda"))


def test_autograd_function_matches_oracle():
    gm, rm = models(6, 8, 2)
    th = init_theta(8, 2, seed=5)
    s = uniform_sz0(6, 11, seed=6)
    w = np.random.default_rng(7).standard_normal(11)
    t = to_dev(th).requires_grad_(True)
    lp = V.log_psi(t, to_dev(s), gm)
    (lp * to_dev(w)).sum().backward()
    ref = R.log_derivs(rm, th, s).T @ w
    np.testing.assert_allclose(host(t.grad), ref, rtol=1e-4, atol=1e-5 * np.abs(ref).max())
    np.testing.assert_allclose(host(lp), R.log_psi(rm, th, s)[0], atol=2e-4)


def test_largest_model_log_psi_and_log_derivs():
    """The largest model the library accepts (24x24, C = 32, n = 16 layers):
    log|psi| in every precision and O_k (FP32) against the oracle on two
    samples.  The log|psi| bars are those of the 10x10 parity test scaled by
    sqrt(N C n) (rounding errors of that many terms adding in quadrature)."""
    L, C, n, B = 24, 32, 16, 2
    th = init_theta(C, n, seed=4)
    s = uniform_sz0(L, B, seed=5)
    scale = np.sqrt((L * L * C * n) / (100 * 16 * 6))
    for prec, tol in ((V.PREC_FP32, 2e-4), (V.PREC_BF16X3, 5e-3), (V.PREC_BF16, 5.0)):
        gm, rm = models(L, C, n, prec)
        ref, rsg = R.log_psi(rm, th, s)
        announce("largest model log_psi", prec)
        sign = torch.empty(B, dtype=torch.int8, device="cuda")
        got = host(V.vqmc_log_psi(gm, to_dev(th), to_dev(s), sign=sign))
        err = np.abs(got - ref).max()
        print("largest model prec=%d log_psi max|err| %.3e (bar %.3e)" % (prec, err, tol * scale))
        assert err <= tol * scale
        assert (host(sign) == rsg).all()
    gm, rm = models(L, C, n)
    announce("largest model log_derivs")
    O = host(V.vqmc_log_derivs(gm, to_dev(th), to_dev(s)))
    ref = R.log_derivs(rm, th, s)
    rel = _rel_fro(O, ref)
    print("largest model O rel fro %.3e" % rel)
    assert rel <= 1e-4
