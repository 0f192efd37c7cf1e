"""GPU parity of the SR step (F, <E>, Var E and the solution of
(S + eps I) delta = F) against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest
import torch

from gpu_common import R, V, models, to_dev, host, announce
from vqmc_inputs import init_theta, uniform_sz0

pytestmark = pytest.mark.gpu


def _rand(B, P, seed):
    rng = np.random.default_rng(seed)
    O = (rng.standard_normal((B, P)) * 0.5 + rng.standard_normal(P)).astype(np.float32)
    E = rng.standard_normal(B) * 3 - 40
    return O, E


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


# sizes span partial 64-blocks, odd orders (unaligned rows, scalar loads),
# several 512-column outer panels (above 1024 the trailing update of the
# later columns runs on the side stream), an order that is a multiple of 128
# (the right-hand side row then opens a block row of its own) and of 256, and
# last outer panels of several sub-panels ending in a partial one (700, 1700:
# the fused per-sub-panel launch with fewer than 64 columns), and the next-panel
# update's 64-row tiles ending in a partial tile (577: 66 rows after the first
# panel) or exactly (1088: 577 rows, the rest of the trailing matrix one tile);
# the last two put a single partial 128-row tile and a partial last K chunk
# on the direct-to-LDS S and Gram kernels (P a multiple of 4, B and P not of 16)
CASES = [(300, 200), (200, 517), (64, 64), (97, 1), (130, 384), (256, 512), (515, 300), (777, 1030),
         (300, 700), (900, 1700), (300, 577), (640, 1088), (17, 44), (129, 132)]


@pytest.mark.parametrize("B,P", CASES)
@pytest.mark.parametrize("method,s_prec", [(V.SR_CHOLESKY, 1), (V.SR_DUAL, 1), (V.SR_CG, 1)])
def test_sr_small_parity(B, P, method, s_prec):
    O, E = _rand(B, P, B + P)
    eps = 1e-2 if method == V.SR_CG else 1e-4
    ref = R.sr_solve(O.astype(np.float64), E, eps)
    announce("sr", B, P, method)
    opts = V.SrOpts(method=method, s_prec=s_prec, eps=eps, tol=1e-12, max_iter=2000)
    d, F, info = V.vqmc_sr_solve(to_dev(O), to_dev(E), opts)
    d, F = host(d), host(F)
    assert info["e_mean"] == pytest.approx(ref["e_mean"], rel=1e-14)
    assert info["e_var"] == pytest.approx(ref["e_var"], rel=1e-12)
    assert _rel(F, ref["F"]) <= 1e-12
    tol = 1e-7 if method == V.SR_CG else 1e-9
    print("B=%d P=%d method=%d delta rel %.3e iters %d" % (B, P, method, _rel(d, ref["delta"]),
                                                         info["iters"]))
    assert _rel(d, ref["delta"]) <= tol
    if method == V.SR_CG:
        assert info["converged"] and info["rel_residual"] <= 1e-12


@pytest.mark.parametrize("method,s_prec", [(V.SR_CHOLESKY, 0), (V.SR_CHOLESKY, 1), (V.SR_DUAL, 1), (V.SR_CG, 1)])
def test_sr_padded_rows(method, s_prec):
    """O as a view into wider rows (row stride ldO > P): with 16-byte rows
    (ldO a multiple of 4) the same kernels run and delta is bit-identical to
    the contiguous O; with an odd stride the scalar-load forms run and agree
    to rounding."""
    B, P = 300, 200
    O, E = _rand(B, P, 21)
    Od, Ed = to_dev(O), to_dev(E)
    announce("sr padded rows", method, s_prec)
    opts = V.SrOpts(method=method, s_prec=s_prec, eps=1e-3, tol=1e-12, max_iter=500)
    d0, F0, _ = V.vqmc_sr_solve(Od, Ed, opts)
    for pad, exact in ((12, True), (1, False)):
        wide = torch.full((B, P + pad), float("nan"), dtype=torch.float32, device="cuda")
        wide[:, :P] = Od
        d1, F1, _ = V.vqmc_sr_solve(wide[:, :P], Ed, opts)
        if exact:
            assert torch.equal(d1, d0) and torch.equal(F1, F0), pad
        else:
            assert _rel(host(d1), host(d0)) <= 1e-12 and _rel(host(F1), host(F0)) <= 1e-14, pad


@pytest.mark.parametrize("method,s_prec", [(V.SR_CHOLESKY, 0), (V.SR_CHOLESKY, 1), (V.SR_DUAL, 1), (V.SR_CG, 1)])
def test_sr_run_to_run_bit_identical(method, s_prec):
    """Two calls on the same inputs give the same bits: no atomics, fixed
    reduction orders, and at this order (above 1024) the Cholesky's trailing
    update runs on the side stream, ordered against the panel chain by events."""
    B, P = 900, 1700
    O, E = _rand(B, P, 5)
    Od, Ed = to_dev(O), to_dev(E)
    announce("sr determinism", method, s_prec)
    opts = V.SrOpts(method=method, s_prec=s_prec, eps=1e-3, tol=1e-10, max_iter=300)
    d1, F1, i1 = V.vqmc_sr_solve(Od, Ed, opts)
    d2, F2, i2 = V.vqmc_sr_solve(Od, Ed, opts)
    assert torch.equal(d1, d2) and torch.equal(F1, F2)
    assert i1["iters"] == i2["iters"] and i1["rel_residual"] == i2["rel_residual"]


def test_sr_fp32_s_is_reported_not_exact():
    B, P = 300, 200
    O, E = _rand(B, P, 11)
    ref = R.sr_solve(O.astype(np.float64), E, 1e-4)
    d, _, _ = V.vqmc_sr_solve(to_dev(O), to_dev(E), V.SrOpts(method=V.SR_CHOLESKY, s_prec=0))
    err = _rel(host(d), ref["delta"])
    print("FP32-accumulated S: delta rel err %.3e" % err)
    assert err < 1e-2


def test_sr_pipeline_10x10_against_oracle():
    """O and E_loc from the GPU library at 10x10 (B = 256), then SR with
    eps = 1e-4 by every solver, against the oracle's exact solve of the same
    inputs."""
    gm, rm = models(10, 16, 6)
    th = to_dev(init_theta(16, 6, seed=0))
    s = to_dev(uniform_sz0(10, 256, seed=1))
    announce("sr pipeline 10x10")
    O = V.vqmc_log_derivs(gm, th, s)
    E = V.vqmc_local_energy(gm, th, s)
    ref = R.sr_solve(host(O).astype(np.float64), host(E), 1e-4)
    for method in (V.SR_CHOLESKY, V.SR_DUAL):
        d, F, info = V.vqmc_sr_solve(O, E, V.SrOpts(method=method))
        e = _rel(host(d), ref["delta"])
        print("method %d delta rel %.3e" % (method, e))
        assert e <= 1e-6
        assert _rel(host(F), ref["F"]) <= 1e-10
    d, F, info = V.vqmc_sr_solve(O, E, V.SrOpts(method=V.SR_CG, tol=1e-10, max_iter=5000))
    print("CG: iters %d rel res %.3e delta rel %.3e" % (info["iters"], info["rel_residual"],
                                                        _rel(host(d), ref["delta"])))
    assert info["converged"]
    assert _rel(host(d), ref["delta"]) <= 1e-4


def test_sr_cg_capped_reports_not_converged():
    O, E = _rand(128, 300, 5)
    d, F, info = V.vqmc_sr_solve(to_dev(O), to_dev(E), V.SrOpts(method=V.SR_CG, eps=1e-6,
                                                              tol=1e-14, max_iter=3))
    assert info["iters"] == 3 and not info["converged"]
    # three CG steps from x0 = 0: the residual must have dropped
    assert info["rel_residual"] < 1.0


def test_sr_residual_full_size_10x10():
    """The explicit-S Cholesky at the full 10x10 size (B = 4096, P = 14080):
    the residual ||(S + eps I) delta - F|| / ||F|| computed on the host in
    FP64 from the same O (S applied matrix-free)."""
    B, P = 4096, 14080
    rng = np.random.default_rng(3)
    O = (rng.standard_normal((B, P)) * 0.1).astype(np.float32)
    O[:, :50] += rng.standard_normal((B, 1)).astype(np.float32)  # correlated block
    E = rng.standard_normal(B) - 50
    announce("sr full size")
    Od = to_dev(O)
    for method in (V.SR_CHOLESKY, V.SR_DUAL):
        d, F, info = V.vqmc_sr_solve(Od, to_dev(E), V.SrOpts(method=method, eps=1e-4))
        d, F = host(d), host(F)
        O64 = O.astype(np.float64)
        Oc = O64 - O64.mean(axis=0)
        res = Oc.T @ (Oc @ d) / B + 1e-4 * d - F
        rr = np.linalg.norm(res) / np.linalg.norm(F)
        print("method %d full-size residual %.3e" % (method, rr))
        assert rr <= 1e-8
