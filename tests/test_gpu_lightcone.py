"""GPU parity of the light-cone local energy (incremental evaluation of every
exchanged configuration) against the FP64 oracle, through the C ABI."""
import json
import os

import numpy as np
import pytest
import torch

from gpu_common import R, V, models, to_dev, host, announce
from vqmc_inputs import init_theta, neel, uniform_sz0, ferro_like_sz0

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "oracle_large.json")


def _lc(L, C, n, prec, **kw):
    gm, rm = models(L, C, n, prec, **kw)
    return gm.with_eloc(V.ELOC_LIGHTCONE), rm


def _check(gm, rm, th, s, tol_mean, tol_each=None):
    ref = R.local_energy(rm, th, s)
    flags = torch.full((s.shape[0],), -1, dtype=torch.int32, device="cuda")
    announce("lightcone", gm, s.shape[0])
    got = host(V.vqmc_local_energy(gm, to_dev(th), to_dev(s), flags=flags))
    assert (host(flags) == 0).all()
    rel_mean = abs(got.mean() - ref.mean()) / abs(ref.mean())
    rel_each = np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)
    print("LC L=%d prec=%d |dE/N| rel %.3e max per-sample %.3e" % (gm.L, gm.prec, rel_mean, rel_each.max()))
    assert rel_mean <= tol_mean
    if tol_each is not None:
        assert rel_each.max() <= tol_each
    return got


# batch-mean bar |dE/N| and per-sample bound, per precision of the
# difference convolutions (FP32: the FP32 tolerance of the dense path;
# split-BF16: the 1e-4 energy bar)
TOL = {V.PREC_FP32: (1e-5, 1e-4), V.PREC_BF16X3: (1e-4, 1e-3)}


# (14, 32, 5) and (18, 16, 3) use the twelve-wave shapes (2 and 3 row tiles
# per wave) with an odd depth, where the next configuration's lift waits for a
# barrier of its own; (16, 32, 8) (every precision) and (16, 16, 8) (FP32) an
# even depth at which two exchanged configurations share the first three
# layer steps
@pytest.mark.parametrize("L,C,n,B", [(6, 16, 2, 9), (8, 16, 3, 7), (10, 16, 6, 12), (12, 32, 4, 5),
                                     (14, 32, 5, 2), (18, 16, 3, 3), (16, 32, 8, 3), (16, 16, 8, 3)])
@pytest.mark.parametrize("prec", [V.PREC_FP32, V.PREC_BF16X3])
def test_lightcone_parity(L, C, n, B, prec):
    gm, rm = _lc(L, C, n, prec)
    th = init_theta(C, n, seed=0)
    _check(gm, rm, th, uniform_sz0(L, B, seed=1), *TOL[prec])


@pytest.mark.parametrize("L,C,n,B", [(10, 16, 6, 12), (16, 32, 8, 3)])
def test_lightcone_single_bf16_is_bounded(L, C, n, B):
    gm, rm = _lc(L, C, n, V.PREC_BF16)
    th = init_theta(C, n, seed=0)
    _check(gm, rm, th, uniform_sz0(L, B, seed=1), 1e-2)


def test_lightcone_edge_configs_and_couplings():
    th = init_theta(16, 2, seed=4)
    s = np.concatenate([neel(8, 1), ferro_like_sz0(8), uniform_sz0(8, 3, seed=9)])
    for kw in ({}, {"J2": 0.0}, {"marshall": 0, "J1": 0.7, "J2": -0.3}):
        gm, rm = _lc(8, 16, 2, V.PREC_FP32, **kw)
        _check(gm, rm, th, s, 1e-5, 1e-4)


def test_lightcone_paired_edge_configs():
    # 16x16, n = 8: the paired form (two exchanged configurations per layer
    # step for layers 1 .. 3) on Neel (every J1 bond antiparallel: 512
    # exchanged configurations) and on a half-up / half-down configuration (96)
    L, C, n = 16, 32, 8
    th = init_theta(C, n, seed=4)
    s = np.concatenate([neel(L, 1), ferro_like_sz0(L)])
    for prec in (V.PREC_FP32, V.PREC_BF16X3):
        gm, rm = _lc(L, C, n, prec)
        _check(gm, rm, th, s, *TOL[prec])
    # all spins up: no exchanged configuration, the diagonal term alone (4N
    # bonds with s_i s_j = 1: N (2 J1 + 2 J2) / 4), flagged as Sz != 0
    gm, _ = _lc(L, C, n, V.PREC_FP32)
    flags = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    e = host(V.vqmc_local_energy(gm, to_dev(th), to_dev(np.ones((1, L * L), np.int8)), flags=flags))
    assert e[0] == L * L * (2 * 1.0 + 2 * 0.5) / 4
    assert host(flags)[0] == 2


def test_lightcone_matches_dense_and_zero_params():
    gm, _ = _lc(10, 16, 6, V.PREC_FP32)
    th = to_dev(init_theta(16, 6, seed=0))
    s = to_dev(uniform_sz0(10, 32, seed=3))
    a = host(V.vqmc_local_energy(gm, th, s))
    b = host(V.vqmc_local_energy(gm.with_eloc(V.ELOC_DENSE), th, s))
    # both are FP32 evaluations within 1e-4 of the oracle per sample
    np.testing.assert_allclose(a, b, rtol=3e-4)
    z = torch.zeros_like(th)
    e = host(V.vqmc_local_energy(gm, z, to_dev(neel(10, 2))))
    np.testing.assert_allclose(e / 100, -1.25, rtol=0, atol=1e-12)
    # run-to-run identical
    c = host(V.vqmc_local_energy(gm, th, s))
    assert (a == c).all()


@pytest.mark.parametrize("L", [16, 24])
@pytest.mark.parametrize("prec", [V.PREC_FP32, V.PREC_BF16X3])
def test_lightcone_large_lattices_against_stored_oracle(L, prec):
    g = {c["L"]: c for c in json.load(open(GOLD))["cases"]}[L]
    gm, _ = _lc(L, g["C"], g["n"], prec)
    s = uniform_sz0(L, g["n_samples"], seed=1)
    announce("lightcone large", L, prec)
    el = host(V.vqmc_local_energy(gm, to_dev(init_theta(g["C"], g["n"], seed=0)), to_dev(s)))
    ref = np.array(g["e_loc"])
    rel = abs(el.mean() - ref.mean()) / abs(ref.mean())
    print("LC L=%d prec=%d E rel %.3e per sample %s" % (L, prec, rel, np.abs(el - ref) / np.abs(ref)))
    assert rel <= 1e-5 if prec == V.PREC_FP32 else rel <= 1e-4
