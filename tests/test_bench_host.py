"""Host-side checks of bench.py's bookkeeping (no GPU): the FLOP and byte
counts the bench divides by its measured times, pinned to the values the
scope table of the method states and to brute force, and the refusal of more
than one GPU."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import bench  # noqa: E402
from vqmc_inputs import neel, uniform_sz0  # noqa: E402


@pytest.mark.parametrize("L,C,n,expect", [(4, 4, 2, 10_368), (10, 16, 6, 2_793_600), (16, 32, 8, 37_896_192),
                                          (24, 32, 8, 85_266_432)])
def test_forward_flops_per_configuration(L, C, n, expect):
    # dense forward of one configuration: 2 N 9 (C + n C^2) FLOPs (the lift
    # and n C -> C layers, 3x3 taps), at the four workloads
    assert bench.f_cfg(L, C, n) == expect


def _antiparallel_brute(s, L):
    """Per bond kind (right, below, lower-right, lower-left), the bonds whose
    two spins differ, by a loop over sites."""
    out = np.zeros((s.shape[0], 4), dtype=np.int64)
    for b in range(s.shape[0]):
        g = s[b].reshape(L, L)
        for y in range(L):
            for x in range(L):
                for k, (dy, dx) in enumerate(((0, 1), (1, 0), (1, 1), (1, -1))):
                    out[b, k] += g[y, x] != g[(y + dy) % L, (x + dx) % L]
    return out


@pytest.mark.parametrize("L", [4, 6, 10])
def test_antiparallel_counts_brute_force(L):
    s = uniform_sz0(L, 7, seed=5)
    np.testing.assert_array_equal(bench.antiparallel_counts(s, L), _antiparallel_brute(s, L))


def test_antiparallel_counts_neel_and_mean():
    # Neel: every J1 bond antiparallel, every J2 bond parallel
    L = 10
    c = bench.antiparallel_counts(neel(L, 3), L)
    np.testing.assert_array_equal(c, np.tile([L * L, L * L, 0, 0], (3, 1)))
    # uniform Sz = 0: each of the 4N bonds is antiparallel with probability
    # 2 (N/2)^2 / (N (N - 1)), so E[n_ap] = 2 N^2 / (N - 1) (202.02 at 10x10)
    N = L * L
    s = uniform_sz0(L, 4000, seed=11)
    m = bench.antiparallel_counts(s, L).sum(axis=1).mean()
    assert abs(m - 2 * N * N / (N - 1)) < 0.01 * 2 * N * N / (N - 1)


def test_local_energy_flops_dense_and_light_cone_limit():
    L, C, n = 4, 4, 2
    s = uniform_sz0(L, 5, seed=2)
    nap = bench.antiparallel_counts(s, L).sum(axis=1)
    f = bench.f_cfg(L, C, n)
    alg, _ = bench.eloc_flops(s, L, C, n, lightcone=False, conv="fp32")
    assert alg == float((1 + nap).sum()) * f
    # on 4x4 the box of every distance >= 2 covers the lattice, so the light
    # cone's layers each convolve all N rows for every exchanged pair: its
    # count is the dense one less the lift (2 N 9 C) per exchanged pair
    alg_lc, _ = bench.eloc_flops(s, L, C, n, lightcone=True, conv="fp32")
    assert alg_lc == pytest.approx(s.shape[0] * f + float(nap.sum()) * (f - 2 * L * L * 9 * C), rel=1e-15)


def test_local_energy_executed_flops_dense_10x10():
    # one Neel configuration at 10x10: 200 antiparallel J1 bonds, so 201
    # configurations.  FP32: 512-row batches of 5 (41 batches, 32 tiles
    # each, K = 144 plus the lift's 12).  BF16: 448-row batches of 4 (50 of
    # 400 rows, whose waves 1..3 skip their last tile: 25 tiles; the last
    # batch of 100 rows skips the last slot of every wave: 24 tiles), K
    # padded to 160, three products in split BF16
    s = neel(10, 1)
    tile = 16 * 16 * 2
    _, f32 = bench.eloc_flops(s, 10, 16, 6, lightcone=False, conv="fp32")
    assert f32 == 41 * 32 * tile * (6 * 144 + 12)
    _, x3 = bench.eloc_flops(s, 10, 16, 6, lightcone=False, conv="bf16x3")
    assert x3 == (50 * 25 + 24) * tile * 6 * 160 * 3
    _, b1 = bench.eloc_flops(s, 10, 16, 6, lightcone=False, conv="bf16")
    assert b1 == x3 / 3


def test_sr_stage_roofline_counts():
    # explicit S at 10x10: B P^2 (lower half of S) = 0.812 TFLOP and P^3 / 3
    # = 0.930 TFLOP for the Cholesky, plus the solves
    B, P = 4096, 14080
    r = bench.sr_stage_roofline("chol64", B, P, 1000.0, 0)
    assert r["flops"] == pytest.approx(B * P * P + P ** 3 / 3 + 2 * P * P)
    assert B * P * P / 1e12 == pytest.approx(0.812, abs=5e-4)
    assert P ** 3 / 3 / 1e12 == pytest.approx(0.930, abs=5e-4)
    assert r["achieved"] == pytest.approx(r["flops"] / 1e12) and r["bound"] == "mfma"
    # CG: two passes over the FP32 O per iteration
    c = bench.sr_stage_roofline("cg", 16384, 74304, 1000.0, 200)
    assert c["bound"] == "hbm" and c["achieved"] == pytest.approx(2 * 16384 * 74304 * 4 * 200 / 1e9)


def test_stored_traffic_lookup():
    d = bench.sources_digest("eloc_kernel")
    assert len(d) == 64 and all(ch in "0123456789abcdef" for ch in d)
    assert bench.stored_traffic("eloc_kernel", "no such workload") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
