"""GPU parity of the rotation-symmetrised amplitude (Eq. sym-ws) against the
FP64 oracle, through the C ABI: log|psi~|, the local energy (dense and light
cone), the log-derivatives and the sampler, plus the rotation invariance every
one of them has and the 4x4 enumeration identity of Eq. (sum-Es)."""
import numpy as np
import pytest
import torch

from gpu_common import R, V, models, to_dev, host, announce
from vqmc_inputs import init_theta, neel, uniform_sz0

pytestmark = pytest.mark.gpu

LP_TOL = {V.PREC_FP32: 2e-4, V.PREC_BF16X3: 5e-3}


def _rot(s, L, k=1):
    """T^k of a batch: (T S) at (y, x) is S at (x, L-1-y)."""
    a = s.reshape(-1, L, L)
    return np.ascontiguousarray(np.rot90(a, k, axes=(1, 2)).reshape(s.shape))


def test_rotation_convention_matches_oracle():
    # the helper's turn is the oracle's: log psi~ of a configuration equals
    # that of its turn, and the unsymmetrised value of T S is one of the four
    _, rm = models(6, 8, 2, symmetry=1)
    _, r0 = models(6, 8, 2)
    th = init_theta(8, 2, seed=4)
    s = uniform_sz0(6, 3, seed=2)
    a, _ = R.log_psi(rm, th, s)
    b, _ = R.log_psi(rm, th, _rot(s, 6))
    np.testing.assert_allclose(a, b, rtol=1e-13)
    parts = np.stack([R.log_psi(r0, th, _rot(s, 6, k))[0] for k in range(4)])
    np.testing.assert_allclose(a, np.log(np.exp(parts).sum(axis=0)), rtol=1e-12)


@pytest.mark.parametrize("L,C,n,B", [(4, 4, 2, 21), (6, 8, 2, 13), (10, 16, 6, 11), (16, 32, 8, 3)])
@pytest.mark.parametrize("prec", [V.PREC_FP32, V.PREC_BF16X3])
def test_sym_log_psi_parity(L, C, n, B, prec):
    if prec != V.PREC_FP32 and C % 8:
        pytest.skip("BF16 forms need C % 8 == 0")
    gm, rm = models(L, C, n, prec, symmetry=1)
    th = init_theta(C, n, seed=0)
    s = uniform_sz0(L, B, seed=1)
    ref, rsg = R.log_psi(rm, th, s)
    announce("sym log_psi", L, C, n, B, prec)
    sign = torch.empty(B, dtype=torch.int8, device="cuda")
    got = host(V.vqmc_log_psi(gm, to_dev(th), to_dev(s), sign=sign))
    err = np.abs(got - ref)
    print("sym log_psi L=%d prec=%d max|err|=%.3e" % (L, prec, err.max()))
    assert err.max() <= LP_TOL[prec]
    assert (host(sign) == rsg).all()


# every kernel shape: rotations in one pass (G >= 4), two passes (G = 2) and
# one per pass (G = 1), for every convolution precision
MULTI = [(6, 4, 2, 9), (8, 8, 2, 9), (10, 16, 3, 7), (12, 32, 2, 5), (14, 32, 2, 3), (16, 16, 2, 3),
         (18, 32, 2, 2), (20, 16, 2, 2), (22, 16, 2, 2), (24, 32, 2, 2)]


@pytest.mark.parametrize("L,C,n,B", MULTI)
def test_sym_log_psi_is_logsumexp_of_rotated_calls(L, C, n, B):
    """log psi~ equals the logsumexp of the unsymmetrised call on the four
    turned batches, however many forward passes the kernel needs per
    configuration (the per-rotation values are the same arithmetic)."""
    th = to_dev(init_theta(C, n, seed=0))
    s = uniform_sz0(L, B, seed=1)
    for prec in (V.PREC_FP32, V.PREC_BF16, V.PREC_BF16X3):
        if prec != V.PREC_FP32 and C % 8:
            continue
        gm, _ = models(L, C, n, prec)
        announce("sym multipass", L, C, n, B, prec)
        got = host(V.vqmc_log_psi(gm.with_symmetry(1), th, to_dev(s)))
        parts = np.stack([host(V.vqmc_log_psi(gm, th, to_dev(_rot(s, L, k)))) for k in range(4)])
        mx = parts.max(axis=0)
        ref = mx + np.log(np.exp(parts - mx).sum(axis=0))
        assert np.isfinite(got).all()
        np.testing.assert_allclose(got, ref, rtol=1e-14, atol=1e-12)


def test_sym_log_psi_rotation_invariance_and_empty():
    gm, _ = models(10, 16, 6, symmetry=1)
    th = to_dev(init_theta(16, 6, seed=0))
    s = uniform_sz0(10, 19, seed=8)
    announce("sym log_psi invariance")
    base = host(V.vqmc_log_psi(gm, th, to_dev(s)))
    for k in (1, 2, 3):
        got = host(V.vqmc_log_psi(gm, th, to_dev(_rot(s, 10, k))))
        # the same four values in another order: rounding of the sum only
        np.testing.assert_allclose(got, base, rtol=1e-13)
    out = V.vqmc_log_psi(gm, th, torch.empty((0, 100), dtype=torch.int8, device="cuda"))
    assert out.numel() == 0


def _sym_eloc(L, C, n, B, prec, eloc, seed=1, tol_each=1e-4, tol_mean=1e-5):
    gm, rm = models(L, C, n, prec, symmetry=1, eloc=eloc)
    th = init_theta(C, n, seed=0)
    s = uniform_sz0(L, B, seed=seed)
    ref = R.local_energy(rm, th, s)
    announce("sym local_energy", L, C, n, B, prec, eloc)
    flags = torch.full((B,), -1, dtype=torch.int32, device="cuda")
    got = host(V.vqmc_local_energy(gm, to_dev(th), to_dev(s), flags=flags))
    assert (host(flags) == 0).all()
    rel_each = np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)
    rel_mean = abs(got.mean() - ref.mean()) / abs(ref.mean())
    print("sym E_loc L=%d prec=%d eloc=%d mean rel %.3e max rel %.3e" % (L, prec, eloc, rel_mean, rel_each.max()))
    assert rel_each.max() <= tol_each
    assert rel_mean <= tol_mean


@pytest.mark.parametrize("L,C,n,B", [(4, 4, 2, 17), (6, 8, 2, 9), (10, 16, 6, 5)])
def test_sym_local_energy_dense_fp32(L, C, n, B):
    _sym_eloc(L, C, n, B, V.PREC_FP32, V.ELOC_DENSE)


def test_sym_local_energy_dense_bf16x3():
    _sym_eloc(10, 16, 6, 5, V.PREC_BF16X3, V.ELOC_DENSE, tol_each=1e-3, tol_mean=1e-4)


@pytest.mark.parametrize("prec", [V.PREC_FP32, V.PREC_BF16X3])
def test_sym_local_energy_lightcone(prec):
    tol = (1e-4, 1e-5) if prec == V.PREC_FP32 else (1e-3, 1e-4)
    _sym_eloc(8, 16, 3, 6, prec, V.ELOC_LIGHTCONE, tol_each=tol[0], tol_mean=tol[1])


@pytest.mark.parametrize("prec", [V.PREC_FP32, V.PREC_BF16X3])
def test_sym_local_energy_lightcone_16x16(prec):
    # 16x16, C = 32, eight layers: the form of the light cone in which two
    # exchanged configurations share the first three layer steps, here over
    # the four rotations of each configuration (FP32 bars scaled by
    # sqrt(N C) as for the unsymmetrised 16x16 energies)
    tol = (1e-4, 5e-5) if prec == V.PREC_FP32 else (1e-3, 1e-4)
    _sym_eloc(16, 32, 8, 2, prec, V.ELOC_LIGHTCONE, tol_each=tol[0], tol_mean=tol[1])


def test_sym_local_energy_lightcone_vs_dense_16x16():
    """Both GPU methods at 16x16, C = 32, eight layers on three more
    configurations, and the rotation invariance of each."""
    th = to_dev(init_theta(32, 8, seed=0))
    s = uniform_sz0(16, 3, seed=3)
    res = {}
    for eloc in (V.ELOC_DENSE, V.ELOC_LIGHTCONE):
        gm, _ = models(16, 32, 8, symmetry=1, eloc=eloc)
        announce("sym 16x16", eloc)
        res[eloc] = host(V.vqmc_local_energy(gm, th, to_dev(s)))
        rot = host(V.vqmc_local_energy(gm, th, to_dev(_rot(s, 16))))
        np.testing.assert_allclose(rot, res[eloc], rtol=1e-12)
    rel = np.abs(res[V.ELOC_DENSE] - res[V.ELOC_LIGHTCONE]) / np.abs(res[V.ELOC_DENSE])
    print("sym 16x16 dense vs light cone max rel %.3e" % rel.max())
    assert rel.max() <= 1e-4


def test_sym_local_energy_flags():
    gm, _ = models(6, 8, 2, symmetry=1, eloc=V.ELOC_DENSE)
    th = to_dev(init_theta(8, 2, seed=0))
    s = uniform_sz0(6, 3, seed=1)
    s[1, 0] = -s[1, 0]          # Sz != 0
    s[2, 5] = 0                 # not a spin value
    flags = torch.full((3,), -1, dtype=torch.int32, device="cuda")
    announce("sym flags")
    V.vqmc_local_energy(gm, th, to_dev(s), flags=flags)
    f = host(flags)
    assert f[0] == 0 and f[1] & 2 and f[2] & 4


def test_sym_enumeration_identity_4x4():
    """sum_s |psi~|^2 E_s / sum_s |psi~|^2 = <psi~|H|psi~> over the 12870
    Sz = 0 states, with the GPU's log|psi~|, sign and E_s and the oracle's H."""
    gm, rm = models(4, 4, 2, symmetry=1)
    th = init_theta(4, 2, seed=0)
    H, states = R.hamiltonian(4, 1.0, 0.5)
    announce("sym enumeration 4x4")
    sd = to_dev(states)
    sign = torch.empty(states.shape[0], dtype=torch.int8, device="cuda")
    la = host(V.vqmc_log_psi(gm, to_dev(th), sd, sign=sign))
    el = host(V.vqmc_local_energy(gm, to_dev(th), sd))
    w = np.exp(2 * (la - la.max()))
    lhs = (w * el).sum() / w.sum()
    assert lhs == pytest.approx(R.exact_energy(H, la, host(sign)), rel=1e-9)
    assert lhs == pytest.approx(R.exact_energy(H, *R.log_psi(rm, th, states)), rel=1e-6)


@pytest.mark.parametrize("L,C,n,B", [(4, 4, 2, 9), (6, 8, 2, 7), (10, 16, 6, 5)])
def test_sym_log_derivs(L, C, n, B):
    gm, rm = models(L, C, n, symmetry=1)
    th = init_theta(C, n, seed=0)
    s = uniform_sz0(L, B, seed=2)
    ref = R.log_derivs(rm, th, s)
    announce("sym log_derivs", L, C, n, B)
    O = host(V.vqmc_log_derivs(gm, to_dev(th), to_dev(s)))
    err = np.linalg.norm(O - ref) / np.linalg.norm(ref)
    row = (np.linalg.norm(O - ref, axis=1) / np.linalg.norm(ref, axis=1)).max()
    print("sym O L=%d Frobenius rel %.3e worst row %.3e" % (L, err, row))
    assert err <= 1e-5 and row <= 2e-5
    rot = host(V.vqmc_log_derivs(gm, to_dev(th), to_dev(_rot(s, L, 3))))
    assert np.linalg.norm(rot - O) / np.linalg.norm(O) <= 2e-6


def test_sym_log_derivs_strided_rows_and_batch_above_grid():
    """ldO > P and more samples than workgroups: rows accumulate in place
    without touching the padding."""
    L, C, n = 4, 4, 2
    gm, rm = models(L, C, n, symmetry=1)
    P = V.num_params(gm)
    th = init_theta(C, n, seed=1)
    B = 2100
    s = uniform_sz0(L, B, seed=4)
    pick = np.array([0, 1, 1000, 2047, 2048, 2099])
    ref = R.log_derivs(rm, th, s[pick])
    O = torch.full((B, P + 7), 7.0, dtype=torch.float32, device="cuda")
    announce("sym log_derivs strided")
    V.vqmc_log_derivs(gm, to_dev(th), to_dev(s), O=O[:, :P])
    Oh = host(O)
    assert (Oh[:, P:] == 7.0).all()
    err = np.linalg.norm(Oh[pick, :P] - ref) / np.linalg.norm(ref)
    assert err <= 1e-5


def test_sym_sampler_trajectories_match_oracle():
    cases = [(4, 4, 2, 128, 2, 0, neel), (6, 8, 2, 32, 1, 1, uniform_sz0), (10, 16, 6, 12, 1, 0, neel)]
    for L, C, n, B, sweeps, prop, init in cases:
        gm, rm = models(L, C, n, symmetry=1)
        th = init_theta(C, n, seed=1)
        s0 = init(L, B) if init is neel else init(L, B, seed=5)
        rs, rla, rna, margin = R.sample(rm, th, s0, n_sweeps=sweeps, seed=11, proposal=prop)
        announce("sym sampler", L, C, n, B, prop)
        sd = to_dev(s0)
        lp = torch.empty(B, dtype=torch.float64, device="cuda")
        na = torch.empty(B, dtype=torch.int32, device="cuda")
        V.vqmc_sample(gm, to_dev(th), sd, n_sweeps=sweeps, seed=11, proposal=prop, log_psi=lp, n_accepted=na)
        gs, gla, gna = host(sd), host(lp), host(na)
        clear = margin > 1e-3
        print("sym sampler L=%d chains compared %d / %d" % (L, clear.sum(), B))
        assert clear.sum() >= 0.8 * B
        assert (gs[clear] == rs[clear]).all()
        assert (gna[clear] == rna[clear]).all()
        np.testing.assert_allclose(gla[clear], rla[clear], atol=2e-4)
        # the returned log psi~ is that of the final configuration
        np.testing.assert_allclose(gla, host(V.vqmc_log_psi(gm, to_dev(th), sd)), atol=1e-9)
