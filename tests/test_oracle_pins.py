"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Every check here compares the oracle with something other than itself:
printed or textbook values, closed forms, invariants, library routines
(scipy eigsh, torch conv2d/autograd, numpy cov/solve) and brute force over all
12870 Sz = 0 states of the 4x4 lattice.  None of these tests touches a GPU.
"""
import math
import os
from itertools import combinations

import numpy as np
import pytest

import oracle as R
from sampler_stats import check_histogram
from vqmc_inputs import init_theta, neel, uniform_sz0, ferro_like_sz0

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    out = {}
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


M4 = R.RefModel(4, 4, 2, 1.0, 0.5, 1)


@pytest.fixture(scope="module")
def ham4():
    H, states = R.hamiltonian(4, 1.0, 0.5)
    return H, states


@pytest.fixture(scope="module")
def theta4():
    return init_theta(4, 2, seed=0).astype(np.float64)


@pytest.fixture(scope="module")
def enum4(ham4, theta4):
    """log|psi|, sign, E_loc of every Sz = 0 state of the 4x4 lattice."""
    H, states = ham4
    la, sg = R.log_psi(M4, theta4, states)
    el = R.local_energy(M4, theta4, states)
    return la, sg, el


# ---------------------------------------------------------------- Philox

def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLD, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = R.philox4x32_10(v[0:4], v[4:6])
        assert list(out) == v[6:10]


# ------------------------------------------------------------ Hamiltonian

def test_bond_count_and_parameter_counts():
    # 4N bonds (Sec. 3.1: half of the four J1 and four J2 bonds per site)
    for L in (4, 6, 10):
        assert len(R.bond_pairs(L, 1.0, 0.5)) == 4 * L * L
    # conv-only model: (9C + C) + n (9C^2 + C)
    assert R.num_params(R.RefModel(4, 4, 2)) == 336
    assert R.num_params(R.RefModel(10, 16, 6)) == 14080
    assert R.num_params(R.RefModel(16, 32, 8)) == 74304
    assert R.num_params(R.RefModel(24, 32, 8)) == 74304


def test_hamiltonian_hermitian_and_trace(ham4):
    H, states = ham4
    assert states.shape == (math.comb(16, 8), 16)
    assert abs(H - H.T).max() == 0.0
    # Tr over Sz = 0: every bond has <s_i s_j> = -1/(N-1) over the sector
    N = 16
    sumJ4 = (2 * N * 1.0 + 2 * N * 0.5) / 4.0
    assert H.diagonal().sum() == pytest.approx(math.comb(N, N // 2) * sumJ4 * (-1.0 / (N - 1)),
                                               abs=1e-9)


def test_hamiltonian_su2(ham4):
    """[H, S^2] = 0 on the Sz = 0 sector (H is SU(2) invariant)."""
    import scipy.sparse as sp
    H, states = ham4
    N = 16
    # S^2 = 3N/4 + 2 sum_{i<j} S_i.S_j with S_i.S_j = (1/4) sigma_i.sigma_j
    allpairs = combinations(range(N), 2)
    masks = ((states > 0).astype(np.int64) << np.arange(N)).sum(axis=1)
    index = -np.ones(1 << N, dtype=np.int64)
    index[masks] = np.arange(states.shape[0])
    M = states.shape[0]
    diag = np.full(M, 0.75 * N)
    rows, cols, vals = [], [], []
    for i, j in allpairs:
        diag += 2 * 0.25 * states[:, i] * states[:, j]
        anti = np.nonzero(states[:, i] != states[:, j])[0]
        rows.append(index[masks[anti] ^ (1 << i) ^ (1 << j)])
        cols.append(anti)
        vals.append(np.full(anti.size, 2 * 0.5))
    S2 = sp.csr_matrix((np.concatenate(vals + [diag]),
                        (np.concatenate(rows + [np.arange(M)]), np.concatenate(cols + [np.arange(M)]))),
                       shape=(M, M))
    comm = H @ S2 - S2 @ H
    assert abs(comm).max() < 1e-10


def test_ground_energy_textbook_and_marshall():
    g = _gold("heisenberg_4x4.txt")
    H0, states = R.hamiltonian(4, 1.0, 0.0)
    e0 = R.ground_energy(H0)[0]
    assert e0 / 16 == pytest.approx(g["e0_per_site_J2_0"], abs=2e-7)
    # at J2 = 0 the ground state obeys the Marshall sign rule exactly
    from scipy.sparse.linalg import eigsh
    w, v = eigsh(H0, k=1, which="SA", tol=1e-12)
    y, x = np.divmod(np.arange(16), 4)
    a = ((x + y) % 2 == 0)
    sign = np.where((states[:, a] > 0).sum(axis=1) % 2 == 1, -1.0, 1.0)
    rot = v[:, 0] * sign
    assert (rot > 0).all() or (rot < 0).all()


def test_neel_diagonal_energy(ham4):
    g = _gold("heisenberg_4x4.txt")
    H, states = ham4
    s = neel(4, 1)[0]
    k = np.nonzero((states == s).all(axis=1))[0][0]
    assert H[k, k] / 16 == pytest.approx(g["neel_diag_per_site_J2_05"], abs=1e-15)


# ------------------------------------------------------------ amplitude

def test_log_psi_matches_torch_circular_conv():
    torch = pytest.importorskip("torch")
    import torch.nn.functional as F
    for (L, C, n) in ((4, 4, 2), (6, 8, 3)):
        m = R.RefModel(L, C, n)
        th = init_theta(C, n, seed=3).astype(np.float64)
        s = uniform_sz0(L, 5, seed=4)
        la, _ = R.log_psi(m, th, s)
        h = torch.tensor(s, dtype=torch.float64).reshape(-1, 1, L, L)
        off = 0
        for l in range(n + 1):
            cin = 1 if l == 0 else C
            W = torch.tensor(th[off: off + C * cin * 9]).reshape(C, cin, 3, 3)
            off += C * cin * 9
            b = torch.tensor(th[off: off + C])
            off += C
            h = torch.tanh(F.conv2d(F.pad(h, (1, 1, 1, 1), mode="circular"), W, b))
        ref = h.sum(dim=(1, 2, 3)).numpy()
        np.testing.assert_allclose(la, ref, rtol=1e-13, atol=1e-12)


def test_log_psi_translation_invariance_and_sign():
    m = R.RefModel(6, 4, 2)
    th = init_theta(4, 2, seed=5).astype(np.float64)
    s = uniform_sz0(6, 3, seed=6)
    base, sg = R.log_psi(m, th, s)
    grid = s.reshape(3, 6, 6)
    for dy, dx in ((0, 1), (1, 0), (2, 3), (5, 5)):
        sh = np.roll(grid, (dy, dx), axis=(1, 2)).reshape(3, 36)
        la, sg2 = R.log_psi(m, th, sh)
        np.testing.assert_allclose(la, base, rtol=1e-13)
        # the Marshall sign flips with an odd shift (sublattices exchange) only
        # by (-1)^{N/2} relative factors; it is a pure function of the spins:
        y, x = np.divmod(np.arange(36), 6)
        a = ((x + y) % 2 == 0)
        expect = np.where((sh[:, a] > 0).sum(axis=1) % 2 == 1, -1, 1)
        assert (sg2 == expect).all()


def test_zero_bias_makes_log_psi_odd():
    m = R.RefModel(4, 4, 2)
    th = init_theta(4, 2, seed=7, zero_bias=True).astype(np.float64)
    s = uniform_sz0(4, 4, seed=8)
    a, _ = R.log_psi(m, th, s)
    b, _ = R.log_psi(m, th, -s)
    np.testing.assert_allclose(a, -b, rtol=1e-13, atol=1e-13)


# --------------------------------------------------------- local energy

def test_local_energy_enumeration_identity(ham4, enum4):
    """sum_s |psi|^2 E_loc(s) = <psi|H|psi> over all 12870 states (Eq. sum-Es)."""
    H, states = ham4
    la, sg, el = enum4
    w = np.exp(2 * (la - la.max()))
    lhs = (w * el).sum() / w.sum()
    rhs = R.exact_energy(H, la, sg)
    assert lhs == pytest.approx(rhs, rel=1e-12)
    # variational bound
    assert rhs >= R.ground_energy(H)[0] - 1e-10
    # and pointwise: E_loc(s) = (H psi)(s) / psi(s)
    psi = sg * np.exp(la - la.max())
    np.testing.assert_allclose(el, (H @ psi) / psi, rtol=1e-11, atol=1e-11)


def test_local_energy_constant_psi_neel():
    """All parameters zero: W = 1, so E_loc(Neel) = -N/4 (diagonal) - N
    (2N J1 exchanges of amplitude -1/2 under the Marshall sign) = -1.25 N."""
    for L in (4, 6, 10):
        m = R.RefModel(L, 4, 1)
        th = np.zeros(R.num_params(m))
        e = R.local_energy(m, th, neel(L, 1))
        assert e[0] / (L * L) == pytest.approx(-1.25, abs=1e-14)


def test_local_energy_translation_and_flags():
    m = R.RefModel(6, 4, 2)
    th = init_theta(4, 2, seed=9).astype(np.float64)
    s = uniform_sz0(6, 2, seed=10)
    e0, f0 = R.local_energy(m, th, s, with_flags=True)
    assert (f0 == 0).all()
    sh = np.roll(s.reshape(2, 6, 6), (1, 2), axis=(1, 2)).reshape(2, 36)
    np.testing.assert_allclose(R.local_energy(m, th, sh), e0, rtol=1e-12)
    bad = s.copy()
    bad[1, 3] = 0
    _, f = R.local_energy(m, th, bad, with_flags=True)
    assert f[1] & 4
    # a configuration with more up than down spins
    up = s[:1].copy()
    up[0, np.nonzero(up[0] < 0)[0][0]] = 1
    _, f = R.local_energy(m, th, up, with_flags=True)
    assert f[0] & 2


def test_local_energy_few_antiparallel_bonds():
    m = R.RefModel(4, 4, 2)
    th = init_theta(4, 2, seed=0).astype(np.float64)
    H, states = R.hamiltonian(4, 1.0, 0.5)
    s = ferro_like_sz0(4)
    la, sg = R.log_psi(m, th, states)
    psi = sg * np.exp(la - la.max())
    k = np.nonzero((states == s[0]).all(axis=1))[0][0]
    e = R.local_energy(m, th, s)
    assert e[0] == pytest.approx((H @ psi)[k] / psi[k], rel=1e-11)


# ------------------------------------------------------ log-derivatives

def test_log_derivs_central_fd():
    m = R.RefModel(4, 4, 2)
    th = init_theta(4, 2, seed=11).astype(np.float64)
    s = uniform_sz0(4, 6, seed=12)
    O = R.log_derivs(m, th, s)
    rng = np.random.default_rng(13)
    h = 1e-6
    for k in rng.choice(th.size, 40, replace=False):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (R.log_psi(m, tp, s)[0] - R.log_psi(m, tm, s)[0]) / (2 * h)
        np.testing.assert_allclose(O[:, k], fd, rtol=1e-6, atol=1e-8)


def test_log_derivs_torch_autograd_and_translation():
    torch = pytest.importorskip("torch")
    import torch.nn.functional as F
    L, C, n = 6, 8, 2
    m = R.RefModel(L, C, n)
    th = init_theta(C, n, seed=14).astype(np.float64)
    s = uniform_sz0(L, 3, seed=15)
    O = R.log_derivs(m, th, s)
    for b in range(3):
        t = torch.tensor(th, requires_grad=True)
        h = torch.tensor(s[b], dtype=torch.float64).reshape(1, 1, L, L)
        off = 0
        for l in range(n + 1):
            cin = 1 if l == 0 else C
            W = t[off: off + C * cin * 9].reshape(C, cin, 3, 3)
            off += C * cin * 9
            bb = t[off: off + C]
            off += C
            h = torch.tanh(F.conv2d(F.pad(h, (1, 1, 1, 1), mode="circular"), W, bb))
        h.sum().backward()
        np.testing.assert_allclose(O[b], t.grad.numpy(), rtol=1e-11, atol=1e-12)
    sh = np.roll(s.reshape(3, L, L), (2, 1), axis=(1, 2)).reshape(3, L * L)
    np.testing.assert_allclose(R.log_derivs(m, th, sh), O, rtol=1e-10, atol=1e-12)


# ----------------------------------------------------------------- SR

def _rand_OE(B, P, seed):
    rng = np.random.default_rng(seed)
    O = rng.standard_normal((B, P)) + 0.3 * rng.standard_normal(P)
    E = rng.standard_normal(B) * 2 - 5
    return O, E


def test_sr_against_numpy_cov_and_solve():
    for B, P in ((40, 12), (12, 40)):
        O, E = _rand_OE(B, P, B * 100 + P)
        eps = 1e-3
        r0 = R.sr_solve(O, E, eps, method=0)
        r1 = R.sr_solve(O, E, eps, method=1)
        cov = np.cov(np.concatenate([O, E[:, None]], axis=1).T, bias=True)
        S, F = cov[:P, :P], cov[:P, P]
        np.testing.assert_allclose(r0["F"], F, rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(R.sr_matrix(O), S, rtol=1e-12, atol=1e-13)
        d = np.linalg.solve(S + eps * np.eye(P), F)
        np.testing.assert_allclose(r0["delta"], d, rtol=1e-9, atol=1e-11)
        np.testing.assert_allclose(r1["delta"], d, rtol=1e-9, atol=1e-11)
        assert r0["e_mean"] == pytest.approx(E.mean(), rel=1e-14)
        assert r0["e_var"] == pytest.approx(E.var(), rel=1e-12)
        # the matrix-free application (S + eps I) v against numpy's covariance
        v = np.random.default_rng(B + P).standard_normal(P)
        np.testing.assert_allclose(R.sr_apply(O, O.mean(axis=0), v, eps), (S + eps * np.eye(P)) @ v,
                                   rtol=1e-12, atol=1e-13)


def test_sr_special_cases():
    O, E = _rand_OE(30, 8, 1)
    # constant energies: no gradient, no update
    r = R.sr_solve(O, np.full(30, -3.0), 1e-4, method=0)
    assert np.abs(r["F"]).max() < 1e-14 and np.abs(r["delta"]).max() < 1e-12
    # a column equal to E: F_k = Var(E)
    O2 = O.copy()
    O2[:, 3] = E
    r = R.sr_solve(O2, E, 1e-4, method=0)
    assert r["F"][3] == pytest.approx(E.var(), rel=1e-12)
    # huge shift: delta -> F / eps
    # (first correction is -S F / eps^2, relative size ||S|| / eps)
    r = R.sr_solve(O, E, 1e6, method=0)
    assert np.linalg.norm(r["delta"] - r["F"] / 1e6) / np.linalg.norm(r["F"] / 1e6) < 1e-5
    # residual of the solve
    r = R.sr_solve(O, E, 1e-4, method=1)
    S = np.cov(O.T, bias=True)
    res = (S + 1e-4 * np.eye(8)) @ r["delta"] - r["F"]
    assert np.linalg.norm(res) / np.linalg.norm(r["F"]) < 1e-10


def test_sr_rank_deficient_primal_equals_dual():
    """P > B: S has rank <= B - 1, the shift keeps the system SPD."""
    O, E = _rand_OE(16, 60, 2)
    S = R.sr_matrix(O)
    w = np.linalg.eigvalsh(S)
    assert (w > -1e-12).all() and (w > 1e-10).sum() <= 15
    r0 = R.sr_solve(O, E, 1e-4, method=0)
    r1 = R.sr_solve(O, E, 1e-4, method=1)
    np.testing.assert_allclose(r0["delta"], r1["delta"], rtol=1e-8,
                               atol=1e-10 * np.abs(r1["delta"]).max())


def test_gradient_is_half_energy_derivative(ham4, theta4, enum4):
    """With |psi|^2 weights over all states, F = <O E> - <O><E> (Eq. Es-Os-G)
    equals half the derivative of the exact energy <psi|H|psi>/<psi|psi>."""
    H, states = ham4
    la, sg, el = enum4
    O = R.log_derivs(M4, theta4, states)
    p = np.exp(2 * (la - la.max()))
    p /= p.sum()
    F = (p[:, None] * O * el[:, None]).sum(0) - (p[:, None] * O).sum(0) * (p * el).sum()
    h = 1e-5
    rng = np.random.default_rng(16)
    for k in rng.choice(theta4.size, 12, replace=False):
        tp, tm = theta4.copy(), theta4.copy()
        tp[k] += h
        tm[k] -= h
        ep = R.exact_energy(H, *R.log_psi(M4, tp, states))
        em = R.exact_energy(H, *R.log_psi(M4, tm, states))
        assert 2 * F[k] == pytest.approx((ep - em) / (2 * h), rel=1e-5, abs=1e-8)


# ------------------------------------------------------------- sampler

def _stag(states, L):
    y, x = np.divmod(np.arange(L * L), L)
    sgn = np.where((x + y) % 2 == 0, 1, -1)
    return np.abs((states * sgn).sum(axis=1)) // 2


@pytest.mark.parametrize("proposal", [0, 1])
def test_sampler_distribution_4x4(ham4, theta4, enum4, proposal):
    """Brute force: independent chains sample |psi|^2 over all 12870 states
    (the histogram over every state, equal-mass bins and a random partition
    of the states), the histogram of |staggered magnetisation|, and the mean
    local energy against the exact <H>.  The same samples must fail against
    |psi|^1 (the acceptance ratio W'/W instead of (W'/W)^2 of Sec. 3.1), so
    the checks can tell the two apart."""
    H, states = ham4
    la, sg, el = enum4
    chains = 8192
    s, lab, nacc, _ = R.sample(M4, theta4, neel(4, chains), n_sweeps=80, seed=1234,
                               proposal=proposal)
    assert (s.sum(axis=1) == 0).all()
    np.testing.assert_allclose(lab, R.log_psi(M4, theta4, s)[0], rtol=1e-12)
    assert (nacc > 0).all()
    p = np.exp(2 * (la - la.max()))
    p /= p.sum()
    stats = check_histogram(s, states, p)
    print(stats)
    p1 = np.exp(la - la.max())
    with pytest.raises(AssertionError):
        check_histogram(s, states, p1 / p1.sum())
    ms = _stag(states, 4)
    hist = np.bincount(_stag(s, 4), minlength=9)[:9]
    exp = np.array([p[ms == k].sum() for k in range(9)]) * chains
    keep = exp > 5
    chi2 = (((hist[keep] - exp[keep]) ** 2) / exp[keep]).sum()
    assert chi2 < 3 * keep.sum() + 20, (hist, exp)
    e_exact = (p * el).sum()
    e_s = R.local_energy(M4, theta4, s)
    se = e_s.std() / math.sqrt(chains)
    assert abs(e_s.mean() - e_exact) < 5 * se


def test_sampler_reproducible_and_counter_split(theta4):
    s0 = neel(4, 8)
    a = R.sample(M4, theta4, s0, n_sweeps=3, seed=7)
    b = R.sample(M4, theta4, s0, n_sweeps=3, seed=7)
    assert (a[0] == b[0]).all()
    # three sweeps at once == one sweep then two with the counter advanced
    c1 = R.sample(M4, theta4, s0, n_sweeps=1, seed=7)
    c2 = R.sample(M4, theta4, c1[0], n_sweeps=2, seed=7, counter_base=16)
    assert (c2[0] == a[0]).all()
    assert ((c1[2] + c2[2]) == a[2]).all()


# ------------------------------------- rotation-symmetrised amplitude

M4S = R.RefModel(4, 4, 2, 1.0, 0.5, 1, 1)


def _rot(states, L, k):
    """numpy's quarter turn of each L x L configuration (k times)."""
    return np.rot90(states.reshape(-1, L, L), k, axes=(1, 2)).reshape(len(states), L * L)


def test_symmetrised_amplitude_definition_and_invariance():
    """Eq. (sym-ws): log|sum_i W(T^i S)| equals the same sum formed here from
    the oracle's own unsymmetrised amplitudes of numpy-rotated
    configurations; it is invariant under the rotation, and for even L the
    four Marshall signs agree (so the sum never cancels)."""
    for L, C, n in ((4, 4, 2), (6, 4, 2), (8, 8, 1)):
        m0 = R.RefModel(L, C, n)
        ms = R.RefModel(L, C, n, 1.0, 0.5, 1, 1)
        th = init_theta(C, n, seed=21).astype(np.float64)
        s = uniform_sz0(L, 5, seed=22)
        la, sg = R.log_psi(ms, th, s)
        parts = [R.log_psi(m0, th, _rot(s, L, k)) for k in range(4)]
        sgs = np.stack([p[1] for p in parts])
        assert (sgs == sgs[0]).all() and (sg == sgs[0]).all()
        lg = np.stack([p[0] for p in parts])
        mx = lg.max(axis=0)
        np.testing.assert_allclose(la, mx + np.log(np.exp(lg - mx).sum(axis=0)), rtol=1e-13)
        for k in (1, 2, 3):
            np.testing.assert_allclose(R.log_psi(ms, th, _rot(s, L, k))[0], la, rtol=1e-13)


def _rotation_invariant_theta(C, n, seed):
    """Every 3x3 kernel averaged over its four quarter turns: then
    W_CNN(T S) = W_CNN(S) for every S."""
    th = init_theta(C, n, seed=seed).astype(np.float64)
    off = 0
    for l in range(n + 1):
        cin = 1 if l == 0 else C
        W = th[off:off + C * cin * 9].reshape(C, cin, 3, 3)
        W[:] = sum(np.rot90(W, k, axes=(2, 3)) for k in range(4)) / 4
        off += C * cin * 9 + C
    return th


def test_symmetrised_closed_form_for_invariant_network():
    """With rotation-invariant kernels the four terms are equal: log|W~| =
    log W_CNN + log 4 and the local energy is that of the unsymmetrised
    amplitude.  The log-derivatives are not: turning the input is turning
    every kernel, so d/dW of the rotated term is the turned gradient, and
    the symmetrised O is the unsymmetrised one averaged over the four quarter
    turns of each 3x3 kernel gradient (biases unchanged)."""
    L, C, n = 6, 4, 2
    m0, ms = R.RefModel(L, C, n), R.RefModel(L, C, n, 1.0, 0.5, 1, 1)
    th = _rotation_invariant_theta(C, n, 23)
    s = uniform_sz0(L, 4, seed=24)
    np.testing.assert_allclose(R.log_psi(ms, th, s)[0], R.log_psi(m0, th, s)[0] + math.log(4), rtol=1e-13)
    np.testing.assert_allclose(R.local_energy(ms, th, s), R.local_energy(m0, th, s), rtol=1e-12)
    O0 = R.log_derivs(m0, th, s)
    Oavg = O0.copy()
    off = 0
    for l in range(n + 1):
        cin = 1 if l == 0 else C
        G = O0[:, off:off + C * cin * 9].reshape(-1, C, cin, 3, 3)
        Oavg[:, off:off + C * cin * 9] = (sum(np.rot90(G, k, axes=(3, 4)) for k in range(4)) / 4).reshape(-1, C * cin * 9)
        off += C * cin * 9 + C
    np.testing.assert_allclose(R.log_derivs(ms, th, s), Oavg, rtol=1e-10, atol=1e-12)


def test_symmetrised_enumeration_identity(ham4, theta4):
    """sum_s |psi~|^2 E_loc(s) = <psi~|H|psi~> and E_loc = (H psi~)/psi~ over
    all 12870 states of 4x4 with the symmetrised amplitude."""
    H, states = ham4
    la, sg = R.log_psi(M4S, theta4, states)
    el = R.local_energy(M4S, theta4, states)
    w = np.exp(2 * (la - la.max()))
    assert (w * el).sum() / w.sum() == pytest.approx(R.exact_energy(H, la, sg), rel=1e-12)
    psi = sg * np.exp(la - la.max())
    np.testing.assert_allclose(el, (H @ psi) / psi, rtol=1e-11, atol=1e-11)


def test_symmetrised_log_derivs_central_fd():
    ms = R.RefModel(4, 4, 2, 1.0, 0.5, 1, 1)
    th = init_theta(4, 2, seed=25).astype(np.float64)
    s = uniform_sz0(4, 5, seed=26)
    O = R.log_derivs(ms, th, s)
    rng = np.random.default_rng(27)
    h = 1e-6
    for k in rng.choice(th.size, 30, replace=False):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (R.log_psi(ms, tp, s)[0] - R.log_psi(ms, tm, s)[0]) / (2 * h)
        np.testing.assert_allclose(O[:, k], fd, rtol=1e-6, atol=1e-8)


def test_symmetrised_sampler_distribution_4x4(ham4, theta4):
    H, states = ham4
    la, sg = R.log_psi(M4S, theta4, states)
    chains = 1024
    s, lab, _, _ = R.sample(M4S, theta4, neel(4, chains), n_sweeps=50, seed=4321)
    np.testing.assert_allclose(lab, R.log_psi(M4S, theta4, s)[0], rtol=1e-12)
    p = np.exp(2 * (la - la.max()))
    p /= p.sum()
    ms = _stag(states, 4)
    hist = np.bincount(_stag(s, 4), minlength=9)[:9]
    exp = np.array([p[ms == k].sum() for k in range(9)]) * chains
    keep = exp > 5
    chi2 = (((hist[keep] - exp[keep]) ** 2) / exp[keep]).sum()
    assert chi2 < 3 * keep.sum() + 20, (hist, exp)
