"""Python side of the FP64 oracle (test infrastructure only).

* ctypes bindings of ``libvqmc_ref.so`` (plain FP64 loops, see vqmc_ref.c);
* exact enumeration of the Sz = 0 sector of small lattices and the sparse
  Hamiltonian of Eq. (J1-J2) built from all site pairs classified by their
  periodic distance (an independent route to the bond set of Sec. 3.1);
* exact energies: <psi|H|psi>/<psi|psi> over all states and the ground energy
  by exact diagonalisation (scipy.sparse.linalg.eigsh).

Nothing here is imported by the product package.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass
from itertools import combinations

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvqmc_ref.so")

__all__ = [
    "RefModel", "lib", "num_params", "log_psi", "local_energy", "log_derivs",
    "sr_solve", "sr_matrix", "sr_apply", "philox4x32_10", "sample", "sz0_states",
    "bond_pairs", "hamiltonian", "exact_energy", "ground_energy",
]


class _Model(ct.Structure):
    _fields_ = [("L", ct.c_int32), ("C", ct.c_int32), ("n", ct.c_int32),
                ("J1", ct.c_double), ("J2", ct.c_double), ("marshall", ct.c_int32),
                ("symmetry", ct.c_int32)]


@dataclass(frozen=True)
class RefModel:
    L: int
    C: int
    n: int
    J1: float = 1.0
    J2: float = 0.5
    marshall: int = 1
    symmetry: int = 0

    def c(self) -> _Model:
        return _Model(self.L, self.C, self.n, self.J1, self.J2, self.marshall, self.symmetry)

    @property
    def N(self) -> int:
        return self.L * self.L


_lib = None


def lib():
    """Load (building if needed) the oracle shared library."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from .build import build
            build()
        L = ct.CDLL(LIB_PATH)
        P = ct.c_void_p
        L.vqmc_ref_num_params.restype = ct.c_int64
        L.vqmc_ref_num_params.argtypes = [ct.POINTER(_Model)]
        L.vqmc_ref_log_psi.argtypes = [ct.POINTER(_Model), P, P, ct.c_int32, P, P]
        L.vqmc_ref_local_energy.argtypes = [ct.POINTER(_Model), P, P, ct.c_int32, P, P]
        L.vqmc_ref_log_derivs.argtypes = [ct.POINTER(_Model), P, P, ct.c_int32, P, ct.c_int64]
        L.vqmc_ref_sr_solve.argtypes = [P, ct.c_int64, P, ct.c_int32, ct.c_int64, ct.c_double,
                                        ct.c_int32, P, P, P, P]
        L.vqmc_ref_sr_matrix.argtypes = [P, ct.c_int64, ct.c_int32, ct.c_int64, P]
        L.vqmc_ref_sr_apply.argtypes = [P, ct.c_int64, ct.c_int32, ct.c_int64, P, ct.c_double, P, P]
        L.vqmc_ref_philox4x32_10.argtypes = [P, P, P]
        L.vqmc_ref_philox4x32_10.restype = None
        L.vqmc_ref_sample.argtypes = [ct.POINTER(_Model), P, P, ct.c_int32, ct.c_int32,
                                      ct.c_uint64, ct.c_uint64, ct.c_int32, P, P, P]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ct.c_void_p)


def _theta(theta) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(theta, dtype=np.float64))


def _spins(spins, N) -> np.ndarray:
    s = np.ascontiguousarray(np.asarray(spins, dtype=np.int8))
    return s.reshape(-1, N)


def num_params(m: RefModel) -> int:
    mc = m.c()
    return int(lib().vqmc_ref_num_params(ct.byref(mc)))


def log_psi(m: RefModel, theta, spins):
    """(log|W_CNN|, Marshall sign) for every row of spins."""
    s = _spins(spins, m.N)
    th = _theta(theta)
    B = s.shape[0]
    out = np.zeros(B)
    sg = np.zeros(B, np.int8)
    mc = m.c()
    rc = lib().vqmc_ref_log_psi(ct.byref(mc), _p(th), _p(s), B, _p(out), _p(sg))
    assert rc == 0, rc
    return out, sg


def local_energy(m: RefModel, theta, spins, with_flags: bool = False):
    s = _spins(spins, m.N)
    th = _theta(theta)
    B = s.shape[0]
    e = np.zeros(B)
    f = np.zeros(B, np.int32)
    mc = m.c()
    rc = lib().vqmc_ref_local_energy(ct.byref(mc), _p(th), _p(s), B, _p(e), _p(f))
    assert rc == 0, rc
    return (e, f) if with_flags else e


def log_derivs(m: RefModel, theta, spins) -> np.ndarray:
    s = _spins(spins, m.N)
    th = _theta(theta)
    B = s.shape[0]
    P = num_params(m)
    O = np.zeros((B, P))
    mc = m.c()
    rc = lib().vqmc_ref_log_derivs(ct.byref(mc), _p(th), _p(s), B, _p(O), P)
    assert rc == 0, rc
    return O


def sr_solve(O, e_loc, eps: float = 1e-4, method: int = -1):
    """Exact SR step: returns dict(delta, F, e_mean, e_var)."""
    O = np.ascontiguousarray(np.asarray(O, dtype=np.float64))
    e = np.ascontiguousarray(np.asarray(e_loc, dtype=np.float64))
    B, P = O.shape
    delta = np.zeros(P)
    F = np.zeros(P)
    em = ct.c_double(0.0)
    ev = ct.c_double(0.0)
    rc = lib().vqmc_ref_sr_solve(_p(O), P, _p(e), B, P, eps, method, _p(delta), _p(F),
                                 ct.cast(ct.pointer(em), ct.c_void_p),
                                 ct.cast(ct.pointer(ev), ct.c_void_p))
    if rc != 0:
        raise RuntimeError("oracle sr_solve failed: %d" % rc)
    return dict(delta=delta, F=F, e_mean=em.value, e_var=ev.value)


def sr_matrix(O) -> np.ndarray:
    O = np.ascontiguousarray(np.asarray(O, dtype=np.float64))
    B, P = O.shape
    S = np.zeros((P, P))
    rc = lib().vqmc_ref_sr_matrix(_p(O), P, B, P, _p(S))
    assert rc == 0, rc
    return S


def sr_apply(O, mean, v, eps: float = 1e-4) -> np.ndarray:
    """(S + eps I) v with S = (1/B) O^cT O^c applied matrix-free; the column
    means of O are passed in."""
    O = np.ascontiguousarray(np.asarray(O, dtype=np.float64))
    mean = np.ascontiguousarray(np.asarray(mean, dtype=np.float64))
    v = np.ascontiguousarray(np.asarray(v, dtype=np.float64))
    B, P = O.shape
    out = np.zeros(P)
    rc = lib().vqmc_ref_sr_apply(_p(O), P, B, P, _p(mean), eps, _p(v), _p(out))
    assert rc == 0, rc
    return out


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, np.uint32)
    lib().vqmc_ref_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def sample(m: RefModel, theta, spins, n_sweeps: int, seed: int, counter_base: int = 0,
           proposal: int = 0):
    """Run the Metropolis chains in place on a copy of spins.  Returns
    (spins, log_abs, n_acc, min_margin)."""
    s = _spins(spins, m.N).copy()
    th = _theta(theta)
    B = s.shape[0]
    la = np.zeros(B)
    na = np.zeros(B, np.int32)
    mm = np.zeros(B)
    mc = m.c()
    rc = lib().vqmc_ref_sample(ct.byref(mc), _p(th), _p(s), B, n_sweeps, seed, counter_base,
                               proposal, _p(la), _p(na), _p(mm))
    assert rc == 0, rc
    return s, la, na, mm


# ------------------------------------------------------- exact enumeration

def sz0_states(L: int) -> np.ndarray:
    """All configurations of the L x L lattice with N/2 up spins, as an int8
    array [n_states][N] (+1 up, -1 down), in increasing bitmask order (bit i
    set = site i up)."""
    N = L * L
    assert N <= 24, "enumeration is for tiny lattices only"
    masks = np.arange(1 << N, dtype=np.int64)
    pop = np.zeros_like(masks)
    for i in range(N):
        pop += (masks >> i) & 1
    masks = masks[pop == N // 2]
    bits = (masks[:, None] >> np.arange(N)[None, :]) & 1
    return np.where(bits == 1, 1, -1).astype(np.int8)


def bond_pairs(L: int, J1: float, J2: float):
    """All unordered site pairs at periodic distance (1,0)/(0,1) (coupling J1)
    or (1,1) (coupling J2), found by scanning every pair of sites.  Returns a
    list of (i, j, J)."""
    N = L * L
    out = []
    for i, j in combinations(range(N), 2):
        yi, xi = divmod(i, L)
        yj, xj = divmod(j, L)
        dx = min(abs(xi - xj), L - abs(xi - xj))
        dy = min(abs(yi - yj), L - abs(yi - yj))
        if (dx, dy) in ((1, 0), (0, 1)):
            out.append((i, j, J1))
        elif (dx, dy) == (1, 1):
            out.append((i, j, J2))
    return out


def hamiltonian(L: int, J1: float, J2: float):
    """Sparse H of Eq. (J1-J2) on the Sz = 0 sector in the sigma^z basis.
    J/4 sigma_i . sigma_j = J/4 (sx sx + sy sy + sz sz): the z part is
    diagonal (J/4 s_i s_j); the x and y parts together move an antiparallel
    pair to its exchanged configuration with amplitude 2 * J/4 = J/2.
    Returns (H as scipy.sparse.csr_matrix, states)."""
    import scipy.sparse as sp
    states = sz0_states(L)
    N = L * L
    M = states.shape[0]
    masks = ((states > 0).astype(np.int64) << np.arange(N)).sum(axis=1)
    index = -np.ones(1 << N, dtype=np.int64)
    index[masks] = np.arange(M)
    rows, cols, vals = [], [], []
    diag = np.zeros(M)
    for i, j, J in bond_pairs(L, J1, J2):
        si = states[:, i].astype(np.float64)
        sj = states[:, j].astype(np.float64)
        diag += 0.25 * J * si * sj
        anti = np.nonzero(states[:, i] != states[:, j])[0]
        flipped = masks[anti] ^ (1 << i) ^ (1 << j)
        rows.append(index[flipped])
        cols.append(anti)
        vals.append(np.full(anti.size, 0.5 * J))
    rows.append(np.arange(M))
    cols.append(np.arange(M))
    vals.append(diag)
    H = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(M, M))
    return H, states


def exact_energy(H, log_abs, sign) -> float:
    """<psi|H|psi>/<psi|psi> with psi = sign * exp(log_abs) over all states."""
    psi = sign.astype(np.float64) * np.exp(log_abs - log_abs.max())
    return float(psi @ (H @ psi) / (psi @ psi))


def ground_energy(H, k: int = 1):
    from scipy.sparse.linalg import eigsh
    w = eigsh(H, k=k, which="SA", return_eigenvectors=False, tol=1e-12)
    return np.sort(w)
