"""The allocation-free local energy (vqmc_local_energy_noalloc) against
vqmc_local_energy with a caller workspace, through the C ABI: the same
kernels read the same packed weights, so the energies and flags must agree
bit for bit.  Two calls in a row on one GPU, the second with a smaller
batch (and another model), so that the second reads what it wrote itself
and not what the first call left in the library's array."""
import numpy as np
import pytest
import torch

from gpu_common import V, to_dev, host, announce
from vqmc_inputs import init_theta, uniform_sz0

pytestmark = pytest.mark.gpu

CASES = [
    # (L, C, n, prec, B): the 10x10 workload first, then smaller calls
    (10, 16, 6, V.PREC_FP32, 4096),
    (10, 16, 6, V.PREC_BF16X3, 333),
    (6, 8, 3, V.PREC_BF16, 77),
    (4, 4, 2, V.PREC_FP32, 5),
]


def _pair(L, C, n, prec, B, seed):
    m = V.Model(L, C, n, 1.0, 0.5, 1, prec, V.ELOC_DENSE)
    th = to_dev(init_theta(C, n, seed=seed))
    s = to_dev(uniform_sz0(L, B, seed=seed + 1))
    announce("noalloc", L, C, n, prec, B)
    ws = torch.empty(max(V.local_energy_workspace(m, B), 1), dtype=torch.uint8, device="cuda")
    f_ref = torch.full((B,), -1, dtype=torch.int32, device="cuda")
    e_ref = V.vqmc_local_energy(m, th, s, flags=f_ref, workspace=ws)
    f = torch.full((B,), -1, dtype=torch.int32, device="cuda")
    e = V.vqmc_local_energy_noalloc(m.with_eloc(V.ELOC_AUTO), th, s, flags=f)
    return host(e), host(e_ref), host(f), host(f_ref)


def test_noalloc_matches_workspace_form_two_calls():
    for k, (L, C, n, prec, B) in enumerate(CASES):
        e, e_ref, f, f_ref = _pair(L, C, n, prec, B, seed=3 * k)
        assert np.isfinite(e).all()
        assert np.array_equal(e.view(np.int64), e_ref.view(np.int64)), (L, C, n, prec, B)
        assert np.array_equal(f, f_ref) and (f == 0).all()


def test_noalloc_rejects_what_needs_a_workspace():
    th = to_dev(init_theta(16, 2, seed=0))
    s = to_dev(uniform_sz0(16, 4, seed=1))
    with pytest.raises(V.VqmcError):
        V.vqmc_local_energy_noalloc(V.Model(16, 16, 2, eloc=V.ELOC_LIGHTCONE), th, s)
    with pytest.raises(V.VqmcError):
        V.vqmc_local_energy_noalloc(V.Model(16, 16, 2, symmetry=1), th, s)
