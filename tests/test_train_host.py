"""Host logic of the optimisation loop module (no GPU): theta transfer
checks and the energy log."""
import pytest
import torch

T = pytest.importorskip("paper_2108_13830_amd.train")
V = pytest.importorskip("paper_2108_13830_amd.vqmc")


def test_transfer_keeps_values_and_checks_shape():
    src = V.Model(6, 8, 2)
    th = torch.arange(V.num_params(src), dtype=torch.float32)
    for dst in (V.Model(10, 8, 2), V.Model(24, 8, 2, J2=0.6), T.with_couplings(src, 1.0, 0.44)):
        out = T.transfer(th, src, dst)
        assert torch.equal(out, th) and out.data_ptr() != th.data_ptr()
    with pytest.raises(ValueError):
        T.transfer(th, src, V.Model(6, 16, 2))
    with pytest.raises(ValueError):
        T.transfer(th, src, V.Model(6, 8, 3))


def test_energy_log_per_site_and_couplings():
    log = T.EnergyLog(e_mean=[-8.0, -11.2], e_var=[1.0, 0.5])
    assert log.per_site(16) == [-0.5, -0.7]
    m = T.with_couplings(V.Model(4, 4, 2), 1.0, 0.3)
    assert (m.J1, m.J2, m.L) == (1.0, 0.3, 4)


def test_chains_counter_advances_by_sweeps():
    ch = T.Chains(torch.zeros((2, 16), dtype=torch.int8), seed=5)
    assert ch.counter == 0 and ch.seed == 5
