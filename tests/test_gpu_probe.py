"""The matrix-core probe (include/vqmc_probe.h): it runs, and the rates it
reports lie between a fifth of the published dense peaks of the MI355X and
those peaks (with 10 % margin for clock variation)."""
import pytest

from gpu_common import V, announce

pytestmark = pytest.mark.gpu

PEAK = {"bf16": 2500.0, "fp32": 157.3, "fp64": 78.6}  # TFLOP/s, dense


@pytest.mark.parametrize("kind", ["bf16", "fp32", "fp64"])
def test_probe_rates_are_plausible(kind):
    announce("probe", kind)
    t = V.probe_mfma(kind, iters=200, blocks=1024)
    print("%s matrix loop: %.1f TFLOP/s (published %.1f)" % (kind, t, PEAK[kind]))
    assert 0.2 * PEAK[kind] <= t <= 1.1 * PEAK[kind]


def test_probe_rejects_bad_arguments():
    import ctypes as ct
    lib = V.lib()
    nul = ct.c_void_p(0)
    assert lib.vqmc_probe_mfma(7, 10, 1, nul, nul, None, nul) == 1
    assert lib.vqmc_probe_mfma(0, 0, 1, nul, nul, None, nul) == 1
