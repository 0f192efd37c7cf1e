"""Entry points captured in a HIP graph (through torch.cuda.graph) and
replayed: every replay, with the program's own eager work and
synchronisations between replays, must give the eager call's bits.

* the SR solve at an order above 1024, whose eager form runs part of the
  Cholesky's trailing update on the library's side stream (under capture it
  runs everything on the captured stream);
* the allocation-free local energy, for callers that cannot allocate."""
import numpy as np
import pytest
import torch

from gpu_common import V, to_dev, announce
from vqmc_inputs import init_theta, uniform_sz0

pytestmark = pytest.mark.gpu


def _capture(fn):
    """fn() warmed up on a side stream, then captured; returns the graph."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fn()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    torch.cuda.synchronize()
    return g


@pytest.mark.parametrize("method", [V.SR_CHOLESKY, V.SR_DUAL, V.SR_CG])
def test_sr_solve_in_a_graph(method):
    B, P = 900, 1700
    rng = np.random.default_rng(5)
    O = to_dev((rng.standard_normal((B, P)) * 0.5 + rng.standard_normal(P)).astype(np.float32))
    E = to_dev(rng.standard_normal(B) * 3 - 40)
    opts = V.SrOpts(method=method, s_prec=1, eps=1e-3, tol=1e-10, max_iter=50)
    ws = torch.empty(V.sr_workspace(B, P, opts), dtype=torch.uint8, device="cuda")
    announce("sr solve in a graph", method)
    d_ref, F_ref, _ = V.vqmc_sr_solve(O, E, opts, workspace=ws, want_info=False)
    d_ref, F_ref = d_ref.clone(), F_ref.clone()
    d = torch.empty(P, dtype=torch.float64, device="cuda")
    F = torch.empty(P, dtype=torch.float64, device="cuda")
    g = _capture(lambda: V.vqmc_sr_solve(O, E, opts, delta=d, F=F, workspace=ws, want_info=False))
    for rep in range(3):
        d.zero_()
        F.fill_(float("nan"))
        junk = (O[:, :64].double() ** 2).sum()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert torch.equal(d, d_ref) and torch.equal(F, F_ref), rep


def test_local_energy_noalloc_in_a_graph():
    L, C, n, B = 10, 16, 6, 257
    m = V.Model(L, C, n, prec=V.PREC_BF16X3, eloc=V.ELOC_DENSE)
    th = to_dev(init_theta(C, n, seed=0))
    s = to_dev(uniform_sz0(L, B, seed=3))
    announce("noalloc local energy in a graph")
    e_ref = V.vqmc_local_energy_noalloc(m, th, s).clone()
    e = torch.empty(B, dtype=torch.float64, device="cuda")
    f = torch.empty(B, dtype=torch.int32, device="cuda")
    g = _capture(lambda: V.vqmc_local_energy_noalloc(m, th, s, out=e, flags=f))
    for rep in range(3):
        e.zero_()
        f.fill_(-1)
        # eager work between replays: another model through the same array
        V.vqmc_local_energy_noalloc(V.Model(6, 8, 3, prec=V.PREC_BF16), to_dev(init_theta(8, 3, seed=1)),
                                    to_dev(uniform_sz0(6, 9, seed=2)))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(e, e_ref) and (f == 0).all(), rep
