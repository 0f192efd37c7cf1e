"""The optimisation loop around vqmc_vmc_step (Sec. 3.1 and 3.2, Fig.
framework): burn-in, then iterations of Step 1 (sampling, the chains carried
from one iteration to the next) and Step 2 (E_s, O_s, SR solve, update), with
a log of the sample energy per iteration; and the transfer of theta across
lattice sizes and couplings (Sec. 3.3): the convolutional amplitude's
parameters do not depend on L or J2/J1, so a trained theta is reused as the
start of another run.

Orchestration only: every step runs in libvqmc's kernels.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import torch

from . import vqmc as V


@dataclass
class EnergyLog:
    """Per-iteration mean and variance of E_s over the B samples (FP64)."""
    e_mean: list = field(default_factory=list)
    e_var: list = field(default_factory=list)
    sr_iters: list = field(default_factory=list)

    def per_site(self, N: int) -> list:
        return [e / N for e in self.e_mean]


@dataclass
class Chains:
    """Configurations of the B Markov chains and the next sampler counter."""
    spins: torch.Tensor
    seed: int
    counter: int = 0


def burn_in(m: V.Model, theta, chains: Chains, n_sweeps: int, proposal: int = 0) -> Chains:
    """n_sweeps sweeps of every chain before the first iteration."""
    V.vqmc_sample(m, theta, chains.spins, n_sweeps=n_sweeps, seed=chains.seed,
                  counter_base=chains.counter, proposal=proposal)
    chains.counter += n_sweeps * m.N
    return chains


def optimise(m: V.Model, theta, chains: Chains, n_iter: int, lr: float,
             opts: V.SrOpts = V.SrOpts(), n_sweeps: int = 1, proposal: int = 0,
             log: EnergyLog | None = None) -> EnergyLog:
    """n_iter iterations in place on theta (FP32, on the GPU) and the chains;
    n_sweeps sweeps (n_sweeps * N proposals) between consecutive samples."""
    log = EnergyLog() if log is None else log
    B = chains.spins.shape[0]
    ws = torch.empty(max(V.vmc_step_workspace(m, B, opts), 1), dtype=torch.uint8,
                     device=chains.spins.device)
    for _ in range(n_iter):
        info = V.vqmc_vmc_step(m, theta, chains.spins, n_sweeps, chains.seed, chains.counter, lr,
                               opts=opts, proposal=proposal, workspace=ws)
        chains.counter += n_sweeps * m.N
        log.e_mean.append(info["e_mean"])
        log.e_var.append(info["e_var"])
        log.sr_iters.append(info["iters"])
    return log


def transfer(theta, src: V.Model, dst: V.Model) -> torch.Tensor:
    """theta of src as the starting point for dst: the same channels and
    layers, any lattice size and couplings."""
    if (src.C, src.n) != (dst.C, dst.n):
        raise ValueError("transfer needs the same channels and layers (%d, %d) vs (%d, %d)"
                         % (src.C, src.n, dst.C, dst.n))
    return theta.detach().clone()


def with_couplings(m: V.Model, J1: float, J2: float) -> V.Model:
    return dataclasses.replace(m, J1=J1, J2=J2)
