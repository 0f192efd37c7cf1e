"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module holds no arithmetic of the method: it only draws the random
parameters and spin configurations that both sides consume, and names the
workload presets.  Everything here is numpy (PCG64) on the host.

Workload recipe (the paper has no dataset; its inputs are the lattice, a
random or transferred parameter vector and Monte Carlo samples, Sec. 3.1):

* parameters: every weight and bias drawn N(0, 1/fan_in) with
  fan_in = 9 * C_in (9 for the 1 -> C lifting layer), PCG64 seed 0, rounded
  to float32 once; both sides receive those float32 values;
* configurations: the Neel state (the chain start of Sec. 3.1), or independent
  uniform random Sz = 0 configurations (each a random placement of N/2 up
  spins, PCG64 seed 1), which stand in for |psi|^2 samples in throughput runs.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = [
    "Preset", "PRESETS", "layer_shapes", "init_theta", "neel", "uniform_sz0",
    "ferro_like_sz0",
]


@dataclass(frozen=True)
class Preset:
    """A named workload: lattice L x L, C channels, n C->C conv layers after the
    1->C lift, couplings J1/J2 and the number of samples B."""
    name: str
    L: int
    C: int
    n: int
    J1: float
    J2: float
    B: int


PRESETS = {
    # 4x4 check: lift + 2 conv layers, 4 channels, 256 samples
    "4x4": Preset("4x4", 4, 4, 2, 1.0, 0.5, 256),
    # 10x10: lift + 6 conv layers, 16 channels (14080 parameters), 4096 samples
    "10x10": Preset("10x10", 10, 16, 6, 1.0, 0.5, 4096),
    # 16x16: lift + 8 conv layers, 32 channels (74304 parameters), 8192 samples
    "16x16": Preset("16x16", 16, 32, 8, 1.0, 0.5, 8192),
    # 24x24: the 16x16 filters reused unchanged, 16384 samples
    "24x24": Preset("24x24", 24, 32, 8, 1.0, 0.5, 16384),
}


def layer_shapes(C: int, n: int):
    """(C_out, C_in) of each 3x3 conv layer: the 1 -> C lift then n C -> C layers."""
    return [(C, 1)] + [(C, C)] * n


def init_theta(C: int, n: int, seed: int = 0, zero_bias: bool = False) -> np.ndarray:
    """Flat float32 parameter vector in layer order; per layer the weight block
    W[c_out][c_in][ky][kx] followed by the bias b[c_out].  Each entry is drawn
    N(0, 1/fan_in), fan_in = 9 * C_in."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for cout, cin in layer_shapes(C, n):
        std = 1.0 / np.sqrt(9.0 * cin)
        parts.append(rng.standard_normal(cout * cin * 9) * std)
        b = rng.standard_normal(cout) * std
        parts.append(np.zeros(cout) if zero_bias else b)
    return np.concatenate(parts).astype(np.float32)


def neel(L: int, B: int) -> np.ndarray:
    """B copies of the Neel state: +1 on sites with x + y even, -1 elsewhere.
    Site index i = y * L + x."""
    y, x = np.divmod(np.arange(L * L), L)
    s = np.where((x + y) % 2 == 0, 1, -1).astype(np.int8)
    return np.tile(s, (B, 1))


def uniform_sz0(L: int, B: int, seed: int = 1) -> np.ndarray:
    """B independent uniform random configurations with N/2 up spins."""
    N = L * L
    rng = np.random.Generator(np.random.PCG64(seed))
    base = np.concatenate([np.ones(N // 2, np.int8), -np.ones(N - N // 2, np.int8)])
    out = np.empty((B, N), np.int8)
    for b in range(B):
        out[b] = rng.permutation(base)
    return out


def ferro_like_sz0(L: int) -> np.ndarray:
    """One Sz = 0 configuration with the upper half of the rows up and the
    lower half down (few antiparallel bonds): an edge case for the
    local-energy generator."""
    N = L * L
    s = -np.ones(N, np.int8)
    s[: N // 2] = 1
    return s[None, :]
