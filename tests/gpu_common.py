"""Helpers shared by the GPU parity tests (no arithmetic of the method here)."""
import os
import sys

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as R  # noqa: E402
from paper_2108_13830_amd import vqmc as V  # noqa: E402

DEV = "cuda:0"


def models(L, C, n, prec=V.PREC_FP32, J1=1.0, J2=0.5, marshall=1, symmetry=0, eloc=V.ELOC_AUTO):
    """The same model for the GPU library and for the oracle."""
    return (V.Model(L, C, n, J1, J2, marshall, prec, eloc, symmetry),
            R.RefModel(L, C, n, J1, J2, marshall, symmetry=symmetry))


def to_dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def announce(*what):
    """Print (and flush) what a GPU step is about to run."""
    print("[gpu]", *what, flush=True)
