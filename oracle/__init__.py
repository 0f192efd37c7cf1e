"""FP64 CPU oracle for the CNN-VQMC + SR hot path of arXiv 2108.13830.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
bench's CPU-baseline leg may import this package; the product library never
does.  It shares no code with the GPU path: the C part (``vqmc_ref.c``) is a
plain double-precision loop nest, the Python part (``ref.py``) adds the exact
4x4 enumeration of the Sz = 0 sector, the sparse Hamiltonian and exact
diagonalisation used to pin it.
"""
from .ref import *  # noqa: F401,F403
