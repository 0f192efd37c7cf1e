"""MI355X-native hot path of CNN variational Monte Carlo with Stochastic
Reconfiguration for the J1-J2 Heisenberg model (arXiv 2108.13830).

The computation lives in libvqmc.so (HIP kernels for gfx950, C ABI in
include/vqmc.h); ``vqmc`` is its Python binding.
"""
from . import vqmc  # noqa: F401
from .vqmc import (Model, SrOpts, num_params, vqmc_log_psi, vqmc_local_energy,  # noqa: F401
                   vqmc_sample, vqmc_log_derivs, vqmc_sr_solve, log_psi, LogPsi,
                   PREC_FP32, PREC_BF16, PREC_BF16X3, SR_AUTO, SR_CHOLESKY, SR_CG, SR_DUAL)
