// common.hpp -- host-side helpers shared by the libvqmc translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vqmc.h"

namespace vqmc {

// Bounds the library supports (LDS sizing of the fused kernels).
constexpr int kMaxL = 24;
constexpr int kMaxLayers = 16;

inline bool model_valid(const vqmc_model *m) {
  if (!m) return false;
  if (m->L < 4 || m->L > kMaxL || (m->L & 1)) return false;
  if (!(m->channels == 4 || m->channels == 8 || m->channels == 16 || m->channels == 32)) return false;
  if (m->n_layers < 1 || m->n_layers > kMaxLayers) return false;
  if (m->activation != VQMC_ACT_TANH) return false;
  if (m->marshall != 0 && m->marshall != 1) return false;
  if (m->conv_prec < VQMC_PREC_FP32 || m->conv_prec > VQMC_PREC_BF16X3) return false;
  if (m->conv_prec != VQMC_PREC_FP32 && m->channels % 8 != 0) return false;
  if (m->eloc_mode < VQMC_ELOC_AUTO || m->eloc_mode > VQMC_ELOC_LIGHTCONE) return false;
  if (m->symmetry != 0 && m->symmetry != 1) return false;
  return true;
}

inline int64_t num_params(int C, int n) { return (int64_t)10 * C + (int64_t)n * (9 * C * C + C); }

// The SR solve's two device status words inside its workspace (the solve
// clears both first): word 0 is set when the Cholesky factorisation meets a
// non-positive pivot, word 1 when the energies or the CG residual are not
// finite.  For options that pass sr_opts_valid.
bool sr_opts_valid(const vqmc_sr_opts *o);
int *sr_status_word(void *workspace, int32_t B, int64_t P, const vqmc_sr_opts *o);

#define VQMC_LAUNCH_CHECK()                                   \
  do {                                                        \
    if (hipGetLastError() != hipSuccess) return VQMC_ERR_DEVICE; \
  } while (0)

}  // namespace vqmc
