// eloc_lc.hpp -- local energy by incremental evaluation inside light cones.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

#include "common.hpp"

namespace vqmc {

// Whether the light-cone kernel handles this model: C = 16 or 32, and the
// cone boxes of distance 1 .. n fit the kernel's two LDS difference buffers
// (at 24x24 in the split-BF16 and FP32 forms: n <= 8).
bool eloc_lc_supported(const vqmc_model *m);

// Device bytes of workspace for B samples: packed weight fragments and one
// slice of FP32 pre-activations (all layers of one sample) per workgroup.
size_t eloc_lc_workspace(const vqmc_model *m, int B);

// Enqueue the light-cone local energy of B samples on st; lp (dev double
// [B], nullable) receives log|W_CNN(s)| of each sample's FP32 pass.
vqmc_status eloc_lc(const vqmc_model *m, const float *theta, const int8_t *spins, int B, double *e_loc,
                    int32_t *flags, double *lp, void *ws, hipStream_t st);

}  // namespace vqmc
