// capi.cpp -- model helpers and status strings of the C ABI.
#include "common.hpp"

extern "C" int64_t vqmc_num_params(const vqmc_model *m) {
  if (!vqmc::model_valid(m)) return -1;
  return vqmc::num_params(m->channels, m->n_layers);
}

extern "C" const char *vqmc_status_string(vqmc_status s) {
  switch (s) {
    case VQMC_OK: return "ok";
    case VQMC_ERR_ARG: return "invalid argument";
    case VQMC_ERR_SHAPE: return "unsupported size";
    case VQMC_ERR_DEVICE: return "HIP launch or runtime error";
    case VQMC_ERR_WORKSPACE: return "workspace missing or too small";
    case VQMC_ERR_NOT_SPD: return "matrix not positive definite";
    case VQMC_WARN_NOT_CONVERGED: return "conjugate gradients did not converge";
    case VQMC_ERR_NONFINITE: return "non-finite energies or residual in the SR solve";
  }
  return "unknown status";
}
