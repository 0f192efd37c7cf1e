// vmc.hip -- one iteration of the variational optimisation: the sampler
// (Step 1), then local energies, log-derivatives, the SR solve and the
// parameter update (Step 2), enqueued on one stream with one workspace.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace vqmc {

// theta_k <- theta_k - lr * delta_k, in FP64, rounded once to FP32; nothing
// is written when the SR solve flagged a non-positive pivot or non-finite
// values (status words 0 and 1 of its workspace).
__global__ void sr_update_kernel(float *__restrict__ theta, const double *__restrict__ delta, int64_t P,
                                 double lr, const int *__restrict__ status) {
  if (status[0] != 0 || status[1] != 0) return;
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < P) theta[k] = (float)((double)theta[k] - lr * delta[k]);
}

static size_t al256(size_t x) { return (x + 255) / 256 * 256; }

// Workspace: E_s [B], O [B][ldO] (ldO = P rounded up to 4 floats, so that
// rows are 16-byte aligned), delta [P], then the workspaces of the local
// energy, the log-derivatives and the SR solve.
struct VmcPlan {
  int64_t P, ldO;
  size_t off_e, off_O, off_delta, off_we, off_wo, off_ws, we, wo, ws, total;
};

static vqmc_status make_plan(const vqmc_model *m, int32_t B, const vqmc_sr_opts *sr, VmcPlan &p) {
  p.P = num_params(m->channels, m->n_layers);
  p.ldO = (p.P + 3) / 4 * 4;
  vqmc_status st = vqmc_local_energy_workspace(m, B, &p.we);
  if (st != VQMC_OK) return st;
  if ((st = vqmc_log_derivs_workspace(m, B, &p.wo)) != VQMC_OK) return st;
  if ((st = vqmc_sr_workspace(B, p.P, sr, &p.ws)) != VQMC_OK) return st;
  size_t off = 0;
  p.off_e = off;
  off += al256((size_t)B * 8);
  p.off_O = off;
  off += al256((size_t)B * p.ldO * 4);
  p.off_delta = off;
  off += al256((size_t)p.P * 8);
  p.off_we = off;
  off += al256(p.we);
  p.off_wo = off;
  off += al256(p.wo);
  p.off_ws = off;
  off += al256(p.ws);
  p.total = off;
  return VQMC_OK;
}

}  // namespace vqmc

using namespace vqmc;

extern "C" vqmc_status vqmc_vmc_step_workspace(const vqmc_model *m, int32_t B, const vqmc_sr_opts *sr,
                                               size_t *bytes) {
  if (!model_valid(m) || !sr_opts_valid(sr) || !bytes) return VQMC_ERR_ARG;
  if (B < 2) return VQMC_ERR_SHAPE;
  VmcPlan p{};
  const vqmc_status st = make_plan(m, B, sr, p);
  if (st != VQMC_OK) return st;
  *bytes = p.total;
  return VQMC_OK;
}

extern "C" vqmc_status vqmc_vmc_step(const vqmc_model *m, float *theta, int8_t *spins, int32_t B,
                                     int32_t n_sweeps, uint64_t seed, uint64_t counter_base, int32_t proposal,
                                     const vqmc_sr_opts *sr, double lr, double *e_loc, void *workspace,
                                     size_t ws_bytes, vqmc_sr_info *info, hipStream_t stream) {
  if (!model_valid(m) || !sr_opts_valid(sr)) return VQMC_ERR_ARG;
  if (B < 2 || n_sweeps < 0) return VQMC_ERR_SHAPE;
  if (!theta || !spins || proposal < 0 || proposal > 1 || !(lr == lr)) return VQMC_ERR_ARG;
  VmcPlan p{};
  vqmc_status st = make_plan(m, B, sr, p);
  if (st != VQMC_OK) return st;
  if (!workspace || ws_bytes < p.total) return VQMC_ERR_WORKSPACE;
  char *w = reinterpret_cast<char *>(workspace);
  double *e = e_loc ? e_loc : reinterpret_cast<double *>(w + p.off_e);
  float *O = reinterpret_cast<float *>(w + p.off_O);
  double *delta = reinterpret_cast<double *>(w + p.off_delta);
  // Step 1: move the chains n_sweeps sweeps on from where they are
  if ((st = vqmc_sample(m, theta, spins, nullptr, B, n_sweeps, seed, counter_base, proposal, nullptr, stream)) !=
      VQMC_OK)
    return st;
  // Step 2: E_s, O_s, (S + eps I) delta = F, theta <- theta - lr delta
  if ((st = vqmc_local_energy(m, theta, spins, B, e, nullptr, p.we ? w + p.off_we : nullptr, p.we, stream)) !=
      VQMC_OK)
    return st;
  if ((st = vqmc_log_derivs(m, theta, spins, B, O, p.ldO, w + p.off_wo, p.wo, stream)) != VQMC_OK) return st;
  const vqmc_status sr_st =
      vqmc_sr_solve(O, p.ldO, e, B, p.P, sr, delta, nullptr, w + p.off_ws, p.ws, info, stream);
  if (sr_st != VQMC_OK && sr_st != VQMC_WARN_NOT_CONVERGED) return sr_st;
  const int *status = sr_status_word(w + p.off_ws, B, p.P, sr);
  sr_update_kernel<<<(unsigned)((p.P + 255) / 256), 256, 0, stream>>>(theta, delta, p.P, lr, status);
  VQMC_LAUNCH_CHECK();
  return sr_st;
}
