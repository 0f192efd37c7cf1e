// probe.hip -- achievable matrix-core throughput on this GPU, the ceiling the
// measured kernels are compared with beside the published peaks.  Every wave
// keeps eight independent accumulator chains of one matrix instruction busy
// for a fixed number of iterations on register operands (no memory traffic
// inside the loop); the caller times the launch.  Not part of the method.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/vqmc_probe.h"
#include "common.hpp"
#include "engine.hpp"

namespace vqmc {
namespace {

constexpr int kChains = 8;

template <int KIND>
__global__ __launch_bounds__(256) void mfma_loop_kernel(const float *__restrict__ in, float *__restrict__ out,
                                                        int iters) {
  const int lane = threadIdx.x & 63;
  const float x = in[lane], y = in[64 + lane];
  float sink = 0.f;
  if constexpr (KIND == VQMC_PROBE_BF16) {
    u16x8 a, b;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      a[j] = bf16_rne(x + j);
      b[j] = bf16_rne(y - j);
    }
    f32x4 acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < kChains; ++c) acc[c] = mma_bf16(a, b, acc[c]);
#pragma unroll
    for (int c = 0; c < kChains; ++c) sink += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  } else if constexpr (KIND == VQMC_PROBE_FP32) {
    f32x4 acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < kChains; ++c) acc[c] = mma_f32(x, y, acc[c]);
#pragma unroll
    for (int c = 0; c < kChains; ++c) sink += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  } else {
    f64x4 acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = f64x4{0.0, 0.0, 0.0, 0.0};
    const double xd = x, yd = y;
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(xd, yd, acc[c], 0, 0, 0);
#pragma unroll
    for (int c = 0; c < kChains; ++c) sink += (float)(acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3]);
  }
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = sink;
}

}  // namespace
}  // namespace vqmc

using namespace vqmc;

extern "C" int vqmc_probe_mfma(int kind, int iters, int blocks, const float *in, float *out, double *flops,
                               hipStream_t stream) {
  if (iters < 1 || blocks < 1 || !in || !out) return VQMC_ERR_ARG;
  double per = 0.0;
  switch (kind) {
    case VQMC_PROBE_BF16:
      mfma_loop_kernel<VQMC_PROBE_BF16><<<blocks, 256, 0, stream>>>(in, out, iters);
      per = 2.0 * 16 * 16 * 32;
      break;
    case VQMC_PROBE_FP32:
      mfma_loop_kernel<VQMC_PROBE_FP32><<<blocks, 256, 0, stream>>>(in, out, iters);
      per = 2.0 * 16 * 16 * 4;
      break;
    case VQMC_PROBE_FP64:
      mfma_loop_kernel<VQMC_PROBE_FP64><<<blocks, 256, 0, stream>>>(in, out, iters);
      per = 2.0 * 16 * 16 * 4;
      break;
    default: return VQMC_ERR_ARG;
  }
  if (hipGetLastError() != hipSuccess) return VQMC_ERR_DEVICE;
  if (flops) *flops = per * kChains * (double)iters * (blocks * 4.0);
  return VQMC_OK;
}
