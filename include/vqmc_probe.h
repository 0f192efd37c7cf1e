/* vqmc_probe.h -- measurement helper of libvqmc (not part of the method):
 * the achievable matrix-core throughput of the GPU, measured by a loop of
 * one matrix instruction per kind with eight independent accumulator chains
 * per wave and register operands only, so that the kernels of the library
 * can be compared with what this GPU sustains as well as with its published
 * peaks.
 *
 * vqmc_probe_mfma enqueues one launch of `blocks` workgroups of 256 threads
 * on `stream`, each wave issuing 8 * iters instructions of the kind:
 *   VQMC_PROBE_BF16  v_mfma_f32_16x16x32_bf16 (16384 FLOPs each),
 *   VQMC_PROBE_FP32  v_mfma_f32_16x16x4_f32   (2048),
 *   VQMC_PROBE_FP64  v_mfma_f64_16x16x4_f64   (2048).
 * in: dev float [128] (operand seeds); out: dev float [blocks * 256]
 * (written so that the loop is kept); *flops (host, nullable) receives the
 * FLOPs of the launch, to be divided by the caller's timing of it.
 * Returns VQMC_OK, VQMC_ERR_ARG (bad kind, iters or blocks < 1, null
 * buffers) or VQMC_ERR_DEVICE (launch failure). */
#ifndef VQMC_PROBE_H
#define VQMC_PROBE_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { VQMC_PROBE_BF16 = 0, VQMC_PROBE_FP32 = 1, VQMC_PROBE_FP64 = 2 };

int vqmc_probe_mfma(int kind, int iters, int blocks, const float *in, float *out, double *flops,
                    hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* VQMC_PROBE_H */
