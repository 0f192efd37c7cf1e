// sr.hip -- the Stochastic Reconfiguration step (Sec. 3.2.2; Eqs. Es-Os-G,
// delta and convar-matrix), all arithmetic in FP64:
//   E^c = E - <E>,  O^c = O - <O>,  F = (1/B) O^cT E^c,  S = (1/B) O^cT O^c,
//   (S + eps I) delta = F.
// Three solvers:
//   1 explicit S (FP64 or FP32 matrix cores) + blocked Cholesky + two
//     triangular solves (the paper's pdgemm / pdpotrf / 2 x pdtrsv);
//   2 matrix-free conjugate gradients, S p = O^cT (O^c p) / B + eps p applied
//     as two streaming passes over O per iteration;
//   3 the same solution through the B x B sample-space system
//     (O^c O^cT / B + eps I) a = E^c / B, delta = O^cT a.
// Every reduction has a fixed order, so results are run-to-run identical.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "common.hpp"
#include "engine.hpp"

namespace vqmc {

// v_mfma_f64_16x16x4f64: A[m = lane%16][k = lane/16], B[k = lane/16][n = lane%16],
// D register i of lane l holds D[row = l/16 + 4 i][col = l%16].
__device__ __forceinline__ f64x4 mma_f64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <int NT>
__device__ __forceinline__ double block_sum_t(double v, double *tmp) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) tmp[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) t += tmp[w];
  __syncthreads();
  return t;
}

// scalar slots in the workspace
enum { S_MEAN = 0, S_VAR, S_SUMEC, S_RR, S_NORMF, S_DONE, S_ITERS, S_REL, S_NSLOT = 16 };

// ------------------------------------------------------------ reductions

__global__ __launch_bounds__(1024) void energy_stats_kernel(const double *__restrict__ e, int B,
                                                            double *__restrict__ ec,
                                                            double *__restrict__ scal,
                                                            int *__restrict__ status) {
  __shared__ double tmp[16];
  if (threadIdx.x < 4) status[threadIdx.x] = 0;
  double s = 0.0;
  for (int b = threadIdx.x; b < B; b += 1024) s += e[b];
  const double mean = block_sum_t<1024>(s, tmp) / B;
  double v = 0.0, c = 0.0;
  for (int b = threadIdx.x; b < B; b += 1024) {
    const double d = e[b] - mean;
    ec[b] = d;
    v += d * d;
    c += d;
  }
  const double var = block_sum_t<1024>(v, tmp) / B;
  const double sc = block_sum_t<1024>(c, tmp);
  if (threadIdx.x == 0) {
    scal[S_MEAN] = mean;
    scal[S_VAR] = var;
    scal[S_SUMEC] = sc;
  }
}

// part_a[c][k] = sum_{b in chunk c} O[b][k] * wa_b (wa = 1 if null, O centred
// by obar if obar != null); part_b likewise with wb (optional).
template <bool CENTRED>
__global__ __launch_bounds__(256) void col_partial_kernel(const float *__restrict__ O, int64_t ldO, int B,
                                                          int64_t P, const double *__restrict__ obar,
                                                          const double *__restrict__ wa,
                                                          const double *__restrict__ wb, int rows_per_chunk,
                                                          double *__restrict__ part_a,
                                                          double *__restrict__ part_b,
                                                          const double *__restrict__ scal) {
  if (scal && scal[S_DONE] != 0.0) return;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= P) return;
  const int c = blockIdx.y;
  const int b0 = c * rows_per_chunk, b1 = min(B, b0 + rows_per_chunk);
  const double ob = CENTRED ? obar[k] : 0.0;
  double sa = 0.0, sb = 0.0;
#pragma unroll 8
  for (int b = b0; b < b1; ++b) {
    const double o = (double)O[(int64_t)b * ldO + k] - ob;
    sa += wa ? o * wa[b] : o;
    if (wb) sb += o * wb[b];
  }
  part_a[(int64_t)c * P + k] = sa;
  if (part_b) part_b[(int64_t)c * P + k] = sb;
}

// <O_k> and F_k = (1/B) (sum_b O_bk E^c_b - <O_k> sum_b E^c_b).
__global__ void col_stats_finish_kernel(const double *__restrict__ part_o, const double *__restrict__ part_f,
                                        int nch, int64_t P, int B, const double *__restrict__ scal,
                                        double *__restrict__ obar, double *__restrict__ F) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P) return;
  double so = 0.0, sf = 0.0;
  for (int c = 0; c < nch; ++c) {
    so += part_o[(int64_t)c * P + k];
    sf += part_f[(int64_t)c * P + k];
  }
  const double ob = so / B;
  obar[k] = ob;
  F[k] = (sf - ob * scal[S_SUMEC]) / B;
}

// out_k = sum_c part[c][k] (delta = O^cT a of the sample-space solve).
__global__ void col_sum_kernel(const double *__restrict__ part, int nch, int64_t P, double *__restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P) return;
  double s = 0.0;
  for (int c = 0; c < nch; ++c) s += part[(int64_t)c * P + k];
  out[k] = s;
}

// ------------------------------------------------ explicit S (primal SYRK)

// Triangular index of a lower-triangular block (bi >= bj).
__device__ __forceinline__ void tri_index(int t, int &bi, int &bj) {
  int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  bi = i;
  bj = t - i * (i + 1) / 2;
}

// S[i][j] = (1/B) sum_b (O[b][i] - <O_i>)(O[b][j] - <O_j>) + eps [i == j],
// lower 64 x 64 blocks; 4 waves in 2 x 2, each 2 x 2 MFMA tiles.  F64: FP64
// operands and accumulation; otherwise the centred values are rounded to
// FP32 and accumulated by the FP32 matrix cores.
template <bool F64>
__global__ __launch_bounds__(256) void syrk_kernel(const float *__restrict__ O, int64_t ldO, int B, int64_t P,
                                                   const double *__restrict__ obar, double eps,
                                                   double *__restrict__ S) {
  constexpr int KC = 32;
  using T = typename std::conditional<F64, double, float>::type;
  __shared__ T sA[KC][64 + 1];
  __shared__ T sB[KC][64 + 1];
  int bi, bj;
  tri_index(blockIdx.x, bi, bj);
  const int64_t i0 = (int64_t)bi * 64, j0 = (int64_t)bj * 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  typedef typename std::conditional<F64, f64x4, f32x4>::type accT;
  accT acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = accT{0, 0, 0, 0};
  const int lc = tid & 63, lr = tid >> 6;
  const double obi = (i0 + lc < P) ? obar[i0 + lc] : 0.0;
  const double obj = (j0 + lc < P) ? obar[j0 + lc] : 0.0;
  for (int kb = 0; kb < B; kb += KC) {
#pragma unroll
    for (int q = 0; q < KC / 4; ++q) {
      const int r = lr + 4 * q, b = kb + r;
      const bool rv = b < B;
      const double vi = (rv && i0 + lc < P) ? (double)O[(int64_t)b * ldO + i0 + lc] - obi : 0.0;
      const double vj = (rv && j0 + lc < P) ? (double)O[(int64_t)b * ldO + j0 + lc] - obj : 0.0;
      sA[r][lc] = (T)vi;
      sB[r][lc] = (T)vj;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int k = ks * 4 + (lane >> 4);
      T a[2], bb[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = sA[k][wm * 32 + t * 16 + (lane & 15)];
        bb[t] = sB[k][wn * 32 + t * 16 + (lane & 15)];
      }
#pragma unroll
      for (int tm = 0; tm < 2; ++tm)
#pragma unroll
        for (int tn = 0; tn < 2; ++tn) {
          if constexpr (F64) acc[tm][tn] = mma_f64(a[tm], bb[tn], acc[tm][tn]);
          else acc[tm][tn] = mma_f32(a[tm], bb[tn], acc[tm][tn]);
        }
    }
    __syncthreads();
  }
  const double inv = 1.0 / B;
#pragma unroll
  for (int tm = 0; tm < 2; ++tm)
#pragma unroll
    for (int tn = 0; tn < 2; ++tn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rl = F64 ? ((lane >> 4) + 4 * r) : (4 * (lane >> 4) + r);
        const int64_t row = i0 + wm * 32 + tm * 16 + rl;
        const int64_t col = j0 + wn * 32 + tn * 16 + (lane & 15);
        if (row < P && col <= row) S[row * P + col] = (double)acc[tm][tn][r] * inv + (row == col ? eps : 0.0);
      }
}

// Sample-space Gram: K[a][c] = (1/B) sum_k (O[a][k]-<O_k>)(O[c][k]-<O_k>) + eps [a == c].
__global__ __launch_bounds__(256) void gram_kernel(const float *__restrict__ O, int64_t ldO, int B, int64_t P,
                                                   const double *__restrict__ obar, double eps,
                                                   double *__restrict__ K) {
  constexpr int KC = 32;
  __shared__ double sA[64][KC + 1];
  __shared__ double sB[64][KC + 1];
  int bi, bj;
  tri_index(blockIdx.x, bi, bj);
  const int a0 = bi * 64, c0 = bj * 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = f64x4{0, 0, 0, 0};
  const int lk = tid & (KC - 1), lr = tid / KC;  // 8 rows per pass
  for (int64_t kb = 0; kb < P; kb += KC) {
    const int64_t k = kb + lk;
    const double ob = k < P ? obar[k] : 0.0;
#pragma unroll
    for (int q = 0; q < 64 / 8; ++q) {
      const int r = lr + 8 * q;
      const int ra = a0 + r, rc = c0 + r;
      sA[r][lk] = (ra < B && k < P) ? (double)O[(int64_t)ra * ldO + k] - ob : 0.0;
      sB[r][lk] = (rc < B && k < P) ? (double)O[(int64_t)rc * ldO + k] - ob : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int kk = ks * 4 + (lane >> 4);
      double a[2], bb[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = sA[wm * 32 + t * 16 + (lane & 15)][kk];
        bb[t] = sB[wn * 32 + t * 16 + (lane & 15)][kk];
      }
#pragma unroll
      for (int tm = 0; tm < 2; ++tm)
#pragma unroll
        for (int tn = 0; tn < 2; ++tn) acc[tm][tn] = mma_f64(a[tm], bb[tn], acc[tm][tn]);
    }
    __syncthreads();
  }
  const double inv = 1.0 / B;
#pragma unroll
  for (int tm = 0; tm < 2; ++tm)
#pragma unroll
    for (int tn = 0; tn < 2; ++tn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = a0 + wm * 32 + tm * 16 + (lane >> 4) + 4 * r;
        const int col = c0 + wn * 32 + tn * 16 + (lane & 15);
        if (row < B && col <= row) K[(int64_t)row * B + col] = acc[tm][tn][r] * inv + (row == col ? eps : 0.0);
      }
}

// ------------------------------------------------------ blocked Cholesky

constexpr int NB = 64;

// Factor the diagonal block kb of the lower triangle in place (one block).
__global__ __launch_bounds__(256) void potrf_diag_kernel(double *__restrict__ M, int64_t n, int kb,
                                                         int *__restrict__ status) {
  __shared__ double A[NB][NB + 1];
  const int64_t o = (int64_t)kb * NB;
  const int m = (int)min((int64_t)NB, n - o);
  for (int idx = threadIdx.x; idx < NB * NB; idx += 256) {
    const int i = idx / NB, t = idx - i * NB;
    A[i][t] = (i < m && t < m) ? (t <= i ? M[(o + i) * n + o + t] : 0.0) : (i == t ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int j = 0; j < NB; ++j) {
    if (threadIdx.x == 0) {
      double d = A[j][j];
      if (!(d > 0.0)) {
        *status = 1;
        d = 1.0;
      }
      A[j][j] = sqrt(d);
    }
    __syncthreads();
    for (int i = j + 1 + threadIdx.x; i < NB; i += 256) A[i][j] /= A[j][j];
    __syncthreads();
    for (int idx = threadIdx.x; idx < NB * NB; idx += 256) {
      const int i = idx / NB, t = idx - i * NB;
      if (t > j && t <= i) A[i][t] -= A[i][j] * A[t][j];
    }
    __syncthreads();
  }
  for (int idx = threadIdx.x; idx < NB * NB; idx += 256) {
    const int i = idx / NB, t = idx - i * NB;
    if (i < m && t <= i) M[(o + i) * n + o + t] = A[i][t];
  }
}

// Panel below the diagonal block: L[i][kb] = A[i][kb] L_kk^-T, one row per
// thread by forward substitution.
__global__ __launch_bounds__(256) void trsm_panel_kernel(double *__restrict__ M, int64_t n, int kb) {
  __shared__ double Lk[NB][NB + 1];
  const int64_t o = (int64_t)kb * NB;
  for (int idx = threadIdx.x; idx < NB * NB; idx += 256) {
    const int i = idx / NB, t = idx - i * NB;
    Lk[i][t] = t <= i ? M[(o + i) * n + o + t] : 0.0;
  }
  __syncthreads();
  const int64_t row = o + NB + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (row >= n) return;
  double x[NB];
  double *a = M + row * n + o;
#pragma unroll
  for (int t = 0; t < NB; ++t) x[t] = a[t];
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    double v = x[t];
#pragma unroll
    for (int s = 0; s < t; ++s) v -= x[s] * Lk[t][s];
    x[t] = v / Lk[t][t];
  }
#pragma unroll
  for (int t = 0; t < NB; ++t) a[t] = x[t];
}

// Trailing update A[i][j] -= sum_t L[i][t] L[j][t] over the panel kb, for the
// lower 64 x 64 blocks below and right of it (FP64 matrix cores).
__global__ __launch_bounds__(256) void syrk_update_kernel(double *__restrict__ M, int64_t n, int kb) {
  __shared__ double sA[64][NB + 1];
  __shared__ double sB[64][NB + 1];
  int bi, bj;
  tri_index(blockIdx.x, bi, bj);
  const int64_t o = (int64_t)kb * NB;
  const int64_t i0 = o + NB + (int64_t)bi * 64, j0 = o + NB + (int64_t)bj * 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  for (int idx = tid; idx < 64 * NB; idx += 256) {
    const int r = idx / NB, t = idx - r * NB;
    sA[r][t] = (i0 + r < n) ? M[(i0 + r) * n + o + t] : 0.0;
    sB[r][t] = (j0 + r < n) ? M[(j0 + r) * n + o + t] : 0.0;
  }
  __syncthreads();
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[a][c] = f64x4{0, 0, 0, 0};
#pragma unroll 4
  for (int ks = 0; ks < NB / 4; ++ks) {
    const int k = ks * 4 + (lane >> 4);
    double a[2], bb[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      a[t] = sA[wm * 32 + t * 16 + (lane & 15)][k];
      bb[t] = sB[wn * 32 + t * 16 + (lane & 15)][k];
    }
#pragma unroll
    for (int tm = 0; tm < 2; ++tm)
#pragma unroll
      for (int tn = 0; tn < 2; ++tn) acc[tm][tn] = mma_f64(a[tm], bb[tn], acc[tm][tn]);
  }
#pragma unroll
  for (int tm = 0; tm < 2; ++tm)
#pragma unroll
    for (int tn = 0; tn < 2; ++tn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = i0 + wm * 32 + tm * 16 + (lane >> 4) + 4 * r;
        const int64_t col = j0 + wn * 32 + tn * 16 + (lane & 15);
        if (row < n && col <= row) M[row * n + col] -= acc[tm][tn][r];
      }
}

// Forward substitution on the diagonal block: rhs_kb <- L_kk^-1 rhs_kb.
__global__ __launch_bounds__(256) void trsv_fwd_diag_kernel(const double *__restrict__ M, int64_t n, int kb,
                                                            double *__restrict__ rhs) {
  __shared__ double Lk[NB][NB + 1];
  __shared__ double y[NB];
  const int64_t o = (int64_t)kb * NB;
  const int m = (int)min((int64_t)NB, n - o);
  for (int idx = threadIdx.x; idx < NB * NB; idx += 256) {
    const int i = idx / NB, t = idx - i * NB;
    Lk[i][t] = (i < m && t <= i) ? M[(o + i) * n + o + t] : 0.0;
  }
  if (threadIdx.x < NB) y[threadIdx.x] = threadIdx.x < m ? rhs[o + threadIdx.x] : 0.0;
  __syncthreads();
  for (int t = 0; t < m; ++t) {
    if (threadIdx.x == 0) y[t] /= Lk[t][t];
    __syncthreads();
    if (threadIdx.x > t && threadIdx.x < m) y[threadIdx.x] -= Lk[threadIdx.x][t] * y[t];
    __syncthreads();
  }
  if (threadIdx.x < m) rhs[o + threadIdx.x] = y[threadIdx.x];
}

// rhs_i -= sum_t L[i][kb*NB + t] y_t for the rows below block kb.
__global__ __launch_bounds__(256) void trsv_fwd_update_kernel(const double *__restrict__ M, int64_t n, int kb,
                                                              double *__restrict__ rhs) {
  __shared__ double y[NB];
  const int64_t o = (int64_t)kb * NB;
  if (threadIdx.x < NB) y[threadIdx.x] = rhs[o + threadIdx.x];
  __syncthreads();
  const int64_t row = o + NB + (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (row >= n) return;
  const double *a = M + row * n + o;
  double s = 0.0;
#pragma unroll 8
  for (int t = 0; t < NB; ++t) s += a[t] * y[t];
  rhs[row] -= s;
}

// Back substitution on the diagonal block: rhs_kb <- L_kk^-T rhs_kb.
__global__ __launch_bounds__(256) void trsv_bwd_diag_kernel(const double *__restrict__ M, int64_t n, int kb,
                                                            double *__restrict__ rhs) {
  __shared__ double Lk[NB][NB + 1];
  __shared__ double x[NB];
  const int64_t o = (int64_t)kb * NB;
  const int m = (int)min((int64_t)NB, n - o);
  for (int idx = threadIdx.x; idx < NB * NB; idx += 256) {
    const int i = idx / NB, t = idx - i * NB;
    Lk[i][t] = (i < m && t <= i) ? M[(o + i) * n + o + t] : 0.0;
  }
  if (threadIdx.x < NB) x[threadIdx.x] = threadIdx.x < m ? rhs[o + threadIdx.x] : 0.0;
  __syncthreads();
  for (int t = m - 1; t >= 0; --t) {
    if (threadIdx.x == 0) x[t] /= Lk[t][t];
    __syncthreads();
    if (threadIdx.x < t) x[threadIdx.x] -= Lk[t][threadIdx.x] * x[t];
    __syncthreads();
  }
  if (threadIdx.x < m) rhs[o + threadIdx.x] = x[threadIdx.x];
}

// rhs_t -= sum_{i in block kb} L[i][t] x_i for t above block kb.
__global__ __launch_bounds__(256) void trsv_bwd_update_kernel(const double *__restrict__ M, int64_t n, int kb,
                                                              double *__restrict__ rhs) {
  __shared__ double x[NB];
  const int64_t o = (int64_t)kb * NB;
  const int m = (int)min((int64_t)NB, n - o);
  if (threadIdx.x < NB) x[threadIdx.x] = threadIdx.x < m ? rhs[o + threadIdx.x] : 0.0;
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= o) return;
  double s = 0.0;
  for (int i = 0; i < m; ++i) s += M[(o + i) * n + t] * x[i];
  rhs[t] -= s;
}

// ---------------------------------------------------------------- CG

__global__ __launch_bounds__(1024) void cg_init_kernel(const double *__restrict__ F, int64_t P,
                                                       double *__restrict__ x, double *__restrict__ r,
                                                       double *__restrict__ p, double *__restrict__ scal) {
  __shared__ double tmp[16];
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < P; k += 1024) {
    const double f = F[k];
    x[k] = 0.0;
    r[k] = f;
    p[k] = f;
    s += f * f;
  }
  const double rr = block_sum_t<1024>(s, tmp);
  if (threadIdx.x == 0) {
    scal[S_RR] = rr;
    scal[S_NORMF] = sqrt(rr);
    scal[S_DONE] = rr > 0.0 ? 0.0 : 1.0;
    scal[S_ITERS] = 0.0;
    scal[S_REL] = 0.0;
  }
}

// u_b = sum_k (O[b][k] - <O_k>) p_k, one workgroup per row.
__global__ __launch_bounds__(256) void cg_rowdot_kernel(const float *__restrict__ O, int64_t ldO, int64_t P,
                                                        const double *__restrict__ obar,
                                                        const double *__restrict__ p, double *__restrict__ u,
                                                        const double *__restrict__ scal) {
  __shared__ double tmp[4];
  if (scal[S_DONE] != 0.0) return;
  const int b = blockIdx.x;
  const float *row = O + (int64_t)b * ldO;
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < P; k += 256) s += ((double)row[k] - obar[k]) * p[k];
  s = block_sum_t<256>(s, tmp);
  if (threadIdx.x == 0) u[b] = s;
}

// q = (sum_c part[c]) / B + eps p, and per-block partial sums of p . q.
__global__ __launch_bounds__(256) void cg_apply_kernel(const double *__restrict__ part, int nch, int64_t P, int B,
                                                       double eps, const double *__restrict__ p,
                                                       double *__restrict__ q, double *__restrict__ pq_part,
                                                       const double *__restrict__ scal) {
  __shared__ double tmp[4];
  if (scal[S_DONE] != 0.0) return;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double v = 0.0;
  if (k < P) {
    double s = 0.0;
    for (int c = 0; c < nch; ++c) s += part[(int64_t)c * P + k];
    const double qk = s / B + eps * p[k];
    q[k] = qk;
    v = p[k] * qk;
  }
  v = block_sum_t<256>(v, tmp);
  if (threadIdx.x == 0) pq_part[blockIdx.x] = v;
}

// alpha = rr / p.q; x += alpha p; r -= alpha q; beta = rr'/rr; p = r + beta p.
__global__ __launch_bounds__(1024) void cg_step_kernel(int64_t P, double *__restrict__ x, double *__restrict__ r,
                                                       double *__restrict__ p, const double *__restrict__ q,
                                                       const double *__restrict__ pq_part, int npq,
                                                       double *__restrict__ scal, double tol) {
  __shared__ double tmp[16];
  if (scal[S_DONE] != 0.0) return;
  double pq = 0.0;
  for (int i = 0; i < npq; ++i) pq += pq_part[i];
  const double rr = scal[S_RR];
  const double alpha = rr / pq;
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < P; k += 1024) {
    x[k] += alpha * p[k];
    const double rk = r[k] - alpha * q[k];
    r[k] = rk;
    s += rk * rk;
  }
  const double rr1 = block_sum_t<1024>(s, tmp);
  const double beta = rr1 / rr;
  for (int64_t k = threadIdx.x; k < P; k += 1024) p[k] = r[k] + beta * p[k];
  if (threadIdx.x == 0) {
    scal[S_RR] = rr1;
    scal[S_ITERS] += 1.0;
    const double rel = sqrt(rr1) / scal[S_NORMF];
    scal[S_REL] = rel;
    if (rel <= tol) scal[S_DONE] = 1.0;
  }
}

__global__ void scale_copy_kernel(const double *__restrict__ a, int64_t n, double s, double *__restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = a[k] * s;
}

// ------------------------------------------------------------- host side

static size_t al(size_t bytes) { return (bytes + 255) / 256 * 256; }

struct SrPlan {
  int method;
  int nch, rows_per_chunk;
  int npq;
  size_t off_scal, off_status, off_ec, off_obar, off_F, off_pa, off_pb, off_M, off_rhs, off_r, off_p, off_q,
      off_u, off_pq, off_alpha, total;
};

static SrPlan make_plan(int B, int64_t P, const vqmc_sr_opts *o) {
  SrPlan s{};
  s.method = o->method == 0 ? (P <= 16384 ? 1 : 2) : o->method;
  const int64_t colblocks = (P + 255) / 256;
  int nch = (int)((4096 + colblocks - 1) / colblocks);
  nch = nch < 1 ? 1 : (nch > 64 ? 64 : nch);
  nch = nch > B ? B : nch;
  s.rows_per_chunk = (B + nch - 1) / nch;
  s.nch = (B + s.rows_per_chunk - 1) / s.rows_per_chunk;
  s.npq = (int)colblocks;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t r = off;
    off += al(bytes);
    return r;
  };
  s.off_scal = take(S_NSLOT * 8);
  s.off_status = take(16);
  s.off_ec = take((size_t)B * 8);
  s.off_obar = take((size_t)P * 8);
  s.off_F = take((size_t)P * 8);
  s.off_pa = take((size_t)s.nch * P * 8);
  s.off_pb = take((size_t)s.nch * P * 8);
  if (s.method == 1) {
    s.off_M = take((size_t)P * P * 8);
  } else if (s.method == 2) {
    s.off_r = take((size_t)P * 8);
    s.off_p = take((size_t)P * 8);
    s.off_q = take((size_t)P * 8);
    s.off_u = take((size_t)B * 8);
    s.off_pq = take((size_t)s.npq * 8);
  } else {
    s.off_M = take((size_t)B * B * 8);
    s.off_alpha = take((size_t)B * 8);
  }
  s.total = off;
  return s;
}

static bool opts_valid(const vqmc_sr_opts *o) {
  return o && o->method >= 0 && o->method <= 3 && (o->s_prec == 0 || o->s_prec == 1) && o->eps > 0.0 &&
         o->tol >= 0.0 && o->max_iter >= 0;
}

// Cholesky factorisation and solve of the n x n SPD matrix M (lower
// triangle), rhs overwritten by the solution.
static vqmc_status chol_solve(double *M, int64_t n, double *rhs, int *status, hipStream_t st) {
  const int nb = (int)((n + NB - 1) / NB);
  for (int kb = 0; kb < nb; ++kb) {
    potrf_diag_kernel<<<1, 256, 0, st>>>(M, n, kb, status);
    const int64_t below = n - (int64_t)(kb + 1) * NB;
    if (below > 0) {
      trsm_panel_kernel<<<(unsigned)((below + 255) / 256), 256, 0, st>>>(M, n, kb);
      const int64_t T = (below + 63) / 64;
      syrk_update_kernel<<<(unsigned)(T * (T + 1) / 2), 256, 0, st>>>(M, n, kb);
    }
  }
  VQMC_LAUNCH_CHECK();
  for (int kb = 0; kb < nb; ++kb) {
    trsv_fwd_diag_kernel<<<1, 256, 0, st>>>(M, n, kb, rhs);
    const int64_t below = n - (int64_t)(kb + 1) * NB;
    if (below > 0) trsv_fwd_update_kernel<<<(unsigned)((below + 255) / 256), 256, 0, st>>>(M, n, kb, rhs);
  }
  for (int kb = nb - 1; kb >= 0; --kb) {
    trsv_bwd_diag_kernel<<<1, 256, 0, st>>>(M, n, kb, rhs);
    const int64_t above = (int64_t)kb * NB;
    if (above > 0) trsv_bwd_update_kernel<<<(unsigned)((above + 255) / 256), 256, 0, st>>>(M, n, kb, rhs);
  }
  VQMC_LAUNCH_CHECK();
  return VQMC_OK;
}

}  // namespace vqmc

using namespace vqmc;

extern "C" vqmc_status vqmc_sr_workspace(int32_t B, int64_t P, const vqmc_sr_opts *o, size_t *bytes) {
  if (!opts_valid(o) || !bytes) return VQMC_ERR_ARG;
  if (B < 2 || P < 1) return VQMC_ERR_SHAPE;
  *bytes = make_plan(B, P, o).total;
  return VQMC_OK;
}

extern "C" vqmc_status vqmc_sr_solve(const float *O, int64_t ldO, const double *e_loc, int32_t B, int64_t P,
                                     const vqmc_sr_opts *o, double *delta, double *F, void *workspace,
                                     size_t ws_bytes, vqmc_sr_info *info, hipStream_t st) {
  if (!opts_valid(o)) return VQMC_ERR_ARG;
  if (B < 2 || P < 1 || ldO < P) return VQMC_ERR_SHAPE;
  if (!O || !e_loc || !delta) return VQMC_ERR_ARG;
  const SrPlan pl = make_plan(B, P, o);
  if (!workspace || ws_bytes < pl.total) return VQMC_ERR_WORKSPACE;
  char *ws = reinterpret_cast<char *>(workspace);
  double *scal = reinterpret_cast<double *>(ws + pl.off_scal);
  int *status = reinterpret_cast<int *>(ws + pl.off_status);
  double *ec = reinterpret_cast<double *>(ws + pl.off_ec);
  double *obar = reinterpret_cast<double *>(ws + pl.off_obar);
  double *Fv = F ? F : reinterpret_cast<double *>(ws + pl.off_F);
  double *pa = reinterpret_cast<double *>(ws + pl.off_pa);
  double *pb = reinterpret_cast<double *>(ws + pl.off_pb);
  // <E>, Var E, E^c (and the Cholesky status cleared); <O>, F
  energy_stats_kernel<<<1, 1024, 0, st>>>(e_loc, B, ec, scal, status);
  const dim3 cgrid((unsigned)((P + 255) / 256), (unsigned)pl.nch);
  col_partial_kernel<false><<<cgrid, 256, 0, st>>>(O, ldO, B, P, nullptr, nullptr, ec, pl.rows_per_chunk, pa, pb,
                                                   nullptr);
  col_stats_finish_kernel<<<(unsigned)((P + 255) / 256), 256, 0, st>>>(pa, pb, pl.nch, P, B, scal, obar, Fv);
  VQMC_LAUNCH_CHECK();
  vqmc_status rc = VQMC_OK;
  if (pl.method == 1) {
    double *S = reinterpret_cast<double *>(ws + pl.off_M);
    const int64_t T = (P + 63) / 64;
    if (o->s_prec == 1)
      syrk_kernel<true><<<(unsigned)(T * (T + 1) / 2), 256, 0, st>>>(O, ldO, B, P, obar, o->eps, S);
    else
      syrk_kernel<false><<<(unsigned)(T * (T + 1) / 2), 256, 0, st>>>(O, ldO, B, P, obar, o->eps, S);
    VQMC_LAUNCH_CHECK();
    scale_copy_kernel<<<(unsigned)((P + 255) / 256), 256, 0, st>>>(Fv, P, 1.0, delta);
    rc = chol_solve(S, P, delta, status, st);
  } else if (pl.method == 3) {
    double *K = reinterpret_cast<double *>(ws + pl.off_M);
    double *alpha = reinterpret_cast<double *>(ws + pl.off_alpha);
    const int64_t T = (B + 63) / 64;
    gram_kernel<<<(unsigned)(T * (T + 1) / 2), 256, 0, st>>>(O, ldO, B, P, obar, o->eps, K);
    scale_copy_kernel<<<(unsigned)((B + 255) / 256), 256, 0, st>>>(ec, B, 1.0 / B, alpha);
    VQMC_LAUNCH_CHECK();
    rc = chol_solve(K, B, alpha, status, st);
    if (rc == VQMC_OK) {
      col_partial_kernel<true><<<cgrid, 256, 0, st>>>(O, ldO, B, P, obar, alpha, nullptr, pl.rows_per_chunk, pa,
                                                      nullptr, nullptr);
      col_sum_kernel<<<(unsigned)((P + 255) / 256), 256, 0, st>>>(pa, pl.nch, P, delta);
      VQMC_LAUNCH_CHECK();
    }
  } else {
    double *r = reinterpret_cast<double *>(ws + pl.off_r);
    double *p = reinterpret_cast<double *>(ws + pl.off_p);
    double *q = reinterpret_cast<double *>(ws + pl.off_q);
    double *u = reinterpret_cast<double *>(ws + pl.off_u);
    double *pq = reinterpret_cast<double *>(ws + pl.off_pq);
    cg_init_kernel<<<1, 1024, 0, st>>>(Fv, P, delta, r, p, scal);
    for (int it = 0; it < o->max_iter; ++it) {
      cg_rowdot_kernel<<<B, 256, 0, st>>>(O, ldO, P, obar, p, u, scal);
      col_partial_kernel<true><<<cgrid, 256, 0, st>>>(O, ldO, B, P, obar, u, nullptr, pl.rows_per_chunk, pa,
                                                      nullptr, scal);
      cg_apply_kernel<<<(unsigned)pl.npq, 256, 0, st>>>(pa, pl.nch, P, B, o->eps, p, q, pq, scal);
      cg_step_kernel<<<1, 1024, 0, st>>>(P, delta, r, p, q, pq, pl.npq, scal, o->tol);
    }
    VQMC_LAUNCH_CHECK();
  }
  if (rc != VQMC_OK) return rc;
  if (info) {
    double h[S_NSLOT];
    int hs[4];
    if (hipMemcpyAsync(h, scal, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess) return VQMC_ERR_DEVICE;
    if (hipMemcpyAsync(hs, status, sizeof(hs), hipMemcpyDeviceToHost, st) != hipSuccess) return VQMC_ERR_DEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return VQMC_ERR_DEVICE;
    info->e_mean = h[S_MEAN];
    info->e_var = h[S_VAR];
    info->iters = pl.method == 2 ? (int32_t)h[S_ITERS] : 0;
    info->rel_residual = pl.method == 2 ? h[S_REL] : 0.0;
    if (hs[0]) return VQMC_ERR_NOT_SPD;
    if (pl.method == 2 && h[S_DONE] == 0.0) return VQMC_WARN_NOT_CONVERGED;
  }
  return VQMC_OK;
}
