// chol.hip -- blocked Cholesky factorisation M = L L^T of an SPD matrix (FP64,
// lower triangle, in place) and the two triangular solves of the SR step
// (Sec. 3.2.2: the Cholesky factor followed by forward and back substitution
// instead of an explicit inverse of M).
//
// Right-looking, two block levels: 256-column outer panels, each factored as
// four 64-column sub-panels.  Per sub-panel: one wavefront factors the 64 x 64
// diagonal block and inverts its triangle; the rows below are then one GEMM
// with that small inverse; the rest of the outer panel is updated.  After each
// outer panel the trailing matrix receives one rank-256 update on the FP64
// matrix cores, so the trailing matrix is read and written once per 256
// columns.  The triangular solves use the stored 64 x 64 inverses: one launch
// per block row applies the inverse and updates the remaining right-hand side.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "chol.hpp"
#include "engine.hpp"
#include "tile128.hpp"

namespace vqmc {

namespace {

constexpr int CB = 64;   // diagonal block / sub-panel width
constexpr int OB = 256;  // outer panel width

__device__ __forceinline__ f64x4 mma64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, l);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Factor the 64 x 64 diagonal block at (c0, c0) and store its inverse.  One
// wavefront: lane i holds row i while factoring (right-looking, column by
// column), then lane c computes column c of L^-1 by forward substitution.
// Rows past n are padded with the identity.
__global__ __launch_bounds__(64) void chol_diag_kernel(double *__restrict__ M, int64_t n, int64_t c0,
                                                       double *__restrict__ Linv, int *__restrict__ status) {
  __shared__ double Ls[CB][CB + 1];
  __shared__ double rdiag[CB];
  const int i = threadIdx.x;
  const int m = (int)((n - c0) < CB ? (n - c0) : CB);
  double a[CB];
#pragma unroll
  for (int t = 0; t < CB; ++t)
    a[t] = (i < m && t <= i) ? M[(c0 + i) * n + c0 + t] : (i == t ? 1.0 : 0.0);
  bool bad = false;
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    double d = readlane_d(a[j], j);
    if (!(d > 0.0)) {
      bad = true;
      d = 1.0;
    }
    d = sqrt(d);
    const double rd = 1.0 / d;
    const double lij = i > j ? a[j] * rd : (i == j ? d : 0.0);
    a[j] = lij;
#pragma unroll
    for (int t = j + 1; t < CB; ++t) {
      const double ltj = readlane_d(lij, t);
      if (t <= i) a[t] -= lij * ltj;
    }
  }
  if (bad && i == 0) *status = 1;
#pragma unroll
  for (int t = 0; t < CB; ++t) {
    Ls[i][t] = t <= i ? a[t] : 0.0;
    if (i < m && t <= i) M[(c0 + i) * n + c0 + t] = a[t];
  }
  rdiag[i] = 1.0 / Ls[i][i];
  __syncthreads();
  const int c = i;
  double x[CB];
#pragma unroll
  for (int r = 0; r < CB; ++r) {
    double v = r == c ? 1.0 : 0.0;
#pragma unroll
    for (int t = 0; t < r; ++t) v -= Ls[r][t] * x[t];
    x[r] = v * rdiag[r];
  }
#pragma unroll
  for (int r = 0; r < CB; ++r) Linv[r * CB + c] = x[r];
}

// Rows below the diagonal block: L[r][c0..c0+63] = A[r][c0..] * Linv^T, 64
// rows per workgroup (4 waves x 16 rows, 4 column tiles each).
__global__ __launch_bounds__(256) void chol_trsm_kernel(double *__restrict__ M, int64_t n, int64_t c0,
                                                       const double *__restrict__ Linv) {
  __shared__ double sA[CB][CB + 1];
  __shared__ double sL[CB][CB + 1];
  const int64_t r0 = c0 + CB + (int64_t)blockIdx.x * CB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int idx = tid; idx < CB * CB; idx += 256) {
    const int r = idx / CB, t = idx - r * CB;
    sA[r][t] = (r0 + r < n) ? M[(r0 + r) * n + c0 + t] : 0.0;
    sL[r][t] = Linv[idx];
  }
  __syncthreads();
  f64x4 acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = f64x4{0, 0, 0, 0};
#pragma unroll 4
  for (int ks = 0; ks < CB / 4; ++ks) {
    const int k = ks * 4 + (lane >> 4);
    const double a = sA[wave * 16 + (lane & 15)][k];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] = mma64(a, sL[q * 16 + (lane & 15)][k], acc[q]);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + wave * 16 + (lane >> 4) + 4 * r;
      if (row < n) M[row * n + c0 + q * 16 + (lane & 15)] = acc[q][r];
    }
}

// Shared body: C[r][c] -= sum_t A[r][t] B[c][t] for one 64 x 64 tile, K taken
// in 64-wide chunks from columns k0..k1 of M, lower triangle only.
__device__ __forceinline__ void tile_syrk(double *__restrict__ M, int64_t n, int64_t r0, int64_t cc0,
                                          int64_t k0, int64_t k1, int64_t cmax,
                                          double (*sR)[CB + 1], double (*sC)[CB + 1]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0, 0, 0, 0};
  for (int64_t kc = k0; kc < k1; kc += CB) {
    const int kw = (int)((k1 - kc) < CB ? (k1 - kc) : CB);
    for (int idx = tid; idx < CB * CB; idx += 256) {
      const int r = idx / CB, t = idx - r * CB;
      sR[r][t] = (r0 + r < n && t < kw) ? M[(r0 + r) * n + kc + t] : 0.0;
      sC[r][t] = (cc0 + r < n && t < kw) ? M[(cc0 + r) * n + kc + t] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int ks = 0; ks < CB / 4; ++ks) {
      const int k = ks * 4 + (lane >> 4);
      double a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = sR[wm * 32 + t * 16 + (lane & 15)][k];
        b[t] = sC[wn * 32 + t * 16 + (lane & 15)][k];
      }
#pragma unroll
      for (int tm = 0; tm < 2; ++tm)
#pragma unroll
        for (int tn = 0; tn < 2; ++tn) acc[tm][tn] = mma64(a[tm], b[tn], acc[tm][tn]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int tm = 0; tm < 2; ++tm)
#pragma unroll
    for (int tn = 0; tn < 2; ++tn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + wm * 32 + tm * 16 + (lane >> 4) + 4 * r;
        const int64_t col = cc0 + wn * 32 + tn * 16 + (lane & 15);
        if (row < n && col < cmax && col <= row) M[row * n + col] -= acc[tm][tn][r];
      }
}

// Remaining columns of the outer panel after sub-panel c0:
// A[r][c] -= sum_t L[r][c0+t] L[c][c0+t] for c in [c0+64, cend), r >= c.
__global__ __launch_bounds__(256) void chol_panel_update_kernel(double *__restrict__ M, int64_t n, int64_t c0,
                                                                int64_t cend) {
  __shared__ double sR[CB][CB + 1];
  __shared__ double sC[CB][CB + 1];
  const int64_t cc0 = c0 + CB + (int64_t)blockIdx.x * CB;
  const int64_t r0 = c0 + CB + (int64_t)blockIdx.y * CB;
  if (cc0 > r0 + CB - 1) return;  // tile strictly above the diagonal
  tile_syrk(M, n, r0, cc0, c0, c0 + CB, cend, sR, sC);
}

// Trailing matrix after the outer panel [p0, p1): lower 128 x 128 tiles,
// M[r][c] -= sum_{t in [p0,p1)} L[r][t] L[c][t].
__global__ __launch_bounds__(256, 2) void chol_trailing_kernel(double *__restrict__ M, int64_t n, int64_t p0,
                                                            int64_t p1) {
  constexpr int KC = 32;
  __shared__ double sR[128][KC + 1];
  __shared__ double sC[128][KC + 1];
  using TT = Tile128<double>;
  int bi, bj;
  lower_block(blockIdx.x, bi, bj);
  const int64_t r0 = p1 + (int64_t)bi * 128, c0 = p1 + (int64_t)bj * 128;
  TT::acc_t acc[4][4];
  TT::zero(acc);
  for (int64_t kc = p0; kc < p1; kc += KC) {
    const int kw = (int)((p1 - kc) < KC ? (p1 - kc) : KC);
#pragma unroll 4
    for (int idx = threadIdx.x; idx < 128 * KC; idx += 256) {
      const int r = idx / KC, t = idx - r * KC;
      sR[r][t] = (r0 + r < n && t < kw) ? M[(r0 + r) * n + kc + t] : 0.0;
      sC[r][t] = (c0 + r < n && t < kw) ? M[(c0 + r) * n + kc + t] : 0.0;
    }
    __syncthreads();
    TT::step<KC, KC + 1>(sR, sC, acc);
    __syncthreads();
  }
#pragma unroll
  for (int tm = 0; tm < 4; ++tm)
#pragma unroll
    for (int tn = 0; tn < 4; ++tn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + TT::row_of(tm, r), col = c0 + TT::col_of(tn);
        if (row < n && col <= row) M[row * n + col] -= acc[tm][tn][r];
      }
}

// Forward substitution for block kb: y_kb = Linv_kb rhs_kb (every workgroup
// computes it; workgroup 0 stores it), then rhs_r -= L[r][kb] . y_kb for the
// rows below, one row per thread.
__global__ __launch_bounds__(256) void chol_fwd_kernel(const double *__restrict__ M, int64_t n, int kb,
                                                      const double *__restrict__ Linv, double *__restrict__ rhs,
                                                      double *__restrict__ y) {
  __shared__ double sr[CB];
  __shared__ double sy[CB];
  const int64_t o = (int64_t)kb * CB;
  const int m = (int)((n - o) < CB ? (n - o) : CB);
  const int tid = threadIdx.x;
  if (tid < CB) sr[tid] = tid < m ? rhs[o + tid] : 0.0;
  __syncthreads();
  if (tid < CB) {
    double s = 0.0;
    for (int t = 0; t <= tid; ++t) s += Linv[(int64_t)kb * CB * CB + tid * CB + t] * sr[t];
    sy[tid] = s;
    if (blockIdx.x == 0 && tid < m) y[o + tid] = s;
  }
  __syncthreads();
  const int64_t r = o + CB + (int64_t)blockIdx.x * 256 + tid;
  if (r >= n) return;
  const double *a = M + r * n + o;
  double s = 0.0;
#pragma unroll 8
  for (int t = 0; t < CB; ++t) s += a[t] * sy[t];
  rhs[r] -= s;
}

// Back substitution for block kb: x_kb = Linv_kb^T rhs_kb, then
// rhs_t -= sum_i L[kb*64+i][t] x_i for t above the block.
__global__ __launch_bounds__(256) void chol_bwd_kernel(const double *__restrict__ M, int64_t n, int kb,
                                                      const double *__restrict__ Linv, double *__restrict__ rhs,
                                                      double *__restrict__ x) {
  __shared__ double sr[CB];
  __shared__ double sx[CB];
  const int64_t o = (int64_t)kb * CB;
  const int m = (int)((n - o) < CB ? (n - o) : CB);
  const int tid = threadIdx.x;
  if (tid < CB) sr[tid] = tid < m ? rhs[o + tid] : 0.0;
  __syncthreads();
  if (tid < CB) {
    double s = 0.0;
    for (int r = tid; r < CB; ++r) s += Linv[(int64_t)kb * CB * CB + r * CB + tid] * sr[r];
    sx[tid] = s;
    if (blockIdx.x == 0 && tid < m) x[o + tid] = s;
  }
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * 256 + tid;
  if (t >= o) return;
  double s = 0.0;
  for (int i = 0; i < m; ++i) s += M[(o + i) * n + t] * sx[i];
  rhs[t] -= s;
}

}  // namespace

size_t chol_workspace_bytes(int64_t n) {
  const int64_t nb = (n + CB - 1) / CB;
  return (size_t)nb * CB * CB * 8 + (size_t)n * 8;
}

vqmc_status chol_factor_solve(double *M, int64_t n, double *rhs, double *x, void *ws, int *status,
                              hipStream_t st) {
  const int64_t nb = (n + CB - 1) / CB;
  double *Linv = reinterpret_cast<double *>(ws);
  double *y = Linv + nb * CB * CB;
  for (int64_t p0 = 0; p0 < n; p0 += OB) {
    const int64_t p1 = (p0 + OB) < n ? p0 + OB : n;
    for (int64_t c0 = p0; c0 < p1; c0 += CB) {
      chol_diag_kernel<<<1, 64, 0, st>>>(M, n, c0, Linv + (c0 / CB) * CB * CB, status);
      const int64_t below = n - (c0 + CB);
      if (below > 0) {
        chol_trsm_kernel<<<(unsigned)((below + CB - 1) / CB), 256, 0, st>>>(M, n, c0, Linv + (c0 / CB) * CB * CB);
        const int64_t rest = p1 - (c0 + CB);
        if (rest > 0) {
          const dim3 g((unsigned)((rest + CB - 1) / CB), (unsigned)((below + CB - 1) / CB));
          chol_panel_update_kernel<<<g, 256, 0, st>>>(M, n, c0, p1);
        }
      }
    }
    if (p1 < n) {
      const int64_t T = (n - p1 + 127) / 128;
      chol_trailing_kernel<<<(unsigned)(T * (T + 1) / 2), 256, 0, st>>>(M, n, p0, p1);
    }
  }
  if (hipGetLastError() != hipSuccess) return VQMC_ERR_DEVICE;
  for (int64_t kb = 0; kb < nb; ++kb) {
    const int64_t below = n - (kb + 1) * CB;
    const unsigned g = below > 0 ? (unsigned)((below + 255) / 256) : 1u;
    chol_fwd_kernel<<<g, 256, 0, st>>>(M, n, (int)kb, Linv, rhs, y);
  }
  for (int64_t kb = nb - 1; kb >= 0; --kb) {
    const int64_t above = kb * CB;
    const unsigned g = above > 0 ? (unsigned)((above + 255) / 256) : 1u;
    chol_bwd_kernel<<<g, 256, 0, st>>>(M, n, (int)kb, Linv, y, x);
  }
  if (hipGetLastError() != hipSuccess) return VQMC_ERR_DEVICE;
  return VQMC_OK;
}

}  // namespace vqmc
