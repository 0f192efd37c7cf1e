// chol.hip -- blocked Cholesky factorisation M = L L^T of an SPD matrix (FP64,
// lower triangle, in place) and the two triangular solves of the SR step
// (Sec. 3.2.2: the Cholesky factor followed by forward and back substitution
// instead of an explicit inverse of M).
//
// Two block levels: 512-column outer panels, right-looking between them (after
// each outer panel the trailing matrix receives one rank-512 update on the
// FP64 matrix cores, so it is read and written once per 512 columns), and
// left-looking inside them over 64-column sub-panels.  A workgroup factors a
// 64 x 64 diagonal block and, in the same sweep, inverts its triangle; the
// rows below are then one GEMM with that small inverse.  One launch per
// sub-panel after the first does the previous sub-panel's row solve, the
// left-looking update of its own columns and the factorisation of its own
// diagonal block (by the workgroup that updated it), so that the chain of
// dependent launches, which competes with the concurrent trailing update for
// compute units, is one launch per 64 columns.  After an outer panel, the
// update of the next panel's columns runs on the caller's stream (its first
// tile's workgroup then factors the next panel's first diagonal block) and
// the rest of the trailing update on a side stream, overlapping the next
// panel's chain.
//
// The right-hand side rides along as an extra last row of the matrix: the
// factorisation of [[M, r], [r^T, *]] leaves y = L^-1 r in that row, so the
// forward substitution costs no launches of its own.  The back substitution
// goes by 256-row blocks: one workgroup solves the block with the stored
// 64 x 64 inverses, then one launch applies it to the rest of y.
//
// Only the lower triangle (row >= column) of M is read or written, except
// that the trailing update may also write the strict upper part of diagonal
// tiles, which nothing reads.  Row stride ld is even (16-byte rows).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <mutex>
#include <type_traits>

#include "chol.hpp"
#include "engine.hpp"
#include "tile128.hpp"

namespace vqmc {

namespace {

constexpr int CB = 64;   // diagonal block / sub-panel width
constexpr int OB = 512;  // outer panel width
constexpr int SB = 256;  // block of the triangular solves

__device__ __forceinline__ f64x4 mma64(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int64_t clamp_row(int64_t r, int64_t n) { return r < n ? r : n - 1; }

typedef double f64x2 __attribute__((ext_vector_type(2)));

// 1/d to full double precision from the hardware reciprocal and two Newton
// steps (d > 0 and normal).
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  r = fma(r, fma(-d, r, 1.0), r);
  return fma(r, fma(-d, r, 1.0), r);
}

// Factor the 64 x 64 diagonal block at (c0, c0) and store the inverse of its
// factor.  256 threads, each holding a 4 x 4 block of the working matrix Z in
// registers.  The lower triangle of Z is the block being factored; its strict
// upper triangle holds the transpose of Y, the unscaled inverse being built
// by Gauss-Jordan elimination on [L | I].  With d_j the j-th pivot and u the
// column j of Z (u_j replaced by 1), step j is the single rank-1 update
//   Z[x][y] -= u_x u_y / d_j   for y > j and (x >= y or x <= j),
// which covers both the trailing Schur complement (x >= y > j) and the
// elimination of column j from the inverse (x <= j < y).  Afterwards
// L[x][y] = Z[x][y] / sqrt(d_y) (x >= y) and Linv[y][x] = Z[x][y] / sqrt(d_y)
// (x < y), Linv[y][y] = 1 / sqrt(d_y).  One barrier per column: the owners of
// column j+1 update and publish it first, and everyone finishes the other
// columns of step j after the barrier.  Rows past n are padded with the
// identity.
__device__ __forceinline__ void diag_factor(double *__restrict__ M, int64_t n, int64_t ld, int64_t c0,
                                            double *__restrict__ Linv, int *__restrict__ status,
                                            double (*colbuf)[CB]) {
  const int tid = threadIdx.x, bx = tid >> 4, by = tid & 15;
  const int x0 = 4 * bx, y0 = 4 * by;
  const int m = (int)((n - c0) < CB ? (n - c0) : CB);
  const bool lowblk = bx > by, upblk = bx < by;
  double z[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int x = x0 + a, y = y0 + b;
      const int xr = x < m ? x : m - 1, yr = y < m ? y : m - 1;
      const double v = M[(c0 + xr) * ld + c0 + yr];
      z[a][b] = x < y ? 0.0 : (x < m ? v : (x == y ? 1.0 : 0.0));
    }
  if (by == 0)
#pragma unroll
    for (int a = 0; a < 4; ++a) colbuf[0][x0 + a] = z[a][0];
  __syncthreads();
  double dcol[4] = {1.0, 1.0, 1.0, 1.0};
  bool bad = false;
  double rlo[4], rhi[4], cf[4];
  // Steps go in groups of four pivots j = 4g + t.  Whether row x0 + a lies
  // at or above pivot j and whether column y0 + a lies past it depend, within
  // a group, only on how bx and by compare with g and on a against t, so the
  // masks of the update are 0/1 factors set once per group and picked at
  // compile time: m_le / m_lt = [bx <= g] / [bx < g], c_ge / c_gt likewise
  // for by; rows of upper blocks take the upper coefficient (x <= j only),
  // rows of lower blocks the lower one (all rows), diagonal blocks by b <= a.
  double m_le, m_lt, c_ge, c_gt, kA_le, kA_lt, kB_le, kB_lt;
  bool xpiv;
  // step j = 4g + t, with column B1 = (t + 1) % 4 of this thread's block done first
  auto step = [&](int g, auto tc, auto b1c) {
    constexpr int T = decltype(tc)::value, B1 = decltype(b1c)::value;
    const int j = 4 * g + T;
    const double *v = colbuf[T & 1];
    double vx[4], vy[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      vx[a] = v[x0 + a];
      vy[a] = v[y0 + a];
    }
    double d = v[j];
    if (!(d > 0.0)) {
      bad = true;
      d = 1.0;
    }
    if (by == g) dcol[T] = d;
    const double q = recip(d);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const double rl = (a == T && xpiv ? 1.0 : vx[a]) * q;
      rlo[a] = rl * (a <= T ? kA_le : kA_lt);
      rhi[a] = rl * (a <= T ? kB_le : kB_lt);
      cf[a] = vy[a] * (a > T ? c_ge : c_gt);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) z[a][B1] -= (B1 <= a ? rlo[a] : rhi[a]) * cf[B1];
    if (T < 3 ? by == g : (g + 1 < CB / 4 && by == g + 1))
#pragma unroll
      for (int a = 0; a < 4; ++a) colbuf[(T + 1) & 1][x0 + a] = z[a][B1];
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (b != B1) z[a][b] -= (b <= a ? rlo[a] : rhi[a]) * cf[b];
  };
  for (int g = 0; g < CB / 4; ++g) {
    m_le = bx <= g ? 1.0 : 0.0;
    m_lt = bx < g ? 1.0 : 0.0;
    c_ge = by >= g ? 1.0 : 0.0;
    c_gt = by > g ? 1.0 : 0.0;
    kA_le = upblk ? m_le : 1.0;
    kA_lt = upblk ? m_lt : 1.0;
    kB_le = lowblk ? 1.0 : m_le;
    kB_lt = lowblk ? 1.0 : m_lt;
    xpiv = bx == g;
    step(g, std::integral_constant<int, 0>{}, std::integral_constant<int, 1>{});
    step(g, std::integral_constant<int, 1>{}, std::integral_constant<int, 2>{});
    step(g, std::integral_constant<int, 2>{}, std::integral_constant<int, 3>{});
    step(g, std::integral_constant<int, 3>{}, std::integral_constant<int, 0>{});
  }
  if (bad && tid == 0) *status = 1;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int y = y0 + b;
    const double sd = sqrt(dcol[b]), rs = 1.0 / sd;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int x = x0 + a;
      if (x > y) {
        if (x < m) M[(c0 + x) * ld + c0 + y] = z[a][b] * rs;
        Linv[y * CB + x] = 0.0;
      } else if (x == y) {
        if (x < m) M[(c0 + x) * ld + c0 + y] = sd;
        Linv[y * CB + y] = rs;
      } else {
        Linv[y * CB + x] = z[a][b] * rs;
      }
    }
  }
}

// side (nullable): receives rows c0 + 64 .. c0 + 127 of the block's columns
// as they are before this sub-panel's row solve (rows past the last one of the
// augmented matrix repeat it).
__global__ __launch_bounds__(256) void chol_diag_kernel(double *__restrict__ M, int64_t n, int64_t ld, int64_t c0,
                                                       double *__restrict__ Linv, int *__restrict__ status,
                                                       double *__restrict__ side) {
  __builtin_amdgcn_s_setprio(3);
  __shared__ double colbuf[2][CB];
  if (side)
    for (int idx = threadIdx.x; idx < CB * CB; idx += 256) {
      const int r = idx >> 6, t = idx & 63;
      side[idx] = M[clamp_row(c0 + CB + r, n + 1) * ld + c0 + t];
    }
  diag_factor(M, n, ld, c0, Linv, status, colbuf);
}

// Stage a 64 x 64 block of doubles (rows r0.. clamped to nr, columns
// k0..k0+63) into LDS: 8 16-byte loads per thread, all issued before the
// first store.
__device__ __forceinline__ void stage64(const double *__restrict__ src, int64_t ld, int64_t r0, int64_t nr,
                                        int64_t k0, double (*dst)[CB + 2]) {
  f64x2 v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int idx = threadIdx.x + 256 * q, r = idx >> 5, j = idx & 31;
    v[q] = *reinterpret_cast<const f64x2 *>(src + clamp_row(r0 + r, nr) * ld + k0 + 2 * j);
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int idx = threadIdx.x + 256 * q, r = idx >> 5, j = idx & 31;
    *reinterpret_cast<f64x2 *>(&dst[r][2 * j]) = v[q];
  }
}

// The same for a block of only kw < 64 valid columns (the last diagonal
// block): columns past kw are zero.
__device__ __forceinline__ void stage64_partial(const double *__restrict__ src, int64_t ld, int64_t r0, int64_t nr,
                                                int64_t k0, int kw, double (*dst)[CB + 2]) {
  double v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = threadIdx.x + 256 * q, r = idx >> 6, t = idx & 63;
    v[q] = src[clamp_row(r0 + r, nr) * ld + k0 + (t < kw ? t : kw - 1)];
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = threadIdx.x + 256 * q, r = idx >> 6, t = idx & 63;
    dst[r][t] = t < kw ? v[q] : 0.0;
  }
}

// Rows below the diagonal block of width m: L[r][c0..c0+m) = A[r][c0..] Linv^T
// Stages rows r0 .. r0+63 of src (clamped to nr - 1), columns k0 .. k0+31,
// into dst; columns at or past kend are zero (FULL: all 32 are inside).
constexpr int KH = 32;  // K chunk of the panel kernels (34.8 KB of LDS for two tiles)
template <bool FULL>
__device__ __forceinline__ void stage32(const double *__restrict__ src, int64_t ld, int64_t r0, int64_t nr,
                                        int64_t k0, int64_t kend, double (*dst)[KH + 2]) {
  if constexpr (FULL) {
    f64x2 v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = threadIdx.x + 256 * q, r = idx >> 4, j = idx & 15;
      v[q] = *reinterpret_cast<const f64x2 *>(src + clamp_row(r0 + r, nr) * ld + k0 + 2 * j);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = threadIdx.x + 256 * q, r = idx >> 4, j = idx & 15;
      *reinterpret_cast<f64x2 *>(&dst[r][2 * j]) = v[q];
    }
  } else {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int idx = threadIdx.x + 256 * q, r = idx >> 5, t = idx & 31;
      const int64_t c = k0 + t < kend ? k0 + t : kend - 1;
      v[q] = src[clamp_row(r0 + r, nr) * ld + c];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int idx = threadIdx.x + 256 * q, r = idx >> 5, t = idx & 31;
      dst[r][t] = k0 + t < kend ? v[q] : 0.0;
    }
  }
}

// for r in [c0+m, nr), 64 rows per workgroup (4 waves x 16 rows, 4 column
// tiles each).  The last row of the augmented matrix is included, so this is
// also the forward substitution step of that block.
template <bool FULL>
__global__ __launch_bounds__(256) void chol_trsm_kernel(double *__restrict__ M, int64_t nr, int64_t ld, int64_t c0,
                                                       int m, const double *__restrict__ Linv) {
  __shared__ double sA[CB][KH + 2];
  __shared__ double sL[CB][KH + 2];
  const int64_t r0 = c0 + m + (int64_t)blockIdx.x * CB;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  f64x4 acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = f64x4{0, 0, 0, 0};
#pragma unroll
  for (int h = 0; h < CB / KH; ++h) {
    stage32<FULL>(M, ld, r0, nr, c0 + KH * h, c0 + m, sA);
    stage32<true>(Linv, CB, 0, CB, KH * h, CB, sL);
    __syncthreads();
#pragma unroll 4
    for (int ks = 0; ks < KH / 4; ++ks) {
      const int k = ks * 4 + (lane >> 4);
      const double a = sA[wave * 16 + (lane & 15)][k];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = mma64(a, sL[q * 16 + (lane & 15)][k], acc[q]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + wave * 16 + (lane >> 4) + 4 * r;
      const int col = q * 16 + (lane & 15);
      if (row < nr && col < m) M[row * ld + c0 + col] = acc[q][r];
    }
}

// One step of the factorisation of an outer panel [p0, ...): the row solve
// of sub-panel c0 (whose diagonal block is factored, its inverse in Linv0)
// fused with the left-looking update and the factorisation of the next
// sub-panel c1 = c0 + 64.  Workgroup b takes rows R = [c1 + 64 b, +64):
//   1. L0[R] = M[R][c0 blk] Linv0^T (written to M), and, recomputed by every
//      workgroup, L0[C] for the rows C = [c1, +64) from side_in (the values
//      of M[C][c0 blk] before this launch, which workgroup 0 overwrites);
//   2. M[R][c] -= sum_{k in [p0, c1)} L[R][k] L[C][k] for c in [c1, cend),
//      r >= c, r < nr: the c0 block from 1., earlier blocks from M;
//      workgroup 1 also copies its updated rows to side_out for the next step;
//   3. workgroup 0 factors the diagonal block of c1 (inverse into Linv1).
__global__ __launch_bounds__(256) void chol_step_kernel(double *__restrict__ M, int64_t nr, int64_t ld, int64_t p0,
                                                        int64_t c0, int64_t cend,
                                                        const double *__restrict__ Linv0,
                                                        double *__restrict__ Linv1, int *__restrict__ status,
                                                        const double *__restrict__ side_in,
                                                        double *__restrict__ side_out) {
  // the panel chain's waves issue ahead of the concurrent trailing update's
  // on a shared compute unit
  __builtin_amdgcn_s_setprio(3);
  __shared__ double sX[CB][CB + 2];
  __shared__ double sY[CB][CB + 2];
  __shared__ double colbuf[2][CB];
  const int64_t c1 = c0 + CB;
  const int64_t r0 = c1 + (int64_t)blockIdx.x * CB;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // ---- 1. row solve of sub-panel c0 for R and C, in two 32-column halves:
  // sX[.][0, 32) = M[R] half, sX[.][34, 66) = Linv0 half, sY[.][0, 32) = side_in half
  f64x4 aR[4], aC[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) aR[q] = aC[q] = f64x4{0, 0, 0, 0};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int idx = threadIdx.x + 256 * q, r = idx >> 4, j = idx & 15;
      const f64x2 vr = *reinterpret_cast<const f64x2 *>(M + clamp_row(r0 + r, nr) * ld + c0 + KH * h + 2 * j);
      const f64x2 vl = *reinterpret_cast<const f64x2 *>(Linv0 + r * CB + KH * h + 2 * j);
      const f64x2 vc = *reinterpret_cast<const f64x2 *>(side_in + r * CB + KH * h + 2 * j);
      *reinterpret_cast<f64x2 *>(&sX[r][2 * j]) = vr;
      *reinterpret_cast<f64x2 *>(&sX[r][KH + 2 + 2 * j]) = vl;
      *reinterpret_cast<f64x2 *>(&sY[r][2 * j]) = vc;
    }
    __syncthreads();
    if (blockIdx.x == 0) {
      // R = C here, and M[C] holds what side_in holds: L0[C] = L0[R]
#pragma unroll 4
      for (int ks = 0; ks < KH / 4; ++ks) {
        const int k = ks * 4 + (lane >> 4);
        const double ar = sX[wave * 16 + (lane & 15)][k];
#pragma unroll
        for (int q = 0; q < 4; ++q) aR[q] = mma64(ar, sX[q * 16 + (lane & 15)][KH + 2 + k], aR[q]);
      }
    } else {
#pragma unroll 4
      for (int ks = 0; ks < KH / 4; ++ks) {
        const int k = ks * 4 + (lane >> 4);
        const double ar = sX[wave * 16 + (lane & 15)][k];
        const double ac = sY[wave * 16 + (lane & 15)][k];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double l = sX[q * 16 + (lane & 15)][KH + 2 + k];
          aR[q] = mma64(ar, l, aR[q]);
          aC[q] = mma64(ac, l, aC[q]);
        }
      }
    }
    __syncthreads();
  }
  if (blockIdx.x == 0)
#pragma unroll
    for (int q = 0; q < 4; ++q) aC[q] = aR[q];
  // L0[R] to M and to sX, L0[C] to sY (row-major [row][k], k in the c0 block)
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int lr = wave * 16 + (lane >> 4) + 4 * r, col = q * 16 + (lane & 15);
      const int64_t row = r0 + lr;
      if (row < nr) M[row * ld + c0 + col] = aR[q][r];
      sX[lr][col] = aR[q][r];
      sY[lr][col] = aC[q][r];
    }
  __syncthreads();
  // ---- 2. left-looking update of the c1 block: first the c0 block ...
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0, 0, 0, 0};
  auto mma_block = [&](int kw) {
    for (int ks = 0; ks < kw / 4; ++ks) {
      const int k = ks * 4 + (lane >> 4);
      double a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = sX[wm * 32 + t * 16 + (lane & 15)][k];
        b[t] = sY[wn * 32 + t * 16 + (lane & 15)][k];
      }
#pragma unroll
      for (int tm = 0; tm < 2; ++tm)
#pragma unroll
        for (int tn = 0; tn < 2; ++tn) acc[tm][tn] = mma64(a[tm], b[tn], acc[tm][tn]);
    }
  };
  mma_block(CB);
  __syncthreads();
  // ... then the earlier blocks of the outer panel, 64 columns at a time
  // (the next chunk loaded into registers while the current one is used)
  auto load = [&](f64x2 (&v)[8], int64_t rb, int64_t k0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int idx = threadIdx.x + 256 * q, r = idx >> 5, j = idx & 31;
      v[q] = *reinterpret_cast<const f64x2 *>(M + clamp_row(rb + r, nr) * ld + k0 + 2 * j);
    }
  };
  auto store = [&](const f64x2 (&v)[8], double (*dst)[CB + 2]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int idx = threadIdx.x + 256 * q, r = idx >> 5, j = idx & 31;
      *reinterpret_cast<f64x2 *>(&dst[r][2 * j]) = v[q];
    }
  };
  if (c0 > p0) {
    f64x2 vr[8], vc[8];
    load(vr, r0, p0);
    load(vc, c1, p0);
    for (int64_t k0 = p0; k0 < c0; k0 += CB) {
      store(vr, sX);
      store(vc, sY);
      __syncthreads();
      if (k0 + CB < c0) {
        load(vr, r0, k0 + CB);
        load(vc, c1, k0 + CB);
      }
      mma_block(CB);
      __syncthreads();
    }
  }
  // M[R][c1 blk] -= acc (lower triangle, existing rows and columns)
#pragma unroll
  for (int tm = 0; tm < 2; ++tm)
#pragma unroll
    for (int tn = 0; tn < 2; ++tn) {
      const int lc = wn * 32 + tn * 16 + (lane & 15);
      const int64_t col = c1 + lc;
      double cur[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + wm * 32 + tm * 16 + (lane >> 4) + 4 * r;
        cur[r] = M[clamp_row(row, nr) * ld + (col < cend ? col : c1)];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int lr = wm * 32 + tm * 16 + (lane >> 4) + 4 * r;
        const int64_t row = r0 + lr;
        const double v = cur[r] - acc[tm][tn][r];
        if (row < nr && col < cend && col <= row) M[row * ld + col] = v;
        if (blockIdx.x == 1 && side_out) side_out[lr * CB + lc] = v;
      }
    }
  // ---- 3. the workgroup of the diagonal block factors it
  if (blockIdx.x == 0) {
    __syncthreads();
    diag_factor(M, nr - 1, ld, c1, Linv1, status, colbuf);
  }
}

// Loader of the trailing update: rows ra0.. (A side) or rb0.. (B side) of M,
// columns k0 + KC c .. +KC-1 for chunk c; rows past nr are clamped (they only
// feed outputs that are not stored).
template <int KC>
struct TrailLoader {
  static constexpr int HALF = KC / 2, NQ = KC / 4;  // f64x2 per row, per thread
  const double *M;
  int64_t ld, nr, ra0, rb0, k0;
  struct Regs {
    f64x2 v[NQ];
  };
  __device__ __forceinline__ void load(Regs &r, int c, bool bside) const {
    const int64_t base = bside ? rb0 : ra0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int idx = threadIdx.x + 256 * q, m = idx / HALF, j = idx % HALF;
      r.v[q] = *reinterpret_cast<const f64x2 *>(M + clamp_row(base + m, nr) * ld + k0 + KC * c + 2 * j);
    }
  }
  __device__ __forceinline__ void store(const Regs &r, Panel<double, KC, false> &P) const {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int idx = threadIdx.x + 256 * q, m = idx / HALF, j = idx % HALF;
      *reinterpret_cast<f64x2 *>(&P.s[m][2 * j]) = r.v[q];
    }
  }
};

// Trailing matrix after the outer panel [p0, p1) (p1 - p0 = OB) past the next
// outer panel: 128 x 128 tiles of rows and columns from p1 + OB on or below
// the diagonal, M[r][c] -= sum_{t in [p0,p1)} L[r][t] L[c][t].  Tile t is
// (bi, bj) of that lower block triangle.
__global__ __launch_bounds__(256, 2) void chol_trailing_kernel(double *__restrict__ M, int64_t n, int64_t nr,
                                                            int64_t ld, int64_t p0, int64_t p1, int ntiles,
                                                            int nchunks) {
  constexpr int KC = 16;
  __shared__ Panel<double, KC, false> sA, sB;
  using TT = Tile128<double>;
  int bi, bj;
  lower_block(xcd_contiguous(blockIdx.x, ntiles), bi, bj);
  const int64_t r0 = p1 + OB + (int64_t)bi * 128, c0 = p1 + OB + (int64_t)bj * 128;
  // the extra block row of the augmented matrix past the last column
  // (uniform per workgroup)
  if (c0 >= n) return;
  TrailLoader<KC> ldr{M, ld, nr, r0, c0, p0};
  TT::acc_t acc[4][4];
  TT::zero(acc);
  TT::run<KC, false>(ldr, nchunks, sA, sB, acc);
#pragma unroll
  for (int tm = 0; tm < 4; ++tm)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + TT::row_of(tm, r);
      double *rp = M + clamp_row(row, nr) * ld + c0;
      double cur[4];
#pragma unroll
      for (int tn = 0; tn < 4; ++tn) {
        const int col = TT::col_of(tn);
        cur[tn] = rp[c0 + col < n ? col : 0];
      }
#pragma unroll
      for (int tn = 0; tn < 4; ++tn) {
        const int col = TT::col_of(tn);
        if (row < nr && c0 + col < n) rp[col] = cur[tn] - acc[tm][tn][r];
      }
    }
}

// The columns of the next outer panel, [p1, p1 + OB), in 64 x 64 tiles:
// M[r][c] -= sum_{t in [p0, p1)} L[r][t] L[c][t] for rows r in [p1, nr) and
// c <= r (diagonal tiles also write their strict upper part, which nothing
// reads).  This update lies on the chain between two outer panels; with four
// times as many workgroups as 128 x 128 tiles it fills the device also when
// few rows remain.  Tile t = (t / ncb, t % ncb); K in chunks of 64 columns,
// the next chunk loaded into registers while the matrix cores use the
// current one.  The workgroup of tile (0, 0), the next panel's first
// diagonal block, then factors that block (inverse into Linv1), and the one of
// tile (1, 0) copies its rows to side (nullable) for the next panel's first
// step, as the panel's diagonal-block launch does for the first panel.
__global__ __launch_bounds__(256, 2) void chol_next_panel_kernel(double *__restrict__ M, int64_t n, int64_t nr,
                                                               int64_t ld, int64_t p0, int64_t p1, int ncb,
                                                               double *__restrict__ Linv1, int *__restrict__ status,
                                                               double *__restrict__ side) {
  __shared__ double sX[CB][CB + 2];
  __shared__ double sY[CB][CB + 2];
  __builtin_amdgcn_s_setprio(3);  // on the chain between two outer panels
  const int bi = (int)blockIdx.x / ncb, bj = (int)blockIdx.x - bi * ncb;
  const int64_t r0 = p1 + (int64_t)bi * CB, c0 = p1 + (int64_t)bj * CB;
  if (bj > bi || c0 >= n) return;  // uniform per workgroup
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  auto load = [&](f64x2 (&v)[8], int64_t rb, int64_t k0) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int idx = threadIdx.x + 256 * q, r = idx >> 5, j = idx & 31;
      v[q] = *reinterpret_cast<const f64x2 *>(M + clamp_row(rb + r, nr) * ld + k0 + 2 * j);
    }
  };
  auto store = [&](const f64x2 (&v)[8], double (*dst)[CB + 2]) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int idx = threadIdx.x + 256 * q, r = idx >> 5, j = idx & 31;
      *reinterpret_cast<f64x2 *>(&dst[r][2 * j]) = v[q];
    }
  };
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0, 0, 0, 0};
  f64x2 vr[8], vc[8];
  load(vr, r0, p0);
  load(vc, c0, p0);
  for (int64_t k0 = p0; k0 < p1; k0 += CB) {
    store(vr, sX);
    store(vc, sY);
    __syncthreads();
    if (k0 + CB < p1) {
      load(vr, r0, k0 + CB);
      load(vc, c0, k0 + CB);
    }
#pragma unroll 4
    for (int ks = 0; ks < CB / 4; ++ks) {
      const int k = ks * 4 + (lane >> 4);
      double a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        a[t] = sX[wm * 32 + t * 16 + (lane & 15)][k];
        b[t] = sY[wn * 32 + t * 16 + (lane & 15)][k];
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
    for (int tn = 0; tn < 2; ++tn) {
      const int64_t col = c0 + wn * 32 + tn * 16 + (lane & 15);
      double cur[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + wm * 32 + tm * 16 + (lane >> 4) + 4 * r;
        cur[r] = M[clamp_row(row, nr) * ld + (col < n ? col : c0)];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int lr = wm * 32 + tm * 16 + (lane >> 4) + 4 * r;
        const int64_t row = r0 + lr;
        const double v = cur[r] - acc[tm][tn][r];
        if (row < nr && col < n) M[row * ld + col] = v;
        if (bi == 1 && bj == 0 && side) side[lr * CB + (int)(col - c0)] = v;
      }
    }
  if (bi == 0 && bj == 0) {
    // sX is free once the K loop is done
    __syncthreads();
    diag_factor(M, n, ld, p1, Linv1, status, reinterpret_cast<double (*)[CB]>(&sX[0][0]));
  }
}

// Back substitution inside block o (mb <= 256 rows): L_KK^T x_K = y_K, where
// y_K has already received the blocks after K.  Sub-blocks from the last:
// t = y_s - L[>s][s]^T x[>s], x_s = Linv_s^T t.  One workgroup; every load
// batch is unconditional (clamped indices) so that it is issued at once.
__global__ __launch_bounds__(256) void chol_bwd_block_kernel(const double *__restrict__ M, int64_t ld,
                                                            int64_t o, int mb, const double *__restrict__ Linv,
                                                            const double *__restrict__ y, double *__restrict__ x) {
  __shared__ double sx[SB];
  __shared__ double st[CB];
  __shared__ double part[4][CB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  sx[tid] = 0.0;  // entries past mb stay zero
  __syncthreads();
  const int nsb = (mb + CB - 1) / CB;
  for (int s = nsb - 1; s >= 0; --s) {
    const int ms = mb - s * CB < CB ? mb - s * CB : CB;
    const int64_t col = o + s * CB + (lane < ms ? lane : ms - 1);
    // t_i = y_i - sum_{r in [64(s+1), mb)} L[o+r][o+64s+i] x_r: lane = column
    // i, wave w takes the rows 64(s+1) + 4k + w
    double acc = 0.0;
    for (int r0 = (s + 1) * CB; r0 < mb; r0 += 64) {
      double v[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const int r = r0 + 4 * k + wave;
        v[k] = M[(o + (r < mb ? r : mb - 1)) * ld + col];
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) acc += v[k] * sx[r0 + 4 * k + wave];  // r0 + 63 < 256
    }
    part[wave][lane] = acc;
    __syncthreads();
    if (tid < CB) st[tid] = (tid < ms ? y[o + s * CB + tid] : 0.0) - (part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid]);
    __syncthreads();
    // x_s[i] = sum_r Linv_s[r][i] t_r (Linv_s is lower triangular): lane = i,
    // wave w takes r = 4k + w
    const double *Li = Linv + (o / CB + s) * CB * CB;
    double v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = Li[(4 * k + wave) * CB + lane];
    acc = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += v[k] * st[4 * k + wave];
    part[wave][lane] = acc;
    __syncthreads();
    if (tid < CB) sx[s * CB + tid] = tid < ms ? part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid] : 0.0;
    __syncthreads();
  }
  if (tid < mb) x[o + tid] = sx[tid];
}

// y_t -= sum_{i < mb} L[o+i][t] x_{o+i} for t < o: 64 columns per workgroup
// (lane = column), the rows split over the 4 waves, 16 loads per batch.
__global__ __launch_bounds__(256) void chol_bwd_update_kernel(const double *__restrict__ M, int64_t ld, int64_t o,
                                                             int mb, const double *__restrict__ x,
                                                             double *__restrict__ y) {
  __shared__ double sx[SB];
  __shared__ double part[4][CB];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  sx[tid] = tid < mb ? x[o + tid] : 0.0;
  __syncthreads();
  const int64_t t = (int64_t)blockIdx.x * CB + lane;
  const int64_t tc = t < o ? t : o - 1;
  double acc = 0.0;
  for (int i0 = wave * 16; i0 < mb; i0 += 64) {
    double v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int i = i0 + k;
      v[k] = M[(o + (i < mb ? i : mb - 1)) * ld + tc];
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) acc += v[k] * sx[i0 + k];  // i0 + 15 < 256, zero past mb
  }
  part[wave][lane] = acc;
  __syncthreads();
  if (tid < CB && t < o) y[t] -= part[0][tid] + part[1][tid] + part[2][tid] + part[3][tid];
}

}  // namespace

size_t chol_workspace_bytes(int64_t n) {
  const int64_t nb = (n + CB - 1) / CB;
  // the inverses of the diagonal blocks, then two 64 x 64 blocks of rows
  // carried from one step of a panel to the next
  return (size_t)(nb + 2) * CB * CB * 8;
}

// A second stream and two events per device, created on first use and kept
// for the life of the process: the trailing update of the columns past the
// next outer panel runs there, concurrently with the factorisation of that
// panel.  A factorisation holds the device's lock while it enqueues, so that
// calls from several host threads pair their event records and waits.
namespace {
struct Side {
  bool tried = false, ok = false;
  hipStream_t s = nullptr;
  hipEvent_t next = nullptr, rest = nullptr;
  std::mutex mu;
};
std::mutex side_mu;
Side side_tab[64];

Side *side_for_current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> g(side_mu);
  Side &sd = side_tab[dev];
  if (!sd.tried) {
    sd.tried = true;
    sd.ok = hipStreamCreateWithFlags(&sd.s, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&sd.next, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&sd.rest, hipEventDisableTiming) == hipSuccess;
  }
  return sd.ok ? &sd : nullptr;
}
}  // namespace

vqmc_status chol_factor_solve(double *M, int64_t n, int64_t ld, double *x, void *ws, int *status, hipStream_t st) {
  if (n < 1 || ld < n || (ld & 1) || (reinterpret_cast<uintptr_t>(M) & 15)) return VQMC_ERR_ARG;
  double *Linv = reinterpret_cast<double *>(ws);
  const int64_t nr = n + 1;  // rows of the augmented matrix; row n carries the right-hand side
  // a stream under graph capture gets every kernel itself (no side stream)
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cap) != hipSuccess) return VQMC_ERR_DEVICE;
  Side *sd = (n > 2 * OB && cap == hipStreamCaptureStatusNone) ? side_for_current_device() : nullptr;
  std::unique_lock<std::mutex> hold;
  if (sd) hold = std::unique_lock<std::mutex>(sd->mu);
  bool rest_pending = false;
  for (int64_t p0 = 0; p0 < n; p0 += OB) {
    const int64_t p1 = (p0 + OB) < n ? p0 + OB : n;
    // first sub-panel: factor its diagonal block (keeping the rows below
    // it for the next step); then one launch per further sub-panel, each
    // solving the previous sub-panel's rows and updating (left-looking inside
    // the panel) and factoring its own; last, the rows of the last sub-panel
    double *side = Linv + ((n + CB - 1) / CB) * CB * CB;
    // the first diagonal block of the later panels is factored by the update
    // of the previous panel's trailing columns (below)
    if (p0 == 0)
      chol_diag_kernel<<<1, 256, 0, st>>>(M, n, ld, p0, Linv + (p0 / CB) * CB * CB, status,
                                          p0 + CB < p1 ? side : nullptr);
    int64_t cl = p0;
    for (int64_t c1 = p0 + CB; c1 < p1; c1 += CB) {
      const int64_t c0 = c1 - CB, m1 = (n - c1) < CB ? (n - c1) : CB;
      const int j = (int)((c0 - p0) / CB);
      chol_step_kernel<<<(unsigned)((nr - c1 + CB - 1) / CB), 256, 0, st>>>(
          M, nr, ld, p0, c0, c1 + m1, Linv + (c0 / CB) * CB * CB, Linv + (c1 / CB) * CB * CB, status,
          side + (j & 1) * CB * CB, c1 + CB < p1 ? side + ((j + 1) & 1) * CB * CB : nullptr);
      cl = c1;
    }
    {
      const int m = (int)((n - cl) < CB ? (n - cl) : CB);
      const int64_t below = nr - (cl + m);
      double *Li = Linv + (cl / CB) * CB * CB;
      if (m == CB)
        chol_trsm_kernel<true><<<(unsigned)((below + CB - 1) / CB), 256, 0, st>>>(M, nr, ld, cl, m, Li);
      else
        chol_trsm_kernel<false><<<(unsigned)((below + CB - 1) / CB), 256, 0, st>>>(M, nr, ld, cl, m, Li);
    }
    if (p1 >= n) break;
    // the next panel's columns must also have the previous rest update
    if (rest_pending && hipStreamWaitEvent(st, sd->rest, 0) != hipSuccess) return VQMC_ERR_DEVICE;
    const int T64 = (int)((nr - p1 + CB - 1) / CB), ncb = T64 < OB / CB ? T64 : OB / CB;
    chol_next_panel_kernel<<<(unsigned)(T64 * ncb), 256, 0, st>>>(M, n, nr, ld, p0, p1, ncb,
                                                                  Linv + (p1 / CB) * CB * CB, status,
                                                                  n - p1 > CB ? side : nullptr);
    if (nr - p1 > OB) {
      const int T = (int)((nr - p1 - OB + 127) / 128), nt = T * (T + 1) / 2;
      if (sd) {
        if (hipEventRecord(sd->next, st) != hipSuccess || hipStreamWaitEvent(sd->s, sd->next, 0) != hipSuccess)
          return VQMC_ERR_DEVICE;
        chol_trailing_kernel<<<(unsigned)nt, 256, 0, sd->s>>>(M, n, nr, ld, p0, p1, nt, OB / 16);
        if (hipEventRecord(sd->rest, sd->s) != hipSuccess) return VQMC_ERR_DEVICE;
        rest_pending = true;
      } else {
        chol_trailing_kernel<<<(unsigned)nt, 256, 0, st>>>(M, n, nr, ld, p0, p1, nt, OB / 16);
      }
    }
  }
  if (rest_pending && hipStreamWaitEvent(st, sd->rest, 0) != hipSuccess) return VQMC_ERR_DEVICE;
  if (hipGetLastError() != hipSuccess) return VQMC_ERR_DEVICE;
  // row n now holds y = L^-1 rhs; L^T x = y from the last block (y is consumed)
  double *y = M + n * ld;
  for (int64_t o = ((n - 1) / SB) * SB; o >= 0; o -= SB) {
    const int mb = (int)((n - o) < SB ? (n - o) : SB);
    chol_bwd_block_kernel<<<1, 256, 0, st>>>(M, ld, o, mb, Linv, y, x);
    if (o > 0) chol_bwd_update_kernel<<<(unsigned)((o + CB - 1) / CB), 256, 0, st>>>(M, ld, o, mb, x, y);
  }
  if (hipGetLastError() != hipSuccess) return VQMC_ERR_DEVICE;
  return VQMC_OK;
}

}  // namespace vqmc
