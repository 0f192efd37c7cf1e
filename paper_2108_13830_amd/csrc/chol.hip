// chol.hip -- blocked Cholesky factorisation M = L L^T of an SPD matrix (FP64,
// lower triangle, in place) and the two triangular solves of the SR step
// (Sec. 3.2.2: the Cholesky factor followed by forward and back substitution
// instead of an explicit inverse of M).
//
// Right-looking, two block levels: 512-column outer panels, each factored as
// eight 64-column sub-panels.  Per sub-panel: one workgroup factors the 64 x 64
// diagonal block and, in the same sweep, inverts its triangle; the rows below
// are then one GEMM with that small inverse; the rest of the outer panel is
// updated.  After each outer panel the trailing matrix receives one rank-512
// update on the FP64 matrix cores, so it is read and written once per 512
// columns.
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
__global__ __launch_bounds__(256) void chol_diag_kernel(double *__restrict__ M, int64_t n, int64_t ld, int64_t c0,
                                                       double *__restrict__ Linv, int *__restrict__ status) {
  __shared__ double colbuf[2][CB];
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
  // one step, with column B1 = (j+1) % 4 of this thread's block done first
  auto step = [&](int j, auto b1c) {
    constexpr int B1 = decltype(b1c)::value;
    const double *v = colbuf[j & 1];
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
    if (by == (j >> 2))
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if ((j & 3) == b) dcol[b] = d;
    const double q = recip(d);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int x = x0 + a;
      const double rl = (x == j ? 1.0 : vx[a]) * q;
      const double ru = x <= j ? rl : 0.0;
      rlo[a] = upblk ? ru : rl;
      rhi[a] = lowblk ? rl : ru;
      cf[a] = (y0 + a > j) ? vy[a] : 0.0;
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) z[a][B1] -= (B1 <= a ? rlo[a] : rhi[a]) * cf[B1];
    if (j + 1 < CB && by == ((j + 1) >> 2))
#pragma unroll
      for (int a = 0; a < 4; ++a) colbuf[(j + 1) & 1][x0 + a] = z[a][B1];
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (b != B1) z[a][b] -= (b <= a ? rlo[a] : rhi[a]) * cf[b];
  };
  for (int j = 0; j < CB; j += 4) {
    step(j, std::integral_constant<int, 1>{});
    step(j + 1, std::integral_constant<int, 2>{});
    step(j + 2, std::integral_constant<int, 3>{});
    step(j + 3, std::integral_constant<int, 0>{});
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
// for r in [c0+m, nr), 64 rows per workgroup (4 waves x 16 rows, 4 column
// tiles each).  The last row of the augmented matrix is included, so this is
// also the forward substitution step of that block.
template <bool FULL>
__global__ __launch_bounds__(256) void chol_trsm_kernel(double *__restrict__ M, int64_t nr, int64_t ld, int64_t c0,
                                                       int m, const double *__restrict__ Linv) {
  __shared__ double sA[CB][CB + 2];
  __shared__ double sL[CB][CB + 2];
  const int64_t r0 = c0 + m + (int64_t)blockIdx.x * CB;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if constexpr (FULL) stage64(M, ld, r0, nr, c0, sA);
  else stage64_partial(M, ld, r0, nr, c0, m, sA);
  stage64(Linv, CB, 0, CB, 0, sL);
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
      const int col = q * 16 + (lane & 15);
      if (row < nr && col < m) M[row * ld + c0 + col] = acc[q][r];
    }
}

// Remaining columns of the outer panel after sub-panel c0, one 64 x 64 tile
// per workgroup: A[r][c] -= sum_t L[r][c0+t] L[c][c0+t] for c in
// [c0+64, cend), r >= c, r < nr.
__global__ __launch_bounds__(256) void chol_panel_update_kernel(double *__restrict__ M, int64_t nr, int64_t ld,
                                                                int64_t c0, int64_t cend) {
  __shared__ double sR[CB][CB + 2];
  __shared__ double sC[CB][CB + 2];
  const int64_t cc0 = c0 + CB + (int64_t)blockIdx.x * CB;
  const int64_t r0 = c0 + CB + (int64_t)blockIdx.y * CB;
  if (cc0 > r0 + CB - 1) return;  // tile strictly above the diagonal (uniform per workgroup)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  stage64(M, ld, r0, nr, c0, sR);
  stage64(M, ld, cc0, nr, c0, sC);
  __syncthreads();
  f64x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0, 0, 0, 0};
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
#pragma unroll
  for (int tm = 0; tm < 2; ++tm)
#pragma unroll
    for (int tn = 0; tn < 2; ++tn) {
      const int64_t col = cc0 + wn * 32 + tn * 16 + (lane & 15);
      double cur[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + wm * 32 + tm * 16 + (lane >> 4) + 4 * r;
        cur[r] = M[clamp_row(row, nr) * ld + (col < cend ? col : c0)];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = r0 + wm * 32 + tm * 16 + (lane >> 4) + 4 * r;
        if (row < nr && col < cend && col <= row) M[row * ld + col] = cur[r] - acc[tm][tn][r];
      }
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

// Trailing matrix after the outer panel [p0, p1) (p1 - p0 = OB): 128 x 128
// tiles of rows [p1, nr) and columns [p1, n) on or below the diagonal,
// M[r][c] -= sum_{t in [p0,p1)} L[r][t] L[c][t].  Tile (bi, bj) counts block
// rows and columns from p1.  ncb > 0: only the block columns bj < ncb (the
// next outer panel), tile t = (t / ncb, t % ncb); ncb == 0: the lower
// triangle of block rows and columns >= OB / 128 (the rest).
__global__ __launch_bounds__(256, 2) void chol_trailing_kernel(double *__restrict__ M, int64_t n, int64_t nr,
                                                            int64_t ld, int64_t p0, int64_t p1, int ntiles,
                                                            int ncb) {
  constexpr int KC = 16;
  __shared__ Panel<double, KC, false> sA, sB;
  using TT = Tile128<double>;
  int bi, bj;
  const int t = xcd_contiguous(blockIdx.x, ntiles);
  if (ncb > 0) {
    bi = t / ncb;
    bj = t - bi * ncb;
  } else {
    lower_block(t, bi, bj);
    bi += OB / 128;
    bj += OB / 128;
  }
  const int64_t r0 = p1 + (int64_t)bi * 128, c0 = p1 + (int64_t)bj * 128;
  // tiles above the diagonal, and the extra block row of the augmented matrix
  // past the last column (uniform per workgroup)
  if (bj > bi || c0 >= n) return;
  TrailLoader<KC> ldr{M, ld, nr, r0, c0, p0};
  TT::acc_t acc[4][4];
  TT::zero(acc);
  TT::run<KC, false>(ldr, OB / KC, sA, sB, acc);
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

// Back substitution inside block o (mb <= 256 rows): L_KK^T x_K = y_K, where
// y_K has already received the blocks after K.  Sub-blocks from the last:
// t = y_s - L[>s][s]^T x[>s], x_s = Linv_s^T t.  One workgroup; every load
// batch is unconditional (clamped indices) so that it is issued at once.
__global__ __launch_bounds__(256) void chol_bwd_block_kernel(const double *__restrict__ M, int64_t n, int64_t ld,
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
  return (size_t)nb * CB * CB * 8;
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
  Side *sd = n > 2 * OB ? side_for_current_device() : nullptr;
  std::unique_lock<std::mutex> hold;
  if (sd) hold = std::unique_lock<std::mutex>(sd->mu);
  bool rest_pending = false;
  for (int64_t p0 = 0; p0 < n; p0 += OB) {
    const int64_t p1 = (p0 + OB) < n ? p0 + OB : n;
    for (int64_t c0 = p0; c0 < p1; c0 += CB) {
      double *Li = Linv + (c0 / CB) * CB * CB;
      const int m = (int)((n - c0) < CB ? (n - c0) : CB);
      chol_diag_kernel<<<1, 256, 0, st>>>(M, n, ld, c0, Li, status);
      const int64_t below = nr - (c0 + m);
      if (m == CB)
        chol_trsm_kernel<true><<<(unsigned)((below + CB - 1) / CB), 256, 0, st>>>(M, nr, ld, c0, m, Li);
      else
        chol_trsm_kernel<false><<<(unsigned)((below + CB - 1) / CB), 256, 0, st>>>(M, nr, ld, c0, m, Li);
      const int64_t rest = p1 - (c0 + CB);
      if (rest > 0) {
        const dim3 g((unsigned)((rest + CB - 1) / CB), (unsigned)((below + CB - 1) / CB));
        chol_panel_update_kernel<<<g, 256, 0, st>>>(M, nr, ld, c0, p1);
      }
    }
    if (p1 >= n) break;
    const int T = (int)((nr - p1 + 127) / 128);
    const int ncb = T < OB / 128 ? T : OB / 128;  // block columns of the next outer panel
    // the next panel's columns must also have the previous rest update
    if (rest_pending && hipStreamWaitEvent(st, sd->rest, 0) != hipSuccess) return VQMC_ERR_DEVICE;
    chol_trailing_kernel<<<(unsigned)(T * ncb), 256, 0, st>>>(M, n, nr, ld, p0, p1, T * ncb, ncb);
    if (T > ncb) {
      const int nt = (T - ncb) * (T - ncb + 1) / 2;
      if (sd) {
        if (hipEventRecord(sd->next, st) != hipSuccess || hipStreamWaitEvent(sd->s, sd->next, 0) != hipSuccess)
          return VQMC_ERR_DEVICE;
        chol_trailing_kernel<<<(unsigned)nt, 256, 0, sd->s>>>(M, n, nr, ld, p0, p1, nt, 0);
        if (hipEventRecord(sd->rest, sd->s) != hipSuccess) return VQMC_ERR_DEVICE;
        rest_pending = true;
      } else {
        chol_trailing_kernel<<<(unsigned)nt, 256, 0, st>>>(M, n, nr, ld, p0, p1, nt, 0);
      }
    }
  }
  if (rest_pending && hipStreamWaitEvent(st, sd->rest, 0) != hipSuccess) return VQMC_ERR_DEVICE;
  if (hipGetLastError() != hipSuccess) return VQMC_ERR_DEVICE;
  // row n now holds y = L^-1 rhs; L^T x = y from the last block (y is consumed)
  double *y = M + n * ld;
  for (int64_t o = ((n - 1) / SB) * SB; o >= 0; o -= SB) {
    const int mb = (int)((n - o) < SB ? (n - o) : SB);
    chol_bwd_block_kernel<<<1, 256, 0, st>>>(M, n, ld, o, mb, Linv, y, x);
    if (o > 0) chol_bwd_update_kernel<<<(unsigned)((o + CB - 1) / CB), 256, 0, st>>>(M, ld, o, mb, x, y);
  }
  if (hipGetLastError() != hipSuccess) return VQMC_ERR_DEVICE;
  return VQMC_OK;
}

}  // namespace vqmc
