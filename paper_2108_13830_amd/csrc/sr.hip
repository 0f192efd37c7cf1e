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

#include "chol.hpp"
#include "common.hpp"
#include "engine.hpp"
#include "tile128.hpp"

namespace vqmc {

// samples per K chunk of the direct-to-LDS S product
constexpr int SYRK_KC = 16;

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
// scal slots; S_RRP + (it & 1): r.r entering CG iteration it (two slots, so
// that the kernel forming the next value never overwrites one its other
// workgroups still read)
enum { S_MEAN = 0, S_VAR, S_SUMEC, S_RR, S_NORMF, S_DONE, S_ITERS, S_REL, S_OBP, S_RRP, S_RRP1, S_NSLOT = 16 };

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
    if (!isfinite(mean) || !isfinite(var)) status[1] = 1;
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

// The same column sums with four adjacent columns per thread (16-byte loads
// of O; needs 16-byte aligned rows).
template <bool CENTRED>
__global__ __launch_bounds__(256) void col_partial4_kernel(const float *__restrict__ O, int64_t ldO, int B,
                                                           int64_t P, const double *__restrict__ obar,
                                                           const double *__restrict__ wa,
                                                           const double *__restrict__ wb, int rows_per_chunk,
                                                           double *__restrict__ part_a,
                                                           double *__restrict__ part_b,
                                                           const double *__restrict__ scal) {
  if (scal && scal[S_DONE] != 0.0) return;
  const int64_t k = ((int64_t)blockIdx.x * 256 + threadIdx.x) * 4;
  if (k >= P) return;
  const int nv = (int)(P - k < 4 ? P - k : 4);
  const int c = blockIdx.y;
  const int b0 = c * rows_per_chunk, b1 = min(B, b0 + rows_per_chunk);
  double ob[4] = {0.0, 0.0, 0.0, 0.0};
  if (CENTRED)
    for (int t = 0; t < nv; ++t) ob[t] = obar[k + t];
  double sa[4] = {0.0, 0.0, 0.0, 0.0}, sb[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int b = b0; b < b1; ++b) {
    const float *row = O + (int64_t)b * ldO + k;
    float v[4];
    if (nv == 4) {
      const float4 q = *reinterpret_cast<const float4 *>(row);
      v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
    } else {
      for (int t = 0; t < 4; ++t) v[t] = t < nv ? row[t] : 0.f;
    }
    const double a = wa ? wa[b] : 1.0;
    const double w2 = wb ? wb[b] : 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const double o = (double)v[t] - ob[t];
      sa[t] += o * a;
      sb[t] += o * w2;
    }
  }
  for (int t = 0; t < nv; ++t) {
    part_a[(int64_t)c * P + k + t] = sa[t];
    if (part_b) part_b[(int64_t)c * P + k + t] = sb[t];
  }
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

// Loader of the primal S tiles: panel rows are columns ia0.. (A side) or
// ib0.. (B side) of O, k runs over samples.  Each thread holds four adjacent
// columns (fixed for the whole K loop) of KC/8 samples per chunk; samples past
// B are zeroed at the LDS store, columns past P are clamped (they only feed
// outputs that are not stored).  Centring happens in FP64 before the
// rounding to T.  Scalar loads: the form for O whose rows are not 16-byte
// aligned or whose P is not a multiple of 4 (syrk_dma_kernel otherwise).
template <typename T, int KC>
struct SyrkLoader {
  static constexpr int NQ = KC / 8;
  const float *O;
  int64_t ldO;
  int B;
  int64_t P, ia0, ib0;
  double oba[4], obb[4];
  struct Regs {
    float v[NQ][4];
    int c;
  };
  __device__ SyrkLoader(const float *O_, int64_t ldO_, int B_, int64_t P_, int64_t ia, int64_t ib,
                        const double *__restrict__ obar)
      : O(O_), ldO(ldO_), B(B_), P(P_), ia0(ia), ib0(ib) {
    const int m4 = threadIdx.x & 31;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t ca = ia0 + 4 * m4 + t, cb = ib0 + 4 * m4 + t;
      oba[t] = ca < P ? obar[ca] : 0.0;
      obb[t] = cb < P ? obar[cb] : 0.0;
    }
  }
  __device__ __forceinline__ void load(Regs &r, int c, bool bside) const {
    const int m4 = threadIdx.x & 31;
    const int64_t col = (bside ? ib0 : ia0) + 4 * m4;
    r.c = c;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int k = (threadIdx.x >> 5) + 8 * q;
      const int b = c * KC + k;
      const float *row = O + (int64_t)(b < B ? b : B - 1) * ldO;
#pragma unroll
      for (int t = 0; t < 4; ++t) r.v[q][t] = row[col + t < P ? col + t : P - 1];
    }
  }
  __device__ __forceinline__ void store(const Regs &r, Panel<T, KC, true> &Pn, bool bside) const {
    const int m4 = threadIdx.x & 31;
    const double *ob = bside ? obb : oba;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int k = (threadIdx.x >> 5) + 8 * q;
      const bool ok = r.c * KC + k < B;
      T w[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) w[t] = ok ? (T)((double)r.v[q][t] - ob[t]) : (T)0;
      if constexpr (sizeof(T) == 4) {
        *reinterpret_cast<float4 *>(&Pn.s[k][4 * m4]) = make_float4(w[0], w[1], w[2], w[3]);
      } else {
        *reinterpret_cast<double2 *>(&Pn.s[k][4 * m4]) = make_double2(w[0], w[1]);
        *reinterpret_cast<double2 *>(&Pn.s[k][4 * m4 + 2]) = make_double2(w[2], w[3]);
      }
    }
  }
};

// The pipelined K loop of Tile128 for loaders whose store needs the side.
template <typename T, int KC, bool KM, class LD>
__device__ __forceinline__ void run_sided(const LD &ld, int nchunks, Panel<T, KC, KM> &sA, Panel<T, KC, KM> &sB,
                                          typename Tile128<T>::acc_t (&acc)[4][4]) {
  typename LD::Regs ra, rb;
  ld.load(ra, 0, false);
  ld.load(rb, 0, true);
  for (int c = 0; c < nchunks; ++c) {
    ld.store(ra, sA, false);
    ld.store(rb, sB, true);
    __syncthreads();
    if (c + 1 < nchunks) {
      ld.load(ra, c + 1, false);
      ld.load(rb, c + 1, true);
    }
    Tile128<T>::template step<KC, KM>(sA, sB, acc);
    __syncthreads();
  }
}

// S[i][j] = (1/B) sum_b (O[b][i] - <O_i>)(O[b][j] - <O_j>) + eps [i == j],
// lower 128 x 128 blocks (row stride ldS).  T = double: FP64 operands and
// accumulation; T = float: the centred values are rounded to FP32 and
// accumulated by the FP32 matrix cores.
template <typename T>
__global__ __launch_bounds__(256, 2) void syrk_kernel(const float *__restrict__ O, int64_t ldO, int B, int64_t P,
                                                   const double *__restrict__ obar, double eps,
                                                   double *__restrict__ S, int64_t ldS, int ntiles) {
  constexpr int KC = sizeof(T) == 4 ? 32 : 16;
  __shared__ Panel<T, KC, true> sA, sB;
  using TT = Tile128<T>;
  int bi, bj;
  lower_block(xcd_contiguous(blockIdx.x, ntiles), bi, bj);
  const int64_t i0 = (int64_t)bi * 128, j0 = (int64_t)bj * 128;
  const SyrkLoader<T, KC> ldr(O, ldO, B, P, i0, j0, obar);
  typename TT::acc_t acc[4][4];
  TT::zero(acc);
  run_sided<T, KC, true>(ldr, (B + KC - 1) / KC, sA, sB, acc);
  const double inv = 1.0 / B;
#pragma unroll
  for (int tm = 0; tm < 4; ++tm)
#pragma unroll
    for (int tn = 0; tn < 4; ++tn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = i0 + TT::row_of(tm, r), col = j0 + TT::col_of(tn);
        if (row < P && col <= row) S[row * ldS + col] = (double)acc[tm][tn][r] * inv + (row == col ? eps : 0.0);
      }
}

// The explicit S on the same 128 x 128 tiles, with the operand panels copied
// from O straight into LDS (direct-to-LDS loads: no registers, no stores) in
// two buffers, so that the copy of chunk c + 1 runs while the matrix cores
// consume chunk c and one barrier per chunk suffices.  A panel chunk is KC
// samples (rows k) of 128 parameters; the 16-float blocks of row k sit at
// block ^ (k & 3), so that the four rows one operand read spans fall on
// disjoint LDS banks.  Operands are centred as they are read, in FP64, and
// then rounded to T: the same values as syrk_kernel forms, hence the same S.
// Needs 16-byte loads (P % 4 == 0, rows 16-byte aligned); rows past B in the
// last chunk read row B - 1 and enter as zeros.
template <typename T, int KC>
__global__ __launch_bounds__(256, 2) void syrk_dma_kernel(const float *__restrict__ O, int64_t ldO, int B, int64_t P,
                                                       const double *__restrict__ obar, double eps,
                                                       double *__restrict__ S, int64_t ldS, int ntiles) {
  static_assert(KC % 8 == 0, "a chunk is whole row pairs for each wave");
  constexpr int PANEL = KC * 128;  // floats per panel chunk
  constexpr int PAIRS = KC / 2;    // wave copy instructions per panel chunk (two rows each)
  __shared__ __align__(16) float sbuf[2][2][PANEL];
  using TT = Tile128<T>;
  int bi, bj;
  lower_block(xcd_contiguous(blockIdx.x, ntiles), bi, bj);
  const int64_t i0 = (int64_t)bi * 128, j0 = (int64_t)bj * 128;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wm = wave >> 1, wn = wave & 1, g = lane >> 4, li = lane & 15;
  // copies: instruction q = wave + 4 j of a chunk moves rows 2 (q % PAIRS) and
  // + 1 of panel q / PAIRS; row & 3 = 2 (wave & 1) + lane / 32 for all of
  // this lane's, so its source column (logical 4-float unit lu of its
  // physical unit lane % 32) is fixed
  const int prow = lane >> 5, pu = lane & 31;
  const int lu = (((pu >> 2) ^ (2 * (wave & 1) + prow)) << 2) | (pu & 3);
  const int64_t colA = i0 + 4 * lu <= P - 4 ? i0 + 4 * lu : P - 4;
  const int64_t colB = j0 + 4 * lu <= P - 4 ? j0 + 4 * lu : P - 4;
  auto copy = [&](int c, int buf) {
#pragma unroll
    for (int j = 0; j < KC / 4; ++j) {
      const int q = wave + 4 * j, side = q / PAIRS, pair = q - side * PAIRS;
      const int b0 = c * KC + 2 * pair + prow;
      const int b = b0 < B ? b0 : B - 1;
      const float *src = O + (int64_t)b * ldO + (side ? colB : colA);
      __builtin_amdgcn_global_load_lds(src, (lds_ptr_t)(&sbuf[buf][side][pair * 256]), 16, 0, 0);
    }
  };
  // operand reads: row k = 4 ks + g (k & 3 = g), logical block wm * 4 + t
  int offA[4], offB[4];
  double oba[4], obb[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    offA[t] = g * 128 + (((wm * 4 + t) ^ g) << 4) + li;
    offB[t] = g * 128 + (((wn * 4 + t) ^ g) << 4) + li;
    const int64_t ca = i0 + wm * 64 + t * 16 + li, cb = j0 + wn * 64 + t * 16 + li;
    oba[t] = ca < P ? obar[ca] : 0.0;
    obb[t] = cb < P ? obar[cb] : 0.0;
  }
  typename TT::acc_t acc[4][4];
  TT::zero(acc);
  auto chunk = [&](const float *pa, const float *pb, int kleft, auto tail) {
    constexpr bool TAIL = decltype(tail)::value;
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      T a[4], b[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double x = (double)pa[offA[t] + ks * 512] - oba[t];
        a[t] = (T)(TAIL && 4 * ks + g >= kleft ? 0.0 : x);
        b[t] = (T)((double)pb[offB[t] + ks * 512] - obb[t]);
      }
#pragma unroll
      for (int tm = 0; tm < 4; ++tm)
#pragma unroll
        for (int tn = 0; tn < 4; ++tn) acc[tm][tn] = TT::mma(a[tm], b[tn], acc[tm][tn]);
    }
  };
  // whole chunks, then (B % KC != 0) the last, partial one
  const int nfull = B / KC, nchunks = (B + KC - 1) / KC;
  copy(0, 0);
  for (int c = 0; c < nfull; ++c) {
    wait_copies();
    __syncthreads();
    if (c + 1 < nchunks) copy(c + 1, (c + 1) & 1);
    chunk(sbuf[c & 1][0], sbuf[c & 1][1], KC, std::false_type{});
  }
  if (nfull < nchunks) {
    wait_copies();
    __syncthreads();
    chunk(sbuf[nfull & 1][0], sbuf[nfull & 1][1], B - nfull * KC, std::true_type{});
  }
  const double inv = 1.0 / B;
#pragma unroll
  for (int tm = 0; tm < 4; ++tm)
#pragma unroll
    for (int tn = 0; tn < 4; ++tn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = i0 + TT::row_of(tm, r), col = j0 + TT::col_of(tn);
        if (row < P && col <= row) S[row * ldS + col] = (double)acc[tm][tn][r] * inv + (row == col ? eps : 0.0);
      }
}

// Loader of the sample-space Gram tiles: panel rows are samples a0.. (A side)
// or c0.. (B side), k runs over parameters in chunks of 16.  Samples past B
// are clamped (outputs not stored); parameters past P are zeroed.  Scalar
// loads: the form for O without 16-byte rows (gram_dma_kernel otherwise).
struct GramLoader {
  const float *O;
  int64_t ldO;
  int B;
  int64_t P;
  int a0, c0;
  const double *obar;
  struct Regs {
    float v[2][4];
    double ob[4];
    int c;
  };
  __device__ __forceinline__ void load(Regs &r, int c, bool bside) const {
    const int k4 = threadIdx.x & 3;
    const int64_t k = (int64_t)c * 16 + 4 * k4;
    r.c = c;
#pragma unroll
    for (int t = 0; t < 4; ++t) r.ob[t] = obar[k + t < P ? k + t : P - 1];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int m = (threadIdx.x + 256 * q) >> 2;
      const int a = (bside ? c0 : a0) + m;
      const float *row = O + (int64_t)(a < B ? a : B - 1) * ldO;
#pragma unroll
      for (int t = 0; t < 4; ++t) r.v[q][t] = row[k + t < P ? k + t : P - 1];
    }
  }
  __device__ __forceinline__ void store(const Regs &r, Panel<double, 16, false> &Pn, bool) const {
    const int k4 = threadIdx.x & 3;
    const int64_t k = (int64_t)r.c * 16 + 4 * k4;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int m = (threadIdx.x + 256 * q) >> 2;
      double w[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) w[t] = k + t < P ? (double)r.v[q][t] - r.ob[t] : 0.0;
      *reinterpret_cast<double2 *>(&Pn.s[m][4 * k4]) = make_double2(w[0], w[1]);
      *reinterpret_cast<double2 *>(&Pn.s[m][4 * k4 + 2]) = make_double2(w[2], w[3]);
    }
  }
};

// Sample-space Gram: K[a][c] = (1/B) sum_k (O[a][k]-<O_k>)(O[c][k]-<O_k>) + eps [a == c]
// (row stride ldK).
__global__ __launch_bounds__(256, 2) void gram_kernel(const float *__restrict__ O, int64_t ldO, int B, int64_t P,
                                                   const double *__restrict__ obar, double eps,
                                                   double *__restrict__ K, int64_t ldK, int ntiles) {
  __shared__ Panel<double, 16, false> sA, sB;
  using TT = Tile128<double>;
  int bi, bj;
  lower_block(xcd_contiguous(blockIdx.x, ntiles), bi, bj);
  const int a0 = bi * 128, c0 = bj * 128;
  const GramLoader ldr{O, ldO, B, P, a0, c0, obar};
  TT::acc_t acc[4][4];
  TT::zero(acc);
  run_sided<double, 16, false>(ldr, (int)((P + 15) / 16), sA, sB, acc);
  const double inv = 1.0 / B;
#pragma unroll
  for (int tm = 0; tm < 4; ++tm)
#pragma unroll
    for (int tn = 0; tn < 4; ++tn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = a0 + TT::row_of(tm, r), col = c0 + TT::col_of(tn);
        if (row < B && col <= row) K[(int64_t)row * ldK + col] = acc[tm][tn][r] * inv + (row == col ? eps : 0.0);
      }
}

// The sample-space Gram matrix with the same direct-to-LDS panel copies as
// syrk_dma_kernel: panel rows are samples, a chunk is 16 parameters (k), so a
// row of a chunk is four 16-byte units, unit u stored at u ^ ((m >> 2) & 3)
// (an operand read then touches 64 distinct banks).  The means of the
// chunk's parameters are loaded beside its copy; parameters past P in the
// last chunk enter as zeros.  Needs 16-byte loads (P % 4 == 0, rows 16-byte
// aligned); the same values enter the matrix cores as in gram_kernel.
__global__ __launch_bounds__(256, 2) void gram_dma_kernel(const float *__restrict__ O, int64_t ldO, int B, int64_t P,
                                                       const double *__restrict__ obar, double eps,
                                                       double *__restrict__ K, int64_t ldK, int ntiles) {
  constexpr int KC = 16, PANEL = 128 * KC;  // floats per panel chunk
  __shared__ __align__(16) float sbuf[2][2][PANEL];
  using TT = Tile128<double>;
  int bi, bj;
  lower_block(xcd_contiguous(blockIdx.x, ntiles), bi, bj);
  const int a0 = bi * 128, c0 = bj * 128;
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // copies: instruction q = wave + 4 j moves rows 16 (q % 8) .. + 15 of
  // panel q / 8, the lane's row 16 (q % 8) + lane / 4, whose swizzle
  // (row >> 2) & 3 = lane / 16: its source unit is fixed
  const int su = (lane & 3) ^ (lane >> 4);
  auto copy = [&](int c, int buf) {
    const int64_t k0 = (int64_t)c * KC + 4 * su;
    const int64_t kc = k0 <= P - 4 ? k0 : P - 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int q = wave + 4 * j, side = q >> 3, blk = q & 7;
      const int row = (side ? c0 : a0) + 16 * blk + (lane >> 2);
      const float *src = O + (int64_t)(row < B ? row : B - 1) * ldO + kc;
      __builtin_amdgcn_global_load_lds(src, (lds_ptr_t)(&sbuf[buf][side][blk * 16 * KC]), 16, 0, 0);
    }
  };
  // operand reads: row m = w*64 + t*16 + lane%16, parameter k = 4 ks + lane/16
  const int lanem = lane & 15, g = lane >> 4, sw = (lanem >> 2) & 3;
  const int wm = wave >> 1, wn = wave & 1;
  int offA[4], offB[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    offA[t] = (wm * 64 + t * 16 + lanem) * KC + g;
    offB[t] = (wn * 64 + t * 16 + lanem) * KC + g;
  }
  // the means of the lane's parameters of chunk c
  auto means = [&](int c, double (&ob)[4]) {
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int64_t k = (int64_t)c * KC + 4 * ks + g;
      ob[ks] = obar[k < P ? k : P - 1];
    }
  };
  TT::acc_t acc[4][4];
  TT::zero(acc);
  auto chunk = [&](const float *pa, const float *pb, const double (&ob)[4], int64_t k0, auto tail) {
    constexpr bool TAIL = decltype(tail)::value;
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int uo = 4 * (ks ^ sw);
      const bool live = !TAIL || k0 + 4 * ks + g < P;
      double a[4], b[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double x = (double)pa[offA[t] + uo] - ob[ks];
        a[t] = live ? x : 0.0;
        b[t] = (double)pb[offB[t] + uo] - ob[ks];
      }
#pragma unroll
      for (int tm = 0; tm < 4; ++tm)
#pragma unroll
        for (int tn = 0; tn < 4; ++tn) acc[tm][tn] = TT::mma(a[tm], b[tn], acc[tm][tn]);
    }
  };
  const int nfull = (int)(P / KC), nchunks = (int)((P + KC - 1) / KC);
  double obc[4], obn[4];
  means(0, obc);
  copy(0, 0);
  for (int c = 0; c < nfull; ++c) {
    wait_copies();
    __syncthreads();
    if (c + 1 < nchunks) {
      copy(c + 1, (c + 1) & 1);
      means(c + 1, obn);
    }
    chunk(sbuf[c & 1][0], sbuf[c & 1][1], obc, (int64_t)c * KC, std::false_type{});
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) obc[ks] = obn[ks];
  }
  if (nfull < nchunks) {
    wait_copies();
    __syncthreads();
    chunk(sbuf[nfull & 1][0], sbuf[nfull & 1][1], obc, (int64_t)nfull * KC, std::true_type{});
  }
  const double inv = 1.0 / B;
#pragma unroll
  for (int tm = 0; tm < 4; ++tm)
#pragma unroll
    for (int tn = 0; tn < 4; ++tn)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = a0 + TT::row_of(tm, r), col = c0 + TT::col_of(tn);
        if (row < B && col <= row) K[(int64_t)row * ldK + col] = acc[tm][tn][r] * inv + (row == col ? eps : 0.0);
      }
}

// ---------------------------------------------------------------- CG

__global__ __launch_bounds__(1024) void cg_init_kernel(const double *__restrict__ F, int64_t P,
                                                       const double *__restrict__ obar,
                                                       double *__restrict__ x, double *__restrict__ r,
                                                       double *__restrict__ p, double *__restrict__ scal,
                                                       int *__restrict__ status) {
  __shared__ double tmp[16];
  double s = 0.0, op = 0.0;
  for (int64_t k = threadIdx.x; k < P; k += 1024) {
    const double f = F[k];
    x[k] = 0.0;
    r[k] = f;
    p[k] = f;
    s += f * f;
    op += obar[k] * f;
  }
  const double rr = block_sum_t<1024>(s, tmp);
  const double obp = block_sum_t<1024>(op, tmp);
  if (threadIdx.x == 0) {
    scal[S_RR] = rr;
    scal[S_RRP] = rr;
    scal[S_NORMF] = sqrt(rr);
    scal[S_DONE] = rr > 0.0 ? 0.0 : 1.0;
    // a non-finite right-hand side (non-finite O or E) stops CG at once
    if (!isfinite(rr)) {
      status[1] = 1;
      scal[S_DONE] = 1.0;
    }
    scal[S_ITERS] = 0.0;
    scal[S_REL] = 0.0;
    scal[S_OBP] = obp;
  }
}

// u_b = sum_k (O[b][k] - <O_k>) p_k = sum_k O[b][k] p_k - <O>.p for R rows
// per workgroup (p is read once for the R rows).  VEC: 16-byte loads of O.
template <int R, bool VEC>
__global__ __launch_bounds__(256) void cg_rowdot_kernel(const float *__restrict__ O, int64_t ldO, int B, int64_t P,
                                                        const double *__restrict__ p, double *__restrict__ u,
                                                        const double *__restrict__ scal) {
  __shared__ double tmp[4 * R];
  if (scal[S_DONE] != 0.0) return;
  const int b0 = blockIdx.x * R;
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  int64_t kdone = 0;
  if constexpr (VEC) {
    const int64_t P4 = P / 4;
    for (int64_t k4 = threadIdx.x; k4 < P4; k4 += 256) {
      const double2 pa = *reinterpret_cast<const double2 *>(p + 4 * k4);
      const double2 pb = *reinterpret_cast<const double2 *>(p + 4 * k4 + 2);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (b0 + r < B) {
          const float4 o = *reinterpret_cast<const float4 *>(O + (int64_t)(b0 + r) * ldO + 4 * k4);
          acc[r] += (double)o.x * pa.x + (double)o.y * pa.y + (double)o.z * pb.x + (double)o.w * pb.y;
        }
      }
    }
    kdone = 4 * P4;
  }
  for (int64_t k = kdone + threadIdx.x; k < P; k += 256) {
    const double pk = p[k];
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (b0 + r < B) acc[r] += (double)O[(int64_t)(b0 + r) * ldO + k] * pk;
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const double v = wave_sum(acc[r]);
    if (lane == 0) tmp[r * 4 + wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < R && b0 + (int)threadIdx.x < B) {
    const int r = threadIdx.x;
    u[b0 + r] = ((tmp[r * 4] + tmp[r * 4 + 1]) + (tmp[r * 4 + 2] + tmp[r * 4 + 3])) - scal[S_OBP];
  }
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

// Sum of the n partials part[0..n) in a fixed order (every workgroup that
// calls it gets the same value): strided per thread, then the block tree.
template <int NT>
__device__ __forceinline__ double sum_partials(const double *__restrict__ part, int n, double *tmp) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += NT) v += part[i];
  return block_sum_t<NT>(v, tmp);
}

// CG iteration it, after q = (S + eps I) p: alpha = rr / p.q; x += alpha p;
// r -= alpha q; per-workgroup partial sums of r.r.
__global__ __launch_bounds__(256) void cg_update_kernel(int64_t P, double *__restrict__ x, double *__restrict__ r,
                                                        const double *__restrict__ p,
                                                        const double *__restrict__ q,
                                                        const double *__restrict__ pq_part, int npq,
                                                        double *__restrict__ rr_part,
                                                        const double *__restrict__ scal, int it) {
  __shared__ double tmp[4];
  if (scal[S_DONE] != 0.0) return;
  const double pq = sum_partials<256>(pq_part, npq, tmp);
  const double alpha = scal[S_RRP + (it & 1)] / pq;
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double v = 0.0;
  if (k < P) {
    x[k] += alpha * p[k];
    const double rk = r[k] - alpha * q[k];
    r[k] = rk;
    v = rk * rk;
  }
  v = block_sum_t<256>(v, tmp);
  if (threadIdx.x == 0) rr_part[blockIdx.x] = v;
}

// beta = rr' / rr; p = r + beta p; per-workgroup partial sums of <O>.p.  The
// first workgroup keeps rr' for the next iteration.
__global__ __launch_bounds__(256) void cg_dir_kernel(int64_t P, const double *__restrict__ r,
                                                     double *__restrict__ p, const double *__restrict__ obar,
                                                     const double *__restrict__ rr_part, int npq,
                                                     double *__restrict__ op_part, double *__restrict__ scal,
                                                     int it) {
  __shared__ double tmp[4];
  if (scal[S_DONE] != 0.0) return;
  const double rr1 = sum_partials<256>(rr_part, npq, tmp);
  const double beta = rr1 / scal[S_RRP + (it & 1)];
  const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double v = 0.0;
  if (k < P) {
    const double pk = r[k] + beta * p[k];
    p[k] = pk;
    v = obar[k] * pk;
  }
  v = block_sum_t<256>(v, tmp);
  if (threadIdx.x == 0) {
    op_part[blockIdx.x] = v;
    if (blockIdx.x == 0) scal[S_RRP + ((it + 1) & 1)] = rr1;
  }
}

// <O>.p for the next matrix-vector product, the residual and the stopping test.
__global__ __launch_bounds__(256) void cg_fin_kernel(const double *__restrict__ op_part, int npq,
                                                     double *__restrict__ scal, int it, double tol,
                                                     int *__restrict__ status) {
  __shared__ double tmp[4];
  if (scal[S_DONE] != 0.0) return;
  const double obp = sum_partials<256>(op_part, npq, tmp);
  if (threadIdx.x == 0) {
    const double rr1 = scal[S_RRP + ((it + 1) & 1)];
    scal[S_RR] = rr1;
    scal[S_OBP] = obp;
    scal[S_ITERS] += 1.0;
    const double rel = sqrt(rr1) / scal[S_NORMF];
    scal[S_REL] = rel;
    if (rel <= tol) scal[S_DONE] = 1.0;
    if (!isfinite(rel)) {
      status[1] = 1;
      scal[S_DONE] = 1.0;
    }
  }
}

__global__ void scale_copy_kernel(const double *__restrict__ a, int64_t n, double s, double *__restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = a[k] * s;
}

// ------------------------------------------------------------- host side

static size_t al(size_t bytes) { return (bytes + 255) / 256 * 256; }

// row stride of the explicit matrices: even, so that rows are 16-byte aligned
static int64_t ld_even(int64_t n) { return (n + 1) & ~(int64_t)1; }

struct SrPlan {
  int method;
  int nch, rows_per_chunk;
  int npq;
  size_t off_scal, off_status, off_ec, off_obar, off_F, off_pa, off_pb, off_M, off_r, off_p, off_q,
      off_u, off_pq, off_rrp, off_opp, off_alpha, off_chol, total;
};

static SrPlan make_plan(int B, int64_t P, const vqmc_sr_opts *o) {
  SrPlan s{};
  if (o->method == 0) {
    // the smaller exact form while its matrix stays within order 65536
    constexpr int64_t kMaxExact = 65536;
    if (B < P) s.method = B <= kMaxExact ? 3 : 2;
    else s.method = P <= kMaxExact ? 1 : 2;
  } else {
    s.method = o->method;
  }
  const int64_t colblocks = (P + 1023) / 1024;  // column blocks of the 4-wide column pass
  int nch = (int)((4096 + colblocks - 1) / colblocks);
  nch = nch < 1 ? 1 : (nch > 64 ? 64 : nch);
  nch = nch > B ? B : nch;
  s.rows_per_chunk = (B + nch - 1) / nch;
  s.nch = (B + s.rows_per_chunk - 1) / s.rows_per_chunk;
  s.npq = (int)((P + 255) / 256);
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
    s.off_M = take((size_t)(P + 1) * ld_even(P) * 8);  // last row: right-hand side
    s.off_chol = take(chol_workspace_bytes(P));
  } else if (s.method == 2) {
    s.off_r = take((size_t)P * 8);
    s.off_p = take((size_t)P * 8);
    s.off_q = take((size_t)P * 8);
    s.off_u = take((size_t)B * 8);
    s.off_pq = take((size_t)s.npq * 8);
    s.off_rrp = take((size_t)s.npq * 8);
    s.off_opp = take((size_t)s.npq * 8);
  } else {
    s.off_M = take((size_t)(B + 1) * ld_even(B) * 8);
    s.off_alpha = take((size_t)B * 8);
    s.off_chol = take(chol_workspace_bytes(B));
  }
  s.total = off;
  return s;
}

bool sr_opts_valid(const vqmc_sr_opts *o) {
  return o && o->method >= 0 && o->method <= 3 && (o->s_prec == 0 || o->s_prec == 1) && o->eps > 0.0 &&
         o->tol >= 0.0 && o->max_iter >= 0;
}

int *sr_status_word(void *workspace, int32_t B, int64_t P, const vqmc_sr_opts *o) {
  return reinterpret_cast<int *>(reinterpret_cast<char *>(workspace) + make_plan(B, P, o).off_status);
}

}  // namespace vqmc

using namespace vqmc;

extern "C" vqmc_status vqmc_sr_workspace(int32_t B, int64_t P, const vqmc_sr_opts *o, size_t *bytes) {
  if (!sr_opts_valid(o) || !bytes) return VQMC_ERR_ARG;
  if (B < 2 || P < 1) return VQMC_ERR_SHAPE;
  *bytes = make_plan(B, P, o).total;
  return VQMC_OK;
}

extern "C" vqmc_status vqmc_sr_solve(const float *O, int64_t ldO, const double *e_loc, int32_t B, int64_t P,
                                     const vqmc_sr_opts *o, double *delta, double *F, void *workspace,
                                     size_t ws_bytes, vqmc_sr_info *info, hipStream_t st) {
  if (!sr_opts_valid(o)) return VQMC_ERR_ARG;
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
  // 16-byte loads of O when every row starts 16-byte aligned
  const bool vec = (reinterpret_cast<uintptr_t>(O) % 16 == 0) && (ldO % 4 == 0);
  // 16-byte loads in the tiled S / Gram kernels also need whole groups of 4 columns
  const bool tvec = vec && (P % 4 == 0);
  // <E>, Var E, E^c (and the Cholesky status cleared); <O>, F
  energy_stats_kernel<<<1, 1024, 0, st>>>(e_loc, B, ec, scal, status);
  const dim3 cgrid((unsigned)((P + 255) / 256), (unsigned)pl.nch);
  const dim3 cgrid4((unsigned)((P + 1023) / 1024), (unsigned)pl.nch);
  if (vec)
    col_partial4_kernel<false><<<cgrid4, 256, 0, st>>>(O, ldO, B, P, nullptr, nullptr, ec, pl.rows_per_chunk, pa,
                                                       pb, nullptr);
  else
    col_partial_kernel<false><<<cgrid, 256, 0, st>>>(O, ldO, B, P, nullptr, nullptr, ec, pl.rows_per_chunk, pa,
                                                     pb, nullptr);
  col_stats_finish_kernel<<<(unsigned)((P + 255) / 256), 256, 0, st>>>(pa, pb, pl.nch, P, B, scal, obar, Fv);
  VQMC_LAUNCH_CHECK();
  vqmc_status rc = VQMC_OK;
  if (pl.method == 1) {
    double *S = reinterpret_cast<double *>(ws + pl.off_M);
    const int64_t T = (P + 127) / 128, ldS = ld_even(P);
    const int nt = (int)(T * (T + 1) / 2);
    if (o->s_prec == 1) {
      if (tvec) syrk_dma_kernel<double, SYRK_KC><<<(unsigned)nt, 256, 0, st>>>(O, ldO, B, P, obar, o->eps, S, ldS, nt);
      else syrk_kernel<double><<<(unsigned)nt, 256, 0, st>>>(O, ldO, B, P, obar, o->eps, S, ldS, nt);
    } else {
      if (tvec) syrk_dma_kernel<float, SYRK_KC><<<(unsigned)nt, 256, 0, st>>>(O, ldO, B, P, obar, o->eps, S, ldS, nt);
      else syrk_kernel<float><<<(unsigned)nt, 256, 0, st>>>(O, ldO, B, P, obar, o->eps, S, ldS, nt);
    }
    VQMC_LAUNCH_CHECK();
    scale_copy_kernel<<<(unsigned)((P + 255) / 256), 256, 0, st>>>(Fv, P, 1.0, S + P * ldS);
    rc = chol_factor_solve(S, P, ldS, delta, ws + pl.off_chol, status, st);
  } else if (pl.method == 3) {
    double *K = reinterpret_cast<double *>(ws + pl.off_M);
    double *alpha = reinterpret_cast<double *>(ws + pl.off_alpha);
    const int64_t T = (B + 127) / 128, ldK = ld_even(B);
    const int nt = (int)(T * (T + 1) / 2);
    if (tvec) gram_dma_kernel<<<(unsigned)nt, 256, 0, st>>>(O, ldO, B, P, obar, o->eps, K, ldK, nt);
    else gram_kernel<<<(unsigned)nt, 256, 0, st>>>(O, ldO, B, P, obar, o->eps, K, ldK, nt);
    scale_copy_kernel<<<(unsigned)((B + 255) / 256), 256, 0, st>>>(ec, B, 1.0 / B, K + B * ldK);
    VQMC_LAUNCH_CHECK();
    rc = chol_factor_solve(K, B, ldK, alpha, ws + pl.off_chol, status, st);
    if (rc == VQMC_OK) {
      if (vec)
        col_partial4_kernel<true><<<cgrid4, 256, 0, st>>>(O, ldO, B, P, obar, alpha, nullptr, pl.rows_per_chunk,
                                                          pa, nullptr, nullptr);
      else
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
    double *rrp = reinterpret_cast<double *>(ws + pl.off_rrp);
    double *opp = reinterpret_cast<double *>(ws + pl.off_opp);
    constexpr int RB = 8;  // rows per workgroup of the row pass
    const unsigned rgrid = (unsigned)((B + RB - 1) / RB);
    cg_init_kernel<<<1, 1024, 0, st>>>(Fv, P, obar, delta, r, p, scal, status);
    for (int it = 0; it < o->max_iter; ++it) {
      if (vec) {
        cg_rowdot_kernel<RB, true><<<rgrid, 256, 0, st>>>(O, ldO, B, P, p, u, scal);
        col_partial4_kernel<true><<<cgrid4, 256, 0, st>>>(O, ldO, B, P, obar, u, nullptr, pl.rows_per_chunk, pa,
                                                          nullptr, scal);
      } else {
        cg_rowdot_kernel<RB, false><<<rgrid, 256, 0, st>>>(O, ldO, B, P, p, u, scal);
        col_partial_kernel<true><<<cgrid, 256, 0, st>>>(O, ldO, B, P, obar, u, nullptr, pl.rows_per_chunk, pa,
                                                        nullptr, scal);
      }
      cg_apply_kernel<<<(unsigned)pl.npq, 256, 0, st>>>(pa, pl.nch, P, B, o->eps, p, q, pq, scal);
      cg_update_kernel<<<(unsigned)pl.npq, 256, 0, st>>>(P, delta, r, p, q, pq, pl.npq, rrp, scal, it);
      cg_dir_kernel<<<(unsigned)pl.npq, 256, 0, st>>>(P, r, p, obar, rrp, pl.npq, opp, scal, it);
      cg_fin_kernel<<<1, 256, 0, st>>>(opp, pl.npq, scal, it, o->tol, status);
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
    if (hs[1]) return VQMC_ERR_NONFINITE;
    if (pl.method == 2 && h[S_DONE] == 0.0) return VQMC_WARN_NOT_CONVERGED;
  }
  return VQMC_OK;
}
