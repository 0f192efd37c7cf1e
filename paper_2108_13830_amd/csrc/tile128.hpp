// tile128.hpp -- 128 x 128 output tile of C += A B^T on the matrix cores.
//
// A and B are staged in LDS as panels of 128 rows (m) by KC (k), either
// k-contiguous ([m][k], "MK") or m-contiguous ([k][m], "KM"), whichever
// matches the source layout so that global loads are 16-byte vectors and LDS
// stores are 16-byte stores.  256 threads = 4 waves in 2 x 2, each wave a
// 64 x 64 sub-tile of 4 x 4 instruction tiles (16 x 16).  The K loop is
// software-pipelined: chunk c+1 is loaded into registers while the matrix
// cores consume chunk c from LDS.  Used by the explicit S (FP64 or FP32), the
// sample-space Gram matrix and the Cholesky trailing update.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "engine.hpp"

namespace vqmc {

template <typename T, int KC, bool KMAJOR>
struct Panel {
  // padding keeps rows 16-byte aligned and puts the four k-groups of an
  // MFMA operand read on disjoint LDS banks
  static constexpr int PAD = KMAJOR ? 16 : 16 / (int)sizeof(T);
  static constexpr int LD = (KMAJOR ? 128 : KC) + PAD;
  static constexpr int ROWS = KMAJOR ? KC : 128;
  T s[ROWS][LD];
  __device__ __forceinline__ T get(int m, int k) const { return KMAJOR ? s[k][m] : s[m][k]; }
};

template <typename T>
struct Tile128 {
  static constexpr bool F64 = sizeof(T) == 8;
  using acc_t = typename std::conditional<F64, f64x4, f32x4>::type;

  __device__ static __forceinline__ acc_t mma(T a, T b, acc_t c) {
    if constexpr (F64) return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }

  __device__ static __forceinline__ void zero(acc_t (&acc)[4][4]) {
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  }

  // acc += A[wm*64 .. +63][0..KC) * B[wn*64 .. +63][0..KC)^T
  template <int KC, bool KM>
  __device__ static __forceinline__ void step(const Panel<T, KC, KM> &A, const Panel<T, KC, KM> &B,
                                              acc_t (&acc)[4][4]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave >> 1, wn = wave & 1;
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int k = ks * 4 + (lane >> 4);
      T a[4], b[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        a[t] = A.get(wm * 64 + t * 16 + (lane & 15), k);
        b[t] = B.get(wn * 64 + t * 16 + (lane & 15), k);
      }
#pragma unroll
      for (int tm = 0; tm < 4; ++tm)
#pragma unroll
        for (int tn = 0; tn < 4; ++tn) acc[tm][tn] = mma(a[tm], b[tn], acc[tm][tn]);
    }
  }

  // Row and column (within the 128 x 128 tile) held by register r of
  // instruction tile (tm, tn) in this lane.  FP64 16x16x4: row l/16 + 4r;
  // FP32 16x16x4: row 4(l/16) + r; column l%16 for both.
  __device__ static __forceinline__ int row_of(int tm, int r) {
    const int lane = threadIdx.x & 63, wm = (threadIdx.x >> 6) >> 1;
    return wm * 64 + tm * 16 + (F64 ? ((lane >> 4) + 4 * r) : (4 * (lane >> 4) + r));
  }
  __device__ static __forceinline__ int col_of(int tn) {
    const int lane = threadIdx.x & 63, wn = (threadIdx.x >> 6) & 1;
    return wn * 64 + tn * 16 + (lane & 15);
  }

  // The pipelined K loop over nchunks chunks.  LD is a loader with
  //   typename LD::Regs;  load(Regs&, int chunk, bool b_side);
  //   store(const Regs&, Panel&)
  // run by all 256 threads.
  template <int KC, bool KM, class LD>
  __device__ static __forceinline__ void run(LD &ld, int nchunks, Panel<T, KC, KM> &sA, Panel<T, KC, KM> &sB,
                                             acc_t (&acc)[4][4]) {
    typename LD::Regs ra, rb;
    ld.load(ra, 0, false);
    ld.load(rb, 0, true);
    for (int c = 0; c < nchunks; ++c) {
      ld.store(ra, sA);
      ld.store(rb, sB);
      __syncthreads();
      if (c + 1 < nchunks) {
        ld.load(ra, c + 1, false);
        ld.load(rb, c + 1, true);
      }
      step<KC, KM>(sA, sB, acc);
      __syncthreads();
    }
  }
};

// Index (bi >= bj) of the t-th block of a lower block triangle.
__device__ __forceinline__ void lower_block(int t, int &bi, int &bj) {
  int i = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
  while ((i + 1) * (i + 2) / 2 <= t) ++i;
  while (i * (i + 1) / 2 > t) --i;
  bi = i;
  bj = t - i * (i + 1) / 2;
}

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2):
// renumber them so that XCD x runs a contiguous range of tiles, whose tiles
// share row panels in that XCD's L2.
__device__ __forceinline__ int xcd_contiguous(int b, int nt) {
  const int q = nt >> 3, r = nt & 7, x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

}  // namespace vqmc
