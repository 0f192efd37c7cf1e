// engine.hpp -- fused forward pass of the convolutional amplitude on gfx950.
//
// The amplitude of Sec. 2.2 (Eq. wcnn) is a stack of periodic 3x3
// convolutions: a 1 -> C lift followed by n C -> C layers, tanh after each,
// and log|W_CNN| = sum over channels and sites of the last layer's output.
//
// One workgroup evaluates a batch of G configurations at once.  The batch's
// G*N lattice sites are the rows of one implicit GEMM per layer:
//   out[row][co] = sum_{tap, ci} act[nb(row, tap)][ci] * W[co][ci][tap],
// with K = 9*C ordered tap-major (k = tap*C + ci).  Activations live in LDS
// for the whole pass (one buffer, updated in place: every wave keeps its
// output tiles in registers until all waves have finished reading the
// layer's input).  The weights of a layer are staged once per batch in LDS in
// the exact per-lane fragment order of the matrix instruction, so each
// K-step reads them with one conflict-free LDS load per lane.
//
// Matrix instructions (64-wide wavefronts, 16x16 output tiles):
//   FP32   v_mfma_f32_16x16x4_f32   A: act[row=lane%16][k=4s+lane/16]
//   BF16   v_mfma_f32_16x16x32_bf16 A: act[row=lane%16][k=32s+8(lane/16)+j]
// both with D[row=4(lane/16)+i][col=lane%16], i = 0..3.  With the operands
// swapped the same instructions give the transposed tile (lane: four
// consecutive channels of one row), which the BF16 forms and the light cone
// use so that outputs leave in 4-channel pieces.
// BF16X3 splits each operand into hi + lo BF16 parts and accumulates
// hi*hi + hi*lo + lo*hi (three products per K-step) in FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vqmc {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

enum Prec { P_F32 = 0, P_BF16 = 1, P_X3 = 2 };

__device__ __forceinline__ int wrapL(int a, int L) { return a < 0 ? a + L : (a >= L ? a - L : a); }

// Site of S read at site i of T^r S, T the quarter turn of Eq. (sym-ws):
// (T S)(y, x) = S(x, L-1-y), so T^2 reads (L-1-y, L-1-x) and T^3 (L-1-x, y).
__device__ __forceinline__ int rot_src(int i, int r, int L) {
  const int y = i / L, x = i - y * L;
  switch (r) {
    case 0: return i;
    case 1: return x * L + (L - 1 - y);
    case 2: return (L - 1 - y) * L + (L - 1 - x);
    default: return (L - 1 - x) * L + y;
  }
}

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  __bf16 h = (__bf16)x;
  return __builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float bf16_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));

// Two floats rounded to nearest-even BF16 by one packed conversion: a in the
// low half, b in the high half.
__device__ __forceinline__ uint32_t bf16x2_rne(float a, float b) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector((f32x2_t{a, b}), bf16x2_t));
}

// Four consecutive values as BF16 pairs hi = bf16(h) and, for the split form,
// lo = bf16(h - hi) (the subtractions are plain FP32 ones).
template <bool SPLIT>
__device__ __forceinline__ void bf16_split4(const float (&h)[4], uint2 &hi, uint2 &lo) {
  hi = uint2{bf16x2_rne(h[0], h[1]), bf16x2_rne(h[2], h[3])};
  if constexpr (SPLIT) {
    const float r0 = h[0] - __uint_as_float(hi.x << 16), r1 = h[1] - __uint_as_float(hi.x & 0xffff0000u);
    const float r2 = h[2] - __uint_as_float(hi.y << 16), r3 = h[3] - __uint_as_float(hi.y & 0xffff0000u);
    lo = uint2{bf16x2_rne(r0, r1), bf16x2_rne(r2, r3)};
  }
}

__device__ __forceinline__ f32x4 mma_f32(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mma_bf16(u16x8 a, u16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a),
                                                  __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
}

typedef __attribute__((address_space(3))) void *lds_ptr_t;

// Starts copying one layer's packed fragments (bytes, a multiple of 1 KiB)
// into LDS with direct-to-LDS loads: no registers are involved and each wave
// instruction moves 1 KiB.  The copy is complete once every thread has
// passed wait_copies() and a barrier.
template <int NTHR>
__device__ __forceinline__ void stage_async(char *dst, const char *__restrict__ src, int bytes) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int c = wave; c < (bytes >> 10); c += NTHR / 64)
    __builtin_amdgcn_global_load_lds(src + (size_t)c * 1024 + lane * 16, (lds_ptr_t)(dst + c * 1024), 16, 0, 0);
}

// The same copy with a fixed, compile-time number of loads per wave
// (ceil(chunks / NW); waves past the last chunk copy it again: the same
// bytes to the same place).  A fixed count lets the compiler wait for loads
// issued before the copy without waiting for the copy itself.
template <int NW, int BYTES>
__device__ __forceinline__ void stage_async_fixed(char *dst, const char *__restrict__ src) {
  constexpr int CH = BYTES >> 10, PER = (CH + NW - 1) / NW;
  static_assert(BYTES % 1024 == 0 && CH > 0, "copies move whole 1 KiB pieces");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int c = wave + p * NW < CH ? wave + p * NW : CH - 1;
    __builtin_amdgcn_global_load_lds(src + (size_t)c * 1024 + lane * 16, (lds_ptr_t)(dst + c * 1024), 16, 0, 0);
  }
}

// Waits for this thread's outstanding memory operations (the direct-to-LDS
// copies included).
__device__ __forceinline__ void wait_copies() { __builtin_amdgcn_s_waitcnt(0); }

// tanh(x) = 1 - 2 / (exp(2x) + 1): one exponential and one hardware
// reciprocal (1 ulp); absolute error ~2e-7 over the whole real line
// (saturates to +-1).
__device__ __forceinline__ float tanh_f(float x) {
  const float e = __expf(2.f * x);
  return 1.f - 2.f * __builtin_amdgcn_rcpf(e + 1.f);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

// Parameter offsets in the flat theta vector (layer 0: lift, then C -> C).
__host__ __device__ inline int64_t layer_offset(int C, int l) {
  return l == 0 ? 0 : (int64_t)10 * C + (int64_t)(l - 1) * (9 * C * C + C);
}

template <int C, int PREC, int NW, int TPW>
struct Engine {
  static constexpr int NT = (C + 15) / 16;  // 16-wide output tiles per row tile
  static constexpr bool F32 = PREC == P_F32;
  static constexpr bool X3 = PREC == P_X3;
  static constexpr int KSTEP = F32 ? 4 : 32;
  static constexpr int KS = (9 * C + KSTEP - 1) / KSTEP;
  static constexpr int LDA = F32 ? C + 1 : C;  // FP32 rows padded by one word
  static constexpr int FRAG = F32 ? 4 : (X3 ? 32 : 16);
  // BF16 fragments are stored as 16-byte pieces in [block][part][lane] order
  // (block = idx / 64 of the lane-order index idx, part 0 = hi, 1 = lo), so
  // that the 64 lanes of a wave read one part as 1 KiB of consecutive bytes.
  __host__ __device__ static constexpr int frag_piece(int idx, int part) {
    return ((idx >> 6) * (FRAG / 16) + part) * 64 + (idx & 63);
  }
  static constexpr int NTHR = NW * 64;
  static constexpr int MAXROWS = NW * TPW * 16;
  // FP32: padded rows; BF16 forms: hi (and lo) planes.  At least
  // MAXROWS * C floats, which the head reuses for the last layer's outputs.
  static constexpr int ACT_BYTES = F32 ? MAXROWS * LDA * 4 : MAXROWS * C * 4;
  static constexpr int FRAG_BYTES = KS * NT * 64 * FRAG;
  static_assert(F32 ? (C % 4 == 0) : (C % 8 == 0), "channel count not supported");
  static_assert(MAXROWS * C * 4 <= ACT_BYTES, "the head reuses the activation buffer");

  // BF16 activation planes: rows of 2C bytes, 128/C of them per 256-byte
  // span of the 64 LDS banks.  The 8-element (16-byte) groups of a row are
  // XOR-swizzled by the row's span index, so that the 16 consecutive rows of
  // a tile, read 16 bytes each, fall on 16 distinct 4-bank groups.
  __device__ static __forceinline__ int phys(int row, int c) {
    if constexpr (C >= 16) {
      constexpr int RSH = C == 16 ? 3 : 2;  // log2(128 / C)
      return row * C + ((((c >> 3) ^ ((row >> RSH) & (C / 8 - 1))) << 3) | (c & 7));
    } else {
      return row * C + c;
    }
  }

  // Four consecutive channels co0..co0+3 of one row (co0 a multiple of 4):
  // one 8-byte store per BF16 plane (the four lie in one swizzled 8-group).
  __device__ static __forceinline__ void store_act4(char *act, int row, int co0, const float (&h)[4]) {
    if constexpr (F32) {
      float *p = reinterpret_cast<float *>(act) + row * LDA + co0;
#pragma unroll
      for (int j = 0; j < 4; ++j) p[j] = h[j];
    } else {
      uint16_t *hi = reinterpret_cast<uint16_t *>(act);
      const int pi = phys(row, co0);
      uint2 vh, vl;
      bf16_split4<X3>(h, vh, vl);
      *reinterpret_cast<uint2 *>(hi + pi) = vh;
      if constexpr (X3) *reinterpret_cast<uint2 *>(hi + MAXROWS * C + pi) = vl;
    }
  }

  __device__ static __forceinline__ void store_act(char *act, int row, int c, float h) {
    if constexpr (F32) {
      reinterpret_cast<float *>(act)[row * LDA + c] = h;
    } else {
      uint16_t *hi = reinterpret_cast<uint16_t *>(act);
      const uint16_t bh = bf16_rne(h);
      hi[phys(row, c)] = bh;
      if constexpr (X3) hi[MAXROWS * C + phys(row, c)] = bf16_rne(h - bf16_f32(bh));
    }
  }

  // Weight fragments of a C -> C layer: entry (s, nt, lane) holds
  // B[k][n] = W[n][ci][tap] for n = 16 nt + lane%16 and k = tap*C + ci from
  // the lane's K slice of step s (zero outside the layer).  TRANSPOSED uses
  // B[k][n] = W[ci][n][tap] (k = tap*C + ci): the input-gradient GEMM.
  template <bool TRANSPOSED = false>
  __device__ static __forceinline__ float wsel(const float *W, int k, int n) {
    if (k >= 9 * C || n >= C) return 0.f;
    const int tap = k / C, ci = k - tap * C;
    return TRANSPOSED ? W[(ci * C + n) * 9 + tap] : W[(n * C + ci) * 9 + tap];
  }

  // Stages W_l (theta order W[co][ci][tap], 9C^2 floats) in the fragment
  // order above: the reads are coalesced (thread t takes elements t,
  // t + NTHR, ...) and each element is scattered to its slot; the K padding
  // of the BF16 forms (k in [9C, 32 KS)) and, for C < 16, the columns
  // [C, 16) are written as zeros by slots of their own, so no slot is
  // written twice.
  __device__ static __forceinline__ void stage_weights(const float *__restrict__ W, char *frag) {
    constexpr int WN = 9 * C * C;
    for (int idx = threadIdx.x; idx < WN; idx += NTHR) {
      const float w = W[idx];
      const int n = idx / (9 * C), rem = idx - n * (9 * C), ci = rem / 9, tap = rem - ci * 9;
      const int k = tap * C + ci, nt = n >> 4;
      if constexpr (F32) {
        reinterpret_cast<float *>(frag)[((k >> 2) * NT + nt) * 64 + (k & 3) * 16 + (n & 15)] = w;
      } else {
        const int kk = k & 31;
        const int piece = frag_piece(((k >> 5) * NT + nt) * 64 + (kk >> 3) * 16 + (n & 15), 0);
        uint16_t *f = reinterpret_cast<uint16_t *>(frag);
        const uint16_t hi = bf16_rne(w);
        f[piece * 8 + (kk & 7)] = hi;
        if constexpr (X3) f[(piece + 64) * 8 + (kk & 7)] = bf16_rne(w - bf16_f32(hi));
      }
    }
    if constexpr (C < 16) {
      // columns n in [C, 16) of the one 16-wide output tile are zero
      constexpr int KT = KS * (F32 ? 4 : 32), NP = 16 - C;
      for (int p = threadIdx.x; p < KT * NP; p += NTHR) {
        const int k = p / NP, n = C + (p - (p / NP) * NP);
        if constexpr (F32) {
          reinterpret_cast<float *>(frag)[(k >> 2) * 64 + (k & 3) * 16 + n] = 0.f;
        } else {
          const int kk = k & 31;
          const int piece = frag_piece((k >> 5) * 64 + (kk >> 3) * 16 + n, 0);
          uint16_t *f = reinterpret_cast<uint16_t *>(frag);
          f[piece * 8 + (kk & 7)] = 0;
          if constexpr (X3) f[(piece + 64) * 8 + (kk & 7)] = 0;
        }
      }
    }
    if constexpr (!F32) {
      constexpr int PADK = 32 * KS - 9 * C;  // zero rows of the last K-step
      for (int p = threadIdx.x; p < PADK * C; p += NTHR) {
        const int k = 9 * C + p / C, n = p - (p / C) * C, kk = k & 31, nt = n >> 4;
        const int piece = frag_piece(((k >> 5) * NT + nt) * 64 + (kk >> 3) * 16 + (n & 15), 0);
        uint16_t *f = reinterpret_cast<uint16_t *>(frag);
        f[piece * 8 + (kk & 7)] = 0;
        if constexpr (X3) f[(piece + 64) * 8 + (kk & 7)] = 0;
      }
    }
  }

  // Lift layer: h_1[row][co] = tanh(b0[co] + sum_tap W0[co][tap] s[nb(row,tap)]).
  __device__ static __forceinline__ void lift(const float *__restrict__ theta, const int8_t *sp, int R, int L, int N,
                              char *act) {
    const float *W0 = theta;
    const float *b0 = theta + 9 * C;
    for (int idx = threadIdx.x; idx < R * C; idx += NTHR) {
      const int row = idx / C, co = idx - row * C;
      const int g = row / N, site = row - g * N, y = site / L, x = site - y * L;
      float z = b0[co];
#pragma unroll
      for (int tap = 0; tap < 9; ++tap) {
        const int yy = wrapL(y + tap / 3 - 1, L), xx = wrapL(x + tap % 3 - 1, L);
        z += W0[co * 9 + tap] * (float)sp[g * N + yy * L + xx];
      }
      store_act(act, row, co, tanh_f(z));
    }
  }

  __device__ static __forceinline__ int nbrow(int pk, int dy, int dx, int L) {
    return (pk >> 10) + wrapL(((pk >> 5) & 31) + dy, L) * L + wrapL((pk & 31) + dx, L);
  }

  // K loop of one conv layer over the wave's row tiles; results stay in acc.
  // FRAG_GLOBAL: fragments read from a packed global array (else from LDS).
  // SIGN = -1 gathers act[row - d(tap)] (input-gradient direction).
  template <bool FRAG_GLOBAL, int SIGN>
  __device__ static __forceinline__ void kloop(const char *act, const char *frag, int R, int L,
                                               int N, f32x4 (&acc)[TPW][NT]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // per tile: the lane's row packed as (g*N) << 10 | y << 5 | x
    int pk[TPW];
#pragma unroll
    for (int i = 0; i < TPW; ++i) {
      int r = (wave + i * NW) * 16 + (lane & 15);
      r = r < R ? r : R - 1;
      const int g = r / N, site = r - g * N, y = site / L;
      pk[i] = ((g * N) << 10) | (y << 5) | (site - y * L);
    }
    kloop_pk<FRAG_GLOBAL, SIGN>(act, frag, pk, L, acc);
  }

  // The same K loop for rows given directly as packed (row base, y, x):
  // tile i of this wave reads the lane's row pk[i].  Only the first NTILE
  // tile slots are computed (NTILE <= TPW, compile time).
  template <bool FRAG_GLOBAL, int SIGN, int NTILE = TPW>
  __device__ static __forceinline__ void kloop_pk(const char *act, const char *frag, const int (&pk)[TPW],
                                                  int L, f32x4 (&acc)[TPW][NT]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < TPW; ++i)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[i][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    // Software-pipelined: the A operands of K-step s+1 are requested from
    // LDS before the matrix instructions of step s are issued.  Every tile
    // slot runs (rows past R are clamped copies whose results are never
    // stored), so no branch separates the loads from the matrix
    // instructions.
    if constexpr (F32) {
      const float *actf = reinterpret_cast<const float *>(act);
      const float *fragf = reinterpret_cast<const float *>(frag);
      constexpr int SPT = C / 4;  // K-steps per tap
      int nbo[NTILE];
      float a_cur[NTILE], a_nxt[NTILE];
#pragma unroll
      for (int i = 0; i < NTILE; ++i) {
        nbo[i] = nbrow(pk[i], -SIGN, -SIGN, L) * LDA + (lane >> 4);
        a_cur[i] = actf[nbo[i]];
      }
#pragma unroll 2
      for (int s = 0; s < KS; ++s) {
        float b[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) b[nt] = fragf[(s * NT + nt) * 64 + lane];
        if (s + 1 < KS) {
          const int s1 = s + 1, tap1 = s1 / SPT, c41 = s1 - tap1 * SPT;
          if (c41 == 0) {
            const int dy = SIGN * (tap1 / 3 - 1), dx = SIGN * (tap1 % 3 - 1);
#pragma unroll
            for (int i = 0; i < NTILE; ++i) nbo[i] = nbrow(pk[i], dy, dx, L) * LDA + (lane >> 4);
          }
#pragma unroll
          for (int i = 0; i < NTILE; ++i) a_nxt[i] = actf[nbo[i] + c41 * 4];
        }
#pragma unroll
        for (int i = 0; i < NTILE; ++i)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) acc[i][nt] = mma_f32(a_cur[i], b[nt], acc[i][nt]);
#pragma unroll
        for (int i = 0; i < NTILE; ++i) a_cur[i] = a_nxt[i];
      }
    } else {
      const uint16_t *hi = reinterpret_cast<const uint16_t *>(act);
      for (int s = 0; s < KS; ++s) {
        u16x8 bh[NT], bl[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const u16x8 *f = reinterpret_cast<const u16x8 *>(frag) + frag_piece((s * NT + nt) * 64 + lane, 0);
          bh[nt] = f[0];
          if constexpr (X3) bl[nt] = f[64];
        }
        const int k0 = 32 * s + 8 * (lane >> 4);
        const bool kv = k0 < 9 * C;
        const int tap = kv ? k0 / C : 0, ci0 = kv ? k0 - tap * C : 0;
        const int dy = SIGN * (tap / 3 - 1), dx = SIGN * (tap % 3 - 1);
        // lanes whose K slice lies past 9C read row 0 and multiply zero weights
        u16x8 ah[NTILE], al[NTILE];
#pragma unroll
        for (int i = 0; i < NTILE; ++i) {
          const int nb = kv ? nbrow(pk[i], dy, dx, L) : 0;
          ah[i] = *reinterpret_cast<const u16x8 *>(hi + phys(nb, ci0));
          if constexpr (X3) al[i] = *reinterpret_cast<const u16x8 *>(hi + MAXROWS * C + phys(nb, ci0));
        }
#pragma unroll
        for (int i = 0; i < NTILE; ++i)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            acc[i][nt] = mma_bf16(ah[i], bh[nt], acc[i][nt]);
            if constexpr (X3) {
              acc[i][nt] = mma_bf16(ah[i], bl[nt], acc[i][nt]);
              acc[i][nt] = mma_bf16(al[i], bh[nt], acc[i][nt]);
            }
          }
      }
    }
  }

  // Neighbour table of the implicit GEMM, built once per kernel:
  // nbt[tap][r] = row of site (y + tap/3 - 1, x + tap%3 - 1) (periodic) of
  // the configuration of row r = g*N + y*L + x; rows past G*N use the last
  // row.  It replaces the per-K-step index arithmetic of the gather.
  static constexpr int NBT_ELEMS = 9 * MAXROWS;
  __device__ static __forceinline__ void build_nbt(uint16_t *nbt, int G, int L, int N) {
    const int Rf = G * N;
    for (int idx = threadIdx.x; idx < NBT_ELEMS; idx += NTHR) {
      const int tap = idx / MAXROWS, r0 = idx - tap * MAXROWS;
      const int r = r0 < Rf ? r0 : Rf - 1;
      const int g = r / N, site = r - g * N, y = site / L, x = site - y * L;
      nbt[idx] = (uint16_t)(g * N + wrapL(y + tap / 3 - 1, L) * L + wrapL(x + tap % 3 - 1, L));
    }
  }

  // Lift layer on the FP32 matrix cores: K = 9 taps padded to 12,
  // A[row][tap] = s[nb(row, tap)] (exact +-1), B[tap][co] = W0[co][tap],
  // in the forward pass's tile orientation.
  __device__ static __forceinline__ void lift_tab(const float *__restrict__ theta, const int8_t *sp,
                                                  const uint16_t *nbt, int R, char *act) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const float *W0 = theta;
    f32x4 acc[TPW][NT];
#pragma unroll
    for (int i = 0; i < TPW; ++i)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[i][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      const int k = 4 * s + (lane >> 4);
      const bool kv = k < 9;
      const int kk = kv ? k : 0;
      float b[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int n = nt * 16 + (lane & 15);
        const float w = W0[(n < C ? n : C - 1) * 9 + kk];
        b[nt] = (kv && n < C) ? w : 0.f;
      }
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
        const int row = (wave + i * NW) * 16 + (lane & 15);
        const float a = (float)sp[nbt[kk * MAXROWS + row]];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
          acc[i][nt] = FWD_TR ? mma_f32(b[nt], kv ? a : 0.f, acc[i][nt]) : mma_f32(kv ? a : 0.f, b[nt], acc[i][nt]);
      }
    }
    write_fwd(acc, theta + 9 * C, R, act);
  }

  // K loop of one C -> C layer over the wave's row tiles with the gather
  // rows read from the neighbour table; results stay in acc.  In the BF16
  // forms a last tile slot that starts at or past row R (a batch shorter
  // than MAXROWS) is not computed: its acc stays zero and none of its rows
  // is stored.
  template <bool TR = false>
  __device__ static __forceinline__ void kloop_tab(const char *act, const char *frag, const uint16_t *nbt,
                                                   f32x4 (&acc)[TPW][NT], int R = MAXROWS) {
    const int lane = threadIdx.x & 63;
    const int wave = F32 ? threadIdx.x >> 6 : __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int rowi[TPW];
#pragma unroll
    for (int i = 0; i < TPW; ++i) rowi[i] = (wave + i * NW) * 16 + (lane & 15);
    if constexpr (TPW > 1 && !F32) {
      if ((wave + (TPW - 1) * NW) * 16 >= R) {
        kloop_rows<TPW - 1, TR>(act, frag, nbt, rowi, acc);
        return;
      }
    }
    kloop_rows<TPW, TR>(act, frag, nbt, rowi, acc);
  }

  // The same K loop for tile i of this wave reading the lane's table column
  // rowi[i] (the output row's own index into nbt); only the first NTILE tile
  // slots are computed (compile time).
  // TR: the product is formed transposed, out^T = W^T act^T, by passing the
  // weight fragments as the instruction's first operand (the per-lane
  // layouts of the two operands coincide).  Then acc[i][nt][j] is
  // out[row = 16 T + lane%16][co = 16 nt + 4 (lane/16) + j]: every lane holds
  // four consecutive channels of one row, written with one wide store, and
  // the row is the one the lane gathers for.
  template <int NTILE, bool TR = false>
  __device__ static __forceinline__ void kloop_rows(const char *act, const char *frag, const uint16_t *nbt,
                                                    const int (&rowi)[TPW], f32x4 (&acc)[TPW][NT]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < TPW; ++i)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) acc[i][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    if constexpr (F32) {
      // A: act[nb][4 c4 + lane/16]; the four K-steps of a tap use the same
      // gather row, at immediate offsets
      const float *actf = reinterpret_cast<const float *>(act) + (lane >> 4);
      const float *fragf = reinterpret_cast<const float *>(frag) + lane;
      constexpr int SPT = C / 4;
#pragma unroll 3
      for (int tap = 0; tap < 9; ++tap) {
        int nb[NTILE];
#pragma unroll
        for (int i = 0; i < NTILE; ++i) nb[i] = (int)nbt[tap * MAXROWS + rowi[i]] * LDA;
#pragma unroll
        for (int c4 = 0; c4 < SPT; ++c4) {
          const int s = tap * SPT + c4;
          float b[NT], a[NTILE];
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) b[nt] = fragf[(s * NT + nt) * 64];
#pragma unroll
          for (int i = 0; i < NTILE; ++i) a[i] = actf[nb[i] + 4 * c4];
#pragma unroll
          for (int i = 0; i < NTILE; ++i)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
              acc[i][nt] = TR ? mma_f32(b[nt], a[i], acc[i][nt]) : mma_f32(a[i], b[nt], acc[i][nt]);
        }
      }
    } else {
      const uint16_t *hi = reinterpret_cast<const uint16_t *>(act);
      // fully unrolled: the table and activation reads of step s+1 can be
      // issued while the matrix instructions of step s run
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        u16x8 bh[NT], bl[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const u16x8 *f = reinterpret_cast<const u16x8 *>(frag) + frag_piece((s * NT + nt) * 64 + lane, 0);
          bh[nt] = f[0];
          if constexpr (X3) bl[nt] = f[64];
        }
        const int k0 = 32 * s + 8 * (lane >> 4);
        const bool kv = k0 < 9 * C;
        // lanes whose K slice lies past 9C read a valid row and multiply zero weights
        const int tap = kv ? k0 / C : 0, ci0 = kv ? k0 - tap * C : 0;
        u16x8 ah[NTILE], al[NTILE];
#pragma unroll
        for (int i = 0; i < NTILE; ++i) {
          const int nb = nbt[tap * MAXROWS + rowi[i]];
          ah[i] = *reinterpret_cast<const u16x8 *>(hi + phys(nb, ci0));
          if constexpr (X3) al[i] = *reinterpret_cast<const u16x8 *>(hi + MAXROWS * C + phys(nb, ci0));
        }
#pragma unroll
        for (int i = 0; i < NTILE; ++i)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt) {
            if constexpr (TR) {
              acc[i][nt] = mma_bf16(bh[nt], ah[i], acc[i][nt]);
              if constexpr (X3) {
                acc[i][nt] = mma_bf16(bl[nt], ah[i], acc[i][nt]);
                acc[i][nt] = mma_bf16(bh[nt], al[i], acc[i][nt]);
              }
            } else {
              acc[i][nt] = mma_bf16(ah[i], bh[nt], acc[i][nt]);
              if constexpr (X3) {
                acc[i][nt] = mma_bf16(ah[i], bl[nt], acc[i][nt]);
                acc[i][nt] = mma_bf16(al[i], bh[nt], acc[i][nt]);
              }
            }
          }
      }
    }
  }

  // Writes tanh(acc + bias) of the wave's tiles into the activation buffer
  // (and, when scratch != nullptr, into scratch[row][co] in global memory).
  template <bool ACT = true>
  __device__ static __forceinline__ void write_tiles(const f32x4 (&acc)[TPW][NT], const float *bias,
                                                     int R, char *act, float *scratch) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int co = nt * 16 + (lane & 15);
      const float bv = co < C ? bias[co] : 0.f;
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
        const int T = wave + i * NW;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = T * 16 + (lane >> 4) * 4 + j;
          if (row < R && co < C) {
            const float h = ACT ? tanh_f(acc[i][nt][j] + bv) : acc[i][nt][j];
            store_act(act, row, co, h);
            if (scratch) scratch[row * C + co] = h;
          }
        }
      }
    }
  }

  // write_tiles for transposed tiles (TR above): tanh(acc + bias) of four
  // consecutive channels per lane and row, one wide store each.
  template <bool ACT = true>
  __device__ static __forceinline__ void write_tiles_t(const f32x4 (&acc)[TPW][NT], const float *bias, int R,
                                                       char *act) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int co0 = nt * 16 + 4 * (lane >> 4);
      if (co0 < C) {
        float bv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) bv[j] = bias[co0 + j];
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
          const int row = (wave + i * NW) * 16 + (lane & 15);
          if (row < R) {
            float h[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) h[j] = ACT ? tanh_f(acc[i][nt][j] + bv[j]) : acc[i][nt][j];
            store_act4(act, row, co0, h);
          }
        }
      }
    }
  }

  // head_vals for transposed tiles.
  template <bool ACT = true>
  __device__ static __forceinline__ void head_vals_t(const f32x4 (&acc)[TPW][NT], const float *bias, int R,
                                                     float *hv) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int co0 = nt * 16 + 4 * (lane >> 4);
      if (co0 < C) {
        float bv[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) bv[j] = bias[co0 + j];
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
          const int row = (wave + i * NW) * 16 + (lane & 15);
          if (row < R) {
            f32x4 h;
#pragma unroll
            for (int j = 0; j < 4; ++j) h[j] = ACT ? tanh_f(acc[i][nt][j] + bv[j]) : acc[i][nt][j];
            *reinterpret_cast<f32x4 *>(hv + row * C + co0) = h;
          }
        }
      }
    }
  }

  // The last layer's outputs tanh(acc + bias) as floats hv[row][C] (the
  // activation buffer, free once every wave has finished the layer's K loop).
  template <bool ACT = true>
  __device__ static __forceinline__ void head_vals(const f32x4 (&acc)[TPW][NT], const float *bias, int R,
                                                   float *hv) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int co = nt * 16 + (lane & 15);
      const float bv = co < C ? bias[co] : 0.f;
#pragma unroll
      for (int i = 0; i < TPW; ++i) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int row = (wave + i * NW) * 16 + (lane >> 4) * 4 + j;
          if (row < R && co < C) hv[row * C + co] = ACT ? tanh_f(acc[i][nt][j] + bv) : acc[i][nt][j];
        }
      }
    }
  }

  // Full forward pass of G configurations sp[G][N] (LDS) -> lp[G] (LDS,
  // FP64).  smem_act / smem_frag are this engine's LDS regions; nbt is the
  // neighbour table built by build_nbt for at least G configurations.
  // Begins and ends with the block synchronised.
  // packed (nullable): the C -> C layers' fragments in this order, packed
  // once per call (pack_layer_frags_kernel); each layer then arrives by
  // direct-to-LDS copies that run while the previous layer's outputs are
  // written.  Without it the weights are staged from theta.
  static constexpr int FRAG_LAYER = KS * NT * 64 * FRAG;
  static constexpr bool DMA_OK = FRAG_LAYER % 1024 == 0;
  // Tile orientation of the forward pass: transposed for the BF16 forms,
  // whose per-output work (tanh, rounding, 16-bit stores) outweighs their
  // matrix work at these channel counts; FP32 keeps the row-major tiles,
  // which measured faster there (scalar stores either way).
  static constexpr bool FWD_TR = !F32;
  template <bool ACT = true>
  __device__ static __forceinline__ void write_fwd(const f32x4 (&acc)[TPW][NT], const float *bias, int R,
                                                   char *act) {
    if constexpr (FWD_TR) write_tiles_t<ACT>(acc, bias, R, act);
    else write_tiles<ACT>(acc, bias, R, act, nullptr);
  }

  // tanh(acc + bias) in place, in the forward pass's tile orientation
  __device__ static __forceinline__ void act_tanh(f32x4 (&acc)[TPW][NT], const float *bias) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      float bv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int co = FWD_TR ? nt * 16 + 4 * (lane >> 4) + j : nt * 16 + (lane & 15);
        bv[j] = co < C ? bias[co] : 0.f;
      }
#pragma unroll
      for (int i = 0; i < TPW; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][nt][j] = tanh_f(acc[i][nt][j] + bv[j]);
    }
  }
  __device__ static __forceinline__ void forward(const float *__restrict__ theta, int n_layers, const int8_t *sp,
                                                 int G, int N, char *smem_act, char *smem_frag,
                                                 const uint16_t *nbt, double *lp,
                                                 const char *__restrict__ packed = nullptr) {
    const int R = G * N;
    const bool dma = DMA_OK && packed != nullptr;
    if (dma) stage_async<NTHR>(smem_frag, packed, FRAG_LAYER);
    else stage_weights(theta + layer_offset(C, 1), smem_frag);
    lift_tab(theta, sp, nbt, R, smem_act);
    if (dma) wait_copies();
    __syncthreads();
    for (int l = 1; l <= n_layers; ++l) {
      f32x4 acc[TPW][NT];
      kloop_tab<FWD_TR>(smem_act, smem_frag, nbt, acc, R);
      const float *bias = theta + layer_offset(C, l) + 9 * C * C;
      // FP32: the activation is applied in registers before the barrier, so
      // a wave that finishes its K loop early spends the wait on it and only
      // the stores wait for the other waves' reads of this layer's input; the
      // BF16 forms apply it after the barrier (their 448-row form has no
      // registers to spare)
      if constexpr (F32) act_tanh(acc, bias);
      __syncthreads();
      if (l < n_layers) {
        if (dma) {
          stage_async<NTHR>(smem_frag, packed + (size_t)l * FRAG_LAYER, FRAG_LAYER);
          write_fwd<!F32>(acc, bias, R, smem_act);
          wait_copies();
        } else {
          write_fwd<!F32>(acc, bias, R, smem_act);
          stage_weights(theta + layer_offset(C, l + 1), smem_frag);
        }
      } else if constexpr (FWD_TR) {
        head_vals_t<!F32>(acc, bias, R, reinterpret_cast<float *>(smem_act));
      } else {
        head_vals<!F32>(acc, bias, R, reinterpret_cast<float *>(smem_act));
      }
      __syncthreads();
    }
    // log|W_CNN| of each configuration: its N*C outputs summed in FP64 in a
    // fixed order (lane-strided partial sums, then the wave's xor tree)
    const float *hv = reinterpret_cast<const float *>(smem_act);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int g = wave; g < G; g += NW) {
      double p = 0.0;
      for (int idx = lane; idx < N * C; idx += 64) p += (double)hv[g * N * C + idx];
      p = wave_sum(p);
      if (lane == 0) lp[g] = p;
    }
    __syncthreads();
  }
};



// Packs the C -> C layers' weights in the engine's per-lane fragment order
// for precision PREC: [layer][KS][NT][64] fragments.
template <int C, int PREC>
__global__ void pack_layer_frags_kernel(const float *__restrict__ theta, int n_layers, char *__restrict__ out) {
  using E = Engine<C, PREC, 1, 1>;
  constexpr int PER = E::KS * E::NT * 64;
  const int total = n_layers * PER;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
    const int l = t / PER + 1, idx = t - (l - 1) * PER;
    const int s = idx / (E::NT * 64), r2 = idx - s * (E::NT * 64);
    const int nt = r2 >> 6, ln = r2 & 63;
    const int n = nt * 16 + (ln & 15);
    const float *W = theta + layer_offset(C, l);
    if constexpr (PREC == P_F32) {
      reinterpret_cast<float *>(out)[t] = E::wsel(W, 4 * s + (ln >> 4), n);
    } else {
      const int k0 = 32 * s + 8 * (ln >> 4);
      u16x8 hi, lo;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const float w = E::wsel(W, k0 + j, n);
        hi[j] = bf16_rne(w);
        lo[j] = bf16_rne(w - bf16_f32(hi[j]));
      }
      reinterpret_cast<u16x8 *>(out)[E::frag_piece(t, 0)] = hi;
      if constexpr (PREC == P_X3) reinterpret_cast<u16x8 *>(out)[E::frag_piece(t, 1)] = lo;
    }
  }
}

template <int C, int PREC>
constexpr size_t frag_bytes_per_layer() {
  using E = Engine<C, PREC, 1, 1>;
  return (size_t)E::KS * E::NT * 64 * E::FRAG;
}

}  // namespace vqmc
