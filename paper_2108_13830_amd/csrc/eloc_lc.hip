// eloc_lc.hip -- local energy by incremental evaluation inside light cones.
//
// For an exchanged configuration s' = s with the pair (i, j) swapped, the
// input changes on two sites only, so after the l-th 3x3 convolution the
// activations differ from those of s only within Chebyshev distance l of the
// pair (its "light cone").  The kernel runs the dense forward pass of s once
// per sample (FP32), keeps e^{2 z_l(s)} of every pre-activation z_l(s) in a
// per-workgroup scratch slice, and then for each s' propagates only the
// difference:
//   dz_l = W_l (*) dh_{l-1}           (matrix cores, rows = cone sites)
//   dh_l = tanh(z_l + dz_l) - tanh(z_l) = tanh(dz_l) (1 - tanh(z_l) tanh(z_l + dz_l))
// and log|W(s')| - log|W(s)| = sum over the last cone of dh_{n+1}.  The
// difference of activations is what enters the convolutions, so rounding it to
// BF16 (single or split) costs relative precision of the difference, not of
// the activations.  The local energy is the same sum as in the dense kernel
// (Eq. Es-Os-G with the bonds of Sec. 3.1).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "common.hpp"
#include "eloc_lc.hpp"
#include "engine.hpp"

namespace vqmc {

namespace {

template <int NW>
__device__ __forceinline__ double bsum(double v, double *tmp) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) tmp[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) t += tmp[w];
  __syncthreads();
  return t;
}

template <int NW>
__device__ __forceinline__ int bisum(int v, int *tmp) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) tmp[threadIdx.x >> 6] = v;
  __syncthreads();
  int t = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) t += tmp[w];
  __syncthreads();
  return t;
}

template <int NW>
__device__ __forceinline__ int bscan(int v, int *tmp, int *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) tmp[wave] = x;
  __syncthreads();
  int base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    base += (w < wave) ? tmp[w] : 0;
    tot += tmp[w];
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

// The dense pass stores E_a = e^{2a} of every pre-activation a, clamped to
// a in [-40, 40] (e^80 < FLT_MAX; tanh is exactly +-1 in FP32 long before):
// tanh(a) = 1 - 2 / (E_a + 1).
__device__ __forceinline__ float exp2x(float a) { return __expf(2.f * fminf(fmaxf(a, -40.f), 40.f)); }

// tanh(a + b) - tanh(a) from E_a = e^{2a}, with the relative accuracy of b.
// With E_c = E_a e^{2b}:
//   tanh(a + b) - tanh(a) = 2 (E_c - E_a) / ((E_c + 1)(E_a + 1)),
// where E_c - E_a = 2 E_a sinh(b) e^b is taken as 2 E_a s(b), s(b) =
// (e^{2b} - 1) / 2 from its series (six terms, truncation below 5e-8
// relative) when |b| < 0.125, and as the plain difference otherwise (the two
// then differ by a factor e^{0.25} or more, so the difference loses at most a
// factor 4.5 in relative accuracy).  E_c is formed as the product E_a e^{2b}
// (never as E_a + (E_c - E_a), which cancels when e^{2b} rounds against 1)
// and capped at 1e30: beyond it tanh(a + b) = 1 in FP32.  Where the
// denominator overflows (E_a > 3e8 with E_c capped) the result is 0, within
// 1e-8 of the exact 2 / (E_a + 1).  One exponential (the hardware 2^x of
// 2b log2 e) and one reciprocal.  The factors 2 are folded in exactly (powers
// of two scale without rounding): the series gives 2 s(b), and the
// denominator is (E_c + 1)(E_a + 1) / 2.
__device__ __forceinline__ float tanh_diff(float ea, float b) {
  const float e = __builtin_amdgcn_exp2f(fminf(b * 2.8853900817779268f, 126.f));
  const float ec = fminf(ea * e, 1e30f);
  const float sb2 =
      b * (2.f + b * (2.f + b * (4.f / 3.f + b * (2.f / 3.f + b * (4.f / 15.f + b * (4.f / 45.f))))));
  // both candidates are formed and one is picked bitwise (a conditional
  // expression here compiles to a branch per element)
  const int sel = -(int)(fabsf(b) < 0.125f);
  const int u = __float_as_int(ea * sb2), t = __float_as_int(ec - ea);
  const float num = __int_as_float(t ^ ((t ^ u) & sel));
  const float h = fmaf(ea, 0.5f, 0.5f);  // (E_a + 1) / 2
  return num * __builtin_amdgcn_rcpf(fmaf(ec, h, h));
}

// Unwrapped bounding box of the exchanged pair of bond k: rows y0..y0+ey,
// columns x0..x0+ex (x0 may be -1 for the lower-left bond).
__device__ __forceinline__ void pair_box(int k, int L, int N, int &i, int &j, int &kind, int &y0, int &x0,
                                         int &ey, int &ex) {
  kind = k / N;
  const int site = k - kind * N, y = site / L, x = site - y * L;
  i = site;
  y0 = y;
  ey = kind > 0 ? 1 : 0;
  switch (kind) {
    case 0: x0 = x; ex = 1; j = y * L + wrapL(x + 1, L); break;
    case 1: x0 = x; ex = 0; j = wrapL(y + 1, L) * L + x; break;
    case 2: x0 = x; ex = 1; j = wrapL(y + 1, L) * L + wrapL(x + 1, L); break;
    default: x0 = x - 1; ex = 1; j = wrapL(y + 1, L) * L + wrapL(x - 1, L); break;
  }
}

// The cone box at distance l: start row/col and extent, clipped to the torus.
struct Box {
  int ys, xs, H, W;
  __device__ __forceinline__ void set(int y0, int x0, int ey, int ex, int l, int L) {
    H = ey + 1 + 2 * l;
    W = ex + 1 + 2 * l;
    ys = y0 - l;
    xs = x0 - l;
    if (H >= L) {
      H = L;
      ys = 0;
    }
    if (W >= L) {
      W = L;
      xs = 0;
    }
  }
  // lattice site of box row r (row-major over the box), without integer
  // division: r / W from a float reciprocal with half-row margin
  __device__ __forceinline__ int site(int r, int L) const {
    const int ry = (int)(((float)r + 0.5f) * __builtin_amdgcn_rcpf((float)W));
    const int rx = r - ry * W;
    int y = ys + ry, x = xs + rx;
    y += y < 0 ? L : 0;
    y -= y >= L ? L : 0;
    x += x < 0 ? L : 0;
    x -= x >= L ? L : 0;
    return y * L + x;
  }
};

// LDS plan of the kernel.  One region serves two phases in turn:
//   dense pass of s:  FP32 activations [MR][C+1] | one layer's FP32 fragments
//                     | neighbour table
//   difference pass:  the fragments of two layers (the current one and the
//                     next, copied while the current one runs) | two
//                     difference buffers indexed by the row of the cone box
//                     (odd boxes in one, even boxes in the other), each with
//                     one extra row that stays zero.
template <int C, int PREC, int NW, int TPW>
struct LC {
  using E32 = Engine<C, P_F32, NW, TPW>;
  using EP = Engine<C, PREC, NW, TPW>;
  static constexpr int NT = E32::NT;
  static constexpr int MR = E32::MAXROWS;
  static constexpr int FRAG32 = E32::FRAG_BYTES;
  static constexpr int FRAGP = EP::FRAG_BYTES;
  static constexpr int BASE = E32::ACT_BYTES + FRAG32 + E32::NBT_ELEMS * 2;
  // bytes per difference row: FP32 rows of C + 1 floats, or BF16 planes
  static constexpr int ROWB = PREC == P_F32 ? 4 * (C + 1) : (PREC == P_X3 ? 4 * C : 2 * C);
  static constexpr int SLOTS = 32;  // log-ratio parts in flight (two groups of 16)
  static constexpr int FIXED = MR + 8 * MR + 8 * SLOTS * NW + 8 * NW + 4 * NW;
  static constexpr int LIMIT = 160 * 1024 - 512;
  static constexpr int ROWS_FIT = (LIMIT - FIXED - 2 * FRAGP) / ROWB;
  // rows of both difference buffers together (zero rows included)
  static constexpr int ROWS = ROWS_FIT < 2 * MR + 2 ? ROWS_FIT : 2 * MR + 2;
  static constexpr int SPASS = 2 * FRAGP + ROWS * ROWB;
  // spill slot of a paired configuration's box of distance 4 (at most 100
  // rows), whole 1 KiB pieces for the direct-to-LDS copies
  static constexpr int SPILL_BYTES = (100 * ROWB + 1023) / 1024 * 1024;
  static constexpr int REGION = ((BASE > SPASS ? BASE : SPASS) + 15) / 16 * 16;
  static_assert(REGION + FIXED <= 160 * 1024, "LDS plan exceeds the workgroup's 160 KiB");
  static_assert(FRAGP % 1024 == 0 && FRAG32 % 1024 == 0, "fragment blocks are copied in 1 KiB pieces");
};

// Rows of the largest cone box of distance l (the exchanged pair spans at
// most 2x2 sites; clipped to the torus).
__host__ __device__ inline int box_rows_max(int l, int L) {
  const int e = 2 + 2 * l < L ? 2 + 2 * l : L;
  return e * e;
}

// Capacities (rows, zero row excluded) of the odd-box and even-box buffers
// for n layers: the stored boxes are those of distance 1 .. n.
__host__ __device__ inline void lc_caps(int n, int L, int &cap_odd, int &cap_even) {
  cap_odd = box_rows_max((n & 1) ? n : n - 1, L);
  cap_even = n >= 2 ? box_rows_max((n & 1) ? n - 1 : n, L) : 0;
}

// Difference buffer of cap + 1 rows (row cap stays zero): FP32 rows of C + 1
// floats, or the BF16 hi plane of (cap + 1) * C values followed (split form)
// by the lo plane; rows are swizzled as in the engine.
template <int C, int PREC>
__device__ __forceinline__ void dstore4(char *buf, int cap, int row, int co0, const float (&h)[4]) {
  using E = Engine<C, PREC, 1, 1>;
  if constexpr (PREC == P_F32) {
    float *p = reinterpret_cast<float *>(buf) + row * (C + 1) + co0;
#pragma unroll
    for (int j = 0; j < 4; ++j) p[j] = h[j];
  } else {
    uint16_t *hi = reinterpret_cast<uint16_t *>(buf);
    const int pi = E::phys(row, co0);
    uint2 vh, vl;
    bf16_split4<PREC == P_X3>(h, vh, vl);
    *reinterpret_cast<uint2 *>(hi + pi) = vh;
    if constexpr (PREC == P_X3) *reinterpret_cast<uint2 *>(hi + (cap + 1) * C + pi) = vl;
  }
}

template <int C, int PREC>
__device__ __forceinline__ int dbuf_bytes(int cap) {
  return PREC == P_F32 ? (cap + 1) * (C + 1) * 4 : (cap + 1) * C * (PREC == P_X3 ? 4 : 2);
}

__device__ __forceinline__ int sel3(const int (&v)[3], int d) { return d == 0 ? v[0] : (d == 1 ? v[1] : v[2]); }

// K loop of one C -> C layer of the difference pass over the first NTILE
// tile slots, in transposed tiles (acc[i][nt][j]: channel 16 nt + 4 (lane/16)
// + j of the lane's output row).  The input of the lane's row at tap
// (dy, dx) is row ro[i][dy] + cf[i][dx] of the input box, or the zero row
// cap when that sum is negative (outside the box).
template <int C, int PREC, int TPW, int NTILE>
__device__ __forceinline__ void kloop_box(const char *in, int cap, const char *frag, const int (&ro)[TPW][3],
                                          const int (&cf)[TPW][3], f32x4 (&acc)[TPW][(C + 15) / 16]) {
  using E = Engine<C, PREC, 1, 1>;
  constexpr int NT = E::NT;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < TPW; ++i)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[i][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
  if constexpr (PREC == P_F32) {
    const float *actf = reinterpret_cast<const float *>(in) + (lane >> 4);
    const float *fragf = reinterpret_cast<const float *>(frag) + lane;
    constexpr int SPT = C / 4;
#pragma unroll 3
    for (int tap = 0; tap < 9; ++tap) {
      const int dy = tap / 3, dx = tap - 3 * dy;
      int nb[NTILE];
#pragma unroll
      for (int i = 0; i < NTILE; ++i) {
        const int g = sel3(ro[i], dy) + sel3(cf[i], dx);
        nb[i] = (int)min((unsigned)g, (unsigned)cap) * (C + 1);  // outside the box: the zero row
      }
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
          for (int nt = 0; nt < NT; ++nt) acc[i][nt] = mma_f32(b[nt], a[i], acc[i][nt]);
      }
    }
  } else {
    const uint16_t *hi = reinterpret_cast<const uint16_t *>(in);
    const uint16_t *lo = hi + (cap + 1) * C;
#pragma unroll
    for (int s = 0; s < E::KS; ++s) {
      u16x8 bh[NT], bl[NT];
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const u16x8 *f = reinterpret_cast<const u16x8 *>(frag) + E::frag_piece((s * NT + nt) * 64 + lane, 0);
        bh[nt] = f[0];
        if constexpr (PREC == P_X3) bl[nt] = f[64];
      }
      const int k0 = 32 * s + 8 * (lane >> 4);
      const bool kv = k0 < 9 * C;
      // with C >= 32 a K-step lies within one tap (known at compile time);
      // lanes whose K slice lies past 9C read a valid row and multiply zero
      // weights
      const int tap = C >= 32 ? (32 * s) / C : (kv ? k0 / C : 0);
      const int ci0 = kv ? k0 - tap * C : 0;
      const int dy = tap / 3, dx = tap - 3 * dy;
      u16x8 ah[NTILE], al[NTILE];
#pragma unroll
      for (int i = 0; i < NTILE; ++i) {
        // a negative index (outside the box) is huge as unsigned: the minimum
        // with cap picks the zero row; rows of the box lie below cap
        const int g = sel3(ro[i], dy) + sel3(cf[i], dx);
        const int p = E::phys((int)min((unsigned)g, (unsigned)cap), ci0);
        ah[i] = *reinterpret_cast<const u16x8 *>(hi + p);
        if constexpr (PREC == P_X3) al[i] = *reinterpret_cast<const u16x8 *>(lo + p);
      }
#pragma unroll
      for (int i = 0; i < NTILE; ++i)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          acc[i][nt] = mma_bf16(bh[nt], ah[i], acc[i][nt]);
          if constexpr (PREC == P_X3) {
            acc[i][nt] = mma_bf16(bl[nt], ah[i], acc[i][nt]);
            acc[i][nt] = mma_bf16(bh[nt], al[i], acc[i][nt]);
          }
        }
    }
  }
}

template <int V>
struct IntC {
  static constexpr int value = V;
};

// Calls f(IntC<n>) for the wave-uniform n in [0, TPW].
template <int TPW, int K = 0, class F>
__device__ __forceinline__ void with_tiles(int n, F &f) {
  if constexpr (K <= TPW) {
    if (n == K) {
      f(IntC<K>{});
      return;
    }
    with_tiles<TPW, K + 1>(n, f);
  }
}

// a - b reduced to [0, L) for a - b in (-L, 2L)
__device__ __forceinline__ int mod_once(int v, int L) {
  v += v < 0 ? L : 0;
  return v >= L ? v - L : v;
}

template <int C, int PREC, int NW, int TPW, bool PAIRS>
__global__ __launch_bounds__(NW * 64) void eloc_lc_kernel(const float *__restrict__ theta,
                                                          const char *__restrict__ frag32,
                                                          const char *__restrict__ fragp,
                                                          const int8_t *__restrict__ spins, int B, int L,
                                                          int n_layers, double J1, double J2, int marshall,
                                                          int cap_odd, int cap_even,
                                                          float *__restrict__ zscratch,
                                                          char *__restrict__ spill,
                                                          double *__restrict__ e_loc,
                                                          int32_t *__restrict__ flags,
                                                          double *__restrict__ lp_out) {
  using K = LC<C, PREC, NW, TPW>;
  using E32 = typename K::E32;
  constexpr int NT = K::NT;
  constexpr int MR = K::MR;
  constexpr int NTHR = NW * 64;
  __shared__ __align__(16) char s_region[K::REGION];
  __shared__ int8_t s_sig[MR];
  __shared__ int16_t s_bonds[4 * MR];
  __shared__ double s_dl[K::SLOTS * NW];  // per-wave parts of the log-ratios in flight
  __shared__ double s_red[NW];
  __shared__ int s_ired[NW];
  // dense pass of s
  char *s_act = s_region;
  char *s_frag = s_region + E32::ACT_BYTES;
  uint16_t *s_nbt = reinterpret_cast<uint16_t *>(s_region + E32::ACT_BYTES + K::FRAG32);
  // difference pass
  // fragment buffer i (0, 1) of the difference pass: s_region + i * K::FRAGP
  char *s_dodd = s_region + 2 * K::FRAGP;
  char *s_deven = s_dodd + dbuf_bytes<C, PREC>(cap_odd);
  // the wave index is uniform across the wave: kept in a scalar register,
  // so that per-wave tile counts branch on scalars
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int N = L * L, NB = 4 * N;
  float *zsc = zscratch + (size_t)blockIdx.x * (n_layers + 1) * N * C;
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    const int8_t *s = spins + (size_t)b * N;
    // the first FP32 layer's fragments arrive while the bonds are scanned
    stage_async<NTHR>(s_frag, frag32, K::FRAG32);
    // neighbour table of the single configuration, nbt[tap][site] (the
    // difference pass reuses its room)
    E32::build_nbt(s_nbt, 1, L, N);
    int sz = 0, bad = 0;
    for (int i = tid; i < N; i += NTHR) {
      const int8_t v = s[i];
      s_sig[i] = v;
      sz += v;
      bad += (v != 1 && v != -1);
    }
    sz = bisum<NW>(sz, s_ired);
    bad = bisum<NW>(bad, s_ired);
    // ---- bond scan (diagonal term, ordered antiparallel list)
    const int chunk = (NB + NTHR - 1) / NTHR;
    const int k0 = tid * chunk, k1 = min(k0 + chunk, NB);
    double dsum = 0.0;
    int cnt = 0;
    for (int k = k0; k < k1; ++k) {
      int i, j, kind, y0, x0, ey, ex;
      pair_box(k, L, N, i, j, kind, y0, x0, ey, ex);
      const int si = s_sig[i], sj = s_sig[j];
      dsum += 0.25 * (kind < 2 ? J1 : J2) * (double)(si * sj);
      cnt += (si != sj);
    }
    int total;
    int off = bscan<NW>(cnt, s_ired, &total);
    for (int k = k0; k < k1; ++k) {
      int i, j, kind, y0, x0, ey, ex;
      pair_box(k, L, N, i, j, kind, y0, x0, ey, ex);
      if (s_sig[i] != s_sig[j]) s_bonds[off++] = (int16_t)k;
    }
    const double diag = bsum<NW>(dsum, s_red);

    // ---- dense FP32 forward of s, keeping e^{2 z_l(s)} of every pre-activation
    {
      const float *W0 = theta, *b0 = theta + 9 * C;
      for (int idx = tid; idx < N * C; idx += NTHR) {
        const int row = idx / C, co = idx - row * C;
        float z = b0[co];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) z += W0[co * 9 + tap] * (float)s_sig[s_nbt[tap * MR + row]];
        zsc[idx] = exp2x(z);
        E32::store_act(s_act, row, co, tanh_f(z));
      }
      wait_copies();
      __syncthreads();
      for (int l = 1; l <= n_layers; ++l) {
        // transposed tiles: lane holds channels co0..co0+3 of one row
        f32x4 acc[TPW][NT];
        E32::template kloop_tab<true>(s_act, s_frag, s_nbt, acc);
        __syncthreads();
        // next: the following FP32 layer, or the first layer of the
        // difference pass (into the first fragment buffer, which overlaps
        // room of this pass that is no longer read)
        if (l < n_layers) stage_async<NTHR>(s_frag, frag32 + (size_t)l * K::FRAG32, K::FRAG32);
        else stage_async<NTHR>(s_region, fragp, K::FRAGP);
        const float *bias = theta + layer_offset(C, l) + 9 * C * C;
        float *zl = zsc + (size_t)l * N * C;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int co0 = nt * 16 + 4 * (lane >> 4);
          float bv[4];
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) bv[jj] = bias[co0 + jj];
#pragma unroll
          for (int i = 0; i < TPW; ++i) {
            const int row = (wave + i * NW) * 16 + (lane & 15);
            if (row < N) {
              f32x4 e;
              float h[4];
#pragma unroll
              for (int jj = 0; jj < 4; ++jj) {
                const float z = acc[i][nt][jj] + bv[jj];
                e[jj] = exp2x(z);
                h[jj] = tanh_f(z);
              }
              *reinterpret_cast<f32x4 *>(zl + row * C + co0) = e;
              if (l < n_layers) E32::store_act4(s_act, row, co0, h);
            }
          }
        }
        wait_copies();
        __syncthreads();
      }
      if (lp_out) {
        // log|W_CNN(s)| from the stored last-layer pre-activations
        const float *zn = zsc + (size_t)n_layers * N * C;
        double lp = 0.0;
        for (int idx = tid; idx < N * C; idx += NTHR)
          lp += (double)(1.f - 2.f * __builtin_amdgcn_rcpf(zn[idx] + 1.f));
        lp = bsum<NW>(lp, s_red);
        if (tid == 0) lp_out[b] = lp;
      }
    }

    // ---- every exchanged configuration.  Layer l reads the differences on
    // the box of distance l (odd l: s_dodd, even l: s_deven) and writes those
    // on the box of distance l + 1 into the other buffer, so one barrier per
    // layer suffices; the fragments of the layer after the current one are
    // copied into the other fragment buffer meanwhile.  Each wave leaves its
    // part of the log-ratio in s_dl; thread 0 turns them into terms 16 at a
    // time (in s' order, the waves' parts summed in wave order).
    // zero rows of the odd buffer (nb = 1) or of both (nb = 2; the dense pass
    // used their room)
    auto zero_rows = [&](int nb) {
      const int wb = PREC == P_F32 ? (C + 1) : (PREC == P_X3 ? C : C / 2);  // 32-bit words per zero row
      for (int idx = tid; idx < nb * wb; idx += NTHR) {
        const int bsel = idx / wb, w = idx - bsel * wb;
        char *buf = bsel ? s_deven : s_dodd;
        const int cap = bsel ? cap_even : cap_odd;
        uint32_t *p;
        if constexpr (PREC == P_F32) {
          p = reinterpret_cast<uint32_t *>(buf) + cap * (C + 1) + w;
        } else {
          // hi plane row cap, then (split form) lo plane row cap
          const int half = C / 2;  // words per plane row
          p = w < half ? reinterpret_cast<uint32_t *>(buf) + cap * half + w
                       : reinterpret_cast<uint32_t *>(buf) + (cap + 1) * half + cap * half + (w - half);
        }
        *p = 0u;
      }
    };
    zero_rows(2);
    // lift of s' q into the odd buffer at row base: dz_1 = sum_tap W0[c][tap]
    // ds(x + d(tap)) on the box of distance 1, four channels per item, the
    // items on threads t0 .. t0 + nthr - 1
    auto lift = [&](int q, int base, int t0, int nthr) {
      if (tid < t0 || tid >= t0 + nthr) return;
      int bi, bj, kind, y0, x0, ey, ex;
      pair_box(s_bonds[q], L, N, bi, bj, kind, y0, x0, ey, ex);
      const float dsi = (float)(s_sig[bj] - s_sig[bi]);  // change of spin at bi (at bj: -dsi)
      const int yi = bi / L, xi = bi - yi * L, yj = bj / L, xj = bj - yj * L;
      Box bx;
      bx.set(y0, x0, ey, ex, 1, L);
      const int R = bx.H * bx.W;
      for (int idx = tid - t0; idx < R * (C / 4); idx += nthr) {
        const int r = idx / (C / 4), co0 = 4 * (idx - r * (C / 4));
        const int site = bx.site(r, L), y = site / L, x = site - y * L;
        // bi and bj each enter through one tap of x at most (L >= 4: the nine
        // taps of a site are nine distinct sites): tap (ty, tx), ty = (y_b -
        // y + 1) mod L, tx likewise, when both are at most 2
        const int tyi = mod_once(yi - y + 1, L), txi = mod_once(xi - x + 1, L);
        const int tyj = mod_once(yj - y + 1, L), txj = mod_once(xj - x + 1, L);
        const bool hi_ = tyi <= 2 && txi <= 2, hj = tyj <= 2 && txj <= 2;
        const int ti = hi_ ? 3 * tyi + txi : 0, tj = hj ? 3 * tyj + txj : 0;
        float dz[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const float wi = hi_ ? theta[(co0 + j) * 9 + ti] : 0.f, wj = hj ? theta[(co0 + j) * 9 + tj] : 0.f;
          // the sum of the nine taps' terms (the other seven are zero); + 0
          // keeps a row that neither site reaches at +0
          dz[j] = fmaf(wj, -dsi, wi * dsi) + 0.f;
        }
        const f32x4 e = *reinterpret_cast<const f32x4 *>(zsc + site * C + co0);
        float dh[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) dh[j] = tanh_diff(e[j], dz[j]);
        dstore4<C, PREC>(s_dodd, cap_odd, base + r, co0, dh);
      }
    };
    double eacc = diag;  // thread 0's
    bool finite = true;
    auto flush = [&](int q_end, int count) {
      for (int qq = q_end - count; qq < q_end; ++qq) {
        double dlog = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) dlog += s_dl[(qq & (K::SLOTS - 1)) * NW + w];
        const int kind = s_bonds[qq] / N;
        const double J = kind < 2 ? J1 : J2;
        const double mu = (marshall && kind < 2) ? -1.0 : 1.0;
        finite = finite && isfinite(dlog);
        eacc += 0.5 * J * mu * exp(dlog);
      }
    };
    // Pairs (PAIRS): s' q and q + 1 share the steps of layers 1 .. 3, waves
    // 0 .. NW/2 - 1 on q and the others on q + 1, the second one's boxes at
    // row offsets so (odd buffer) and se (even buffer); its box of distance 4
    // goes to a per-workgroup spill slot in global memory, comes back into
    // the odd buffer by direct-to-LDS copy during the first one's last layer
    // (n even: the odd buffer is free then) and is moved into the even
    // buffer before its own layers 4 .. n (that copy may cover the odd
    // buffer's zero rows: they are cleared again).
    const int so = box_rows_max(3, L), se = box_rows_max(2, L);
    char *spl = PAIRS ? spill + (size_t)blockIdx.x * K::SPILL_BYTES : nullptr;
    auto lift_next = [&](int qn) {
      if (PAIRS && qn + 1 < total) {
        lift(qn, 0, 0, NTHR / 2);
        lift(qn + 1, so, NTHR / 2, NTHR / 2);
      } else {
        lift(qn, 0, 0, NTHR);
      }
    };
    struct PB {
      int y0, x0, ey, ex;
    };
    auto pbox = [&](int q) {
      PB p;
      int bi, bj, kind;
      pair_box(s_bonds[q], L, N, bi, bj, kind, p.y0, p.x0, p.ey, p.ex);
      return p;
    };
    int t = 0;  // layer steps run so far: the current step's fragments are in buffer t & 1
    // One layer step: layer l of the s' whose box is pa (HALF = 0, every
    // wave), or of the pair pa, pb (HALF = 1, l <= 3); the fragments of layer
    // fidx + 1 are copied meanwhile (fidx < 0: none).  Returns the wave's part
    // of the log-ratio at the last layer.
    auto step = [&](auto half_c, int l, const PB &pa, const PB &pb, int fidx) {
      constexpr bool HALF = decltype(half_c)::value;
      constexpr int NWS = HALF ? NW / 2 : NW;
      const int hb = HALF ? (wave >= NW / 2 ? 1 : 0) : 0;
      const int wv = wave - hb * (NW / 2);
      const PB &pq = hb ? pb : pa;
      const int in_base = hb ? ((l & 1) ? so : se) : 0;
      const int out_base = hb ? ((l & 1) ? se : so) : 0;
      const bool to_spill = HALF && hb && l == 3;
      double part = 0.0;
      const char *din = (l & 1) ? s_dodd : s_deven;
      const int cap_in = (l & 1) ? cap_odd : cap_even;
      char *dout = (l & 1) ? s_deven : s_dodd;
      const int cap_out = (l & 1) ? cap_even : cap_odd;
      Box bo, bn;
      bn.set(pq.y0, pq.x0, pq.ey, pq.ex, l, L);      // input box
      bo.set(pq.y0, pq.x0, pq.ey, pq.ex, l + 1, L);  // output box
      const int R = bo.H * bo.W;
      // tiles of this wave in the output box (wave-uniform)
      const int Ttot = (R + 15) / 16;
      const int nti = Ttot > wv ? (Ttot - wv + NWS - 1) / NWS : 0;
      const float *zl = zsc + (size_t)l * N * C;
      const char *fcur = s_region + (t & 1) * K::FRAGP;
      // the next step's fragments go into the other buffer, read last by the
      // previous step
      const bool copy_next = fidx >= 0;
      char *fnext = s_region + ((t + 1) & 1) * K::FRAGP;
      const char *fsrc = fragp + (size_t)(copy_next ? fidx : 0) * K::FRAGP;
      // One compile-time body per tile count of this wave: the loaded
      // exponentials are used only inside it (a register copy at a branch
      // merge would wait for them, and for the fragment copy issued after
      // them, before the K loop).
      auto body = [&](auto ntile) {
        constexpr int NTILE = decltype(ntile)::value;
        // the lane's output row in tile slot i (rows past the box repeat
        // the last one and are not stored): its lattice site, and the rows
        // of the input box that its 3x3 neighbourhood reads
        int site[TPW], ro[TPW][3], cf[TPW][3];
#pragma unroll
        for (int i = 0; i < NTILE; ++i) {
          int r = (wv + i * NWS) * 16 + (lane & 15);
          r = r < R ? r : R - 1;
          const int ry = (int)(((float)r + 0.5f) * __builtin_amdgcn_rcpf((float)bo.W)), rx = r - ry * bo.W;
          const int y = mod_once(bo.ys + ry, L), x = mod_once(bo.xs + rx, L);
          site[i] = y * L + x;
          const int ay = mod_once(y - bn.ys, L), ax = mod_once(x - bn.xs, L);
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            // ay, ax lie in [0, L): only the neighbour above (left) can
            // wrap, to L - 1, and only the one below (right), to 0
            int vy = ay + d - 1, vx = ax + d - 1;
            if (d == 0) {
              vy = vy < 0 ? L - 1 : vy;
              vx = vx < 0 ? L - 1 : vx;
            } else if (d == 2) {
              vy = vy >= L ? 0 : vy;
              vx = vx >= L ? 0 : vx;
            }
            ro[i][d] = vy < bn.H ? in_base + vy * bn.W : -(1 << 20);
            cf[i][d] = vx < bn.W ? vx : -(1 << 20);
          }
        }
        // the stored e^{2 z_l(s)} of the lane's rows, requested before the
        // K loop so that the matrix work covers the memory latency
        f32x4 za[TPW][NT];
#pragma unroll
        for (int i = 0; i < NTILE; ++i)
#pragma unroll
          for (int nt = 0; nt < NT; ++nt)
            za[i][nt] = *reinterpret_cast<const f32x4 *>(zl + site[i] * C + nt * 16 + 4 * (lane >> 4));
        if (copy_next) stage_async_fixed<NW, K::FRAGP>(fnext, fsrc);
        if constexpr (NTILE > 0) {
          f32x4 acc[TPW][NT];
          kloop_box<C, PREC, TPW, NTILE>(din, cap_in, fcur, ro, cf, acc);
#pragma unroll
          for (int i = 0; i < NTILE; ++i) {
            const int r = (wv + i * NWS) * 16 + (lane & 15);
            if (r < R) {
#pragma unroll
              for (int nt = 0; nt < NT; ++nt) {
                float dh[4];
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) dh[jj] = tanh_diff(za[i][nt][jj], acc[i][nt][jj]);
                if (HALF || l < n_layers) {
                  if (to_spill) dstore4<C, PREC>(spl, R - 1, r, nt * 16 + 4 * (lane >> 4), dh);
                  else dstore4<C, PREC>(dout, cap_out, out_base + r, nt * 16 + 4 * (lane >> 4), dh);
                } else {
#pragma unroll
                  for (int jj = 0; jj < 4; ++jj) part += (double)dh[jj];
                }
              }
            }
          }
        }
      };
      // a pair's boxes (at most 100 rows, 7 tiles) give each of the NW / 2
      // waves of a configuration at most two tiles
      with_tiles<(HALF && TPW > 2) ? 2 : TPW>(nti, body);
      return part;
    };
    if (total > 0) lift_next(0);
    __syncthreads();
    if constexpr (!PAIRS) {
      // one s' at a time (kept apart from the paired form's step code, which
      // the compiler schedules differently)
      for (int q = 0; q < total; ++q) {
        int bi, bj, kind, y0, x0, ey, ex;
        pair_box(s_bonds[q], L, N, bi, bj, kind, y0, x0, ey, ex);
        // every wave has written its parts of s' q-16 .. q-1 (before a barrier);
        // the slots written meanwhile (s' q onwards) are the other 16
        if (tid == 0 && q > 0 && (q & 15) == 0) flush(q, 16);
        double part = 0.0;
        for (int l = 1; l <= n_layers; ++l) {
          const char *din = (l & 1) ? s_dodd : s_deven;
          const int cap_in = (l & 1) ? cap_odd : cap_even;
          char *dout = (l & 1) ? s_deven : s_dodd;
          const int cap_out = (l & 1) ? cap_even : cap_odd;
          Box bo, bn;
          bn.set(y0, x0, ey, ex, l, L);      // input box
          bo.set(y0, x0, ey, ex, l + 1, L);  // output box
          const int R = bo.H * bo.W;
          // tiles of this wave in the output box (wave-uniform)
          const int Ttot = (R + 15) / 16;
          const int nti = Ttot > wave ? (Ttot - wave + NW - 1) / NW : 0;
          // the lane's output row in tile slot i (rows past the box repeat the
          // last one and are not stored): its lattice site, and the rows of
          // the input box that its 3x3 neighbourhood reads
          const float *zl = zsc + (size_t)l * N * C;
          const char *fcur = s_region + (t & 1) * K::FRAGP;
          // the next layer's fragments (after the last layer: the first one's,
          // for the next s') go into the other buffer, read last by the
          // previous layer
          const bool copy_next = l < n_layers || q + 1 < total;
          char *fnext = s_region + ((t + 1) & 1) * K::FRAGP;
          const char *fsrc = fragp + (size_t)(l < n_layers ? l : 0) * K::FRAGP;
          // One compile-time body per tile count of this wave: the loaded
          // exponentials are used only inside it (a register copy at a branch
          // merge would wait for them, and for the fragment copy issued after
          // them, before the K loop).
          auto body = [&](auto ntile) {
            constexpr int NTILE = decltype(ntile)::value;
            // the lane's output row in tile slot i (rows past the box repeat
            // the last one and are not stored): its lattice site, and the rows
            // of the input box that its 3x3 neighbourhood reads
            int site[TPW], ro[TPW][3], cf[TPW][3];
#pragma unroll
            for (int i = 0; i < NTILE; ++i) {
              int r = (wave + i * NW) * 16 + (lane & 15);
              r = r < R ? r : R - 1;
              const int ry = (int)(((float)r + 0.5f) * __builtin_amdgcn_rcpf((float)bo.W)), rx = r - ry * bo.W;
              const int y = mod_once(bo.ys + ry, L), x = mod_once(bo.xs + rx, L);
              site[i] = y * L + x;
              const int ay = mod_once(y - bn.ys, L), ax = mod_once(x - bn.xs, L);
#pragma unroll
              for (int d = 0; d < 3; ++d) {
                // ay, ax lie in [0, L): only the neighbour above (left) can
                // wrap, to L - 1, and only the one below (right), to 0
                int vy = ay + d - 1, vx = ax + d - 1;
                if (d == 0) {
                  vy = vy < 0 ? L - 1 : vy;
                  vx = vx < 0 ? L - 1 : vx;
                } else if (d == 2) {
                  vy = vy >= L ? 0 : vy;
                  vx = vx >= L ? 0 : vx;
                }
                ro[i][d] = vy < bn.H ? vy * bn.W : -(1 << 20);
                cf[i][d] = vx < bn.W ? vx : -(1 << 20);
              }
            }
            // the stored e^{2 z_l(s)} of the lane's rows, requested before the
            // K loop so that the matrix work covers the memory latency
            f32x4 za[TPW][NT];
#pragma unroll
            for (int i = 0; i < NTILE; ++i)
#pragma unroll
              for (int nt = 0; nt < NT; ++nt)
                za[i][nt] = *reinterpret_cast<const f32x4 *>(zl + site[i] * C + nt * 16 + 4 * (lane >> 4));
            if (copy_next) stage_async_fixed<NW, K::FRAGP>(fnext, fsrc);
            if constexpr (NTILE > 0) {
              f32x4 acc[TPW][NT];
              kloop_box<C, PREC, TPW, NTILE>(din, cap_in, fcur, ro, cf, acc);
#pragma unroll
              for (int i = 0; i < NTILE; ++i) {
                const int r = (wave + i * NW) * 16 + (lane & 15);
                if (r < R) {
#pragma unroll
                  for (int nt = 0; nt < NT; ++nt) {
                    float dh[4];
#pragma unroll
                    for (int jj = 0; jj < 4; ++jj) dh[jj] = tanh_diff(za[i][nt][jj], acc[i][nt][jj]);
                    if (l < n_layers) {
                      dstore4<C, PREC>(dout, cap_out, r, nt * 16 + 4 * (lane >> 4), dh);
                    } else {
#pragma unroll
                      for (int jj = 0; jj < 4; ++jj) part += (double)dh[jj];
                    }
                  }
                }
              }
            }
          };
          with_tiles<TPW>(nti, body);
          if (l == n_layers) {
            part = wave_sum(part);
            if (lane == 0) s_dl[(q & (K::SLOTS - 1)) * NW + wave] = part;
            // with n even the last layer reads the even buffer: the next s'
            // lift fills the odd one now
            if (!(n_layers & 1) && q + 1 < total) lift(q + 1, 0, 0, NTHR);
          }
          wait_copies();
          __syncthreads();
          ++t;
        }
        if ((n_layers & 1) && q + 1 < total) {
          lift(q + 1, 0, 0, NTHR);
          __syncthreads();
        }
      }
    } else {
      for (int q = 0; q < total;) {
        // every wave has written its parts of s' q-16 .. q-1 (before a barrier);
        // the slots written meanwhile (s' q onwards) are the other 16
        if (tid == 0 && q > 0 && (q & 15) == 0) flush(q, 16);
        const bool pr = PAIRS && q + 1 < total;
        const int qn = q + (pr ? 2 : 1);  // the next unit's first s'
        const PB pa = pbox(q), pb = pr ? pbox(q + 1) : pa;
        // steps: the pair's layers 1 .. 3, then layers 4 .. n of q and of q + 1;
        // or layers 1 .. n of q alone
        const int nsteps = pr ? 2 * n_layers - 3 : n_layers;
        for (int st = 0; st < nsteps; ++st) {
          if (pr && st < 3) {
            step(IntC<1>{}, st + 1, pa, pb, st + 1);
          } else {
            const int second = pr && st >= n_layers;  // s' q + 1 of a pair
            const int l = second ? st - n_layers + 4 : st + 1;
            const int fidx = l < n_layers ? l : ((pr && !second) ? 3 : (qn < total ? 0 : -1));
            // the first of a pair's last layer: its partner's spilled box comes
            // back into the odd buffer (issued before this step's loads, so
            // that their waits are not lengthened by it; the K loop covers it)
            if (pr && !second && l == n_layers) stage_async_fixed<NW, K::SPILL_BYTES>(s_dodd, spl);
            double part = step(IntC<0>{}, l, second ? pb : pa, pb, fidx);
            if (l == n_layers) {
              part = wave_sum(part);
              if (lane == 0) s_dl[((q + second) & (K::SLOTS - 1)) * NW + wave] = part;
              // with n even the last layer reads the even buffer: the next
              // lift fills the odd one now (for the first of a pair: the copy
              // above does)
              if (!(n_layers & 1) && !(pr && !second) && qn < total) lift_next(qn);
            }
          }
          wait_copies();
          __syncthreads();
          ++t;
          if (pr && st == n_layers - 1) {
            // the partner's box of distance 4: odd buffer -> even rows 0 .. R4 - 1
            Box b4;
            b4.set(pb.y0, pb.x0, pb.ey, pb.ex, 4, L);
            const int R4 = b4.H * b4.W;
            if constexpr (PREC == P_F32) {
              const uint32_t *src = reinterpret_cast<const uint32_t *>(s_dodd);
              uint32_t *dst = reinterpret_cast<uint32_t *>(s_deven);
              for (int w = tid; w < R4 * (C + 1); w += NTHR) dst[w] = src[w];
            } else {
              const int pw = R4 * C / 8;  // 16-byte pieces per plane
              for (int w = tid; w < (PREC == P_X3 ? 2 : 1) * pw; w += NTHR) {
                const int pl = w >= pw ? 1 : 0, o = w - pl * pw;
                const uint4 v = *reinterpret_cast<const uint4 *>(s_dodd + (size_t)pl * R4 * C * 2 + o * 16);
                *reinterpret_cast<uint4 *>(s_deven + (size_t)pl * (cap_even + 1) * C * 2 + o * 16) = v;
              }
            }
            __syncthreads();
            zero_rows(1);
          }
        }
        if ((n_layers & 1) && qn < total) {
          lift_next(qn);
          __syncthreads();
        }
        q = qn;
      }
    }
    if (tid == 0) {
      if (total > 0) flush(total, total - ((total - 1) & ~15));
      e_loc[b] = eacc;
      if (flags) flags[b] = ((!isfinite(eacc) || !finite) ? 1 : 0) | (sz != 0 ? 2 : 0) | (bad ? 4 : 0);
    }
    __syncthreads();
  }
}

inline size_t al256(size_t b) { return (b + 255) / 256 * 256; }

// Whether two s' can share the first three layer steps (see the kernel):
// twelve waves, n even and at least 4, both configurations' boxes of
// distance 1 .. 3 side by side in the buffers, a box of distance 4 in the
// even one, and the spill slot's copy within the odd buffer.
template <int C, int PREC, int NW, int TPW>
bool lc_pairs(int L, int n) {
  using K = LC<C, PREC, NW, TPW>;
  if (NW != 12 || (n & 1) || n < 4) return false;
  int cap_odd, cap_even;
  lc_caps(n, L, cap_odd, cap_even);
  return 2 * box_rows_max(3, L) <= cap_odd && 2 * box_rows_max(2, L) <= cap_even &&
         (box_rows_max(4, L) + 15) / 16 <= 2 * (NW / 2) && box_rows_max(4, L) <= cap_even &&
         box_rows_max(4, L) * K::ROWB <= K::SPILL_BYTES && K::SPILL_BYTES <= (cap_odd + 1) * K::ROWB;
}

template <int C, int PREC, int NW, int TPW>
bool lc_fits(int L, int n) {
  using K = LC<C, PREC, NW, TPW>;
  int cap_odd, cap_even;
  lc_caps(n, L, cap_odd, cap_even);
  return L * L <= K::MR && cap_odd + cap_even + 2 <= K::ROWS;
}

// Launch shapes by lattice size: (waves per workgroup, row tiles per wave),
// with NW * TPW * 16 >= N rows for the dense pass of s.  Twelve waves (three
// per SIMD) above 128 sites, so that one wave's memory and barrier waits are
// covered by the others' work (measured against eight waves at 16x16 and
// 24x24).
int lc_shape(int N) { return N <= 64 ? 0 : N <= 128 ? 1 : N <= 256 ? 2 : 3; }

template <int C, int PREC, int NW, int TPW>
int lc_grid(int B) {
  using K = LC<C, PREC, NW, TPW>;
  const int lds = K::REGION + K::FIXED + 256;
  int per_cu = 160 * 1024 / lds;
  const int thr = 2048 / (NW * 64);
  per_cu = per_cu < 1 ? 1 : (per_cu > thr ? thr : per_cu);
  const int g = 256 * per_cu;
  return B < g ? B : g;
}

template <int C, int PREC>
int lc_grid_c(int N, int B) {
  switch (lc_shape(N)) {
    case 0: return lc_grid<C, PREC, 4, 1>(B);
    case 1: return lc_grid<C, PREC, 4, 2>(B);
    case 2: return lc_grid<C, PREC, 12, 2>(B);
    default: return lc_grid<C, PREC, 12, 3>(B);
  }
}

template <int C, int PREC>
int lc_spill_c(int N) {
  switch (lc_shape(N)) {
    case 0: return LC<C, PREC, 4, 1>::SPILL_BYTES;
    case 1: return LC<C, PREC, 4, 2>::SPILL_BYTES;
    case 2: return LC<C, PREC, 12, 2>::SPILL_BYTES;
    default: return LC<C, PREC, 12, 3>::SPILL_BYTES;
  }
}

// packed FP32 fragments | packed fragments of the difference pass | per
// workgroup: the stored exponentials of s, then a spill slot
template <int C, int PREC>
size_t lc_ws(const vqmc_model *m, int B) {
  const int N = m->L * m->L, n = m->n_layers;
  const int grid = B > 0 ? lc_grid_c<C, PREC>(N, B) : 0;
  return al256(n * frag_bytes_per_layer<C, P_F32>()) + al256(n * frag_bytes_per_layer<C, PREC>()) +
         al256((size_t)grid * (n + 1) * N * C * 4) + (size_t)grid * lc_spill_c<C, PREC>(N);
}

template <int C, int PREC, int NW, int TPW>
vqmc_status lc_launch(const vqmc_model *m, const float *theta, const int8_t *spins, int B, double *e_loc,
                      int32_t *flags, double *lp, char *ws, hipStream_t st) {
  // the workgroup's LDS rows hold one configuration's sites, and the two
  // difference buffers the boxes of distance 1 .. n
  if (!lc_fits<C, PREC, NW, TPW>(m->L, m->n_layers)) return VQMC_ERR_SHAPE;
  const int n = m->n_layers;
  int cap_odd, cap_even;
  lc_caps(n, m->L, cap_odd, cap_even);
  char *f32 = ws;
  char *fp = ws + al256(n * frag_bytes_per_layer<C, P_F32>());
  float *z = reinterpret_cast<float *>(fp + al256(n * frag_bytes_per_layer<C, PREC>()));
  const int grid = lc_grid<C, PREC, NW, TPW>(B);
  char *spill = reinterpret_cast<char *>(z) + al256((size_t)grid * (n + 1) * m->L * m->L * C * 4);
  const int t32 = n * Engine<C, P_F32, 1, 1>::KS * Engine<C, P_F32, 1, 1>::NT * 64;
  const int tp = n * Engine<C, PREC, 1, 1>::KS * Engine<C, PREC, 1, 1>::NT * 64;
  pack_layer_frags_kernel<C, P_F32><<<(t32 + 255) / 256, 256, 0, st>>>(theta, n, f32);
  if (PREC != P_F32) pack_layer_frags_kernel<C, PREC><<<(tp + 255) / 256, 256, 0, st>>>(theta, n, fp);
  else fp = f32;
  // the paired form is a kernel of its own, so that the plain one keeps its
  // registers
  if (NW == 12 && lc_pairs<C, PREC, NW, TPW>(m->L, n))
    eloc_lc_kernel<C, PREC, NW, TPW, true><<<grid, NW * 64, 0, st>>>(
        theta, f32, fp, spins, B, m->L, n, m->J1, m->J2, m->marshall, cap_odd, cap_even, z, spill, e_loc, flags, lp);
  else
    eloc_lc_kernel<C, PREC, NW, TPW, false><<<grid, NW * 64, 0, st>>>(
        theta, f32, fp, spins, B, m->L, n, m->J1, m->J2, m->marshall, cap_odd, cap_even, z, spill, e_loc, flags, lp);
  if (hipGetLastError() != hipSuccess) return VQMC_ERR_DEVICE;
  return VQMC_OK;
}

template <int C, int PREC>
vqmc_status lc_launch_c(const vqmc_model *m, const float *theta, const int8_t *spins, int B, double *e_loc,
                        int32_t *flags, double *lp, char *ws, hipStream_t st) {
  switch (lc_shape(m->L * m->L)) {
    case 0: return lc_launch<C, PREC, 4, 1>(m, theta, spins, B, e_loc, flags, lp, ws, st);
    case 1: return lc_launch<C, PREC, 4, 2>(m, theta, spins, B, e_loc, flags, lp, ws, st);
    case 2: return lc_launch<C, PREC, 12, 2>(m, theta, spins, B, e_loc, flags, lp, ws, st);
    default:
      return lc_launch<C, PREC, 12, 3>(m, theta, spins, B, e_loc, flags, lp, ws, st);
  }
}

}  // namespace

size_t eloc_lc_workspace(const vqmc_model *m, int B) {
  switch (m->channels) {
    case 16:
      return m->conv_prec == P_F32 ? lc_ws<16, P_F32>(m, B)
                                   : m->conv_prec == P_BF16 ? lc_ws<16, P_BF16>(m, B) : lc_ws<16, P_X3>(m, B);
    case 32:
      return m->conv_prec == P_F32 ? lc_ws<32, P_F32>(m, B)
                                   : m->conv_prec == P_BF16 ? lc_ws<32, P_BF16>(m, B) : lc_ws<32, P_X3>(m, B);
    default: return 0;
  }
}

template <int C, int PREC>
bool lc_fits_c(int L, int n) {
  switch (lc_shape(L * L)) {
    case 0: return lc_fits<C, PREC, 4, 1>(L, n);
    case 1: return lc_fits<C, PREC, 4, 2>(L, n);
    case 2: return lc_fits<C, PREC, 12, 2>(L, n);
    default: return lc_fits<C, PREC, 12, 3>(L, n);
  }
}

bool eloc_lc_supported(const vqmc_model *m) {
  const int L = m->L, n = m->n_layers;
  switch (m->channels) {
    case 16:
      return m->conv_prec == P_F32 ? lc_fits_c<16, P_F32>(L, n)
             : m->conv_prec == P_BF16 ? lc_fits_c<16, P_BF16>(L, n) : lc_fits_c<16, P_X3>(L, n);
    case 32:
      return m->conv_prec == P_F32 ? lc_fits_c<32, P_F32>(L, n)
             : m->conv_prec == P_BF16 ? lc_fits_c<32, P_BF16>(L, n) : lc_fits_c<32, P_X3>(L, n);
    default: return false;
  }
}

vqmc_status eloc_lc(const vqmc_model *m, const float *theta, const int8_t *spins, int B, double *e_loc,
                    int32_t *flags, double *lp, void *ws, hipStream_t st) {
  char *w = reinterpret_cast<char *>(ws);
  switch (m->channels) {
    case 16:
      return m->conv_prec == P_F32 ? lc_launch_c<16, P_F32>(m, theta, spins, B, e_loc, flags, lp, w, st)
             : m->conv_prec == P_BF16 ? lc_launch_c<16, P_BF16>(m, theta, spins, B, e_loc, flags, lp, w, st)
                                      : lc_launch_c<16, P_X3>(m, theta, spins, B, e_loc, flags, lp, w, st);
    case 32:
      return m->conv_prec == P_F32 ? lc_launch_c<32, P_F32>(m, theta, spins, B, e_loc, flags, lp, w, st)
             : m->conv_prec == P_BF16 ? lc_launch_c<32, P_BF16>(m, theta, spins, B, e_loc, flags, lp, w, st)
                                      : lc_launch_c<32, P_X3>(m, theta, spins, B, e_loc, flags, lp, w, st);
    default: return VQMC_ERR_ARG;
  }
}

}  // namespace vqmc
