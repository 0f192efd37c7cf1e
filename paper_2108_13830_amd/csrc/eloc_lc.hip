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
// where E_c - E_a = E_a (e^{2b} - 1) is taken from the series of e^x - 1
// (six terms) when |2b| < 0.25 (truncation below 5e-8 relative) and as the
// plain difference otherwise (the two then differ by a factor e^{0.25} or
// more, so the difference loses at most a factor 4.5 in relative accuracy).
// E_c is capped at 1e30: beyond it tanh(a + b) = 1 in FP32.  Where the
// denominator overflows (E_a > 3e8 with E_c capped) the result is 0, within
// 1e-8 of the exact 2 / (E_a + 1).  One exponential and one reciprocal.
__device__ __forceinline__ float tanh_diff(float ea, float b) {
  const float x = 2.f * b;
  const float ec = fminf(ea * __expf(fminf(x, 88.f)), 1e30f);
  const float em1 =
      x * (1.f + x * (1.f / 2.f + x * (1.f / 6.f + x * (1.f / 24.f + x * (1.f / 120.f + x * (1.f / 720.f))))));
  // both candidates are formed and one is picked bitwise (no branch)
  const int sel = -(int)(fabsf(x) < 0.25f);
  const int u = __float_as_int(ea * em1), t = __float_as_int(ec - ea);
  const float num = __int_as_float(t ^ ((t ^ u) & sel));
  return 2.f * num * __builtin_amdgcn_rcpf((ec + 1.f) * (ea + 1.f));
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

template <int C, int PREC, int NW, int TPW>
struct LC {
  using E32 = Engine<C, P_F32, NW, TPW>;
  using EP = Engine<C, PREC, NW, TPW>;
  static constexpr int NT = E32::NT;
  static constexpr int ACT = E32::ACT_BYTES > EP::ACT_BYTES ? E32::ACT_BYTES : EP::ACT_BYTES;
  static constexpr int MR = E32::MAXROWS;
  static constexpr int FRAG = E32::FRAG_BYTES > EP::FRAG_BYTES ? E32::FRAG_BYTES : EP::FRAG_BYTES;
};

// The engine's K loop over the first n tile slots only (n wave-uniform,
// 0 <= n <= TPW), dispatched to a compile-time trip count.  rows[i] is the
// lattice site of the lane's output row in tile slot i.
template <class EP, int TPW, int K = 1>
__device__ __forceinline__ void kloop_n(int n, const char *act, const char *frag, const uint16_t *nbt,
                                        const int (&rows)[TPW], f32x4 (&acc)[TPW][EP::NT]) {
  if constexpr (K <= TPW) {
    if (n <= K) {
      EP::template kloop_rows<K>(act, frag, nbt, rows, acc);
      return;
    }
    kloop_n<EP, TPW, K + 1>(n, act, frag, nbt, rows, acc);
  }
}


template <int C, int PREC, int NW, int TPW>
__global__ __launch_bounds__(NW * 64) void eloc_lc_kernel(const float *__restrict__ theta,
                                                          const char *__restrict__ frag32,
                                                          const char *__restrict__ fragp,
                                                          const int8_t *__restrict__ spins, int B, int L,
                                                          int n_layers, double J1, double J2, int marshall,
                                                          float *__restrict__ zscratch,
                                                          double *__restrict__ e_loc,
                                                          int32_t *__restrict__ flags,
                                                          double *__restrict__ lp_out) {
  using K = LC<C, PREC, NW, TPW>;
  using E32 = typename K::E32;
  using EP = typename K::EP;
  constexpr int NT = K::NT;
  constexpr int MR = K::MR;
  __shared__ __align__(16) char s_act[K::ACT];
  __shared__ __align__(16) char s_frag[K::FRAG];
  __shared__ uint16_t s_nbt[E32::NBT_ELEMS];
  __shared__ int8_t s_sig[MR];
  __shared__ int16_t s_bonds[4 * MR];
  __shared__ double s_red[NW];
  __shared__ int s_ired[NW];
  __shared__ double s_dl[16 * NW];  // per-wave parts of the last 16 log-ratios
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int N = L * L, NB = 4 * N;
  const int per_frag32 = E32::KS * NT * 64 * E32::FRAG;
  const int per_fragp = EP::KS * NT * 64 * EP::FRAG;
  static_assert((E32::KS * NT * 64 * E32::FRAG) % 1024 == 0 && (EP::KS * NT * 64 * EP::FRAG) % 1024 == 0,
                "fragment blocks are copied in 1 KiB pieces");
  float *zsc = zscratch + (size_t)blockIdx.x * (n_layers + 1) * N * C;
  // neighbour table of the single configuration: nbt[tap][site]
  E32::build_nbt(s_nbt, 1, L, N);
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    const int8_t *s = spins + (size_t)b * N;
    // the first FP32 layer's fragments arrive while the bonds are scanned
    stage_async<NW * 64>(s_frag, frag32, per_frag32);
    int sz = 0, bad = 0;
    for (int i = tid; i < N; i += NW * 64) {
      const int8_t v = s[i];
      s_sig[i] = v;
      sz += v;
      bad += (v != 1 && v != -1);
    }
    sz = bisum<NW>(sz, s_ired);
    bad = bisum<NW>(bad, s_ired);
    // ---- bond scan (diagonal term, ordered antiparallel list)
    const int chunk = (NB + NW * 64 - 1) / (NW * 64);
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
      for (int idx = tid; idx < N * C; idx += NW * 64) {
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
        f32x4 acc[TPW][NT];
        E32::kloop_tab(s_act, s_frag, s_nbt, acc);
        __syncthreads();
        // next: the following FP32 layer, or the first layer of the s' pass
        if (l < n_layers) stage_async<NW * 64>(s_frag, frag32 + (size_t)l * per_frag32, per_frag32);
        else stage_async<NW * 64>(s_frag, fragp, per_fragp);
        const float *bias = theta + layer_offset(C, l) + 9 * C * C;
        float *zl = zsc + (size_t)l * N * C;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
          const int co = nt * 16 + (lane & 15);
          const float bv = co < C ? bias[co] : 0.f;
#pragma unroll
          for (int i = 0; i < TPW; ++i)
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
              const int row = (wave + i * NW) * 16 + (lane >> 4) * 4 + jj;
              if (row < N && co < C) {
                const float z = acc[i][nt][jj] + bv;
                zl[row * C + co] = exp2x(z);
                if (l < n_layers) E32::store_act(s_act, row, co, tanh_f(z));
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
        for (int idx = tid; idx < N * C; idx += NW * 64)
          lp += (double)(1.f - 2.f * __builtin_amdgcn_rcpf(zn[idx] + 1.f));
        lp = bsum<NW>(lp, s_red);
        if (tid == 0) lp_out[b] = lp;
      }
    }

    // ---- every exchanged configuration, one at a time.  On entry to each
    // s' the fragments of its first layer are in (or on their way to) LDS.
    // Each wave leaves its part of the log-ratio in s_dl; thread 0 turns
    // them into terms 16 at a time (in s' order, the waves' parts summed in
    // wave order), so that no s' waits on a block-wide reduction.
    double eacc = diag;  // thread 0's
    bool finite = true;
    auto flush = [&](int q_end, int count) {
      for (int qq = q_end - count; qq < q_end; ++qq) {
        double dlog = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) dlog += s_dl[(qq & 15) * NW + w];
        const int kind = s_bonds[qq] / N;
        const double J = kind < 2 ? J1 : J2;
        const double mu = (marshall && kind < 2) ? -1.0 : 1.0;
        finite = finite && isfinite(dlog);
        eacc += 0.5 * J * mu * exp(dlog);
      }
    };
    for (int q = 0; q < total; ++q) {
      int bi, bj, kind, y0, x0, ey, ex;
      pair_box(s_bonds[q], L, N, bi, bj, kind, y0, x0, ey, ex);
      const float dsi = (float)(s_sig[bj] - s_sig[bi]);  // change of spin at bi (at bj: -dsi)
      // clear the difference buffer
      {
        uint4 *p = reinterpret_cast<uint4 *>(s_act);
        for (int idx = tid; idx < K::ACT / 16; idx += NW * 64) p[idx] = uint4{0, 0, 0, 0};
      }
      __syncthreads();
      // every wave has written its parts of s' q-16 .. q-1 (before the barrier)
      if (tid == 0 && q > 0 && (q & 15) == 0) flush(q, 16);
      // lift: dz_1[x][c] = sum_tap W0[c][tap] ds[x + d(tap)] on the distance-1 box
      {
        Box bx;
        bx.set(y0, x0, ey, ex, 1, L);
        const int R = bx.H * bx.W;
        for (int idx = tid; idx < R * C; idx += NW * 64) {
          const int r = idx / C, co = idx - r * C;
          const int site = bx.site(r, L);
          float dz = 0.f;
#pragma unroll
          for (int tap = 0; tap < 9; ++tap) {
            const int nb = s_nbt[tap * MR + site];
            const float w = theta[co * 9 + tap];
            dz += nb == bi ? w * dsi : (nb == bj ? -w * dsi : 0.f);
          }
          EP::store_act(s_act, site, co, tanh_diff(zsc[site * C + co], dz));
        }
      }
      wait_copies();
      __syncthreads();
      double part = 0.0;
      for (int l = 1; l <= n_layers; ++l) {
        Box bx;
        bx.set(y0, x0, ey, ex, l + 1, L);
        const int R = bx.H * bx.W;
        int rows[TPW];
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
          int r = (wave + i * NW) * 16 + (lane & 15);
          r = r < R ? r : R - 1;
          rows[i] = bx.site(r, L);
        }
        // tiles of this wave in the current box (wave-uniform)
        const int Ttot = (R + 15) / 16;
        const int nti = Ttot > wave ? (Ttot - wave + NW - 1) / NW : 0;
        // the lane's output sites (four rows r0..r0+3 of each of its tiles,
        // walking the box row-major; rows past the box reuse a valid site)
        // and the stored e^{2 z_l(s)} there, requested before the K loop so
        // that the matrix work covers the memory latency
        const float *zl = zsc + (size_t)l * N * C;
        int osite[TPW][4];
        float za[TPW][4][NT];
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
          if (i < nti) {
            const int r0 = (wave + i * NW) * 16 + (lane >> 4) * 4;
            // r0 / W from a float reciprocal with half-row margin (r0 < 2^10)
            int ry = (int)(((float)r0 + 0.5f) * __builtin_amdgcn_rcpf((float)bx.W)), rx = r0 - ry * bx.W;
            int y = bx.ys + ry, x = bx.xs + rx;
            y = y < 0 ? y + L : (y >= L ? y - L : y);
            x = x < 0 ? x + L : (x >= L ? x - L : x);
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
              osite[i][jj] = y * L + x;
              ++rx;
              x = x + 1 == L ? 0 : x + 1;
              if (rx == bx.W) {
                rx = 0;
                x = bx.xs < 0 ? bx.xs + L : bx.xs;
                y = y + 1 == L ? 0 : y + 1;
              }
            }
#pragma unroll
            for (int jj = 0; jj < 4; ++jj)
#pragma unroll
              for (int nt = 0; nt < NT; ++nt) {
                const int co = nt * 16 + (lane & 15);
                za[i][jj][nt] = zl[osite[i][jj] * C + (co < C ? co : 0)];
              }
          }
        }
        f32x4 acc[TPW][NT];
        kloop_n<EP, TPW>(nti, s_act, s_frag, s_nbt, rows, acc);
        __syncthreads();
        // next layer's fragments (after the last layer: the first layer's,
        // for the next s') arrive while this layer's differences are formed
        stage_async<NW * 64>(s_frag, fragp + (size_t)(l < n_layers ? l : 0) * per_fragp, per_fragp);
#pragma unroll
        for (int i = 0; i < TPW; ++i) {
          if (i < nti) {
            const int r0 = (wave + i * NW) * 16 + (lane >> 4) * 4;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
              if (r0 + jj < R) {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) {
                  const int co = nt * 16 + (lane & 15);
                  if (co < C) {
                    const float dh = tanh_diff(za[i][jj][nt], acc[i][nt][jj]);
                    if (l < n_layers) EP::store_act(s_act, osite[i][jj], co, dh);
                    else part += (double)dh;
                  }
                }
              }
            }
          }
        }
        if (l < n_layers) wait_copies();
        __syncthreads();
      }
      part = wave_sum(part);
      if (lane == 0) s_dl[(q & 15) * NW + wave] = part;
    }
    // the copy started by the last layer of the last s' must land before the
    // next sample overwrites the buffer
    wait_copies();
    __syncthreads();
    if (tid == 0) {
      if (total > 0) flush(total, total - ((total - 1) & ~15));
      e_loc[b] = eacc;
      if (flags) flags[b] = ((!isfinite(eacc) || !finite) ? 1 : 0) | (sz != 0 ? 2 : 0) | (bad ? 4 : 0);
    }
    __syncthreads();
  }
}

inline size_t al256(size_t b) { return (b + 255) / 256 * 256; }

// Launch shapes by lattice size: (waves per workgroup, row tiles per wave),
// with NW * TPW * 16 >= N rows for the dense pass of s.  Eight waves (two
// per SIMD) from 16x16 up, so that one wave's memory and barrier waits are
// covered by the other's matrix work.
int lc_shape(int N) { return N <= 64 ? 0 : N <= 128 ? 1 : N <= 256 ? 2 : 3; }

template <int C, int PREC, int NW, int TPW>
int lc_grid(int B) {
  using K = LC<C, PREC, NW, TPW>;
  const int lds = K::ACT + K::FRAG + 23 * K::MR + 256;
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
    case 2: return lc_grid<C, PREC, 8, 2>(B);
    default: return PREC == P_F32 ? lc_grid<C, PREC, 8, 5>(B) : lc_grid<C, PREC, 12, 3>(B);
  }
}

template <int C, int PREC>
size_t lc_ws(const vqmc_model *m, int B) {
  const int N = m->L * m->L, n = m->n_layers;
  const int grid = B > 0 ? lc_grid_c<C, PREC>(N, B) : 0;
  return al256(n * frag_bytes_per_layer<C, P_F32>()) + al256(n * frag_bytes_per_layer<C, PREC>()) +
         (size_t)grid * (n + 1) * N * C * 4;
}

template <int C, int PREC, int NW, int TPW>
vqmc_status lc_launch(const vqmc_model *m, const float *theta, const int8_t *spins, int B, double *e_loc,
                      int32_t *flags, double *lp, char *ws, hipStream_t st) {
  // the workgroup's LDS rows hold one configuration's sites
  if (m->L * m->L > LC<C, PREC, NW, TPW>::MR) return VQMC_ERR_SHAPE;
  const int n = m->n_layers;
  char *f32 = ws;
  char *fp = ws + al256(n * frag_bytes_per_layer<C, P_F32>());
  float *z = reinterpret_cast<float *>(fp + al256(n * frag_bytes_per_layer<C, PREC>()));
  const int t32 = n * Engine<C, P_F32, 1, 1>::KS * Engine<C, P_F32, 1, 1>::NT * 64;
  const int tp = n * Engine<C, PREC, 1, 1>::KS * Engine<C, PREC, 1, 1>::NT * 64;
  pack_layer_frags_kernel<C, P_F32><<<(t32 + 255) / 256, 256, 0, st>>>(theta, n, f32);
  if (PREC != P_F32) pack_layer_frags_kernel<C, PREC><<<(tp + 255) / 256, 256, 0, st>>>(theta, n, fp);
  else fp = f32;
  eloc_lc_kernel<C, PREC, NW, TPW><<<lc_grid<C, PREC, NW, TPW>(B), NW * 64, 0, st>>>(
      theta, f32, fp, spins, B, m->L, n, m->J1, m->J2, m->marshall, z, e_loc, flags, lp);
  if (hipGetLastError() != hipSuccess) return VQMC_ERR_DEVICE;
  return VQMC_OK;
}

template <int C, int PREC>
vqmc_status lc_launch_c(const vqmc_model *m, const float *theta, const int8_t *spins, int B, double *e_loc,
                        int32_t *flags, double *lp, char *ws, hipStream_t st) {
  switch (lc_shape(m->L * m->L)) {
    case 0: return lc_launch<C, PREC, 4, 1>(m, theta, spins, B, e_loc, flags, lp, ws, st);
    case 1: return lc_launch<C, PREC, 4, 2>(m, theta, spins, B, e_loc, flags, lp, ws, st);
    case 2: return lc_launch<C, PREC, 8, 2>(m, theta, spins, B, e_loc, flags, lp, ws, st);
    // BF16 forms: 12 waves of 3 tiles (more waves to hide the cone's latencies);
    // FP32: 8 waves of 5 tiles
    default:
      return PREC == P_F32 ? lc_launch<C, PREC, 8, 5>(m, theta, spins, B, e_loc, flags, lp, ws, st)
                           : lc_launch<C, PREC, 12, 3>(m, theta, spins, B, e_loc, flags, lp, ws, st);
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

bool eloc_lc_supported(const vqmc_model *m) { return m->channels == 16 || m->channels == 32; }

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
