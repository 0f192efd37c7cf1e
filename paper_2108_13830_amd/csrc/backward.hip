// backward.hip -- per-sample log-derivatives O_k = d log|W| / d theta_k
// (the O_s of Eq. Es-Os-G), FP32 on the matrix cores.
//
// One workgroup per sample (grid-stride).  The forward pass is recomputed
// with the fused engine and every hidden activation h_1..h_n is written to a
// per-workgroup scratch slice in global memory (the activations of a whole
// batch are never stored: memory stays O(grid), not O(B)).  The reverse pass
// then walks the layers top-down with two LDS buffers, D (the error signal
// delta_{l+1} = dlog|W|/dz_{l+1}) and H (the layer input h_l):
//   dW_l[co][ci][tap] = sum_site D[site][co] H[site + d(tap)][ci]    (GEMM, K = sites)
//   db_l[co]          = sum_site D[site][co]                        (extra column of ones)
//   g_l[j][ci]        = sum_{tap,co} D[j - d(tap)][co] W_l[co][ci][tap]   (transposed conv)
//   D <- g_l * (1 - H^2)
// and finishes with the 1 -> C lift, whose input is the spin configuration.
//
// Symmetrised amplitude (R = 4 rotations): d log|W~| = sum_r p_r O(T^r S)
// with p_r the softmax of log W_CNN(T^r S).  The passes run rotation by
// rotation and accumulate into the sample's row of O in place: after
// rotation r the row holds sum_{i<=r} exp(lw_i - M_r) O_i (M_r the running
// maximum), so each pass scales the row by exp(M_{r-1} - M_r) and its own
// delta_{n+1} by exp(lw_r - M_r); the last pass also divides both by the
// normaliser.  With R = 1 the row is simply written.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"
#include "engine.hpp"

namespace vqmc {

// Fragments of every C -> C layer in the engine's FP32 B-operand order:
// [layer 1..n][forward | transposed][KS][NT][64].
template <int C>
__global__ void pack_frags_kernel(const float *__restrict__ theta, int n_layers, float *__restrict__ frags) {
  using E = Engine<C, P_F32, 1, 1>;
  constexpr int PER = E::KS * E::NT * 64;
  const int total = n_layers * 2 * PER;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
    const int l = t / (2 * PER) + 1, rem = t - (l - 1) * 2 * PER;
    const bool tr = rem >= PER;
    const int idx = tr ? rem - PER : rem;
    const int s = idx / (E::NT * 64), r2 = idx - s * (E::NT * 64);
    const int nt = r2 >> 6, ln = r2 & 63;
    const int k = 4 * s + (ln >> 4), n = nt * 16 + (ln & 15);
    const float *W = theta + layer_offset(C, l);
    frags[t] = tr ? E::template wsel<true>(W, k, n) : E::template wsel<false>(W, k, n);
  }
}

template <int C, int NW, int TPW>
struct Bwd {
  using E = Engine<C, P_F32, NW, TPW>;
  static constexpr int LDA = E::LDA;
  static constexpr int PER = E::KS * E::NT * 64;
  static constexpr int MT = (C + 15) / 16;              // dW row tiles (c_out)
  static constexpr int NCOL = 9 * C + 1;                // (ci, tap) columns + bias column
  static constexpr int NTN = (NCOL + 15) / 16;          // dW column tiles
  static constexpr int NPW = (NTN + NW - 1) / NW;       // column tiles per wave
  static constexpr int LDS_BYTES = 2 * E::MAXROWS * LDA * 4 + E::MAXROWS;
};

template <int C, int NW, int TPW>
__global__ __launch_bounds__(NW * 64) void logderiv_kernel(const float *__restrict__ theta,
                                                           const float *__restrict__ frags,
                                                           const int8_t *__restrict__ spins, int B,
                                                           int L, int n_layers, int R, float *__restrict__ O,
                                                           int64_t ldO, float *__restrict__ scratch_all) {
  using K = Bwd<C, NW, TPW>;
  using E = typename K::E;
  constexpr int LDA = K::LDA;
  __shared__ __align__(16) float s_D[E::MAXROWS * LDA];
  __shared__ __align__(16) float s_H[E::MAXROWS * LDA];
  __shared__ int8_t s_sp[E::MAXROWS];
  __shared__ double s_red[NW];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int N = L * L;
  float *scratch = scratch_all + (size_t)blockIdx.x * n_layers * N * C;
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    float *Ob = O + (size_t)b * ldO;
    double mx = -INFINITY, zsum = 0.0;  // running maximum and normaliser (uniform)
    for (int rr = 0; rr < R; ++rr) {
      for (int i = tid; i < N; i += E::NTHR) s_sp[i] = spins[(size_t)b * N + rot_src(i, rr, L)];
      __syncthreads();
      // ---- forward, keeping h_1..h_n
      E::lift(theta, s_sp, N, L, N, reinterpret_cast<char *>(s_D));
      __syncthreads();
      for (int idx = tid; idx < N * C; idx += E::NTHR) {
        const int r = idx / C, c = idx - r * C;
        scratch[idx] = s_D[r * LDA + c];
      }
      for (int l = 1; l <= n_layers; ++l) {
        f32x4 acc[TPW][E::NT];
        E::template kloop<true, 1>(reinterpret_cast<const char *>(s_D),
                                   reinterpret_cast<const char *>(frags + (size_t)(l - 1) * 2 * K::PER),
                                   N, L, N, acc);
        __syncthreads();
        E::write_tiles(acc, theta + layer_offset(C, l) + 9 * C * C, N, reinterpret_cast<char *>(s_D),
                       l < n_layers ? scratch + (size_t)l * N * C : nullptr);
        __syncthreads();
      }
      // ---- this rotation's weight: row <- alpha row + beta O(T^r S)
      float alpha = 0.f, beta = 1.f;
      if (R > 1) {
        double part = 0.0;
        for (int idx = tid; idx < N * C; idx += E::NTHR) {
          const int row = idx / C, c = idx - row * C;
          part += (double)s_D[row * LDA + c];
        }
        part = wave_sum(part);
        if (lane == 0) s_red[wave] = part;
        __syncthreads();
        double lw = 0.0;
  #pragma unroll
        for (int w = 0; w < NW; ++w) lw += s_red[w];
        __syncthreads();
        const double m2 = fmax(mx, lw), sc = exp(mx - m2), wr = exp(lw - m2);
        zsum = zsum * sc + wr;
        mx = m2;
        const double norm = rr == R - 1 ? 1.0 / zsum : 1.0;
        alpha = (float)(sc * norm);
        beta = (float)(wr * norm);
      }
      // ---- delta_{n+1} = beta (1 - h_{n+1}^2) (the head sums h_{n+1})
      for (int idx = tid; idx < N * C; idx += E::NTHR) {
        const int row = idx / C, c = idx - row * C;
        const float h = s_D[row * LDA + c];
        s_D[row * LDA + c] = beta * (1.f - h * h);
      }
      // ---- reverse pass over the C -> C layers
      for (int l = n_layers; l >= 1; --l) {
        const float *hl = scratch + (size_t)(l - 1) * N * C;
        for (int idx = tid; idx < N * C; idx += E::NTHR) {
          const int r = idx / C, c = idx - r * C;
          s_H[r * LDA + c] = hl[idx];
        }
        __syncthreads();
        const int64_t off = layer_offset(C, l);
        // dW_l and db_l: M = c_out, columns n' = ci*9 + tap (n' = 9C: bias), K = sites
        {
          f32x4 acc[K::MT][K::NPW];
          int cdy[K::NPW], cdx[K::NPW], cci[K::NPW];
          bool cval[K::NPW], cone[K::NPW];
  #pragma unroll
          for (int q = 0; q < K::NPW; ++q) {
            const int np = (wave + q * NW) * 16 + (lane & 15);
            const int ci = np / 9, tap = np - ci * 9;
            cval[q] = np < 9 * C;
            cone[q] = np == 9 * C;
            cci[q] = cval[q] ? ci : 0;
            cdy[q] = tap / 3 - 1;
            cdx[q] = tap % 3 - 1;
  #pragma unroll
            for (int mt = 0; mt < K::MT; ++mt) acc[mt][q] = f32x4{0.f, 0.f, 0.f, 0.f};
          }
          int site = lane >> 4;
          int y = site / L, x = site - y * L;
          for (int ks = 0; ks < N / 4; ++ks) {
            float a[K::MT];
  #pragma unroll
            for (int mt = 0; mt < K::MT; ++mt) {
              const int co = mt * 16 + (lane & 15);
              a[mt] = co < C ? s_D[site * LDA + co] : 0.f;
            }
  #pragma unroll
            for (int q = 0; q < K::NPW; ++q) {
              if ((wave + q * NW) < K::NTN) {
                const int nb = wrapL(y + cdy[q], L) * L + wrapL(x + cdx[q], L);
                const float bv = cval[q] ? s_H[nb * LDA + cci[q]] : (cone[q] ? 1.f : 0.f);
  #pragma unroll
                for (int mt = 0; mt < K::MT; ++mt) acc[mt][q] = mma_f32(a[mt], bv, acc[mt][q]);
              }
            }
            site += 4;
            x += 4;
            while (x >= L) {
              x -= L;
              ++y;
            }
          }
  #pragma unroll
          for (int q = 0; q < K::NPW; ++q) {
            const int np = (wave + q * NW) * 16 + (lane & 15);
            if ((wave + q * NW) < K::NTN) {
  #pragma unroll
              for (int mt = 0; mt < K::MT; ++mt)
  #pragma unroll
                for (int j = 0; j < 4; ++j) {
                  const int co = mt * 16 + (lane >> 4) * 4 + j;
                  if (co < C) {
                    float *dst = np < 9 * C ? Ob + off + (int64_t)co * 9 * C + np : Ob + off + 9 * C * C + co;
                    if (np <= 9 * C) *dst = rr ? fmaf(alpha, *dst, acc[mt][q][j]) : acc[mt][q][j];
                  }
                }
            }
          }
        }
        // g_l = transposed conv of delta_{l+1}; then delta_l = g_l (1 - h_l^2)
        f32x4 acc[TPW][E::NT];
        E::template kloop<true, -1>(reinterpret_cast<const char *>(s_D),
                                    reinterpret_cast<const char *>(frags + (size_t)(l - 1) * 2 * K::PER + K::PER),
                                    N, L, N, acc);
        __syncthreads();
  #pragma unroll
        for (int nt = 0; nt < E::NT; ++nt) {
          const int ci = nt * 16 + (lane & 15);
  #pragma unroll
          for (int i = 0; i < TPW; ++i) {
  #pragma unroll
            for (int j = 0; j < 4; ++j) {
              const int row = (wave + i * NW) * 16 + (lane >> 4) * 4 + j;
              if (row < N && ci < C) {
                const float h = s_H[row * LDA + ci];
                s_D[row * LDA + ci] = acc[i][nt][j] * (1.f - h * h);
              }
            }
          }
        }
        __syncthreads();
      }
      // ---- the 1 -> C lift: dW_0[co][tap] = sum_site D[site][co] s[site + d(tap)]
      for (int o = tid; o < 10 * C; o += E::NTHR) {
        const int co = o < 9 * C ? o / 9 : o - 9 * C;
        const int tap = o < 9 * C ? o - co * 9 : -1;
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        float sum = 0.f;
        for (int y = 0; y < L; ++y) {
          const int yy = wrapL(y + dy, L) * L;
          for (int x = 0; x < L; ++x) {
            const float d = s_D[(y * L + x) * LDA + co];
            sum += tap < 0 ? d : d * (float)s_sp[yy + wrapL(x + dx, L)];
          }
        }
        Ob[o] = rr ? fmaf(alpha, Ob[o], sum) : sum;
      }
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------- dispatch

constexpr int kBwdMaxGrid = 2048;

// Launch shapes by lattice size (selector 1, 2, 4 or 9): (waves, row tiles
// per wave) = (4, 1), (4, 2), (8, 2), (12, 3), so that NW * TPW * 16 >= N.
// Above 128 sites the two FP32 row buffers leave room for one or two
// workgroups per compute unit, so more waves per workgroup (two or three per
// SIMD) hide the latency of the gathers and of the matrix instructions
// (24x24: 25.9 -> 15.1 ms, 16x16: 12.7 -> 8.5 ms for 4096 samples, the same
// bits).
static int bwd_tpw(int N) { return N <= 64 ? 1 : N <= 128 ? 2 : N <= 256 ? 4 : 9; }

template <int C, int NW, int TPW>
static int bwd_grid(int B) {
  const int lds = Bwd<C, NW, TPW>::LDS_BYTES;
  int per_cu = 160 * 1024 / (lds + 1024);
  per_cu = per_cu < 1 ? 1 : (per_cu > 8 ? 8 : per_cu);
  int g = 256 * per_cu;
  g = g > kBwdMaxGrid ? kBwdMaxGrid : g;
  return B < g ? B : g;
}

template <int C>
static int grid_for(int N, int B) {
  switch (bwd_tpw(N)) {
    case 1: return bwd_grid<C, 4, 1>(B);
    case 2: return bwd_grid<C, 4, 2>(B);
    case 4: return bwd_grid<C, 8, 2>(B);
    default: return bwd_grid<C, 12, 3>(B);
  }
}

static int grid_any(int C, int N, int B) {
  switch (C) {
    case 4: return grid_for<4>(N, B);
    case 8: return grid_for<8>(N, B);
    case 16: return grid_for<16>(N, B);
    default: return grid_for<32>(N, B);
  }
}

static size_t frag_floats(int C, int n) {
  const int KS = (9 * C + 3) / 4, NT = (C + 15) / 16;
  return (size_t)n * 2 * KS * NT * 64;
}

static size_t ws_bytes_needed(const vqmc_model *m, int B) {
  const int N = m->L * m->L, C = m->channels, n = m->n_layers;
  const int grid = B > 0 ? grid_any(C, N, B) : 0;
  const size_t frag = (frag_floats(C, n) * 4 + 255) / 256 * 256;
  return frag + (size_t)grid * n * N * C * 4;
}

template <int C, int NW, int TPW>
static vqmc_status launch_bwd(const vqmc_model *m, const float *theta, const int8_t *spins, int B,
                              float *O, int64_t ldO, char *ws, hipStream_t stream) {
  const int N = m->L * m->L, n = m->n_layers;
  float *frags = reinterpret_cast<float *>(ws);
  float *scratch = reinterpret_cast<float *>(ws + (frag_floats(C, n) * 4 + 255) / 256 * 256);
  const int total = (int)frag_floats(C, n);
  pack_frags_kernel<C><<<(total + 255) / 256, 256, 0, stream>>>(theta, n, frags);
  VQMC_LAUNCH_CHECK();
  logderiv_kernel<C, NW, TPW><<<bwd_grid<C, NW, TPW>(B), NW * 64, 0, stream>>>(
      theta, frags, spins, B, m->L, n, m->symmetry ? 4 : 1, O, ldO, scratch);
  VQMC_LAUNCH_CHECK();
  (void)N;
  return VQMC_OK;
}

template <int C>
static vqmc_status launch_c(const vqmc_model *m, const float *theta, const int8_t *spins, int B,
                            float *O, int64_t ldO, char *ws, hipStream_t stream) {
  switch (bwd_tpw(m->L * m->L)) {
    case 1: return launch_bwd<C, 4, 1>(m, theta, spins, B, O, ldO, ws, stream);
    case 2: return launch_bwd<C, 4, 2>(m, theta, spins, B, O, ldO, ws, stream);
    case 4: return launch_bwd<C, 8, 2>(m, theta, spins, B, O, ldO, ws, stream);
    default: return launch_bwd<C, 12, 3>(m, theta, spins, B, O, ldO, ws, stream);
  }
}

}  // namespace vqmc

using namespace vqmc;

extern "C" vqmc_status vqmc_log_derivs_workspace(const vqmc_model *m, int32_t B, size_t *bytes) {
  if (!model_valid(m) || !bytes) return VQMC_ERR_ARG;
  if (B < 0) return VQMC_ERR_SHAPE;
  *bytes = ws_bytes_needed(m, B);
  return VQMC_OK;
}

extern "C" vqmc_status vqmc_log_derivs(const vqmc_model *m, const float *theta, const int8_t *spins,
                                       int32_t B, float *O, int64_t ldO, void *workspace,
                                       size_t ws_bytes, hipStream_t stream) {
  if (!model_valid(m)) return VQMC_ERR_ARG;
  if (B < 0) return VQMC_ERR_SHAPE;
  const int64_t P = num_params(m->channels, m->n_layers);
  if (ldO < P) return VQMC_ERR_SHAPE;
  if (B == 0) return VQMC_OK;
  if (!theta || !spins || !O) return VQMC_ERR_ARG;
  if (!workspace || ws_bytes < ws_bytes_needed(m, B)) return VQMC_ERR_WORKSPACE;
  char *ws = reinterpret_cast<char *>(workspace);
  switch (m->channels) {
    case 4: return launch_c<4>(m, theta, spins, B, O, ldO, ws, stream);
    case 8: return launch_c<8>(m, theta, spins, B, O, ldO, ws, stream);
    case 16: return launch_c<16>(m, theta, spins, B, O, ldO, ws, stream);
    case 32: return launch_c<32>(m, theta, spins, B, O, ldO, ws, stream);
    default: return VQMC_ERR_ARG;
  }
}
