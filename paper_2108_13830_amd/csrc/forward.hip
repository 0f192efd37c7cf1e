// forward.hip -- log|psi|, the local-energy generator and the Metropolis
// exchange sampler, all built on the fused conv engine (engine.hpp).
#include <hip/hip_runtime.h>

#include <mutex>
#include <math.h>
#include <stdint.h>

#include "common.hpp"
#include "eloc_lc.hpp"
#include "engine.hpp"

namespace vqmc {

// ---------------------------------------------------------------- helpers

template <int NW>
__device__ __forceinline__ double block_sum(double v, double *tmp) {
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
__device__ __forceinline__ int block_isum(int v, int *tmp) {
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

// Exclusive prefix sum over the block (thread order); *total gets the sum.
template <int NW>
__device__ __forceinline__ int block_excl_scan(int v, int *tmp, int *total) {
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

// Bond k of the 4N bonds (Sec. 3.1): kind k / N = 0 right (J1), 1 below
// (J1), 2 lower-right (J2), 3 lower-left (J2) neighbour of site k % N.
__device__ __forceinline__ void decode_bond(int k, int L, int N, int &i, int &j, int &kind) {
  kind = k / N;
  const int site = k - kind * N, y = site / L, x = site - y * L;
  i = site;
  const int yd = wrapL(y + (kind > 0 ? 1 : 0), L);
  const int xd = wrapL(x + (kind == 0 || kind == 2 ? 1 : (kind == 3 ? -1 : 0)), L);
  j = yd * L + xd;
}

// Philox4x32-10 block function (Salmon et al., SC'11): ten rounds, each two
// 32x32 -> 64-bit products, the round key bumped by the Weyl constants.
__device__ __forceinline__ void philox(uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t &c3,
                                       uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
}

// ------------------------------------------------------------- log |psi|

// logsumexp of v[0..R) in FP64 (the largest term factored out).
__device__ __forceinline__ double lse(const double *v, int R) {
  double mx = v[0];
  for (int r = 1; r < R; ++r) mx = fmax(mx, v[r]);
  double t = 0.0;
  for (int r = 0; r < R; ++r) t += exp(v[r] - mx);
  return mx + log(t);
}

// SYM = false: one configuration per slot, G per workgroup.  SYM (R = 4
// rotations, the symmetrised amplitude): every configuration fills R
// consecutive slots with its rotations T^r S, read straight from global
// memory through rot_src.  When R slots fit a batch (G >= R) a workgroup
// takes G/R whole configurations per forward pass; otherwise it takes one
// configuration and thread 0 folds the log|W| of its rotations, G per pass,
// into a running logsumexp kept in LDS.
template <int C, int PREC, int NW, int TPW, bool SYM>
__global__ __launch_bounds__(NW * 64, C <= 16 ? 2 : 1) void logpsi_kernel(const float *__restrict__ theta,
                                                         const int8_t *__restrict__ spins, int B,
                                                         int L, int n_layers, int marshall, int G,
                                                         double *__restrict__ out,
                                                         int8_t *__restrict__ sign) {
  using E = Engine<C, PREC, NW, TPW>;
  constexpr int R = SYM ? 4 : 1;
  __shared__ __align__(16) char s_act[E::ACT_BYTES];
  __shared__ __align__(16) char s_frag[E::FRAG_BYTES];
  __shared__ int8_t s_sp[E::MAXROWS];
  __shared__ uint16_t s_nbt[E::NBT_ELEMS];
  __shared__ double s_lp[64];
  __shared__ int s_ired[NW];
  __shared__ double s_run[2];  // running maximum and sum of the logsumexp
  const int N = L * L;
  const bool whole = G >= R;  // every configuration's slots in one pass
  const int SP = whole ? G / R : 1;
  E::build_nbt(s_nbt, whole ? SP * R : G, L, N);
  for (int base = blockIdx.x * SP; base < B; base += gridDim.x * SP) {
    const int Sb = min(SP, B - base);
    if constexpr (!SYM) {
      for (int idx = threadIdx.x; idx < Sb * N; idx += E::NTHR) s_sp[idx] = spins[(size_t)base * N + idx];
      __syncthreads();
      E::forward(theta, n_layers, s_sp, Sb, N, s_act, s_frag, s_nbt, s_lp);
      for (int q = threadIdx.x; q < Sb; q += E::NTHR) out[base + q] = s_lp[q];
    } else {
      const int V = Sb * R;
      for (int v0 = 0; v0 < V; v0 += G) {
        const int Gb = min(G, V - v0);
        for (int idx = threadIdx.x; idx < Gb * N; idx += E::NTHR) {
          const int g = idx / N, i = idx - g * N, v = v0 + g, q = v / R;
          s_sp[idx] = spins[(size_t)(base + q) * N + rot_src(i, v - q * R, L)];
        }
        __syncthreads();
        E::forward(theta, n_layers, s_sp, Gb, N, s_act, s_frag, s_nbt, s_lp);
        if (whole) {
          for (int q = threadIdx.x; q < Sb; q += E::NTHR) out[base + q] = lse(s_lp + q * R, R);
        } else if (threadIdx.x == 0) {
          double mx = v0 == 0 ? -INFINITY : s_run[0], t = v0 == 0 ? 0.0 : s_run[1];
          for (int g = 0; g < Gb; ++g) {
            const double v = s_lp[g], m2 = fmax(mx, v);
            t = t * exp(mx - m2) + exp(v - m2);
            mx = m2;
          }
          s_run[0] = mx;
          s_run[1] = t;
        }
        __syncthreads();
      }
      if (!whole && threadIdx.x == 0) out[base] = s_run[0] + log(s_run[1]);
    }
    if (sign) {
      // the Marshall sign of S (its rotations share it when Sz = 0)
      for (int q = 0; q < Sb; ++q) {
        const int8_t *sq = spins + (size_t)(base + q) * N;
        int up = 0;
        for (int i = threadIdx.x; i < N; i += E::NTHR) {
          const int y = i / L, x = i - y * L;
          up += (((x + y) & 1) == 0 && sq[i] > 0);
        }
        up = block_isum<NW>(up, s_ired);
        if (threadIdx.x == 0) sign[base + q] = (marshall && (up & 1)) ? -1 : 1;
      }
    }
    __syncthreads();
  }
}

// ----------------------------------------------------------- local energy

// One workgroup per sample.  The 4N bonds are scanned in parallel for the
// diagonal term and the ordered list of antiparallel bonds; then the sample
// itself and all its exchanged configurations s' are evaluated by the fused
// engine in batches of G, and the off-diagonal terms J/2 mu exp(dlog) are
// accumulated in FP64 in bond order.
template <int C, int PREC, int NW, int TPW>
__global__ __launch_bounds__(NW * 64, C <= 16 ? (TPW <= 7 ? 3 : 2) : 1) void eloc_kernel(const float *__restrict__ theta,
                                                       const int8_t *__restrict__ spins, int B, int L,
                                                       int n_layers, double J1, double J2,
                                                       int marshall, int G,
                                                       double *__restrict__ e_loc,
                                                       int32_t *__restrict__ flags,
                                                       double *__restrict__ lp_out,
                                                       const char *__restrict__ packed) {
  using E = Engine<C, PREC, NW, TPW>;
  constexpr int MR = E::MAXROWS;
  __shared__ __align__(16) char s_act[E::ACT_BYTES];
  __shared__ __align__(16) char s_frag[E::FRAG_BYTES];
  __shared__ int8_t s_sp[MR];
  __shared__ int8_t s_sig[MR];
  __shared__ int16_t s_bonds[4 * MR];
  __shared__ double s_lp[64];
  __shared__ double s_terms[64];
  __shared__ double s_red[NW];
  __shared__ int s_ired[NW];
  __shared__ uint16_t s_nbt[E::NBT_ELEMS];
  const int tid = threadIdx.x;
  const int N = L * L, NB = 4 * N;
  E::build_nbt(s_nbt, G, L, N);
  for (int b = blockIdx.x; b < B; b += gridDim.x) {
    const int8_t *s = spins + (size_t)b * N;
    int sz = 0, bad = 0;
    for (int i = tid; i < N; i += E::NTHR) {
      const int8_t v = s[i];
      s_sig[i] = v;
      sz += v;
      bad += (v != 1 && v != -1);
    }
    sz = block_isum<NW>(sz, s_ired);
    bad = block_isum<NW>(bad, s_ired);
    // bond scan: contiguous chunks per thread keep the list in bond order
    const int chunk = (NB + E::NTHR - 1) / E::NTHR;
    const int k0 = tid * chunk, k1 = min(k0 + chunk, NB);
    double dsum = 0.0;
    int cnt = 0;
    for (int k = k0; k < k1; ++k) {
      int i, j, kind;
      decode_bond(k, L, N, i, j, kind);
      const int si = s_sig[i], sj = s_sig[j];
      dsum += 0.25 * (kind < 2 ? J1 : J2) * (double)(si * sj);
      cnt += (si != sj);
    }
    int total;
    int off = block_excl_scan<NW>(cnt, s_ired, &total);
    for (int k = k0; k < k1; ++k) {
      int i, j, kind;
      decode_bond(k, L, N, i, j, kind);
      if (s_sig[i] != s_sig[j]) s_bonds[off++] = (int16_t)k;
    }
    const double diag = block_sum<NW>(dsum, s_red);
    const int nconf = 1 + total;
    double lp0 = 0.0, eacc = diag;
    for (int q0 = 0; q0 < nconf; q0 += G) {
      const int Gb = min(G, nconf - q0);
      for (int idx = tid; idx < Gb * N; idx += E::NTHR) {
        const int g = idx / N, i = idx - g * N, q = q0 + g;
        int8_t v = s_sig[i];
        if (q > 0) {
          int bi, bj, kind;
          decode_bond(s_bonds[q - 1], L, N, bi, bj, kind);
          if (i == bi) v = s_sig[bj];
          if (i == bj) v = s_sig[bi];
        }
        s_sp[idx] = v;
      }
      __syncthreads();
      E::forward(theta, n_layers, s_sp, Gb, N, s_act, s_frag, s_nbt, s_lp, packed);
      if (q0 == 0) lp0 = s_lp[0];
      for (int g = tid; g < Gb; g += E::NTHR) {
        const int q = q0 + g;
        double t = 0.0;
        if (q > 0) {
          const int kind = s_bonds[q - 1] / N;
          const double J = kind < 2 ? J1 : J2;
          const double mu = (marshall && kind < 2) ? -1.0 : 1.0;
          t = 0.5 * J * mu * exp(s_lp[g] - lp0);
        }
        s_terms[g] = t;
      }
      __syncthreads();
      if (tid == 0)
        for (int g = 0; g < Gb; ++g) eacc += s_terms[g];
      __syncthreads();
    }
    if (tid == 0) {
      e_loc[b] = eacc;
      if (flags) flags[b] = ((!isfinite(eacc) || !isfinite(lp0)) ? 1 : 0) | (sz != 0 ? 2 : 0) | (bad ? 4 : 0);
      if (lp_out) lp_out[b] = lp0;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- sampler

// One chain per workgroup (a single wavefront for small lattices).  Every
// thread computes the same Philox words and reads the same LDS state, so all
// control flow below is uniform across the workgroup.  With R = 4 the chain's
// configuration is kept apart (s_cfg) and every evaluation fills the batch
// with its four rotations, at most G of them per forward pass.
template <int C, int PREC, int NW, int TPW>
__global__ __launch_bounds__(NW * 64) void sample_kernel(const float *__restrict__ theta,
                                                         int8_t *__restrict__ spins, int L,
                                                         int n_layers, int n_sweeps, uint64_t seed,
                                                         uint64_t counter_base, int proposal, int R,
                                                         int G, double *__restrict__ log_psi,
                                                         int32_t *__restrict__ n_acc) {
  using E = Engine<C, PREC, NW, TPW>;
  __shared__ __align__(16) char s_act[E::ACT_BYTES];
  __shared__ __align__(16) char s_frag[E::FRAG_BYTES];
  __shared__ int8_t s_sp[E::MAXROWS];
  __shared__ int8_t s_rot[E::MAXROWS];
  __shared__ double s_lp[64];
  __shared__ int s_ired[NW];
  __shared__ int s_pick[2];
  __shared__ uint16_t s_nbt[E::NBT_ELEMS];
  const int tid = threadIdx.x;
  const int N = L * L;
  const int b = blockIdx.x;
  int8_t *s = spins + (size_t)b * N;
  int8_t *s_cfg = R == 1 ? s_sp : s_rot;  // the chain's configuration
  E::build_nbt(s_nbt, R == 1 ? 1 : G, L, N);
  // log|W| (or log|W~|) of the configuration in s_cfg; uniform result
  // (one call site of the engine keeps the kernel's register budget)
  auto evaluate = [&]() -> double {
    double mx = -INFINITY, t = 0.0;
    for (int r0 = 0; r0 < R; r0 += G) {
      const int Gb = min(G, R - r0);
      if (R > 1) {
        for (int idx = tid; idx < Gb * N; idx += E::NTHR) {
          const int g = idx / N, i = idx - g * N;
          s_sp[idx] = s_cfg[rot_src(i, r0 + g, L)];
        }
        __syncthreads();
      }
      E::forward(theta, n_layers, s_sp, Gb, N, s_act, s_frag, s_nbt, s_lp);
      if (R == 1) return s_lp[0];
      for (int g = 0; g < Gb; ++g) {
        const double v = s_lp[g], m2 = fmax(mx, v);
        t = t * exp(mx - m2) + exp(v - m2);
        mx = m2;
      }
      __syncthreads();
    }
    return mx + log(t);
  };
  for (int i = tid; i < N; i += E::NTHR) s_cfg[i] = s[i];
  __syncthreads();
  double lp = evaluate();
  int acc = 0;
  const uint32_t key0 = (uint32_t)seed, key1 = (uint32_t)(seed >> 32);
  const int chunk = (2 * N + E::NTHR - 1) / E::NTHR;
  const int k0 = tid * chunk, k1 = min(k0 + chunk, 2 * N);
  const int64_t steps = (int64_t)n_sweeps * N;
  for (int64_t t = 0; t < steps; ++t) {
    const uint64_t tt = counter_base + (uint64_t)t;
    uint32_t c0 = (uint32_t)tt, c1 = (uint32_t)(tt >> 32), c2 = (uint32_t)b, c3 = 0u;
    philox(c0, c1, c2, c3, key0, key1);
    int i = 0, j = 0, nap = 0;
    if (proposal == 0) {
      int kind;
      const int k = (int)(((uint64_t)c0 * (uint64_t)(2 * N)) >> 32);
      decode_bond(k, L, N, i, j, kind);
      if (s_cfg[i] == s_cfg[j]) continue;  // parallel pair: rejected move
    } else {
      int cnt = 0;
      for (int k = k0; k < k1; ++k) {
        int a, c, kind;
        decode_bond(k, L, N, a, c, kind);
        cnt += (s_cfg[a] != s_cfg[c]);
      }
      int off = block_excl_scan<NW>(cnt, s_ired, &nap);
      if (nap == 0) continue;
      const int pick = (int)(((uint64_t)c0 * (uint64_t)nap) >> 32);
      if (pick >= off && pick < off + cnt) {
        int seen = off;
        for (int k = k0; k < k1; ++k) {
          int a, c, kind;
          decode_bond(k, L, N, a, c, kind);
          if (s_cfg[a] != s_cfg[c]) {
            if (seen == pick) {
              s_pick[0] = a;
              s_pick[1] = c;
            }
            ++seen;
          }
        }
      }
      __syncthreads();
      i = s_pick[0];
      j = s_pick[1];
    }
    __syncthreads();
    if (tid == 0) {
      const int8_t v = s_cfg[i];
      s_cfg[i] = s_cfg[j];
      s_cfg[j] = v;
    }
    __syncthreads();
    const double lpn = evaluate();
    double hast = 0.0;
    if (proposal == 1) {
      int cnt = 0;
      for (int k = k0; k < k1; ++k) {
        int a, c, kind;
        decode_bond(k, L, N, a, c, kind);
        cnt += (s_cfg[a] != s_cfg[c]);
      }
      const int napn = block_isum<NW>(cnt, s_ired);
      hast = log((double)nap) - log((double)napn);
    }
    const double r = ((double)c1 + 0.5) * (1.0 / 4294967296.0);
    if (2.0 * (lpn - lp) + hast - log(r) >= 0.0) {
      lp = lpn;
      ++acc;
    } else {
      if (tid == 0) {
        const int8_t v = s_cfg[i];
        s_cfg[i] = s_cfg[j];
        s_cfg[j] = v;
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < N; i += E::NTHR) s[i] = s_cfg[i];
  if (tid == 0) {
    if (log_psi) log_psi[b] = lp;
    if (n_acc) n_acc[b] = acc;
  }
}

// ------------------------------------------------- rotation-symmetrised E_s

// rot[4b + r] = T^r spins[b] (Eq. sym-ws), one thread per output byte.
__global__ void rotate_kernel(const int8_t *__restrict__ spins, int B, int L, int8_t *__restrict__ rot) {
  const int N = L * L;
  const int64_t total = (int64_t)4 * B * N;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = t / N;
    const int i = (int)(t - v * N);
    rot[t] = spins[(v >> 2) * N + rot_src(i, (int)(v & 3), L)];
  }
}

// E_s = sum_r p_r E_CNN(T^r s), p_r = softmax_r log W_CNN(T^r s); the flags
// of the four rotations are merged (bit 1 also for a non-finite result).
__global__ void sym_combine_kernel(const double *__restrict__ e4, const double *__restrict__ lp4,
                                   const int32_t *__restrict__ f4, int B, double *__restrict__ e_loc,
                                   int32_t *__restrict__ flags) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const double *l = lp4 + 4 * (size_t)b, *e = e4 + 4 * (size_t)b;
  const double mx = fmax(fmax(l[0], l[1]), fmax(l[2], l[3]));
  double z = 0.0, acc = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const double w = exp(l[r] - mx);
    z += w;
    acc += w * e[r];
  }
  const double E = acc / z;
  e_loc[b] = E;
  if (flags) {
    const int32_t *f = f4 + 4 * (size_t)b;
    flags[b] = f[0] | f[1] | f[2] | f[3] | (isfinite(E) ? 0 : 1);
  }
}

// ------------------------------------------------------------- dispatch

template <int C>
struct Inst {
  static constexpr int NW = 4;
  static constexpr int TPW = (C == 32) ? 9 : 8;  // rows per block: 576 / 512
  static constexpr int SNW = 1;                   // sampler, small lattices
  static constexpr int STPW = 9;                  // 144 rows
  // dense local energy in the BF16 forms at C = 16: 448 rows, so that three
  // workgroups share a compute unit (their per-output work then overlaps
  // each other's matrix work); used while a configuration fits (FP32
  // measured faster with 512 rows and two workgroups)
  static constexpr int ETPW = 7;
};

enum Kind { K_LOGPSI, K_ELOC, K_SAMPLE };

struct FwdArgs {
  const float *theta;
  const int8_t *spins_in;
  int8_t *spins_io;
  int B, L, n_layers, marshall;
  double J1, J2;
  double *out_d;
  int8_t *out_sign;
  int32_t *out_i;
  int n_sweeps, proposal;
  uint64_t seed, counter_base;
  int R;           // 1, or 4 for the rotation-symmetrised amplitude
  double *lp_out;  // local energy: log|W_CNN(s)| per sample (nullable)
  char *ws;        // local energy: room for the packed weight fragments (nullable)
  size_t ws_bytes;
  hipStream_t stream;
};

template <int C, int PREC>
static vqmc_status launch(Kind kind, const FwdArgs &a) {
  using I = Inst<C>;
  using E = Engine<C, PREC, I::NW, I::TPW>;
  using ES = Engine<C, PREC, I::SNW, I::STPW>;
  const int N = a.L * a.L;
  if (N > E::MAXROWS) return VQMC_ERR_SHAPE;
  if (a.B == 0) return VQMC_OK;
  if (kind == K_SAMPLE) {
    if (a.n_sweeps < 0) return VQMC_OK;
    // the small engine (one wavefront) when all R evaluations fit one batch
    if (a.R * N <= ES::MAXROWS) {
      sample_kernel<C, PREC, I::SNW, I::STPW><<<a.B, I::SNW * 64, 0, a.stream>>>(
          a.theta, a.spins_io, a.L, a.n_layers, a.n_sweeps, a.seed, a.counter_base, a.proposal, a.R,
          a.R, a.out_d, a.out_i);
    } else {
      const int G = min(a.R, E::MAXROWS / N);
      sample_kernel<C, PREC, I::NW, I::TPW><<<a.B, I::NW * 64, 0, a.stream>>>(
          a.theta, a.spins_io, a.L, a.n_layers, a.n_sweeps, a.seed, a.counter_base, a.proposal, a.R,
          G, a.out_d, a.out_i);
    }
    VQMC_LAUNCH_CHECK();
    return VQMC_OK;
  }
  int G = E::MAXROWS / N;
  G = G > 64 ? 64 : G;
  if (kind == K_LOGPSI) {
    // whole configurations per workgroup: G rounded down to a multiple of R
    if (G >= a.R) G -= G % a.R;
    const int SP = a.R == 1 ? G : (G >= a.R ? G / a.R : 1);
    const int grid = (a.B + SP - 1) / SP;
    if (a.R == 1)
      logpsi_kernel<C, PREC, I::NW, I::TPW, false><<<grid, I::NW * 64, 0, a.stream>>>(
          a.theta, a.spins_in, a.B, a.L, a.n_layers, a.marshall, G, a.out_d, a.out_sign);
    else
      logpsi_kernel<C, PREC, I::NW, I::TPW, true><<<grid, I::NW * 64, 0, a.stream>>>(
          a.theta, a.spins_in, a.B, a.L, a.n_layers, a.marshall, G, a.out_d, a.out_sign);
  } else {
    // the C -> C layers' fragments packed once for the whole call, when the
    // caller provided the room
    const char *packed = nullptr;
    if (E::DMA_OK && a.ws && a.ws_bytes >= (size_t)a.n_layers * E::FRAG_LAYER) {
      const int total = a.n_layers * E::KS * E::NT * 64;
      pack_layer_frags_kernel<C, PREC><<<(total + 255) / 256, 256, 0, a.stream>>>(a.theta, a.n_layers, a.ws);
      packed = a.ws;
    }
    bool done = false;
    if constexpr (C == 16 && PREC != P_F32) {
      using E7 = Engine<C, PREC, I::NW, I::ETPW>;
      if (N <= E7::MAXROWS) {
        const int G7 = E7::MAXROWS / N < 64 ? E7::MAXROWS / N : 64;
        eloc_kernel<C, PREC, I::NW, I::ETPW><<<a.B, I::NW * 64, 0, a.stream>>>(
            a.theta, a.spins_in, a.B, a.L, a.n_layers, a.J1, a.J2, a.marshall, G7, a.out_d, a.out_i, a.lp_out,
            packed);
        done = true;
      }
    }
    if (!done)
      eloc_kernel<C, PREC, I::NW, I::TPW><<<a.B, I::NW * 64, 0, a.stream>>>(
          a.theta, a.spins_in, a.B, a.L, a.n_layers, a.J1, a.J2, a.marshall, G, a.out_d, a.out_i, a.lp_out,
          packed);
  }
  VQMC_LAUNCH_CHECK();
  return VQMC_OK;
}

static vqmc_status dispatch(Kind kind, int C, int prec, const FwdArgs &a) {
  switch (C) {
    case 4: return launch<4, P_F32>(kind, a);
    case 8:
      return prec == P_F32 ? launch<8, P_F32>(kind, a)
                           : prec == P_BF16 ? launch<8, P_BF16>(kind, a) : launch<8, P_X3>(kind, a);
    case 16:
      return prec == P_F32 ? launch<16, P_F32>(kind, a)
                           : prec == P_BF16 ? launch<16, P_BF16>(kind, a) : launch<16, P_X3>(kind, a);
    case 32:
      return prec == P_F32 ? launch<32, P_F32>(kind, a)
                           : prec == P_BF16 ? launch<32, P_BF16>(kind, a) : launch<32, P_X3>(kind, a);
    default: return VQMC_ERR_ARG;
  }
}

}  // namespace vqmc

using namespace vqmc;

extern "C" vqmc_status vqmc_log_psi(const vqmc_model *m, const float *theta, const int8_t *spins,
                                    int32_t B, double *log_abs_psi, int8_t *sign,
                                    hipStream_t stream) {
  if (!model_valid(m)) return VQMC_ERR_ARG;
  if (B < 0) return VQMC_ERR_SHAPE;
  if (B > 0 && (!theta || !spins || !log_abs_psi)) return VQMC_ERR_ARG;
  FwdArgs a{};
  a.theta = theta;
  a.spins_in = spins;
  a.B = B;
  a.L = m->L;
  a.n_layers = m->n_layers;
  a.marshall = m->marshall;
  a.out_d = log_abs_psi;
  a.out_sign = sign;
  a.R = m->symmetry ? 4 : 1;
  a.stream = stream;
  return dispatch(K_LOGPSI, m->channels, m->conv_prec, a);
}

// Light cones pay off once they stay well inside the lattice for most layers.
static bool use_lightcone(const vqmc_model *m) {
  if (m->eloc_mode == VQMC_ELOC_DENSE) return false;
  if (!eloc_lc_supported(m)) return false;
  return m->eloc_mode == VQMC_ELOC_LIGHTCONE || m->L >= 14;
}

static size_t al256(size_t x) { return (x + 255) / 256 * 256; }

// Symmetrised local energy: rotated copies, per-rotation E and log|W_CNN|,
// flags, then the workspace of the inner evaluation of 4B configurations.
static size_t sym_head_bytes(const vqmc_model *m, int B) {
  const size_t V = (size_t)4 * B, N = (size_t)m->L * m->L;
  return al256(V * N) + 2 * al256(V * 8) + al256(V * 4);
}

// Dense evaluation: room for the packed fragments of the C -> C layers (the
// call also runs without it, staging the weights from theta per batch).
static size_t dense_ws_bytes(const vqmc_model *m) {
  const int C = m->channels, prec = m->conv_prec;
  size_t per = 0;
  switch (C) {
    case 4: per = Engine<4, P_F32, 1, 1>::FRAG_LAYER; break;
    case 8: per = prec == P_F32 ? Engine<8, P_F32, 1, 1>::FRAG_LAYER
                  : prec == P_BF16 ? Engine<8, P_BF16, 1, 1>::FRAG_LAYER : Engine<8, P_X3, 1, 1>::FRAG_LAYER; break;
    case 16: per = prec == P_F32 ? Engine<16, P_F32, 1, 1>::FRAG_LAYER
                   : prec == P_BF16 ? Engine<16, P_BF16, 1, 1>::FRAG_LAYER : Engine<16, P_X3, 1, 1>::FRAG_LAYER; break;
    default: per = prec == P_F32 ? Engine<32, P_F32, 1, 1>::FRAG_LAYER
                   : prec == P_BF16 ? Engine<32, P_BF16, 1, 1>::FRAG_LAYER : Engine<32, P_X3, 1, 1>::FRAG_LAYER; break;
  }
  return per % 1024 == 0 ? al256((size_t)m->n_layers * per) : 0;
}

static size_t eloc_ws_bytes(const vqmc_model *m, int B) {
  const size_t inner = use_lightcone(m) ? eloc_lc_workspace(m, m->symmetry ? 4 * B : B) : dense_ws_bytes(m);
  return (m->symmetry ? sym_head_bytes(m, B) : 0) + inner;
}

extern "C" vqmc_status vqmc_local_energy_method(const vqmc_model *m, int32_t *method) {
  if (!model_valid(m) || !method) return VQMC_ERR_ARG;
  if (m->eloc_mode == VQMC_ELOC_LIGHTCONE && !eloc_lc_supported(m)) return VQMC_ERR_ARG;
  *method = use_lightcone(m) ? VQMC_ELOC_LIGHTCONE : VQMC_ELOC_DENSE;
  return VQMC_OK;
}

extern "C" vqmc_status vqmc_local_energy_workspace(const vqmc_model *m, int32_t B, size_t *bytes) {
  if (!model_valid(m) || !bytes) return VQMC_ERR_ARG;
  if (B < 0 || (m->symmetry && B > INT32_MAX / 4)) return VQMC_ERR_SHAPE;
  if (m->eloc_mode == VQMC_ELOC_LIGHTCONE && !eloc_lc_supported(m)) return VQMC_ERR_ARG;
  *bytes = eloc_ws_bytes(m, B);
  return VQMC_OK;
}

// The unsymmetrised evaluation of B configurations (dense or light cone).
static vqmc_status eloc_plain(const vqmc_model *m, const float *theta, const int8_t *spins, int32_t B,
                              double *e_loc, int32_t *flags, double *lp, void *ws, size_t ws_bytes,
                              hipStream_t stream) {
  if (use_lightcone(m)) {
    if (!ws || ws_bytes < eloc_lc_workspace(m, B)) return VQMC_ERR_WORKSPACE;
    return eloc_lc(m, theta, spins, B, e_loc, flags, lp, ws, stream);
  }
  FwdArgs a{};
  a.theta = theta;
  a.spins_in = spins;
  a.B = B;
  a.L = m->L;
  a.n_layers = m->n_layers;
  a.marshall = m->marshall;
  a.J1 = m->J1;
  a.J2 = m->J2;
  a.out_d = e_loc;
  a.out_i = flags;
  a.R = 1;
  a.lp_out = lp;
  a.ws = reinterpret_cast<char *>(ws);
  a.ws_bytes = ws ? ws_bytes : 0;
  a.stream = stream;
  return dispatch(K_ELOC, m->channels, m->conv_prec, a);
}

extern "C" vqmc_status vqmc_local_energy(const vqmc_model *m, const float *theta,
                                         const int8_t *spins, int32_t B, double *e_loc,
                                         int32_t *chain_flags, void *workspace, size_t ws_bytes,
                                         hipStream_t stream) {
  if (!model_valid(m)) return VQMC_ERR_ARG;
  if (B < 0 || (m->symmetry && B > INT32_MAX / 4)) return VQMC_ERR_SHAPE;
  if (m->eloc_mode == VQMC_ELOC_LIGHTCONE && !eloc_lc_supported(m)) return VQMC_ERR_ARG;
  if (B > 0 && (!theta || !spins || !e_loc)) return VQMC_ERR_ARG;
  if (!m->symmetry) {
    if (B == 0 && use_lightcone(m)) return VQMC_OK;
    return eloc_plain(m, theta, spins, B, e_loc, chain_flags, nullptr, workspace, ws_bytes, stream);
  }
  const int N = m->L * m->L;
  if (B == 0) return VQMC_OK;
  if (!workspace || ws_bytes < eloc_ws_bytes(m, B)) return VQMC_ERR_WORKSPACE;
  char *w = reinterpret_cast<char *>(workspace);
  const size_t V = (size_t)4 * B;
  int8_t *rot = reinterpret_cast<int8_t *>(w);
  double *e4 = reinterpret_cast<double *>(w + al256(V * N));
  double *lp4 = reinterpret_cast<double *>(w + al256(V * N) + al256(V * 8));
  int32_t *f4 = reinterpret_cast<int32_t *>(w + al256(V * N) + 2 * al256(V * 8));
  char *inner = w + sym_head_bytes(m, B);
  const int64_t total = (int64_t)V * N;
  const int blocks = (int)((total + 255) / 256 < 8192 ? (total + 255) / 256 : 8192);
  rotate_kernel<<<blocks, 256, 0, stream>>>(spins, B, m->L, rot);
  VQMC_LAUNCH_CHECK();
  const vqmc_status st = eloc_plain(m, theta, rot, (int32_t)V, e4, f4, lp4, inner,
                                    ws_bytes - sym_head_bytes(m, B), stream);
  if (st != VQMC_OK) return st;
  sym_combine_kernel<<<(B + 255) / 256, 256, 0, stream>>>(e4, lp4, f4, B, e_loc, chain_flags);
  VQMC_LAUNCH_CHECK();
  return VQMC_OK;
}

// ------------------------------------------------- allocation-free variant

namespace vqmc {

// Room for the C -> C layers' packed fragments of the dense local energy for
// every supported model: kMaxLayers layers of the largest engine (C = 32,
// split-BF16: 36 KiB per layer, 576 KiB in all).
constexpr size_t kScratchBytes = (size_t)kMaxLayers * Engine<32, P_X3, 1, 1>::FRAG_LAYER;
static_assert(kScratchBytes <= (1u << 20), "the no-allocation scratch stays below 1 MiB");

// The library's own device memory for vqmc_local_energy_noalloc, one copy
// per GPU, held until the process ends.  Its host-side name is not a device
// address: host code uses the per-device pointer from hipGetSymbolAddress.
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mutex;
static void *g_scratch_ptr[kMaxDevices];

// The current device's address of `scratch`, looked up on the first call on
// that device (with the device current) and kept; nullptr on failure.
static void *scratch_ptr() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace vqmc

extern "C" vqmc_status vqmc_local_energy_noalloc(const vqmc_model *m, const float *theta, const int8_t *spins,
                                                 int32_t B, double *e_loc, int32_t *chain_flags,
                                                 hipStream_t stream) {
  if (!model_valid(m)) return VQMC_ERR_ARG;
  if (m->symmetry || m->eloc_mode == VQMC_ELOC_LIGHTCONE) return VQMC_ERR_ARG;
  if (B < 0) return VQMC_ERR_SHAPE;
  if (B > 0 && (!theta || !spins || !e_loc)) return VQMC_ERR_ARG;
  vqmc_model dm = *m;
  dm.eloc_mode = VQMC_ELOC_DENSE;
  const size_t need = dense_ws_bytes(&dm);
  if (need > kScratchBytes) return VQMC_ERR_WORKSPACE;
  if (B == 0) return VQMC_OK;
  void *ws = need ? scratch_ptr() : nullptr;
  if (need && !ws) return VQMC_ERR_DEVICE;
  return eloc_plain(&dm, theta, spins, B, e_loc, chain_flags, nullptr, ws, need, stream);
}

extern "C" vqmc_status vqmc_sample(const vqmc_model *m, const float *theta, int8_t *spins,
                                   double *log_psi, int32_t B, int32_t n_sweeps, uint64_t seed,
                                   uint64_t counter_base, int32_t proposal, int32_t *n_accepted,
                                   hipStream_t stream) {
  if (!model_valid(m)) return VQMC_ERR_ARG;
  if (B < 0 || n_sweeps < 0) return VQMC_ERR_SHAPE;
  if (proposal != 0 && proposal != 1) return VQMC_ERR_ARG;
  if (B > 0 && (!theta || !spins)) return VQMC_ERR_ARG;
  FwdArgs a{};
  a.theta = theta;
  a.spins_io = spins;
  a.B = B;
  a.L = m->L;
  a.n_layers = m->n_layers;
  a.marshall = m->marshall;
  a.out_d = log_psi;
  a.out_i = n_accepted;
  a.n_sweeps = n_sweeps;
  a.proposal = proposal;
  a.seed = seed;
  a.counter_base = counter_base;
  a.R = m->symmetry ? 4 : 1;
  a.stream = stream;
  return dispatch(K_SAMPLE, m->channels, m->conv_prec, a);
}
