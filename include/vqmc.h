/* vqmc.h -- C ABI of libvqmc: the hot path of CNN variational Monte Carlo
 * with Stochastic Reconfiguration for the spin-1/2 J1-J2 Heisenberg model on
 * periodic L x L lattices (Li et al., arXiv 2108.13830), on one MI355X GPU.
 *
 * Every entry point is extern "C", takes plain pointers and sizes, returns a
 * vqmc_status, never throws and never allocates device memory: the caller
 * owns every buffer (device buffers are marked "dev", host ones "host").
 * Calls only enqueue work on the given HIP stream; the one exception is
 * vqmc_sr_solve with info != NULL, which synchronises the stream before it
 * returns to fill *info.  Argument and shape errors are detected before any
 * launch and return VQMC_ERR_ARG / VQMC_ERR_SHAPE with no side effect; a
 * failed launch returns VQMC_ERR_DEVICE; faults inside kernels surface at the
 * caller's next synchronisation.  Calls on different streams that write the
 * same buffers race.  The library keeps no data between calls; the one
 * resource it holds is, per device, an internal HIP stream and two events
 * (created by the first Cholesky solve of order > 1024 and kept until the
 * process ends) on which that solve overlaps part of its trailing updates
 * with the factorisation of the next panel; the call's own stream waits for
 * that work before the call's remaining kernels, so the call still behaves
 * as work enqueued on its own stream.  On a stream under HIP graph capture
 * the solve uses no side stream (every kernel goes to the captured stream).
 *
 * Layouts (a specification the FP64 test oracle also follows):
 *   - site i = y*L + x, periodic boundaries, spin +1 = up, -1 = down (Sec. 2.1);
 *   - sublattice A = {x + y even};
 *   - spins: int8 [B][N], N = L*L, row-major;
 *   - theta: float32 [P], for layer l = 0..n the weights W_l[c_out][c_in][ky][kx]
 *     then the biases b_l[c_out]; layer 0 lifts 1 -> C channels, layers
 *     1..n map C -> C; tap (ky,kx) multiplies h[(y+ky-1) mod L][(x+kx-1) mod L];
 *   - O: float32 [B][ldO], column k = d log|psi| / d theta_k in theta order.
 */
#ifndef VQMC_H
#define VQMC_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VQMC_OK = 0,
  VQMC_ERR_ARG = 1,       /* a null pointer, bad enum value or bad model   */
  VQMC_ERR_SHAPE = 2,     /* sizes out of the supported range              */
  VQMC_ERR_DEVICE = 3,    /* a HIP call or a kernel launch failed          */
  VQMC_ERR_WORKSPACE = 4, /* workspace missing or smaller than required    */
  VQMC_ERR_NOT_SPD = 5,   /* Cholesky met a non-positive pivot             */
  VQMC_WARN_NOT_CONVERGED = 6, /* CG reached max_iter; delta and info hold the
                                  last iterate                             */
  VQMC_ERR_NONFINITE = 7  /* the SR solve met non-finite energies, or a
                             non-finite CG residual (non-finite O)         */
} vqmc_status;

/* Arithmetic of the convolutions (all accumulate in FP32):
 *   FP32   -- FP32 operands on the FP32 matrix cores;
 *   BF16   -- operands rounded to nearest-even BF16, one product;
 *   BF16X3 -- each operand split x = hi + lo (hi = bf16(x), lo = bf16(x - hi))
 *             and hi*hi + hi*lo + lo*hi accumulated.
 * BF16 and BF16X3 need channels % 8 == 0. */
typedef enum { VQMC_PREC_FP32 = 0, VQMC_PREC_BF16 = 1, VQMC_PREC_BF16X3 = 2 } vqmc_prec;

typedef enum { VQMC_ACT_TANH = 0 } vqmc_act;

/* How vqmc_local_energy evaluates the exchanged configurations s':
 *   DENSE     -- the full forward pass of every s' (batched per workgroup);
 *   LIGHTCONE -- one FP32 forward pass of s per sample, then for every s'
 *                only the change of the activations inside the growing
 *                neighbourhood of the exchanged pair (needs channels 16 or
 *                32 and a workspace);
 *   AUTO      -- LIGHTCONE when supported and L >= 14, else DENSE. */
typedef enum { VQMC_ELOC_AUTO = 0, VQMC_ELOC_DENSE = 1, VQMC_ELOC_LIGHTCONE = 2 } vqmc_eloc_mode;

/* The variational state and the Hamiltonian.
 *   L          lattice side, even, 4 <= L <= 24;
 *   channels   C in {4, 8, 16, 32};
 *   n_layers   n >= 1 C -> C conv layers after the 1 -> C lift (n <= 16);
 *   activation VQMC_ACT_TANH after every conv; log|W_CNN| is the sum of the
 *              last layer's outputs over channels and sites (Sec. 2.2,
 *              Eq. wcnn);
 *   J1, J2     couplings of Eq. (J1-J2), H = J1/4 sum_<ij> s_i.s_j
 *              + J2/4 sum_<<ij>> s_i.s_j;
 *   marshall   1: W = (-1)^{N_up(A)} W_CNN (Sec. 2.2), 0: W = W_CNN;
 *   conv_prec  vqmc_prec of the forward convolutions (log psi, local energy
 *              and sampler; with LIGHTCONE, of the convolutions of the
 *              activation changes).  The log-derivative path always runs FP32;
 *   eloc_mode  vqmc_eloc_mode;
 *   symmetry   0: the amplitude W above; 1: the rotation-symmetrised
 *              W~(S) = sum_{i=0..3} W(T^i S) of Eq. (sym-ws), T the quarter
 *              turn of the lattice, (T S) at (y, x) = S at (x, L-1-y).  On an
 *              even lattice T maps sublattice A onto B, and for Sz = 0 N/2 is
 *              even, so the four Marshall signs agree: every entry point
 *              evaluates log|W~| = logsumexp_i log W_CNN(T^i S) with the sign
 *              of S (for Sz != 0, which the local energy flags, the unsigned
 *              sum).  Costs four forward passes per configuration. */
typedef struct {
  int32_t L, channels, n_layers, activation;
  double J1, J2;
  int32_t marshall;
  int32_t conv_prec;
  int32_t eloc_mode;
  int32_t symmetry;
} vqmc_model;

/* Number of parameters P = (9C + C) + n (9C^2 + C); < 0 for an invalid model. */
int64_t vqmc_num_params(const vqmc_model *m);

/* Static description of a status code (never NULL). */
const char *vqmc_status_string(vqmc_status s);

/* Metropolis exchange sampler (Sec. 3.1, Fig. framework b/c).
 * Each of the B chains performs n_sweeps * N proposals in place on its row of
 * spins (dev int8 [B][N], +-1, Sz = 0 is conserved).  Proposal t of chain c
 * draws Philox4x32-10 (Salmon et al., SC'11) with counter
 * (t_lo, t_hi, c, 0), t = counter_base + t_local, key (seed_lo, seed_hi):
 *   proposal 0: bond k = floor(u0 * 2N / 2^32) among the 2N J1 bonds (site k
 *               to its right neighbour for k < N, site k - N to the one below
 *               otherwise); a parallel pair is a rejected move;
 *   proposal 1: the floor(u0 * n_ap / 2^32)-th antiparallel J1 bond in that
 *               order, with the Hastings factor n_ap(s) / n_ap(s');
 * and accepts iff 2 (log|W'| - log|W|) [+ ln Hastings] >= ln r with
 * r = (u1 + 1/2) 2^-32 (the paper's P = (W'/W)^2 >= r, r in (0,1)).
 * log_psi (dev double [B], nullable) receives the final log|W_CNN| (with
 * symmetry, log|W~|: every proposal then evaluates the four rotations);
 * n_accepted (dev int32 [B], nullable) the accepted moves.  B >= 0. */
vqmc_status vqmc_sample(const vqmc_model *m, const float *theta, int8_t *spins,
                        double *log_psi, int32_t B, int32_t n_sweeps,
                        uint64_t seed, uint64_t counter_base, int32_t proposal,
                        int32_t *n_accepted, hipStream_t stream);

/* log|W_CNN(sigma_b)| (dev double [B]) and the Marshall sign (dev int8 [B],
 * nullable; +1 when marshall = 0) of B configurations (Sec. 2.2); with
 * symmetry, log|W~(sigma_b)|, the logsumexp over the four rotations. */
vqmc_status vqmc_log_psi(const vqmc_model *m, const float *theta,
                         const int8_t *spins, int32_t B, double *log_abs_psi,
                         int8_t *sign, hipStream_t stream);

/* Local energy E_s of Eq. (Es-Os-G) for B configurations:
 *   E_s = sum_b J_b/4 s_i s_j  over the 4N bonds (J1: right and below
 *         neighbours, J2: lower-right and lower-left; Sec. 3.1)
 *       + sum over antiparallel bonds of J_b/2 * mu_b * exp(log|W(s')| - log|W(s)|),
 * s' = s with the pair exchanged, mu_b the ratio of Marshall signs (-1 for
 * J1 and +1 for J2 bonds when marshall = 1).  Every s' of a sample is built
 * on chip and evaluated in the same launch.  e_loc: dev double [B].
 * chain_flags (dev int32 [B], nullable): bit 1 non-finite log psi or E_s,
 * bit 2 Sz != 0, bit 4 a spin value other than +-1; the status stays OK.
 * With symmetry, W~(s')/W~(s) = sum_i p_i mu W_CNN(T^i s')/W_CNN(T^i s) with
 * p_i = W_CNN(T^i s)/sum_j W_CNN(T^j s), and the exchanges of T^i s are the
 * rotated exchanges of s (the bond set maps onto itself, J1 to J1 and J2 to
 * J2), so E_s = sum_i p_i E_CNN(T^i s): the 4B rotated configurations are
 * written to the workspace, evaluated by either method above, and combined;
 * bit 1 of chain_flags is set if any rotation's value is non-finite.
 * workspace: dev, at least vqmc_local_energy_workspace bytes (may be NULL
 * for the dense evaluation without symmetry). */
vqmc_status vqmc_local_energy(const vqmc_model *m, const float *theta,
                              const int8_t *spins, int32_t B, double *e_loc,
                              int32_t *chain_flags, void *workspace,
                              size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the local energy
 * of vqmc_local_energy in the dense evaluation, with the packed layer weights
 * kept in the library's own device array (576 KiB per GPU, taken on the first
 * call on a device and held until the process ends) instead of a workspace.
 * Same arguments and results as vqmc_local_energy with eloc_mode DENSE (AUTO
 * is taken as DENSE); VQMC_ERR_ARG for symmetry = 1 or eloc_mode LIGHTCONE,
 * which need a caller workspace; VQMC_ERR_WORKSPACE if the model's packed
 * weights exceed the array (never for the models vqmc_num_params accepts);
 * VQMC_ERR_DEVICE if the array's address cannot be obtained.  The call
 * allocates nothing.  Every call on a GPU uses that GPU's one array: calls
 * that overlap on one GPU (several streams or host threads) race. */
vqmc_status vqmc_local_energy_noalloc(const vqmc_model *m, const float *theta,
                                      const int8_t *spins, int32_t B, double *e_loc,
                                      int32_t *chain_flags, hipStream_t stream);

/* The method vqmc_local_energy uses for this model (*method: VQMC_ELOC_DENSE
 * or VQMC_ELOC_LIGHTCONE, AUTO resolved); VQMC_ERR_ARG when the model asks
 * for the light cone and the light cone does not support it. */
vqmc_status vqmc_local_energy_method(const vqmc_model *m, int32_t *method);

/* Workspace (device bytes) vqmc_local_energy needs for this model and B.
 * For the dense evaluation without symmetry it is the room for the C -> C
 * layers' weights packed once per call (n layers x 5-36 KiB), and optional:
 * with a NULL workspace (or a smaller one) the weights are staged from theta
 * for every batch instead, with the same results, more slowly. */
vqmc_status vqmc_local_energy_workspace(const vqmc_model *m, int32_t B, size_t *bytes);

/* Workspace (device bytes) needed by vqmc_log_derivs for this model. */
vqmc_status vqmc_log_derivs_workspace(const vqmc_model *m, int32_t B, size_t *bytes);

/* Per-sample log-derivatives O[b][k] = d log|W(sigma_b)| / d theta_k (the
 * O_s of Eq. Es-Os-G), FP32, by a hand-written reverse pass that recomputes
 * the forward activations per sample.  With symmetry, d log|W~| =
 * sum_i p_i d log W_CNN(T^i S) (p_i as for the local energy): the reverse
 * pass runs once per rotation and the rows are accumulated in place with
 * running rescaling (the largest weight kept at 1 until the final
 * normalisation).  O: dev float [B][ldO], ldO >= P.
 * workspace: dev, at least the bytes vqmc_log_derivs_workspace reports. */
vqmc_status vqmc_log_derivs(const vqmc_model *m, const float *theta,
                            const int8_t *spins, int32_t B, float *O, int64_t ldO,
                            void *workspace, size_t ws_bytes, hipStream_t stream);

/* Options of the SR solve (Sec. 3.2.2).
 *   method   0 auto: the smaller of the two exact forms (B < P: method 3,
 *            else method 1) while its order is at most 65536, else CG;
 *            1 Cholesky of the explicit P x P matrix, 2 matrix-free
 *            conjugate gradients, 3 Cholesky of the equivalent B x B
 *            sample-space matrix (the same delta, by the push-through
 *            identity Oc^T (Oc Oc^T/B + eps I)^-1 = (Oc^T Oc/B + eps I)^-1 Oc^T);
 *   s_prec   (method 1) 0: S accumulated by FP32 matrix cores from FP32
 *            centred O; 1: FP64 accumulation (FP64 matrix cores);
 *   eps      diagonal shift (> 0);
 *   tol      CG stop: ||r|| / ||F|| <= tol;
 *   max_iter CG iteration cap. */
typedef struct {
  int32_t method;
  int32_t s_prec;
  double eps;
  double tol;
  int32_t max_iter;
} vqmc_sr_opts;

/* Host-side report of one SR solve. */
typedef struct {
  double e_mean;       /* <E_s>                                  */
  double e_var;        /* <(E_s - <E_s>)^2>                      */
  int32_t iters;       /* CG iterations (0 for Cholesky)         */
  double rel_residual; /* CG ||r|| / ||F|| (0 for Cholesky)      */
} vqmc_sr_info;

/* Workspace (device bytes) needed by vqmc_sr_solve. */
vqmc_status vqmc_sr_workspace(int32_t B, int64_t P, const vqmc_sr_opts *o, size_t *bytes);

/* SR step (Sec. 3.2.2; Eqs. delta and convar-matrix), all arithmetic FP64:
 *   E^c = E - <E>, O^c = O - <O>,
 *   F = (1/B) O^cT E^c            (= <O E> - <O><E>, the gradient G),
 *   S = (1/B) O^cT O^c            (= <O O> - <O><O>),
 *   delta solves (S + eps I) delta = F.
 * O: dev float [B][ldO]; e_loc: dev double [B]; delta: dev double [P];
 * F: dev double [P] (nullable); info: host (nullable, forces a stream
 * synchronisation).  B >= 2, P >= 1.  Only with info are the device-side
 * failures returned: VQMC_ERR_NOT_SPD when the factorisation met a
 * non-positive pivot (it then finishes with unit pivots, so delta is
 * finite but wrong), VQMC_ERR_NONFINITE when the energies or the CG
 * residual are not finite (CG then stops). */
vqmc_status vqmc_sr_solve(const float *O, int64_t ldO, const double *e_loc,
                          int32_t B, int64_t P, const vqmc_sr_opts *o,
                          double *delta, double *F, void *workspace,
                          size_t ws_bytes, vqmc_sr_info *info, hipStream_t stream);

/* One iteration of the optimisation loop (Sec. 3.1 and 3.2, Fig. framework):
 *   Step 1: n_sweeps sweeps of vqmc_sample on the B chains, in place, from
 *           where the previous iteration left them (proposal, seed and
 *           counters as there: this call uses counters counter_base ..
 *           counter_base + n_sweeps*N - 1, so the caller advances
 *           counter_base by n_sweeps*N per call);
 *   Step 2: E_s (vqmc_local_energy), O_s (vqmc_log_derivs, FP32), the SR
 *           solve (S + eps I) delta = F with options sr, and the update
 *           theta <- theta - lr * delta (FP64 arithmetic, rounded once to
 *           FP32), in place on theta.
 * e_loc (dev double [B], nullable) receives the local energies of the
 * sampled configurations (under the theta the call started with).  info
 * (host, nullable) receives their mean and variance and the SR report, and
 * forces a stream synchronisation.  The update kernel reads the SR solve's
 * device status and leaves theta bit-unchanged when the factorisation met a
 * non-positive pivot or the energies or CG residual were not finite, with or
 * without info; only with info is that failure also returned
 * (VQMC_ERR_NOT_SPD or VQMC_ERR_NONFINITE).  With CG that reaches max_iter
 * the update uses the last iterate and VQMC_WARN_NOT_CONVERGED is returned
 * (with info).  workspace: dev, vqmc_vmc_step_workspace bytes (E_s, O, delta
 * and the three inner workspaces).  B >= 2, n_sweeps >= 0. */
vqmc_status vqmc_vmc_step(const vqmc_model *m, float *theta, int8_t *spins,
                          int32_t B, int32_t n_sweeps, uint64_t seed,
                          uint64_t counter_base, int32_t proposal,
                          const vqmc_sr_opts *sr, double lr, double *e_loc,
                          void *workspace, size_t ws_bytes, vqmc_sr_info *info,
                          hipStream_t stream);

/* Workspace (device bytes) of vqmc_vmc_step for this model, B and solver. */
vqmc_status vqmc_vmc_step_workspace(const vqmc_model *m, int32_t B,
                                    const vqmc_sr_opts *sr, size_t *bytes);

#ifdef __cplusplus
}
#endif
#endif /* VQMC_H */
