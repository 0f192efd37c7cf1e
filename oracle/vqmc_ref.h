/* vqmc_ref.h -- FP64 CPU oracle for the CNN-VQMC + SR hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library
 * against a plain, slow, obviously correct implementation of what the paper
 * computes.  Only the tests, the smoke check and the bench's CPU-baseline leg
 * may load it; the product path never does.  It shares no source with the GPU
 * path.
 *
 * Paper: Li et al., "Bridging the Gap between Deep Learning and Frustrated
 * Quantum Spin System for Extreme-scale Simulations on New Generation of
 * Sunway Supercomputer" (arXiv 2108.13830).  Citations name the paper's
 * sections and equations.
 *
 * Conventions (shared with the GPU library by specification, not by code):
 *   site i = y*L + x, periodic; spin +1 = up, -1 = down (Sec. 2.1);
 *   sublattice A = {x + y even};
 *   theta (double here) ordered per layer l = 0..n as W_l[c_out][c_in][ky][kx]
 *   then b_l[c_out]; tap (ky,kx) reads h[(y+ky-1) mod L][(x+kx-1) mod L].
 *
 * Every function returns 0 on success, a negative value on bad arguments.
 */
#ifndef VQMC_REF_H
#define VQMC_REF_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t L;        /* lattice side, even, >= 4 */
  int32_t C;        /* channels */
  int32_t n;        /* C->C conv layers after the 1->C lift */
  double J1, J2;    /* couplings of Eq. (J1-J2) */
  int32_t marshall; /* 1: sign (-1)^{N_up(A)} (Sec. 2.2), 0: all signs +1 */
  int32_t symmetry; /* 1: the rotation-symmetrised amplitude of Eq. (sym-ws),
                       W~(S) = sum_{i=0..3} W(T^i S), T the 90-degree rotation
                       of the L x L configuration; 0: W itself */
} vqmc_ref_model;

int64_t vqmc_ref_num_params(const vqmc_ref_model *m);

/* log|W| and the sign of W for B configurations [B][N]: W = (-1)^{N_up(A)}
 * W_CNN (Sec. 2.2), or its rotation-symmetrised sum (Eq. sym-ws) when
 * m->symmetry; log_abs is then log|sum_i W(T^i sigma)|. */
int vqmc_ref_log_psi(const vqmc_ref_model *m, const double *theta,
                     const int8_t *spins, int32_t B, double *log_abs,
                     int8_t *sign);

/* Local energy E_s of Eq. (Es-Os-G); flags bit 1 non-finite, bit 2 Sz != 0,
 * bit 4 a spin value other than +-1.  flags may be NULL. */
int vqmc_ref_local_energy(const vqmc_ref_model *m, const double *theta,
                          const int8_t *spins, int32_t B, double *e_loc,
                          int32_t *flags);

/* O[b][k] = d log|W(sigma_b)| / d theta_k (W symmetrised when
 * m->symmetry), row stride ldO >= P. */
int vqmc_ref_log_derivs(const vqmc_ref_model *m, const double *theta,
                        const int8_t *spins, int32_t B, double *O,
                        int64_t ldO);

/* SR step (Sec. 3.2.2): E mean/var, F = <O E> - <O><E>, and the exact
 * solution of (S + eps I) delta = F, S = <O O> - <O><O>.  method 0: primal
 * Cholesky of the P x P matrix, 1: the equivalent B x B sample-space system,
 * -1: primal if P <= B else sample-space.  F, e_mean, e_var may be NULL. */
int vqmc_ref_sr_solve(const double *O, int64_t ldO, const double *e_loc,
                      int32_t B, int64_t P, double eps, int32_t method,
                      double *delta, double *F, double *e_mean, double *e_var);

/* S = <O O> - <O><O> written to S [P][P] (for tests at small P). */
/* out = (S + eps I) v with S of Eq. (convar-matrix) applied without
 * forming it; mean: the column means <O> [P]. */
int vqmc_ref_sr_apply(const double *O, int64_t ldO, int32_t B, int64_t P, const double *mean,
                      double eps, const double *v, double *out);

int vqmc_ref_sr_matrix(const double *O, int64_t ldO, int32_t B, int64_t P,
                       double *S);

/* Philox4x32-10 block function (Salmon et al., SC'11). */
void vqmc_ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2],
                            uint32_t out[4]);

/* Metropolis exchange sampler (Sec. 3.1).  proposal 0: a uniformly drawn J1
 * bond, parallel pairs rejected; proposal 1: a uniformly drawn antiparallel
 * J1 bond with the Hastings factor.  spins [B][N] in/out; log_abs [B] out;
 * n_acc [B] out; min_margin [B] out: the smallest |log-acceptance - ln r|
 * over the chain's decisions (how close the chain came to a tie).  Any of the
 * three outputs may be NULL. */
int vqmc_ref_sample(const vqmc_ref_model *m, const double *theta,
                    int8_t *spins, int32_t B, int32_t n_sweeps, uint64_t seed,
                    uint64_t counter_base, int32_t proposal, double *log_abs,
                    int32_t *n_acc, double *min_margin);

#ifdef __cplusplus
}
#endif
#endif
