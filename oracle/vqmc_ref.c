/* vqmc_ref.c -- FP64 CPU oracle for the CNN-VQMC + SR hot path.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * bench's CPU-baseline leg, never by the product path.  Plain loops in double
 * precision, OpenMP only over independent samples / rows; no blocking, no
 * fusion.  Shares no code with the GPU library.
 *
 * Paper: arXiv 2108.13830 (Li et al.).  Each function names the section or
 * equation it follows.
 */
#include "vqmc_ref.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ model */

static int model_ok(const vqmc_ref_model *m) {
  return m && m->L >= 4 && (m->L % 2) == 0 && m->C >= 1 && m->n >= 0;
}

/* Layer l has C_in = 1 for the lift (l = 0) and C otherwise; 9 weights per
 * (c_out, c_in) pair and one bias per c_out. */
static int64_t layer_cin(const vqmc_ref_model *m, int l) { return l == 0 ? 1 : m->C; }

int64_t vqmc_ref_num_params(const vqmc_ref_model *m) {
  if (!model_ok(m)) return -1;
  int64_t P = 0;
  for (int l = 0; l <= m->n; ++l) P += (int64_t)m->C * layer_cin(m, l) * 9 + m->C;
  return P;
}

static int64_t weight_offset(const vqmc_ref_model *m, int l) {
  int64_t off = 0;
  for (int k = 0; k < l; ++k) off += (int64_t)m->C * layer_cin(m, k) * 9 + m->C;
  return off;
}

static int wrap(int a, int L) { return ((a % L) + L) % L; }

/* ------------------------------------------------------- CNN amplitude */

/* Forward pass of the convolutional amplitude, Sec. 2.2, Eq. (wcnn):
 *   h_0 = spins (one channel),
 *   h_l[co][y][x] = tanh(b_l[co] + sum_{ci,ky,kx} W_l[co][ci][ky][kx]
 *                          * h_{l-1}[ci][(y+ky-1) mod L][(x+kx-1) mod L]),
 *   log|W_CNN| = sum_{c,i} h_{n+1}[c][i].
 * acts (optional) receives every layer's output h_1..h_{n+1}, each [C][N],
 * for the reverse pass. */
static double forward(const vqmc_ref_model *m, const double *theta,
                      const int8_t *s, double *acts) {
  const int L = m->L, N = L * L, C = m->C;
  double *prev = (double *)malloc(sizeof(double) * (size_t)C * N);
  double *cur = (double *)malloc(sizeof(double) * (size_t)C * N);
  /* the layer's weights as wt[ky][kx][ci][co] and one site's outputs z[co]:
   * the same sums as the formula above, taken tap by tap so that the
   * innermost loop runs over independent outputs */
  double *wt = (double *)malloc(sizeof(double) * (size_t)9 * C * C);
  double *z = (double *)malloc(sizeof(double) * (size_t)C);
  for (int i = 0; i < N; ++i) prev[i] = (double)s[i];
  for (int l = 0; l <= m->n; ++l) {
    const int cin = (int)layer_cin(m, l);
    const double *W = theta + weight_offset(m, l);
    const double *bias = W + (int64_t)C * cin * 9;
    for (int co = 0; co < C; ++co)
      for (int ci = 0; ci < cin; ++ci)
        for (int t = 0; t < 9; ++t) wt[((size_t)t * cin + ci) * C + co] = W[(co * cin + ci) * 9 + t];
    for (int y = 0; y < L; ++y)
      for (int x = 0; x < L; ++x) {
        for (int co = 0; co < C; ++co) z[co] = bias[co];
        for (int ky = 0; ky < 3; ++ky)
          for (int kx = 0; kx < 3; ++kx) {
            const int src = wrap(y + ky - 1, L) * L + wrap(x + kx - 1, L);
            const double *w = wt + (size_t)(ky * 3 + kx) * cin * C;
            for (int ci = 0; ci < cin; ++ci) {
              const double v = prev[ci * N + src];
              for (int co = 0; co < C; ++co) z[co] += w[ci * C + co] * v;
            }
          }
        for (int co = 0; co < C; ++co) cur[co * N + y * L + x] = tanh(z[co]);
      }
    if (acts) memcpy(acts + (size_t)l * C * N, cur, sizeof(double) * (size_t)C * N);
    double *t = prev; prev = cur; cur = t;
  }
  double sum = 0.0;
  for (int i = 0; i < C * N; ++i) sum += prev[i];
  free(prev);
  free(cur);
  free(wt);
  free(z);
  return sum;
}

/* Marshall-Peierls sign (-1)^{N_up(A)}, Sec. 2.2; A = {x + y even}. */
static int marshall_sign(const vqmc_ref_model *m, const int8_t *s) {
  if (!m->marshall) return 1;
  const int L = m->L;
  int up_a = 0;
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x)
      if (((x + y) & 1) == 0 && s[y * L + x] > 0) ++up_a;
  return (up_a & 1) ? -1 : 1;
}

/* T^i S for the 90-degree rotation T of the L x L configuration (Eq.
 * sym-ws): the element at (y, x) of T S is the element of S at (x, L-1-y),
 * i.e. the whole square turned a quarter counter-clockwise. */
static void rotate_config(int L, const int8_t *s, int i, int8_t *out) {
  for (int y = 0; y < L; ++y)
    for (int x = 0; x < L; ++x) {
      int sy = y, sx = x;
      for (int k = 0; k < i; ++k) {
        const int ty = sx, tx = L - 1 - sy;
        sy = ty;
        sx = tx;
      }
      out[y * L + x] = s[sy * L + sx];
    }
}

/* log|W| and sign(W) of Sec. 2.2, W = (-1)^{N_up(A)} W_CNN with
 * W_CNN = exp(sum of the last layer); with m->symmetry the sum of Eq.
 * (sym-ws), W~ = sum_i W(T^i S), formed literally as a signed sum (scaled by
 * the largest term).  lw (optional, [4]) receives the weights
 * W(T^i S) / W~ of the four terms, which give d log|W~| = sum_i lw_i
 * d log|W_CNN(T^i S)|. */
static double amplitude(const vqmc_ref_model *m, const double *theta, const int8_t *s, int *sign,
                        double *lw) {
  if (!m->symmetry) {
    if (sign) *sign = marshall_sign(m, s);
    if (lw) lw[0] = 1.0;
    return forward(m, theta, s, NULL);
  }
  const int L = m->L, N = L * L;
  int8_t *r = (int8_t *)malloc((size_t)N);
  double lg[4];
  int sg[4];
  double mx = -INFINITY;
  for (int i = 0; i < 4; ++i) {
    rotate_config(L, s, i, r);
    lg[i] = forward(m, theta, r, NULL);
    sg[i] = marshall_sign(m, r);
    if (lg[i] > mx) mx = lg[i];
  }
  free(r);
  double a = 0.0;
  for (int i = 0; i < 4; ++i) a += sg[i] * exp(lg[i] - mx);
  if (sign) *sign = a < 0.0 ? -1 : 1;
  if (lw)
    for (int i = 0; i < 4; ++i) lw[i] = sg[i] * exp(lg[i] - mx) / a;
  return mx + log(fabs(a));
}

int vqmc_ref_log_psi(const vqmc_ref_model *m, const double *theta,
                     const int8_t *spins, int32_t B, double *log_abs,
                     int8_t *sign) {
  if (!model_ok(m) || B < 0 || (B > 0 && (!theta || !spins || !log_abs))) return -1;
  const int N = m->L * m->L;
#pragma omp parallel for schedule(dynamic)
  for (int b = 0; b < B; ++b) {
    int sg;
    log_abs[b] = amplitude(m, theta, spins + (size_t)b * N, &sg, NULL);
    if (sign) sign[b] = (int8_t)sg;
  }
  return 0;
}

/* ---------------------------------------------------------- local energy */

/* The 4N bonds of Sec. 3.1 (each pair counted once): for every site the J1
 * bonds to the right and below neighbours, and the J2 bonds to the
 * lower-right and lower-left diagonal neighbours. */
static void bond(const vqmc_ref_model *m, int k, int *i, int *j, double *J) {
  const int L = m->L, N = L * L;
  const int kind = k / N, site = k % N, y = site / L, x = site % L;
  *i = site;
  switch (kind) {
    case 0: *j = y * L + wrap(x + 1, L); *J = m->J1; break;
    case 1: *j = wrap(y + 1, L) * L + x; *J = m->J1; break;
    case 2: *j = wrap(y + 1, L) * L + wrap(x + 1, L); *J = m->J2; break;
    default: *j = wrap(y + 1, L) * L + wrap(x - 1, L); *J = m->J2; break;
  }
}

/* E_s(sigma) = sum_{sigma'} (W(sigma')/W(sigma)) <sigma|H|sigma'>, Eq.
 * (sum-Es) and (Es-Os-G), with H of Eq. (J1-J2): J/4 sigma_i.sigma_j has the
 * diagonal element J/4 s_i s_j and the element J/2 between a configuration
 * and the one with the antiparallel pair (i, j) exchanged.  The amplitude
 * ratio is exp(log|W'| - log|W|) times the ratio of Marshall signs. */
int vqmc_ref_local_energy(const vqmc_ref_model *m, const double *theta,
                          const int8_t *spins, int32_t B, double *e_loc,
                          int32_t *flags) {
  if (!model_ok(m) || B < 0 || (B > 0 && (!theta || !spins || !e_loc))) return -1;
  const int N = m->L * m->L, NB = 4 * N;
  /* all (sample, bond) pairs, so that OpenMP spreads the sigma' forwards */
  double *lp = (double *)malloc(sizeof(double) * ((size_t)B + 1));
  double *lpp = (double *)malloc(sizeof(double) * ((size_t)B * NB + 1));
  int *sg0 = (int *)malloc(sizeof(int) * ((size_t)B + 1));
  int *sgp = (int *)malloc(sizeof(int) * ((size_t)B * NB + 1));
#pragma omp parallel for schedule(dynamic)
  for (int b = 0; b < B; ++b) lp[b] = amplitude(m, theta, spins + (size_t)b * N, &sg0[b], NULL);
#pragma omp parallel for schedule(dynamic)
  for (int64_t t = 0; t < (int64_t)B * NB; ++t) {
    const int b = (int)(t / NB), k = (int)(t % NB);
    const int8_t *s = spins + (size_t)b * N;
    int i, j;
    double J;
    bond(m, k, &i, &j, &J);
    lpp[t] = 0.0;
    sgp[t] = 1;
    if (s[i] != s[j]) {
      int8_t *sp = (int8_t *)malloc((size_t)N);
      memcpy(sp, s, (size_t)N);
      sp[i] = s[j];
      sp[j] = s[i];
      lpp[t] = amplitude(m, theta, sp, &sgp[t], NULL);
      free(sp);
    }
  }
  for (int b = 0; b < B; ++b) {
    const int8_t *s = spins + (size_t)b * N;
    const int sg = sg0[b];
    double e = 0.0;
    int f = 0, sz = 0;
    for (int i = 0; i < N; ++i) {
      sz += s[i];
      if (s[i] != 1 && s[i] != -1) f |= 4;
    }
    if (sz != 0) f |= 2;
    for (int k = 0; k < NB; ++k) {
      int i, j;
      double J;
      bond(m, k, &i, &j, &J);
      e += 0.25 * J * (double)s[i] * (double)s[j];
      if (s[i] != s[j]) {
        const double mu = (double)(sgp[(size_t)b * NB + k] * sg);
        e += 0.5 * J * mu * exp(lpp[(size_t)b * NB + k] - lp[b]);
      }
    }
    if (!isfinite(e) || !isfinite(lp[b])) f |= 1;
    e_loc[b] = e;
    if (flags) flags[b] = f;
  }
  free(lp);
  free(lpp);
  free(sg0);
  free(sgp);
  return 0;
}

/* ------------------------------------------------------- log-derivatives */

/* O_k = (1/W) dW/d a_k of Eq. (Es-Os-G) = d log|W_CNN| / d theta_k (the
 * Marshall sign does not depend on theta).  Reverse-mode differentiation of
 * the forward pass above:
 *   g_{n+1} = 1;  delta_l = g_l (1 - h_l^2);
 *   dL/dW_l[co][ci][ky][kx] = sum_{y,x} delta_l[co][y][x] h_{l-1}[ci][y+ky-1][x+kx-1];
 *   dL/db_l[co] = sum_{y,x} delta_l[co][y][x];
 *   g_{l-1}[ci][y+ky-1][x+kx-1] += W_l[co][ci][ky][kx] delta_l[co][y][x]. */
static void log_derivs_one(const vqmc_ref_model *m, const double *theta,
                           const int8_t *s, double *O) {
  const int L = m->L, N = L * L, C = m->C, nl = m->n + 1;
  double *acts = (double *)malloc(sizeof(double) * (size_t)nl * C * N);
  double *h0 = (double *)malloc(sizeof(double) * (size_t)N);
  double *g = (double *)malloc(sizeof(double) * (size_t)C * N);
  double *gp = (double *)malloc(sizeof(double) * (size_t)C * N);
  double *dl = (double *)malloc(sizeof(double) * (size_t)C * N);
  forward(m, theta, s, acts);
  for (int i = 0; i < N; ++i) h0[i] = (double)s[i];
  for (int i = 0; i < C * N; ++i) g[i] = 1.0;
  for (int l = m->n; l >= 0; --l) {
    const int cin = (int)layer_cin(m, l);
    const double *h = acts + (size_t)l * C * N;
    const double *hp = (l == 0) ? h0 : acts + (size_t)(l - 1) * C * N;
    const int64_t off = weight_offset(m, l);
    const double *W = theta + off;
    double *dW = O + off;
    double *db = dW + (int64_t)C * cin * 9;
    for (int i = 0; i < C * N; ++i) dl[i] = g[i] * (1.0 - h[i] * h[i]);
    for (int co = 0; co < C; ++co) {
      double sb = 0.0;
      for (int i = 0; i < N; ++i) sb += dl[co * N + i];
      db[co] = sb;
      for (int ci = 0; ci < cin; ++ci)
        for (int ky = 0; ky < 3; ++ky)
          for (int kx = 0; kx < 3; ++kx) {
            double sw = 0.0;
            for (int y = 0; y < L; ++y)
              for (int x = 0; x < L; ++x)
                sw += dl[co * N + y * L + x] *
                      hp[ci * N + wrap(y + ky - 1, L) * L + wrap(x + kx - 1, L)];
            dW[((co * cin + ci) * 3 + ky) * 3 + kx] = sw;
          }
    }
    if (l > 0) {
      for (int i = 0; i < cin * N; ++i) gp[i] = 0.0;
      for (int co = 0; co < C; ++co)
        for (int ci = 0; ci < cin; ++ci)
          for (int ky = 0; ky < 3; ++ky)
            for (int kx = 0; kx < 3; ++kx)
              for (int y = 0; y < L; ++y)
                for (int x = 0; x < L; ++x)
                  gp[ci * N + wrap(y + ky - 1, L) * L + wrap(x + kx - 1, L)] +=
                      W[((co * cin + ci) * 3 + ky) * 3 + kx] * dl[co * N + y * L + x];
      double *t = g; g = gp; gp = t;
    }
  }
  free(acts); free(h0); free(g); free(gp); free(dl);
}

/* With the symmetrised amplitude (Eq. sym-ws), d log|W~| = sum_i lw_i
 * d log|W_CNN(T^i S)| with the term weights lw_i = W(T^i S) / W~. */
int vqmc_ref_log_derivs(const vqmc_ref_model *m, const double *theta,
                        const int8_t *spins, int32_t B, double *O,
                        int64_t ldO) {
  const int64_t P = vqmc_ref_num_params(m);
  if (P < 0 || B < 0 || ldO < P || (B > 0 && (!theta || !spins || !O))) return -1;
  const int N = m->L * m->L;
#pragma omp parallel for schedule(dynamic)
  for (int b = 0; b < B; ++b) {
    const int8_t *s = spins + (size_t)b * N;
    double *Ob = O + (size_t)b * ldO;
    if (!m->symmetry) {
      log_derivs_one(m, theta, s, Ob);
      continue;
    }
    double lw[4];
    amplitude(m, theta, s, NULL, lw);
    int8_t *r = (int8_t *)malloc((size_t)N);
    double *Oi = (double *)malloc(sizeof(double) * (size_t)P);
    for (int64_t k = 0; k < P; ++k) Ob[k] = 0.0;
    for (int i = 0; i < 4; ++i) {
      rotate_config(m->L, s, i, r);
      log_derivs_one(m, theta, r, Oi);
      for (int64_t k = 0; k < P; ++k) Ob[k] += lw[i] * Oi[k];
    }
    free(r);
    free(Oi);
  }
  return 0;
}

/* ------------------------------------------------------------------- SR */

/* Column means <O_k> and the centred copy O^c = O - <O>. */
static double *centred(const double *O, int64_t ldO, int32_t B, int64_t P, double *mean) {
  for (int64_t k = 0; k < P; ++k) {
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += O[(size_t)b * ldO + k];
    mean[k] = s / B;
  }
  double *Oc = (double *)malloc(sizeof(double) * (size_t)B * P);
  for (int b = 0; b < B; ++b)
    for (int64_t k = 0; k < P; ++k) Oc[(size_t)b * P + k] = O[(size_t)b * ldO + k] - mean[k];
  return Oc;
}

/* Cholesky factorisation A = L L^T of an SPD n x n matrix (row-major, lower
 * triangle used), in place; the textbook column-by-column recurrence.
 * Returns -2 if a pivot is not positive. */
static int cholesky(double *A, int64_t n) {
  for (int64_t j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int64_t k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
    if (!(d > 0.0)) return -2;
    const double ljj = sqrt(d);
    A[j * n + j] = ljj;
#pragma omp parallel for schedule(static)
    for (int64_t i = j + 1; i < n; ++i) {
      double v = A[i * n + j];
      for (int64_t k = 0; k < j; ++k) v -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = v / ljj;
    }
  }
  return 0;
}

/* Solve L L^T x = r: forward substitution L y = r, then back substitution
 * L^T x = y (the two triangular solves of Sec. 3.2.2). */
static void chol_solve(const double *Lm, int64_t n, const double *r, double *x) {
  for (int64_t i = 0; i < n; ++i) {
    double v = r[i];
    for (int64_t k = 0; k < i; ++k) v -= Lm[i * n + k] * x[k];
    x[i] = v / Lm[i * n + i];
  }
  for (int64_t i = n - 1; i >= 0; --i) {
    double v = x[i];
    for (int64_t k = i + 1; k < n; ++k) v -= Lm[k * n + i] * x[k];
    x[i] = v / Lm[i * n + i];
  }
}

/* One application of the shifted SR matrix of Eq. (convar-matrix) to a
 * vector, without forming it: out = (1/B) sum_b (O_b - <O>) ((O_b - <O>) . v)
 * + eps v, with the column means <O> given (the work of one iteration of an
 * iterative solve of Eq. delta).  Two passes over O: the row products u_b,
 * then the columns summed over b in order. */
int vqmc_ref_sr_apply(const double *O, int64_t ldO, int32_t B, int64_t P, const double *mean,
                      double eps, const double *v, double *out) {
  if (!O || !mean || !v || !out || B < 1 || P < 1 || ldO < P) return -1;
  double *u = (double *)malloc(sizeof(double) * (size_t)B);
#pragma omp parallel for schedule(static)
  for (int b = 0; b < B; ++b) {
    double s = 0.0;
    for (int64_t k = 0; k < P; ++k) s += (O[(size_t)b * ldO + k] - mean[k]) * v[k];
    u[b] = s;
  }
  for (int64_t k = 0; k < P; ++k) out[k] = 0.0;
  for (int b = 0; b < B; ++b) {
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < P; ++k) out[k] += (O[(size_t)b * ldO + k] - mean[k]) * u[b];
  }
  for (int64_t k = 0; k < P; ++k) out[k] = out[k] / B + eps * v[k];
  free(u);
  return 0;
}

int vqmc_ref_sr_matrix(const double *O, int64_t ldO, int32_t B, int64_t P, double *S) {
  if (!O || !S || B < 1 || P < 1 || ldO < P) return -1;
  double *mean = (double *)malloc(sizeof(double) * (size_t)P);
  double *Oc = centred(O, ldO, B, P, mean);
#pragma omp parallel for schedule(dynamic)
  for (int64_t k = 0; k < P; ++k)
    for (int64_t q = 0; q < P; ++q) {
      double s = 0.0;
      for (int b = 0; b < B; ++b) s += Oc[(size_t)b * P + k] * Oc[(size_t)b * P + q];
      S[k * P + q] = s / B;
    }
  free(mean);
  free(Oc);
  return 0;
}

/* SR step of Sec. 3.2.2 with Eqs. (Es-Os-G), (delta), (convar-matrix):
 *   E = <E_s>, G = F = <O E> - <O><E> = (1/B) O^cT E^c,
 *   M = S + eps I with S = (1/B) O^cT O^c,
 *   delta = M^{-1} F by Cholesky and two triangular solves.
 * The sample-space form solves (1/B O^c O^cT + eps I) a = E^c / B and sets
 * delta = O^cT a, which is the same vector (push-through identity). */
int vqmc_ref_sr_solve(const double *O, int64_t ldO, const double *e_loc,
                      int32_t B, int64_t P, double eps, int32_t method,
                      double *delta, double *F, double *e_mean, double *e_var) {
  if (!O || !e_loc || !delta || B < 1 || P < 1 || ldO < P || !(eps >= 0.0)) return -1;
  if (method < 0) method = (P <= B) ? 0 : 1;
  double em = 0.0;
  for (int b = 0; b < B; ++b) em += e_loc[b];
  em /= B;
  double ev = 0.0;
  for (int b = 0; b < B; ++b) ev += (e_loc[b] - em) * (e_loc[b] - em);
  ev /= B;
  if (e_mean) *e_mean = em;
  if (e_var) *e_var = ev;
  double *mean = (double *)malloc(sizeof(double) * (size_t)P);
  double *Oc = centred(O, ldO, B, P, mean);
  double *Ec = (double *)malloc(sizeof(double) * (size_t)B);
  for (int b = 0; b < B; ++b) Ec[b] = e_loc[b] - em;
  double *Fv = (double *)malloc(sizeof(double) * (size_t)P);
  for (int64_t k = 0; k < P; ++k) {
    double s = 0.0;
    for (int b = 0; b < B; ++b) s += Oc[(size_t)b * P + k] * Ec[b];
    Fv[k] = s / B;
  }
  if (F) memcpy(F, Fv, sizeof(double) * (size_t)P);
  int rc = 0;
  if (method == 0) {
    double *S = (double *)malloc(sizeof(double) * (size_t)P * P);
#pragma omp parallel for schedule(dynamic)
    for (int64_t k = 0; k < P; ++k)
      for (int64_t q = 0; q <= k; ++q) {
        double s = 0.0;
        for (int b = 0; b < B; ++b) s += Oc[(size_t)b * P + k] * Oc[(size_t)b * P + q];
        S[k * P + q] = s / B + (k == q ? eps : 0.0);
      }
    rc = cholesky(S, P);
    if (rc == 0) chol_solve(S, P, Fv, delta);
    free(S);
  } else {
    double *K = (double *)malloc(sizeof(double) * (size_t)B * B);
#pragma omp parallel for schedule(dynamic)
    for (int a = 0; a < B; ++a)
      for (int c = 0; c <= a; ++c) {
        double s = 0.0;
        for (int64_t k = 0; k < P; ++k) s += Oc[(size_t)a * P + k] * Oc[(size_t)c * P + k];
        K[(size_t)a * B + c] = s / B + (a == c ? eps : 0.0);
      }
    rc = cholesky(K, B);
    if (rc == 0) {
      double *rhs = (double *)malloc(sizeof(double) * (size_t)B);
      double *alpha = (double *)malloc(sizeof(double) * (size_t)B);
      for (int b = 0; b < B; ++b) rhs[b] = Ec[b] / B;
      chol_solve(K, B, rhs, alpha);
      for (int64_t k = 0; k < P; ++k) {
        double s = 0.0;
        for (int b = 0; b < B; ++b) s += Oc[(size_t)b * P + k] * alpha[b];
        delta[k] = s;
      }
      free(rhs);
      free(alpha);
    }
    free(K);
  }
  free(mean); free(Oc); free(Ec); free(Fv);
  return rc;
}

/* -------------------------------------------------------------- sampler */

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies with the
 * round keys bumped by the Weyl constants between rounds. */
void vqmc_ref_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n1 = (uint32_t)p1;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    const uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The random words of one proposal: counter (t_lo, t_hi, chain, 0) with
 * t = counter_base + sweep*N + step, key (seed_lo, seed_hi). */
static void proposal_words(uint64_t seed, uint64_t t, int chain, uint32_t w[4]) {
  const uint32_t ctr[4] = {(uint32_t)t, (uint32_t)(t >> 32), (uint32_t)chain, 0u};
  const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  vqmc_ref_philox4x32_10(ctr, key, w);
}

static int count_antiparallel_j1(const vqmc_ref_model *m, const int8_t *s) {
  const int N = m->L * m->L;
  int c = 0;
  for (int k = 0; k < 2 * N; ++k) {
    int i, j;
    double J;
    bond(m, k, &i, &j, &J);
    if (s[i] != s[j]) ++c;
  }
  return c;
}

/* Metropolis chain of Sec. 3.1: from the current configuration propose the
 * exchange of the two spins of a J1 bond, evaluate the amplitude of the
 * proposal and accept iff P = (W'/W)^2 >= r with r in (0,1), i.e.
 * 2 (log|W'| - log|W|) >= ln r.  A sweep is N proposals.  r = (u + 1/2)
 * 2^-32 from the second random word; the bond index is floor(u0 * n / 2^32)
 * from the first. */
int vqmc_ref_sample(const vqmc_ref_model *m, const double *theta,
                    int8_t *spins, int32_t B, int32_t n_sweeps, uint64_t seed,
                    uint64_t counter_base, int32_t proposal, double *log_abs,
                    int32_t *n_acc, double *min_margin) {
  if (!model_ok(m) || B < 0 || n_sweeps < 0 || (proposal != 0 && proposal != 1)) return -1;
  if (B > 0 && (!theta || !spins)) return -1;
  const int N = m->L * m->L;
#pragma omp parallel for schedule(dynamic)
  for (int b = 0; b < B; ++b) {
    int8_t *s = spins + (size_t)b * N;
    int8_t *sp = (int8_t *)malloc((size_t)N);
    double lp = amplitude(m, theta, s, NULL, NULL);
    int acc = 0;
    double mm = INFINITY;
    for (int64_t t = 0; t < (int64_t)n_sweeps * N; ++t) {
      uint32_t w[4];
      proposal_words(seed, counter_base + (uint64_t)t, b, w);
      int i = -1, j = -1;
      double J, hastings = 0.0;
      if (proposal == 0) {
        const int k = (int)(((uint64_t)w[0] * (uint64_t)(2 * N)) >> 32);
        bond(m, k, &i, &j, &J);
        if (s[i] == s[j]) continue; /* parallel pair: the move is rejected */
      } else {
        const int nap = count_antiparallel_j1(m, s);
        if (nap == 0) continue;
        int pick = (int)(((uint64_t)w[0] * (uint64_t)nap) >> 32);
        for (int k = 0; k < 2 * N; ++k) {
          int a, c;
          bond(m, k, &a, &c, &J);
          if (s[a] != s[c] && pick-- == 0) { i = a; j = c; break; }
        }
      }
      memcpy(sp, s, (size_t)N);
      sp[i] = s[j];
      sp[j] = s[i];
      if (proposal == 1) hastings = log((double)count_antiparallel_j1(m, s)) -
                                    log((double)count_antiparallel_j1(m, sp));
      const double lpn = amplitude(m, theta, sp, NULL, NULL);
      const double r = ((double)w[1] + 0.5) * (1.0 / 4294967296.0);
      const double a = 2.0 * (lpn - lp) + hastings - log(r);
      if (fabs(a) < mm) mm = fabs(a);
      if (a >= 0.0) {
        memcpy(s, sp, (size_t)N);
        lp = lpn;
        ++acc;
      }
    }
    if (log_abs) log_abs[b] = lp;
    if (n_acc) n_acc[b] = acc;
    if (min_margin) min_margin[b] = mm;
    free(sp);
  }
  return 0;
}
