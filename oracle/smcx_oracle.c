/*
 * Plain FP64 CPU oracle for the population likelihood of a transdimensional
 * SMC sampler (Demasi & Del Pozzo, "Massively parallel transdimensional
 * sampling with data assimilation").
 *
 * TEST INFRASTRUCTURE ONLY. This file is the checker, not the product: only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load it. It shares no code, header, table or helper with the GPU
 * library. Every quantity is the plain definition, written out in double
 * precision and summed in index order; there is no blocking, fusion or
 * reordering. OpenMP only distributes whole particles over threads, so the
 * result of a particle does not depend on the thread count.
 *
 * Conventions (readings of the paper, stated once here):
 *  - sample times are t_s = t_start + s*dt, s = 0..T-1;
 *  - a particle is (K, theta_K) in the disjoint union over K of the
 *    K-component parameter spaces (Sec. "Reversible Jump MCMC"), stored as
 *    CSR rows: components of particle i are rows offsets[i]..offsets[i+1]-1
 *    of theta[M][P];
 *  - the residual is r_s = d_s - (h_0(t_s) + h_1(t_s) + ... + h_{K-1}(t_s)),
 *    the template sum accumulated left to right;
 *  - log L = -(1/(2 sigma^2)) sum_s r_s^2 for white noise of standard
 *    deviation sigma (the time-domain form of the noise-weighted inner
 *    product, eq. gw_likelihood with a uniform PSD); the constant
 *    -(T/2) log(2 pi sigma^2) is dropped;
 *  - every per-particle output is tempered: the tempered bridge
 *    (eq. prior_bridge) raises L to beta, so outputs are beta * (.).
 *
 * Models:
 *  - MODEL_PULSE (P=3, theta = A, t0, w):
 *        h(t) = A exp(-(t - t0)^2 / (2 w^2))           (Sec. Gaussian pulses)
 *    w is read as a standard deviation.
 *  - MODEL_GBSINE (P=4, theta = A', f0, fdot, phi0):
 *        h(t) = A' sin(2 pi f0 t + pi fdot t^2 + phi0)
 *    a single-channel, time-domain stand-in for the Galactic-binary signal
 *    of Sec. "LISA Galactic binaries" (parameters f0, fdot, A, phi0 of the
 *    source list there; sky position, polarisation and inclination are not
 *    modelled).
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#include <omp.h>

#define MODEL_PULSE 0
#define MODEL_GBSINE 1

#define OR_OK 0
#define OR_EINVAL (-1)

static const double TWO_PI = 6.283185307179586476925286766559;
static const double PI = 3.141592653589793238462643383279;

int oracle_n_params(int model) {
  if (model == MODEL_PULSE) return 3;
  if (model == MODEL_GBSINE) return 4;
  if (model == 2) return 8; /* the frequency-domain Galactic binaries (gblisa_oracle.c) */
  return -1;
}

void oracle_set_threads(int n) { if (n > 0) omp_set_num_threads(n); }
int oracle_get_threads(void) { return omp_get_max_threads(); }

/* One component template h(t) (model definitions above). */
static double template_value(int model, const double* th, double t) {
  if (model == MODEL_PULSE) {
    double A = th[0], t0 = th[1], w = th[2];
    double x = t - t0;
    return A * exp(-(x * x) / (2.0 * w * w));
  } else {
    double A = th[0], f0 = th[1], fdot = th[2], phi0 = th[3];
    double phase = TWO_PI * f0 * t + PI * fdot * t * t + phi0;
    return A * sin(phase);
  }
}

/* Analytic partial derivatives dh/dtheta_p of one template at time t.
 * Pulse:  dh/dA = e, dh/dt0 = A e x / w^2, dh/dw = A e x^2 / w^3 with
 *         e = exp(-x^2/(2w^2)), x = t - t0.
 * GB:     dh/dA' = sin(Phi), dh/df0 = 2 pi t A' cos(Phi),
 *         dh/dfdot = pi t^2 A' cos(Phi), dh/dphi0 = A' cos(Phi). */
static void template_partials(int model, const double* th, double t, double* dh) {
  if (model == MODEL_PULSE) {
    double A = th[0], t0 = th[1], w = th[2];
    double x = t - t0;
    double e = exp(-(x * x) / (2.0 * w * w));
    dh[0] = e;
    dh[1] = A * e * x / (w * w);
    dh[2] = A * e * x * x / (w * w * w);
  } else {
    double A = th[0], f0 = th[1], fdot = th[2], phi0 = th[3];
    double phase = TWO_PI * f0 * t + PI * fdot * t * t + phi0;
    double s = sin(phase), c = cos(phase);
    dh[0] = s;
    dh[1] = TWO_PI * t * A * c;
    dh[2] = PI * t * t * A * c;
    dh[3] = A * c;
  }
}

/* Sum of K templates at every sample: out[s] = sum_k h_k(t_s). */
int oracle_template_sum(int model, int64_t K, const double* theta, int64_t T, double t_start,
                        double dt, double* out) {
  int P = oracle_n_params(model);
  if (P < 0 || K < 0 || T < 0 || (K > 0 && !theta) || (T > 0 && !out)) return OR_EINVAL;
  for (int64_t s = 0; s < T; ++s) {
    double t = t_start + (double)s * dt;
    double hs = 0.0;
    for (int64_t k = 0; k < K; ++k) hs += template_value(model, theta + k * P, t);
    out[s] = hs;
  }
  return OR_OK;
}

static int check_population(int model, int64_t N, const int64_t* offsets, const double* theta) {
  if (oracle_n_params(model) < 0 || N < 0 || (N > 0 && !offsets)) return OR_EINVAL;
  if (N == 0) return OR_OK;
  if (offsets[0] != 0) return OR_EINVAL;
  for (int64_t i = 0; i < N; ++i)
    if (offsets[i + 1] < offsets[i]) return OR_EINVAL;
  if (offsets[N] > 0 && !theta) return OR_EINVAL;
  return OR_OK;
}

/* Residual at sample s for the components of one particle, skipping the
 * component with local index `skip` (pass -1 to skip none). */
static double residual_at(int model, const double* d, double t_start, double dt, int64_t s,
                          int64_t K, const double* th, int P, int64_t skip) {
  double t = t_start + (double)s * dt;
  double hs = 0.0;
  for (int64_t k = 0; k < K; ++k)
    if (k != skip) hs += template_value(model, th + k * P, t);
  return d[s] - hs;
}

/* Tempered log-likelihood of every particle (eq. prior_bridge applied to
 * the white-noise likelihood of eq. gw_likelihood). */
int oracle_logl(int model, const double* d, int64_t T, double t_start, double dt, double sigma,
                int64_t N, const int64_t* offsets, const double* theta, const double* beta,
                double* logl) {
  if (check_population(model, N, offsets, theta) != OR_OK || T < 0 || (T > 0 && !d) ||
      (N > 0 && !logl))
    return OR_EINVAL;
  int P = oracle_n_params(model);
#pragma omp parallel for schedule(dynamic)
  for (int64_t i = 0; i < N; ++i) {
    int64_t K = offsets[i + 1] - offsets[i];
    const double* th = theta ? theta + offsets[i] * P : NULL;
    double ss = 0.0;
    for (int64_t s = 0; s < T; ++s) {
      double r = residual_at(model, d, t_start, dt, s, K, th, P, -1);
      ss += r * r;
    }
    double b = beta ? beta[i] : 1.0;
    logl[i] = b * (-0.5 * ss / (sigma * sigma));
  }
  return OR_OK;
}

/* Tempered log-likelihood and gradient of one particle (K components th). */
static void particle_logl_grad(int model, const double* d, int64_t T, double t_start, double dt,
                               double sigma, int64_t K, const double* th, double b, double* logl,
                               double* g) {
  int P = oracle_n_params(model);
  double ss = 0.0;
  for (int64_t k = 0; k < K * P; ++k) g[k] = 0.0;
  for (int64_t s = 0; s < T; ++s) {
    double r = residual_at(model, d, t_start, dt, s, K, th, P, -1);
    ss += r * r;
    double t = t_start + (double)s * dt;
    for (int64_t k = 0; k < K; ++k) {
      double dh[4];
      template_partials(model, th + k * P, t, dh);
      for (int p = 0; p < P; ++p) g[k * P + p] += r * dh[p];
    }
  }
  for (int64_t k = 0; k < K * P; ++k) g[k] = b * (g[k] / (sigma * sigma));
  *logl = b * (-0.5 * ss / (sigma * sigma));
}

/* Tempered log-likelihood and its gradient with respect to every component
 * parameter: grad[m][p] = beta * (1/sigma^2) sum_s r_s dh_m(t_s)/dtheta_p.
 * The gradient is what the NUTS kernel of Sec. "No-U-Turn-Sampler" needs
 * (Hamilton's equations use the gradient of the potential). `logl` may be
 * NULL. */
int oracle_logl_grad(int model, const double* d, int64_t T, double t_start, double dt,
                     double sigma, int64_t N, const int64_t* offsets, const double* theta,
                     const double* beta, double* logl, double* grad) {
  if (check_population(model, N, offsets, theta) != OR_OK || T < 0 || (T > 0 && !d))
    return OR_EINVAL;
  if (N > 0 && offsets[N] > 0 && !grad) return OR_EINVAL;
  int P = oracle_n_params(model);
#pragma omp parallel for schedule(dynamic)
  for (int64_t i = 0; i < N; ++i) {
    int64_t K = offsets[i + 1] - offsets[i];
    const double* th = theta ? theta + offsets[i] * P : NULL;
    double* g = grad ? grad + offsets[i] * P : NULL;
    double b = beta ? beta[i] : 1.0;
    double ss = 0.0;
    for (int64_t k = 0; k < K * P; ++k) g[k] = 0.0;
    for (int64_t s = 0; s < T; ++s) {
      double r = residual_at(model, d, t_start, dt, s, K, th, P, -1);
      ss += r * r;
      double t = t_start + (double)s * dt;
      for (int64_t k = 0; k < K; ++k) {
        double dh[4];
        template_partials(model, th + k * P, t, dh);
        for (int p = 0; p < P; ++p) g[k * P + p] += r * dh[p];
      }
    }
    for (int64_t k = 0; k < K * P; ++k) g[k] = b * (g[k] / (sigma * sigma));
    if (logl) logl[i] = b * (-0.5 * ss / (sigma * sigma));
  }
  return OR_OK;
}

/* ---- posterior-start bridge (eq. reuse_bridge) ----
 * For white noise the likelihood factorises over samples, so the bridge
 * p(theta|d1) (p(theta|d2)/p(theta|d1))^beta between the posterior on the
 * first `split` samples (d1) and the posterior on all T samples (d2) has the
 * log-likelihood part
 *   logL_split = -(1/(2 sigma^2)) [ sum_{s<split} r_s^2 + beta sum_{s>=split} r_s^2 ]
 * i.e. samples before the split enter untempered and the later ones tempered
 * by beta. split = 0 is the prior bridge (eq. prior_bridge), split = T the
 * untempered posterior. The functions below are the tempered ones above
 * with that per-sample weight. */
static double sample_weight(int64_t s, int64_t split, double b) { return s < split ? 1.0 : b; }

int oracle_logl_split(int model, const double* d, int64_t T, double t_start, double dt,
                      double sigma, int64_t N, const int64_t* offsets, const double* theta,
                      const double* beta, int64_t split, double* logl) {
  if (check_population(model, N, offsets, theta) != OR_OK || T < 0 || (T > 0 && !d) ||
      (N > 0 && !logl) || split < 0)
    return OR_EINVAL;
  int P = oracle_n_params(model);
#pragma omp parallel for schedule(dynamic)
  for (int64_t i = 0; i < N; ++i) {
    int64_t K = offsets[i + 1] - offsets[i];
    const double* th = theta ? theta + offsets[i] * P : NULL;
    double b = beta ? beta[i] : 1.0;
    double ss = 0.0;
    for (int64_t s = 0; s < T; ++s) {
      double r = residual_at(model, d, t_start, dt, s, K, th, P, -1);
      ss += sample_weight(s, split, b) * (r * r);
    }
    logl[i] = -0.5 * ss / (sigma * sigma);
  }
  return OR_OK;
}

static void particle_logl_grad_split(int model, const double* d, int64_t T, double t_start,
                                     double dt, double sigma, int64_t K, const double* th,
                                     double b, int64_t split, double* logl, double* g) {
  int P = oracle_n_params(model);
  double ss = 0.0;
  for (int64_t k = 0; k < K * P; ++k) g[k] = 0.0;
  for (int64_t s = 0; s < T; ++s) {
    double r = residual_at(model, d, t_start, dt, s, K, th, P, -1);
    double ws = sample_weight(s, split, b);
    ss += ws * (r * r);
    double t = t_start + (double)s * dt;
    for (int64_t k = 0; k < K; ++k) {
      double dh[4];
      template_partials(model, th + k * P, t, dh);
      for (int p = 0; p < P; ++p) g[k * P + p] += ws * (r * dh[p]);
    }
  }
  for (int64_t k = 0; k < K * P; ++k) g[k] = g[k] / (sigma * sigma);
  *logl = -0.5 * ss / (sigma * sigma);
}

int oracle_logl_grad_split(int model, const double* d, int64_t T, double t_start, double dt,
                           double sigma, int64_t N, const int64_t* offsets, const double* theta,
                           const double* beta, int64_t split, double* logl, double* grad) {
  if (check_population(model, N, offsets, theta) != OR_OK || T < 0 || (T > 0 && !d) ||
      split < 0)
    return OR_EINVAL;
  if (N > 0 && offsets[N] > 0 && !grad) return OR_EINVAL;
  int P = oracle_n_params(model);
#pragma omp parallel for schedule(dynamic)
  for (int64_t i = 0; i < N; ++i) {
    int64_t K = offsets[i + 1] - offsets[i];
    const double* th = theta ? theta + offsets[i] * P : NULL;
    double l;
    particle_logl_grad_split(model, d, T, t_start, dt, sigma, K, th, beta ? beta[i] : 1.0, split,
                             &l, grad ? grad + offsets[i] * P : NULL);
    if (logl) logl[i] = l;
  }
  return OR_OK;
}

/* Birth/death changes of logL_split: the inner products of
 * oracle_delta_logl_birth_death with the per-sample weight. */
int oracle_delta_split(int model, const double* d, int64_t T, double t_start, double dt,
                       double sigma, int64_t N, const int64_t* offsets, const double* theta,
                       const double* beta, const double* theta_birth, const int32_t* death_idx,
                       int64_t split, double* d_birth, double* d_death) {
  if (check_population(model, N, offsets, theta) != OR_OK || T < 0 || (T > 0 && !d) ||
      split < 0)
    return OR_EINVAL;
  if (N > 0 && ((theta_birth && !d_birth) || (death_idx && !d_death))) return OR_EINVAL;
  for (int64_t i = 0; death_idx && i < N; ++i) {
    int64_t K = offsets[i + 1] - offsets[i];
    if (death_idx[i] < -1 || death_idx[i] >= K) return OR_EINVAL;
  }
  int P = oracle_n_params(model);
#pragma omp parallel for schedule(dynamic)
  for (int64_t i = 0; i < N; ++i) {
    int64_t K = offsets[i + 1] - offsets[i];
    const double* th = theta ? theta + offsets[i] * P : NULL;
    double b = beta ? beta[i] : 1.0;
    if (theta_birth) {
      const double* tb = theta_birth + i * P;
      double x = 0.0, y = 0.0;
      for (int64_t s = 0; s < T; ++s) {
        double r = residual_at(model, d, t_start, dt, s, K, th, P, -1);
        double h = template_value(model, tb, t_start + (double)s * dt);
        double ws = sample_weight(s, split, b);
        x += ws * (r * h);
        y += ws * (h * h);
      }
      d_birth[i] = (x - 0.5 * y) / (sigma * sigma);
    }
    if (death_idx) {
      int64_t j = death_idx[i];
      if (j < 0) {
        d_death[i] = 0.0;
      } else {
        double x = 0.0, y = 0.0;
        for (int64_t s = 0; s < T; ++s) {
          double r = residual_at(model, d, t_start, dt, s, K, th, P, j);
          double h = template_value(model, th + j * P, t_start + (double)s * dt);
          double ws = sample_weight(s, split, b);
          x += ws * (r * h);
          y += ws * (h * h);
        }
        d_death[i] = -((x - 0.5 * y) / (sigma * sigma));
      }
    }
  }
  return OR_OK;
}

/* Change of tempered log-likelihood for the nested birth/death moves of
 * Sec. "Reversible Jump MCMC" (k' = k +- 1, unit Jacobian):
 *   birth of theta_new appended at index K:
 *     D_birth = beta [ <r, h_new> - 0.5 <h_new, h_new> ] / sigma^2
 *   death of local index j:
 *     D_death = -beta [ <r_not_j, h_j> - 0.5 <h_j, h_j> ] / sigma^2
 * where r is the residual of the current particle and r_not_j the residual
 * with component j left out of the index-order sum. Both follow from
 * expanding -|r'|^2/(2 sigma^2) + |r|^2/(2 sigma^2). death_idx[i] = -1
 * gives D_death = 0; theta_birth or death_idx may be NULL (that output is
 * then not written). */
int oracle_delta_logl_birth_death(int model, const double* d, int64_t T, double t_start,
                                  double dt, double sigma, int64_t N, const int64_t* offsets,
                                  const double* theta, const double* beta,
                                  const double* theta_birth, const int32_t* death_idx,
                                  double* d_birth, double* d_death) {
  if (check_population(model, N, offsets, theta) != OR_OK || T < 0 || (T > 0 && !d))
    return OR_EINVAL;
  if (N > 0 && ((theta_birth && !d_birth) || (death_idx && !d_death))) return OR_EINVAL;
  for (int64_t i = 0; death_idx && i < N; ++i) {
    int64_t K = offsets[i + 1] - offsets[i];
    if (death_idx[i] < -1 || death_idx[i] >= K) return OR_EINVAL;
  }
  int P = oracle_n_params(model);
#pragma omp parallel for schedule(dynamic)
  for (int64_t i = 0; i < N; ++i) {
    int64_t K = offsets[i + 1] - offsets[i];
    const double* th = theta ? theta + offsets[i] * P : NULL;
    double b = beta ? beta[i] : 1.0;
    if (theta_birth) {
      const double* tb = theta_birth + i * P;
      double x = 0.0, y = 0.0;
      for (int64_t s = 0; s < T; ++s) {
        double r = residual_at(model, d, t_start, dt, s, K, th, P, -1);
        double h = template_value(model, tb, t_start + (double)s * dt);
        x += r * h;
        y += h * h;
      }
      d_birth[i] = b * (x - 0.5 * y) / (sigma * sigma);
    }
    if (death_idx) {
      int64_t j = death_idx[i];
      if (j < 0) {
        d_death[i] = 0.0;
      } else {
        double x = 0.0, y = 0.0;
        for (int64_t s = 0; s < T; ++s) {
          double r = residual_at(model, d, t_start, dt, s, K, th, P, j);
          double h = template_value(model, th + j * P, t_start + (double)s * dt);
          x += r * h;
          y += h * h;
        }
        d_death[i] = -(b * (x - 0.5 * y) / (sigma * sigma));
      }
    }
  }
  return OR_OK;
}

/* Data-assimilation reweighting (eq. reuse_bridge with the incremental
 * weight of eq. incremental_weight, the ESS of eq. ess and the evidence
 * ratio Z_t/Z_{t-1} of Sec. "Sequential Monte Carlo").
 *
 * For white noise the likelihood factorises over samples, so the ratio
 * p(theta|d2)/p(theta|d1) of eq. reuse_bridge equals, up to a constant,
 * exp(logl_ext) with logl_ext the untempered log-likelihood of the new
 * samples [T1, T2) only:
 *   logl_ext_i = -(1/(2 sigma^2)) sum_{s=T1}^{T2-1} r_s^2
 * (templates at the absolute times t_s of the longer segment d, which has
 * T2 samples). Raising the ratio to beta and stepping beta by delta_beta
 * gives the log incremental weight
 *   logw_i = logw_prev_i + delta_beta * logl_ext_i
 * (logw_prev = 0 when NULL, i.e. uniform previous weights). Then, with
 * m = max_i logw_i:
 *   w_norm_i = exp(logw_i - m) / sum_j exp(logw_j - m)
 *   ESS = (sum w)^2 / sum w^2 = 1 / sum_i w_norm_i^2
 *   logZ increment = log sum_i exp(logw_i) - log sum_i exp(logw_prev_i)
 *                  (= ... - log N for uniform previous weights).
 * scalars = {ESS, logZ increment, m}. N = 0 gives {0, 0, -inf}. */
int oracle_reweight_extend(int model, const double* d, double t_start, double dt, double sigma,
                           int64_t T1, int64_t T2, int64_t N, const int64_t* offsets,
                           const double* theta, double delta_beta, const double* logw_prev,
                           double* logl_ext, double* logw, double* w_norm, double* scalars) {
  if (check_population(model, N, offsets, theta) != OR_OK || T1 < 0 || T2 < T1 ||
      (T2 > 0 && !d) || !scalars)
    return OR_EINVAL;
  if (N > 0 && (!logl_ext || !logw || !w_norm)) return OR_EINVAL;
  int P = oracle_n_params(model);
#pragma omp parallel for schedule(dynamic)
  for (int64_t i = 0; i < N; ++i) {
    int64_t K = offsets[i + 1] - offsets[i];
    const double* th = theta ? theta + offsets[i] * P : NULL;
    double ss = 0.0;
    for (int64_t s = T1; s < T2; ++s) {
      double r = residual_at(model, d, t_start, dt, s, K, th, P, -1);
      ss += r * r;
    }
    logl_ext[i] = -0.5 * ss / (sigma * sigma);
  }
  if (N == 0) {
    scalars[0] = 0.0;
    scalars[1] = 0.0;
    scalars[2] = -INFINITY;
    return OR_OK;
  }
  double m = -INFINITY;
  for (int64_t i = 0; i < N; ++i) {
    logw[i] = (logw_prev ? logw_prev[i] : 0.0) + delta_beta * logl_ext[i];
    if (logw[i] > m) m = logw[i];
  }
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    double e = exp(logw[i] - m);
    s1 += e;
    s2 += e * e;
  }
  for (int64_t i = 0; i < N; ++i) w_norm[i] = exp(logw[i] - m) / s1;
  double lse_prev;
  if (logw_prev) {
    double mp = -INFINITY, sp = 0.0;
    for (int64_t i = 0; i < N; ++i)
      if (logw_prev[i] > mp) mp = logw_prev[i];
    for (int64_t i = 0; i < N; ++i) sp += exp(logw_prev[i] - mp);
    lse_prev = mp + log(sp);
  } else {
    lse_prev = log((double)N);
  }
  scalars[0] = s1 * s1 / s2;
  scalars[1] = m + log(s1) - lse_prev;
  scalars[2] = m;
  return OR_OK;
}

/* One leapfrog step of Hamiltonian dynamics (Sec. "No-U-Turn-Sampler"),
 * H = -log p(theta) + 0.5 r^T r with an identity mass matrix, for the
 * tempered target whose log density is beta * logL (uniform prior: zero
 * gradient inside its box):
 *   p_half = p + (eps/2) grad(beta logL)(q)
 *   q'     = q + eps p_half
 *   p'     = p_half + (eps/2) grad(beta logL)(q')
 * Particles with active[i] == 0 (active may be NULL = all active) are copied
 * unchanged. Outputs q', p' and the tempered logL and gradient at q'. */
/* Population gradient of the tempered target: the prior bridge when
 * split == 0, the posterior-start bridge otherwise. */
static int target_logl_grad(int model, const double* d, int64_t T, double t_start, double dt,
                            double sigma, int64_t N, const int64_t* offsets, const double* q,
                            const double* beta, int64_t split, double* logl, double* grad) {
  if (split == 0)
    return oracle_logl_grad(model, d, T, t_start, dt, sigma, N, offsets, q, beta, logl, grad);
  return oracle_logl_grad_split(model, d, T, t_start, dt, sigma, N, offsets, q, beta, split, logl,
                                grad);
}

static int leapfrog_impl(int model, const double* d, int64_t T, double t_start, double dt,
                         double sigma, int64_t N, const int64_t* offsets, const double* q,
                         const double* p, const double* beta, double eps, const uint8_t* active,
                         int64_t split, double* q_out, double* p_out, double* logl_out,
                         double* grad_out) {
  if (check_population(model, N, offsets, q) != OR_OK || T < 0 || (T > 0 && !d)) return OR_EINVAL;
  int64_t M = N > 0 ? offsets[N] : 0;
  if (M > 0 && (!p || !q_out || !p_out || !grad_out)) return OR_EINVAL;
  if (N > 0 && !logl_out) return OR_EINVAL;
  int P = oracle_n_params(model);
  /* gradient at the start point, into grad_out as scratch */
  int rc = target_logl_grad(model, d, T, t_start, dt, sigma, N, offsets, q, beta, split, logl_out,
                            grad_out);
  if (rc != OR_OK) return rc;
  for (int64_t i = 0; i < N; ++i) {
    int on = active ? active[i] != 0 : 1;
    for (int64_t m = offsets[i] * P; m < offsets[i + 1] * P; ++m) {
      if (on) {
        double ph = p[m] + 0.5 * eps * grad_out[m];
        p_out[m] = ph;
        q_out[m] = q[m] + eps * ph;
      } else {
        p_out[m] = p[m];
        q_out[m] = q[m];
      }
    }
  }
  rc = target_logl_grad(model, d, T, t_start, dt, sigma, N, offsets, q_out, beta, split, logl_out,
                        grad_out);
  if (rc != OR_OK) return rc;
  for (int64_t i = 0; i < N; ++i) {
    int on = active ? active[i] != 0 : 1;
    if (!on) continue;
    for (int64_t m = offsets[i] * P; m < offsets[i + 1] * P; ++m)
      p_out[m] = p_out[m] + 0.5 * eps * grad_out[m];
  }
  return OR_OK;
}

int oracle_leapfrog(int model, const double* d, int64_t T, double t_start, double dt,
                    double sigma, int64_t N, const int64_t* offsets, const double* q,
                    const double* p, const double* beta, double eps, const uint8_t* active,
                    double* q_out, double* p_out, double* logl_out, double* grad_out) {
  return leapfrog_impl(model, d, T, t_start, dt, sigma, N, offsets, q, p, beta, eps, active, 0,
                       q_out, p_out, logl_out, grad_out);
}

/* The leapfrog step for the posterior-start bridge target (split > 0). */
int oracle_leapfrog_split(int model, const double* d, int64_t T, double t_start, double dt,
                          double sigma, int64_t N, const int64_t* offsets, const double* q,
                          const double* p, const double* beta, double eps, const uint8_t* active,
                          int64_t split, double* q_out, double* p_out, double* logl_out,
                          double* grad_out) {
  if (split < 0) return OR_EINVAL;
  return leapfrog_impl(model, d, T, t_start, dt, sigma, N, offsets, q, p, beta, eps, active, split,
                       q_out, p_out, logl_out, grad_out);
}

/* One No-U-Turn transition per particle (Sec. "No-U-Turn-Sampler"; the
 * stopping rule of Hoffman & Gelman, in its multinomial form). Reading used
 * here, written out step by step:
 *  - potential U = -beta logL inside the uniform prior box, +inf outside;
 *    H = U + |p|^2 / 2 (identity metric); the momentum is an input draw;
 *  - the trajectory grows by doublings j = 0, 1, ..., max_depth - 1 in
 *    direction dirs[j]; doubling j adds 2^j leapfrog steps (oracle_leapfrog's
 *    arithmetic) continuing from the trajectory end on that side;
 *  - leaf n of doubling j replaces the subtree's proposal with probability
 *    exp(-H_n) / (sum of exp(-H) over the subtree's leaves so far), decided
 *    by u_leaf[2^j - 1 + n] < that probability;
 *  - a leaf with H_n - H_0 > 1000 (or outside the box) is a divergence;
 *  - every block of 2^m consecutive leaves of the subtree (m = 1..j, aligned
 *    to the subtree start) is tested when it completes: with rho the sum of
 *    the block's momenta and p_a, p_b its first and last momenta, it has
 *    turned if rho.p_a <= 0 or rho.p_b <= 0;
 *  - a divergence or turn inside the subtree discards the subtree and ends
 *    the transition; otherwise the subtree's proposal replaces the
 *    trajectory's with probability min(1, W_sub / W_traj) (u_tree[j]), the
 *    weights and momentum sums are merged, and the whole trajectory is
 *    tested the same way (end momenta p_left, p_right);
 *  - the transition ends after max_depth doublings at the latest.
 * Outputs: the proposal's position, tempered logL and gradient; depth = the
 * number of completed doublings; steps = leapfrog steps taken; status 0 (no
 * components), 1 (U-turn), 2 (divergence), 3 (maximum depth). */
static double dot(const double* a, const double* b, int64_t n) {
  double s = 0.0;
  for (int64_t x = 0; x < n; ++x) s += a[x] * b[x];
  return s;
}
/* y = W v (trans == 0) or W^T v (trans == 1) for an n x n row-major W */
static void matvec(const double* W, int64_t n, int trans, const double* v, double* y) {
  for (int64_t a = 0; a < n; ++a) {
    double s = 0.0;
    for (int64_t c = 0; c < n; ++c) s += (trans ? W[c * n + a] : W[a * n + c]) * v[c];
    y[a] = s;
  }
}
static double logaddexp(double a, double b) {
  double m = a > b ? a : b;
  if (m == -INFINITY) return -INFINITY;
  return m + log(exp(a - m) + exp(b - m));
}
static int inside_box(const double* q, int64_t n, int P, const double* lo, const double* hi) {
  if (!lo) return 1;
  for (int64_t x = 0; x < n; ++x)
    if (!(q[x] >= lo[x % P] && q[x] <= hi[x % P])) return 0;
  return 1;
}

#include <stdlib.h>
#include <string.h>

static int nuts_impl(int model, const double* d, int64_t T, double t_start, double dt,
                     double sigma, int64_t N, const int64_t* offsets, const double* beta,
                     double eps, int max_depth, const double* prior_lo, const double* prior_hi,
                     const double* momentum, const int8_t* dirs, const double* u_leaf,
                     const double* u_tree, int64_t split, const int64_t* w_off, const double* W,
                     double* q, double* logl, double* grad, int32_t* depth_out,
                     int32_t* steps_out, int32_t* status_out) {
  if (check_population(model, N, offsets, q) != OR_OK || max_depth < 1 || max_depth > 16)
    return OR_EINVAL;
  int P = oracle_n_params(model);
  if (W) {
    if (!w_off) return OR_EINVAL;
    for (int64_t i = 0; i < N; ++i) {
      int64_t n = (offsets[i + 1] - offsets[i]) * P;
      if (w_off[i + 1] - w_off[i] != n * n || w_off[i] < 0) return OR_EINVAL;
    }
  }
  int64_t nleaf = ((int64_t)1 << max_depth) - 1;
#pragma omp parallel for schedule(dynamic)
  for (int64_t i = 0; i < N; ++i) {
    int64_t K = offsets[i + 1] - offsets[i];
    int64_t n = K * P;
    double* qi = q + offsets[i] * P;
    double* gi = grad + offsets[i] * P;
    double b = beta ? beta[i] : 1.0;
    int depth = 0, steps = 0, status = 0;
    if (n == 0) {
      depth_out[i] = 0; steps_out[i] = 0; status_out[i] = 0;
      continue;
    }
    /* 16 + 2*max_depth state vectors of n doubles */
    double* buf = (double*)calloc((size_t)(16 + 2 * max_depth) * n, sizeof(double));
    double *qL = buf, *pL = buf + n, *gL = buf + 2 * n, *qR = buf + 3 * n, *pR = buf + 4 * n,
           *gR = buf + 5 * n, *qF = buf + 6 * n, *pF = buf + 7 * n, *gF = buf + 8 * n,
           *qP = buf + 9 * n, *gP = buf + 10 * n, *qS = buf + 11 * n, *gS = buf + 12 * n,
           *rhoT = buf + 13 * n, *rhoS = buf + 14 * n, *tmp = buf + 15 * n;
    double* ckP = buf + 16 * n;                 /* [max_depth][n] */
    double* ckR = buf + (16 + max_depth) * n;  /* [max_depth][n] */
    const double* Wi = W ? W + w_off[i] : NULL;
    double* wv = W ? (double*)malloc((size_t)n * sizeof(double)) : NULL;
    const double* p0 = momentum + offsets[i] * P;
    double l0 = logl[i];
    double H0 = -l0 + 0.5 * dot(p0, p0, n);
    for (int64_t x = 0; x < n; ++x) {
      qL[x] = qR[x] = qP[x] = qi[x];
      pL[x] = pR[x] = rhoT[x] = p0[x];
      gL[x] = gR[x] = gP[x] = gi[x];
    }
    double lL = l0, lR = l0, lP = l0, lS = l0, lF = l0;
    double lw_tree = -H0;
    if (!inside_box(qi, n, P, prior_lo, prior_hi) || !isfinite(H0)) {
      status = 2;
    } else {
      status = 3;
      for (int j = 0; j < max_depth; ++j) {
        int v = dirs[i * max_depth + j];
        double e = eps * (double)v;
        memcpy(qF, v > 0 ? qR : qL, n * sizeof(double));
        memcpy(pF, v > 0 ? pR : pL, n * sizeof(double));
        memcpy(gF, v > 0 ? gR : gL, n * sizeof(double));
        lF = v > 0 ? lR : lL;
        double lw_sub = -INFINITY;
        for (int64_t x = 0; x < n; ++x) rhoS[x] = 0.0;
        int stop = 0;
        for (int64_t leaf = 0; leaf < ((int64_t)1 << j); ++leaf) {
          /* leapfrog step from the frontier; with a metric the momentum is
           * the whitened one: kicks by W grad, drift by W^T p */
          if (!Wi) {
            for (int64_t x = 0; x < n; ++x) {
              pF[x] = pF[x] + 0.5 * e * gF[x];
              qF[x] = qF[x] + e * pF[x];
            }
          } else {
            matvec(Wi, n, 0, gF, wv);
            for (int64_t x = 0; x < n; ++x) pF[x] = pF[x] + 0.5 * e * wv[x];
            matvec(Wi, n, 1, pF, wv);
            for (int64_t x = 0; x < n; ++x) qF[x] = qF[x] + e * wv[x];
          }
          if (split == 0)
            particle_logl_grad(model, d, T, t_start, dt, sigma, K, qF, b, &lF, gF);
          else
            particle_logl_grad_split(model, d, T, t_start, dt, sigma, K, qF, b, split, &lF, gF);
          if (Wi) matvec(Wi, n, 0, gF, wv);
          for (int64_t x = 0; x < n; ++x) pF[x] = pF[x] + 0.5 * e * (Wi ? wv[x] : gF[x]);
          steps += 1;
          double H = inside_box(qF, n, P, prior_lo, prior_hi) ? -lF + 0.5 * dot(pF, pF, n)
                                                              : INFINITY;
          if (!(H - H0 <= 1000.0)) { status = 2; stop = 1; break; }
          double lws = logaddexp(lw_sub, -H);
          if (u_leaf[i * nleaf + ((int64_t)1 << j) - 1 + leaf] < exp(-H - lws)) {
            memcpy(qS, qF, n * sizeof(double));
            memcpy(gS, gF, n * sizeof(double));
            lS = lF;
          }
          lw_sub = lws;
          for (int64_t x = 0; x < n; ++x) tmp[x] = rhoS[x];
          for (int64_t x = 0; x < n; ++x) rhoS[x] += pF[x];
          for (int m = 1; m <= j; ++m) {
            if (leaf % ((int64_t)1 << m) != 0) break;
            memcpy(ckP + (m - 1) * n, pF, n * sizeof(double));
            memcpy(ckR + (m - 1) * n, tmp, n * sizeof(double));
          }
          int turn = 0;
          for (int m = 1; m <= j && !turn; ++m) {
            if ((leaf + 1) % ((int64_t)1 << m) != 0) break;
            double dl = 0.0, dr = 0.0;
            for (int64_t x = 0; x < n; ++x) {
              double rb = rhoS[x] - ckR[(m - 1) * n + x];
              dl += rb * ckP[(m - 1) * n + x];
              dr += rb * pF[x];
            }
            turn = dl <= 0.0 || dr <= 0.0;
          }
          if (turn) { status = 1; stop = 1; break; }
        }
        if (stop) break;
        if (u_tree[i * max_depth + j] < exp(lw_sub - lw_tree)) {
          memcpy(qP, qS, n * sizeof(double));
          memcpy(gP, gS, n * sizeof(double));
          lP = lS;
        }
        lw_tree = logaddexp(lw_tree, lw_sub);
        for (int64_t x = 0; x < n; ++x) rhoT[x] += rhoS[x];
        if (v > 0) {
          memcpy(qR, qF, n * sizeof(double)); memcpy(pR, pF, n * sizeof(double));
          memcpy(gR, gF, n * sizeof(double)); lR = lF;
        } else {
          memcpy(qL, qF, n * sizeof(double)); memcpy(pL, pF, n * sizeof(double));
          memcpy(gL, gF, n * sizeof(double)); lL = lF;
        }
        depth = j + 1;
        if (dot(rhoT, pL, n) <= 0.0 || dot(rhoT, pR, n) <= 0.0) { status = 1; break; }
      }
    }
    memcpy(qi, qP, n * sizeof(double));
    memcpy(gi, gP, n * sizeof(double));
    logl[i] = lP;
    depth_out[i] = depth;
    steps_out[i] = steps;
    status_out[i] = status;
    free(buf);
    free(wv);
  }
  return OR_OK;
}

int oracle_nuts_transition(int model, const double* d, int64_t T, double t_start, double dt,
                           double sigma, int64_t N, const int64_t* offsets, const double* beta,
                           double eps, int max_depth, const double* prior_lo,
                           const double* prior_hi, const double* momentum, const int8_t* dirs,
                           const double* u_leaf, const double* u_tree, double* q, double* logl,
                           double* grad, int32_t* depth_out, int32_t* steps_out,
                           int32_t* status_out) {
  return nuts_impl(model, d, T, t_start, dt, sigma, N, offsets, beta, eps, max_depth, prior_lo,
                   prior_hi, momentum, dirs, u_leaf, u_tree, 0, NULL, NULL, q, logl, grad, depth_out,
                   steps_out, status_out);
}

/* The NUTS transition for the posterior-start bridge target (split > 0). */
int oracle_nuts_transition_split(int model, const double* d, int64_t T, double t_start, double dt,
                                 double sigma, int64_t N, const int64_t* offsets,
                                 const double* beta, double eps, int max_depth,
                                 const double* prior_lo, const double* prior_hi,
                                 const double* momentum, const int8_t* dirs, const double* u_leaf,
                                 const double* u_tree, int64_t split, double* q, double* logl,
                                 double* grad, int32_t* depth_out, int32_t* steps_out,
                                 int32_t* status_out) {
  if (split < 0) return OR_EINVAL;
  return nuts_impl(model, d, T, t_start, dt, sigma, N, offsets, beta, eps, max_depth, prior_lo,
                   prior_hi, momentum, dirs, u_leaf, u_tree, split, NULL, NULL, q, logl, grad,
                   depth_out, steps_out, status_out);
}

/* The NUTS transition with a mass matrix M given through a factor W with
 * M^{-1} = W^T W (one n x n row-major block per particle at W + w_off[i],
 * n = K P; for example W = L^{-1} with M = L L^T, as oracle_metric_factor
 * gives). The momentum input is the whitened momentum r = W p_M, so the
 * draw stays N(0, I) and the kinetic energy |r|^2 / 2 equals
 * p_M^T M^{-1} p_M / 2. Hamilton's equations in (q, r) read
 *   dq/dt = W^T r,   dr/dt = W grad(beta logL),
 * so a leapfrog step kicks by (eps/2) W g and drifts by eps W^T r, and the
 * U-turn test rho.r is the metric's generalised criterion. split > 0 selects
 * the posterior-start bridge target as in oracle_nuts_transition_split. */
int oracle_nuts_transition_metric(int model, const double* d, int64_t T, double t_start,
                                  double dt, double sigma, int64_t N, const int64_t* offsets,
                                  const double* beta, double eps, int max_depth,
                                  const double* prior_lo, const double* prior_hi,
                                  const double* momentum, const int8_t* dirs,
                                  const double* u_leaf, const double* u_tree, int64_t split,
                                  const int64_t* w_off, const double* W, double* q, double* logl,
                                  double* grad, int32_t* depth_out, int32_t* steps_out,
                                  int32_t* status_out) {
  if (split < 0 || !W) return OR_EINVAL;
  return nuts_impl(model, d, T, t_start, dt, sigma, N, offsets, beta, eps, max_depth, prior_lo,
                   prior_hi, momentum, dirs, u_leaf, u_tree, split, w_off, W, q, logl, grad,
                   depth_out, steps_out, status_out);
}

/* ------------------------------------------------------------------ SMC steps
 * The steps of one SMC iteration around the likelihood (Sec. "Sequential
 * Monte Carlo" and Sec. "Algorithm and implementation"): choice of the next
 * inverse temperature, reweighting, resampling, and the accept/reject of the
 * birth and death moves of the mutation kernel (eq. kernel_mixture,
 * eq. rj_acceptance). */

/* ESS of w_i = exp(logw_prev_i + db * logl_i) (eq. ess), by a max-shifted sum.
 * Also returns the shift m and s1 = sum_i exp(log w_i - m). */
static double ess_at(int64_t N, const double* logl, const double* logw_prev, double db,
                     double* m_out, double* s1_out) {
  double m = -INFINITY;
  for (int64_t i = 0; i < N; ++i) {
    double lw = (logw_prev ? logw_prev[i] : 0.0) + db * logl[i];
    if (lw > m) m = lw;
  }
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = 0; i < N; ++i) {
    double lw = (logw_prev ? logw_prev[i] : 0.0) + db * logl[i];
    double e = exp(lw - m);
    s1 += e;
    s2 += e * e;
  }
  if (m_out) *m_out = m;
  if (s1_out) *s1_out = s1;
  return s1 * s1 / s2;
}

/* Next inverse temperature of the prior bridge (eq. prior_bridge) by the ESS
 * condition (eq. ess_target), for the incremental weights of
 * eq. incremental_weight: log w_i = logw_prev_i + (beta - beta_prev) logl_i with
 * untempered log-likelihoods logl (logw_prev NULL: uniform previous weights).
 *   beta = 1 if ESS(1) >= alpha N; otherwise bisection on [beta_prev, 1]: the
 *   bracket is halved (at most 60 times, and no further once its midpoint is
 *   no longer strictly inside), keeping its lower end where ESS >= alpha N;
 *   the result is the lower end, or the upper end if the lower end never
 *   moved (ESS(beta_prev) < alpha N, possible only with uneven logw_prev).
 * Outputs log w_i, normalised weights w_norm_i, and
 * scalars = {beta, ESS(beta), log Z_t/Z_{t-1}, number of ESS evaluations in
 * the bisection}, the evidence increment being log sum exp(log w) minus
 * log sum exp(logw_prev) (log N for uniform previous weights). */
int oracle_next_beta(int64_t N, const double* logl, const double* logw_prev, double beta_prev,
                     double alpha, double* logw, double* w_norm, double* scalars) {
  if (N < 1 || !logl || !logw || !w_norm || !scalars || !(beta_prev >= 0.0 && beta_prev <= 1.0) ||
      !(alpha > 0.0 && alpha <= 1.0))
    return OR_EINVAL;
  const double target = alpha * (double)N;
  double beta = 1.0;
  int evals = 0;
  if (!(ess_at(N, logl, logw_prev, 1.0 - beta_prev, NULL, NULL) >= target)) {
    double lo = beta_prev, hi = 1.0;
    int moved = 0;
    for (int it = 0; it < 60; ++it) {
      double mid = 0.5 * (lo + hi);
      if (!(mid > lo && mid < hi)) break;
      double e = ess_at(N, logl, logw_prev, mid - beta_prev, NULL, NULL);
      ++evals;
      if (e >= target) {
        lo = mid;
        moved = 1;
      } else {
        hi = mid;
      }
    }
    beta = moved ? lo : hi;
  }
  const double db = beta - beta_prev;
  double m, s1;
  const double ess = ess_at(N, logl, logw_prev, db, &m, &s1);
  for (int64_t i = 0; i < N; ++i) {
    logw[i] = (logw_prev ? logw_prev[i] : 0.0) + db * logl[i];
    w_norm[i] = exp(logw[i] - m) / s1;
  }
  double lse_prev;
  if (logw_prev) {
    double mp = -INFINITY, sp = 0.0;
    for (int64_t i = 0; i < N; ++i)
      if (logw_prev[i] > mp) mp = logw_prev[i];
    for (int64_t i = 0; i < N; ++i) sp += exp(logw_prev[i] - mp);
    lse_prev = mp + log(sp);
  } else {
    lse_prev = log((double)N);
  }
  scalars[0] = beta;
  scalars[1] = ess;
  scalars[2] = m + log(s1) - lse_prev;
  scalars[3] = (double)evals;
  return OR_OK;
}

/* Systematic resampling (the scheme is a reading: the paper resamples by the
 * normalised weights without naming one). With weights carried as integers
 * c_i = round(w_norm_i * 2^40) (0 for non-positive or NaN weights), inclusive
 * prefix sums C_i and their total C, offspring j = 0..N-1 takes position
 * U_j = floor(((j + u) * C) / N) (in double precision, evaluated in that
 * order; capped at C - 1) and the ancestor a_j = min{i : C_i > U_j}.
 * The new population is the ancestors' rows in CSR form: offsets_out[N+1],
 * theta_out[offsets_out[N]][P], which must not exceed m_cap rows. */
int oracle_resample_systematic(int model, int64_t N, const int64_t* offsets, const double* theta,
                               const double* w_norm, double u, int64_t m_cap, int32_t* ancestors,
                               int64_t* offsets_out, double* theta_out) {
  if (check_population(model, N, offsets, theta) != OR_OK || N < 1 || !w_norm || !ancestors ||
      !offsets_out || !(u >= 0.0 && u < 1.0))
    return OR_EINVAL;
  int P = oracle_n_params(model);
  int64_t* C = (int64_t*)malloc((size_t)N * sizeof(int64_t));
  if (!C) return OR_EINVAL;
  int64_t run = 0;
  for (int64_t i = 0; i < N; ++i) {
    double w = w_norm[i];
    int64_t c = 0;
    if (w > 0.0) c = (int64_t)rint((w < 1.0 ? w : 1.0) * 1099511627776.0);
    run += c;
    C[i] = run;
  }
  const int64_t total = run;
  if (total <= 0) {
    free(C);
    return OR_EINVAL;
  }
  int64_t a = 0; /* U_j does not decrease with j, so the scan resumes where it stopped */
  for (int64_t j = 0; j < N; ++j) {
    int64_t U = (int64_t)floor(((double)j + u) * (double)total / (double)N);
    if (U >= total) U = total - 1;
    while (C[a] <= U) ++a; /* the first index whose prefix exceeds U */
    ancestors[j] = (int32_t)a;
  }
  free(C);
  offsets_out[0] = 0;
  for (int64_t j = 0; j < N; ++j) {
    int64_t a = ancestors[j];
    offsets_out[j + 1] = offsets_out[j] + (offsets[a + 1] - offsets[a]);
  }
  if (offsets_out[N] > m_cap) return OR_EINVAL;
  for (int64_t j = 0; j < N; ++j) {
    int64_t a = ancestors[j];
    for (int64_t x = 0; x < (offsets[a + 1] - offsets[a]) * P; ++x)
      theta_out[offsets_out[j] * P + x] = theta[offsets[a] * P + x];
  }
  return OR_OK;
}

/* Accept/reject of the transdimensional moves of the mutation kernel
 * (Sec. "Reversible Jump Markov Chain Monte Carlo", eq. rj_acceptance) and
 * the new population. move[i]: 0 keeps particle i, 1 proposes the birth of
 * theta_birth[i] (drawn from the single-component prior), 2 proposes the
 * death of its component death_idx[i]. Reading of the acceptance ratio:
 * components are exchangeable, so a birth is taken to insert the new
 * component at a uniformly chosen one of the k+1 positions (appending it is
 * the same state up to order, which the likelihood and prior ignore) and a
 * death removes a uniformly chosen one of the k+1 (resp. k) components; the
 * 1/(k+1) position and selection probabilities then cancel, the prior
 * density of the new component cancels its proposal density, the Jacobian is
 * one, and with a uniform prior on k over [k_lo, k_hi]:
 *   birth: log alpha = dlogl_birth + log(p_death / p_birth)  if k + 1 <= k_hi
 *   death: log alpha = dlogl_death - log(p_death / p_birth)  if k - 1 >= k_lo
 * (-inf outside the k range), with the tempered log-likelihood changes of
 * delta_logl_birth_death. The move is accepted when log_u[i] < log alpha.
 * An accepted birth appends theta_birth[i] as the particle's last row; an
 * accepted death removes row death_idx[i]; other rows keep their order.
 * accepted[i] = 1 for an accepted move, else 0. The new population must not
 * exceed m_cap rows. */
int oracle_rj_apply(int model, int64_t N, const int64_t* offsets, const double* theta,
                    const int8_t* move, const double* theta_birth, const int32_t* death_idx,
                    const double* dlogl_birth, const double* dlogl_death, const double* log_u,
                    int32_t k_lo, int32_t k_hi, double log_pd_over_pb, int64_t m_cap,
                    int64_t* offsets_out, double* theta_out, int8_t* accepted) {
  if (check_population(model, N, offsets, theta) != OR_OK || !move || !log_u || !offsets_out ||
      !accepted || k_lo < 0 || k_hi < k_lo)
    return OR_EINVAL;
  int P = oracle_n_params(model);
  offsets_out[0] = 0;
  for (int64_t i = 0; i < N; ++i) {
    int64_t K = offsets[i + 1] - offsets[i];
    int acc = 0;
    if (move[i] == 1 && theta_birth && dlogl_birth && K + 1 <= k_hi)
      acc = log_u[i] < dlogl_birth[i] + log_pd_over_pb;
    else if (move[i] == 2 && death_idx && dlogl_death && K - 1 >= k_lo && death_idx[i] >= 0 &&
             death_idx[i] < K)
      acc = log_u[i] < dlogl_death[i] - log_pd_over_pb;
    accepted[i] = (int8_t)acc;
    offsets_out[i + 1] = offsets_out[i] + K + (acc ? (move[i] == 1 ? 1 : -1) : 0);
  }
  if (offsets_out[N] > m_cap) return OR_EINVAL;
  for (int64_t i = 0; i < N; ++i) {
    int64_t K = offsets[i + 1] - offsets[i];
    int64_t skip = (accepted[i] && move[i] == 2) ? death_idx[i] : -1;
    int64_t o = offsets_out[i];
    for (int64_t k = 0; k < K; ++k) {
      if (k == skip) continue;
      for (int p = 0; p < P; ++p) theta_out[o * P + p] = theta[(offsets[i] + k) * P + p];
      ++o;
    }
    if (accepted[i] && move[i] == 1) {
      for (int p = 0; p < P; ++p) theta_out[o * P + p] = theta_birth[i * P + p];
      ++o;
    }
  }
  return OR_OK;
}

/* ------------------------------------------------------------------ metric
 * Gauss-Newton (Fisher) approximation of the Hessian of the tempered
 * negative log-likelihood, for the NUTS mass matrix (Sec. "No-U-Turn-Sampler"
 * takes the Hessian of the negative log posterior as the metric; a uniform
 * prior adds nothing inside its box). With J_s the vector of template
 * partials dh_k(t_s)/dtheta_{k,p} of one particle (entry k P + p):
 *   F = (beta / sigma^2) sum_s J_s J_s^T
 * which is the Hessian of -beta logL without the term in r_s d2h/dtheta2
 * (exact when the residual vanishes). Output: the (K P) x (K P) matrix of
 * particle i, row-major, at F + f_offsets[i], where the caller's
 * f_offsets[i+1] - f_offsets[i] must equal (K_i P)^2. */
static int fisher_impl(int model, int64_t T, double t_start, double dt, double sigma, int64_t N,
                       const int64_t* offsets, const double* theta, const double* beta,
                       int64_t split, const int64_t* f_offsets, double* F);

int oracle_fisher(int model, int64_t T, double t_start, double dt, double sigma, int64_t N,
                  const int64_t* offsets, const double* theta, const double* beta,
                  const int64_t* f_offsets, double* F) {
  return fisher_impl(model, T, t_start, dt, sigma, N, offsets, theta, beta, 0, f_offsets, F);
}

/* The metric of the posterior-start bridge target (eq. reuse_bridge):
 * samples before `split` enter with weight 1, later ones with beta_i,
 *   F = (1 / sigma^2) sum_s w_s J_s J_s^T,  w_s = 1 (s < split) or beta_i. */
int oracle_fisher_split(int model, int64_t T, double t_start, double dt, double sigma, int64_t N,
                        const int64_t* offsets, const double* theta, const double* beta,
                        int64_t split, const int64_t* f_offsets, double* F) {
  if (split < 0) return OR_EINVAL;
  return fisher_impl(model, T, t_start, dt, sigma, N, offsets, theta, beta, split, f_offsets, F);
}

static int fisher_impl(int model, int64_t T, double t_start, double dt, double sigma, int64_t N,
                       const int64_t* offsets, const double* theta, const double* beta,
                       int64_t split, const int64_t* f_offsets, double* F) {
  if (check_population(model, N, offsets, theta) != OR_OK || T < 0 || !f_offsets)
    return OR_EINVAL;
  int P = oracle_n_params(model);
  for (int64_t i = 0; i < N; ++i) {
    int64_t n = (offsets[i + 1] - offsets[i]) * P;
    if (f_offsets[i + 1] - f_offsets[i] != n * n) return OR_EINVAL;
  }
  if (N > 0 && f_offsets[N] > 0 && !F) return OR_EINVAL;
#pragma omp parallel for schedule(dynamic)
  for (int64_t i = 0; i < N; ++i) {
    int64_t K = offsets[i + 1] - offsets[i];
    int64_t n = K * P;
    const double* th = theta ? theta + offsets[i] * P : NULL;
    double* Fi = F ? F + f_offsets[i] : NULL;
    double b = beta ? beta[i] : 1.0;
    if (n == 0) continue;
    double* J = (double*)malloc((size_t)n * sizeof(double));
    for (int64_t x = 0; x < n * n; ++x) Fi[x] = 0.0;
    for (int64_t s = 0; s < T; ++s) {
      double t = t_start + (double)s * dt;
      double ws = split == 0 ? 1.0 : sample_weight(s, split, b);
      for (int64_t k = 0; k < K; ++k) template_partials(model, th + k * P, t, J + k * P);
      for (int64_t a = 0; a < n; ++a)
        for (int64_t c = 0; c < n; ++c) Fi[a * n + c] += ws * (J[a] * J[c]);
    }
    /* without a split the tempering is one factor outside the sum */
    double outer = split == 0 ? b : 1.0;
    for (int64_t x = 0; x < n * n; ++x) Fi[x] = outer * (Fi[x] / (sigma * sigma));
    free(J);
  }
  return OR_OK;
}

/* Factor of the NUTS mass matrix from the metric: M = F + diag(ridge) with
 * ridge[p] added to the diagonal entry of parameter p of every component (a
 * floor where F is singular, e.g. the prior's precision), factored as
 * M = L L^T (Cholesky, row by row) and inverted by forward substitution:
 * W = L^{-1}, lower triangular, so M^{-1} = W^T W. Only the lower triangle of
 * each F block is read. Blocks share f_offsets' layout; W may not alias F.
 * status[i] = 0, or 1 when M is not numerically positive definite (a pivot
 * <= 0 or NaN), in which case particle i's W block is all NaN. */
int oracle_metric_factor(int model, int64_t N, const int64_t* offsets, const int64_t* f_offsets,
                         const double* F, const double* ridge, double* W, int32_t* status) {
  if (N < 0 || (N > 0 && (!offsets || !f_offsets || !ridge || !status))) return OR_EINVAL;
  int P = oracle_n_params(model);
  for (int64_t i = 0; i < N; ++i) {
    int64_t n = (offsets[i + 1] - offsets[i]) * P;
    if (n < 0 || f_offsets[i + 1] - f_offsets[i] != n * n) return OR_EINVAL;
  }
  if (N > 0 && f_offsets[N] > 0 && (!F || !W)) return OR_EINVAL;
#pragma omp parallel for schedule(dynamic)
  for (int64_t i = 0; i < N; ++i) {
    int64_t n = (offsets[i + 1] - offsets[i]) * P;
    status[i] = 0;
    if (n == 0) continue;
    const double* Fi = F + f_offsets[i];
    double* Wi = W + f_offsets[i];
    double* L = (double*)calloc((size_t)(n * n), sizeof(double));
    int ok = 1;
    for (int64_t r = 0; r < n && ok; ++r) {
      for (int64_t c = 0; c <= r; ++c) {
        double v = Fi[r * n + c] + (r == c ? ridge[r % P] : 0.0);
        for (int64_t k = 0; k < c; ++k) v -= L[r * n + k] * L[c * n + k];
        if (r == c) {
          if (!(v > 0.0)) { ok = 0; break; }
          L[r * n + r] = sqrt(v);
        } else {
          L[r * n + c] = v / L[c * n + c];
        }
      }
    }
    if (!ok) {
      status[i] = 1;
      for (int64_t x = 0; x < n * n; ++x) Wi[x] = NAN;
    } else {
      /* column c of W solves L w = e_c */
      for (int64_t c = 0; c < n; ++c)
        for (int64_t r = 0; r < n; ++r) {
          if (r < c) { Wi[r * n + c] = 0.0; continue; }
          double v = r == c ? 1.0 : 0.0;
          for (int64_t k = c; k < r; ++k) v -= L[r * n + k] * Wi[k * n + c];
          Wi[r * n + c] = v / L[r * n + r];
        }
    }
    free(L);
  }
  return OR_OK;
}
