/* FP64 oracle of the LISA Galactic-binary model in the frequency domain
 * (Sec. "LISA Galactic binaries"): eight parameters per source
 *   theta = (f0, fdot, log10 A, beta, lambda, psi, iota, phi0)
 * (reference frequency [Hz], its derivative [Hz/s], log10 of the strain
 * amplitude, ecliptic latitude and longitude, polarisation angle,
 * inclination, initial phase), the two noise-orthogonal TDI channels A and
 * E, and the likelihood of eq. gw_likelihood with a constant PSD S:
 *   log L = -(1/2) sum_{c in A,E} (4 df / S) sum_k |d_c[k] - h_c[k]|^2,
 * df = 1 / T_obs, over the bins k of a band [k0, k0 + B).
 *
 * TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
 * leg of the benchmark call it; the product path never links it. Plain
 * loops in double precision, written from the definitions below.
 *
 * Response (long-wavelength limit of the LISA constellation, as in Cutler
 * 1998 and Cornish & Rubbo 2003). Spacecraft k = 0, 1, 2 on the first-order
 * circular-orbit solution, with orbital phase a = 2 pi t / year and
 * b_k = 2 pi k / 3:
 *   x_k = R cos a + (e R / 2) (cos(2a - b_k) - 3 cos b_k)
 *   y_k = R sin a + (e R / 2) (sin(2a - b_k) - 3 sin b_k)
 *   z_k = -sqrt(3) e R cos(a - b_k),      e = L / (2 sqrt(3) R),
 * which keeps the arms at length L (to first order) in a plane inclined by
 * 60 degrees to the ecliptic, the guiding centre at R (cos a, sin a, 0).
 * The Michelson tensor with vertex k is M_k = (u u - v v) / 2 with u, v the
 * unit vectors from spacecraft k to k+1 and to k+2; the channels are
 *   A = (M_2 - M_0) / sqrt(2),   E = (M_0 - 2 M_1 + M_2) / sqrt(6)
 * (the T combination vanishes in this limit). The TDI transfer factor is a
 * constant over the narrow band and is absorbed into the PSD.
 *
 * Source: direction n = (cos b cos l, cos b sin l, sin b); u = (sin b cos l,
 * sin b sin l, -cos b), v = (-sin l, cos l, 0); e+ = cos 2psi (uu - vv) +
 * sin 2psi (uv + vu), ex = -sin 2psi (uu - vv) + cos 2psi (uv + vu);
 * h+ = A (1 + cos^2 i) cos Phi, hx = -2 A cos i sin Phi, with the phase at
 * the retarded time tau = t + n.x0(t) / c of the guiding centre:
 *   Phi = 2 pi (f0 tau + fdot tau^2 / 2) + phi0.
 * Channel strain h_c(t) = (D_c : e+) h+ + (D_c : ex) hx = Re[a_c e^{i Phi}]
 * with a_c = F+ A+ - i Fx Ax, A+ = A (1 + cos^2 i), Ax = -2 A cos i.
 * Amplitudes are in units of 1e-21 strain: A = 10^(log10 A + 21).
 *
 * Template spectrum (the fast/slow decomposition of FastGB / JAXGB, which
 * the paper's waveforms come from): with carrier bin q = floor(f0 T_obs) and
 * the slowly varying envelope z_c(t) = (1/2) a_c(t) exp(i (Phi - 2 pi q t /
 * T_obs)) sampled at t_j = j T_obs / Ns, j < Ns,
 *   h_c[q + m] = (T_obs / Ns) sum_j z_c(t_j) exp(-2 pi i m j / Ns),
 * m = -Ns/2 .. Ns/2 - 1 (bins outside the band dropped). The spectrum's
 * Fourier convention is h[k] = dt sum_n h(t_n) exp(-2 pi i k n / Nt);
 * oracle_gblisa_spectrum_dft computes exactly that from the time series,
 * which pins the decomposition within its aliasing error. */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_EINVAL 1
#define GB_P 8

static const double kPi = 3.14159265358979323846;
static const double kYear = 31557600.0;       /* Julian year [s] */
static const double kAU = 1.495978707e11;     /* orbital radius R [m] */
static const double kC = 299792458.0;         /* [m/s] */
static const double kArm = 2.5e9;             /* arm length L [m] */
static const double kAmpUnit = 1e21;          /* amplitudes in units of 1e-21 */

/* ------------------------------------------------------------ geometry */
static void sc_positions(double t, double x[3][3]) {
  double a = 2.0 * kPi * t / kYear;
  double e = kArm / (2.0 * sqrt(3.0) * kAU);
  for (int k = 0; k < 3; ++k) {
    double b = 2.0 * kPi * k / 3.0;
    x[k][0] = kAU * cos(a) + 0.5 * e * kAU * (cos(2.0 * a - b) - 3.0 * cos(b));
    x[k][1] = kAU * sin(a) + 0.5 * e * kAU * (sin(2.0 * a - b) - 3.0 * sin(b));
    x[k][2] = -sqrt(3.0) * e * kAU * cos(a - b);
  }
}

static void unit(const double* from, const double* to, double* u) {
  double d[3] = {to[0] - from[0], to[1] - from[1], to[2] - from[2]};
  double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  for (int i = 0; i < 3; ++i) u[i] = d[i] / n;
}

/* Michelson tensor with vertex k */
static void michelson(double x[3][3], int k, double M[3][3]) {
  double u[3], v[3];
  unit(x[k], x[(k + 1) % 3], u);
  unit(x[k], x[(k + 2) % 3], v);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[i][j] = 0.5 * (u[i] * u[j] - v[i] * v[j]);
}

/* Detector tensors of the A and E channels at time t */
void oracle_gblisa_tensors(double t, double* DA9, double* DE9) {
  double x[3][3], M[3][3][3];
  sc_positions(t, x);
  for (int k = 0; k < 3; ++k) michelson(x, k, M[k]);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      DA9[3 * i + j] = (M[2][i][j] - M[0][i][j]) / sqrt(2.0);
      DE9[3 * i + j] = (M[0][i][j] - 2.0 * M[1][i][j] + M[2][i][j]) / sqrt(6.0);
    }
}

void oracle_gblisa_positions(double t, double* x9) {
  double x[3][3];
  sc_positions(t, x);
  memcpy(x9, x, sizeof(x));
}

static double contract(const double* D9, double T[3][3]) {
  double s = 0.0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) s += D9[3 * i + j] * T[i][j];
  return s;
}

/* Polarisation basis tensors eps+ = uu - vv, epsx = uv + vu of the source
 * direction, and (when d != NULL) their derivatives with respect to the
 * latitude (d[0], d[1]) and longitude (d[2], d[3]). */
static void basis(double b, double l, double ep[3][3], double ex[3][3], double d[4][3][3]) {
  double u[3] = {sin(b) * cos(l), sin(b) * sin(l), -cos(b)};
  double v[3] = {-sin(l), cos(l), 0.0};
  double ub[3] = {cos(b) * cos(l), cos(b) * sin(l), sin(b)};   /* du/db */
  double ul[3] = {-sin(b) * sin(l), sin(b) * cos(l), 0.0};     /* du/dl */
  double vl[3] = {-cos(l), -sin(l), 0.0};                      /* dv/dl */
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      ep[i][j] = u[i] * u[j] - v[i] * v[j];
      ex[i][j] = u[i] * v[j] + v[i] * u[j];
      if (d) {
        d[0][i][j] = ub[i] * u[j] + u[i] * ub[j];
        d[1][i][j] = ub[i] * v[j] + v[i] * ub[j];
        d[2][i][j] = ul[i] * u[j] + u[i] * ul[j] - vl[i] * v[j] - v[i] * vl[j];
        d[3][i][j] = ul[i] * v[j] + vl[i] * u[j] + u[i] * vl[j] + v[i] * ul[j];
      }
    }
}

/* Antenna patterns of both channels at time t for direction (b, l) and
 * polarisation psi: Fp[c] = D_c : e+, Fx[c] = D_c : ex (c = 0: A, 1: E). */
void oracle_gblisa_response(double t, double b, double l, double psi, double* Fp, double* Fx) {
  double DA[9], DE[9], ep[3][3], ex[3][3];
  oracle_gblisa_tensors(t, DA, DE);
  basis(b, l, ep, ex, NULL);
  for (int c = 0; c < 2; ++c) {
    const double* D = c == 0 ? DA : DE;
    double P = contract(D, ep), X = contract(D, ex);
    Fp[c] = cos(2.0 * psi) * P + sin(2.0 * psi) * X;
    Fx[c] = -sin(2.0 * psi) * P + cos(2.0 * psi) * X;
  }
}

/* Retarded time at the guiding centre, tau = t + n . x0(t) / c */
static double retarded(double t, double b, double l) {
  double a = 2.0 * kPi * t / kYear;
  return t + kAU * cos(b) * cos(a - l) / kC;
}

/* ------------------------------------------------------------ waveform */
/* Time-domain strain of one source in both channels at time t. */
void oracle_gblisa_strain(const double* th, double t, double* h2) {
  double f0 = th[0], fd = th[1], A = pow(10.0, th[2]) * kAmpUnit;
  double b = th[3], l = th[4], psi = th[5], inc = th[6], phi0 = th[7];
  double Fp[2], Fx[2];
  oracle_gblisa_response(t, b, l, psi, Fp, Fx);
  double tau = retarded(t, b, l);
  double Phi = 2.0 * kPi * (f0 * tau + 0.5 * fd * tau * tau) + phi0;
  double Ap = A * (1.0 + cos(inc) * cos(inc)), Ax = -2.0 * A * cos(inc);
  for (int c = 0; c < 2; ++c) h2[c] = Fp[c] * Ap * cos(Phi) + Fx[c] * Ax * sin(Phi);
}

/* Envelope z_c(t_j) of one source (re, im per channel) and, when dz != NULL,
 * its derivatives with respect to the eight parameters, dz[p][c][re/im]. */
static void envelope(const double* th, double T_obs, int Ns, int64_t q, int j, double z[2][2],
                     double dz[GB_P][2][2]) {
  double f0 = th[0], fd = th[1], A = pow(10.0, th[2]) * kAmpUnit;
  double b = th[3], l = th[4], psi = th[5], inc = th[6], phi0 = th[7];
  double t = (double)j * T_obs / (double)Ns;
  double DA[9], DE[9], ep[3][3], ex[3][3], dB[4][3][3];
  oracle_gblisa_tensors(t, DA, DE);
  basis(b, l, ep, ex, dz ? dB : NULL);
  double a = 2.0 * kPi * t / kYear;
  double tau = t + kAU * cos(b) * cos(a - l) / kC;
  /* phase in cycles, reduced: f0 tau + fdot tau^2 / 2 - q j / Ns + phi0 / (2 pi) */
  double cyc = f0 * tau + 0.5 * fd * tau * tau - (double)(q % Ns) * (double)j / (double)Ns;
  cyc = cyc - floor(cyc) + phi0 / (2.0 * kPi);
  double ph = 2.0 * kPi * cyc;
  double cph = cos(ph), sph = sin(ph);
  double ci = cos(inc), si = sin(inc);
  double Ap = A * (1.0 + ci * ci), Ax = -2.0 * A * ci;
  double c2 = cos(2.0 * psi), s2 = sin(2.0 * psi);
  double Fp[2], Fx[2], dFp[2][2], dFx[2][2]; /* d[latitude / longitude] */
  for (int c = 0; c < 2; ++c) {
    const double* D = c == 0 ? DA : DE;
    double P = contract(D, ep), X = contract(D, ex);
    Fp[c] = c2 * P + s2 * X;
    Fx[c] = -s2 * P + c2 * X;
    if (dz)
      for (int s = 0; s < 2; ++s) {
        double dP = contract(D, dB[2 * s]), dX = contract(D, dB[2 * s + 1]);
        dFp[c][s] = c2 * dP + s2 * dX;
        dFx[c][s] = -s2 * dP + c2 * dX;
      }
  }
  for (int c = 0; c < 2; ++c) {
    /* a = Fp Ap - i Fx Ax; z = a e^{i ph} / 2 */
    double ar = Fp[c] * Ap, ai = -Fx[c] * Ax;
    z[c][0] = 0.5 * (ar * cph - ai * sph);
    z[c][1] = 0.5 * (ar * sph + ai * cph);
  }
  if (!dz) return;
  /* phase derivatives: dPhi/dtheta, and the derivative of the complex
   * amplitude a for each parameter */
  double dphi[GB_P] = {0};
  dphi[0] = 2.0 * kPi * tau;
  dphi[1] = kPi * tau * tau;
  double fi = f0 + fd * tau; /* dPhi/dtau / (2 pi) */
  dphi[3] = 2.0 * kPi * fi * (-kAU * sin(b) * cos(a - l) / kC);
  dphi[4] = 2.0 * kPi * fi * (kAU * cos(b) * sin(a - l) / kC);
  dphi[7] = 1.0;
  for (int c = 0; c < 2; ++c) {
    double da[GB_P][2];
    memset(da, 0, sizeof(da));
    double ln10 = log(10.0);
    da[2][0] = ln10 * Fp[c] * Ap;
    da[2][1] = -ln10 * Fx[c] * Ax;
    da[3][0] = dFp[c][0] * Ap;
    da[3][1] = -dFx[c][0] * Ax;
    da[4][0] = dFp[c][1] * Ap;
    da[4][1] = -dFx[c][1] * Ax;
    /* dF+/dpsi = 2 Fx, dFx/dpsi = -2 F+ */
    da[5][0] = 2.0 * Fx[c] * Ap;
    da[5][1] = 2.0 * Fp[c] * Ax;
    /* dA+/di = -2 A cos i sin i, dAx/di = 2 A sin i */
    da[6][0] = Fp[c] * (-2.0 * A * ci * si);
    da[6][1] = -Fx[c] * (2.0 * A * si);
    for (int p = 0; p < GB_P; ++p) {
      /* d z = (da e^{i ph}) / 2 + i dphi z */
      double r = 0.5 * (da[p][0] * cph - da[p][1] * sph) - dphi[p] * z[c][1];
      double i = 0.5 * (da[p][0] * sph + da[p][1] * cph) + dphi[p] * z[c][0];
      dz[p][c][0] = r;
      dz[p][c][1] = i;
    }
  }
}

static int64_t carrier_bin(double f0, double T_obs) { return (int64_t)floor(f0 * T_obs); }

/* Adds sign * the spectrum of one source (and, if dh != NULL, writes the
 * spectra of its eight derivatives, dh[p][c][k][re/im] over the band) */
static void add_source(const double* th, double T_obs, int Ns, int64_t k0, int64_t B, double sign,
                       double* out, double* dh) {
  int64_t q = carrier_bin(th[0], T_obs);
  double (*z)[2][2] = malloc((size_t)Ns * sizeof(*z));
  double (*dz)[GB_P][2][2] = dh ? malloc((size_t)Ns * sizeof(*dz)) : NULL;
  for (int j = 0; j < Ns; ++j) envelope(th, T_obs, Ns, q, j, z[j], dz ? dz[j] : NULL);
  double scale = T_obs / (double)Ns;
  for (int m = -Ns / 2; m < Ns / 2; ++m) {
    int64_t k = q + m - k0;
    if (k < 0 || k >= B) continue;
    double s[2][2] = {{0, 0}, {0, 0}}, ds[GB_P][2][2];
    if (dh) memset(ds, 0, sizeof(ds));
    for (int j = 0; j < Ns; ++j) {
      double w = -2.0 * kPi * (double)(((int64_t)m * j) % Ns) / (double)Ns;
      double cw = cos(w), sw = sin(w);
      for (int c = 0; c < 2; ++c) {
        s[c][0] += z[j][c][0] * cw - z[j][c][1] * sw;
        s[c][1] += z[j][c][0] * sw + z[j][c][1] * cw;
        if (dh)
          for (int p = 0; p < GB_P; ++p) {
            ds[p][c][0] += dz[j][p][c][0] * cw - dz[j][p][c][1] * sw;
            ds[p][c][1] += dz[j][p][c][0] * sw + dz[j][p][c][1] * cw;
          }
      }
    }
    for (int c = 0; c < 2; ++c) {
      out[(c * B + k) * 2 + 0] += sign * scale * s[c][0];
      out[(c * B + k) * 2 + 1] += sign * scale * s[c][1];
      if (dh)
        for (int p = 0; p < GB_P; ++p) {
          dh[((p * 2 + c) * B + k) * 2 + 0] = scale * ds[p][c][0];
          dh[((p * 2 + c) * B + k) * 2 + 1] = scale * ds[p][c][1];
        }
    }
  }
  free(z);
  free(dz);
}

/* Template spectrum of K sources over the band, out[2][B][2] (channel, bin,
 * re/im), by the fast/slow decomposition with Ns envelope samples. */
int oracle_gblisa_spectrum(int64_t K, const double* theta, double T_obs, int Ns, int64_t k0,
                           int64_t B, double* out) {
  if (K < 0 || B < 0 || !(T_obs > 0) || Ns < 2 || (Ns & (Ns - 1)) || (B > 0 && !out) ||
      (K > 0 && !theta))
    return OR_EINVAL;
  memset(out, 0, (size_t)(4 * B) * sizeof(double));
  for (int64_t k = 0; k < K; ++k) add_source(theta + k * GB_P, T_obs, Ns, k0, B, 1.0, out, NULL);
  return OR_OK;
}

/* The same band from the plain DFT of the strain sampled at Nt points,
 * h[k] = dt sum_n h(t_n) exp(-2 pi i k n / Nt), dt = T_obs / Nt. */
int oracle_gblisa_spectrum_dft(int64_t K, const double* theta, double T_obs, int64_t Nt,
                               int64_t k0, int64_t B, double* out) {
  if (K < 0 || B < 0 || !(T_obs > 0) || Nt < 2 || (B > 0 && !out) || (K > 0 && !theta))
    return OR_EINVAL;
  memset(out, 0, (size_t)(4 * B) * sizeof(double));
  double dt = T_obs / (double)Nt;
  double* h = malloc((size_t)(2 * Nt) * sizeof(double));
  for (int64_t n = 0; n < Nt; ++n) {
    double acc[2] = {0, 0};
    for (int64_t k = 0; k < K; ++k) {
      double h2[2];
      oracle_gblisa_strain(theta + k * GB_P, (double)n * dt, h2);
      acc[0] += h2[0];
      acc[1] += h2[1];
    }
    h[2 * n] = acc[0];
    h[2 * n + 1] = acc[1];
  }
#pragma omp parallel for schedule(dynamic)
  for (int64_t k = 0; k < B; ++k) {
    double s[2][2] = {{0, 0}, {0, 0}};
    for (int64_t n = 0; n < Nt; ++n) {
      double w = -2.0 * kPi * (double)(((k0 + k) * n) % Nt) / (double)Nt;
      double cw = cos(w), sw = sin(w);
      for (int c = 0; c < 2; ++c) {
        s[c][0] += h[2 * n + c] * cw;
        s[c][1] += h[2 * n + c] * sw;
      }
    }
    for (int c = 0; c < 2; ++c) {
      out[(c * B + k) * 2 + 0] = dt * s[c][0];
      out[(c * B + k) * 2 + 1] = dt * s[c][1];
    }
  }
  free(h);
  return OR_OK;
}

static int check_population_ok(int64_t N, const int64_t* offsets, const double* theta) {
  if (N < 0 || (N > 0 && !offsets)) return OR_EINVAL;
  if (N > 0 && offsets[0] != 0) return OR_EINVAL;
  for (int64_t i = 0; i < N; ++i)
    if (offsets[i + 1] < offsets[i]) return OR_EINVAL;
  if (N > 0 && offsets[N] > 0 && !theta) return OR_EINVAL;
  return OR_OK;
}

/* Tempered log-likelihood (and gradient when grad != NULL) of every
 * particle: logl_i = beta_i log L, grad = beta_i d log L / d theta with
 *   d log L / d theta = (4 df / S) Re sum_c sum_k conj(r_c[k]) dh_c[k]/dtheta,
 * r = d - sum of the particle's templates; d is [2][B][2]. */
int oracle_gblisa_logl_grad(const double* d, int64_t k0, int64_t B, double T_obs, double S, int Ns,
                            int64_t N, const int64_t* offsets, const double* theta,
                            const double* beta, double* logl, double* grad) {
  if (check_population_ok(N, offsets, theta) != OR_OK || B < 0 || !(T_obs > 0) || !(S > 0) ||
      (B > 0 && !d) || (N > 0 && !logl))
    return OR_EINVAL;
  double cnorm = 4.0 / (T_obs * S);
#pragma omp parallel for schedule(dynamic)
  for (int64_t i = 0; i < N; ++i) {
    int64_t K = offsets[i + 1] - offsets[i];
    const double* th = theta ? theta + offsets[i] * GB_P : NULL;
    double b = beta ? beta[i] : 1.0;
    double* r = malloc((size_t)(4 * B + 1) * sizeof(double));
    for (int64_t x = 0; x < 4 * B; ++x) r[x] = d[x];
    for (int64_t k = 0; k < K; ++k) add_source(th + k * GB_P, T_obs, Ns, k0, B, -1.0, r, NULL);
    double ss = 0.0;
    for (int64_t x = 0; x < 4 * B; ++x) ss += r[x] * r[x];
    logl[i] = b * (-0.5 * cnorm * ss);
    if (grad && K > 0) {
      double* dh = malloc((size_t)(GB_P * 4 * B + 1) * sizeof(double));
      double* junk = malloc((size_t)(4 * B + 1) * sizeof(double));
      for (int64_t k = 0; k < K; ++k) {
        memset(dh, 0, (size_t)(GB_P * 4 * B) * sizeof(double));
        memset(junk, 0, (size_t)(4 * B) * sizeof(double));
        add_source(th + k * GB_P, T_obs, Ns, k0, B, 1.0, junk, dh);
        for (int p = 0; p < GB_P; ++p) {
          double s = 0.0;
          for (int64_t x = 0; x < 2 * B; ++x)
            s += r[2 * x] * dh[(p * 2 * B) * 2 + 2 * x] + r[2 * x + 1] * dh[(p * 2 * B) * 2 + 2 * x + 1];
          grad[(offsets[i] + k) * GB_P + p] = b * cnorm * s;
        }
      }
      free(dh);
      free(junk);
    }
    free(r);
  }
  return OR_OK;
}

/* Birth and death changes of the tempered log-likelihood (the reversible-jump
 * deltas of eq. rj_acceptance for this model): with c = beta (4 df / S) and
 * r the particle's residual,
 *   birth:  c (Re<r, h_new> - |h_new|^2 / 2)
 *   death:  -c (Re<r, h_j> + |h_j|^2 / 2)   (death_idx[i] = j, or -1: 0). */
int oracle_gblisa_delta(const double* d, int64_t k0, int64_t B, double T_obs, double S, int Ns,
                        int64_t N, const int64_t* offsets, const double* theta, const double* beta,
                        const double* theta_birth, const int32_t* death_idx, double* d_birth,
                        double* d_death) {
  if (check_population_ok(N, offsets, theta) != OR_OK || B < 0 || !(T_obs > 0) || !(S > 0) ||
      (B > 0 && !d))
    return OR_EINVAL;
  if (N > 0 && ((theta_birth && !d_birth) || (death_idx && !d_death))) return OR_EINVAL;
  for (int64_t i = 0; death_idx && i < N; ++i)
    if (death_idx[i] < -1 || death_idx[i] >= offsets[i + 1] - offsets[i]) return OR_EINVAL;
  double cnorm = 4.0 / (T_obs * S);
#pragma omp parallel for schedule(dynamic)
  for (int64_t i = 0; i < N; ++i) {
    int64_t K = offsets[i + 1] - offsets[i];
    const double* th = theta ? theta + offsets[i] * GB_P : NULL;
    double b = beta ? beta[i] : 1.0;
    double* r = malloc((size_t)(4 * B + 1) * sizeof(double));
    double* h = malloc((size_t)(4 * B + 1) * sizeof(double));
    for (int64_t x = 0; x < 4 * B; ++x) r[x] = d[x];
    for (int64_t k = 0; k < K; ++k) add_source(th + k * GB_P, T_obs, Ns, k0, B, -1.0, r, NULL);
    double rh = 0.0, hh = 0.0;
    if (theta_birth) {
      memset(h, 0, (size_t)(4 * B) * sizeof(double));
      add_source(theta_birth + i * GB_P, T_obs, Ns, k0, B, 1.0, h, NULL);
      for (int64_t x = 0; x < 4 * B; ++x) {
        rh += r[x] * h[x];
        hh += h[x] * h[x];
      }
      d_birth[i] = b * cnorm * (rh - 0.5 * hh);
    }
    int32_t j = death_idx ? death_idx[i] : -2;
    if (j == -1) {
      d_death[i] = 0.0;
    } else if (j >= 0) {
      memset(h, 0, (size_t)(4 * B) * sizeof(double));
      add_source(th + j * GB_P, T_obs, Ns, k0, B, 1.0, h, NULL);
      rh = hh = 0.0;
      for (int64_t x = 0; x < 4 * B; ++x) {
        rh += r[x] * h[x];
        hh += h[x] * h[x];
      }
      d_death[i] = -(b * cnorm * (rh + 0.5 * hh));
    }
    free(r);
    free(h);
  }
  return OR_OK;
}

/* Gauss-Newton metric of the frequency-domain model, per source: for every
 * particle the (8K) x (8K) matrix whose diagonal 8 x 8 block k is
 *   F_k = beta (4 df / S) Re sum_c sum_k conj(dh_c[k] / dtheta_a) dh_c[k] / dtheta_b
 * over the band (the Hessian of -beta logL in that source's parameters
 * without its residual term), and whose blocks between different sources
 * are zero. Blocks at F + f_offsets[i], row-major; f_offsets[i+1] -
 * f_offsets[i] must be (8 K_i)^2. */
int oracle_gblisa_fisher(int64_t k0, int64_t B, double T_obs, double S, int Ns, int64_t N,
                         const int64_t* offsets, const double* theta, const double* beta,
                         const int64_t* f_offsets, double* F) {
  if (check_population_ok(N, offsets, theta) != OR_OK || B < 0 || !(T_obs > 0) || !(S > 0) ||
      (N > 0 && !f_offsets))
    return OR_EINVAL;
  for (int64_t i = 0; i < N; ++i) {
    int64_t n = (offsets[i + 1] - offsets[i]) * GB_P;
    if (f_offsets[i + 1] - f_offsets[i] != n * n) return OR_EINVAL;
  }
  if (N > 0 && f_offsets[N] > 0 && !F) return OR_EINVAL;
  double cnorm = 4.0 / (T_obs * S);
#pragma omp parallel for schedule(dynamic)
  for (int64_t i = 0; i < N; ++i) {
    int64_t K = offsets[i + 1] - offsets[i], n = K * GB_P;
    double b = beta ? beta[i] : 1.0;
    double* Fi = F ? F + f_offsets[i] : NULL;
    if (n == 0) continue;
    for (int64_t x = 0; x < n * n; ++x) Fi[x] = 0.0;
    double* dh = malloc((size_t)(GB_P * 4 * B + 1) * sizeof(double));
    double* junk = malloc((size_t)(4 * B + 1) * sizeof(double));
    for (int64_t k = 0; k < K; ++k) {
      memset(dh, 0, (size_t)(GB_P * 4 * B) * sizeof(double));
      memset(junk, 0, (size_t)(4 * B) * sizeof(double));
      add_source(theta + (offsets[i] + k) * GB_P, T_obs, Ns, k0, B, 1.0, junk, dh);
      for (int pa = 0; pa < GB_P; ++pa)
        for (int pb = 0; pb < GB_P; ++pb) {
          double s = 0.0;
          for (int64_t x = 0; x < 4 * B; ++x) s += dh[pa * 4 * B + x] * dh[pb * 4 * B + x];
          Fi[(k * GB_P + pa) * n + k * GB_P + pb] = b * cnorm * s;
        }
    }
    free(dh);
    free(junk);
  }
  return OR_OK;
}
