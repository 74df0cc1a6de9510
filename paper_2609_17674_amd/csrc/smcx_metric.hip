// Gauss-Newton (Fisher) metric of every particle on the matrix cores.
//
// F_i = (beta_i / sigma^2) sum_s J_s J_s^T with J_s the template partials
// dh_k(t_s)/dtheta_{k,p} of particle i (coordinate k P + p): the Hessian of the
// tempered negative log-likelihood without its residual term, the mass matrix
// the NUTS section of the paper asks for (the Hessian of the negative log
// posterior; a uniform prior adds nothing inside its box).
//
// One wave owns one particle and walks the samples in steps of 8. Per step
// each lane forms J at 4 samples for its coordinate in each block of 32
// coordinates, in natural units (J~ = J * s with s = (1, w, w) for pulses and
// (1, 1/T_obs, 1/T_obs^2, 1) for sinusoids, so every entry is of order one),
// rounds them to FP16 and feeds them as both operands of
// v_mfma_f32_32x32x8_f16: with A[i][k] held by lane i + 32 (k/4), element
// k%4, and B[k][j] by lane j + 32 (k/4), a lane's own values are its row of
// A and column of B, and D = J~_block_i^T J~_block_j. The FP32 accumulators
// are flushed into the FP64 output after each window of 4096 samples (one
// launch per window), each entry owned by one lane (read-add-write, no
// atomics), so the result is deterministic; entries
// below the diagonal are written as copies of those above it.
// Error: FP16 rounding of J~ (2^-11 relative) bounds |dF~_ac| by about
// 2^-10 sqrt(F~_aa F~_cc), plus FP32 accumulation over 512 steps.
#include "smcx_internal.h"

#include <algorithm>

#include <math.h>

namespace smcx {
namespace {

typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef float float16v __attribute__((ext_vector_type(16)));

constexpr double kTwoPiM = 6.283185307179586476925286766559;
constexpr double kPiM = 3.141592653589793238462643383279;
constexpr double kHalfLog2eRoot = 0.84932180028801904272150283410289;  // sqrt(log2(e) / 2)
constexpr int kFlushSamples = 4096;

struct MetricArgs {
  int P;
  int64_t N, M, T;
  double t_start, dt, inv_sigma2, t_obs;
  int32_t k_max;
  const int64_t* offsets;
  const double* theta;
  const double* beta;
  const int64_t* f_offsets;
  int64_t f_size;  // entries of F: every block must fit
  double* F;
  int* flag;
  int64_t w0, w1;  // sample window of this launch; the first window writes F, later ones add
  int tempered;    // 1: the window's samples carry beta_i (0: before a bridge split)
  int blocks;      // 1: only each component's P x P block, at F + m P P (source row m)
  const uint8_t* mask;  // [N] or nullptr: particles with mask[i] == 0 get zero blocks
};

// Per-lane description of one coordinate (component k, parameter p), set up
// so that J~ needs no branch on p; padding lanes get zero coefficients.
template <int MODEL>
struct Coord;

// pulse: x = s - nf (exact), z = x a - fa, J~ = e (c0 + c1 z + c2 z^2) with
// e = 2^(-z^2): (c0, c1, c2) = (1, 0, 0), (0, A k, 0), (0, 0, A k^2) for
// p = 0, 1, 2, k = 1 / sqrt(log2(e)/2) so that k z = (t - t0)/w
template <>
struct Coord<SMCX_PULSE> {
  float nf, a, fa, c0, c1, c2;
};

// sinusoid: phase in cycles ph0 + ph1 s + ph2 s^2 (FP64);
// J~ = sin(2 pi (phase + shift)) (k0 + k1 tr + k2 tr^2), tr = t / T_obs
// = tr0 + s dtr: shift 0 and (1, 0, 0) for A'; a quarter cycle (the cosine)
// and (0, 2 pi A', 0), (0, 0, pi A'), (A', 0, 0) for f0, fdot, phi0
template <>
struct Coord<SMCX_GBSINE> {
  double ph0, ph1, ph2;
  float shift, k0, k1, k2, tr0, dtr;
};

template <int MODEL>
__device__ Coord<MODEL> make_coord(const MetricArgs& a, const double* th, int c, int n,
                                   double* scale) {
  Coord<MODEL> q{};
  *scale = 1.0;
  if (c >= n) return q;  // all coefficients zero
  const int p = c % a.P;
  const double* r = th + (int64_t)(c / a.P) * a.P;
  if constexpr (MODEL == SMCX_PULSE) {
    const double A = r[0], t0 = r[1], w = r[2];
    const double cc = (t0 - a.t_start) / a.dt;
    double nn = floor(cc);
    nn = fmin(fmax(nn, -4194304.0), 4194304.0);
    const double al = kHalfLog2eRoot * a.dt / w;
    const double k = 1.0 / kHalfLog2eRoot;
    q.nf = (float)nn;
    q.a = (float)al;
    q.fa = (float)((cc - nn) * al);
    q.c0 = p == 0 ? 1.f : 0.f;
    q.c1 = p == 1 ? (float)(A * k) : 0.f;
    q.c2 = p == 2 ? (float)(A * k * k) : 0.f;
    *scale = p == 0 ? 1.0 : w;
  } else {
    const double A = r[0], f0 = r[1], fd = r[2], phi0 = r[3];
    const double ts = a.t_start, dt = a.dt;
    q.ph0 = f0 * ts + 0.5 * fd * ts * ts + phi0 / kTwoPiM;
    q.ph1 = (f0 + fd * ts) * dt;
    q.ph2 = 0.5 * fd * dt * dt;
    q.shift = p == 0 ? 0.f : 0.25f;
    q.k0 = p == 0 ? 1.f : (p == 3 ? (float)A : 0.f);
    q.k1 = p == 1 ? (float)(kTwoPiM * A) : 0.f;
    q.k2 = p == 2 ? (float)(kPiM * A) : 0.f;
    q.tr0 = (float)(ts / a.t_obs);
    q.dtr = (float)(dt / a.t_obs);
    *scale = p == 1 ? 1.0 / a.t_obs : (p == 2 ? 1.0 / (a.t_obs * a.t_obs) : 1.0);
  }
  return q;
}

// J~ of one coordinate at sample s.
template <int MODEL>
__device__ __forceinline__ float jvalue(const Coord<MODEL>& q, int s) {
  if constexpr (MODEL == SMCX_PULSE) {
    const float z = __builtin_fmaf((float)s - q.nf, q.a, -q.fa);
    const float e = __builtin_amdgcn_exp2f(-(z * z));
    return e * __builtin_fmaf(__builtin_fmaf(q.c2, z, q.c1), z, q.c0);
  } else {
    const double sd = (double)s;
    const double ph = fma(fma(q.ph2, sd, q.ph1), sd, q.ph0);
    const float rev = (float)(ph - rint(ph)) + q.shift;  // revolutions in [-0.5, 0.75]
    const float tr = __builtin_fmaf((float)s, q.dtr, q.tr0);
    return __builtin_amdgcn_sinf(rev) * __builtin_fmaf(__builtin_fmaf(q.k2, tr, q.k1), tr, q.k0);
  }
}

template <int MODEL, int NB>
__global__ __launch_bounds__(256) void metric_kernel(MetricArgs a) {
  constexpr int NP = NB * (NB + 1) / 2;
  extern __shared__ double scl[];  // [4 waves][32 NB] inverse natural scales of the coordinates
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 4 + wid;
  if (i >= a.N) return;
  const int64_t o0 = a.offsets[i], o1 = a.offsets[i + 1];
  if (!(o0 >= 0 && o1 >= o0 && o1 <= a.M && o1 - o0 <= a.k_max)) {
    if (lane == 0) atomicOr(a.flag, kFlagOffsets);
    return;
  }
  const int n = (int)(o1 - o0) * a.P;
  const int64_t fo = a.blocks ? o0 * a.P * a.P : a.f_offsets[i];
  if (n > 32 * NB ||
      (!a.blocks && (a.f_offsets[i + 1] - fo != (int64_t)n * n || fo < 0 ||
                     fo + (int64_t)n * n > a.f_size))) {
    if (lane == 0) atomicOr(a.flag, kFlagOffsets);
    return;
  }
  if (n == 0) return;
  if (a.mask && !a.mask[i]) {
    // not selected: zero blocks (the factor's ridge makes them definite),
    // written by the first window; later windows add nothing
    if (a.w0 == 0) {
      const int64_t cnt = a.blocks ? (int64_t)n * a.P : (int64_t)n * n;
      for (int64_t e = lane; e < cnt; e += 64) a.F[fo + e] = 0.0;
    }
    return;
  }
  const double* th = a.theta + o0 * a.P;
  Coord<MODEL> q[NB];
  double* my = scl + wid * 32 * NB;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    double sc;
    q[b] = make_coord<MODEL>(a, th, 32 * b + (lane & 31), n, &sc);
    if (lane < 32) my[32 * b + lane] = 1.0 / sc;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const double bs = (a.tempered && a.beta ? a.beta[i] : 1.0) * a.inv_sigma2;
  const int half = lane >> 5;  // which group of 4 samples of a step this lane feeds
  float16v acc[NP];
#pragma unroll
  for (int x = 0; x < NP; ++x) acc[x] = float16v{};
  const int w1 = (int)a.w1;  // sample indices fit in 32 bits (T <= 2^22)
#pragma unroll 1
  for (int s0 = (int)a.w0 + 4 * half; s0 < w1 + 4 * half; s0 += 8) {
    half4 j[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float v = jvalue<MODEL>(q[b], s0 + e);
        j[b][e] = (_Float16)(s0 + e < w1 ? v : 0.f);
      }
    int x = 0;
#pragma unroll
    for (int bi = 0; bi < NB; ++bi)
#pragma unroll
      for (int bj = bi; bj < NB; ++bj, ++x)
        acc[x] = __builtin_amdgcn_mfma_f32_32x32x8f16(j[bi], j[bj], acc[x], 0, 0, 0);
  }
  // flush: lane holds D[r_i][c_j] with c_j = lane % 32, r_i = 8 (r/4) + 4 half + r % 4
  const bool first = a.w0 == 0;
  int x = 0;
#pragma unroll
  for (int bi = 0; bi < NB; ++bi)
#pragma unroll
    for (int bj = bi; bj < NB; ++bj, ++x) {
      const int c = 32 * bj + (lane & 31);
      if (c >= n) continue;
      const double sc = bs * my[c];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int rr = 32 * bi + 8 * (r >> 2) + 4 * half + (r & 3);
        // inside a diagonal block only the upper triangle is taken and
        // mirrored, so the result is exactly symmetric
        if (rr >= n || (bi == bj && rr > c)) continue;
        const double v = (double)acc[x][r] * sc * my[rr];
        if (a.blocks) {
          // a component's block starts at coordinate P k: entries (rr, c) of
          // one component only, at F + (o0 + k) P P
          if (rr / a.P != c / a.P) continue;
          const int64_t bo = fo + (int64_t)(rr / a.P) * a.P * a.P;
          const int pr = rr % a.P, pc = c % a.P;
          double* e1 = a.F + bo + pr * a.P + pc;
          *e1 = first ? v : *e1 + v;
          if (pr != pc) {
            double* e2 = a.F + bo + pc * a.P + pr;
            *e2 = first ? v : *e2 + v;
          }
          continue;
        }
        double* e1 = a.F + fo + (int64_t)rr * n + c;
        *e1 = first ? v : *e1 + v;
        if (rr != c) {
          double* e2 = a.F + fo + (int64_t)c * n + rr;
          *e2 = first ? v : *e2 + v;
        }
      }
    }
}

// ---------------------------------------------------------------- factor
// W = L^{-1} of M = F + diag(ridge) (M = L L^T), the NUTS mass matrix's
// factor with M^{-1} = W^T W. One workgroup of one wave per particle keeps
// the lower triangle of its block packed in LDS (row r at r (r + 1) / 2):
// right-looking Cholesky, one column per step (the subtractions into each
// entry come in column order, as in the row-by-row textbook form), then the
// in-place inversion of the triangle from the last column to the first with
// W_rj = -(sum_{j<k<=r} W_rk L_kj) / L_jj, W_jj = 1 / L_jj. Lanes own rows;
// barriers separate the steps. A pivot that is not > 0 (or NaN) stops the
// factorisation: the block is filled with NaN and a flag is raised.
struct FactorArgs {
  int P;
  int64_t N, M;
  int32_t k_max;
  const int64_t* offsets;
  const int64_t* f_offsets;
  int64_t f_size;
  const double* F;
  double* W;
  double ridge[8];  // per parameter, P <= 8
  int block;        // 0: the whole block; b: its block-diagonal part in b x b blocks
  int* flag;
  const uint8_t* mask;  // [N] or nullptr: particles with mask[i] == 0 are skipped
};

__device__ __forceinline__ int tri(int r, int c) { return r * (r + 1) / 2 + c; }

// Factor of the diagonal block [o, o + m) of particle block Fi (n x n), its
// W written into Wi at the same place; L is the LDS triangle (m (m+1)/2
// doubles). Returns false (in every lane) if a pivot is not > 0.
__device__ bool factor_block(const FactorArgs& a, const double* Fi, double* Wi, int n, int o, int m,
                             double* L, int lane) {
  for (int r = 0; r < m; ++r)
    for (int c = lane; c <= r; c += 64)
      L[tri(r, c)] = Fi[(int64_t)(o + r) * n + o + c] + (r == c ? a.ridge[(o + c) % a.P] : 0.0);
  __syncthreads();
  for (int j = 0; j < m; ++j) {
    const double d = L[tri(j, j)];
    if (!(d > 0.0)) {  // the same value in every lane: a uniform exit
      __syncthreads();
      return false;
    }
    const double ljj = sqrt(d);
    __syncthreads();
    for (int r = j + 1 + lane; r < m; r += 64) L[tri(r, j)] = L[tri(r, j)] / ljj;
    if (lane == 0) L[tri(j, j)] = ljj;
    __syncthreads();
    for (int r = j + 1 + lane; r < m; r += 64) {
      const double lrj = L[tri(r, j)];
      for (int c = j + 1; c <= r; ++c) L[tri(r, c)] = fma(-lrj, L[tri(c, j)], L[tri(r, c)]);
    }
    __syncthreads();
  }
  for (int j = m - 1; j >= 0; --j) {
    const double ljj = L[tri(j, j)];
    double acc[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int r = j + 1 + lane + 64 * t;
      double s = 0.0;
      if (r < m)
        for (int k = j + 1; k <= r; ++k) s = fma(L[tri(r, k)], L[tri(k, j)], s);
      acc[t] = s;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int r = j + 1 + lane + 64 * t;
      if (r < m) L[tri(r, j)] = -acc[t] / ljj;
    }
    if (lane == 0) L[tri(j, j)] = 1.0 / ljj;
    __syncthreads();
  }
  for (int e = lane; e < m * m; e += 64) {
    const int r = e / m, c = e % m;
    Wi[(int64_t)(o + r) * n + o + c] = c <= r ? L[tri(r, c)] : 0.0;
  }
  __syncthreads();  // L is reused by the next block
  return true;
}

__global__ __launch_bounds__(64) void factor_kernel(FactorArgs a) {
  extern __shared__ double L[];
  const int lane = threadIdx.x;
  const int64_t i = blockIdx.x;
  if (i >= a.N) return;
  const int64_t o0 = a.offsets[i], o1 = a.offsets[i + 1];
  if (!(o0 >= 0 && o1 >= o0 && o1 <= a.M && o1 - o0 <= a.k_max)) {
    if (lane == 0) atomicOr(a.flag, kFlagOffsets);
    return;
  }
  const int n = (int)(o1 - o0) * a.P;
  const int64_t fo = a.f_offsets[i];
  if (a.f_offsets[i + 1] - fo != (int64_t)n * n || fo < 0 || fo + (int64_t)n * n > a.f_size) {
    if (lane == 0) atomicOr(a.flag, kFlagOffsets);
    return;
  }
  if (a.mask && !a.mask[i]) return;
  if (n == 0) return;
  const double* Fi = a.F + fo;
  double* Wi = a.W + fo;
  bool ok = true;
  if (a.block == 0) {
    ok = factor_block(a, Fi, Wi, n, 0, n, L, lane);
  } else {
    // block-diagonal part only: the blocks between diagonal blocks are zero
    // in W (when W is F itself they are overwritten after every read)
    for (int o = 0; o < n && ok; o += a.block) ok = factor_block(a, Fi, Wi, n, o, a.block, L, lane);
    if (ok)
      for (int64_t e = lane; e < (int64_t)n * n; e += 64) {
        const int r = (int)(e / n), c = (int)(e % n);
        if (r / a.block != c / a.block) Wi[e] = 0.0;
      }
  }
  if (!ok) {
    if (lane == 0) atomicOr(a.flag, kFlagNotPD);
    for (int64_t e = lane; e < (int64_t)n * n; e += 64) Wi[e] = __builtin_nan("");
  }
}

// One P x P block per thread, W_m = L^{-1} with L L^T = F_m + diag(ridge),
// in registers: the same steps in the same order as factor_block, so a block
// comes out bitwise as the workgroup factor's block mode gives it. A pivot
// that is not > 0 (or NaN) fills the block with NaN and raises the flag.
struct RidgeP {
  double r[8];
};

template <int P>
__global__ __launch_bounds__(256) void factor_blocks_kernel(const double* F, double* W, int64_t M,
                                                            RidgeP rg, int* flag) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const double* f = F + m * P * P;
  double L[P][P];
#pragma unroll
  for (int r = 0; r < P; ++r)
#pragma unroll
    for (int c = 0; c <= r; ++c) L[r][c] = f[r * P + c] + (r == c ? rg.r[c] : 0.0);
  bool ok = true;
#pragma unroll
  for (int j = 0; j < P; ++j) {
    const double d = L[j][j];
    ok = ok && d > 0.0;
    const double ljj = sqrt(d);
#pragma unroll
    for (int r = j + 1; r < P; ++r) L[r][j] = L[r][j] / ljj;
    L[j][j] = ljj;
#pragma unroll
    for (int r = j + 1; r < P; ++r) {
      const double lrj = L[r][j];
#pragma unroll
      for (int c = j + 1; c <= r; ++c) L[r][c] = fma(-lrj, L[c][j], L[r][c]);
    }
  }
#pragma unroll
  for (int j = P - 1; j >= 0; --j) {
    const double ljj = L[j][j];
    double acc[P];
#pragma unroll
    for (int r = j + 1; r < P; ++r) {
      double s = 0.0;
#pragma unroll
      for (int k = j + 1; k <= r; ++k) s = fma(L[r][k], L[k][j], s);
      acc[r] = s;
    }
#pragma unroll
    for (int r = j + 1; r < P; ++r) L[r][j] = -acc[r] / ljj;
    L[j][j] = 1.0 / ljj;
  }
  double* w = W + m * P * P;
#pragma unroll
  for (int r = 0; r < P; ++r)
#pragma unroll
    for (int c = 0; c < P; ++c) w[r * P + c] = !ok ? __builtin_nan("") : (c <= r ? L[r][c] : 0.0);
  if (!ok) atomicOr(flag, kFlagNotPD);
}

}  // namespace

// The population-level mass matrix: the mean of M P x P blocks. Stage one
// sums contiguous row ranges, one lane per entry and four waves taking every
// fourth row, the waves combined in order; stage two adds the range sums in
// order and divides by M. The partition depends only on M and the scratch
// size, so the result is reproducible bit for bit.
constexpr int kPoolWaves = 4;

__global__ __launch_bounds__(64 * kPoolWaves) void pool_partial_kernel(int PP, int64_t M,
                                                                         int64_t rows, const double* F,
                                                                         double* part) {
  __shared__ double sh[kPoolWaves][64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * rows;
  const int64_t r1 = min(M, r0 + rows);
  // four running sums per lane (rows r0 + wid + kPoolWaves (4 j + u) go to
  // sum u), so that four loads are in flight; combined in a fixed order
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  if (lane < PP) {
    int64_t m = r0 + wid;
    for (; m + 3 * kPoolWaves < r1; m += 4 * kPoolWaves)
#pragma unroll
      for (int u = 0; u < 4; ++u) s[u] += F[(m + u * kPoolWaves) * PP + lane];
    for (int u = 0; m < r1; m += kPoolWaves, ++u) s[u] += F[m * PP + lane];
  }
  sh[wid][lane] = (s[0] + s[1]) + (s[2] + s[3]);
  __syncthreads();
  if (wid == 0 && lane < PP) {
    double t = sh[0][lane];
    for (int w = 1; w < kPoolWaves; ++w) t += sh[w][lane];
    part[(size_t)blockIdx.x * PP + lane] = t;
  }
}

// The range sums of the G workgroups: 16 waves take every 16th range each,
// then the first wave adds the 16 wave sums in order.
constexpr int kFinalWaves = 16;
__global__ __launch_bounds__(64 * kFinalWaves) void pool_final_kernel(int PP, int G, int64_t M,
                                                                      const double* part,
                                                                      double* out) {
  __shared__ double sh[kFinalWaves][64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  double s[2] = {0.0, 0.0};
  if (lane < PP) {
    int g = wid, u = 0;
    for (; g < G; g += kFinalWaves, u ^= 1) s[u] += part[(size_t)g * PP + lane];
  }
  sh[wid][lane] = s[0] + s[1];
  __syncthreads();
  if (wid == 0 && lane < PP) {
    double t = sh[0][lane];
    for (int w = 1; w < kFinalWaves; ++w) t += sh[w][lane];
    out[lane] = t / (double)M;
  }
}

hipError_t launch_metric_factor_blocks(int P, int64_t M, const double* F, const double* ridge,
                                       double* W, int* flag, hipStream_t st) {
  if (M == 0) return hipSuccess;
  RidgeP rg{};
  if (P > 8) return hipErrorInvalidValue;
  for (int p = 0; p < P; ++p) rg.r[p] = ridge[p];
  const dim3 grid((unsigned)((M + 255) / 256)), block(256);
  switch (P) {
    case 3: hipLaunchKernelGGL(factor_blocks_kernel<3>, grid, block, 0, st, F, W, M, rg, flag); break;
    case 4: hipLaunchKernelGGL(factor_blocks_kernel<4>, grid, block, 0, st, F, W, M, rg, flag); break;
    case 8: hipLaunchKernelGGL(factor_blocks_kernel<8>, grid, block, 0, st, F, W, M, rg, flag); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_metric_pool(int P, int64_t M, const double* F, double* F_mean, double* part,
                              size_t part_cap, hipStream_t st) {
  const int PP = P * P;
  if (PP > 64 || M < 1) return hipErrorInvalidValue;
  // about 256 rows per workgroup, at most 1024 workgroups and what the scratch
  // holds; with no room for a range sum, one workgroup sums into F_mean itself
  int64_t G = std::min<int64_t>((M + 255) / 256, 1024);
  G = std::min<int64_t>(G, (int64_t)(part_cap / PP));
  if (G < 1) {
    G = 1;
    part = F_mean;
  }
  const int64_t rows = (M + G - 1) / G;
  G = (M + rows - 1) / rows;
  hipLaunchKernelGGL(pool_partial_kernel, dim3((unsigned)G), dim3(64 * kPoolWaves), 0, st, PP, M,
                     rows, F, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pool_final_kernel, dim3(1), dim3(64 * kFinalWaves), 0, st, PP, (int)G, M, part,
                     F_mean);
  return hipGetLastError();
}

size_t factor_lds_bytes(int nmax) { return (size_t)nmax * (nmax + 1) / 2 * sizeof(double); }

hipError_t launch_metric_factor(int P, int64_t N, int64_t M, int32_t k_max,
                                const int64_t* offsets, const int64_t* f_offsets, int64_t f_size,
                                const double* F, const double* ridge, int block, double* W,
                                int* flag, hipStream_t st, const uint8_t* mask) {
  FactorArgs a{};
  a.P = P;
  a.N = N;
  a.M = M;
  a.k_max = k_max;
  a.offsets = offsets;
  a.f_offsets = f_offsets;
  a.f_size = f_size;
  a.F = F;
  a.W = W;
  if (P > 8) return hipErrorInvalidValue;
  for (int p = 0; p < P; ++p) a.ridge[p] = ridge[p];
  a.flag = flag;
  a.mask = mask;
  a.block = block;
  hipLaunchKernelGGL(factor_kernel, dim3((unsigned)N), dim3(64),
                     factor_lds_bytes(block > 0 ? block : k_max * P), st, a);
  return hipGetLastError();
}

hipError_t launch_metric(int model, int P, int64_t N, int64_t M, int64_t T, double t_start,
                         double dt, double inv_sigma2, int32_t k_max, const int64_t* offsets,
                         const double* theta, const double* beta, const int64_t* f_offsets,
                         int64_t f_size, double* F, int64_t split, int blocks, int* flag,
                         hipStream_t st, const uint8_t* mask) {
  MetricArgs a{P, N, M, T, t_start, dt, inv_sigma2, (double)T * dt, k_max, offsets, theta,
               beta, f_offsets, f_size, F, flag, 0, 0, 1, blocks, mask};
  const int nmax = k_max * P;
  const dim3 grid((unsigned)((N + 3) / 4)), block(256);
  const int nb = nmax <= 32 ? 1 : (nmax <= 64 ? 2 : 4);
  if (nmax > 128) return hipErrorInvalidValue;
  const size_t lds = 4 * 32 * (size_t)nb * sizeof(double);
  // one launch per window of samples: later windows add to what earlier ones
  // wrote; with a bridge split the windows stop at the split, and only those
  // after it are tempered
  for (int64_t w0 = 0; w0 < T; w0 = a.w1) {
    const int64_t end = split > 0 && w0 < split ? split : T;  // windows never straddle the split
    a.w0 = w0;
    a.w1 = w0 + kFlushSamples < end ? w0 + kFlushSamples : end;
    a.tempered = split == 0 || w0 >= split ? 1 : 0;
    if (model == SMCX_PULSE) {
      if (nb == 1) hipLaunchKernelGGL((metric_kernel<SMCX_PULSE, 1>), grid, block, lds, st, a);
      else if (nb == 2) hipLaunchKernelGGL((metric_kernel<SMCX_PULSE, 2>), grid, block, lds, st, a);
      else hipLaunchKernelGGL((metric_kernel<SMCX_PULSE, 4>), grid, block, lds, st, a);
    } else {
      if (nb == 1) hipLaunchKernelGGL((metric_kernel<SMCX_GBSINE, 1>), grid, block, lds, st, a);
      else if (nb == 2) hipLaunchKernelGGL((metric_kernel<SMCX_GBSINE, 2>), grid, block, lds, st, a);
      else hipLaunchKernelGGL((metric_kernel<SMCX_GBSINE, 4>), grid, block, lds, st, a);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

}  // namespace smcx
