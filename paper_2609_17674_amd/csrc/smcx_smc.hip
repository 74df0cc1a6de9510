// SMC steps around the likelihood (Sec. "Sequential Monte Carlo",
// Sec. "Algorithm and implementation"): the ESS choice of the next
// inverse temperature with its weights and evidence increment, systematic
// resampling, the accept/reject of birth and death moves (eq. rj_acceptance),
// and the CSR rebuild the last two share.
//
// Population-wide reductions run in one block with a fixed combination order
// (butterfly within a wave, then waves in order), so results do not depend on
// timing. Resampling works on integer weights so that its prefix sums, and
// therefore the ancestors, are exact.
#include "smcx_internal.h"

#include <math.h>

namespace smcx {
namespace {

constexpr int kBlock = 1024;  // single-block kernels
constexpr int kBlockWaves = kBlock / 64;
constexpr double kWeightUnit = 1099511627776.0;  // 2^40: integer weight units

// Sum of a and b over the block, the same bits in every thread.
__device__ void block_sum2(double& a, double& b, double* sh) {
  for (int o = 32; o >= 1; o >>= 1) {  // butterfly: each step is commutative, so all lanes agree
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    sh[w] = a;
    sh[kBlockWaves + w] = b;
  }
  __syncthreads();
  a = 0.0;
  b = 0.0;
  for (int i = 0; i < kBlockWaves; ++i) {
    a += sh[i];
    b += sh[kBlockWaves + i];
  }
}

// Loads per batch in the single-block prefix passes: the loads of a batch are
// in flight together.
constexpr int kScanBatch = 16;

// Prefix sums over the block of the int64 values value(i), i < N, for the
// single-block rebuild passes: wave w takes a contiguous segment of items in
// chunks of 64, lane l holding item c + l, so every load is coalesced and
// kScanBatch chunks are in flight together. out(i, before, through) receives
// the sums of the items before i and through i. Integer sums are exact, so
// the grouping does not change them. Returns the total (all threads).
template <class Val, class Out>
__device__ int64_t block_prefix(int64_t N, Val value, Out out, int64_t* wsum) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t seg = ((N + kBlockWaves - 1) / kBlockWaves + 63) / 64 * 64;
  const int64_t s0 = (int64_t)w * seg, s1 = s0 + seg < N ? s0 + seg : N;
  constexpr int64_t kSpan = 64 * kScanBatch;
  int64_t s = 0;
  for (int64_t c0 = s0; c0 < s1; c0 += kSpan) {
    int64_t v[kScanBatch];
#pragma unroll
    for (int u = 0; u < kScanBatch; ++u) {
      const int64_t i = c0 + 64 * u + lane;
      v[u] = i < s1 ? value(i) : 0;
    }
#pragma unroll
    for (int u = 0; u < kScanBatch; ++u) s += v[u];
  }
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
  if (lane == 0) wsum[w] = s;
  __syncthreads();
  int64_t run = 0, total = 0;
  for (int i = 0; i < kBlockWaves; ++i) {
    const int64_t x = wsum[i];
    run += i < w ? x : 0;
    total += x;
  }
  __syncthreads();  // wsum may be reused
  for (int64_t c0 = s0; c0 < s1; c0 += kSpan) {
    int64_t v[kScanBatch];
#pragma unroll
    for (int u = 0; u < kScanBatch; ++u) {
      const int64_t i = c0 + 64 * u + lane;
      v[u] = i < s1 ? value(i) : 0;
    }
#pragma unroll
    for (int u = 0; u < kScanBatch; ++u) {
      int64_t x = v[u];
      for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
      }
      const int64_t i = c0 + 64 * u + lane;
      if (i < s1) out(i, run + x - v[u], run + x);
      run += __shfl(x, 63);
    }
  }
  return total;
}

__device__ double block_max(double a, double* sh) {
  for (int o = 32; o >= 1; o >>= 1) a = fmax(a, __shfl_xor(a, o));
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[w] = a;
  __syncthreads();
  a = -INFINITY;
  for (int i = 0; i < kBlockWaves; ++i) a = fmax(a, sh[i]);
  return a;
}

// The search stops when the bracket is 1e-14 of the step or a few units in
// the last place of beta, whichever is wider (a step much smaller than
// beta_prev cannot be resolved to 1e-14 of itself).
constexpr double kBracketUlps = 8.0 * 2.220446049250313e-16;
// ... or when the lower end itself meets the condition to 1e-12 in log ESS
// (ESS >= alpha N still holds there).
constexpr double kRootTol = 1e-12;

struct NextBetaArgs {
  int64_t N;
  const double* logl;
  const double* logw_prev;
  double beta_prev, alpha;
  double* beta_out;
  double* logw;
  double* w_norm;
  double* scalars;
};

__device__ __forceinline__ double log_weight(const NextBetaArgs& a, int64_t i, double db) {
  return (a.logw_prev ? a.logw_prev[i] : 0.0) + db * a.logl[i];
}

// ESS of the weights at increment db (eq. ess), with the shift and sum.
__device__ double ess_at(const NextBetaArgs& a, double db, double* sh, double* m_out,
                         double* s1_out) {
  double m = -INFINITY;
  for (int64_t i = threadIdx.x; i < a.N; i += kBlock) m = fmax(m, log_weight(a, i, db));
  m = block_max(m, sh);
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = threadIdx.x; i < a.N; i += kBlock) {
    const double e = exp(log_weight(a, i, db) - m);
    s1 += e;
    s2 += e * e;
  }
  block_sum2(s1, s2, sh);
  if (m_out) *m_out = m;
  if (s1_out) *s1_out = s1;
  return s1 * s1 / s2;
}

// One block: the root of ESS = alpha N on [beta_prev, 1] (eq. ess_target),
// then the weights of eq. incremental_weight and the evidence increment.
__global__ __launch_bounds__(kBlock) void next_beta_kernel(NextBetaArgs a) {
  __shared__ double sh[2 * kBlockWaves];
  const double target = a.alpha * (double)a.N;
  double beta = 1.0;
  int evals = 0;
  const double e1 = ess_at(a, 1.0 - a.beta_prev, sh, nullptr, nullptr);
  if (!(e1 >= target)) {
    // The root of ESS(beta) = target in [beta_prev, 1], kept bracketed:
    // ESS(lo) >= target > ESS(hi). Each step tries the regula-falsi point of
    // f = log(ESS / target) (the Illinois variant halves the value kept at an
    // end that stays twice in a row), or the midpoint where that point is not
    // strictly inside; about ten evaluations reach the bracket width the
    // plain bisection reaches in fifty. The result is lo, a tested point, so
    // ESS(beta) >= target holds as for the bisection.
    double lo = a.beta_prev, hi = 1.0;
    const double f0 = a.logw_prev ? log(ess_at(a, 0.0, sh, nullptr, nullptr) / target)
                                  : log((double)a.N / target);
    double flo = f0, fhi = log(e1 / target);
    if (!(flo >= 0.0)) {
      // the previous weights alone are below the target: plain bisection
      // (it ends next to beta_prev)
      bool moved = false;
      for (int it = 0; it < 60; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (!(mid > lo && mid < hi)) break;
        const double e = ess_at(a, mid - a.beta_prev, sh, nullptr, nullptr);
        ++evals;
        if (e >= target) {
          lo = mid;
          moved = true;
        } else {
          hi = mid;
        }
      }
      beta = moved ? lo : hi;
    } else {
      int side = 0;
      for (int it = 0; it < 100; ++it) {
        double x = fhi == fhi && flo - fhi > 0.0 ? hi - fhi * (hi - lo) / (fhi - flo) : 0.5 * (lo + hi);
        if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
        if (!(x > lo && x < hi)) break;
        const double fx = log(ess_at(a, x - a.beta_prev, sh, nullptr, nullptr) / target);
        ++evals;
        if (fx >= 0.0) {
          lo = x;
          flo = fx;
          if (side == 1) fhi *= 0.5;
          side = 1;
        } else {
          hi = x;
          fhi = fx == fx ? fx : -INFINITY;
          if (side == -1) flo *= 0.5;
          side = -1;
        }
        if (hi - lo <= fmax(1e-14 * (hi - a.beta_prev), kBracketUlps * hi) ||
            (fx >= 0.0 && fx <= kRootTol))
          break;
      }
      beta = lo;
    }
  }
  const double db = beta - a.beta_prev;
  double m, s1;
  const double ess = ess_at(a, db, sh, &m, &s1);
  for (int64_t i = threadIdx.x; i < a.N; i += kBlock) {
    const double lw = log_weight(a, i, db);
    a.logw[i] = lw;
    a.w_norm[i] = exp(lw - m) / s1;
    if (a.beta_out) a.beta_out[i] = beta;
  }
  double lse_prev = log((double)a.N);
  if (a.logw_prev) {
    double mp = -INFINITY;
    for (int64_t i = threadIdx.x; i < a.N; i += kBlock) mp = fmax(mp, a.logw_prev[i]);
    mp = block_max(mp, sh);
    double sp = 0.0, unused = 0.0;
    for (int64_t i = threadIdx.x; i < a.N; i += kBlock) sp += exp(a.logw_prev[i] - mp);
    block_sum2(sp, unused, sh);
    lse_prev = mp + log(sp);
  }
  if (threadIdx.x == 0) {
    a.scalars[0] = beta;
    a.scalars[1] = ess;
    a.scalars[2] = m + log(s1) - lse_prev;
    a.scalars[3] = (double)evals;
  }
}

// ---------------------------------------------------------------- next beta, many workgroups
// The same search for uniform previous weights (no logw_prev), spread over
// the device: one launch per ESS evaluation. A launch's workgroups each sum
// exp(db l_i - m) and its square over their slice of particles (m = db
// max_i l_i, exact since db >= 0); the next launch's workgroups first add the
// range sums in slice order and take the search's next step from them, every
// workgroup computing the same bits (so they agree on the point to evaluate),
// and workgroup 0 records the step. A fixed number of evaluation launches is
// queued; the ones after the search has ended return at once, and a one-block
// pass finishes a search that would still be running. The evaluation at the
// bracket's lower end is kept, so the weights need no further pass.
constexpr int kNbBlock = 256;
constexpr int kNbPer = 4;                      // particles per thread per launch
constexpr int kNbSlice = kNbBlock * kNbPer;    // particles per workgroup
constexpr int kNbLaunches = 12;                // evaluation launches queued
constexpr int kNbState = 16;                   // doubles per search state

// search state (doubles): lo, hi, flo, fhi, x (point evaluated by the launch),
// side, evals, phase (0: evaluate beta = 1; 1: bracketing search; 2: done),
// beta, s1_lo, s2_lo (sums at beta), L (max l)
enum { kLo, kHi, kFlo, kFhi, kX, kSide, kEvals, kPhase, kBeta, kS1, kS2, kL };

struct NbMultiArgs {
  int64_t N;
  const double* logl;
  double beta_prev, alpha, target;
  double* beta_out;
  double* logw;
  double* w_norm;
  double* scalars;
  double* state;  // [2][kNbState]
  double* pmax;   // [G]
  double* psum;   // [2][G][2]
  int G;
};

__device__ __forceinline__ double nb_max_l(const NbMultiArgs& a) {
  double L = -INFINITY;
  for (int g = 0; g < a.G; ++g) L = fmax(L, a.pmax[g]);
  return L;
}

// The search's step after an evaluation at st[kX] with sums (s1, s2); the
// same arithmetic as next_beta_kernel's bracketing search.
__device__ void nb_advance(const NbMultiArgs& a, double* st, double s1, double s2) {
  const double ess = s1 * s1 / s2;
  if (st[kPhase] == 0.0) {  // the evaluation at beta = 1
    if (ess >= a.target) {
      st[kPhase] = 2.0;
      st[kBeta] = 1.0;
      st[kS1] = s1;
      st[kS2] = s2;
      return;
    }
    st[kLo] = a.beta_prev;
    st[kHi] = 1.0;
    st[kFlo] = log((double)a.N / a.target);
    st[kFhi] = log(ess / a.target);
    st[kSide] = 0.0;
    st[kPhase] = 1.0;
    // sums at beta_prev: uniform weights
    st[kS1] = (double)a.N;
    st[kS2] = (double)a.N;
  } else {
    const double x = st[kX];
    const double fx = log(ess / a.target);
    st[kEvals] += 1.0;
    if (fx >= 0.0) {
      st[kLo] = x;
      st[kFlo] = fx;
      if (st[kSide] == 1.0) st[kFhi] *= 0.5;
      st[kSide] = 1.0;
      st[kS1] = s1;
      st[kS2] = s2;
    } else {
      st[kHi] = x;
      st[kFhi] = fx == fx ? fx : -INFINITY;
      if (st[kSide] == -1.0) st[kFlo] *= 0.5;
      st[kSide] = -1.0;
    }
    if (st[kHi] - st[kLo] <= fmax(1e-14 * (st[kHi] - a.beta_prev), kBracketUlps * st[kHi]) ||
        (fx >= 0.0 && fx <= kRootTol) || st[kEvals] >= 100.0) {
      st[kPhase] = 2.0;
      st[kBeta] = st[kLo];
      return;
    }
  }
  const double lo = st[kLo], hi = st[kHi], flo = st[kFlo], fhi = st[kFhi];
  double x = fhi == fhi && flo - fhi > 0.0 ? hi - fhi * (hi - lo) / (fhi - flo) : 0.5 * (lo + hi);
  if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
  if (!(x > lo && x < hi)) {
    st[kPhase] = 2.0;
    st[kBeta] = lo;
    return;
  }
  st[kX] = x;
}

__global__ __launch_bounds__(kNbBlock) void nb_max_kernel(NbMultiArgs a) {
  __shared__ double sh[kNbBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kNbSlice;
  double m = -INFINITY;
#pragma unroll
  for (int u = 0; u < kNbPer; ++u) {
    const int64_t i = base + u * kNbBlock + threadIdx.x;
    if (i < a.N) m = fmax(m, a.logl[i]);
  }
  for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sh[0];
    for (int w = 1; w < kNbBlock / 64; ++w) r = fmax(r, sh[w]);
    a.pmax[blockIdx.x] = r;
  }
}

// Launch k: take the step after launch k - 1's evaluation (k > 0), then
// evaluate the new point.
__global__ __launch_bounds__(kNbBlock) void nb_eval_kernel(NbMultiArgs a, int k) {
  __shared__ double st[kNbState];
  __shared__ double sh[2 * (kNbBlock / 64)];
  if (threadIdx.x == 0) {
    if (k == 0) {
      for (int q = 0; q < kNbState; ++q) st[q] = 0.0;
      st[kX] = 1.0;
      st[kL] = nb_max_l(a);
    } else {
      const double* prev = a.state + ((k - 1) & 1) * kNbState;
      for (int q = 0; q < kNbState; ++q) st[q] = prev[q];
      if (st[kPhase] != 2.0) {
        const double* ps = a.psum + (size_t)((k - 1) & 1) * a.G * 2;
        double s1 = 0.0, s2 = 0.0;
        for (int g = 0; g < a.G; ++g) {
          s1 += ps[2 * g];
          s2 += ps[2 * g + 1];
        }
        nb_advance(a, st, s1, s2);
      }
    }
    if (blockIdx.x == 0) {
      double* cur = a.state + (k & 1) * kNbState;
      for (int q = 0; q < kNbState; ++q) cur[q] = st[q];
    }
  }
  __syncthreads();
  if (st[kPhase] == 2.0) return;
  const double db = st[kX] - a.beta_prev;
  const double m = db * st[kL];
  const int64_t base = (int64_t)blockIdx.x * kNbSlice;
  double s1 = 0.0, s2 = 0.0;
#pragma unroll
  for (int u = 0; u < kNbPer; ++u) {
    const int64_t i = base + u * kNbBlock + threadIdx.x;
    if (i < a.N) {
      const double e = exp(db * a.logl[i] - m);
      s1 += e;
      s2 += e * e;
    }
  }
  for (int o = 32; o >= 1; o >>= 1) {
    s1 += __shfl_xor(s1, o);
    s2 += __shfl_xor(s2, o);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[threadIdx.x >> 6] = s1;
    sh[kNbBlock / 64 + (threadIdx.x >> 6)] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t1 = 0.0, t2 = 0.0;
    for (int w = 0; w < kNbBlock / 64; ++w) {
      t1 += sh[w];
      t2 += sh[kNbBlock / 64 + w];
    }
    double* ps = a.psum + (size_t)(k & 1) * a.G * 2;
    ps[2 * blockIdx.x] = t1;
    ps[2 * blockIdx.x + 1] = t2;
  }
}

// One block: take the step after the last queued evaluation and, should the
// search still be running, finish it with block-wide evaluations.
__global__ __launch_bounds__(kBlock) void nb_finish_kernel(NbMultiArgs a) {
  __shared__ double st[kNbState];
  __shared__ double sh[2 * kBlockWaves];
  constexpr int k = kNbLaunches;  // the step after launch kNbLaunches - 1
  if (threadIdx.x == 0) {
    const double* prev = a.state + ((k - 1) & 1) * kNbState;
    for (int q = 0; q < kNbState; ++q) st[q] = prev[q];
    if (st[kPhase] != 2.0) {
      const double* ps = a.psum + (size_t)((k - 1) & 1) * a.G * 2;
      double s1 = 0.0, s2 = 0.0;
      for (int g = 0; g < a.G; ++g) {
        s1 += ps[2 * g];
        s2 += ps[2 * g + 1];
      }
      nb_advance(a, st, s1, s2);
    }
  }
  __syncthreads();
  while (st[kPhase] != 2.0) {
    const double db = st[kX] - a.beta_prev;
    const double m = db * st[kL];
    double s1 = 0.0, s2 = 0.0;
    for (int64_t i = threadIdx.x; i < a.N; i += kBlock) {
      const double e = exp(db * a.logl[i] - m);
      s1 += e;
      s2 += e * e;
    }
    block_sum2(s1, s2, sh);  // the same bits in every thread
    __syncthreads();
    if (threadIdx.x == 0) nb_advance(a, st, s1, s2);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* cur = a.state + (k & 1) * kNbState;
    for (int q = 0; q < kNbState; ++q) cur[q] = st[q];
  }
}

// Weights at the chosen beta (eq. incremental_weight), normalised by the
// kept sums, and the scalars.
__global__ __launch_bounds__(kNbBlock) void nb_weights_kernel(NbMultiArgs a) {
  const double* st = a.state + (kNbLaunches & 1) * kNbState;
  const double beta = st[kBeta], db = beta - a.beta_prev;
  const double m = db * st[kL], s1 = st[kS1];
  const int64_t base = (int64_t)blockIdx.x * kNbSlice;
#pragma unroll
  for (int u = 0; u < kNbPer; ++u) {
    const int64_t i = base + u * kNbBlock + threadIdx.x;
    if (i < a.N) {
      const double lw = db * a.logl[i];
      a.logw[i] = lw;
      a.w_norm[i] = exp(lw - m) / s1;
      if (a.beta_out) a.beta_out[i] = beta;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.scalars[0] = beta;
    a.scalars[1] = s1 * s1 / st[kS2];
    a.scalars[2] = m + log(s1) - log((double)a.N);
    a.scalars[3] = st[kEvals];
  }
}

// ---------------------------------------------------------------- CSR rebuild
// Output particle j takes rows src_row[j] .. src_row[j] + src_len[j] - 1 of
// theta, without row skip[j] (local index, -1 = none), followed by row j of
// theta_add when append[j] != 0.
struct RebuildArgs {
  int64_t N, M;
  int P;
  int32_t k_max;
  const int64_t* offsets;  // source population
  const double* theta;
  int64_t* src_row;   // [N] workspace
  int32_t* src_len;   // [N]
  int32_t* skip;      // [N]
  int32_t* append;    // [N]
  int64_t* count;     // [N] rows of output particle j
  const double* theta_add;  // [N][P] rows appended (births)
  int64_t* offsets_out;     // [N + 1]
  double* theta_out;        // [m_cap][P]
  int64_t m_cap;
  int* flag;
};

// Rows of source particle i, validated against [0, M] and k_max (an invalid
// particle contributes no rows and raises the flag).
__device__ __forceinline__ bool source_rows(const RebuildArgs& a, int64_t i, int64_t& row,
                                            int32_t& len) {
  const int64_t o0 = a.offsets[i], o1 = a.offsets[i + 1];
  if (!(o0 >= 0 && o1 >= o0 && o1 <= a.M && o1 - o0 <= a.k_max)) {
    atomicOr(a.flag, (o1 - o0 > a.k_max && o0 >= 0 && o1 <= a.M) ? kFlagKMax : kFlagOffsets);
    row = 0;
    len = 0;
    return false;
  }
  row = o0;
  len = (int32_t)(o1 - o0);
  return true;
}

// Exclusive prefix sum of count[0..N) into offsets_out[0..N] (one block).
__global__ __launch_bounds__(kBlock) void csr_scan_kernel(RebuildArgs a) {
  __shared__ int64_t wsum[kBlockWaves];
  const int64_t total = block_prefix(
      a.N, [&](int64_t i) { return a.count[i]; },
      [&](int64_t i, int64_t before, int64_t) { a.offsets_out[i] = before; }, wsum);
  if (threadIdx.x == 0) {
    a.offsets_out[a.N] = total;
    if (total > a.m_cap) atomicOr(a.flag, kFlagCapacity);
  }
}

// One wave per output particle copies its rows; rows at or past m_cap are
// not written (the capacity flag is raised by the scan).
__global__ __launch_bounds__(256) void csr_gather_kernel(RebuildArgs a) {
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= a.N) return;
  const int64_t start = a.offsets_out[j];
  const int64_t row = a.src_row[j];
  const int32_t len = a.src_len[j], skip = a.skip[j];
  const int P = a.P;
  for (int64_t x = lane; x < (int64_t)len * P; x += 64) {
    const int32_t k = (int32_t)(x / P);
    const int p = (int)(x - (int64_t)k * P);
    if (k == skip) continue;
    const int64_t out = start + k - (skip >= 0 && k > skip ? 1 : 0);
    if (out < a.m_cap) a.theta_out[out * P + p] = a.theta[(row + k) * P + p];
  }
  if (a.append[j] && lane < P) {
    const int64_t out = start + len - (skip >= 0 ? 1 : 0);
    if (out < a.m_cap) a.theta_out[out * P + lane] = a.theta_add[j * P + lane];
  }
}

// ---------------------------------------------------------------- resampling
struct ResampleArgs {
  RebuildArgs r;
  const double* w_norm;
  double u;
  int64_t* cum;       // [N] inclusive prefix sums of the integer weights
  int32_t* ancestors; // [N]
};

// Integer weights c_i = round(w_i 2^40) (0 unless w_i > 0) and their inclusive
// prefix sums, exact in int64 (one block).
__device__ __forceinline__ int64_t weight_units(double w) {
  return w > 0.0 ? (int64_t)rint((w < 1.0 ? w : 1.0) * kWeightUnit) : 0;
}

__global__ __launch_bounds__(kBlock) void resample_prefix_kernel(ResampleArgs a) {
  __shared__ int64_t wsum[kBlockWaves];
  const int64_t total = block_prefix(
      a.r.N, [&](int64_t i) { return weight_units(a.w_norm[i]); },
      [&](int64_t i, int64_t, int64_t through) { a.cum[i] = through; }, wsum);
  if (threadIdx.x == 0 && total <= 0) atomicOr(a.r.flag, kFlagWeights);
}

// Offspring j: position U_j = floor(((j + u) C) / N), ancestor = first i with
// cum[i] > U_j (binary search); then its rows for the rebuild.
__global__ __launch_bounds__(256) void resample_ancestor_kernel(ResampleArgs a) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t N = a.r.N;
  if (j >= N) return;
  const int64_t total = a.cum[N - 1];
  int64_t anc = j;  // no positive weight: every particle keeps itself (flagged)
  if (total > 0) {
    int64_t U = (int64_t)floor(((double)j + a.u) * (double)total / (double)N);
    if (U >= total) U = total - 1;
    int64_t lo = 0, hi = N - 1;  // cum[hi] = total > U
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      if (a.cum[mid] > U) hi = mid;
      else lo = mid + 1;
    }
    anc = lo;
  }
  a.ancestors[j] = (int32_t)anc;
  int64_t row;
  int32_t len;
  source_rows(a.r, anc, row, len);
  a.r.src_row[j] = row;
  a.r.src_len[j] = len;
  a.r.skip[j] = -1;
  a.r.append[j] = 0;
  a.r.count[j] = len;
}

// ---------------------------------------------------------------- birth/death
struct RjArgs {
  RebuildArgs r;
  const int8_t* move;
  const int32_t* death_idx;
  const double* dlogl_birth;
  const double* dlogl_death;
  const double* log_u;
  int32_t k_lo, k_hi;
  double log_pd_over_pb;
  int8_t* accepted;
};

// Accept/reject per particle: log alpha = dlogl_birth + log(p_death/p_birth)
// for a birth with K + 1 <= k_hi, dlogl_death - log(p_death/p_birth) for a
// death of a valid index with K - 1 >= k_lo (the reading of eq. rj_acceptance
// for exchangeable components, a birth proposal equal to the prior and a
// uniform prior on K); accepted when log_u < log alpha.
__global__ __launch_bounds__(256) void rj_decide_kernel(RjArgs a) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.r.N) return;
  int64_t row;
  int32_t K;
  const bool ok = source_rows(a.r, i, row, K);
  const int mv = a.move[i];
  bool acc = false;
  int32_t skip = -1;
  if (ok && mv == 1 && a.r.theta_add && a.dlogl_birth && K + 1 <= a.k_hi) {
    acc = a.log_u[i] < a.dlogl_birth[i] + a.log_pd_over_pb;
  } else if (ok && mv == 2 && a.death_idx && a.dlogl_death && K - 1 >= a.k_lo) {
    const int32_t j = a.death_idx[i];
    if (j >= 0 && j < K) {
      acc = a.log_u[i] < a.dlogl_death[i] - a.log_pd_over_pb;
      if (acc) skip = j;
    }
  }
  a.accepted[i] = acc ? 1 : 0;
  a.r.src_row[i] = row;
  a.r.src_len[i] = K;
  a.r.skip[i] = skip;
  a.r.append[i] = (acc && mv == 1) ? 1 : 0;
  a.r.count[i] = K + (acc ? (mv == 1 ? 1 : -1) : 0);
}

hipError_t launch_rebuild(const RebuildArgs& r, hipStream_t st) {
  hipLaunchKernelGGL(csr_scan_kernel, dim3(1), dim3(kBlock), 0, st, r);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(csr_gather_kernel, dim3((unsigned)((r.N + 3) / 4)), dim3(256), 0, st, r);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_next_beta(int64_t N, const double* logl, const double* logw_prev,
                            double beta_prev, double alpha, double* beta_out, double* logw,
                            double* w_norm, double* scalars, double* work, size_t work_cap,
                            hipStream_t st) {
  const int64_t G = (N + kNbSlice - 1) / kNbSlice;
  if (logw_prev || !work || work_cap < (size_t)(2 * kNbState + 5 * G)) {
    NextBetaArgs a{N, logl, logw_prev, beta_prev, alpha, beta_out, logw, w_norm, scalars};
    hipLaunchKernelGGL(next_beta_kernel, dim3(1), dim3(kBlock), 0, st, a);
    return hipGetLastError();
  }
  NbMultiArgs a;
  a.N = N;
  a.logl = logl;
  a.beta_prev = beta_prev;
  a.alpha = alpha;
  a.target = alpha * (double)N;
  a.beta_out = beta_out;
  a.logw = logw;
  a.w_norm = w_norm;
  a.scalars = scalars;
  a.state = work;
  a.pmax = work + 2 * kNbState;
  a.psum = a.pmax + G;
  a.G = (int)G;
  const dim3 grid((unsigned)G), block(kNbBlock);
  hipLaunchKernelGGL(nb_max_kernel, grid, block, 0, st, a);
  for (int k = 0; k < kNbLaunches; ++k) hipLaunchKernelGGL(nb_eval_kernel, grid, block, 0, st, a, k);
  hipLaunchKernelGGL(nb_finish_kernel, dim3(1), dim3(kBlock), 0, st, a);
  hipLaunchKernelGGL(nb_weights_kernel, grid, block, 0, st, a);
  return hipGetLastError();
}

hipError_t launch_resample(const SmcWork& w, int model, int32_t k_max, int64_t N,
                           const int64_t* offsets, int64_t M, const double* theta,
                           const double* w_norm, double u, int64_t m_cap, int32_t* ancestors,
                           int64_t* offsets_out, double* theta_out, int* flag, hipStream_t st) {
  ResampleArgs a;
  a.r = RebuildArgs{N, M, n_params(model), k_max, offsets, theta, w.src_row, w.src_len, w.skip,
                    w.append, w.count, nullptr, offsets_out, theta_out, m_cap, flag};
  a.w_norm = w_norm;
  a.u = u;
  a.cum = w.cum;
  a.ancestors = ancestors;
  hipLaunchKernelGGL(resample_prefix_kernel, dim3(1), dim3(kBlock), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(resample_ancestor_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st,
                     a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_rebuild(a.r, st);
}

hipError_t launch_rj_apply(const SmcWork& w, int model, int32_t k_max, int64_t N,
                           const int64_t* offsets, int64_t M, const double* theta,
                           const int8_t* move, const double* theta_birth, const int32_t* death_idx,
                           const double* dlogl_birth, const double* dlogl_death,
                           const double* log_u, int32_t k_lo, int32_t k_hi, double log_pd_over_pb,
                           int64_t m_cap, int64_t* offsets_out, double* theta_out,
                           int8_t* accepted, int* flag, hipStream_t st) {
  RjArgs a;
  a.r = RebuildArgs{N, M, n_params(model), k_max, offsets, theta, w.src_row, w.src_len, w.skip,
                    w.append, w.count, theta_birth, offsets_out, theta_out, m_cap, flag};
  a.move = move;
  a.death_idx = death_idx;
  a.dlogl_birth = dlogl_birth;
  a.dlogl_death = dlogl_death;
  a.log_u = log_u;
  a.k_lo = k_lo;
  a.k_hi = k_hi;
  a.log_pd_over_pb = log_pd_over_pb;
  a.accepted = accepted;
  hipLaunchKernelGGL(rj_decide_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_rebuild(a.r, st);
}

}  // namespace smcx
