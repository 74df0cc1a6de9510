// C ABI of libsmcx: problem handle, argument checks, workspace, launches.
#include <hip/hip_runtime.h>

#include <cerrno>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <climits>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/smcx.h"
#include "smcx_internal.h"
#include "smcx_problem.h"

using smcx::Tiling;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

}  // namespace

namespace smcx {
int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}
}  // namespace smcx

namespace {

int hip_fail(hipError_t e, const char* what) {
  return fail(SMCX_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool capturing(hipStream_t st) {
  hipStreamCaptureStatus s = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &s) != hipSuccess) return false;
  return s != hipStreamCaptureStatusNone;
}

int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// The cap on one handle's device workspace: SMCX_WORKSPACE_MAX in bytes,
// with an optional k, m or g suffix (2^10, 2^20, 2^30); unset means none.
// Returns SMCX_OK when `bytes` fits, SMCX_ENOMEM when it does not and
// SMCX_EINVAL for a value that does not parse; nothing is allocated either way.
int check_workspace(size_t bytes, const char* what) {
  const char* v = std::getenv("SMCX_WORKSPACE_MAX");
  if (!v || !*v) return SMCX_OK;
  char* end = nullptr;
  errno = 0;
  const unsigned long long n = std::strtoull(v, &end, 10);
  unsigned shift = 0;
  if (end && (*end == 'k' || *end == 'K')) shift = 10, ++end;
  else if (end && (*end == 'm' || *end == 'M')) shift = 20, ++end;
  else if (end && (*end == 'g' || *end == 'G')) shift = 30, ++end;
  if (errno || end == v || *end || (shift && n > (~0ull >> shift)))
    return fail(SMCX_EINVAL, "SMCX_WORKSPACE_MAX = '%s' is not a byte count", v);
  const unsigned long long cap = n << shift;
  if (bytes > cap)
    return fail(SMCX_ENOMEM, "%s needs %zu bytes of device workspace, over SMCX_WORKSPACE_MAX = %llu",
                what, bytes, cap);
  return SMCX_OK;
}

}  // namespace

// Default tiling per (model, kind, T). It depends only on the model and the
// length of the sample axis, never on N, so a particle's arithmetic (and
// hence its result bit pattern) does not depend on the batch it is in.
Tiling smcx::default_tiling(int model, int kind, int64_t T) {
  Tiling t;
  if (model == SMCX_PULSE) {
    if (kind == kDelta)
      t.S = 16;
    else
      t.S = T >= 2048 ? 32 : (T >= 512 ? 16 : 8);
    const int64_t tile = 64 * (int64_t)t.S;
    t.chunk_len = T <= 8192 ? round_up(T, tile) : round_up(8192, tile);
  } else {
    t.S = 16;
    t.chunk_len = 4096;
  }
  t.nch = (int)((T + t.chunk_len - 1) / t.chunk_len);
  t.sorted = 1;
  return t;
}

namespace {

// Workspace capacities fixed at create: any tiling with at most this many
// chunks per particle fits the partial-sum buffers.
int cap_chunks(int64_t T) { return (int)std::min<int64_t>(64, (T + 1023) / 1024); }
int cap_chunks_grad(int64_t T) { return (int)std::min<int64_t>(32, (T + 4095) / 4096); }

Tiling with_range(Tiling t, int64_t len) {
  t.nch = len <= 0 ? 0 : (int)((len + t.chunk_len - 1) / t.chunk_len);
  return t;
}

}  // namespace


namespace {

void free_problem(smcx_problem* p) {
  if (!p) return;
  for (hipEvent_t e : p->prof_ev) (void)hipEventDestroy(e);
  for (hipGraphExec_t g : p->nuts_graph)
    if (g) (void)hipGraphExecDestroy(g);
  if (p->nuts_capture) (void)hipStreamDestroy(p->nuts_capture);
  (void)hipFree(p->nuts_vec);
  (void)hipFree(p->nuts_state);
  (void)hipFree(p->nuts_logl);
  (void)hipFree(p->nuts_active);
  (void)hipFree(p->nuts_dir);
  (void)hipFree(p->nuts_count);
  (void)hipFree(p->nuts_list);
  (void)hipFree(p->d32);
  (void)hipFree(p->d64);
  (void)hipFree(p->fd_data);
  (void)hipFree(p->fd_src);
  (void)hipFree(p->fd_table);
  (void)hipFree(p->order);
  (void)hipFree(p->n_active);
  (void)hipFree(p->prep_hist);
  (void)hipFree(p->smc.cum);
  (void)hipFree(p->smc.src_row);
  (void)hipFree(p->smc.src_len);
  (void)hipFree(p->smc.skip);
  (void)hipFree(p->smc.append);
  (void)hipFree(p->smc.count);
  (void)hipFree(p->flag);
  (void)hipFree(p->part);
  (void)hipFree(p->part_g);
  (void)hipFree(p->rbuf);
  (void)hipFree(p->bpart);
  delete p;
}

int check_pop(const smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
              const double* theta) {
  if (!p) return fail(SMCX_EINVAL, "problem handle is NULL");
  if (N < 0) return fail(SMCX_EINVAL, "N = %lld is negative", (long long)N);
  if (N > p->n_max)
    return fail(SMCX_EINVAL, "N = %lld exceeds n_max = %lld of the handle", (long long)N,
                (long long)p->n_max);
  if (M < 0) return fail(SMCX_EINVAL, "M = %lld is negative", (long long)M);
  if (M > p->m_max)
    return fail(SMCX_EINVAL, "M = %lld exceeds m_max = %lld of the handle", (long long)M,
                (long long)p->m_max);
  if (N > 0 && !offsets) return fail(SMCX_EINVAL, "offsets is NULL");
  if (M > 0 && !theta) return fail(SMCX_EINVAL, "theta is NULL");
  return SMCX_OK;
}

// Bracket the batched kernels of one call with events when profiling is on.
// With `inner` the stop event is recorded by the launcher right after the
// population kernel (before any pass that combines chunk partials).
struct ProfScope {
  smcx_problem* p;
  hipStream_t st;
  bool on;
  bool inner = false;
  ProfScope(smcx_problem* p_, hipStream_t st_) : p(p_), st(st_), on(false) {
    if (p->prof_on && 2 * (size_t)p->prof_n + 1 < p->prof_ev.size() && !capturing(st)) {
      on = hipEventRecord(p->prof_ev[2 * p->prof_n], st) == hipSuccess;
    }
  }
  ~ProfScope() {
    if (!on) return;
    if (inner || hipEventRecord(p->prof_ev[2 * p->prof_n + 1], st) == hipSuccess) ++p->prof_n;
  }
};

// A batched launch under the profiling events. On the frequency-domain model
// the pass that writes the source constants runs before the first event
// when profiling is on, so that the events time the likelihood kernel alone.
// `pop` marks launches of the time-domain population kernel, whose launcher
// records the stop event itself (a.prof_stop).
template <class Launch>
hipError_t profiled(smcx_problem* p, smcx::PopArgs a, hipStream_t st, Launch launch,
                    bool pop = false) {
  if (p->fd && p->prof_on) {
    hipError_t e = smcx::launch_fd_src(a, st);
    if (e != hipSuccess) return e;
    a.fd_src_ready = 1;
  }
  ProfScope ps(p, st);
  if (ps.on && pop && !p->fd) {
    a.prof_stop = p->prof_ev[2 * p->prof_n + 1];
    ps.inner = true;
  }
  hipError_t e = launch(a);
  if (e != hipSuccess) ps.inner = false;
  return e;
}

smcx::PopArgs base_args(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
                        const double* theta, const double* beta, const Tiling& t, int64_t s_lo,
                        int64_t s_hi, double k0) {
  smcx::PopArgs a;
  std::memset(&a, 0, sizeof(a));
  a.M = M;
  a.k0 = k0;
  a.d32 = p->d32;
  a.s_lo = s_lo;
  a.s_hi = s_hi;
  a.t_start = p->t_start;
  a.dt = p->dt;
  a.inv_sigma2 = p->inv_sigma2;
  a.offsets = offsets;
  a.theta = theta;
  a.beta = beta;
  a.N = N;
  a.k_max = p->k_max;
  a.m_max = p->m_max;
  a.order = t.sorted ? p->order : nullptr;
  a.persist = t.sorted == 2;
  a.n_cu = p->n_cu;
  a.n_active = p->n_active;
  a.nch = t.nch;
  a.chunk_len = t.chunk_len;
  a.part = p->part;
  a.part_g = p->part_g;
  a.flag = p->flag;
  if (p->fd) {
    a.fd_data = p->fd_data;
    a.fd_src = p->fd_src;
    a.fd_table = p->fd_table;
    a.fd_k0 = p->fd_k0;
    a.fd_B = p->fd_B;
    a.fd_T_obs = p->fd_T_obs;
    a.fd_scale = p->fd_T_obs / 64.0;
    a.n_cu = p->n_cu;
    // three workgroups of the gradient kernel fit a compute unit at once; its
    // grid holds at least this many (six per unit, or one per four particles)
    a.fd_split = std::min<int64_t>(3 * (int64_t)p->n_cu, (N + 3) / 4);
    if (p->partner) {
      const smcx_problem* q = p->partner;
      a.fd_bridge = 1;
      a.fd2_data = q->fd_data;
      a.fd2_table = q->fd_table;
      a.fd2_k0 = q->fd_k0;
      a.fd2_B = q->fd_B;
      a.fd2_T_obs = q->fd_T_obs;
      a.fd2_cnorm = q->inv_sigma2;
    }
  }
  return a;
}

// Coarse-grid constants of the frequency-domain model for observation time
// T_obs: per envelope sample t_j = j T_obs / 64 the symmetric detector tensors
// of the A and E channels, cos and sin of the orbital phase, t_j; then the
// per-lane FFT twiddles. The constellation follows the first-order
// circular-orbit solution (guiding centre on the 1 AU circle, arms of length L
// in a plane inclined by 60 degrees to the ecliptic); the Michelson tensor
// with vertex k is (u u - v v) / 2 for the unit vectors towards spacecraft
// k+1 and k+2, A = (M_2 - M_0) / sqrt(2), E = (M_0 - 2 M_1 + M_2) / sqrt(6).
void fd_table_host(double T_obs, std::vector<double>& tab) {
  const double kPi = 3.14159265358979323846, R = 1.495978707e11, L = 2.5e9, year = 31557600.0;
  const double ecc = L / (2.0 * std::sqrt(3.0) * R);
  tab.assign(smcx::kFdTableSize, 0.0);
  for (int j = 0; j < 64; ++j) {
    const double t = j * T_obs / 64.0, a = 2.0 * kPi * t / year;
    double x[3][3];
    for (int k = 0; k < 3; ++k) {
      const double b = 2.0 * kPi * k / 3.0;
      x[k][0] = R * std::cos(a) + 0.5 * ecc * R * (std::cos(2.0 * a - b) - 3.0 * std::cos(b));
      x[k][1] = R * std::sin(a) + 0.5 * ecc * R * (std::sin(2.0 * a - b) - 3.0 * std::sin(b));
      x[k][2] = -std::sqrt(3.0) * ecc * R * std::cos(a - b);
    }
    double M[3][3][3];
    for (int k = 0; k < 3; ++k) {
      double u[3], v[3], nu = 0.0, nv = 0.0;
      for (int c = 0; c < 3; ++c) {
        u[c] = x[(k + 1) % 3][c] - x[k][c];
        v[c] = x[(k + 2) % 3][c] - x[k][c];
        nu += u[c] * u[c];
        nv += v[c] * v[c];
      }
      nu = std::sqrt(nu);
      nv = std::sqrt(nv);
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) M[k][r][c] = 0.5 * (u[r] * u[c] / (nu * nu) - v[r] * v[c] / (nv * nv));
    }
    static const int ri[6] = {0, 1, 2, 0, 0, 1}, ci[6] = {0, 1, 2, 1, 2, 2};
    double* row = tab.data() + j * smcx::kFdTableStride;
    for (int e = 0; e < 6; ++e) {
      const int r = ri[e], c = ci[e];
      row[e] = (M[2][r][c] - M[0][r][c]) / std::sqrt(2.0);
      row[6 + e] = (M[0][r][c] - 2.0 * M[1][r][c] + M[2][r][c]) / std::sqrt(6.0);
    }
    row[12] = std::cos(a);
    row[13] = std::sin(a);
    row[14] = t;
  }
  // Stage s (span H = 32 >> s) of the transform: lane l's butterfly has index
  // l & (H - 1) in its block, root exp(-2 pi i (l & (H - 1)) (32 / H) / 64).
  // For H <= 2 the forward root carries the sign of the lane's difference
  // (-1 where bit H of the lane is set); the inverse takes the conjugate.
  // (The kernels apply the span-1 roots, all 1 up to that sign, without
  // reading them.)
  for (int st = 0; st < 6; ++st) {
    const int H = 32 >> st;
    for (int l = 0; l < 64; ++l) {
      const int k = (l & (H - 1)) * (32 / H);
      const double c = std::cos(2.0 * kPi * k / 64.0), sn = -std::sin(2.0 * kPi * k / 64.0);
      const double sg = (H <= 2 && (l & H)) ? -1.0 : 1.0;
      tab[smcx::kFdTwiddleFwd + st * 128 + 2 * l] = sg * c;
      tab[smcx::kFdTwiddleFwd + st * 128 + 2 * l + 1] = sg * sn;
      tab[smcx::kFdTwiddleInv + st * 128 + 2 * l] = c;
      tab[smcx::kFdTwiddleInv + st * 128 + 2 * l + 1] = -sn;
    }
  }
  // the phase table of the envelope: cos and sin of 2 pi k / 128 (from
  // long double, so that each entry is the double nearest its value)
  const long double kPiL = 3.141592653589793238462643383279502884L;
  for (int k = -smcx::kFdTrigSteps / 2; k <= smcx::kFdTrigSteps / 2; ++k) {
    const long double x = 2.0L * kPiL * k / smcx::kFdTrigSteps;
    tab[smcx::kFdTrig + 2 * (k + smcx::kFdTrigSteps / 2)] = (double)std::cos(x);
    tab[smcx::kFdTrig + 2 * (k + smcx::kFdTrigSteps / 2) + 1] = (double)std::sin(x);
  }
}

// logL of a particle without components, split at the posterior-start bridge
// sample (0 without one): the part from the split on, tempered by beta, and
// the untempered part before it (FP64 prefix sums of d^2).
// Under a bridge between two frequency-domain records the K = 0 value is
// (1 - beta) E_partner + beta E_own = E_partner + beta (E_own - E_partner).
double k0_fd(const smcx_problem* p) { return -0.5 * p->prefix[1] * p->inv_sigma2; }
double k0_tempered(const smcx_problem* p) {
  if (p->fd && p->partner) return k0_fd(p) - k0_fd(p->partner);
  return -0.5 * (p->prefix[p->T] - p->prefix[p->split]) * p->inv_sigma2;
}
double k0_untempered(const smcx_problem* p) {
  if (p->fd && p->partner) return k0_fd(p->partner);
  return -0.5 * p->prefix[p->split] * p->inv_sigma2;
}

smcx::PrepArgs prep_args(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
                         const double* beta, double k0, int tempered) {
  smcx::PrepArgs a;
  std::memset(&a, 0, sizeof(a));
  a.offsets = offsets;
  a.beta = beta;
  a.N = N;
  a.M = M;
  a.k_max = p->k_max;
  a.m_max = p->m_max;
  a.k0_value = k0;
  a.P = p->P;
  a.order = p->order;
  a.n_active = p->n_active;
  a.block_hist = p->prep_hist;
  a.flag = p->flag;
  a.tempered = tempered;
  return a;
}

}  // namespace

extern "C" {

const char* smcx_last_error(void) { return g_last_error.c_str(); }

int smcx_problem_create(int model, const double* d_dev, int64_t T, double t_start, double dt,
                        double sigma, int32_t k_max, int64_t n_max, int64_t m_max,
                        void* hip_stream, smcx_problem** out) {
  g_last_error.clear();
  if (!out) return fail(SMCX_EINVAL, "out is NULL");
  *out = nullptr;
  if (model != SMCX_PULSE && model != SMCX_GBSINE)
    return fail(SMCX_EINVAL, "unknown model %d", model);
  if (!d_dev) return fail(SMCX_EINVAL, "d_dev is NULL");
  if (T < 1 || T > (int64_t(1) << 22)) return fail(SMCX_EINVAL, "T = %lld outside [1, 2^22]", (long long)T);
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(SMCX_EINVAL, "dt must be finite and > 0");
  if (!std::isfinite(t_start)) return fail(SMCX_EINVAL, "t_start must be finite");
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(SMCX_EINVAL, "sigma must be finite and > 0");
  if (k_max < 1 || k_max > 512) return fail(SMCX_EINVAL, "k_max = %d outside [1, 512]", k_max);
  if (n_max < 0 || n_max > (int64_t(1) << 30)) return fail(SMCX_EINVAL, "n_max = %lld out of range", (long long)n_max);
  if (m_max < 0 || m_max > (int64_t(1) << 34)) return fail(SMCX_EINVAL, "m_max = %lld out of range", (long long)m_max);
  hipStream_t st = (hipStream_t)hip_stream;
  if (capturing(st)) return fail(SMCX_ECAPTURE, "smcx_problem_create called during stream capture");

  smcx_problem* p = new smcx_problem();
  p->model = model;
  p->P = smcx::n_params(model);
  p->T = T;
  p->t_start = t_start;
  p->dt = dt;
  p->sigma = sigma;
  p->inv_sigma2 = 1.0 / (sigma * sigma);
  p->k_max = k_max;
  p->n_max = n_max;
  p->m_max = m_max;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) { free_problem(p); return hip_fail(e, "hipGetDevice"); }
  e = hipDeviceGetAttribute(&p->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device);
  if (e != hipSuccess) { free_problem(p); return hip_fail(e, "hipDeviceGetAttribute"); }

  p->max_nch = cap_chunks(T);
  p->max_nch_grad = cap_chunks_grad(T);
  for (int k = 0; k < kNumKinds; ++k) {
    p->tiling[k] = smcx::default_tiling(model, k, T);
    p->max_nch = std::max(p->max_nch, p->tiling[k].nch);
  }
  p->max_nch_grad = std::max(p->max_nch_grad, p->tiling[kGrad].nch);
  // data: FP64 copy (plain form), FP32 copy (batched kernels), FP64 energy prefix sums (host)
  std::vector<double> h(T);
  e = hipMemcpyAsync(h.data(), d_dev, T * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) { free_problem(p); return hip_fail(e, "copy of d"); }
  // FP32 copy zero-padded by one full 4096-sample tile past T (tile loads need no guard)
  const int64_t T_pad = round_up(T, 4096) + 4096;
  std::vector<float> h32(T_pad, 0.0f);
  p->prefix.assign(T + 1, 0.0);
  for (int64_t s = 0; s < T; ++s) {
    h32[s] = (float)h[s];
    p->prefix[s + 1] = p->prefix[s] + h[s] * h[s];
  }
  const size_t part_elems = (size_t)p->max_nch * (size_t)std::max<int64_t>(n_max, 1) * 4;
  p->part_cap = part_elems;
  const size_t partg_elems = p->max_nch_grad > 1
                                 ? (size_t)p->max_nch_grad * (size_t)std::max<int64_t>(m_max, 1) * p->P
                                 : 1;
  const int nb = (int)((T + 255) / 256);
  const size_t n1 = (size_t)std::max<int64_t>(n_max, 1);
  struct { void** ptr; size_t bytes; } allocs[] = {
      {(void**)&p->d32, T_pad * sizeof(float)},
      {(void**)&p->d64, T * sizeof(double)},
      {(void**)&p->order, (size_t)std::max<int64_t>(n_max, 1) * sizeof(int32_t)},
      {(void**)&p->n_active, sizeof(int32_t)},
      {(void**)&p->prep_hist,
       (size_t)smcx::prep_slices(std::max<int64_t>(n_max, 1)) * (k_max + 1) * sizeof(int32_t)},
      {(void**)&p->smc.cum, n1 * sizeof(int64_t)},
      {(void**)&p->smc.src_row, n1 * sizeof(int64_t)},
      {(void**)&p->smc.src_len, n1 * sizeof(int32_t)},
      {(void**)&p->smc.skip, n1 * sizeof(int32_t)},
      {(void**)&p->smc.append, n1 * sizeof(int32_t)},
      {(void**)&p->smc.count, n1 * sizeof(int64_t)},
      {(void**)&p->flag, sizeof(int)},
      {(void**)&p->part, part_elems * sizeof(double)},
      {(void**)&p->part_g, partg_elems * sizeof(double)},
      {(void**)&p->rbuf, T * sizeof(double)},
      {(void**)&p->bpart, nb * sizeof(double)},
  };
  size_t total = 0;
  for (auto& al : allocs) total += al.bytes;
  if (int rc = check_workspace(total, "the problem handle")) {
    free_problem(p);
    return rc;
  }
  for (auto& al : allocs) {
    e = hipMalloc(al.ptr, al.bytes);
    if (e != hipSuccess) {
      free_problem(p);
      return fail(SMCX_ENOMEM, "hipMalloc of %zu bytes failed: %s", al.bytes, hipGetErrorString(e));
    }
  }
  p->ws_bytes = total;
  const int zero = 0;
  e = hipMemcpyAsync(p->d32, h32.data(), T_pad * sizeof(float), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(p->d64, d_dev, T * sizeof(double), hipMemcpyDeviceToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(p->flag, &zero, sizeof(int), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(p->n_active, &zero, sizeof(int), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) { free_problem(p); return hip_fail(e, "upload of d"); }
  *out = p;
  return SMCX_OK;
}

int smcx_problem_create_fd(int model, const double* d_dev, int64_t k0, int64_t B, double T_obs,
                           double psd, int32_t k_max, int64_t n_max, int64_t m_max,
                           void* hip_stream, smcx_problem** out) {
  g_last_error.clear();
  if (!out) return fail(SMCX_EINVAL, "out is NULL");
  *out = nullptr;
  if (model != SMCX_GBLISA) return fail(SMCX_EINVAL, "model %d has no frequency-domain form", model);
  if (!d_dev) return fail(SMCX_EINVAL, "d_dev is NULL");
  if (B < 1 || B > 256) return fail(SMCX_EINVAL, "B = %lld outside [1, 256]", (long long)B);
  if (k0 < 0) return fail(SMCX_EINVAL, "k0 must be >= 0");
  if (!(T_obs > 0.0) || !std::isfinite(T_obs)) return fail(SMCX_EINVAL, "T_obs must be finite and > 0");
  if (!(psd > 0.0) || !std::isfinite(psd)) return fail(SMCX_EINVAL, "psd must be finite and > 0");
  if (k_max < 1 || k_max > 512) return fail(SMCX_EINVAL, "k_max = %d outside [1, 512]", k_max);
  if (n_max < 0 || n_max > (int64_t(1) << 30)) return fail(SMCX_EINVAL, "n_max = %lld out of range", (long long)n_max);
  if (m_max < 0 || m_max > (int64_t(1) << 34)) return fail(SMCX_EINVAL, "m_max = %lld out of range", (long long)m_max);
  hipStream_t st = (hipStream_t)hip_stream;
  if (capturing(st)) return fail(SMCX_ECAPTURE, "smcx_problem_create_fd called during stream capture");

  smcx_problem* p = new smcx_problem();
  p->model = model;
  p->P = smcx::n_params(model);
  p->T = 1;  // no time axis: one "sample" carries the band's energy
  p->t_start = 0.0;
  p->dt = 1.0;
  p->sigma = 1.0;
  p->inv_sigma2 = 4.0 / (T_obs * psd);  // the inner product's 4 df / S
  p->k_max = k_max;
  p->n_max = n_max;
  p->m_max = m_max;
  p->fd = true;
  p->fd_k0 = k0;
  p->fd_B = B;
  p->fd_T_obs = T_obs;
  p->fd_S = psd;
  hipError_t e = hipGetDevice(&p->device);
  if (e != hipSuccess) { free_problem(p); return hip_fail(e, "hipGetDevice"); }
  e = hipDeviceGetAttribute(&p->lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, p->device);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&p->n_cu, hipDeviceAttributeMultiprocessorCount, p->device);
  if (e != hipSuccess) { free_problem(p); return hip_fail(e, "hipDeviceGetAttribute"); }
  for (int k = 0; k < kNumKinds; ++k) p->tiling[k] = Tiling{16, 1024, 1, 1};
  p->max_nch = p->max_nch_grad = 1;
  const int64_t Bp = smcx::kFdBandStride;
  std::vector<double> h(4 * B), hp(4 * Bp, 0.0), tab;
  e = hipMemcpyAsync(h.data(), d_dev, 4 * B * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) { free_problem(p); return hip_fail(e, "copy of d"); }
  double energy = 0.0;
  for (int c = 0; c < 2; ++c)
    for (int64_t b = 0; b < B; ++b)
      for (int x = 0; x < 2; ++x) {
        const double v = h[(c * B + b) * 2 + x];
        hp[(c * Bp + b) * 2 + x] = v;
        energy += v * v;
      }
  p->prefix = {0.0, energy};
  fd_table_host(T_obs, tab);
  const size_t n1 = (size_t)std::max<int64_t>(n_max, 1);
  p->part_cap = n1 * 4;
  struct { void** ptr; size_t bytes; } allocs[] = {
      {(void**)&p->fd_data, 4 * Bp * sizeof(double)},
      {(void**)&p->fd_src, (size_t)std::max<int64_t>(m_max, 1) * smcx::kFdSrcWords * sizeof(double)},
      {(void**)&p->fd_table, tab.size() * sizeof(double)},
      {(void**)&p->order, n1 * sizeof(int32_t)},
      {(void**)&p->n_active, sizeof(int32_t)},
      {(void**)&p->prep_hist, (size_t)smcx::prep_slices((int64_t)n1) * (k_max + 1) * sizeof(int32_t)},
      {(void**)&p->smc.cum, n1 * sizeof(int64_t)},
      {(void**)&p->smc.src_row, n1 * sizeof(int64_t)},
      {(void**)&p->smc.src_len, n1 * sizeof(int32_t)},
      {(void**)&p->smc.skip, n1 * sizeof(int32_t)},
      {(void**)&p->smc.append, n1 * sizeof(int32_t)},
      {(void**)&p->smc.count, n1 * sizeof(int64_t)},
      {(void**)&p->flag, sizeof(int)},
      {(void**)&p->part, n1 * 4 * sizeof(double)},
      {(void**)&p->part_g, sizeof(double)},
  };
  size_t total = 0;
  for (auto& al : allocs) total += al.bytes;
  if (int rc = check_workspace(total, "the problem handle")) {
    free_problem(p);
    return rc;
  }
  for (auto& al : allocs) {
    e = hipMalloc(al.ptr, al.bytes);
    if (e != hipSuccess) {
      free_problem(p);
      return fail(SMCX_ENOMEM, "hipMalloc of %zu bytes failed: %s", al.bytes, hipGetErrorString(e));
    }
  }
  p->ws_bytes = total;
  const int zero = 0;
  e = hipMemcpyAsync(p->fd_data, hp.data(), hp.size() * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->fd_table, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(p->flag, &zero, sizeof(int), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipMemcpyAsync(p->n_active, &zero, sizeof(int), hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) { free_problem(p); return hip_fail(e, "upload of d"); }
  *out = p;
  return SMCX_OK;
}

int smcx_template_spectrum(int model, int64_t K, const double* theta, double T_obs, int64_t k0,
                           int64_t B, double* out, void* hip_stream) {
  g_last_error.clear();
  if (model != SMCX_GBLISA) return fail(SMCX_EINVAL, "model %d has no frequency-domain form", model);
  if (K < 0) return fail(SMCX_EINVAL, "negative K");
  if (K > 0 && !theta) return fail(SMCX_EINVAL, "theta is NULL");
  if (B < 1 || B > 256) return fail(SMCX_EINVAL, "B = %lld outside [1, 256]", (long long)B);
  if (!out) return fail(SMCX_EINVAL, "out is NULL");
  if (!(T_obs > 0.0) || !std::isfinite(T_obs)) return fail(SMCX_EINVAL, "T_obs must be finite and > 0");
  hipStream_t st = (hipStream_t)hip_stream;
  if (capturing(st)) return fail(SMCX_ECAPTURE, "smcx_template_spectrum called during stream capture");
  std::vector<double> tab;
  fd_table_host(T_obs, tab);
  double* dtab = nullptr;
  hipError_t e = hipMalloc(&dtab, tab.size() * sizeof(double));
  if (e != hipSuccess) return fail(SMCX_ENOMEM, "hipMalloc failed: %s", hipGetErrorString(e));
  e = hipMemcpyAsync(dtab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, st);
  smcx::PopArgs a;
  std::memset(&a, 0, sizeof(a));
  a.theta = theta;
  a.fd_table = dtab;
  a.fd_k0 = k0;
  a.fd_B = B;
  a.fd_T_obs = T_obs;
  a.fd_scale = T_obs / 64.0;
  if (e == hipSuccess) e = smcx::launch_fd_spectrum(a, K, out, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipFree(dtab);
  if (e != hipSuccess) return hip_fail(e, "template spectrum");
  return SMCX_OK;
}

int smcx_problem_destroy(smcx_problem* prob) {
  g_last_error.clear();
  if (!prob) return SMCX_OK;
  (void)hipDeviceSynchronize();
  free_problem(prob);
  return SMCX_OK;
}

int smcx_device_status(smcx_problem* p, void* hip_stream) {
  g_last_error.clear();
  if (!p) return fail(SMCX_EINVAL, "problem handle is NULL");
  hipStream_t st = (hipStream_t)hip_stream;
  if (capturing(st)) return fail(SMCX_ECAPTURE, "smcx_device_status called during stream capture");
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "stream synchronize");
  int flag = 0;
  const int zero = 0;
  e = hipMemcpy(&flag, p->flag, sizeof(int), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(p->flag, &zero, sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "device flag read");
  if (flag == 0) return SMCX_OK;
  std::string msg = "device-side argument errors:";
  if (flag & smcx::kFlagOffsets) msg += " offsets (or metric block offsets) not a valid prefix sum;";
  if (flag & smcx::kFlagKMax) msg += " a particle has K > k_max;";
  if (flag & smcx::kFlagMMax) msg += " offsets[N] differs from M;";
  if (flag & smcx::kFlagDeath) msg += " death index outside [-1, K);";
  if (flag & smcx::kFlagPhase) msg += " sinusoid phase of 2^19 cycles or more over the samples, or chirp too fast for the tile;";
  if (flag & smcx::kFlagCapacity) msg += " rebuilt population exceeds the output rows (m_cap);";
  if (flag & smcx::kFlagWeights) msg += " resampling weights have no positive entry;";
  if (flag & smcx::kFlagNotPD) msg += " a metric block is not positive definite (its factor is NaN);";
  return fail(SMCX_EDEVICE, "%s", msg.c_str());
}

int logl_batch(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
               const double* theta, const double* beta, double* logl, void* hip_stream) {
  g_last_error.clear();
  int rc = check_pop(p, N, offsets, M, theta);
  if (rc) return rc;
  if (N > 0 && !logl) return fail(SMCX_EINVAL, "logl is NULL");
  if (N == 0) return SMCX_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  const double k0 = k0_tempered(p);
  const Tiling& t = p->tiling[kFwd];
  hipError_t e = hipSuccess;
  if (t.sorted) {
    smcx::PrepArgs pa = prep_args(p, N, offsets, M, beta, k0, 1);
    pa.k0_lo = k0_untempered(p);
    pa.logl = logl;
    e = smcx::launch_prep(pa, st);
    if (e != hipSuccess) return hip_fail(e, "prep launch");
  }
  smcx::PopArgs a = base_args(p, N, offsets, M, theta, beta, t, 0, p->T, k0);
  a.split = p->split;
  a.k0_lo = k0_untempered(p);
  a.logl = logl;
  e = profiled(p, a, st, [&](const smcx::PopArgs& b) {
    return smcx::launch_forward(p->model, t, b, st);
  }, true);
  if (e != hipSuccess) return hip_fail(e, "logl launch");
  return SMCX_OK;
}

static int grad_batch(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
                      const double* theta, const double* beta, const uint8_t* mask, double* logl,
                      double* grad, void* hip_stream) {
  int rc = check_pop(p, N, offsets, M, theta);
  if (rc) return rc;
  if (M > 0 && !grad) return fail(SMCX_EINVAL, "grad is NULL");
  if (N == 0) return SMCX_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  const double k0 = k0_tempered(p);
  const Tiling& t = p->tiling[kGrad];
  hipError_t e = hipSuccess;
  if (t.sorted) {
    smcx::PrepArgs pa = prep_args(p, N, offsets, M, beta, k0, 1);
    pa.k0_lo = k0_untempered(p);
    pa.logl = logl;
    pa.grad = grad;
    e = smcx::launch_prep(pa, st);
    if (e != hipSuccess) return hip_fail(e, "prep launch");
  }
  smcx::PopArgs a = base_args(p, N, offsets, M, theta, beta, t, 0, p->T, k0);
  a.split = p->split;
  a.k0_lo = k0_untempered(p);
  a.logl = logl;
  a.grad = grad;
  a.active = mask;
  e = profiled(p, a, st, [&](const smcx::PopArgs& b) {
    return smcx::launch_fused(p->model, t, b, st);
  }, true);
  if (e != hipSuccess) return hip_fail(e, "logl_grad launch");
  return SMCX_OK;
}

int logl_grad_batch(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
                    const double* theta, const double* beta, double* logl, double* grad,
                    void* hip_stream) {
  g_last_error.clear();
  return grad_batch(p, N, offsets, M, theta, beta, nullptr, logl, grad, hip_stream);
}

int logl_grad_batch_masked(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
                           const double* theta, const double* beta, const uint8_t* mask,
                           double* logl, double* grad, void* hip_stream) {
  g_last_error.clear();
  if (N > 0 && !mask) return fail(SMCX_EINVAL, "mask is NULL");
  return grad_batch(p, N, offsets, M, theta, beta, mask, logl, grad, hip_stream);
}

static int delta_batch(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
                       const double* theta, const double* beta, const uint8_t* mask,
                       const double* theta_birth, const int32_t* death_idx, double* dlogl_birth,
                       double* dlogl_death, void* hip_stream) {
  int rc = check_pop(p, N, offsets, M, theta);
  if (rc) return rc;
  if (N > 0 && theta_birth && !dlogl_birth) return fail(SMCX_EINVAL, "dlogl_birth is NULL");
  if (N > 0 && death_idx && !dlogl_death) return fail(SMCX_EINVAL, "dlogl_death is NULL");
  if (N == 0 || (!theta_birth && !death_idx)) return SMCX_OK;
  if (p->k_max + 1 > 513) return fail(SMCX_EINVAL, "k_max too large for the birth slot");
  hipStream_t st = (hipStream_t)hip_stream;
  const Tiling& t = p->tiling[kDelta];
  hipError_t e = hipSuccess;
  if (t.sorted) {
    smcx::PrepArgs pa = prep_args(p, N, offsets, M, beta, 0.0, 1);
    pa.include_k0 = 1;
    pa.death_idx = death_idx;
    pa.dlogl_birth = theta_birth ? dlogl_birth : nullptr;
    pa.dlogl_death = death_idx ? dlogl_death : nullptr;
    e = smcx::launch_prep(pa, st);
    if (e != hipSuccess) return hip_fail(e, "prep launch");
  }
  smcx::PopArgs a = base_args(p, N, offsets, M, theta, beta, t, 0, p->T, 0.0);
  a.split = p->split;
  a.k0_lo = k0_untempered(p);
  a.theta_birth = theta_birth;
  a.death_idx = death_idx;
  a.dlogl_birth = dlogl_birth;
  a.dlogl_death = dlogl_death;
  a.active = mask;
  e = profiled(p, a, st, [&](const smcx::PopArgs& b) {
    return smcx::launch_delta(p->model, t, b, st);
  });
  if (e != hipSuccess) return hip_fail(e, "delta launch");
  return SMCX_OK;
}

int delta_logl_birth_death(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
                           const double* theta, const double* beta, const double* theta_birth,
                           const int32_t* death_idx, double* dlogl_birth, double* dlogl_death,
                           void* hip_stream) {
  g_last_error.clear();
  return delta_batch(p, N, offsets, M, theta, beta, nullptr, theta_birth, death_idx, dlogl_birth,
                     dlogl_death, hip_stream);
}

int delta_logl_birth_death_masked(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
                                  const double* theta, const double* beta, const uint8_t* mask,
                                  const double* theta_birth, const int32_t* death_idx,
                                  double* dlogl_birth, double* dlogl_death, void* hip_stream) {
  g_last_error.clear();
  if (N > 0 && !mask) return fail(SMCX_EINVAL, "mask is NULL");
  return delta_batch(p, N, offsets, M, theta, beta, mask, theta_birth, death_idx, dlogl_birth,
                     dlogl_death, hip_stream);
}

int reweight_extend(smcx_problem* p, int64_t T1, int64_t T2, int64_t N, const int64_t* offsets,
                    int64_t M, const double* theta, double delta_beta, const double* logw_prev,
                    double* logl_ext, double* logw, double* w_norm, double* scalars,
                    void* hip_stream) {
  g_last_error.clear();
  if (p && p->fd)
    return fail(SMCX_EINVAL, "reweight_extend needs a time-domain problem; for the frequency-domain "
                             "model evaluate logl_batch on both problems");
  int rc = check_pop(p, N, offsets, M, theta);
  if (rc) return rc;
  if (T1 < 0 || T2 <= T1 || T2 > p->T)
    return fail(SMCX_EINVAL, "sample range [%lld, %lld) not inside [0, %lld)", (long long)T1,
                (long long)T2, (long long)p->T);
  if (!std::isfinite(delta_beta)) return fail(SMCX_EINVAL, "delta_beta must be finite");
  if (!scalars) return fail(SMCX_EINVAL, "scalars is NULL");
  if (N > 0 && (!logl_ext || !logw || !w_norm)) return fail(SMCX_EINVAL, "an output array is NULL");
  hipStream_t st = (hipStream_t)hip_stream;
  if (N > 0) {
    const double k0 = -0.5 * (p->prefix[T2] - p->prefix[T1]) * p->inv_sigma2;
    const Tiling t = with_range(p->tiling[kFwd], T2 - T1);
    hipError_t e = hipSuccess;
    if (t.sorted) {
      smcx::PrepArgs pa = prep_args(p, N, offsets, M, nullptr, k0, 0);
      pa.logl = logl_ext;
      e = smcx::launch_prep(pa, st);
      if (e != hipSuccess) return hip_fail(e, "prep launch");
    }
    smcx::PopArgs a = base_args(p, N, offsets, M, theta, nullptr, t, T1, T2, k0);
    a.logl = logl_ext;
    e = profiled(p, a, st, [&](const smcx::PopArgs& b) {
      return smcx::launch_forward(p->model, t, b, st);
    }, true);
    if (e != hipSuccess) return hip_fail(e, "segment logl launch");
  }
  hipError_t e = smcx::launch_reweight_reduce(N, delta_beta, logl_ext, logw_prev, logw, w_norm,
                                              scalars, p->part, p->part_cap, st);
  if (e != hipSuccess) return hip_fail(e, "reweight launch");
  return SMCX_OK;
}

int smcx_template_sum(int model, int64_t K, const double* theta, int64_t T, double t_start,
                      double dt, double* out, void* hip_stream) {
  g_last_error.clear();
  if (model != SMCX_PULSE && model != SMCX_GBSINE) return fail(SMCX_EINVAL, "unknown model %d", model);
  if (K < 0 || T < 0) return fail(SMCX_EINVAL, "negative size");
  if (K > 0 && !theta) return fail(SMCX_EINVAL, "theta is NULL");
  if (T > 0 && !out) return fail(SMCX_EINVAL, "out is NULL");
  hipError_t e = smcx::launch_template_sum(model, K, theta, T, t_start, dt, out,
                                           (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "template_sum launch");
  return SMCX_OK;
}

int smcx_plain_logl_grad(smcx_problem* p, int64_t N, const int64_t* offsets_host, int64_t M,
                         const double* theta, const double* beta, double* logl, double* grad,
                         void* hip_stream) {
  g_last_error.clear();
  if (p && p->split != 0)
    return fail(SMCX_EINVAL, "the plain form evaluates the prior bridge only (bridge split is set)");
  if (p && p->fd) return fail(SMCX_EINVAL, "the plain form is defined for time-domain problems only");
  int rc = check_pop(p, N, offsets_host, M, theta);
  if (rc) return rc;
  if (N > 0 && !logl) return fail(SMCX_EINVAL, "logl is NULL");
  if (N == 0) return SMCX_OK;
  if (offsets_host[0] != 0) return fail(SMCX_EINVAL, "offsets[0] != 0");
  for (int64_t i = 0; i < N; ++i) {
    const int64_t K = offsets_host[i + 1] - offsets_host[i];
    if (K < 0 || K > p->k_max) return fail(SMCX_EINVAL, "particle %lld has K = %lld", (long long)i, (long long)K);
  }
  if (offsets_host[N] != M) return fail(SMCX_EINVAL, "offsets[N] != M");
  if (offsets_host[N] > 0 && !grad) return fail(SMCX_EINVAL, "grad is NULL");
  hipStream_t st = (hipStream_t)hip_stream;
  for (int64_t i = 0; i < N; ++i) {
    const int64_t m0 = offsets_host[i];
    const int K = (int)(offsets_host[i + 1] - m0);
    hipError_t e = smcx::launch_plain_particle(p->model, p->d64, p->T, p->t_start, p->dt,
                                               p->inv_sigma2, theta + m0 * p->P, K, beta, i,
                                               p->rbuf, p->bpart, logl, grad + m0 * p->P, st);
    if (e != hipSuccess) return hip_fail(e, "plain launch");
  }
  return SMCX_OK;
}

int smcx_leapfrog(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M, const double* beta,
                  double eps, const int8_t* dir, const uint8_t* active, const double* q_in,
                  const double* p_in, const double* g_in, double* q_out, double* p_out,
                  double* g_out, double* logl_out, void* hip_stream) {
  g_last_error.clear();
  int rc = check_pop(p, N, offsets, M, q_in);
  if (rc) return rc;
  if (!std::isfinite(eps)) return fail(SMCX_EINVAL, "eps must be finite");
  if (N > 0 && !logl_out) return fail(SMCX_EINVAL, "logl_out is NULL");
  if (M > 0 && (!p_in || !g_in || !q_out || !p_out || !g_out))
    return fail(SMCX_EINVAL, "a state array is NULL");
  const size_t bytes = (size_t)M * p->P * sizeof(double);
  const double* ins[3] = {q_in, p_in, g_in};
  const double* outs[3] = {q_out, p_out, g_out};
  for (const double* x : ins)
    for (const double* y : outs)
      if (M > 0 && (const char*)x < (const char*)y + bytes && (const char*)y < (const char*)x + bytes)
        return fail(SMCX_EINVAL, "input and output state arrays overlap");
  if (N == 0) return SMCX_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  hipError_t e = smcx::launch_drift(p->model, N, M, offsets, eps, dir, active, q_in, p_in, g_in,
                                    q_out, p_out, g_out, st);
  if (e != hipSuccess) return hip_fail(e, "drift launch");
  const double k0 = k0_tempered(p);
  const Tiling& t = p->tiling[kGrad];
  if (t.sorted) {
    smcx::PrepArgs pa = prep_args(p, N, offsets, M, beta, k0, 1);
    pa.k0_lo = k0_untempered(p);
    pa.logl = logl_out;
    pa.grad = g_out;
    e = smcx::launch_prep(pa, st);
    if (e != hipSuccess) return hip_fail(e, "prep launch");
  }
  smcx::PopArgs a = base_args(p, N, offsets, M, q_out, beta, t, 0, p->T, k0);
  a.split = p->split;
  a.k0_lo = k0_untempered(p);
  a.logl = logl_out;
  a.grad = g_out;
  a.active = active;
  a.p_half = p_out;
  a.p_out = p_out;
  a.eps = eps;
  a.dir = dir;
  e = profiled(p, a, st, [&](const smcx::PopArgs& b) {
    return smcx::launch_fused(p->model, t, b, st);
  }, true);
  if (e != hipSuccess) return hip_fail(e, "leapfrog gradient launch");
  return SMCX_OK;
}

int smcx_nuts_reserve(smcx_problem* p, int32_t max_depth) {
  g_last_error.clear();
  if (!p) return fail(SMCX_EINVAL, "problem handle is NULL");
  if (max_depth < 1 || max_depth > smcx::kNutsMaxDepth)
    return fail(SMCX_EINVAL, "max_depth = %d outside [1, %d]", max_depth, smcx::kNutsMaxDepth);
  if (p->nuts_depth >= max_depth) return SMCX_OK;
  const size_t stride = (size_t)std::max<int64_t>(p->m_max, 1) * p->P;
  const size_t nN = (size_t)std::max<int64_t>(p->n_max, 1);
  auto depth_bytes = [&](int D) {
    return D > 0 ? stride * smcx::kNutsSlots(D) * sizeof(double) + (D + 1) * sizeof(int) : 0;
  };
  const size_t per_particle = nN * (sizeof(smcx::NutsState) + sizeof(double) + 2 + 2 * sizeof(int32_t));
  // the cap is checked before anything is released: a refused reserve keeps
  // the handle, and its smaller NUTS workspace, as they were
  const size_t grown = p->ws_bytes - depth_bytes(p->nuts_depth) + depth_bytes(max_depth) +
                       (p->nuts_state ? 0 : per_particle);
  if (int rc = check_workspace(grown, "the NUTS workspace")) return rc;
  if (p->nuts_vec) {  // grow: release the smaller workspace first
    (void)hipDeviceSynchronize();
    (void)hipFree(p->nuts_vec);
    p->nuts_vec = nullptr;
    (void)hipFree(p->nuts_count);
    p->nuts_count = nullptr;
    p->ws_bytes -= depth_bytes(p->nuts_depth);
    p->nuts_depth = 0;
  }
  hipError_t e = hipMalloc(&p->nuts_vec, stride * smcx::kNutsSlots(max_depth) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc(&p->nuts_count, (max_depth + 1) * sizeof(int));
  if (e != hipSuccess) {
    (void)hipFree(p->nuts_vec);
    p->nuts_vec = nullptr;
    return fail(SMCX_ENOMEM, "NUTS workspace allocation failed: %s", hipGetErrorString(e));
  }
  p->ws_bytes += depth_bytes(max_depth);
  if (!p->nuts_state) {
    e = hipMalloc(&p->nuts_state, nN * sizeof(smcx::NutsState));
    if (e == hipSuccess) e = hipMalloc(&p->nuts_logl, nN * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&p->nuts_active, nN);
    if (e == hipSuccess) e = hipMalloc(&p->nuts_dir, nN);
    if (e == hipSuccess) e = hipMalloc(&p->nuts_list, 2 * nN * sizeof(int32_t));
    if (e != hipSuccess) {
      for (void** q : {(void**)&p->nuts_state, (void**)&p->nuts_logl, (void**)&p->nuts_active,
                       (void**)&p->nuts_dir, (void**)&p->nuts_list}) {
        (void)hipFree(*q);
        *q = nullptr;
      }
      return fail(SMCX_ENOMEM, "NUTS workspace allocation failed: %s", hipGetErrorString(e));
    }
    p->ws_bytes += per_particle;
  }
  if (!p->nuts_capture) e = hipStreamCreateWithFlags(&p->nuts_capture, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "NUTS capture stream");
  p->nuts_depth = max_depth;
  for (hipGraphExec_t g : p->nuts_graph)
    if (g) (void)hipGraphExecDestroy(g);
  p->nuts_graph.assign(max_depth, nullptr);
  p->nuts_graph_key.assign(max_depth, 0);
  return SMCX_OK;
}

namespace {
uint64_t mix_key(uint64_t h, uint64_t v) {
  h ^= v + 0x9e3779b97f4a7c15ull + (h << 6) + (h >> 2);
  return h;
}
}  // namespace

namespace {
int nuts_transition(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
                    const double* beta, double eps, int32_t max_depth, const double* prior_lo,
                    const double* prior_hi, const double* momentum, const int8_t* dirs,
                    const double* u_leaf, const double* u_tree, const uint8_t* mask,
                    const int64_t* w_offsets, int64_t w_size, const double* W, int w_blocks,
                    double* q, double* logl, double* grad, int32_t* depth_out, int32_t* steps_out,
                    int32_t* status_out, int32_t use_graph, void* hip_stream) {
  int rc = check_pop(p, N, offsets, M, q);
  if (rc) return rc;
  if (W) {
    if (!w_blocks && !w_offsets) return fail(SMCX_EINVAL, "w_offsets is NULL");
    if (w_size < 0) return fail(SMCX_EINVAL, "w_size must be >= 0");
    if ((int64_t)p->k_max * p->P > smcx::kNutsMetricMax)
      return fail(SMCX_EINVAL, "a NUTS metric needs k_max * P <= %d (here %d)", smcx::kNutsMetricMax,
                  p->k_max * p->P);
  }
  if (!(eps > 0.0) || !std::isfinite(eps)) return fail(SMCX_EINVAL, "eps must be finite and > 0");
  if (max_depth < 1 || max_depth > p->nuts_depth)
    return fail(SMCX_EINVAL, "max_depth = %d exceeds the reserved NUTS depth %d (smcx_nuts_reserve)",
                max_depth, p->nuts_depth);
  if ((prior_lo == nullptr) != (prior_hi == nullptr))
    return fail(SMCX_EINVAL, "prior_lo and prior_hi must both be given or both be NULL");
  if (N > 0 && (!logl || !dirs || !u_leaf || !u_tree)) return fail(SMCX_EINVAL, "an input array is NULL");
  if (M > 0 && (!momentum || !grad)) return fail(SMCX_EINVAL, "momentum or grad is NULL");
  hipStream_t st = (hipStream_t)hip_stream;
  if (capturing(st)) return fail(SMCX_ECAPTURE, "smcx_nuts_transition called during stream capture");
  if (N == 0) return SMCX_OK;

  smcx::NutsArgs na;
  std::memset(&na, 0, sizeof(na));
  na.P = p->P;
  na.D = max_depth;
  na.n_cu = p->n_cu;
  na.k_max = p->k_max;
  na.N = N;
  na.M = M;
  na.offsets = offsets;
  na.eps = eps;
  na.prior_lo = prior_lo;
  na.prior_hi = prior_hi;
  na.momentum = momentum;
  na.dirs = dirs;
  na.u_leaf = u_leaf;
  na.u_tree = u_tree;
  na.mask = mask;
  na.q = q;
  na.logl = logl;
  na.grad = grad;
  na.depth_out = depth_out;
  na.steps_out = steps_out;
  na.status_out = status_out;
  na.vec = p->nuts_vec;
  na.stride = std::max<int64_t>(p->m_max, 1) * p->P;
  na.state = (smcx::NutsState*)p->nuts_state;
  na.logl_front = p->nuts_logl;
  na.active = p->nuts_active;
  na.dir = p->nuts_dir;
  na.count = p->nuts_count;
  na.list_next = nullptr;  // init lists nothing: the first doubling runs in natural order
  na.wmat = W;
  na.w_off = W && !w_blocks ? w_offsets : nullptr;
  na.w_size = w_size;
  na.w_blocks = W && w_blocks ? 1 : 0;
  na.flag = p->flag;
  double* qF = p->nuts_vec + 6 * na.stride;
  double* pF = p->nuts_vec + 7 * na.stride;
  double* gF = p->nuts_vec + 8 * na.stride;
  double* pH = p->nuts_vec + 9 * na.stride;

  const double k0 = k0_tempered(p);
  const Tiling& t = p->tiling[kGrad];
  hipError_t e = hipSuccess;
  if (t.sorted) {  // one ordering pass serves every leapfrog step of the transition
    smcx::PrepArgs pa = prep_args(p, N, offsets, M, beta, k0, 1);
    pa.k0_lo = k0_untempered(p);
    pa.logl = p->nuts_logl;
    e = smcx::launch_prep(pa, st);
    if (e != hipSuccess) return hip_fail(e, "prep launch");
  }
  smcx::PopArgs a = base_args(p, N, offsets, M, qF, beta, t, 0, p->T, k0);
  a.split = p->split;
  a.k0_lo = k0_untempered(p);
  a.logl = p->nuts_logl;
  a.grad = gF;
  a.active = p->nuts_active;
  // with a metric the closing kick needs W times the whole gradient: the
  // leaf kernel applies it instead of the gradient pass's epilogue
  a.p_half = W ? nullptr : pH;
  a.p_out = W ? nullptr : pF;
  a.eps = eps;
  a.dir = p->nuts_dir;

  // For the frequency-domain model every launch of doubling j >= 1 (gradient,
  // leaf, merge) walks the particles still extending at its start, which the
  // previous merge listed, so its cost shrinks with the active set; the lists
  // alternate between two buffers. The first doubling, where nearly every
  // particle is active, runs in natural order. The time-domain models keep the
  // natural order in the leaf and merge launches and the longest-first order
  // in the gradient: their short launches pay more for the list's extra
  // dependent load than they save, and their chunked gradient balances
  // better longest-first (measured on the pulse NUTS workload).
  const size_t nlist = (size_t)std::max<int64_t>(p->n_max, 1);
  auto doubling = [&](int j, hipStream_t s) -> hipError_t {
    smcx::NutsArgs nj = na;
    smcx::PopArgs aj = a;
    // From the third doubling on few particles are still extending (trees
    // end after one or two doublings for most): on the frequency-domain
    // model the leaf, merge and gradient launches step through them on fixed
    // grids, which removes the floor of grids sized to the population. The
    // time-domain workloads' populations are smaller, and there the
    // one-pass kernels (half the registers) measured faster.
    nj.stride_grid = aj.stride_grid = p->fd && j >= 2 ? 1 : 0;
    if (p->fd) {
      nj.list_next = p->nuts_list + (size_t)((j + 1) & 1) * nlist;
      if (j > 0) {
        nj.list = p->nuts_list + (size_t)(j & 1) * nlist;
        nj.nlist = p->nuts_count + j;
        aj.order = nj.list;
        aj.n_active = nj.nlist;
      }
    }
    for (int n = 0; n < (1 << j); ++n) {
      hipError_t err = smcx::launch_fused(p->model, t, aj, s);
      if (err == hipSuccess) err = smcx::launch_nuts_leaf(nj, j, n, s);
      if (err != hipSuccess) return err;
    }
    return smcx::launch_nuts_merge(nj, j, s);
  };

  uint64_t key = 0;
  for (uint64_t v : {(uint64_t)N, (uint64_t)M, (uint64_t)(uintptr_t)offsets, (uint64_t)(uintptr_t)beta,
                     (uint64_t)(uintptr_t)prior_lo, (uint64_t)(uintptr_t)prior_hi,
                     (uint64_t)(uintptr_t)momentum, (uint64_t)(uintptr_t)dirs,
                     (uint64_t)(uintptr_t)u_leaf, (uint64_t)(uintptr_t)u_tree,
                     (uint64_t)(uintptr_t)q, (uint64_t)(uintptr_t)logl, (uint64_t)(uintptr_t)grad,
                     (uint64_t)t.S, (uint64_t)t.chunk_len, (uint64_t)t.sorted, (uint64_t)max_depth,
                     (uint64_t)p->split, (uint64_t)(uintptr_t)W, (uint64_t)(uintptr_t)w_offsets,
                     (uint64_t)w_size, (uint64_t)w_blocks, (uint64_t)(uintptr_t)p->partner})
    key = mix_key(key, v);
  uint64_t eb;
  std::memcpy(&eb, &eps, sizeof(eb));
  key = mix_key(key, eb);

  e = smcx::launch_nuts_init(na, st);
  if (e != hipSuccess) return hip_fail(e, "NUTS init launch");
  for (int j = 0; j < max_depth; ++j) {
    if (use_graph) {
      if (!p->nuts_graph[j] || p->nuts_graph_key[j] != key) {
        if (p->nuts_graph[j]) (void)hipGraphExecDestroy(p->nuts_graph[j]);
        p->nuts_graph[j] = nullptr;
        hipGraph_t g = nullptr;
        e = hipStreamBeginCapture(p->nuts_capture, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
          hipError_t e2 = doubling(j, p->nuts_capture);
          e = hipStreamEndCapture(p->nuts_capture, &g);
          if (e2 != hipSuccess) e = e2;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&p->nuts_graph[j], g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(e, "NUTS graph capture");
        p->nuts_graph_key[j] = key;
      }
      e = hipGraphLaunch(p->nuts_graph[j], st);
    } else {
      e = doubling(j, st);
    }
    if (e != hipSuccess) return hip_fail(e, "NUTS doubling");
    if (j + 1 < max_depth) {  // stop as soon as no trajectory is still extending
      int alive = 0;
      e = hipMemcpyAsync(&alive, p->nuts_count + (j + 1), sizeof(int), hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return hip_fail(e, "NUTS active count");
      if (alive == 0) break;
    }
  }
  e = smcx::launch_nuts_finalize(na, st);
  if (e != hipSuccess) return hip_fail(e, "NUTS finalize launch");
  return SMCX_OK;
}
}  // namespace

int smcx_nuts_transition(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
                         const double* beta, double eps, int32_t max_depth,
                         const double* prior_lo, const double* prior_hi, const double* momentum,
                         const int8_t* dirs, const double* u_leaf, const double* u_tree,
                         const uint8_t* mask, double* q, double* logl, double* grad,
                         int32_t* depth_out, int32_t* steps_out, int32_t* status_out,
                         int32_t use_graph, void* hip_stream) {
  g_last_error.clear();
  return nuts_transition(p, N, offsets, M, beta, eps, max_depth, prior_lo, prior_hi, momentum, dirs,
                         u_leaf, u_tree, mask, nullptr, 0, nullptr, 0, q, logl, grad, depth_out,
                         steps_out, status_out, use_graph, hip_stream);
}

int smcx_nuts_transition_metric(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
                                const double* beta, double eps, int32_t max_depth,
                                const double* prior_lo, const double* prior_hi,
                                const double* momentum, const int8_t* dirs, const double* u_leaf,
                                const double* u_tree, const uint8_t* mask,
                                const int64_t* w_offsets, int64_t w_size, const double* W,
                                double* q, double* logl, double* grad, int32_t* depth_out,
                                int32_t* steps_out, int32_t* status_out, int32_t use_graph,
                                void* hip_stream) {
  g_last_error.clear();
  if (!p) return fail(SMCX_EINVAL, "problem handle is NULL");
  if (!W && N > 0) return fail(SMCX_EINVAL, "W is NULL");
  return nuts_transition(p, N, offsets, M, beta, eps, max_depth, prior_lo, prior_hi, momentum, dirs,
                         u_leaf, u_tree, mask, w_offsets, w_size, W, 0, q, logl, grad, depth_out,
                         steps_out, status_out, use_graph, hip_stream);
}

int smcx_nuts_transition_metric_blocks(smcx_problem* p, int64_t N, const int64_t* offsets,
                                       int64_t M, const double* beta, double eps,
                                       int32_t max_depth, const double* prior_lo,
                                       const double* prior_hi, const double* momentum,
                                       const int8_t* dirs, const double* u_leaf,
                                       const double* u_tree, const uint8_t* mask, const double* W,
                                       double* q, double* logl, double* grad, int32_t* depth_out,
                                       int32_t* steps_out, int32_t* status_out, int32_t use_graph,
                                       void* hip_stream) {
  g_last_error.clear();
  if (!p) return fail(SMCX_EINVAL, "problem handle is NULL");
  if (!W && M > 0) return fail(SMCX_EINVAL, "W is NULL");
  return nuts_transition(p, N, offsets, M, beta, eps, max_depth, prior_lo, prior_hi, momentum, dirs,
                         u_leaf, u_tree, mask, nullptr, M * p->P * p->P, M > 0 ? W : nullptr,
                         M > 0 ? 1 : 0, q, logl, grad, depth_out, steps_out, status_out, use_graph,
                         hip_stream);
}

int smcx_set_bridge_split(smcx_problem* p, int64_t split) {
  g_last_error.clear();
  if (!p) return fail(SMCX_EINVAL, "problem handle is NULL");
  if (p->fd && split != 0) return fail(SMCX_EINVAL, "frequency-domain problems have no bridge split");
  if (split < 0 || split > p->T)
    return fail(SMCX_EINVAL, "split = %lld outside [0, T = %lld]", (long long)split, (long long)p->T);
  p->split = split;
  return SMCX_OK;
}

int smcx_set_bridge_partner(smcx_problem* p, smcx_problem* partner) {
  g_last_error.clear();
  if (!p) return fail(SMCX_EINVAL, "problem handle is NULL");
  if (partner) {
    if (!p->fd || !partner->fd)
      return fail(SMCX_EINVAL, "a bridge partner joins two frequency-domain handles");
    if (partner == p) return fail(SMCX_EINVAL, "a handle cannot be its own bridge partner");
    if (partner->model != p->model) return fail(SMCX_EINVAL, "the partner has another model");
    if (partner->partner) return fail(SMCX_EINVAL, "the partner has a bridge partner itself");
  }
  p->partner = partner;
  return SMCX_OK;
}

int smcx_get_bridge_split(smcx_problem* p, int64_t* split) {
  g_last_error.clear();
  if (!p || !split) return fail(SMCX_EINVAL, "problem handle or output is NULL");
  *split = p->split;
  return SMCX_OK;
}

int smcx_set_tiling(smcx_problem* p, int32_t kind, int32_t S, int64_t chunk_len, int32_t sorted) {
  g_last_error.clear();
  if (!p) return fail(SMCX_EINVAL, "problem handle is NULL");
  if (p->fd) return fail(SMCX_EINVAL, "frequency-domain problems have no sample tiling");
  if (kind < 0 || kind >= kNumKinds) return fail(SMCX_EINVAL, "unknown call kind %d", kind);
  const bool s_ok = kind == kDelta ? (S == 8 || S == 16) : (S == 8 || S == 16 || S == 32 || S == 64);
  if (!s_ok) return fail(SMCX_EINVAL, "S = %d not supported for this call kind", S);
  if (chunk_len <= 0 || chunk_len % (64 * (int64_t)S) != 0)
    return fail(SMCX_EINVAL, "chunk_len must be a positive multiple of 64*S");
  if (sorted < 0 || sorted > 2) return fail(SMCX_EINVAL, "sorted must be 0, 1 or 2");
  Tiling t;
  t.S = S;
  t.chunk_len = chunk_len;
  t.nch = (int)((p->T + chunk_len - 1) / chunk_len);
  t.sorted = sorted;
  if (t.nch > p->max_nch) return fail(SMCX_EINVAL, "%d chunks exceed the workspace (%d)", t.nch, p->max_nch);
  if (kind == kGrad && t.nch > 1 && t.nch > p->max_nch_grad)
    return fail(SMCX_EINVAL, "%d gradient chunks exceed the workspace (%d)", t.nch, p->max_nch_grad);
  p->tiling[kind] = t;
  return SMCX_OK;
}

int smcx_get_tiling(smcx_problem* p, int32_t kind, int32_t* S, int64_t* chunk_len, int32_t* sorted) {
  g_last_error.clear();
  if (!p) return fail(SMCX_EINVAL, "problem handle is NULL");
  if (kind < 0 || kind >= kNumKinds) return fail(SMCX_EINVAL, "unknown call kind %d", kind);
  if (S) *S = p->tiling[kind].S;
  if (chunk_len) *chunk_len = p->tiling[kind].chunk_len;
  if (sorted) *sorted = p->tiling[kind].sorted;
  return SMCX_OK;
}

int smcx_profile_begin(smcx_problem* p, int32_t max_launches) {
  g_last_error.clear();
  if (!p) return fail(SMCX_EINVAL, "problem handle is NULL");
  if (max_launches < 1 || max_launches > (1 << 16)) return fail(SMCX_EINVAL, "max_launches out of range");
  const size_t need = 2 * (size_t)max_launches;
  while (p->prof_ev.size() < need) {
    hipEvent_t e;
    hipError_t err = hipEventCreate(&e);
    if (err != hipSuccess) return hip_fail(err, "hipEventCreate");
    p->prof_ev.push_back(e);
  }
  p->prof_n = 0;
  p->prof_on = true;
  return SMCX_OK;
}

int smcx_profile_end(smcx_problem* p, double* total_ms, int64_t* launches) {
  g_last_error.clear();
  if (!p) return fail(SMCX_EINVAL, "problem handle is NULL");
  p->prof_on = false;
  double tot = 0.0;
  for (int i = 0; i < p->prof_n; ++i) {
    hipError_t e = hipEventSynchronize(p->prof_ev[2 * i + 1]);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, p->prof_ev[2 * i], p->prof_ev[2 * i + 1]);
    if (e != hipSuccess) return hip_fail(e, "profile event");
    tot += ms;
  }
  if (total_ms) *total_ms = tot;
  if (launches) *launches = p->prof_n;
  p->prof_n = 0;
  return SMCX_OK;
}

int smcx_next_beta(smcx_problem* p, int64_t N, const double* logl, const double* logw_prev,
                   double beta_prev, double alpha, double* beta_out, double* logw,
                   double* w_norm, double* scalars, void* hip_stream) {
  g_last_error.clear();
  if (!p) return fail(SMCX_EINVAL, "problem handle is NULL");
  if (N < 1 || N > p->n_max)
    return fail(SMCX_EINVAL, "N = %lld outside [1, n_max = %lld]", (long long)N,
                (long long)p->n_max);
  if (!logl || !logw || !w_norm || !scalars)
    return fail(SMCX_EINVAL, "logl, logw, w_norm and scalars are required");
  if (!(beta_prev >= 0.0 && beta_prev <= 1.0))
    return fail(SMCX_EINVAL, "beta_prev = %g outside [0, 1]", beta_prev);
  if (!(alpha > 0.0 && alpha <= 1.0)) return fail(SMCX_EINVAL, "alpha = %g outside (0, 1]", alpha);
  hipStream_t st = (hipStream_t)hip_stream;
  hipError_t e = smcx::launch_next_beta(N, logl, logw_prev, beta_prev, alpha, beta_out, logw,
                                        w_norm, scalars, p->part, p->part_cap, st);
  if (e != hipSuccess) return hip_fail(e, "next_beta launch");
  return SMCX_OK;
}

int smcx_resample_systematic(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
                             const double* theta, const double* w_norm, double u, int64_t m_cap,
                             int32_t* ancestors, int64_t* offsets_out, double* theta_out,
                             void* hip_stream) {
  g_last_error.clear();
  int rc = check_pop(p, N, offsets, M, theta);
  if (rc) return rc;
  if (N < 1) return fail(SMCX_EINVAL, "N must be positive");
  if (N > INT32_MAX) return fail(SMCX_EINVAL, "N too large for int32 ancestors");
  if (!w_norm || !ancestors || !offsets_out) return fail(SMCX_EINVAL, "null output or weights");
  if (m_cap < 0 || (m_cap > 0 && !theta_out)) return fail(SMCX_EINVAL, "bad m_cap / theta_out");
  if (!(u >= 0.0 && u < 1.0)) return fail(SMCX_EINVAL, "u = %g outside [0, 1)", u);
  hipStream_t st = (hipStream_t)hip_stream;
  hipError_t e = smcx::launch_resample(p->smc, p->model, p->k_max, N, offsets, M, theta, w_norm, u,
                                       m_cap, ancestors, offsets_out, theta_out, p->flag, st);
  if (e != hipSuccess) return hip_fail(e, "resample launch");
  return SMCX_OK;
}

int smcx_rj_apply(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
                  const double* theta, const int8_t* move, const double* theta_birth,
                  const int32_t* death_idx, const double* dlogl_birth, const double* dlogl_death,
                  const double* log_u, int32_t k_lo, int32_t k_hi, double log_pd_over_pb,
                  int64_t m_cap, int64_t* offsets_out, double* theta_out, int8_t* accepted,
                  void* hip_stream) {
  g_last_error.clear();
  int rc = check_pop(p, N, offsets, M, theta);
  if (rc) return rc;
  if (N == 0) return SMCX_OK;
  if (!move || !log_u || !offsets_out || !accepted)
    return fail(SMCX_EINVAL, "move, log_u, offsets_out and accepted are required");
  if (m_cap < 0 || (m_cap > 0 && !theta_out)) return fail(SMCX_EINVAL, "bad m_cap / theta_out");
  if (k_lo < 0 || k_hi < k_lo || k_hi > p->k_max)
    return fail(SMCX_EINVAL, "k range [%d, %d] not inside [0, k_max = %d]", k_lo, k_hi, p->k_max);
  if (!(log_pd_over_pb == log_pd_over_pb)) return fail(SMCX_EINVAL, "log_pd_over_pb is NaN");
  hipStream_t st = (hipStream_t)hip_stream;
  hipError_t e = smcx::launch_rj_apply(p->smc, p->model, p->k_max, N, offsets, M, theta, move,
                                       theta_birth, death_idx, dlogl_birth, dlogl_death, log_u,
                                       k_lo, k_hi, log_pd_over_pb, m_cap, offsets_out, theta_out,
                                       accepted, p->flag, st);
  if (e != hipSuccess) return hip_fail(e, "rj_apply launch");
  return SMCX_OK;
}

static int gn_metric(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
                     const double* theta, const double* beta, const uint8_t* mask,
                     const int64_t* f_offsets, int64_t f_size, double* F, void* hip_stream) {
  int rc = check_pop(p, N, offsets, M, theta);
  if (rc) return rc;
  if (N == 0) return SMCX_OK;
  if (!f_offsets) return fail(SMCX_EINVAL, "f_offsets is NULL");
  if (f_size < 0 || (f_size > 0 && !F)) return fail(SMCX_EINVAL, "bad f_size / F");
  if (p->fd) {
    smcx::PopArgs a = base_args(p, N, offsets, M, theta, beta, p->tiling[kGrad], 0, p->T, 0.0);
    a.active = mask;
    hipError_t e = smcx::launch_fd_metric(a, f_offsets, f_size, F, 0, (hipStream_t)hip_stream);
    if (e != hipSuccess) return hip_fail(e, "metric launch");
    return SMCX_OK;
  }
  if ((int64_t)p->k_max * p->P > 128)
    return fail(SMCX_EINVAL, "the metric supports k_max * P <= 128 (k_max = %d)", p->k_max);
  hipStream_t st = (hipStream_t)hip_stream;
  hipError_t e = smcx::launch_metric(p->model, p->P, N, M, p->T, p->t_start, p->dt, p->inv_sigma2,
                                     p->k_max, offsets, theta, beta, f_offsets, f_size, F,
                                     p->split, 0, p->flag, st, mask);
  if (e != hipSuccess) return hip_fail(e, "metric launch");
  return SMCX_OK;
}

int smcx_gauss_newton_metric(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
                             const double* theta, const double* beta, const int64_t* f_offsets,
                             int64_t f_size, double* F, void* hip_stream) {
  g_last_error.clear();
  return gn_metric(p, N, offsets, M, theta, beta, nullptr, f_offsets, f_size, F, hip_stream);
}

int smcx_gauss_newton_metric_masked(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
                                    const double* theta, const double* beta, const uint8_t* mask,
                                    const int64_t* f_offsets, int64_t f_size, double* F,
                                    void* hip_stream) {
  g_last_error.clear();
  if (N > 0 && !mask) return fail(SMCX_EINVAL, "mask is NULL");
  return gn_metric(p, N, offsets, M, theta, beta, mask, f_offsets, f_size, F, hip_stream);
}

static int gn_metric_blocks(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
                            const double* theta, const double* beta, const uint8_t* mask,
                            double* F, void* hip_stream) {
  int rc = check_pop(p, N, offsets, M, theta);
  if (rc) return rc;
  if (N == 0) return SMCX_OK;
  if (M > 0 && !F) return fail(SMCX_EINVAL, "F is NULL");
  hipStream_t st = (hipStream_t)hip_stream;
  if (p->fd) {
    smcx::PopArgs a = base_args(p, N, offsets, M, theta, beta, p->tiling[kGrad], 0, p->T, 0.0);
    a.active = mask;
    hipError_t e = smcx::launch_fd_metric(a, nullptr, 0, F, 1, st);
    if (e != hipSuccess) return hip_fail(e, "metric launch");
    return SMCX_OK;
  }
  if ((int64_t)p->k_max * p->P > 128)
    return fail(SMCX_EINVAL, "the metric supports k_max * P <= 128 (k_max = %d)", p->k_max);
  hipError_t e = smcx::launch_metric(p->model, p->P, N, M, p->T, p->t_start, p->dt, p->inv_sigma2,
                                     p->k_max, offsets, theta, beta, nullptr, 0, F, p->split, 1,
                                     p->flag, st, mask);
  if (e != hipSuccess) return hip_fail(e, "metric launch");
  return SMCX_OK;
}

int smcx_gauss_newton_metric_blocks(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
                                    const double* theta, const double* beta, double* F,
                                    void* hip_stream) {
  g_last_error.clear();
  return gn_metric_blocks(p, N, offsets, M, theta, beta, nullptr, F, hip_stream);
}

int smcx_gauss_newton_metric_blocks_masked(smcx_problem* p, int64_t N, const int64_t* offsets,
                                           int64_t M, const double* theta, const double* beta,
                                           const uint8_t* mask, double* F, void* hip_stream) {
  g_last_error.clear();
  if (N > 0 && !mask) return fail(SMCX_EINVAL, "mask is NULL");
  return gn_metric_blocks(p, N, offsets, M, theta, beta, mask, F, hip_stream);
}

int smcx_metric_pool_blocks(smcx_problem* p, int64_t M, const double* F, double* F_mean,
                            void* hip_stream) {
  g_last_error.clear();
  if (!p) return fail(SMCX_EINVAL, "problem handle is NULL");
  if (M < 1 || M > p->m_max)
    return fail(SMCX_EINVAL, "M = %lld outside [1, m_max = %lld]", (long long)M,
                (long long)p->m_max);
  if (!F || !F_mean) return fail(SMCX_EINVAL, "F or F_mean is NULL");
  hipError_t e = smcx::launch_metric_pool(p->P, M, F, F_mean, p->part, p->part_cap,
                                          (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "metric pool launch");
  return SMCX_OK;
}

int smcx_metric_factor_blocks(smcx_problem* p, int64_t M, const double* F, const double* ridge,
                              double* W, void* hip_stream) {
  g_last_error.clear();
  if (!p) return fail(SMCX_EINVAL, "problem handle is NULL");
  if (M < 0) return fail(SMCX_EINVAL, "M = %lld must be >= 0", (long long)M);
  if (M > 0 && (!F || !W)) return fail(SMCX_EINVAL, "F or W is NULL");
  if (!ridge) return fail(SMCX_EINVAL, "ridge is NULL");
  for (int q = 0; q < p->P; ++q)
    if (!(ridge[q] >= 0.0) || !std::isfinite(ridge[q]))
      return fail(SMCX_EINVAL, "ridge[%d] must be finite and >= 0", q);
  hipError_t e = smcx::launch_metric_factor_blocks(p->P, M, F, ridge, W, p->flag,
                                                   (hipStream_t)hip_stream);
  if (e != hipSuccess) return hip_fail(e, "metric factor launch");
  return SMCX_OK;
}

static int metric_factor(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
                         const uint8_t* mask, const int64_t* f_offsets, int64_t f_size,
                         const double* F, const double* ridge, int32_t block, double* W,
                         void* hip_stream) {
  int rc = check_pop(p, N, offsets, M, F ? F : W);  // theta is not read: only the sizes matter
  if (rc) return rc;
  if (N == 0) return SMCX_OK;
  if (!f_offsets) return fail(SMCX_EINVAL, "f_offsets is NULL");
  if (f_size < 0 || (f_size > 0 && (!F || !W))) return fail(SMCX_EINVAL, "bad f_size / F / W");
  if (!ridge) return fail(SMCX_EINVAL, "ridge is NULL");
  for (int q = 0; q < p->P; ++q)
    if (!(ridge[q] >= 0.0) || !std::isfinite(ridge[q]))
      return fail(SMCX_EINVAL, "ridge[%d] must be finite and >= 0", q);
  const int nmax = p->k_max * p->P;
  if (nmax > smcx::kNutsMetricMax)
    return fail(SMCX_EINVAL, "the metric factor supports k_max * P <= %d", smcx::kNutsMetricMax);
  if (block < 0 || (block > 0 && p->P % block != 0))
    return fail(SMCX_EINVAL, "block = %d must be 0 or divide P = %d", block, p->P);
  if ((int64_t)smcx::factor_lds_bytes(block > 0 ? block : nmax) > (int64_t)p->lds_max)
    return fail(SMCX_EINVAL, "k_max * P = %d needs %zu bytes of LDS per workgroup; the device has %d",
                nmax, smcx::factor_lds_bytes(nmax), p->lds_max);
  hipStream_t st = (hipStream_t)hip_stream;
  hipError_t e = smcx::launch_metric_factor(p->P, N, M, p->k_max, offsets, f_offsets, f_size, F,
                                            ridge, block, W, p->flag, st, mask);
  if (e != hipSuccess) return hip_fail(e, "metric factor launch");
  return SMCX_OK;
}

int smcx_metric_factor(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
                       const int64_t* f_offsets, int64_t f_size, const double* F,
                       const double* ridge, int32_t block, double* W, void* hip_stream) {
  g_last_error.clear();
  return metric_factor(p, N, offsets, M, nullptr, f_offsets, f_size, F, ridge, block, W,
                       hip_stream);
}

int smcx_metric_factor_masked(smcx_problem* p, int64_t N, const int64_t* offsets, int64_t M,
                              const uint8_t* mask, const int64_t* f_offsets, int64_t f_size,
                              const double* F, const double* ridge, int32_t block, double* W,
                              void* hip_stream) {
  g_last_error.clear();
  if (N > 0 && !mask) return fail(SMCX_EINVAL, "mask is NULL");
  return metric_factor(p, N, offsets, M, mask, f_offsets, f_size, F, ridge, block, W,
                       hip_stream);
}

}  // extern "C"
