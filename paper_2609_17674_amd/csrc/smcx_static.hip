// logl_grad_batch_static: the fused log-likelihood + gradient pass without a
// problem handle and without any allocation. Its workspace (the FP32 copy of
// the data, the K = 0 energy, the longest-K-first work list and the chunk
// partial sums) lives in one file-scope device array of fixed size; each
// device holds its own copy, whose address is looked up once per device.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>

#include "../../include/smcx.h"
#include "smcx_internal.h"
#include "smcx_problem.h"

namespace {

constexpr size_t kScratchBytes = (size_t)SMCX_STATIC_SCRATCH_BYTES;
constexpr int kStageBlock = 256;
constexpr int kStageSpan = 4096;  // samples per staging block (16 per thread)

// The shared workspace. Host code must not use this name as an address:
// scratch_base() returns the device address of the current device's copy.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_base[kMaxDevices] = {};

int scratch_base(unsigned char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess)
    return smcx::set_error(SMCX_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return smcx::set_error(SMCX_EDEVICE, "device %d outside the supported range", dev);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_base[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return smcx::set_error(SMCX_EDEVICE, "hipGetSymbolAddress of the static scratch: %s",
                             hipGetErrorString(e));
    g_base[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_base[dev];
  return SMCX_OK;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }

// Byte offsets of the workspace parts for one call.
struct Layout {
  size_t flag, n_active, k0, energy, d32, order, hist, part, part_g, total;
};

Layout layout(int64_t T_pad, int64_t N, int64_t M, int P, int32_t k_max, int nch) {
  Layout L;
  size_t o = 0;
  L.flag = o;     o += align256(sizeof(int));
  L.n_active = o; o += align256(sizeof(int32_t));
  L.k0 = o;       o += align256(sizeof(double));
  L.energy = o;   o += align256((size_t)(T_pad / kStageSpan) * sizeof(double));
  L.d32 = o;      o += align256((size_t)T_pad * sizeof(float));
  L.order = o;    o += align256((size_t)N * sizeof(int32_t));
  L.hist = o;     o += align256((size_t)smcx::prep_slices(N) * (k_max + 1) * sizeof(int32_t));
  L.part = o;     o += nch > 1 ? align256((size_t)nch * N * sizeof(double)) : 0;
  L.part_g = o;   o += nch > 1 ? align256((size_t)nch * M * P * sizeof(double)) : 0;
  L.total = o;
  return L;
}

// FP32 copy of d zero-padded to T_pad, one FP64 partial of sum d^2 per block
// of kStageSpan samples (fixed order), and the device flag cleared.
__global__ __launch_bounds__(kStageBlock) void stage_kernel(const double* d, int64_t T,
                                                            float* d32, double* energy,
                                                            int* flag) {
  __shared__ double sh[kStageBlock];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kStageSpan;
  double s = 0.0;
  for (int j = 0; j < kStageSpan / kStageBlock; ++j) {
    const int64_t x = base + (int64_t)j * kStageBlock + tid;
    const double v = x < T ? d[x] : 0.0;
    d32[x] = (float)v;
    s = fma(v, v, s);
  }
  sh[tid] = s;
  __syncthreads();
  for (int h = kStageBlock / 2; h > 0; h >>= 1) {
    if (tid < h) sh[tid] += sh[tid + h];
    __syncthreads();
  }
  if (tid == 0) {
    energy[blockIdx.x] = sh[0];
    if (blockIdx.x == 0) *flag = 0;
  }
}

// log L of a particle without components: -||d||^2 / (2 sigma^2), the block
// partials summed in a fixed order.
__global__ __launch_bounds__(kStageBlock) void k0_kernel(const double* energy, int64_t nb,
                                                         double inv_sigma2, double* k0) {
  __shared__ double sh[kStageBlock];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int64_t b = tid; b < nb; b += kStageBlock) s += energy[b];
  sh[tid] = s;
  __syncthreads();
  for (int h = kStageBlock / 2; h > 0; h >>= 1) {
    if (tid < h) sh[tid] += sh[tid + h];
    __syncthreads();
  }
  if (tid == 0) *k0 = -0.5 * sh[0] * inv_sigma2;
}

}  // namespace

extern "C" int logl_grad_batch_static(int model, const double* d, int64_t T, double t_start,
                                      double dt, double sigma, int32_t k_max, int64_t N,
                                      const int64_t* offsets, int64_t M, const double* theta,
                                      const double* beta, double* logl, double* grad,
                                      void* hip_stream) {
  using smcx::set_error;
  if (model != SMCX_PULSE && model != SMCX_GBSINE)
    return set_error(SMCX_EINVAL, "unknown or unsupported model %d (time-domain models only)",
                     model);
  if (T < 1) return set_error(SMCX_EINVAL, "T = %lld must be at least 1", (long long)T);
  if (!d) return set_error(SMCX_EINVAL, "d is NULL");
  if (!(dt > 0.0) || !std::isfinite(dt)) return set_error(SMCX_EINVAL, "dt must be finite and > 0");
  if (!std::isfinite(t_start)) return set_error(SMCX_EINVAL, "t_start must be finite");
  if (!(sigma > 0.0) || !std::isfinite(sigma))
    return set_error(SMCX_EINVAL, "sigma must be finite and > 0");
  if (k_max < 1 || k_max > 512) return set_error(SMCX_EINVAL, "k_max = %d outside [1, 512]", k_max);
  if (N < 0 || N > INT32_MAX) return set_error(SMCX_EINVAL, "N = %lld out of range", (long long)N);
  if (M < 0) return set_error(SMCX_EINVAL, "M = %lld is negative", (long long)M);
  if (N > 0 && !offsets) return set_error(SMCX_EINVAL, "offsets is NULL");
  if (M > 0 && (!theta || !grad)) return set_error(SMCX_EINVAL, "theta or grad is NULL");
  if (N == 0) return SMCX_OK;

  const int P = smcx::n_params(model);
  const int64_t T_pad = round_up(T, kStageSpan) + kStageSpan;
  // the default tiling of the gradient pass, with longer chunks where its
  // partial sums would not fit
  Tiling t = smcx::default_tiling(model, kGrad, T);
  Layout L = layout(T_pad, N, M, P, k_max, t.nch);
  while (L.total > kScratchBytes && t.nch > 1) {
    t.chunk_len *= 2;
    t.nch = (int)((T + t.chunk_len - 1) / t.chunk_len);
    L = layout(T_pad, N, M, P, k_max, t.nch);
  }
  if (L.total > kScratchBytes)
    return set_error(SMCX_ENOMEM,
                     "logl_grad_batch_static needs %zu bytes of static scratch for T = %lld, "
                     "N = %lld, M = %lld; the limit is %zu bytes",
                     L.total, (long long)T, (long long)N, (long long)M, kScratchBytes);

  unsigned char* base = nullptr;
  int rc = scratch_base(&base);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)hip_stream;
  int* flag = reinterpret_cast<int*>(base + L.flag);
  double* k0 = reinterpret_cast<double*>(base + L.k0);
  double* energy = reinterpret_cast<double*>(base + L.energy);
  float* d32 = reinterpret_cast<float*>(base + L.d32);
  const int64_t nb = T_pad / kStageSpan;

  hipLaunchKernelGGL(stage_kernel, dim3((unsigned)nb), dim3(kStageBlock), 0, st, d, T, d32,
                     energy, flag);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k0_kernel, dim3(1), dim3(kStageBlock), 0, st, energy, nb,
                       1.0 / (sigma * sigma), k0);
    e = hipGetLastError();
  }
  if (e != hipSuccess)
    return set_error(SMCX_EDEVICE, "staging launch: %s", hipGetErrorString(e));

  smcx::PrepArgs pa;
  std::memset(&pa, 0, sizeof(pa));
  pa.offsets = offsets;
  pa.beta = beta;
  pa.N = N;
  pa.M = M;
  pa.k_max = k_max;
  pa.m_max = M;
  pa.k0_dev = k0;
  pa.P = P;
  pa.logl = logl;
  pa.grad = grad;
  pa.order = reinterpret_cast<int32_t*>(base + L.order);
  pa.n_active = reinterpret_cast<int32_t*>(base + L.n_active);
  pa.block_hist = reinterpret_cast<int32_t*>(base + L.hist);
  pa.flag = flag;
  pa.tempered = 1;
  e = smcx::launch_prep(pa, st);
  if (e != hipSuccess) return set_error(SMCX_EDEVICE, "prep launch: %s", hipGetErrorString(e));

  smcx::PopArgs a;
  std::memset(&a, 0, sizeof(a));
  a.d32 = d32;
  a.s_lo = 0;
  a.s_hi = T;
  a.t_start = t_start;
  a.dt = dt;
  a.inv_sigma2 = 1.0 / (sigma * sigma);
  a.offsets = offsets;
  a.theta = theta;
  a.beta = beta;
  a.N = N;
  a.M = M;
  a.k_max = k_max;
  a.m_max = M;
  a.k0_dev = k0;
  a.order = pa.order;
  a.n_active = pa.n_active;
  a.nch = t.nch;
  a.chunk_len = t.chunk_len;
  a.logl = logl;
  a.grad = grad;
  a.part = t.nch > 1 ? reinterpret_cast<double*>(base + L.part) : nullptr;
  a.part_g = t.nch > 1 ? reinterpret_cast<double*>(base + L.part_g) : nullptr;
  a.flag = flag;
  e = smcx::launch_fused(model, t, a, st);
  if (e != hipSuccess)
    return set_error(SMCX_EDEVICE, "logl_grad launch: %s", hipGetErrorString(e));
  return SMCX_OK;
}
