// Plain FP64 form of the fused log-likelihood + gradient, one particle per
// pair of launches. It exists as the comparison point for the batched
// kernels: straightforward thread-per-sample FP64 arithmetic with device-libm
// exp/sin/cos, the residual stored in global memory between the forward and
// adjoint launches, block tree reductions, no batching and no tiling.
#include "smcx_internal.h"

#include <math.h>

namespace smcx {
namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kPi = 3.141592653589793238462643383279;

__device__ inline double plain_h(int model, const double* th, double t) {
  if (model == SMCX_PULSE) {
    const double x = t - th[1];
    return th[0] * exp(-(x * x) / (2.0 * th[2] * th[2]));
  }
  return th[0] * sin(kTwoPi * th[1] * t + kPi * th[2] * t * t + th[3]);
}

__device__ inline void plain_dh(int model, const double* th, double t, double* dh) {
  if (model == SMCX_PULSE) {
    const double A = th[0], w = th[2], x = t - th[1];
    const double e = exp(-(x * x) / (2.0 * w * w));
    dh[0] = e;
    dh[1] = A * e * x / (w * w);
    dh[2] = A * e * x * x / (w * w * w);
    dh[3] = 0.0;
  } else {
    const double A = th[0];
    const double ph = kTwoPi * th[1] * t + kPi * th[2] * t * t + th[3];
    const double s = sin(ph), c = cos(ph);
    dh[0] = s;
    dh[1] = kTwoPi * t * A * c;
    dh[2] = kPi * t * t * A * c;
    dh[3] = A * c;
  }
}

__device__ inline double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void plain_fwd_kernel(int model, const double* d, int64_t T,
                                                        double t_start, double dt,
                                                        const double* th, int K, double* rbuf,
                                                        double* bpart) {
  __shared__ double red[256];
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double r = 0.0;
  if (s < T) {
    const double t = t_start + (double)s * dt;
    double h = 0.0;
    for (int k = 0; k < K; ++k) h += plain_h(model, th + k * n_params(model), t);
    r = d[s] - h;
    rbuf[s] = r;
  }
  const double ss = block_sum(r * r, red);
  if (threadIdx.x == 0) bpart[blockIdx.x] = ss;
}

__global__ __launch_bounds__(256) void plain_adj_kernel(int model, const double* rbuf, int64_t T,
                                                        double t_start, double dt,
                                                        const double* th, int K,
                                                        const double* beta, int64_t i,
                                                        double inv_sigma2, const double* bpart,
                                                        int nb, double* logl, double* grad_rows) {
  __shared__ double red[256];
  const double b = beta ? beta[i] : 1.0;
  const int k = blockIdx.x;
  if (k == K) {  // last block: the log-likelihood from the forward partials
    if (threadIdx.x == 0) {
      double ss = 0.0;
      for (int q = 0; q < nb; ++q) ss += bpart[q];
      logl[i] = b * (-0.5 * ss * inv_sigma2);
    }
    return;
  }
  const int P = n_params(model);
  const double* tk = th + k * P;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t s = threadIdx.x; s < T; s += blockDim.x) {
    double dh[4];
    plain_dh(model, tk, t_start + (double)s * dt, dh);
    const double r = rbuf[s];
    for (int p = 0; p < 4; ++p) acc[p] += r * dh[p];
  }
  for (int p = 0; p < P; ++p) {
    const double v = block_sum(acc[p], red);
    if (threadIdx.x == 0) grad_rows[k * P + p] = b * v * inv_sigma2;
  }
}

}  // namespace

hipError_t launch_plain_particle(int model, const double* d64, int64_t T, double t_start,
                                 double dt, double inv_sigma2, const double* theta_rows, int K,
                                 const double* beta, int64_t i, double* rbuf, double* bpart,
                                 double* logl, double* grad_rows, hipStream_t st) {
  const int nb = (int)((T + 255) / 256);
  hipLaunchKernelGGL(plain_fwd_kernel, dim3(nb), dim3(256), 0, st, model, d64, T, t_start, dt,
                     theta_rows, K, rbuf, bpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(plain_adj_kernel, dim3(K + 1), dim3(256), 0, st, model, rbuf, T, t_start, dt,
                     theta_rows, K, beta, i, inv_sigma2, bpart, nb, logl, grad_rows);
  return hipGetLastError();
}

}  // namespace smcx
