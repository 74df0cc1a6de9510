// VALU issue-rate probe: the measured ceilings the population kernels are
// compared with. Each lane runs eight independent dependency chains of one
// instruction kind (enough to cover its latency), so the kernel's time is the
// issue time of that kind at the chosen occupancy.
#include <hip/hip_runtime.h>

#include "../../include/smcx.h"
#include "smcx_internal.h"
#include "smcx_problem.h"

namespace {

constexpr int kChains = 8;
constexpr int kReps = 4;  // repetitions of the eight chains per loop iteration

template <int OP>
__device__ __forceinline__ void step(float (&x)[kChains], double (&y)[kChains],
                                     unsigned (&u)[kChains], float b, float c, double bd,
                                     double cd, unsigned ui) {
#pragma unroll
  for (int k = 0; k < kChains; ++k) {
    if constexpr (OP == SMCX_PROBE_FMA_F32) {
      x[k] = __builtin_fmaf(x[k], b, c);
    } else if constexpr (OP == SMCX_PROBE_MUL_F32) {
      x[k] = x[k] * b;
    } else if constexpr (OP == SMCX_PROBE_EXP_F32) {
      x[k] = __builtin_amdgcn_exp2f(-__builtin_fabsf(x[k]));  // modifiers are free
    } else if constexpr (OP == SMCX_PROBE_SIN_F32) {
      x[k] = __builtin_amdgcn_sinf(x[k]);
    } else if constexpr (OP == SMCX_PROBE_FMA_F64) {
      y[k] = fma(y[k], bd, cd);
    } else if constexpr (OP == SMCX_PROBE_ADD_U32) {
      // written out: the compiler would otherwise sum the chain in closed form
      asm volatile("v_add_u32 %0, %0, %1" : "+v"(u[k]) : "v"(ui));
    } else if constexpr (OP == SMCX_PROBE_CVT) {
      // v_cvt_f32_i32 of the previous result's bit pattern
      u[k] = __builtin_bit_cast(unsigned, (float)(int)u[k]);
    } else if constexpr (OP == SMCX_PROBE_FMAC_F32) {
      x[k] = __builtin_fmaf(b, c, x[k]);  // accumulator form: v_fmac_f32
    } else if constexpr (OP == SMCX_PROBE_ADD_F32) {
      x[k] = x[k] + b;
    } else if constexpr (OP == SMCX_PROBE_MUL_F64) {
      y[k] = y[k] * bd;
    } else if constexpr (OP == SMCX_PROBE_ADD_F64) {
      y[k] = y[k] + bd;
    } else if constexpr (OP == SMCX_PROBE_DPP) {
      // v_mov_b32 with a row rotation by one lane: the value walks round its row
      u[k] = (unsigned)__builtin_amdgcn_mov_dpp((int)u[k], 0x121, 0xF, 0xF, false);
    } else if constexpr (OP == SMCX_PROBE_PERMLANE32) {
      // v_permlane32_swap_b32 between chains k and k + 1 (counted once per pair)
      if ((k & 1) == 0) {
        const auto r = __builtin_amdgcn_permlane32_swap(u[k], u[k + 1], false, false);
        u[k] = r[0];
        u[k + 1] = r[1];
      }
    } else if constexpr (OP == SMCX_PROBE_ALIGNBIT) {
      // v_alignbit_b32, the funnel shift that builds the sinusoids' phase
      // float (written out: repeated shifts of one value fold to a constant)
      asm volatile("v_alignbit_b32 %0, %1, %0, 9" : "+v"(u[k]) : "v"(ui));
    } else if constexpr (OP == SMCX_PROBE_SIN_4FMA) {
      // one transcendental and four FP32 FMAs (accumulator form) per chain
      // step: whether the transcendental unit overlaps with the FP32 issue
      const float s = __builtin_amdgcn_sinf(x[k]);
      x[k] = __builtin_fmaf(b, c, s);
      x[k] = __builtin_fmaf(b, c, x[k]);
      x[k] = __builtin_fmaf(b, c, x[k]);
      x[k] = __builtin_fmaf(b, c, x[k]);
    }
  }
}

template <int OP>
__global__ __launch_bounds__(256) void probe_kernel(int32_t iters, const float* in, float* out) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const float v = in[threadIdx.x & 63];
  const float b = in[64 + (threadIdx.x & 63)], c = in[128 + (threadIdx.x & 63)];
  float x[kChains];
  double y[kChains];
  unsigned u[kChains];
#pragma unroll
  for (int k = 0; k < kChains; ++k) {
    x[k] = v + 0.01f * (float)k;
    y[k] = (double)x[k];
    u[k] = (unsigned)tid + 977u * (unsigned)k;
  }
  const double bd = (double)b, cd = (double)c;
  const unsigned ui = (unsigned)(in[192] * 16.0f) | 1u;
  for (int32_t it = 0; it < iters; ++it) {
#pragma unroll
    for (int r = 0; r < kReps; ++r) step<OP>(x, y, u, b, c, bd, cd, ui);
  }
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < kChains; ++k) acc += x[k] + (float)y[k] + (float)u[k];
  out[tid] = acc;
}

template <int OP>
hipError_t launch(int32_t blocks, int32_t iters, const float* in, float* out, hipStream_t st) {
  hipLaunchKernelGGL(probe_kernel<OP>, dim3((unsigned)blocks), dim3(256), 0, st, iters, in, out);
  return hipGetLastError();
}

}  // namespace

extern "C" int smcx_issue_probe(int op, int32_t blocks, int32_t iters, const float* in,
                                float* out, int64_t* lane_ops, void* hip_stream) {
  if (blocks < 1 || iters < 1) return smcx::set_error(SMCX_EINVAL, "blocks and iters must be >= 1");
  if (!in || !out || !lane_ops) return smcx::set_error(SMCX_EINVAL, "a pointer is NULL");
  // lane-instructions per chain and step, times two
  const int64_t per_step2 = op == SMCX_PROBE_SIN_4FMA ? 10 : op == SMCX_PROBE_PERMLANE32 ? 1 : 2;
  hipStream_t st = (hipStream_t)hip_stream;
  hipError_t e;
  switch (op) {
    case SMCX_PROBE_FMA_F32: e = launch<SMCX_PROBE_FMA_F32>(blocks, iters, in, out, st); break;
    case SMCX_PROBE_MUL_F32: e = launch<SMCX_PROBE_MUL_F32>(blocks, iters, in, out, st); break;
    case SMCX_PROBE_EXP_F32: e = launch<SMCX_PROBE_EXP_F32>(blocks, iters, in, out, st); break;
    case SMCX_PROBE_SIN_F32: e = launch<SMCX_PROBE_SIN_F32>(blocks, iters, in, out, st); break;
    case SMCX_PROBE_FMA_F64: e = launch<SMCX_PROBE_FMA_F64>(blocks, iters, in, out, st); break;
    case SMCX_PROBE_ADD_U32: e = launch<SMCX_PROBE_ADD_U32>(blocks, iters, in, out, st); break;
    case SMCX_PROBE_CVT: e = launch<SMCX_PROBE_CVT>(blocks, iters, in, out, st); break;
    case SMCX_PROBE_SIN_4FMA: e = launch<SMCX_PROBE_SIN_4FMA>(blocks, iters, in, out, st); break;
    case SMCX_PROBE_FMAC_F32: e = launch<SMCX_PROBE_FMAC_F32>(blocks, iters, in, out, st); break;
    case SMCX_PROBE_ADD_F32: e = launch<SMCX_PROBE_ADD_F32>(blocks, iters, in, out, st); break;
    case SMCX_PROBE_MUL_F64: e = launch<SMCX_PROBE_MUL_F64>(blocks, iters, in, out, st); break;
    case SMCX_PROBE_ADD_F64: e = launch<SMCX_PROBE_ADD_F64>(blocks, iters, in, out, st); break;
    case SMCX_PROBE_DPP: e = launch<SMCX_PROBE_DPP>(blocks, iters, in, out, st); break;
    case SMCX_PROBE_PERMLANE32: e = launch<SMCX_PROBE_PERMLANE32>(blocks, iters, in, out, st); break;
    case SMCX_PROBE_ALIGNBIT: e = launch<SMCX_PROBE_ALIGNBIT>(blocks, iters, in, out, st); break;
    default: return smcx::set_error(SMCX_EINVAL, "unknown probe %d", op);
  }
  if (e != hipSuccess) return smcx::set_error(SMCX_EDEVICE, "probe launch: %s", hipGetErrorString(e));
  *lane_ops = (int64_t)blocks * 256 * iters * kReps * kChains * per_step2 / 2;
  return SMCX_OK;
}
