// Definition of the problem handle, shared by the ABI and autotuner units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "smcx_internal.h"

using smcx::Tiling;

enum Kind { kFwd = 0, kGrad = 1, kDelta = 2, kNumKinds = 3 };

struct smcx_problem {
  int model = 0;
  int P = 0;
  int64_t T = 0;
  double t_start = 0, dt = 0, sigma = 0, inv_sigma2 = 0;
  int32_t k_max = 0;
  int64_t n_max = 0, m_max = 0;
  int device = 0;
  int lds_max = 0;  // LDS bytes per workgroup of the device
  int n_cu = 0;     // compute units of the device
  float* d32 = nullptr;
  double* d64 = nullptr;
  std::vector<double> prefix;  // FP64 prefix sums of d^2, prefix[s] = sum_{q<s} d_q^2
  Tiling tiling[kNumKinds];
  int64_t split = 0;  // posterior-start bridge split (smcx_set_bridge_split); 0 = prior bridge
  // frequency-domain problems (smcx_problem_create_fd)
  bool fd = false;
  int64_t fd_k0 = 0, fd_B = 0;
  double fd_T_obs = 0, fd_S = 0;
  double* fd_data = nullptr;   // [2][kFdBandStride][2], zero past B
  double* fd_src = nullptr;    // [m_max][34] source constants, rewritten by every launch
  double* fd_table = nullptr;  // kFdTableSize doubles
  smcx_problem* partner = nullptr;  // bridge partner (smcx_set_bridge_partner), or none
  int max_nch = 0;       // capacity of part (chunks per particle)
  int max_nch_grad = 0;  // capacity of part_g
  int32_t* order = nullptr;
  int32_t* n_active = nullptr;
  int32_t* prep_hist = nullptr;  // [prep_slices(n_max)][k_max + 1]
  smcx::SmcWork smc{};            // SMC-step workspace, [n_max] each
  int* flag = nullptr;
  double* part = nullptr;   // [max_nch][n_max][4]
  size_t part_cap = 0;      // doubles in part
  double* part_g = nullptr; // [nch_grad][m_max][P]
  double* rbuf = nullptr;   // plain form residual [T]
  double* bpart = nullptr;  // plain form block partials
  size_t ws_bytes = 0;      // device workspace this handle holds (all of the above and below)
  // NUTS workspace (smcx_nuts_reserve)
  int nuts_depth = 0;
  double* nuts_vec = nullptr;      // [nuts_slots][m_max * P] per-row state vectors
  void* nuts_state = nullptr;      // [n_max] per-particle scalars
  double* nuts_logl = nullptr;     // [n_max] tempered logL at the frontier
  uint8_t* nuts_active = nullptr;  // [n_max]
  int8_t* nuts_dir = nullptr;      // [n_max] direction of the current doubling
  int* nuts_count = nullptr;       // [nuts_depth + 1] particles still extending
  int32_t* nuts_list = nullptr;    // [2][n_max] active particles of a doubling and of the next
  hipStream_t nuts_capture = nullptr;
  std::vector<hipGraphExec_t> nuts_graph;  // one per doubling depth
  std::vector<uint64_t> nuts_graph_key;
  // measurement hooks
  bool prof_on = false;
  int prof_n = 0;
  std::vector<hipEvent_t> prof_ev;  // [2 * capacity]
};

namespace smcx {
// Set the thread's last-error message and return `code`.
int set_error(int code, const char* fmt, ...);
// Default tiling of call kind `kind` (Kind) for a data length T.
Tiling default_tiling(int model, int kind, int64_t T);
}  // namespace smcx
