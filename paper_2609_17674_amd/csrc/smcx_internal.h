// Internal declarations shared by the HIP translation units of libsmcx.
// Device helpers (wave reductions on gfx950 DPP), kernel argument blocks and
// the launch entry points the C ABI layer calls.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/smcx.h"

namespace smcx {

constexpr int kWave = 64;

// Device-side error flag bits (see smcx_device_status).
enum : int {
  kFlagOffsets = 1,   // offsets not monotone / offsets[0] != 0
  kFlagKMax = 2,      // a particle has K_i > k_max
  kFlagMMax = 4,      // offsets[N] != M (rows of theta passed by the caller)
  kFlagDeath = 8,     // death index outside [-1, K_i)
  kFlagPhase = 16,    // GB phase increment too large for the per-tile reduction
  kFlagCapacity = 32, // a rebuilt population needs more rows than the output holds
  kFlagWeights = 64,  // resampling weights without a positive entry
  kFlagNotPD = 128,   // a metric block is not positive definite (its factor is NaN)
};

// Per-particle workspace of the SMC steps (resampling, birth/death rebuild).
struct SmcWork {
  int64_t* cum;      // [n_max] integer weight prefix sums
  int64_t* src_row;  // [n_max] first source row of each output particle
  int32_t* src_len;  // [n_max] source rows
  int32_t* skip;     // [n_max] source row left out (-1 none)
  int32_t* append;   // [n_max] 1: a row of theta_add follows
  int64_t* count;    // [n_max] rows of each output particle
};

// Number of parameters per component.
__host__ __device__ constexpr int n_params(int model) {
  return model == SMCX_PULSE ? 3 : (model == SMCX_GBSINE ? 4 : 8);
}

// ---------------------------------------------------------------------------
// Tiling of the sample axis. A wave owns one work item = (particle, chunk);
// a chunk is walked in tiles of 64*S samples, lane l holding samples
// tile + 64*j + l, j < S, so that every load of the data is one coalesced
// 256-byte line per j. Chunks split long sample ranges across waves; their
// per-chunk partial sums are combined in a fixed order afterwards.
struct Tiling {
  int S;              // samples per lane per tile (8, 16, 32 or 64)
  int64_t chunk_len;  // samples per chunk (multiple of 64*S)
  int nch;            // chunks covering [s_lo, s_hi)
  int sorted;         // 1: items ordered by K descending (ordering pass), 0: particle order,
                      // 2: as 1 on a persistent grid (waves step through the items)
};

// Arguments of the batched population kernels (forward, fused forward +
// adjoint, birth/death, segment forward).
struct PopArgs {
  const float* d32;        // [T] data in FP32
  int64_t s_lo, s_hi;      // sample range [s_lo, s_hi)
  double t_start, dt, inv_sigma2;
  const int64_t* offsets;  // [N+1]
  const double* theta;     // [M][P]
  const double* beta;      // [N] or nullptr (beta = 1)
  int64_t N;
  int64_t M;               // rows of theta (offsets[N] must equal it)
  int32_t k_max;
  int64_t m_max;
  double k0;               // logL of a particle without components (tempered part)
  double k0_lo;            // its untempered part: samples before the split (0 without one)
  const double* k0_dev;    // device scalar used in place of k0 when set (nullptr: k0)
  int64_t split;           // posterior-start bridge: samples s < split are untempered
                           // (weight 1), later ones weighted by beta; 0 (or <= s_lo) = off
  const int32_t* order;    // [N] particles sorted by K descending, or nullptr: particle order
  const int32_t* n_active; // device scalar: number of entries of order (sorted mode)
  int nch;
  int64_t chunk_len;
  // outputs
  double* logl;            // [N] or nullptr
  double* grad;            // [M][P] or nullptr
  double* part;            // [nch][N][n_part] chunk partials when nch > 1
  double* part_g;          // [nch][m_max][P] chunk gradient partials when nch > 1
  // leapfrog mode of the fused pass (p_half != nullptr): theta holds the
  // drifted positions q'; after the gradient g' the momenta are kicked,
  // p_out = p_half + (eps_i / 2) g', with eps_i = eps * dir[i]
  const uint8_t* active;   // [N] or nullptr: particles with active[i] == 0 are skipped
  const double* p_half;    // [M][P] half-step momenta
  double* p_out;           // [M][P] full-step momenta (may be p_half itself)
  double eps;
  const int8_t* dir;       // [N] +-1 or nullptr (+1)
  // birth / death
  const double* theta_birth;  // [N][P] or nullptr
  const int32_t* death_idx;   // [N] or nullptr
  double* dlogl_birth;
  double* dlogl_death;
  int* flag;
  void* prof_stop;         // hipEvent_t the launcher records right after the population
                           // kernel (profiling), or nullptr
  // frequency-domain (LISA Galactic-binary) problems
  const double* fd_data;   // [2][kFdBandStride][2] band spectrum of A and E (re, im), zero past B
  double* fd_src;           // [M][34] source constants (the handle's workspace)
  const double* fd_table;  // per-lane coarse-grid constants and FFT twiddles
  int64_t fd_k0;           // first bin of the band
  int64_t fd_B;            // bins in the band
  double fd_T_obs;         // observation time [s]
  double fd_scale;         // T_obs / 64
  int64_t fd_split;        // gradient launches over at most this many listed particles
                           // give each particle a whole workgroup (0: never); at most
                           // the launch's workgroups
  int n_cu;                // compute units of the device (grid sizes)
  int persist;             // 1: the population kernel's grid holds what the device runs
                           // at once and each wave steps through the work items
  int stride_grid;         // 1: launches whose kernels step through the listed particles
                           // take a fixed grid per compute unit (few listed), 0: a
                           // workgroup per group of particles
  int fd_src_ready;        // 1: the caller has written fd_src for this launch's particles
  // bridge between two records (eq. reuse_bridge): the partner handle's data
  int fd_bridge;           // 1: target (1 - beta) logL_partner + beta logL_own
  const double* fd2_data;
  const double* fd2_table;
  int64_t fd2_k0, fd2_B;
  double fd2_T_obs, fd2_cnorm;
};
// Band spectra are stored at one stride, the largest band (256 bins), so
// that a kernel sized for the wider of two bridged bands reads either.
constexpr int kFdBandStride = 256;
// Doubles per row of the frequency-domain source constants (one row per
// row of theta).
constexpr int kFdSrcWords = 46;
// Layout of fd_table: [64][kFdTableStride] (tensors of A, E; cos, sin of
// the orbital phase; t_j), then the per-lane twiddles of the six FFT stages,
// [6][64][2] for the forward transform and [6][64][2] for the inverse (stage
// s has span 32 >> s; see the transform in the frequency-domain kernels for
// the lane layout), then [129][2] cos and sin of 2 pi k / 128, k = -64..64.
constexpr int kFdTableStride = 16;
constexpr int kFdTwiddleFwd = 64 * kFdTableStride;
constexpr int kFdTwiddleInv = kFdTwiddleFwd + 6 * 128;
constexpr int kFdTrig = kFdTwiddleInv + 6 * 128;
constexpr int kFdTrigSteps = 128;
constexpr int kFdTableSize = kFdTrig + 2 * (kFdTrigSteps + 1);

// Sort particles by K (descending) and settle K = 0 / invalid particles.
struct PrepArgs {
  const int64_t* offsets;
  const double* beta;
  int64_t N;
  int32_t k_max;
  int64_t m_max;
  int64_t M;           // rows of theta: offsets[N] must equal it
  double k0_value;     // untempered logL of a particle with no components (tempered part)
  double k0_lo;        // part of it before the bridge split, added untempered (0: no split)
  const double* k0_dev;  // device scalar used in place of k0_value when set (nullptr: k0_value)
  double* logl;        // written for K = 0 (tempered) and invalid (NaN) particles
  double* logl2;       // optional second output set to the K=0 value (nullptr)
  int P;
  double* grad;        // NaN rows for invalid particles (nullptr to skip)
  double* dlogl_birth; // birth/death outputs for invalid particles (nullptr to skip)
  double* dlogl_death;
  const int32_t* death_idx;  // validated against [-1, K_i) when dlogl_death is set
  int32_t* order;
  int32_t* n_active;
  int32_t* block_hist; // [prep_slices(N)][k_max + 1] workspace of the ordering pass
  int* flag;
  int tempered;        // 1: K=0 value times beta_i, 0: untempered
  int include_k0;      // 1: K = 0 particles stay in the work list (birth pass)
};

// Per-particle scalars of a NUTS transition.
struct NutsState {
  double H0;         // energy at the start point
  double lw_tree;    // log of the summed weights exp(-H) of the trajectory
  double lw_sub;     // same for the subtree being built
  double logl_prop;  // tempered logL at the trajectory proposal
  double logl_sub;   // tempered logL at the subtree proposal
  int depth;         // completed doublings
  int steps;         // leapfrog steps taken
  int status;        // 0 no components, 1 U-turn, 2 divergence, 3 maximum depth, 4 running
  int pad;
};

struct NutsArgs {
  int P;
  int D;                   // maximum tree depth
  int k_max;               // components per particle the likelihood kernels accept
  int64_t N, M;
  const int64_t* offsets;
  double eps;
  const double* prior_lo;  // [P] or nullptr
  const double* prior_hi;  // [P]
  const double* momentum;  // [M][P] standard normal draws
  const int8_t* dirs;      // [N][D]
  const double* u_leaf;    // [N][2^D - 1]
  const double* u_tree;    // [N][D]
  const uint8_t* mask;     // [N] or nullptr: particles with mask[i] == 0 stay put
  double* q;               // [M][P] in/out
  double* logl;            // [N] in/out (tempered)
  double* grad;            // [M][P] in/out (tempered)
  int32_t* depth_out;
  int32_t* steps_out;
  int32_t* status_out;
  double* vec;             // state vectors, slot k at vec + k * stride
  int64_t stride;
  NutsState* state;        // [N]
  double* logl_front;      // [N]
  uint8_t* active;         // [N]
  int8_t* dir;             // [N]
  int* count;              // [D + 1]
  // mass matrix (W^T W)^{-1}: per-particle n x n row-major blocks W at
  // wmat + w_off[i] (n = K P <= kNutsMetricMax), or with w_blocks one P x P
  // block per source row m at wmat + m P P (W block diagonal), or
  // wmat == nullptr for the identity; the momentum is then the whitened one
  const double* wmat;
  const int64_t* w_off;    // [N + 1]
  int64_t w_size;          // entries of wmat
  int w_blocks;
  // The particles still extending at the start of the current doubling,
  // list[0 .. *nlist) in no particular order (or nullptr: natural order),
  // and the list the merge fills for the next doubling (or nullptr), counting
  // in count[depth]. Particles only leave the set within a doubling.
  const int32_t* list;
  const int* nlist;
  int32_t* list_next;
  int* flag;
  int n_cu;                // compute units of the device (grid sizes)
  int stride_grid;         // 1: leaf and merge take a fixed grid per compute unit
                           // (few listed particles), 0: a workgroup per particle
};
constexpr int kNutsMetricMax = 128;  // coordinates per particle with a metric (two per lane)
constexpr int kNutsMaxDepth = 10;
constexpr int kNutsSlots(int D) { return 16 + 2 * D; }

hipError_t launch_nuts_init(const NutsArgs& a, hipStream_t st);
hipError_t launch_nuts_leaf(const NutsArgs& a, int j, int n, hipStream_t st);
hipError_t launch_nuts_merge(const NutsArgs& a, int j, hipStream_t st);
hipError_t launch_nuts_finalize(const NutsArgs& a, hipStream_t st);

// Host launchers (defined in smcx_kernels.hip / smcx_plain.hip).
hipError_t launch_prep(const PrepArgs& a, hipStream_t st);
// Number of particle slices of the ordering pass (its histogram workspace rows).
int64_t prep_slices(int64_t N);

// Gauss-Newton metric on the matrix cores (smcx_metric.hip); k_max * P <= 128.
// blocks: write only the P x P block of each component, at F + m P P for its
// source row m (f_offsets unused).
hipError_t launch_metric(int model, int P, int64_t N, int64_t M, int64_t T, double t_start,
                         double dt, double inv_sigma2, int32_t k_max, const int64_t* offsets,
                         const double* theta, const double* beta, const int64_t* f_offsets,
                         int64_t f_size, double* F, int64_t split, int blocks, int* flag,
                         hipStream_t st, const uint8_t* mask = nullptr);
// Factor W = L^{-1} of F + diag(ridge) per particle (smcx_metric.hip); ridge is
// a host array of P values; LDS bytes of one workgroup for k_max * P = nmax.
// Factor of M independent P x P blocks ([M][P][P], one thread each).
// Mean of M P x P blocks in a fixed order (part: scratch of part_cap doubles).
hipError_t launch_metric_pool(int P, int64_t M, const double* F, double* F_mean, double* part,
                              size_t part_cap, hipStream_t st);
hipError_t launch_metric_factor_blocks(int P, int64_t M, const double* F, const double* ridge,
                                       double* W, int* flag, hipStream_t st);
hipError_t launch_metric_factor(int P, int64_t N, int64_t M, int32_t k_max,
                                const int64_t* offsets, const int64_t* f_offsets, int64_t f_size,
                                const double* F, const double* ridge, int block, double* W,
                                int* flag, hipStream_t st, const uint8_t* mask = nullptr);
size_t factor_lds_bytes(int nmax);

// SMC steps (smcx_smc.hip).
// Next beta by the ESS condition; with uniform previous weights and a
// workspace of work_cap doubles large enough, spread over the device.
hipError_t launch_next_beta(int64_t N, const double* logl, const double* logw_prev,
                            double beta_prev, double alpha, double* beta_out, double* logw,
                            double* w_norm, double* scalars, double* work, size_t work_cap,
                            hipStream_t st);
hipError_t launch_resample(const SmcWork& w, int model, int32_t k_max, int64_t N,
                           const int64_t* offsets, int64_t M, const double* theta,
                           const double* w_norm, double u, int64_t m_cap, int32_t* ancestors,
                           int64_t* offsets_out, double* theta_out, int* flag, hipStream_t st);
hipError_t launch_rj_apply(const SmcWork& w, int model, int32_t k_max, int64_t N,
                           const int64_t* offsets, int64_t M, const double* theta,
                           const int8_t* move, const double* theta_birth, const int32_t* death_idx,
                           const double* dlogl_birth, const double* dlogl_death,
                           const double* log_u, int32_t k_lo, int32_t k_hi, double log_pd_over_pb,
                           int64_t m_cap, int64_t* offsets_out, double* theta_out,
                           int8_t* accepted, int* flag, hipStream_t st);
hipError_t launch_forward(int model, const Tiling& t, const PopArgs& a, hipStream_t st);
// Frequency-domain model (smcx_gblisa.hip): mode 0 logL, 1 logL + gradient
// (leapfrog kick when p_half is set), 2 birth / death changes.
hipError_t launch_fd(int mode, const PopArgs& a, hipStream_t st);
// The source constants of the particles a launch of launch_fd works on
// (launch_fd runs it first unless a.fd_src_ready).
hipError_t launch_fd_src(const PopArgs& a, hipStream_t st);
hipError_t launch_fd_spectrum(const PopArgs& a, int64_t K, double* out, hipStream_t st);
hipError_t launch_fd_metric(const PopArgs& a, const int64_t* f_offsets, int64_t f_size, double* F,
                            int blocks, hipStream_t st);
hipError_t launch_fused(int model, const Tiling& t, const PopArgs& a, hipStream_t st);
hipError_t launch_delta(int model, const Tiling& t, const PopArgs& a, hipStream_t st);
// Weights, ESS and evidence increment of reweight_extend; over many
// workgroups when the workspace (part_cap doubles) holds their range sums.
hipError_t launch_reweight_reduce(int64_t N, double delta_beta, const double* logl_ext,
                                  const double* logw_prev, double* logw, double* w_norm,
                                  double* scalars, double* part, size_t part_cap, hipStream_t st);
hipError_t launch_drift(int model, int64_t N, int64_t M, const int64_t* offsets, double eps,
                        const int8_t* dir, const uint8_t* active, const double* q_in,
                        const double* p_in, const double* g_in, double* q_out, double* p_out,
                        double* g_out, hipStream_t st);
hipError_t launch_template_sum(int model, int64_t K, const double* theta, int64_t T,
                               double t_start, double dt, double* out, hipStream_t st);
hipError_t launch_plain_particle(int model, const double* d64, int64_t T, double t_start,
                                 double dt, double inv_sigma2, const double* theta_rows, int K,
                                 const double* beta, int64_t i, double* rbuf, double* bpart,
                                 double* logl, double* grad_rows, hipStream_t st);

size_t pop_lds_bytes_per_wave(int model, int32_t k_max, bool grad);

}  // namespace smcx
