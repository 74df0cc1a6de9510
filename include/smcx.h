/*
 * smcx.h — C ABI of the population likelihood library for transdimensional
 * Sequential Monte Carlo (Demasi & Del Pozzo, "Massively parallel
 * transdimensional sampling with data assimilation").
 *
 * What the library computes. A population of N particles, particle i being
 * (K_i, theta_i) with K_i components of P parameters each (the disjoint
 * union over k of {k} x theta_k, Sec. "Reversible Jump MCMC"). Data d are T
 * samples at times t_s = t_start + s*dt with white noise of standard
 * deviation sigma. For each particle the library synthesises the summed
 * template, forms the residual
 *     r_s = d_s - sum_{k=0}^{K_i-1} h_k(t_s)
 * and reduces the noise-weighted inner product into the log-likelihood
 *     log L_i = -(1/(2 sigma^2)) sum_s r_s^2
 * (the time-domain white-noise form of eq. gw_likelihood; the constant
 * -(T/2) log(2 pi sigma^2) is dropped). All per-particle outputs are
 * tempered, i.e. multiplied by the particle's inverse temperature beta_i
 * (eq. prior_bridge raises the likelihood to beta).
 *
 * Models (component templates):
 *   SMCX_PULSE  (P=3, theta = A, t0, w):  h = A exp(-(t-t0)^2 / (2 w^2))
 *               (Sec. "Sequence of gaussian pulses"; w is a standard
 *               deviation).
 *   SMCX_GBSINE (P=4, theta = A', f0 [Hz], fdot [Hz/s], phi0 [rad]):
 *               h = A' sin(2 pi f0 t + pi fdot t^2 + phi0)
 *               (single-channel time-domain stand-in for the Galactic
 *               binaries of Sec. "LISA Galactic binaries"; A' is the
 *               amplitude after rescaling the data by 1e21).
 *   SMCX_GBLISA (P=8, theta = f0 [Hz], fdot [Hz/s], log10 A, ecliptic
 *               latitude, ecliptic longitude, psi, iota, phi0 [rad]): the
 *               Galactic binaries of Sec. "LISA Galactic binaries" in the
 *               frequency domain (smcx_problem_create_fd): channels A and E
 *               of the constellation in its long-wavelength limit, and
 *                 logL = -(1/2) (4 / (T_obs S)) sum_c sum_k |d_c[k] - h_c[k]|^2
 *               over the bins of a band (eq. gw_likelihood with a constant
 *               PSD S). Templates by the fast/slow decomposition: the
 *               heterodyned envelope at 64 points over the record, its
 *               64-point DFT filling bins floor(f0 T_obs) - 32 .. + 31.
 *               Amplitudes in units of 1e-21 strain (A = 10^(log10 A + 21)).
 *               Supported: logl_batch, logl_grad_batch, delta_logl_birth_death,
 *               smcx_leapfrog, smcx_nuts_transition(_metric) and the SMC
 *               steps and smcx_gauss_newton_metric (per-source blocks); not
 *               the time-domain calls (reweight_extend, the plain form,
 *               tiling, the bridge split).
 *
 * Layout. The population is CSR: offsets[N+1] (int64, offsets[0] = 0,
 * non-decreasing, K_i = offsets[i+1]-offsets[i]), theta[M][P] (FP64,
 * row-major, M = offsets[N]); gradients use the layout of theta.
 *
 * Ownership and streams. Every array argument is a DEVICE pointer owned by
 * the caller (for example torch.Tensor.data_ptr()). The library owns only
 * the problem handle and the device workspace it allocates in
 * smcx_problem_create. Compute calls allocate nothing, never synchronise
 * the host, and run asynchronously on `hip_stream` (a hipStream_t; NULL is
 * the default stream); results are valid in stream order. Calls that share
 * one problem handle must be ordered on one stream (they share workspace).
 *
 * Precision. Template synthesis and residual arithmetic run in FP32; the
 * Galactic-binary phase is formed and reduced modulo one cycle in FP64 (it
 * must stay below 2^19 cycles over the sample range, i.e. f t below about
 * 5e5: a component beyond that, or whose chirp moves the phase by 1/64 cycle
 * or more across a tile, gets NaN outputs and raises the device flag); the
 * per-particle inner products are accumulated in FP64 and all outputs are
 * FP64. In logl_batch, logl_grad_batch, reweight_extend and the leapfrog and
 * NUTS calls, a pulse is truncated to |t - t0| < sqrt(128 ln 2) |w| (about
 * 9.42 |w|), outside which its template is below 2^-64 of its peak. Blocks of
 * 64 samples that meet the support are evaluated whole. The truncation is far
 * under the FP32 resolution of the residual; only a component lying entirely
 * outside the sample range notices it, whose negligible gradient may then come
 * out as exactly zero. delta_logl_birth_death and smcx_plain_logl_grad
 * evaluate pulses on every sample.
 *
 * Errors. Every call returns SMCX_OK or a negative code and never throws
 * across the ABI; smcx_last_error() gives a message for the calling thread.
 * Argument errors the host can see (null pointers, negative sizes, sizes
 * above what the handle was created for, empty sample ranges) are reported
 * before any launch and leave all outputs untouched. Errors that depend on
 * device data (non-monotone offsets, offsets[N] != M, K_i > k_max, a death index
 * >= K_i) cannot be seen by the host: the kernels write NaN into the
 * affected particle's outputs and raise a device flag that
 * smcx_device_status() reports (and clears). NaN or Inf parameters only
 * affect their own particle's per-particle outputs.
 */
#ifndef SMCX_H
#define SMCX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct smcx_problem smcx_problem;

enum {
  SMCX_OK = 0,
  SMCX_EINVAL = -1,   /* bad argument, detected before launch */
  SMCX_ENOMEM = -2,   /* device allocation failed, or a size beyond a fixed workspace */
  SMCX_EDEVICE = -3,  /* HIP runtime error, or a device-side flag was raised */
  SMCX_ECAPTURE = -4  /* call not allowed while the stream is being captured */
};

enum { SMCX_PULSE = 0, SMCX_GBSINE = 1, SMCX_GBLISA = 2 };

/* Create a problem handle for one data vector.
 *   model      SMCX_PULSE or SMCX_GBSINE
 *   d_dev      [T] FP64 device data; copied (to FP32, plus FP64 energy
 *              prefix sums) during the call, need not outlive the handle
 *   T          number of samples, 1 <= T <= 2^22
 *   t_start,dt time of sample 0 and sample spacing (dt > 0)
 *   sigma      white-noise standard deviation (> 0)
 *   k_max      largest K_i any call will pass (1..512)
 *   n_max      largest N any call will pass (>= 0)
 *   m_max      largest M = offsets[N] any call will pass (>= 0)
 *   hip_stream stream used for the set-up copies; the call synchronises it
 *   out        receives the handle
 * Returns SMCX_EINVAL for bad sizes, SMCX_ENOMEM if the workspace cannot be
 * allocated or exceeds the cap below. This is the only call that allocates
 * or synchronises (with smcx_nuts_reserve).
 *
 * Workspace cap: when the environment variable SMCX_WORKSPACE_MAX holds a
 * byte count (decimal, optional suffix k, m or g for 2^10, 2^20, 2^30), the
 * calls that allocate a handle's device workspace (the two creates and
 * smcx_nuts_reserve) first add up what the handle would then hold and return
 * SMCX_ENOMEM, allocating nothing, when it exceeds the cap; an existing
 * handle stays usable as it was. A value that does not parse gives
 * SMCX_EINVAL. The variable is read at each such call. */
int smcx_problem_create(int model, const double* d_dev, int64_t T, double t_start, double dt,
                        double sigma, int32_t k_max, int64_t n_max, int64_t m_max,
                        void* hip_stream, smcx_problem** out);

/* Create a frequency-domain problem (model SMCX_GBLISA).
 *   d_dev      [2][B][2] FP64 device data: the A and E spectra (re, im) of
 *              bins k0 .. k0 + B - 1, in the convention
 *              d[k] = dt sum_n d(t_n) exp(-2 pi i k n / N_t); copied during
 *              the call
 *   k0, B      first bin and number of bins, 1 <= B <= 256
 *   T_obs      record length [s] (bin spacing 1 / T_obs); envelope samples
 *              sit at j T_obs / 64 from the start of the record
 *   psd        constant one-sided PSD S of both channels (> 0)
 *   k_max, n_max, m_max, hip_stream, out   as smcx_problem_create
 * Source windows that reach outside the band are cut at its edges. The
 * handle's calls run in FP64 throughout. Allocates and synchronises. */
int smcx_problem_create_fd(int model, const double* d_dev, int64_t k0, int64_t B, double T_obs,
                           double psd, int32_t k_max, int64_t n_max, int64_t m_max,
                           void* hip_stream, smcx_problem** out);

/* Band spectrum of K sources of the frequency-domain model (for building
 * data): out [2][B][2] FP64 (device), theta [K][8] (device), as the
 * templates of a handle with the same T_obs, k0, B. A set-up call: it
 * allocates a small table, launches one wave and synchronises. */
int smcx_template_spectrum(int model, int64_t K, const double* theta, double T_obs, int64_t k0,
                           int64_t B, double* out, void* hip_stream);

/* Free the handle and its workspace (after synchronising its last stream).
 * NULL is accepted. */
int smcx_problem_destroy(smcx_problem* prob);

/* Message describing the last error on the calling thread ("" if none). */
const char* smcx_last_error(void);

/* Synchronise `hip_stream`, then report and clear the device-side error
 * flag: SMCX_OK if no kernel saw invalid device data since the last call,
 * SMCX_EDEVICE otherwise (smcx_last_error() names the first cause). */
int smcx_device_status(smcx_problem* prob, void* hip_stream);

/* Tempered log-likelihood of every particle.
 *   logl[i] = beta_i * ( -(1/(2 sigma^2)) sum_{s<T} r_s^2 )
 * (eq. prior_bridge with the white-noise likelihood of eq. gw_likelihood).
 *   N          number of particles, 0 <= N <= n_max
 *   offsets    [N+1] int64 CSR offsets
 *   M          rows of theta, 0 <= M <= m_max; the kernels check
 *              offsets[N] == M on the device and touch no row >= M
 *   theta      [M][P] FP64
 *   beta       [N] FP64 inverse temperatures, or NULL for beta = 1
 *   logl       [N] FP64 output
 * A particle with K_i = 0 gets beta_i * (-||d||^2 / (2 sigma^2)), with
 * ||d||^2 taken in FP64 at create. */
int logl_batch(smcx_problem* prob, int64_t N, const int64_t* offsets, int64_t M,
               const double* theta, const double* beta, double* logl, void* hip_stream);

/* Tempered log-likelihood and its gradient with respect to every component
 * parameter, in one fused forward + adjoint pass that recomputes templates
 * instead of storing them:
 *   grad[m][p] = beta_i * (1/sigma^2) sum_s r_s dh_m(t_s)/dtheta_p
 * for the rows m of particle i. Hamilton's equations of the NUTS kernel
 * (Sec. "No-U-Turn-Sampler") need this gradient of the log target.
 *   logl       [N] FP64 output, or NULL to skip it
 *   grad       [M][P] FP64 output (may be NULL only if M = 0)
 * Other arguments as logl_batch. */
int logl_grad_batch(smcx_problem* prob, int64_t N, const int64_t* offsets, int64_t M,
                    const double* theta, const double* beta, double* logl, double* grad,
                    void* hip_stream);

/* logl_grad_batch for the particles with mask[i] != 0 only, as the mixture
 * kernel of eq. kernel_mixture needs: the NUTS move starts from the
 * gradient of the particles it moves. mask [N] uint8 (NULL: SMCX_EINVAL).
 * The logl and grad entries of the other particles are not computed: on
 * return they hold unspecified values. The selected particles' entries are
 * bitwise those of logl_grad_batch. */
int logl_grad_batch_masked(smcx_problem* prob, int64_t N, const int64_t* offsets, int64_t M,
                           const double* theta, const double* beta, const uint8_t* mask,
                           double* logl, double* grad, void* hip_stream);

/* Bytes of the library's static scratch array (one copy per device). */
#define SMCX_STATIC_SCRATCH_BYTES (32u << 20)

/* logl_grad_batch for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * It needs no problem handle and allocates nothing, here or in any library
 * routine it calls. Its workspace (the FP32 copy of d, the K = 0 energy, the
 * work list and the chunk partial sums) lives in a file-scope device array
 * of SMCX_STATIC_SCRATCH_BYTES per device, held until the process ends.
 *   model, T, t_start, dt, sigma, k_max   as smcx_problem_create (time-domain
 *              models only); d [T] FP64 device data, read on every call
 *   N, offsets, M, theta, beta, logl, grad   as logl_grad_batch (no n_max /
 *              m_max: the sizes are bounded by the scratch instead)
 * The pass is the default gradient tiling of the handle path, with longer
 * sample chunks where the partial sums would not fit; results agree with
 * logl_grad_batch to the library's tolerances (and are bitwise equal when
 * the tiling is the same, except for K = 0 particles, whose ||d||^2 is summed
 * on the device). Sizes whose workspace exceeds the scratch return
 * SMCX_ENOMEM before any launch; other host-visible argument errors return
 * SMCX_EINVAL. Invalid device data gives NaN outputs for the particle (there
 * is no status call for this form). Every call on a device shares that
 * device's scratch and leaves its contents behind: calls that may overlap on
 * one device (several streams or threads) race and must be serialised by the
 * caller. */
int logl_grad_batch_static(int model, const double* d, int64_t T, double t_start, double dt,
                           double sigma, int32_t k_max, int64_t N, const int64_t* offsets,
                           int64_t M, const double* theta, const double* beta, double* logl,
                           double* grad, void* hip_stream);

/* Change of the tempered log-likelihood under the nested birth and death
 * moves of Sec. "Reversible Jump MCMC" (k' = k +- 1, unit Jacobian; the
 * acceptance ratio of eq. rj_acceptance needs exactly this change):
 *   birth of theta_birth[i] appended after the K_i existing components:
 *     dlogl_birth[i] =  beta_i (<r, h_new> - <h_new, h_new>/2) / sigma^2
 *   death of the component with local index j = death_idx[i]:
 *     dlogl_death[i] = -beta_i (<r_-j, h_j> - <h_j, h_j>/2) / sigma^2
 * where r_-j is the residual with component j left out of the index-order
 * template sum. Both are computed in one pass over the data. A birth
 * followed by the death of the appended component gives exactly
 * dlogl_birth + dlogl_death = 0 (same arithmetic on both sides).
 *   theta_birth [N][P] FP64, or NULL (then dlogl_birth is not written)
 *   death_idx   [N] int32 local index in [0, K_i) or -1 for "no death"
 *               (dlogl_death[i] = 0), or NULL (dlogl_death not written)
 *   dlogl_birth, dlogl_death  [N] FP64 outputs (NULL allowed only together
 *               with a NULL theta_birth / death_idx respectively) */
int delta_logl_birth_death(smcx_problem* prob, int64_t N, const int64_t* offsets, int64_t M,
                           const double* theta, const double* beta, const double* theta_birth,
                           const int32_t* death_idx, double* dlogl_birth, double* dlogl_death,
                           void* hip_stream);

/* delta_logl_birth_death for the particles with mask[i] != 0 only (in the
 * mixture kernel of eq. kernel_mixture, those that propose a birth or a
 * death). mask [N] uint8 (NULL: SMCX_EINVAL). The other particles'
 * dlogl_birth and dlogl_death entries hold unspecified values on return;
 * the selected ones are bitwise those of delta_logl_birth_death. */
int delta_logl_birth_death_masked(smcx_problem* prob, int64_t N, const int64_t* offsets,
                                  int64_t M, const double* theta, const double* beta,
                                  const uint8_t* mask, const double* theta_birth,
                                  const int32_t* death_idx, double* dlogl_birth,
                                  double* dlogl_death, void* hip_stream);

/* Data-assimilation reweighting (eq. reuse_bridge, eq. incremental_weight,
 * eq. ess and the evidence ratio of Sec. "Sequential Monte Carlo").
 * The handle is built over the longer data segment d2; samples [0, T1) are
 * the earlier segment d1 and [T1, T2) the new samples. For white noise the
 * ratio p(theta|d2)/p(theta|d1) of eq. reuse_bridge is, up to a constant,
 * exp(logl_ext) with the untempered log-likelihood of the new samples
 *   logl_ext[i] = -(1/(2 sigma^2)) sum_{s=T1}^{T2-1} r_s^2
 * (templates at the absolute times of d2), so the log incremental weight
 * for a step delta_beta is
 *   logw[i] = logw_prev[i] + delta_beta * logl_ext[i]
 * and, with m = max_i logw[i],
 *   w_norm[i]  = exp(logw[i] - m) / sum_j exp(logw[j] - m)
 *   scalars[0] = ESS = (sum w)^2 / sum w^2
 *   scalars[1] = log Z_t/Z_{t-1} = log sum exp(logw) - log sum exp(logw_prev)
 *                (log N for uniform previous weights)
 *   scalars[2] = m
 *   T1, T2     0 <= T1 < T2 <= T (the handle's T)
 *   logw_prev  [N] FP64 previous log weights, or NULL for uniform
 *   logl_ext, logw, w_norm [N] FP64 outputs, scalars [3] FP64 output
 * The population reductions are done in a fixed order (deterministic).
 * N = 0 gives scalars {0, 0, -inf}. */
int reweight_extend(smcx_problem* prob, int64_t T1, int64_t T2, int64_t N, const int64_t* offsets,
                    int64_t M, const double* theta, double delta_beta, const double* logw_prev,
                    double* logl_ext, double* logw, double* w_norm, double* scalars,
                    void* hip_stream);

/* Synthesise a noise-free signal: out[s] = sum_{k<K} h_k(t_s), s < T, in
 * FP64 (device libm exp/sin), for building injected data sets.
 *   theta [K][P] FP64 device, out [T] FP64 device. K >= 0, T >= 0. */
int smcx_template_sum(int model, int64_t K, const double* theta, int64_t T, double t_start,
                      double dt, double* out, void* hip_stream);

/* Plain reference form of logl_grad_batch, the comparison point for the
 * batched kernels: one particle per pair of launches (a forward kernel that
 * stores the FP64 residual, then an adjoint kernel), FP64 arithmetic and
 * FP64 device-libm exp/sin/cos throughout, block reductions, no batching.
 * Same outputs as logl_grad_batch (logl may not be NULL here), but the CSR
 * offsets are a HOST array (offsets_host[N+1]) because the host loop over
 * particles needs each K_i to size its launches. It is a baseline, not a
 * production path. */
int smcx_plain_logl_grad(smcx_problem* prob, int64_t N, const int64_t* offsets_host, int64_t M,
                         const double* theta, const double* beta, double* logl, double* grad,
                         void* hip_stream);

/* One leapfrog step of Hamiltonian dynamics (Sec. "No-U-Turn-Sampler":
 * Hamilton's equations integrated with the symplectic leapfrog scheme) for
 * every active particle, with an identity mass matrix and the tempered log
 * target beta * logL (a uniform prior adds nothing inside its box):
 *   p_half = p + (e/2) g,   q' = q + e p_half,   p' = p_half + (e/2) g'
 * where e = eps * dir[i], g = beta grad logL(q) is supplied by the caller
 * (for example from logl_grad_batch or the previous step) and g' is
 * computed at q' by the fused forward + adjoint pass, whose epilogue applies
 * the closing half kick.
 *   dir        [N] int8 +1/-1 (integration direction) or NULL for +1
 *   active     [N] uint8, or NULL for all; an inactive particle's q, p, g
 *              are copied to the outputs and its logl_out is not written
 *   q_in, p_in, g_in     [M][P] FP64 state at the start
 *   q_out, p_out, g_out  [M][P] FP64 state after the step (must not overlap
 *              the inputs); logl_out [N] tempered logL at q'
 * Other arguments as logl_grad_batch. Capture-safe: two kernel launches
 * (three with the ordering pass), no allocation, no host synchronisation. */
int smcx_leapfrog(smcx_problem* prob, int64_t N, const int64_t* offsets, int64_t M,
                  const double* beta, double eps, const int8_t* dir, const uint8_t* active,
                  const double* q_in, const double* p_in, const double* g_in, double* q_out,
                  double* p_out, double* g_out, double* logl_out, void* hip_stream);

/* Reserve the device workspace of smcx_nuts_transition for trees of depth
 * up to max_depth (1..10): about (16 + 2 max_depth) m_max P doubles plus
 * small per-particle arrays. A set-up call: allocates, may synchronise.
 * SMCX_ENOMEM when the grown workspace would exceed SMCX_WORKSPACE_MAX
 * (the handle and its reserved depth are then unchanged) or an allocation
 * fails (the reserved depth is then 0 until a reserve succeeds). */
int smcx_nuts_reserve(smcx_problem* prob, int32_t max_depth);

/* One No-U-Turn transition (Sec. "No-U-Turn-Sampler") for every particle,
 * all trajectories built in lockstep on the device (multinomial NUTS,
 * generalised U-turn criterion on every balanced sub-block and on the whole
 * trajectory, divergence when the energy rises by more than 1000 or a
 * position leaves the prior box, tree depth <= max_depth, identity metric;
 * smcx_nuts_transition_metric below takes a dense mass matrix).
 * Each doubling of depth j runs 2^j batched leapfrog steps (smcx_leapfrog's
 * arithmetic) each followed by a controller pass, and is captured once into
 * a hipGraph and replayed when use_graph != 0 (the graph is rebuilt when any
 * pointer or size argument changes). The host synchronises once per
 * doubling to learn whether any trajectory is still growing.
 *   beta, eps          tempering and leapfrog step size (eps > 0)
 *   max_depth          at most the depth reserved with smcx_nuts_reserve
 *   prior_lo, prior_hi [P] box of the uniform prior, or both NULL
 *   momentum           [M][P] standard-normal draws (initial momenta)
 *   dirs               [N][max_depth] int8 +1/-1 doubling directions
 *   u_leaf             [N][2^max_depth - 1] uniforms in [0,1); leaf n of the
 *                      doubling at depth j uses column 2^j - 1 + n
 *   u_tree             [N][max_depth] uniforms for merging subtrees
 *   mask               [N] uint8 or NULL: a particle with mask[i] == 0 is
 *                      left as it is (status 0), for mixtures of moves
 *   q, logl, grad      in: state, tempered logL and gradient at q (for
 *                      example from logl_grad_batch); out: the new state
 *   depth_out, steps_out, status_out  [N] int32 or NULL: completed
 *                      doublings, leapfrog steps, and the reason the
 *                      trajectory stopped (0 no components or masked, 1 U-turn,
 *                      2 divergence, 3 maximum depth, -1 invalid rows)
 * Returns SMCX_ECAPTURE if called during stream capture. */
int smcx_nuts_transition(smcx_problem* prob, int64_t N, const int64_t* offsets, int64_t M,
                         const double* beta, double eps, int32_t max_depth,
                         const double* prior_lo, const double* prior_hi, const double* momentum,
                         const int8_t* dirs, const double* u_leaf, const double* u_tree,
                         const uint8_t* mask, double* q, double* logl, double* grad,
                         int32_t* depth_out, int32_t* steps_out, int32_t* status_out,
                         int32_t use_graph, void* hip_stream);

/* smcx_nuts_transition with the mass matrix M_i = (W_i^T W_i)^{-1} of each
 * particle (Sec. "No-U-Turn-Sampler": momentum ~ N(0, M), kinetic energy
 * r^T M^{-1} r / 2, M the Hessian of the negative log posterior), given by
 * a factor W_i such as the one smcx_metric_factor returns: a dense
 * (K_i P)^2 row-major block at W + w_offsets[i] (device, int64 [N+1]; w_size
 * entries in W). The transition runs in whitened momentum: `momentum` holds
 * the standard-normal draws z = W p_M, each leapfrog step kicks by
 * (eps/2) W grad and drifts by eps W^T z, and the energy and the U-turn test
 * use |z|^2 and rho.z (the metric's generalised criterion). eps is then in
 * the metric's units (order one when M is the posterior's Hessian). Needs
 * k_max P <= 128. A particle whose block does not match (K_i P)^2 or lies
 * outside W keeps its state, reports status -1 and raises a device flag.
 * Other arguments and behaviour as smcx_nuts_transition; with W_i = I the
 * result equals it bitwise. */
int smcx_nuts_transition_metric(smcx_problem* prob, int64_t N, const int64_t* offsets, int64_t M,
                                const double* beta, double eps, int32_t max_depth,
                                const double* prior_lo, const double* prior_hi,
                                const double* momentum, const int8_t* dirs, const double* u_leaf,
                                const double* u_tree, const uint8_t* mask,
                                const int64_t* w_offsets, int64_t w_size, const double* W,
                                double* q, double* logl, double* grad, int32_t* depth_out,
                                int32_t* steps_out, int32_t* status_out, int32_t use_graph,
                                void* hip_stream);

/* smcx_nuts_transition_metric with a block-diagonal factor: W [M][P][P] in
 * the layout of smcx_metric_factor_blocks (the factor of source row m at
 * W + m P P), so each product with W takes P terms per coordinate instead of
 * K_i P. The result equals smcx_nuts_transition_metric's with the dense W
 * that has these blocks on its diagonal and zeros elsewhere. Other arguments
 * and behaviour as smcx_nuts_transition_metric (k_max P <= 128). */
int smcx_nuts_transition_metric_blocks(smcx_problem* prob, int64_t N, const int64_t* offsets,
                                       int64_t M, const double* beta, double eps,
                                       int32_t max_depth, const double* prior_lo,
                                       const double* prior_hi, const double* momentum,
                                       const int8_t* dirs, const double* u_leaf,
                                       const double* u_tree, const uint8_t* mask, const double* W,
                                       double* q, double* logl, double* grad, int32_t* depth_out,
                                       int32_t* steps_out, int32_t* status_out, int32_t use_graph,
                                       void* hip_stream);

/* Tiling of the sample axis, per call kind: SMCX_KIND_LOGL (logl_batch and
 * the segment pass of reweight_extend), SMCX_KIND_GRAD (logl_grad_batch),
 * SMCX_KIND_DELTA (delta_logl_birth_death). A wave owns one (particle,
 * chunk) work item and walks the chunk in tiles of 64*S samples.
 *   S          samples per lane per tile: 8, 16, 32 or 64 (DELTA: 8 or 16)
 *   chunk_len  samples per chunk, a positive multiple of 64*S; the number of
 *              chunks ceil(T / chunk_len) must fit the workspace sized at
 *              create (at most min(64, ceil(T/1024)) chunks, and for GRAD
 *              with more than one chunk at most min(32, ceil(T/4096)))
 *   sorted     1: an ordering pass schedules particles longest-K first;
 *              0: particles are scheduled in index order; 2: longest-K first
 *              on a persistent grid (SMCX_KIND_LOGL and SMCX_KIND_GRAD: as
 *              many workgroups as the device holds at once, each wave taking
 *              the work items at a fixed stride; SMCX_KIND_DELTA runs as 1)
 * The tiling fixes the summation order inside a particle, so results are
 * bitwise reproducible for a fixed tiling (and independent of N and of the
 * other particles), and change only within rounding when it changes. The
 * defaults depend on the model and T only. Returns SMCX_EINVAL for values
 * outside these ranges. */
enum { SMCX_KIND_LOGL = 0, SMCX_KIND_GRAD = 1, SMCX_KIND_DELTA = 2 };
int smcx_set_tiling(smcx_problem* prob, int32_t kind, int32_t S, int64_t chunk_len,
                    int32_t sorted);
int smcx_get_tiling(smcx_problem* prob, int32_t kind, int32_t* S, int64_t* chunk_len,
                    int32_t* sorted);

/* Autotuner: for call kind `kind`, time every supported tiling (S, chunk
 * length, ordering) on the given population with HIP events (one warm-up
 * and `reps` timed calls each), apply the fastest to the handle and report
 * it. If `cache_path` is not NULL it names a plain-text cache: a matching
 * entry for (device architecture, model, T, kind, k_max) is applied without
 * timing, and a new result is appended. The population arguments are those
 * of the call kind (for SMCX_KIND_DELTA the population's own rows serve as
 * birth candidates). This is a set-up call: it allocates temporary device
 * buffers, synchronises `hip_stream`, and returns SMCX_ECAPTURE during
 * stream capture. Needs N >= 1 and M >= 1. */
int smcx_autotune(smcx_problem* prob, int32_t kind, int64_t N, const int64_t* offsets, int64_t M,
                  const double* theta, const double* beta, int32_t reps, const char* cache_path,
                  void* hip_stream, int32_t* out_S, int64_t* out_chunk_len, int32_t* out_sorted,
                  double* out_ms);

/* Gauss-Newton mass matrix for NUTS (Sec. "No-U-Turn-Sampler" takes the
 * Hessian of the negative log posterior as the metric): per particle
 *   F_i = (beta_i / sigma^2) sum_s J_s J_s^T,
 * J_s = the template partials dh_k(t_s)/dtheta_{k,p} (entry k P + p), i.e.
 * the Hessian of -beta logL without its residual term (exact where the
 * residual vanishes), as a dense (K_i P) x (K_i P) FP64 row-major matrix at
 * F + f_offsets[i]. f_offsets [N+1] (device, int64) are the caller's block
 * starts: f_offsets[i+1] - f_offsets[i] must equal (K_i P)^2 (else the
 * particle is skipped and the device flag raised); f_size is the length of F.
 * Computed on the matrix cores: J is formed in FP32 in natural units
 * (s = (1, w, w) for pulses, (1, 1/T_obs, 1/T_obs^2, 1) for sinusoids),
 * rounded to FP16, and J^T J accumulated in FP32 (flushed to FP64 every 4096
 * samples). The relative error of an entry is then bounded by about 1e-3 of
 * sqrt(F_aa F_cc), ample for a preconditioner. Requires k_max P <= 128.
 * With a bridge split set (smcx_set_bridge_split) it is the metric of the
 * bridge target: samples before the split enter with weight 1, later ones
 * with beta_i. beta may be NULL (1). Every sample is evaluated (no pulse
 * truncation). For the frequency-domain model (SMCX_GBLISA) the metric is
 * kept per source: block k is the Gauss-Newton Hessian in that source's
 * eight parameters over its 64-bin window, computed in FP64 from the
 * envelope derivatives by Parseval's identity, and blocks between sources
 * are zero; there k_max is not limited (the k_max P <= 128 bound above is
 * the time-domain kernel's). */
int smcx_gauss_newton_metric(smcx_problem* prob, int64_t N, const int64_t* offsets, int64_t M,
                             const double* theta, const double* beta, const int64_t* f_offsets,
                             int64_t f_size, double* F, void* hip_stream);

/* smcx_gauss_newton_metric for the particles with mask[i] != 0 (in the
 * mixture kernel of eq. kernel_mixture, those the NUTS move takes); the
 * others get zero matrices, which the ridge of smcx_metric_factor makes
 * definite. mask [N] uint8 (NULL: SMCX_EINVAL). The selected particles'
 * matrices are bitwise those of smcx_gauss_newton_metric. */
int smcx_gauss_newton_metric_masked(smcx_problem* prob, int64_t N, const int64_t* offsets,
                                    int64_t M, const double* theta, const double* beta,
                                    const uint8_t* mask, const int64_t* f_offsets, int64_t f_size,
                                    double* F, void* hip_stream);

/* Factor of the NUTS mass matrix built from the metric (Sec. "No-U-Turn-
 * Sampler": mass matrix = Hessian of the negative log posterior). Per
 * particle M_i = F_i + diag(ridge), ridge[p] (host array, P values >= 0)
 * added to the diagonal entry of parameter p of every component -- a floor
 * where F is singular, e.g. the uniform prior's precision 12 / width^2 --
 * factored as M_i = L L^T (Cholesky, FP64) and inverted: W_i = L^{-1}, lower
 * triangular, written as a dense (K_i P)^2 row-major block at W + f_offsets[i]
 * with zeros above the diagonal, so that M_i^{-1} = W_i^T W_i. Only the lower
 * triangle of each F block is read; W may equal F (in place). A block that
 * is not numerically positive definite (a pivot <= 0 or NaN) is written as
 * NaN and raises a device flag; offsets that disagree with (K_i P)^2 or
 * blocks beyond f_size skip the particle and raise a flag. One workgroup per
 * particle keeps its triangle in LDS: needs k_max P <= 128 and
 * (k_max P)(k_max P + 1)/2 doubles of LDS per workgroup (SMCX_EINVAL
 * otherwise). block = 0 factors the whole matrix; block = b (dividing P)
 * factors its block-diagonal part in b x b blocks and writes zeros between
 * them -- exact when F is block-diagonal, as the frequency-domain model's
 * per-source metric is with b = 8 -- using b (b + 1)/2 doubles of LDS.
 * Capture-safe: one launch, no allocation. */
int smcx_metric_factor(smcx_problem* prob, int64_t N, const int64_t* offsets, int64_t M,
                       const int64_t* f_offsets, int64_t f_size, const double* F,
                       const double* ridge, int32_t block, double* W, void* hip_stream);

/* smcx_metric_factor for the particles with mask[i] != 0 (those the NUTS
 * move of eq. kernel_mixture takes, whose transition reads nothing else of
 * W); the other particles' W entries are not written. mask [N] uint8 (NULL:
 * SMCX_EINVAL). The selected particles' factors are bitwise those of
 * smcx_metric_factor. */
int smcx_metric_factor_masked(smcx_problem* prob, int64_t N, const int64_t* offsets, int64_t M,
                              const uint8_t* mask, const int64_t* f_offsets, int64_t f_size,
                              const double* F, const double* ridge, int32_t block, double* W,
                              void* hip_stream);

/* Block-diagonal mass matrices kept per source (Sec. "No-U-Turn-Sampler";
 * the frequency-domain model's metric is exactly block diagonal, one P x P
 * block per source). The three calls below use one layout: a device FP64
 * array [M][P][P], the row-major block of source row m of theta at m P P.
 * It holds M P^2 doubles where the dense layout holds sum_i (K_i P)^2.
 *
 * smcx_gauss_newton_metric_blocks: the diagonal blocks of the metric of
 * smcx_gauss_newton_metric (same definition, precision and bridge
 * behaviour), F [M][P][P] written for the source rows of the N particles.
 * Nothing between blocks is written or needed. Time-domain models compute
 * the whole metric on the matrix cores and keep its per-component blocks
 * (k_max P <= 128); the frequency-domain model computes only its blocks
 * (any k_max). Capture-safe. */
int smcx_gauss_newton_metric_blocks(smcx_problem* prob, int64_t N, const int64_t* offsets,
                                    int64_t M, const double* theta, const double* beta, double* F,
                                    void* hip_stream);

/* smcx_gauss_newton_metric_blocks for the particles with mask[i] != 0; the
 * other particles' blocks are zero (see smcx_gauss_newton_metric_masked).
 * mask [N] uint8 (NULL: SMCX_EINVAL). */
int smcx_gauss_newton_metric_blocks_masked(smcx_problem* prob, int64_t N, const int64_t* offsets,
                                           int64_t M, const double* theta, const double* beta,
                                           const uint8_t* mask, double* F, void* hip_stream);

/* smcx_metric_factor for the block layout: for each of the M blocks,
 * W_m = L_m^{-1} with L_m L_m^T = F_m + diag(ridge) (ridge: host array of P
 * values >= 0), lower triangular with zeros above the diagonal, so that
 * M_m^{-1} = W_m^T W_m. Each block is factored as smcx_metric_factor's block
 * mode factors it. A block with a pivot that is not > 0 (or NaN) is written
 * as NaN and raises the device flag; the others are unaffected. W may equal
 * F. One thread per block, no LDS; capture-safe. */
int smcx_metric_factor_blocks(smcx_problem* prob, int64_t M, const double* F, const double* ridge,
                              double* W, void* hip_stream);

/* The population-level mass matrix of a mutation step: the mean of the M
 * per-source blocks F [M][P][P] (smcx_gauss_newton_metric_blocks' layout),
 * written to F_mean [P][P]. Sec. "No-U-Turn-Sampler" sets the mass matrix to
 * the Hessian of the negative log posterior without saying where it is
 * taken; a matrix taken at each particle's own position would make the NUTS
 * move not leave the tempered target invariant (the reverse move would use
 * another matrix), while one matrix for the whole population, fixed for the
 * step, does. Summed in a fixed order (bitwise reproducible); 1 <= M <=
 * m_max. Uses the handle's workspace: order calls on one stream. */
int smcx_metric_pool_blocks(smcx_problem* prob, int64_t M, const double* F, double* F_mean,
                            void* hip_stream);

/* Posterior-start bridge (eq. reuse_bridge). For white noise the bridge
 * p(theta|d1) (p(theta|d2)/p(theta|d1))^beta from the posterior on the first
 * `split` samples d1 to the posterior on all T samples d2 has the
 * log-likelihood part
 *   logL_split = -(1/(2 sigma^2)) [ sum_{s<split} r_s^2 + beta sum_{s>=split} r_s^2 ]
 * After smcx_set_bridge_split(prob, split) every tempered call on the handle
 * (logl_batch, logl_grad_batch, delta_logl_birth_death, smcx_leapfrog,
 * smcx_nuts_transition) evaluates this target with beta_i from its beta
 * argument: samples before the split enter untempered, later ones weighted
 * by beta_i (gradients and birth/death changes likewise). split = 0, the
 * default, is the prior bridge of eq. prior_bridge (beta times logL);
 * split = T the untempered posterior. reweight_extend is not affected (its
 * segment log-likelihood is untempered), and smcx_plain_logl_grad refuses
 * to run while a split is set. The incremental weights of this bridge are
 * (beta - beta_prev) times the untempered log-likelihood of samples
 * [split, T), which reweight_extend(prob, split, T, ...) computes.
 * smcx_gauss_newton_metric follows the split as well.
 * 0 <= split <= T. */
int smcx_set_bridge_split(smcx_problem* prob, int64_t split);

/* Posterior-start bridge between two frequency-domain records (eq.
 * reuse_bridge for the Galactic-binary model, whose bins all change when
 * the record grows): after smcx_set_bridge_partner(prob, partner) every
 * tempered call on prob (logl_batch, logl_grad_batch, delta_logl_birth_death,
 * smcx_leapfrog, smcx_nuts_transition(_metric), smcx_gauss_newton_metric)
 * evaluates
 *   (1 - beta_i) logL_partner + beta_i logL_prob
 * (and the matching gradients, changes and metric), where partner holds the
 * shorter record d1 and prob the longer one d2; beta = NULL gives logL_prob.
 * The incremental weights of this bridge are (beta - beta_prev) times
 * logL_prob - logL_partner (two untempered logl_batch calls, one per handle).
 * Both handles must be frequency-domain handles of the same model; the
 * partner must outlive the setting and have no partner itself; NULL clears.
 * The partner's data are read, its workspace is not used. */
int smcx_set_bridge_partner(smcx_problem* prob, smcx_problem* partner);
int smcx_get_bridge_split(smcx_problem* prob, int64_t* split);

/* ---- SMC steps around the likelihood (Sec. "Sequential Monte Carlo",
 * Sec. "Algorithm and implementation") ---------------------------------- */

/* Next inverse temperature of the prior bridge (eq. prior_bridge), chosen by
 * the ESS condition of eq. ess_target, with the incremental weights of
 * eq. incremental_weight, log w_i = logw_prev_i + (beta - beta_prev) logl_i,
 * and the ESS of eq. ess.
 *   logl       [N] UNTEMPERED log-likelihoods (logl_batch with beta = NULL)
 *   logw_prev  [N] log weights carried over, or NULL for uniform ones
 *   beta_prev  current inverse temperature in [0, 1]; alpha in (0, 1]
 * beta = 1 when ESS(1) >= alpha N; otherwise the root in the bracket
 * [beta_prev, 1], found by a bracketing search that keeps the lower end where
 * ESS >= alpha N: regula falsi on log(ESS / alpha N) in its Illinois form,
 * with the midpoint wherever the secant point is not strictly inside, until
 * the bracket is 1e-14 of (upper end - beta_prev) or no point lies strictly
 * inside. beta is that lower end, a tested point, so ESS(beta) >= alpha N;
 * it is the bisection root of eq. ess_target to that width. If the previous
 * weights alone have ESS < alpha N the bracket is halved instead (at most 60
 * times) and beta is its upper end, next to beta_prev.
 * Outputs (device): beta_out [N] every entry set to beta (ready for the
 * tempered calls; may be NULL), logw [N], w_norm [N] normalised weights,
 * scalars [4] = {beta, ESS(beta), log Z_t/Z_{t-1}, ESS evaluations of the
 * search}; the evidence increment is log sum exp(log w) - log sum
 * exp(logw_prev) (log N for uniform previous weights). N in [1, n_max].
 * One single-block launch; no allocation, no host synchronisation. */
int smcx_next_beta(smcx_problem* prob, int64_t N, const double* logl, const double* logw_prev,
                   double beta_prev, double alpha, double* beta_out, double* logw,
                   double* w_norm, double* scalars, void* hip_stream);

/* Systematic resampling of the population by its normalised weights (the
 * paper leaves the scheme open; systematic resampling is the reading taken).
 * Weights become integers c_i = round(w_norm_i 2^40) (0 unless w_norm_i > 0),
 * with exact int64 prefix sums C_i and total C; offspring j takes position
 * U_j = floor(((j + u) C) / N) in double precision (evaluated in that order,
 * capped at C - 1) and ancestor a_j = min{i : C_i > U_j}. The same inputs
 * therefore give the same ancestors on any implementation.
 *   offsets, M, theta   the population (validated on the device as for
 *                       logl_batch; an invalid particle contributes no rows)
 *   w_norm [N], u in [0, 1)
 *   ancestors [N] int32, offsets_out [N+1] int64, theta_out [m_cap][P]
 * The new population is the ancestors' rows in CSR form. If it needs more
 * than m_cap rows the device flag is raised (smcx_device_status) and rows
 * past m_cap are not written; m_cap = N k_max always suffices. Weights
 * without a positive entry raise the flag and keep every particle. The
 * outputs must not overlap the inputs. N in [1, n_max]. */
int smcx_resample_systematic(smcx_problem* prob, int64_t N, const int64_t* offsets, int64_t M,
                             const double* theta, const double* w_norm, double u, int64_t m_cap,
                             int32_t* ancestors, int64_t* offsets_out, double* theta_out,
                             void* hip_stream);

/* Accept/reject of the birth and death moves of the mutation kernel
 * (eq. kernel_mixture; Sec. "Reversible Jump Markov Chain Monte Carlo",
 * eq. rj_acceptance) and the rebuilt population.
 *   move [N] int8: 0 keep, 1 birth of theta_birth[i] (drawn from the
 *       single-component prior), 2 death of component death_idx[i]
 *   dlogl_birth, dlogl_death [N]: the tempered changes from
 *       delta_logl_birth_death for the same proposals
 *   log_u [N]: logs of uniforms; k_lo <= k_hi <= k_max: the uniform prior
 *       range of K; log_pd_over_pb = log(p_death / p_birth)
 * Reading of the ratio: components are exchangeable, so a birth is taken to
 * insert at one of the k+1 positions uniformly (equal to appending, up to an
 * order the target ignores) and a death to remove a uniformly chosen
 * component; the 1/(k+1) factors cancel, the prior density of the new
 * component cancels its proposal density and the Jacobian is one, leaving
 *   birth: log alpha = dlogl_birth + log_pd_over_pb   (K + 1 <= k_hi)
 *   death: log alpha = dlogl_death - log_pd_over_pb   (K - 1 >= k_lo,
 *                                                       0 <= death_idx < K)
 * and -inf otherwise; a move is accepted when log_u < log alpha (a NaN
 * change is rejected). An accepted birth appends its row last, an accepted
 * death removes its row, the other rows keep their order.
 * Outputs: offsets_out [N+1], theta_out [m_cap][P] (capacity handled as in
 * smcx_resample_systematic; m_cap = M + N always suffices), accepted [N]
 * int8. The outputs must not overlap the inputs. */
int smcx_rj_apply(smcx_problem* prob, int64_t N, const int64_t* offsets, int64_t M,
                  const double* theta, const int8_t* move, const double* theta_birth,
                  const int32_t* death_idx, const double* dlogl_birth, const double* dlogl_death,
                  const double* log_u, int32_t k_lo, int32_t k_hi, double log_pd_over_pb,
                  int64_t m_cap, int64_t* offsets_out, double* theta_out, int8_t* accepted,
                  void* hip_stream);

/* Measurement hooks. Between smcx_profile_begin and smcx_profile_end every
 * compute call on the handle brackets its batched kernel launches (the
 * population kernel and, for split sample ranges, its combine pass; not the
 * ordering pass) with a pair of HIP events recorded on the call's stream,
 * for at most max_launches calls. smcx_profile_end synchronises those
 * events and returns the summed elapsed time and the number of bracketed
 * calls. Calls made while the stream is being captured are not bracketed.
 * begin creates the events (host-side HIP objects, no device memory). */
int smcx_profile_begin(smcx_problem* prob, int32_t max_launches);
int smcx_profile_end(smcx_problem* prob, double* total_ms, int64_t* launches);

/* Instruction kinds of smcx_issue_probe. */
enum {
  SMCX_PROBE_FMA_F32 = 0,   /* v_fma_f32 */
  SMCX_PROBE_MUL_F32 = 1,   /* v_mul_f32 */
  SMCX_PROBE_EXP_F32 = 2,   /* v_exp_f32 (base 2) */
  SMCX_PROBE_SIN_F32 = 3,   /* v_sin_f32 (argument in revolutions) */
  SMCX_PROBE_FMA_F64 = 4,   /* v_fma_f64 */
  SMCX_PROBE_ADD_U32 = 5,   /* v_add_u32 */
  SMCX_PROBE_CVT = 6,       /* v_cvt_f32_i32 */
  SMCX_PROBE_SIN_4FMA = 7,  /* one v_sin_f32 and four v_fmac_f32 per step */
  SMCX_PROBE_FMAC_F32 = 8,  /* v_fmac_f32 (the two-operand accumulator form) */
  SMCX_PROBE_ADD_F32 = 9,   /* v_add_f32 */
  SMCX_PROBE_MUL_F64 = 10,  /* v_mul_f64 */
  SMCX_PROBE_ADD_F64 = 11,  /* v_add_f64 */
  SMCX_PROBE_DPP = 12,      /* v_mov_b32 with a DPP row rotation */
  SMCX_PROBE_PERMLANE32 = 13, /* v_permlane32_swap_b32 */
  SMCX_PROBE_ALIGNBIT = 14    /* v_alignbit_b32 */
};

/* The measured VALU ceilings the roofline of the population kernels refers
 * to (the vector issue limit of the chip, not an operation of the paper's
 * method). Launches `blocks` workgroups of 256 lanes; every lane runs
 * 32 * iters steps of eight independent dependency chains of instruction
 * kind `op`, so the kernel time divided into *lane_ops (set on return: the
 * number of lane-instructions the launch issues) is that kind's issue rate
 * at the occupancy the grid gives (blocks = compute units x waves per SIMD).
 * in: [256] FP32 device inputs (chain seeds); out: [blocks * 256] FP32
 * device outputs (chain results, so that nothing is optimised away). The
 * caller times the launch (events on hip_stream). */
int smcx_issue_probe(int op, int32_t blocks, int32_t iters, const float* in, float* out,
                     int64_t* lane_ops, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* SMCX_H */
