// Batched No-U-Turn transition kernels (Sec. "No-U-Turn-Sampler").
//
// Every particle builds its own trajectory by repeated doubling; since a
// doubling at depth j always has 2^j leapfrog steps, all particles that are
// still extending sit at the same (depth, leaf) position and advance in
// lockstep, one batched gradient evaluation per leaf. A particle that stops
// (U-turn, divergence, maximum depth) simply drops out of the active mask,
// so trajectory lengths are ragged. The variant is multinomial NUTS:
//  * within a subtree, leaf n replaces the subtree proposal with probability
//    w_n / (sum of subtree weights so far), w = exp(-H);
//  * a completed subtree replaces the trajectory proposal with probability
//    min(1, W_subtree / W_trajectory);
//  * the generalised U-turn test on a segment with momentum sum rho and end
//    momenta p_a, p_b stops when rho.p_a <= 0 or rho.p_b <= 0; it is applied
//    to every balanced block of the subtree as the block completes, and to
//    the whole trajectory after each doubling;
//  * a leaf whose energy exceeds the initial one by more than 1000, or that
//    leaves the prior box, is a divergence and stops the trajectory;
//  * a subtree that turns or diverges is discarded.
// Random numbers are inputs: one direction per doubling, one uniform per
// leaf and one per doubling.
//
// With a mass matrix M = (W^T W)^{-1} (the section's Hessian metric, W the
// inverse Cholesky factor of the Gauss-Newton metric) the state carries the
// whitened momentum r = W p_M, drawn N(0, I): kicks add (e/2) W g, drifts add
// e W^T r, and the energy and U-turn test keep the identity form in r. The
// closing kick of a leapfrog step then needs the whole gradient of the
// particle, so it moves from the gradient pass's epilogue into the leaf
// kernel.
//
// One workgroup of one wave handles one particle at a time; lanes run over its K*P
// coordinates (at most two each when a metric is used).
#include "smcx_internal.h"

#include <math.h>

#include <algorithm>

namespace smcx {
namespace {

__device__ __forceinline__ double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ int wany(int v) {
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o);
  return v;
}
__device__ __forceinline__ double logaddexp(double a, double b) {
  const double m = fmax(a, b);
  if (m == -INFINITY) return -INFINITY;
  return m + log(exp(a - m) + exp(b - m));
}

struct View {
  int lane;
  int64_t i, x0, x1;  // particle and its coordinate range [x0, x1)
  int K;
  bool ok;
};

__device__ __forceinline__ View view_of(const NutsArgs& a) {
  View v;
  v.lane = threadIdx.x & 63;
  v.i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  v.ok = v.i < a.N;
  if (!v.ok) return v;
  const int64_t o0 = a.offsets[v.i], o1 = a.offsets[v.i + 1];
  v.ok = o0 >= 0 && o1 >= o0 && o1 <= a.M;
  v.x0 = o0 * a.P;
  v.x1 = o1 * a.P;
  v.K = (int)(o1 - o0);
  return v;
}

// The workgroup's particle in the current doubling's list (leaf and merge),
// or in natural order when no list is given.
__device__ __forceinline__ int64_t list_count(const NutsArgs& a) {
  return a.list ? (int64_t)*a.nlist : a.N;
}
// Particle at rank r < list_count(a): the r-th listed one, or particle r.
__device__ __forceinline__ View view_at(const NutsArgs& a, int64_t r) {
  View v;
  v.lane = threadIdx.x & 63;
  v.i = a.list ? (int64_t)a.list[r] : r;
  const int64_t o0 = a.offsets[v.i], o1 = a.offsets[v.i + 1];
  v.ok = o0 >= 0 && o1 >= o0 && o1 <= a.M;
  v.x0 = o0 * a.P;
  v.x1 = o1 * a.P;
  v.K = (int)(o1 - o0);
  return v;
}

__device__ __forceinline__ double* slot(const NutsArgs& a, int k) { return a.vec + (size_t)k * a.stride; }

enum Slot { qL = 0, pL, gL, qR, pR, gR, qF, pF, gF, pH, qP, gP, qS, gS, rhoT, rhoS, kFirstCk };

__device__ __forceinline__ bool in_box(const NutsArgs& a, int64_t x, double q) {
  if (!a.prior_lo) return true;
  const int p = (int)(x % a.P);
  return q >= a.prior_lo[p] && q <= a.prior_hi[p];
}

// ---- products with the metric factor (one wave per workgroup, n <= 128)
// sh[c] = src[x0 + c], visible to the whole wave on return
__device__ __forceinline__ void stage(double* sh, const double* src, const View& v) {
  const int n = (int)(v.x1 - v.x0);
  for (int c = v.lane; c < n; c += 64) sh[c] = src[v.x0 + c];
  __syncthreads();
}
// y[t] = (W sh)_c for c = lane + 64 t (TRANS: (W^T sh)_c), c < n; the sum
// runs over c' in index order with fused multiply-adds. bs > 0: W is block
// diagonal, one bs x bs block per source (bs = P) stored one after another,
// and the sum runs over the block of c only (the dense form's other terms
// are products with zero, so both give the same value).
template <bool TRANS>
__device__ __forceinline__ void wmul(const double* W, int n, int bs, const double* sh, int lane,
                                     double y[2]) {
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int c = lane + 64 * t;
    double s = 0.0;
    if (c < n) {
      if (bs) {
        const int r = c % bs, b = c - r;  // first coordinate of c's source
        const double* B = W + (int64_t)b * bs;
        for (int k = 0; k < bs; ++k) s = fma(TRANS ? B[k * bs + r] : B[r * bs + k], sh[b + k], s);
      } else {
        for (int k = 0; k < n; ++k)
          s = fma(TRANS ? W[(int64_t)k * n + c] : W[(int64_t)c * n + k], sh[k], s);
      }
    }
    y[t] = s;
  }
}
__device__ __forceinline__ const double* wblock(const NutsArgs& a, const View& v) {
  return a.w_blocks ? a.wmat + v.x0 * a.P : a.wmat + a.w_off[v.i];
}
__device__ __forceinline__ int wbs(const NutsArgs& a) { return a.w_blocks ? a.P : 0; }

// Drift of the frontier: pH = pF + (e/2) gF, qF += e pH; with a metric
// pH = pF + (e/2) W gF, qF += e W^T pH (wg: W gF when the caller has it).
__device__ __forceinline__ void drift(const NutsArgs& a, const View& v, double e, double* sh,
                                      const double* wg_in = nullptr) {
  double *q = slot(a, qF), *p = slot(a, pF), *g = slot(a, gF), *h = slot(a, pH);
  if (!a.wmat) {
    for (int64_t x = v.x0 + v.lane; x < v.x1; x += 64) {
      const double ph = fma(0.5 * e, g[x], p[x]);
      h[x] = ph;
      q[x] = fma(e, ph, q[x]);
    }
    return;
  }
  const int n = (int)(v.x1 - v.x0);
  const double* W = wblock(a, v);
  double wg[2], y[2];
  if (wg_in) {
    wg[0] = wg_in[0];
    wg[1] = wg_in[1];
  } else {
    stage(sh, g, v);
    wmul<false>(W, n, wbs(a), sh, v.lane, wg);
    __syncthreads();
  }
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int c = v.lane + 64 * t;
    if (c < n) {
      const double ph = fma(0.5 * e, wg[t], p[v.x0 + c]);
      h[v.x0 + c] = ph;
      sh[c] = ph;
    }
  }
  __syncthreads();
  wmul<true>(W, n, wbs(a), sh, v.lane, y);
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int c = v.lane + 64 * t;
    if (c < n) q[v.x0 + c] = fma(e, y[t], q[v.x0 + c]);
  }
  __syncthreads();
}

__global__ __launch_bounds__(64) void nuts_init_kernel(NutsArgs a) {
  __shared__ double sh[kNutsMetricMax];
  if (blockIdx.x == 0 && (int)threadIdx.x <= a.D) a.count[threadIdx.x] = 0;
  const View v = view_of(a);
  if (!v.ok) {
    if (v.i < a.N && v.lane == 0) {
      a.active[v.i] = 0;
      a.state[v.i].status = -1;
    }
    return;
  }
  NutsState& s = a.state[v.i];
  double pp = 0.0;
  int out = 0;
  for (int64_t x = v.x0 + v.lane; x < v.x1; x += 64) {
    const double q = a.q[x], p = a.momentum[x], g = a.grad[x];
    pp = fma(p, p, pp);
    out |= !in_box(a, x, q);
    slot(a, qL)[x] = q; slot(a, pL)[x] = p; slot(a, gL)[x] = g;
    slot(a, qR)[x] = q; slot(a, pR)[x] = p; slot(a, gR)[x] = g;
    slot(a, qF)[x] = q; slot(a, pF)[x] = p; slot(a, gF)[x] = g;
    slot(a, qP)[x] = q; slot(a, gP)[x] = g;
    slot(a, rhoT)[x] = p;
    slot(a, rhoS)[x] = 0.0;
  }
  pp = wsum(pp);
  out = wany(out);
  const double H0 = -a.logl[v.i] + 0.5 * pp;
  // a metric block that does not match (K P)^2 or lies outside the array:
  // the particle is kept as it is, with status -1 and the offsets flag
  bool bad_w = false;
  if (a.wmat && v.K > 0) {
    const int64_t n = v.x1 - v.x0;
    if (a.w_blocks) {
      bad_w = n > kNutsMetricMax;
    } else {
      const int64_t w0 = a.w_off[v.i], w1 = a.w_off[v.i + 1];
      bad_w = n > kNutsMetricMax || w1 - w0 != n * n || w0 < 0 || w1 > a.w_size;
    }
    if (bad_w && v.lane == 0) atomicOr(a.flag, kFlagOffsets);
  }
  // more components than the likelihood kernels accept: kept, status -1, flag
  const bool bad_k = v.K > a.k_max;
  if (bad_k && v.lane == 0) atomicOr(a.flag, kFlagKMax);
  bad_w = bad_w || bad_k;
  const bool still = v.K == 0 || (a.mask && !a.mask[v.i]) || bad_w;  // no move: kept as it is
  const bool go = !still && !out && (H0 == H0) && fabs(H0) < INFINITY;
  const int8_t d = go ? a.dirs[v.i * a.D] : (int8_t)1;
  if (v.lane == 0) {
    s.H0 = H0;
    s.lw_tree = -H0;
    s.lw_sub = -INFINITY;
    s.logl_prop = a.logl[v.i];
    s.logl_sub = a.logl[v.i];
    s.depth = 0;
    s.steps = 0;
    s.status = bad_w ? -1 : (still ? 0 : (go ? 4 : 2));
    a.active[v.i] = go ? 1 : 0;
    a.dir[v.i] = d;
  }
  if (go) drift(a, v, a.eps * (double)d, sh);
}

// Leaf n of the doubling at depth j (the frontier has just been moved by one
// leapfrog step: qF, pF, gF and the frontier logL are current).
__device__ __forceinline__ void leaf_step(const NutsArgs& a, const View& v, int j, int n,
                                          double* sh) {
  if (!a.active[v.i]) return;
  NutsState& s = a.state[v.i];
  const double e = a.eps * (double)a.dir[v.i];
  double wg[2];
  if (a.wmat) {  // closing half-kick of the step: pF = pH + (e/2) W gF
    const int nc = (int)(v.x1 - v.x0);
    stage(sh, slot(a, gF), v);
    wmul<false>(wblock(a, v), nc, wbs(a), sh, v.lane, wg);
    __syncthreads();
    const double* h = slot(a, pH);
    double* pf = slot(a, pF);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int c = v.lane + 64 * t;
      if (c < nc) pf[v.x0 + c] = fma(0.5 * e, wg[t], h[v.x0 + c]);
    }
  }
  const double* q = slot(a, qF);
  const double* p = slot(a, pF);
  double pp = 0.0;
  int out = 0;
  for (int64_t x = v.x0 + v.lane; x < v.x1; x += 64) {
    pp = fma(p[x], p[x], pp);
    out |= !in_box(a, x, q[x]);
  }
  pp = wsum(pp);
  out = wany(out);
  const double lf = a.logl_front[v.i];
  const double H = out ? INFINITY : -lf + 0.5 * pp;
  if (!(H - s.H0 <= 1000.0)) {  // divergence (also NaN)
    if (v.lane == 0) {
      s.steps += 1;
      s.status = 2;
      a.active[v.i] = 0;
    }
    return;
  }
  // multinomial choice inside the subtree
  const double lw = -H;
  const double lws = logaddexp(s.lw_sub, lw);
  const double u = a.u_leaf[v.i * ((1ll << a.D) - 1) + ((1ll << j) - 1) + n];
  const bool take = u < exp(lw - lws);
  // momentum sum and checkpoints at block starts
  double* rs = slot(a, rhoS);
  const double* g = slot(a, gF);
  for (int64_t x = v.x0 + v.lane; x < v.x1; x += 64) {
    if (take) {
      slot(a, qS)[x] = q[x];
      slot(a, gS)[x] = g[x];
    }
    const double before = rs[x];
    rs[x] = before + p[x];
    for (int m = 1; m <= j; ++m) {
      if ((n & ((1 << m) - 1)) != 0) break;  // n starts blocks of 2^1 .. 2^m leaves
      slot(a, kFirstCk + (m - 1))[x] = p[x];
      slot(a, kFirstCk + a.D + (m - 1))[x] = before;
    }
  }
  // U-turn test of every block of 2^m leaves that ends at leaf n
  bool turn = false;
  for (int m = 1; m <= j && !turn; ++m) {
    if (((n + 1) & ((1 << m) - 1)) != 0) break;
    const double* ckp = slot(a, kFirstCk + (m - 1));
    const double* ckr = slot(a, kFirstCk + a.D + (m - 1));
    double dl = 0.0, dr = 0.0;
    for (int64_t x = v.x0 + v.lane; x < v.x1; x += 64) {
      const double rb = rs[x] - ckr[x];
      dl = fma(rb, ckp[x], dl);
      dr = fma(rb, p[x], dr);
    }
    dl = wsum(dl);
    dr = wsum(dr);
    turn = dl <= 0.0 || dr <= 0.0;
  }
  if (v.lane == 0) {
    if (take) s.logl_sub = lf;
    s.lw_sub = lws;
    s.steps += 1;
    if (turn) {
      s.status = 1;
      a.active[v.i] = 0;
    }
  }
  if (!turn && n < (1 << j) - 1) drift(a, v, e, sh, wg);
}

// End of the doubling at depth j: merge the (valid) subtree into the trajectory.
__device__ __forceinline__ void merge_step(const NutsArgs& a, const View& v, int j, double* sh) {
  if (!a.active[v.i]) return;
  NutsState& s = a.state[v.i];
  const bool take = a.u_tree[v.i * a.D + j] < exp(s.lw_sub - s.lw_tree);
  const int8_t d = a.dir[v.i];
  const int e0 = d > 0 ? qR : qL;
  double dl = 0.0, dr = 0.0;
  for (int64_t x = v.x0 + v.lane; x < v.x1; x += 64) {
    if (take) {
      slot(a, qP)[x] = slot(a, qS)[x];
      slot(a, gP)[x] = slot(a, gS)[x];
    }
    const double rt = slot(a, rhoT)[x] + slot(a, rhoS)[x];
    slot(a, rhoT)[x] = rt;
    slot(a, e0)[x] = slot(a, qF)[x];
    slot(a, e0 + 1)[x] = slot(a, pF)[x];
    slot(a, e0 + 2)[x] = slot(a, gF)[x];
    dl = fma(rt, slot(a, pL)[x], dl);
    dr = fma(rt, slot(a, pR)[x], dr);
  }
  dl = wsum(dl);
  dr = wsum(dr);
  const bool turn = dl <= 0.0 || dr <= 0.0;
  const int depth = j + 1;
  const bool more = !turn && depth < a.D;
  const int8_t dn = more ? a.dirs[v.i * a.D + depth] : d;
  if (v.lane == 0) {
    if (take) s.logl_prop = s.logl_sub;
    s.lw_tree = logaddexp(s.lw_tree, s.lw_sub);
    s.depth = depth;
    if (!more) {
      s.status = turn ? 1 : 3;
      a.active[v.i] = 0;
    } else {
      s.lw_sub = -INFINITY;
      a.dir[v.i] = dn;
      const int slot = atomicAdd(&a.count[depth], 1);
      if (a.list_next) a.list_next[slot] = (int32_t)v.i;
    }
  }
  if (!more) return;
  const int e1 = dn > 0 ? qR : qL;
  for (int64_t x = v.x0 + v.lane; x < v.x1; x += 64) {
    slot(a, qF)[x] = slot(a, e1)[x];
    slot(a, pF)[x] = slot(a, e1 + 1)[x];
    slot(a, gF)[x] = slot(a, e1 + 2)[x];
    slot(a, rhoS)[x] = 0.0;
  }
  drift(a, v, a.eps * (double)dn, sh);
}

// Leaf and merge over the listed particles (all of them in natural order),
// one wave per particle. STRIDED (late doublings, few listed): a grid of a
// fixed size whose workgroups step through them, as a grid as large as the
// population would pay a dispatch per particle there. Otherwise one
// workgroup per particle: a loop around the step keeps about twice the
// registers live (64 -> 127 VGPRs for the leaf), which halves the occupancy
// of full passes.
template <bool STRIDED>
__global__ __launch_bounds__(64) void nuts_leaf_kernel(NutsArgs a, int j, int n) {
  __shared__ double sh[kNutsMetricMax];
  const int64_t cnt = list_count(a);
  if constexpr (!STRIDED) {
    if ((int64_t)blockIdx.x >= cnt) return;
    const View v = view_at(a, blockIdx.x);
    if (v.ok) leaf_step(a, v, j, n, sh);
  } else {
    for (int64_t r = blockIdx.x; r < cnt; r += gridDim.x) {
      const View v = view_at(a, r);
      if (v.ok) leaf_step(a, v, j, n, sh);
      // sh is the next particle's; no barrier after the last one, whose
      // release would hold the wave until its stores complete
      if (r + gridDim.x < cnt) __syncthreads();
    }
  }
}

template <bool STRIDED>
__global__ __launch_bounds__(64) void nuts_merge_kernel(NutsArgs a, int j) {
  __shared__ double sh[kNutsMetricMax];
  const int64_t cnt = list_count(a);
  if constexpr (!STRIDED) {
    if ((int64_t)blockIdx.x >= cnt) return;
    const View v = view_at(a, blockIdx.x);
    if (v.ok) merge_step(a, v, j, sh);
  } else {
    for (int64_t r = blockIdx.x; r < cnt; r += gridDim.x) {
      const View v = view_at(a, r);
      if (v.ok) merge_step(a, v, j, sh);
      if (r + gridDim.x < cnt) __syncthreads();
    }
  }
}

__global__ __launch_bounds__(64) void nuts_finalize_kernel(NutsArgs a) {
  const View v = view_of(a);
  if (!v.ok) {
    if (v.i < a.N && v.lane == 0) {
      if (a.status_out) a.status_out[v.i] = -1;
      if (a.depth_out) a.depth_out[v.i] = 0;
      if (a.steps_out) a.steps_out[v.i] = 0;
    }
    return;
  }
  const NutsState& s = a.state[v.i];
  for (int64_t x = v.x0 + v.lane; x < v.x1; x += 64) {
    a.q[x] = slot(a, qP)[x];
    a.grad[x] = slot(a, gP)[x];
  }
  if (v.lane == 0) {
    a.logl[v.i] = s.logl_prop;
    if (a.depth_out) a.depth_out[v.i] = s.depth;
    if (a.steps_out) a.steps_out[v.i] = s.steps;
    if (a.status_out) a.status_out[v.i] = s.status;
  }
}

dim3 grid_of(int64_t N) { return dim3((unsigned)N); }  // one wave-sized workgroup per particle
// The strided leaf and merge grid: 32 wave-sized workgroups per compute unit
// (the one-pass kernels' full occupancy), at most N.
dim3 stride_grid(const NutsArgs& a) {
  const int64_t cap = 32 * (int64_t)(a.n_cu > 0 ? a.n_cu : 256);
  return dim3((unsigned)std::max<int64_t>(1, std::min(a.N, cap)));
}

}  // namespace

hipError_t launch_nuts_init(const NutsArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(nuts_init_kernel, grid_of(a.N), dim3(64), 0, st, a);
  return hipGetLastError();
}
hipError_t launch_nuts_leaf(const NutsArgs& a, int j, int n, hipStream_t st) {
  if (a.stride_grid)
    hipLaunchKernelGGL(nuts_leaf_kernel<true>, stride_grid(a), dim3(64), 0, st, a, j, n);
  else
    hipLaunchKernelGGL(nuts_leaf_kernel<false>, grid_of(a.N), dim3(64), 0, st, a, j, n);
  return hipGetLastError();
}
hipError_t launch_nuts_merge(const NutsArgs& a, int j, hipStream_t st) {
  if (a.stride_grid)
    hipLaunchKernelGGL(nuts_merge_kernel<true>, stride_grid(a), dim3(64), 0, st, a, j);
  else
    hipLaunchKernelGGL(nuts_merge_kernel<false>, grid_of(a.N), dim3(64), 0, st, a, j);
  return hipGetLastError();
}
hipError_t launch_nuts_finalize(const NutsArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(nuts_finalize_kernel, grid_of(a.N), dim3(64), 0, st, a);
  return hipGetLastError();
}

}  // namespace smcx
