// LISA Galactic binaries in the frequency domain (Sec. "LISA Galactic
// binaries"): eight parameters per source (f0, fdot, log10 A, ecliptic
// latitude and longitude, psi, iota, phi0), the A and E channels in the
// long-wavelength limit of the constellation, and the likelihood of
// eq. gw_likelihood with a constant PSD over a band of bins [k0, k0 + B):
//   logL = -(1/2) (4 / (T_obs S)) sum_c sum_k |d_c[k] - h_c[k]|^2.
//
// Templates use the fast/slow decomposition the paper's waveforms come from:
// the heterodyned envelope z_c(t) = a_c(t) e^{i(Phi(tau) - 2 pi q t / T_obs)} / 2
// (carrier bin q = floor(f0 T_obs), tau the retarded time at the guiding
// centre) is sampled at t_j = j T_obs / 64 and its 64-point DFT fills bins
// q - 32 .. q + 31:  h_c[q + m] = (T_obs / 64) sum_j z_c(t_j) e^{-2 pi i m j / 64}.
//
// Mapping: one wave per particle; lane j owns envelope sample j and band
// bins j + 64 r. A source's 64 samples go through one FFT across the wave
// (radix 2, six stages over lane pairs lane ^ h, both channels at once,
// FP64), then each lane fetches the window value of its own bins from the
// lane holding it.
// The residual stays in registers; the adjoint contracts the inverse FFT of
// each source's residual window with the analytic envelope derivatives, so
// d logL / d theta = beta (4 / (T_obs S)) (T_obs / 64) Re sum_j conj(w_j) dz_j.
// Everything is FP64: a source concentrates its signal in a few bins, where
// an FP32 template would not hold the likelihood to 1e-6.
#include "smcx_internal.h"

#include <math.h>

// The library is built without floating-point contraction so that the
// time-domain kernels round as written. These FP64 kernels are held to a
// tolerance and rely on no particular rounding of a product followed by a
// sum, so here a * b + c may fuse into one FMA.
#pragma clang fp contract(fast)

namespace smcx {
namespace {

constexpr int kNs = 64;
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kLn10 = 2.302585092994045684017991454684;
constexpr double kAuLight = 1.495978707e11 / 299792458.0;  // R / c [s]

// Per-lane constants of the coarse time grid: symmetric detector tensors
// of A and E (xx, yy, zz, xy, xz, yz), cos and sin of the orbital phase,
// t_j. Each workgroup stages them in LDS as [field][lane], so that a wave
// reads one field of all its lanes without bank conflicts; g points at this
// lane's column. Read where used, they keep 15 doubles out of the registers
// of the particle's whole pass.
constexpr int kGeoFields = 15;
struct LaneGeom {
  const double* g;
  __device__ __forceinline__ double d(int c, int x) const { return g[(6 * c + x) * 64]; }
  __device__ __forceinline__ double ca() const { return g[12 * 64]; }
  __device__ __forceinline__ double sa() const { return g[13 * 64]; }
  __device__ __forceinline__ double t() const { return g[14 * 64]; }
};

// The lane tables of a workgroup, in the dynamic LDS of the launch: the FFT
// twiddles, forward then inverse, [stage][lane][re, im] each; the phase
// table of the envelope; the grid of the handle's record; under a bridge
// that of its partner (otherwise geo[1] aliases geo[0] and takes no space).
// The gradient kernel adds one residual copy per wave after them
// (fd_lds_words).
constexpr int kTwWords = 2 * 6 * 128;
constexpr int kTrigWords = 2 * (kFdTrigSteps + 1);
constexpr int kGeoWords = kGeoFields * 64;
struct FdTables {
  const double* tw;
  const double* trig;
  const double* geo[2];
};

extern __shared__ double fd_lds[];

// Doubles of dynamic LDS a frequency-domain launch needs: the tables, plus
// resid_words per wave.
constexpr size_t fd_lds_words(bool bridge, int waves, int resid_words) {
  return (size_t)kTwWords + kTrigWords + (bridge ? 2 : 1) * kGeoWords + (size_t)waves * resid_words;
}

// Every thread of the workgroup calls this before any of them returns.
// Returns the first word after the tables.
__device__ __forceinline__ double* stage_tables(FdTables& t, const double* own, const double* partner) {
  double* tw = fd_lds;
  double* trig = tw + kTwWords;
  double* g0 = trig + kTrigWords;
  double* g1 = partner ? g0 + kGeoWords : g0;
  for (int x = threadIdx.x; x < kGeoWords; x += blockDim.x) {
    const int f = x >> 6, l = x & 63;
    g0[x] = own[l * kFdTableStride + f];
    if (partner) g1[x] = partner[l * kFdTableStride + f];
  }
  for (int x = threadIdx.x; x < kTwWords; x += blockDim.x) tw[x] = own[kFdTwiddleFwd + x];
  for (int x = threadIdx.x; x < kTrigWords; x += blockDim.x) trig[x] = own[kFdTrig + x];
  __syncthreads();
  t.tw = tw;
  t.trig = trig;
  t.geo[0] = g0;
  t.geo[1] = g1;
  return (partner ? g1 : g0) + kGeoWords;
}

// Orders the LDS accesses of one wave around it (they complete in order;
// this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct V3 {
  double x, y, z;
};
__device__ __forceinline__ double dot3(const V3& a, const V3& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 mul_sym(const double* d, const V3& v) {
  return {d[0] * v.x + d[3] * v.y + d[4] * v.z, d[3] * v.x + d[1] * v.y + d[5] * v.z,
          d[4] * v.x + d[5] * v.y + d[2] * v.z};
}

// Source constants, the same in every lane.
struct Src {
  double f0, fd, A, cb, sb, cl, sl, c2p, s2p, ci, si, cyc0;
  double Ap, Ax;  // amplitudes of h+ and hx
  // The antenna patterns Fp = cos(2 psi) P + sin(2 psi) X and
  // Fx = -sin(2 psi) P + cos(2 psi) X of the quadratic forms P = u.D u - v.D v
  // and X = 2 u.D v of a detector tensor D, as weights of its six components
  // (xx, yy, zz, xy, xz, yz): Fp = sum fpw[e] D[e], Fx = sum fxw[e] D[e].
  double fpw[6], fxw[6];
  // The weights of the forms n.D u and n.D v in the same way (the
  // zz weight of n.D v is zero, v having no z component: five words).
  double wnu[6], wnv[5];
  V3 n, u, v;  // v = (-sin l, cos l, 0)
  int64_t q;
};

// Source constants, one row of kSrcWords doubles per row of theta, written
// by fd_src_kernel before each frequency-domain launch (one thread per
// source) and read by the kernels at wave-uniform addresses through a
// restrict-qualified pointer, so they arrive by scalar loads into scalar
// registers instead of occupying vector registers in every lane. Words 0-32
// hold the constants with the carrier bin q of the handle's record, word 33
// the carrier bin under the bridge partner's observation time, words 34-44
// the weights of n.D u and n.D v, word 45 is zero.
constexpr int kSrcWords = kFdSrcWords;
constexpr int kQOwn = 32, kQPartner = 33, kWnu = 34, kWnv = 40;

// All words but the partner's carrier bin.
__device__ __forceinline__ void src_store(double* c, const Src& s) {
  const double v[33] = {s.f0,    s.fd,    s.A,     s.cb,    s.sb,    s.cl,    s.sl,
                        s.c2p,    s.s2p,    s.ci,     s.si,     s.cyc0,   s.Ap,     s.Ax,
                        s.fpw[0], s.fpw[1], s.fpw[2], s.fpw[3], s.fpw[4], s.fpw[5], s.fxw[0],
                        s.fxw[1], s.fxw[2], s.fxw[3], s.fxw[4], s.fxw[5], s.n.x,    s.n.y,
                        s.n.z,   s.u.x,   s.u.y,   s.u.z,   __builtin_bit_cast(double, s.q)};
#pragma unroll
  for (int x = 0; x < 33; ++x) c[x] = v[x];
#pragma unroll
  for (int x = 0; x < 6; ++x) c[kWnu + x] = s.wnu[x];
#pragma unroll
  for (int x = 0; x < 5; ++x) c[kWnv + x] = s.wnv[x];
  c[kSrcWords - 1] = 0.0;
}

__device__ __forceinline__ Src src_load(const double* c, int qslot) {
  Src s;
  s.f0 = c[0]; s.fd = c[1]; s.A = c[2]; s.cb = c[3]; s.sb = c[4]; s.cl = c[5]; s.sl = c[6];
  s.c2p = c[7]; s.s2p = c[8]; s.ci = c[9]; s.si = c[10]; s.cyc0 = c[11]; s.Ap = c[12]; s.Ax = c[13];
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    s.fpw[e] = c[14 + e];
    s.fxw[e] = c[20 + e];
  }
  s.n = {c[26], c[27], c[28]};
  s.u = {c[29], c[30], c[31]};
  s.v = {-s.sl, s.cl, 0.0};
  s.q = __builtin_bit_cast(int64_t, c[qslot]);  // stored as its bit pattern
#pragma unroll
  for (int x = 0; x < 6; ++x) s.wnu[x] = c[kWnu + x];
#pragma unroll
  for (int x = 0; x < 5; ++x) s.wnv[x] = c[kWnv + x];
  return s;
}

__device__ __forceinline__ Src make_src(const double* th, double T_obs) {
  Src s;
  s.f0 = th[0];
  s.fd = th[1];
  s.A = exp10(th[2] + 21.0);
  sincos(th[3], &s.sb, &s.cb);
  sincos(th[4], &s.sl, &s.cl);
  sincos(2.0 * th[5], &s.s2p, &s.c2p);
  sincos(th[6], &s.si, &s.ci);
  s.cyc0 = th[7] / kTwoPi;
  s.n = {s.cb * s.cl, s.cb * s.sl, s.sb};
  s.u = {s.sb * s.cl, s.sb * s.sl, -s.cb};
  s.v = {-s.sl, s.cl, 0.0};
  s.q = (int64_t)floor(s.f0 * T_obs);
  s.Ap = s.A * (1.0 + s.ci * s.ci);
  s.Ax = -2.0 * s.A * s.ci;
  const V3& u = s.u;
  const V3& v = s.v;
  // weights of P and X, then of the antenna patterns
  const double ep[6] = {u.x * u.x - v.x * v.x,         u.y * u.y - v.y * v.y,
                        u.z * u.z - v.z * v.z,         2.0 * (u.x * u.y - v.x * v.y),
                        2.0 * (u.x * u.z - v.x * v.z), 2.0 * (u.y * u.z - v.y * v.z)};
  const double ex[6] = {2.0 * u.x * v.x,               2.0 * u.y * v.y,
                        2.0 * u.z * v.z,               2.0 * (u.x * v.y + u.y * v.x),
                        2.0 * (u.x * v.z + u.z * v.x), 2.0 * (u.y * v.z + u.z * v.y)};
  for (int x = 0; x < 6; ++x) {
    s.fpw[x] = s.c2p * ep[x] + s.s2p * ex[x];
    s.fxw[x] = -s.s2p * ep[x] + s.c2p * ex[x];
  }
  const V3& n = s.n;
  s.wnu[0] = n.x * u.x;
  s.wnu[1] = n.y * u.y;
  s.wnu[2] = n.z * u.z;
  s.wnu[3] = n.x * u.y + n.y * u.x;
  s.wnu[4] = n.x * u.z + n.z * u.x;
  s.wnu[5] = n.y * u.z + n.z * u.y;
  s.wnv[0] = n.x * v.x;  // xx, yy, xy, xz, yz
  s.wnv[1] = n.y * v.y;
  s.wnv[2] = n.x * v.y + n.y * v.x;
  s.wnv[3] = n.z * v.x;
  s.wnv[4] = n.z * v.y;
  return s;
}

// Envelope of one source at this lane's sample, both channels (no (-1)^j).
struct Env {
  double zr[2], zi[2];  // z_c
  double ar[2], ai[2];  // complex amplitude a_c
  double Fp[2], Fx[2];  // antenna patterns
  double cph, sph, tau, doppler;  // doppler = cos(a - l) (R/c)
};

// The amplitude part of the envelope: antenna patterns, complex amplitudes,
// Doppler delay and retarded time (no phase).
__device__ __forceinline__ Env envelope_amp(const Src& s, const LaneGeom& g) {
  Env e;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    double Fp = 0.0, Fx = 0.0;
#pragma unroll
    for (int x = 0; x < 6; ++x) {
      const double D = g.d(c, x);
      Fp = fma(s.fpw[x], D, Fp);
      Fx = fma(s.fxw[x], D, Fx);
    }
    e.Fp[c] = Fp;
    e.Fx[c] = Fx;
    e.ar[c] = e.Fp[c] * s.Ap;
    e.ai[c] = -e.Fx[c] * s.Ax;
  }
  e.doppler = kAuLight * (g.ca() * s.cl + g.sa() * s.sl);
  e.tau = g.t() + s.cb * e.doppler;
  return e;
}

// cos and sin of 2 pi cyc: the nearest step k / 128 of the phase (t = 128 cyc
// and its nearest integer are exact, and so is their difference), turned
// by the remainder x = 2 pi (cyc - k / 128), |x| <= pi / 128, whose sine
// and cosine are their Taylor series cut after x^7 and x^6 (the next terms
// are below 1e-20 and 4e-18). The cut is relative to the double-precision
// ulp far smaller than the rounding of the two products that turn the step.
// The table (trig) holds cos, sin of 2 pi k / 128 for k = -64..64; the step
// is taken modulo 128, so any phase (a NaN one converts to some integer)
// indexes inside it.
__device__ __forceinline__ void cis_cycles(double cyc, const double* trig, double* c, double* s) {
  const double t = cyc * (double)kFdTrigSteps;  // exact
  const double kf = rint(t);
  const double x = (t - kf) * (kTwoPi / kFdTrigSteps);  // t - kf is exact
  const double x2 = x * x;
  const double sx = fma(x * x2, fma(x2, fma(x2, -1.0 / 5040.0, 1.0 / 120.0), -1.0 / 6.0), x);
  const double cx = fma(x2, fma(x2, fma(x2, -1.0 / 720.0, 1.0 / 24.0), -0.5), 1.0);
  const int k = ((int)kf + kFdTrigSteps / 2) & (kFdTrigSteps - 1);  // entry of the step modulo 128
  const double ck = trig[2 * k], sk = trig[2 * k + 1];
  *c = fma(ck, cx, -(sk * sx));
  *s = fma(sk, cx, ck * sx);
}

// zs: the factor of z (1/2 for the envelope itself).
__device__ __forceinline__ Env envelope(const Src& s, const LaneGeom& g, const double* trig,
                                        int lane, double zs = 0.5) {
  Env e = envelope_amp(s, g);
  // phase in cycles (heterodyned at the carrier bin q), reduced by cis_cycles
  // before the product with 2 pi
  const double cyc = fma(e.tau, fma(0.5 * s.fd, e.tau, s.f0),
                         fma(-(double)(int)(s.q & (kNs - 1)), (double)lane * (1.0 / kNs), s.cyc0));
  cis_cycles(cyc, trig, &e.cph, &e.sph);
  // zs (a_c e^{i ph}) with a_c = Ap Fp_c - i Ax Fx_c
  const double zp = zs * s.Ap, zx = zs * s.Ax;
  const double pc = zp * e.cph, ps = zp * e.sph, xc = zx * e.cph, xs = zx * e.sph;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    e.zr[c] = e.Fp[c] * pc + e.Fx[c] * xs;
    e.zi[c] = e.Fp[c] * ps - e.Fx[c] * xc;
  }
  return e;
}

// The value of lane (lane ^ H), H a power of two below 64, with no trip
// through the LDS crossbar: DPP row permutations for H <= 8 (H = 4 and 8 as
// the half-row mirror i -> i ^ 7 followed by i -> i ^ 3 or the row mirror
// i -> i ^ 15) and the row-swap instructions for H = 16 and 32.
template <int H>
__device__ __forceinline__ int xor_lane_u32(int v, int lane) {
  if constexpr (H == 1) {
    return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);  // quad_perm [1,0,3,2]
  } else if constexpr (H == 2) {
    return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);  // quad_perm [2,3,0,1]
  } else if constexpr (H == 4) {
    const int t = __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true);  // row_half_mirror
    return __builtin_amdgcn_mov_dpp(t, 0x1B, 0xF, 0xF, true);          // quad_perm [3,2,1,0]
  } else if constexpr (H == 8) {
    const int t = __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true);  // row_half_mirror
    return __builtin_amdgcn_mov_dpp(t, 0x140, 0xF, 0xF, true);         // row_mirror
  } else if constexpr (H == 16) {
    // both operands a copy of v: the first ends with rows (0, 0, 2, 2), the
    // second with rows (1, 1, 3, 3)
    const auto r = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
    return (int)((lane & 16) ? r[0] : r[1]);
  } else {
    static_assert(H == 32, "xor distance");
    const auto r = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
    return (int)((lane & 32) ? r[0] : r[1]);
  }
}

template <int H>
__device__ __forceinline__ double xor_lane(double v, int lane) {
  const int64_t b = __builtin_bit_cast(int64_t, v);
  const int lo = xor_lane_u32<H>((int)(uint32_t)b, lane), hi = xor_lane_u32<H>((int)(b >> 32), lane);
  return __builtin_bit_cast(double, (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

__device__ __forceinline__ double join_words(unsigned lo, unsigned hi) {
  return __builtin_bit_cast(double, (uint64_t)lo | ((uint64_t)hi << 32));
}

// Half-lane moves at distance H = 4 or 8, where a DPP row shift can write
// only the lanes of one side (its bank mask selects groups of four lanes):
// from_above gives the lanes with bit H clear the value src of lane L + H and
// leaves old in the others; from_below gives the lanes with bit H set src of
// lane L - H and leaves old in the rest. Two of them make a trade between
// lane pairs with no select.
template <int H, bool ABOVE>
__device__ __forceinline__ double half_move(double old, double src) {
  static_assert(H == 4 || H == 8, "bank-masked move distance");
  constexpr int kCtrl = ABOVE ? 0x100 + H : 0x110 + H;  // row_shl:H or row_shr:H
  constexpr int kBanks = ABOVE ? (H == 8 ? 0x3 : 0x5) : (H == 8 ? 0xC : 0xA);
  const uint64_t uo = __builtin_bit_cast(uint64_t, old), us = __builtin_bit_cast(uint64_t, src);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)uo, (int)(unsigned)us,
                                                            kCtrl, 0xF, kBanks, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)(uo >> 32),
                                                            (int)(unsigned)(us >> 32), kCtrl, 0xF,
                                                            kBanks, false);
  return join_words(lo, hi);
}
template <int H>
__device__ __forceinline__ double from_above(double old, double src) { return half_move<H, true>(old, src); }
template <int H>
__device__ __forceinline__ double from_below(double old, double src) { return half_move<H, false>(old, src); }

// v of lane L - N within the row of 16 lanes (lanes with L mod 16 < N get 0).
template <int N>
__device__ __forceinline__ double row_shr(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)u, 0x110 + N, 0xF, 0xF, true);
  const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(u >> 32), 0x110 + N, 0xF, 0xF, true);
  return join_words(lo, hi);
}

// Transposed sums: a stage over lane pairs (L, L ^ H) takes two partial sums
// per lane and leaves one, lanes with bit H clear keeping the first value's
// pair sum and the others the second's. Each value's total is formed over
// the same pairs, level by level, as in a butterfly, so it is bitwise the
// same; a stage costs one exchange per pair of values instead of one per
// value. At H = 32 and 16 the row swaps do it without selects: after
// swapping the upper rows of a with the lower rows of b, a + b holds a's pair
// sum in the lower rows and b's in the upper ones; at H = 8 and 4 the
// half-lane moves do the same.
template <int H>
__device__ __forceinline__ double pair_sum(double a, double b, int lane) {
  if constexpr (H == 32 || H == 16) {
    const uint64_t ua = __builtin_bit_cast(uint64_t, a), ub = __builtin_bit_cast(uint64_t, b);
    const unsigned alo = (unsigned)ua, ahi = (unsigned)(ua >> 32), blo = (unsigned)ub, bhi = (unsigned)(ub >> 32);
    if constexpr (H == 32) {
      const auto lo = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
      const auto hi = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
      return join_words(lo[0], hi[0]) + join_words(lo[1], hi[1]);
    } else {
      const auto lo = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
      const auto hi = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
      return join_words(lo[0], hi[0]) + join_words(lo[1], hi[1]);
    }
  } else if constexpr (H == 8 || H == 4) {
    // lanes with bit H clear: (own a, a of L + H); set: (b of L - H, own b)
    return from_below<H>(a, b) + from_above<H>(b, a);
  } else {
    const bool up = lane & H;
    const double send = up ? a : b, keep = up ? b : a;
    return keep + xor_lane<H>(send, lane);
  }
}

// Wave totals of eight values: lane L with L mod 8 = 7 ends with the total
// of v[L >> 3]. The last three levels add the value of lane L - 4, L - 2 and
// L - 1, which pairs the same partial sums as a butterfly would.
__device__ __forceinline__ double transposed_sum8(const double v[8], int lane) {
  double t5[4], t4[2];
#pragma unroll
  for (int i = 0; i < 4; ++i) t5[i] = pair_sum<32>(v[i], v[i + 4], lane);
#pragma unroll
  for (int i = 0; i < 2; ++i) t4[i] = pair_sum<16>(t5[i], t5[i + 2], lane);
  double t = pair_sum<8>(t4[0], t4[1], lane);
  t += row_shr<4>(t);
  t += row_shr<2>(t);
  t += row_shr<1>(t);
  return t;
}

// Wave totals of 36 values. Value x is given the lane slot kSlot36[x]; the
// slots are R5 and R5 + 32 with R5 = R4 and R4 + 16, R4 = {0,1,2,4,5,8,9,10,12},
// so each stage halves the number of live partial sums (36, 18, 9, 5, 3, 2,
// 1) and pairs absent from a stage are zero. Lane L ends with the total of
// the value whose slot is L.
__constant__ const int kSlot36[36] = {0,  1,  2,  4,  5,  8,  9,  10, 12, 16, 17, 18,
                                      20, 21, 24, 25, 26, 28, 32, 33, 34, 36, 37, 40,
                                      41, 42, 44, 48, 49, 50, 52, 53, 56, 57, 58, 60};

__device__ __forceinline__ double transposed_sum36(const double v[36], int lane) {
  double t5[18], t4[9], t3[5], t2[3], t1[2];
#pragma unroll
  for (int i = 0; i < 18; ++i) t5[i] = pair_sum<32>(v[i], v[i + 18], lane);
#pragma unroll
  for (int i = 0; i < 9; ++i) t4[i] = pair_sum<16>(t5[i], t5[i + 9], lane);
#pragma unroll
  for (int i = 0; i < 5; ++i) t3[i] = pair_sum<8>(t4[i], i + 5 < 9 ? t4[i + 5] : 0.0, lane);
#pragma unroll
  for (int i = 0; i < 3; ++i) t2[i] = pair_sum<4>(t3[i], i + 3 < 5 ? t3[i + 3] : 0.0, lane);
#pragma unroll
  for (int i = 0; i < 2; ++i) t1[i] = pair_sum<2>(t2[i], i + 2 < 3 ? t2[i + 2] : 0.0, lane);
  return pair_sum<1>(t1[0], t1[1], lane);
}

// The 64-point transforms keep two complex values per lane, A and B; at the
// start A is channel A's and B channel E's sample of the lane. A stage of
// span H first trades values between lanes L and L ^ H so that a lane with
// bit H clear holds (its A, the partner's A) and one with bit H set (the
// partner's B, its B): a butterfly pair of one sub-transform. The lane then
// forms both outputs of that butterfly, so no lane computes a result it
// throws away. At H = 32 and 16 the row swaps make the trade, one
// instruction per register; at H = 8 and 4 two half-lane moves; at H = 2
// and 1 one DPP exchange and selects. After the
// six forward stages lane 32c + i holds channel c's window bins bitrev5(i)
// and 32 + bitrev5(i); one more row swap at span 32 leaves lane 32s + i with
// both channels of bin 32s + bitrev5(i). Each trade is its own inverse, so
// the inverse transform runs the stages backwards. The twiddles come from
// the table, one complex number per lane and stage.
struct Pair {
  double ar, ai, br, bi;  // A = ar + i ai, B = br + i bi
};

// the trade at span 32 or 16 of one register pair
template <int H>
__device__ __forceinline__ void row_swap(double& a, double& b) {
  const uint64_t ua = __builtin_bit_cast(uint64_t, a), ub = __builtin_bit_cast(uint64_t, b);
  const unsigned alo = (unsigned)ua, ahi = (unsigned)(ua >> 32), blo = (unsigned)ub, bhi = (unsigned)(ub >> 32);
  if constexpr (H == 32) {
    const auto lo = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
    a = join_words(lo[0], hi[0]);
    b = join_words(lo[1], hi[1]);
  } else {
    static_assert(H == 16, "row swap span");
    const auto lo = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
    a = join_words(lo[0], hi[0]);
    b = join_words(lo[1], hi[1]);
  }
}

template <int H>
__device__ __forceinline__ void trade(Pair& p, int lane) {
  if constexpr (H >= 16) {
    row_swap<H>(p.ar, p.br);
    row_swap<H>(p.ai, p.bi);
  } else if constexpr (H >= 4) {
    // lanes with bit H clear keep A and take the B of lane L + H; the others
    // keep B and take the A of lane L - H
    const double nbr = from_above<H>(p.br, p.ar), nbi = from_above<H>(p.bi, p.ai);
    p.ar = from_below<H>(p.ar, p.br);
    p.ai = from_below<H>(p.ai, p.bi);
    p.br = nbr;
    p.bi = nbi;
  } else {
    const bool set = lane & H;
    const double rr = xor_lane<H>(set ? p.ar : p.br, lane), ri = xor_lane<H>(set ? p.ai : p.bi, lane);
    p.ar = set ? rr : p.ar;
    p.ai = set ? ri : p.ai;
    p.br = set ? p.br : rr;
    p.bi = set ? p.bi : ri;
  }
}

// Forward stage S (span 32 >> S), decimation in frequency: (a, b) ->
// (a + b, (a - b) w). Down to span 4 the pair arrives in order (x the
// element of the lower index). At spans 2 and 1 the lane keeps x (its A, or
// its B with bit H set) and receives y, so the pair is (x, y) or (y, x); the
// sign of the difference in the second case is folded into the lane's
// twiddle, which at span 1 is that sign alone (the root is 1), applied by
// flipping the sign bit.
template <int S>
__device__ __forceinline__ void fwd_stage(Pair& p, const double* tw, int lane) {
  constexpr int H = 32 >> S;
  double xr, xi, yr, yi;
  if constexpr (H >= 16) {
    row_swap<H>(p.ar, p.br);
    row_swap<H>(p.ai, p.bi);
    xr = p.ar;
    xi = p.ai;
    yr = p.br;
    yi = p.bi;
  } else if constexpr (H >= 4) {
    // lanes with bit H clear: (own A, A of lane L + H); set: (B of L - H, own B)
    xr = from_below<H>(p.ar, p.br);
    xi = from_below<H>(p.ai, p.bi);
    yr = from_above<H>(p.br, p.ar);
    yi = from_above<H>(p.bi, p.ai);
  } else {
    const bool set = lane & H;
    xr = set ? p.br : p.ar;
    xi = set ? p.bi : p.ai;
    yr = xor_lane<H>(set ? p.ar : p.br, lane);
    yi = xor_lane<H>(set ? p.ai : p.bi, lane);
  }
  const double dr = xr - yr, di = xi - yi;
  p.ar = xr + yr;
  p.ai = xi + yi;
  if constexpr (H == 1) {
    const uint64_t sgn = (uint64_t)(lane & 1) << 63;
    p.br = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, dr) ^ sgn);
    p.bi = __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, di) ^ sgn);
  } else {
    const double wr = tw[S * 128 + 2 * lane], wi = tw[S * 128 + 2 * lane + 1];
    p.br = dr * wr - di * wi;
    p.bi = dr * wi + di * wr;
  }
}

// Inverse stage S: (s, d) -> (s + conj(w) d, s - conj(w) d), then the trade
// (at span 1 the root is 1).
template <int S>
__device__ __forceinline__ void inv_stage(Pair& p, const double* tw, int lane) {
  constexpr int H = 32 >> S;
  double tr = p.br, ti = p.bi;
  if constexpr (H > 1) {
    const double wr = tw[S * 128 + 2 * lane], wi = tw[S * 128 + 2 * lane + 1];
    tr = p.br * wr - p.bi * wi;
    ti = p.br * wi + p.bi * wr;
  }
  const double sr = p.ar, si = p.ai;
  p.ar = sr + tr;
  p.ai = si + ti;
  p.br = sr - tr;
  p.bi = si - ti;
  trade<H>(p, lane);
}

__device__ __forceinline__ int bitrev5(int x) { return (int)(__builtin_bitreverse32((unsigned)x) >> 27); }

// The lane holding window bin m (0 <= m < 64) after the forward transform,
// and the bin a lane holds: the map is its own inverse.
__device__ __forceinline__ int bin_lane(int m) { return (m & 32) | bitrev5(m & 31); }

// Forward DFT of both channels over the wave: lane j holds sample j of each
// channel in (re[c], im[c]); lane bin_lane(m) ends with bin m of each.
// tw: the forward twiddles ([stage][lane][re, im]).
__device__ __forceinline__ void fft_fwd(double re[2], double im[2], const double* tw, int lane) {
  Pair p{re[0], im[0], re[1], im[1]};
  fwd_stage<0>(p, tw, lane);
  fwd_stage<1>(p, tw, lane);
  fwd_stage<2>(p, tw, lane);
  fwd_stage<3>(p, tw, lane);
  fwd_stage<4>(p, tw, lane);
  fwd_stage<5>(p, tw, lane);
  row_swap<32>(p.ar, p.br);
  row_swap<32>(p.ai, p.bi);
  re[0] = p.ar;
  im[0] = p.ai;
  re[1] = p.br;
  im[1] = p.bi;
}

// Inverse (unnormalised, e^{+2 pi i m j / 64}) DFT of both channels: lane L
// holds bin bin_lane(L) of each channel, or with SPLIT lane 32c + i holds
// channel c's bins bitrev5(i) in (re[0], im[0]) and 32 + bitrev5(i) in
// (re[1], im[1]) (the layout of the forward stages before their last row
// swap); lane j ends with sample j. tw: the inverse twiddles.
template <bool SPLIT = false>
__device__ __forceinline__ void fft_inv(double re[2], double im[2], const double* tw, int lane) {
  Pair p{re[0], im[0], re[1], im[1]};
  if constexpr (!SPLIT) {
    row_swap<32>(p.ar, p.br);
    row_swap<32>(p.ai, p.bi);
  }
  inv_stage<5>(p, tw, lane);
  inv_stage<4>(p, tw, lane);
  inv_stage<3>(p, tw, lane);
  inv_stage<2>(p, tw, lane);
  inv_stage<1>(p, tw, lane);
  inv_stage<0>(p, tw, lane);
  re[0] = p.ar;
  im[0] = p.ai;
  re[1] = p.br;
  im[1] = p.bi;
}

// Butterfly sum: every lane ends with the same (bitwise) total, since each
// stage adds the same two values in both lanes of a pair.
__device__ __forceinline__ double wave_sum(double v, int lane) {
  v += xor_lane<32>(v, lane);
  v += xor_lane<16>(v, lane);
  v += xor_lane<8>(v, lane);
  v += xor_lane<4>(v, lane);
  v += xor_lane<2>(v, lane);
  v += xor_lane<1>(v, lane);
  return v;
}

// The source's window spectrum (times T_obs / 64) across the wave: lane L
// holds bin q - 32 + bin_lane(L).
__device__ __forceinline__ void window_spectrum(const Src& s, const LaneGeom& g, const double* tw,
                                                const double* trig, double scale, int lane,
                                                double re[2], double im[2]) {
  // (-1)^j centres the window on q
  const Env e = envelope(s, g, trig, lane, (lane & 1) ? -0.5 * scale : 0.5 * scale);
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    re[c] = e.zr[c];
    im[c] = e.zi[c];
  }
  fft_fwd(re, im, tw, lane);
}

// Value of the window spectrum at band bin b (0 outside the window), read
// from the lane that holds it. All lanes must call this together.
__device__ __forceinline__ void window_at(const double re[2], const double im[2], int64_t b_abs,
                                          int64_t q, double out_re[2], double out_im[2]) {
  const int64_t m = b_abs - (q - kNs / 2);
  const bool in = m >= 0 && m < kNs;
  const int src = bin_lane((int)(m & (kNs - 1)));
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    const double vr = __shfl(re[c], src), vi = __shfl(im[c], src);
    out_re[c] = in ? vr : 0.0;
    out_im[c] = in ? vi : 0.0;
  }
}

// One data set of the likelihood: the handle's own, or under a bridge
// (eq. reuse_bridge between two records) also its partner's.
struct FdSide {
  const double* data;
  const double* tw;  // twiddles in LDS, forward then inverse
  const double* trig;  // phase table in LDS
  LaneGeom g;        // this lane's grid constants in LDS
  int64_t k0, B;
  double T_obs, scale, cnorm;
  int qslot;         // word of the source rows with this record's carrier bin
};

__device__ __forceinline__ FdSide own_side(const PopArgs& a, const FdTables& t, int lane) {
  return {a.fd_data, t.tw, t.trig, LaneGeom{t.geo[0] + lane}, a.fd_k0, a.fd_B, a.fd_T_obs,
          a.fd_scale, a.inv_sigma2, kQOwn};
}
__device__ __forceinline__ FdSide partner_side(const PopArgs& a, const FdTables& t, int lane) {
  return {a.fd2_data, t.tw, t.trig, LaneGeom{t.geo[1] + lane}, a.fd2_k0, a.fd2_B, a.fd2_T_obs,
          a.fd2_T_obs / 64.0, a.fd2_cnorm, kQPartner};
}

template <int NR>
struct Resid {
  double re[2][NR], im[2][NR];
};

template <int NR>
__device__ __forceinline__ void load_resid(const FdSide& sd, int lane, Resid<NR>& R) {
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const int b = lane + kNs * r;
      R.re[c][r] = sd.data[(c * kFdBandStride + b) * 2];
      R.im[c][r] = sd.data[(c * kFdBandStride + b) * 2 + 1];
    }
}

// Band index of the source's window bin 0 (wave-uniform), clamped to
// [-2 kNs, B], which leaves every test of a band bin against the window and
// the band as it was and keeps the index arithmetic in 32 bits.
__device__ __forceinline__ int window_start(int64_t q, const FdSide& sd) {
  const int64_t lo = q - kNs / 2 - sd.k0;
  return (int)(lo < -2 * kNs ? -2 * kNs : (lo > sd.B ? sd.B : lo));
}

// R -= sign h over the band (sign = +-1). Each band bin takes the window
// value from the lane holding it, weighted by sign where the bin lies in both
// the window and the band and by 0 elsewhere: one FMA per value, which
// rounds as R - sign v.
template <int NR>
__device__ __forceinline__ void subtract_source(const FdSide& sd, const Src& s, const LaneGeom& g,
                                                int lane, Resid<NR>& R, double sign) {
  double re[2], im[2];
  window_spectrum(s, g, sd.tw, sd.trig, sd.scale, lane, re, im);
  const int lo = window_start(s.q, sd);  // band index of window bin 0
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int b = lane + kNs * r, m = b - lo;
    const double f = ((unsigned)m < (unsigned)kNs && b < (int)sd.B) ? -sign : 0.0;
    const int from = bin_lane(m & (kNs - 1));
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      R.re[c][r] = fma(f, __shfl(re[c], from), R.re[c][r]);
      R.im[c][r] = fma(f, __shfl(im[c], from), R.im[c][r]);
    }
  }
}

// Re<R, h> and |h|^2 over the band for one source (both channels).
template <int NR>
__device__ __forceinline__ void overlap(const FdSide& sd, const Src& s, const LaneGeom& g, int lane,
                                        const Resid<NR>& R, double* rh, double* hh) {
  double re[2], im[2];
  window_spectrum(s, g, sd.tw, sd.trig, sd.scale, lane, re, im);
  double x = 0.0, y = 0.0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int64_t b = lane + kNs * r;
    double vr[2], vi[2];
    window_at(re, im, sd.k0 + b, s.q, vr, vi);
    if (b < sd.B)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        x = fma(R.re[c][r], vr[c], fma(R.im[c][r], vi[c], x));
        y = fma(vr[c], vr[c], fma(vi[c], vi[c], y));
      }
  }
  *rh = wave_sum(x, lane);
  *hh = wave_sum(y, lane);
}

// Derivatives of the envelope z_c = a_c e^{i ph} / 2 (channel c) with respect
// to the eight parameters at this lane's sample: dz_p = (da_p e^{i ph}) / 2 +
// i dphi_p z = (e^{i ph} / 2) g_p with g_p = da_p + i dphi_p a_c, a the complex
// amplitude and ph the heterodyned phase. This returns g_p; the phase factor
// has modulus one and drops out of the metric entries Re(conj(dz_a) dz_b).
__device__ __forceinline__ void amp_phase_derivs(const Src& s, const LaneGeom& g, const Env& e, int c,
                                                 double gr[8], double gi[8]) {
  const double Ap = s.Ap, Ax = s.Ax;
  const double fi = s.f0 + s.fd * e.tau;
  const double dphi[8] = {kTwoPi * e.tau, 0.5 * kTwoPi * e.tau * e.tau, 0.0,
                          kTwoPi * fi * (-s.sb * e.doppler),
                          kTwoPi * fi * (s.cb * kAuLight * (g.sa() * s.cl - g.ca() * s.sl)), 0.0, 0.0,
                          1.0};
  const V3 ul = {s.sb * s.v.x, s.sb * s.v.y, 0.0};
  const V3 vl = {-s.cl, -s.sl, 0.0};
  double D[6];
#pragma unroll
  for (int x = 0; x < 6; ++x) D[x] = g.d(c, x);
  const V3 Du = mul_sym(D, s.u), Dv = mul_sym(D, s.v);
  const double dPb = 2.0 * dot3(s.n, Du), dXb = 2.0 * dot3(s.n, Dv);
  const double dPl = 2.0 * (dot3(ul, Du) - dot3(vl, Dv));
  const double dXl = 2.0 * (dot3(ul, Dv) + dot3(vl, Du));
  double da_r[8], da_i[8];
  da_r[0] = da_i[0] = da_r[1] = da_i[1] = da_r[7] = da_i[7] = 0.0;
  da_r[2] = kLn10 * e.ar[c];
  da_i[2] = kLn10 * e.ai[c];
  da_r[3] = (s.c2p * dPb + s.s2p * dXb) * Ap;
  da_i[3] = -(-s.s2p * dPb + s.c2p * dXb) * Ax;
  da_r[4] = (s.c2p * dPl + s.s2p * dXl) * Ap;
  da_i[4] = -(-s.s2p * dPl + s.c2p * dXl) * Ax;
  da_r[5] = 2.0 * e.Fx[c] * Ap;
  da_i[5] = 2.0 * e.Fp[c] * Ax;
  da_r[6] = e.Fp[c] * (-2.0 * s.A * s.ci * s.si);
  da_i[6] = -e.Fx[c] * (2.0 * s.A * s.si);
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    gr[p] = da_r[p] - dphi[p] * e.ai[c];
    gi[p] = da_i[p] + dphi[p] * e.ar[c];
  }
}



// This lane's share of the gradient of one source, sum_c Re(conj(w_c) dz_c,p)
// for the eight parameters, without forming dz_c,p = (da_c,p / 2) e^{i ph} +
// i dphi_p z_c (amp_phase_derivs): per channel
//   Re(conj(w) dz_p) = Re(da_p) ur + Im(da_p) ui + dphi_p (Im w Re z - Re w Im z),
// ur = (Re w cos ph + Im w sin ph) / 2, ui = (Im w cos ph - Re w sin ph) / 2.
// The caller passes w up to a sign, which half (+-1/2) restores. With the
// amplitudes a_c = Ap Fp_c - i Ax Fx_c, every amplitude and phase term is a
// combination of four channel sums S1 = sum Fp ur, S2 = sum Fp ui,
// S3 = sum Fx ur, S4 = sum Fx ui: the phase factor shared by the dphi terms
// is G = sum (Im w Re z - Re w Im z) = sum (Re a ui - Im a ur) = Ap S2 + Ax S3,
// the amplitude's own term sum (Re a ur + Im a ui) = Ap S1 - Ax S4, the
// polarisation angle's sum (Fx Ap ur + Fp Ax ui) = Ap S3 + Ax S2 and the
// inclination's sum (cos(i) Fp ur + Fx ui) = cos(i) S1 + S4. The two sky
// derivatives are linear in (dP, dX), which are bilinear in the detector
// tensor D_c, so with the weights alpha_c = c2p Ap ur + s2p Ax ui,
// beta_c = s2p Ap ur - c2p Ax ui that the polarisation angle and the
// amplitudes give dP and dX they contract to 2 n.D y1 (latitude) and
// 2 (ul.D y1 + vl.D y2) (longitude), y1 = alpha u + beta v, y2 = beta u - alpha v,
// ul = sin(b) v and vl = -(cos(b) n + sin(b) u) the derivatives of u and v
// with respect to the longitude. With D symmetric these reduce to the forms
// n.D u and n.D v and the patterns P and X:
//   latitude:  2 sum (alpha n.D u + beta n.D v)
//   longitude: 2 sum (alpha (sin(b) X + cos(b) n.D v) - beta (sin(b) P + cos(b) n.D u)),
// where sum (alpha X - beta P) is the polarisation angle's sum above (P and X
// rotated by 2 psi are Fp and Fx), and the rest is linear in the four sums
// U1 = sum ur n.D u, U2 = sum ui n.D u, V1 = sum ur n.D v, V2 = sum ui n.D v.
__device__ __forceinline__ void grad_terms(const Src& s, const LaneGeom& g, const Env& e,
                                           const double wr[2], const double wi[2], double half,
                                           double gp[8]) {
  const double Ap = s.Ap, Ax = s.Ax;
  const double hc = half * e.cph, hs = half * e.sph;
  double ur[2], ui[2];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    ur[c] = wr[c] * hc + wi[c] * hs;
    ui[c] = wi[c] * hc - wr[c] * hs;
  }
  const double S1 = e.Fp[0] * ur[0] + e.Fp[1] * ur[1], S2 = e.Fp[0] * ui[0] + e.Fp[1] * ui[1];
  const double S3 = e.Fx[0] * ur[0] + e.Fx[1] * ur[1], S4 = e.Fx[0] * ui[0] + e.Fx[1] * ui[1];
  const double G = Ap * S2 + Ax * S3;
  const double t5 = Ap * S3 + Ax * S2;
  // the phase derivatives times G: 2 pi (tau, tau^2 / 2) and 2 pi f_i times
  // the Doppler delay's derivatives, f_i = f0 + fdot tau
  const double G2 = kTwoPi * G;
  const double Gf = (s.f0 + s.fd * e.tau) * G2;
  gp[0] = e.tau * G2;
  gp[1] = (0.5 * e.tau) * gp[0];
  gp[2] = kLn10 * (Ap * S1 - Ax * S4);
  gp[5] = 2.0 * t5;
  gp[6] = -2.0 * s.A * s.si * (s.ci * S1 + S4);
  gp[7] = G;
  // the sky derivatives, one channel at a time (the barrier keeps the two
  // channels' temporaries from being live together)
  static constexpr int kVx[5] = {0, 1, 3, 4, 5};  // the tensor entries of the n.D v weights
  double U1 = 0.0, U2 = 0.0, V1 = 0.0, V2 = 0.0;
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    double nDu = 0.0, nDv = 0.0;
#pragma unroll
    for (int x = 0; x < 6; ++x) nDu = fma(s.wnu[x], g.d(c, x), nDu);
#pragma unroll
    for (int x = 0; x < 5; ++x) nDv = fma(s.wnv[x], g.d(c, kVx[x]), nDv);
    U1 = fma(ur[c], nDu, U1);
    U2 = fma(ui[c], nDu, U2);
    V1 = fma(ur[c], nDv, V1);
    V2 = fma(ui[c], nDv, V2);
    __builtin_amdgcn_sched_barrier(0);
  }
  const double kPa = s.c2p * Ap, kXa = s.s2p * Ax, kPb = s.s2p * Ap, kXb = s.c2p * Ax;
  const double lat = (kPa * U1 + kXa * U2) + (kPb * V1 - kXb * V2);
  const double lon = (kPa * V1 + kXa * V2) - (kPb * U1 - kXb * U2);
  gp[3] = (-s.sb * e.doppler) * Gf + 2.0 * lat;
  gp[4] = (s.cb * kAuLight) * (g.sa() * s.cl - g.ca() * s.sl) * Gf + 2.0 * (s.sb * t5 + s.cb * lon);
}

struct FdItem {
  int64_t i, m0;
  int K;
};

// Listed work items of a launch: the ordering pass's count in sorted mode
// (valid particles with K > 0, or all valid ones for birth/death), else N.
__device__ __forceinline__ int64_t fd_count(const PopArgs& a) {
  return a.order ? (int64_t)*a.n_active : a.N;
}

// Work item at rank < fd_count(a); false for a particle whose offsets are
// invalid or exceed k_max.
__device__ __forceinline__ bool fd_item_at(const PopArgs& a, int64_t rank, FdItem& it) {
  it.i = a.order ? (int64_t)a.order[rank] : rank;
  const int64_t o0 = a.offsets[it.i], o1 = a.offsets[it.i + 1];
  if (!(o0 >= 0 && o1 >= o0 && o1 <= a.M && o1 - o0 <= a.k_max)) return false;
  it.m0 = o0;
  it.K = (int)(o1 - o0);
  return true;
}

__device__ __forceinline__ bool fd_active_at(const PopArgs& a, int64_t rank, FdItem& it) {
  return fd_item_at(a, rank, it) && !(a.active && !a.active[it.i]);
}

// A wave's residual copy in LDS (the gradient pass): four rows (re, im of
// A, re, im of E) of kNs NR band bins and one zero word that gathers from
// outside the band read.
template <int NR>
constexpr int resid_row() { return kNs * NR + 2; }
template <int NR>
constexpr int resid_words() { return 4 * resid_row<NR>(); }

// One particle on one data set, weighted by w; the first side writes the
// outputs, a second one adds to them, and the leapfrog kick (p_half set)
// follows the last side's gradient. rl: the wave's residual copy in LDS
// (MODE 1).
template <int MODE, int NR>
__device__ __forceinline__ void fd_particle(const PopArgs& a, const FdSide& sd, const FdItem& it,
                                            int lane, double w, bool first, bool last,
                                            const double* __restrict__ src, double* rl,
                                            int k_first = 0, int k_step = 1) {
  const int64_t i = it.i;
  const double wc = w * sd.cnorm;  // weight * 4 / (T_obs S)
  const LaneGeom g = sd.g;
  Resid<NR> R;
  load_resid<NR>(sd, lane, R);
  for (int k = 0; k < it.K; ++k) {
    const int row = __builtin_amdgcn_readfirstlane((int)(it.m0 + k));
    // the lane index, opaque in each pass, so that the lane's grid constants
    // are read from LDS for every source instead of held in 30 registers
    // through the loop
    int ln = lane;
    asm volatile("" : "+v"(ln));
    const LaneGeom gk{g.g + (ln - lane)};
    subtract_source<NR>(sd, src_load(src + (int64_t)row * kSrcWords, sd.qslot), gk, lane, R, 1.0);
  }
  if constexpr (MODE == 2) {
    if (a.theta_birth && a.dlogl_birth) {
      const Src s = make_src(a.theta_birth + i * 8, sd.T_obs);
      double rh, hh;
      overlap<NR>(sd, s, g, lane, R, &rh, &hh);
      const double v = wc * (rh - 0.5 * hh);
      if (lane == 0) a.dlogl_birth[i] = first ? v : a.dlogl_birth[i] + v;
    }
    if (a.death_idx && a.dlogl_death) {
      const int j = a.death_idx[i];
      if (j >= 0 && j < it.K) {
        const int row = __builtin_amdgcn_readfirstlane((int)(it.m0 + j));
        const Src s = src_load(src + (int64_t)row * kSrcWords, sd.qslot);
        double rh, hh;
        overlap<NR>(sd, s, g, lane, R, &rh, &hh);
        const double v = -(wc * (rh + 0.5 * hh));
        if (lane == 0) a.dlogl_death[i] = first ? v : a.dlogl_death[i] + v;
      } else if (lane == 0 && first) {
        a.dlogl_death[i] = j == -1 ? 0.0 : __builtin_nan("");
        if (j != -1) atomicOr(a.flag, kFlagDeath);
      }
    }
    return;
  }
  double ss = 0.0;
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int r = 0; r < NR; ++r) ss = fma(R.re[c][r], R.re[c][r], fma(R.im[c][r], R.im[c][r], ss));
  ss = wave_sum(ss, lane);
  if (lane == 0 && k_first == 0 && a.logl) {
    const double v = -0.5 * wc * ss;
    a.logl[i] = first ? v : a.logl[i] + v;
  }
  if constexpr (MODE == 1) {
    const double he = a.p_half ? 0.5 * a.eps * (a.dir ? (double)a.dir[i] : 1.0) : 0.0;
    // the window bins this lane gathers, in the split layout of the inverse
    // transform: channel lane >> 5, bins m0 and m0 + 32
    const int wc0 = (lane >> 5) * 2, m0 = bitrev5(lane & 31);
    // The residual goes to the wave's LDS copy ([re, im of A, re, im of E]
    // [band position]); the loop gathers each source's window from there,
    // and its registers are free for the adjoint.
    constexpr int Bp = kNs * NR, rs = resid_row<NR>();
    wave_lds_sync();
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        rl[(2 * c) * rs + lane + kNs * r] = R.re[c][r];
        rl[(2 * c + 1) * rs + lane + kNs * r] = R.im[c][r];
      }
    if (lane < 4) rl[lane * rs + Bp] = 0.0;
    wave_lds_sync();
    for (int k = k_first; k < it.K; k += k_step) {
      const int row = __builtin_amdgcn_readfirstlane((int)(it.m0 + k));
      const Src s = src_load(src + (int64_t)row * kSrcWords, sd.qslot);
      // residual window of the source in the inverse transform's input order
      const int lo = window_start(s.q, sd);  // band index of window bin 0
      double wr[2], wi[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int bw = lo + m0 + 32 * h;  // band index this lane gathers
        const int bi = (unsigned)bw < (unsigned)sd.B ? bw : Bp;  // the zero word outside the band
        wr[h] = rl[wc0 * rs + bi];
        wi[h] = rl[(wc0 + 1) * rs + bi];
      }
      fft_inv<true>(wr, wi, sd.tw + 6 * 128, lane);
      // w_j = sum_m R[q + m] e^{2 pi i m j / 64} = (-1)^j times the inverse DFT
      // of the window (indexed from q - 32); the sign goes with the factor 1/2
      // Re(conj(w) dz) per parameter
      const Env e = envelope(s, g, sd.trig, lane);
      double gp[8];
      grad_terms(s, g, e, wr, wi, (lane & 1) ? -0.5 : 0.5, gp);
      // lane 8p + 7 ends with parameter p's total
      double gv = transposed_sum8(gp, lane) * (wc * sd.scale);
      if ((lane & 7) == 7) {
        const int64_t x = (it.m0 + k) * 8 + (lane >> 3);
        if (!first && a.grad) gv += a.grad[x];
        if (a.grad) a.grad[x] = gv;
        if (last && a.p_half) a.p_out[x] = fma(he, gv, a.p_half[x]);
      }
    }
  }
}

// MODE 0: logL; 1: logL and gradient (with the leapfrog kick when p_half
// is set); 2: birth / death changes. Under a bridge (fd_bridge) the target
// is (1 - beta) logL_partner + beta logL_own, so each particle runs on both
// data sets.
template <int MODE, int NR>
__device__ __forceinline__ void fd_run(const PopArgs& a, const FdTables& tabs, const FdItem& it,
                                       int lane, const double* __restrict__ src, double* rl,
                                       int k_first, int k_step) {
  const double b = a.beta ? a.beta[it.i] : 1.0;
  if (a.fd_bridge) {
    fd_particle<MODE, NR>(a, partner_side(a, tabs, lane), it, lane, 1.0 - b, true, false, src,
                          rl, k_first, k_step);
    fd_particle<MODE, NR>(a, own_side(a, tabs, lane), it, lane, b, false, true, src, rl, k_first,
                          k_step);
  } else {
    fd_particle<MODE, NR>(a, own_side(a, tabs, lane), it, lane, b, true, true, src, rl, k_first,
                          k_step);
  }
}

// STRIDED (the leapfrog gradient of late NUTS doublings on the 128-bin band):
// a grid smaller than the population whose workgroups step through the
// listed particles. Otherwise one pass, one particle per wave, as in full
// passes, where the hardware hands the workgroups out in the K-sorted order
// (measured faster than the loop, whose form also keeps more registers live
// in the other variants).
template <int MODE, int NR, bool STRIDED>
__global__ __launch_bounds__(256) void fd_kernel(PopArgs a, const double* __restrict__ src) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
  const int64_t n = fd_count(a);
  FdTables tabs;
  FdItem it;
  if constexpr (!STRIDED) {
    const int64_t rank = (int64_t)blockIdx.x * waves + wave;
    const bool work = rank < n && fd_active_at(a, rank, it);
    // a workgroup without an active particle leaves at once
    if (!__syncthreads_or(work)) return;
    double* rl = stage_tables(tabs, a.fd_table, a.fd_bridge ? a.fd2_table : nullptr) +
                 wave * resid_words<NR>();
    if (work) fd_run<MODE, NR>(a, tabs, it, lane, src, rl, 0, 1);
  } else {
    // Few listed particles (late NUTS leaves): the waves of a workgroup
    // share one particle. Each builds the whole residual and takes every
    // waves-th source of the gradient pass, so the results are those of one
    // wave per particle while the latency of a particle drops to about half
    // and four times as many SIMDs hold work.
    const bool split = a.order && a.fd_split > 0 && n <= a.fd_split;
    const int64_t per = split ? 1 : waves;  // particles of one workgroup pass
    const int64_t stride = (int64_t)gridDim.x * per;
    const int k_first = split ? wave : 0, k_step = split ? waves : 1;
    // this wave's first active item, found before the tables are staged (a
    // workgroup without one leaves at once); the next is looked for after
    // each particle
    int64_t r0 = (int64_t)blockIdx.x * per;
    bool have = false;
    for (; r0 < n && !have; r0 += stride) {
      const int64_t rank = split ? r0 : r0 + wave;
      have = rank < n && fd_active_at(a, rank, it);
    }
    if (!__syncthreads_or(have)) return;
    double* rl = stage_tables(tabs, a.fd_table, a.fd_bridge ? a.fd2_table : nullptr) +
                 wave * resid_words<NR>();
    while (have) {
      // the lane index, opaque to the compiler in each pass: nothing derived
      // from it (table addresses, lane geometry) stays live from one
      // particle to the next, which would cost a wave per SIMD
      int ln = lane;
      asm volatile("" : "+v"(ln));
      fd_run<MODE, NR>(a, tabs, it, ln, src, rl, k_first, k_step);
      have = false;
      for (; r0 < n && !have; r0 += stride) {
        const int64_t rank = split ? r0 : r0 + wave;
        have = rank < n && fd_active_at(a, rank, it);
      }
    }
  }
}

// Per-source Gauss-Newton metric: block k of particle i is
//   beta (4 / (T_obs S)) Re sum_c sum_m conj(dh_c / dtheta_a) dh_c / dtheta_b
// over the source's 64-bin window, which by Parseval's identity for the
// 64-point DFT equals beta (4 / (T_obs S)) (T_obs / 64)^2 64 Re sum_c sum_j
// conj(dz_c,a(t_j)) dz_c,b(t_j) = (1/4) Re sum_c sum_j conj(g_c,a) g_c,b (the
// phase drops out, see amp_phase_derivs); blocks between sources are zero.
// One wave per particle; 36 sums per source.
// blocks: F is [M][8][8], block k of particle i at F + (o0 + k) 64 (nothing
// between blocks is written); otherwise the dense n x n block at F + f_off[i].
// Held to 168 VGPRs (it needs 171 unconstrained; the excess goes to SGPR
// spills into VGPR lanes, no scratch), which gives three waves per SIMD.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 3))) void fd_metric_kernel(PopArgs a, const double* __restrict__ src,
                                                        const int64_t* f_off, int64_t f_size, double* F,
                                                        int blocks) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  FdTables tabs;
  stage_tables(tabs, a.fd_table, a.fd_bridge ? a.fd2_table : nullptr);
  if (i >= a.N) return;
  const int64_t o0 = a.offsets[i], o1 = a.offsets[i + 1];
  if (!(o0 >= 0 && o1 >= o0 && o1 <= a.M && o1 - o0 <= a.k_max)) {
    if (lane == 0) atomicOr(a.flag, kFlagOffsets);
    return;
  }
  const int K = (int)(o1 - o0), n = 8 * K;
  const int64_t fo = blocks ? o0 * 64 : f_off[i];
  if (!blocks && (f_off[i + 1] - fo != (int64_t)n * n || fo < 0 || fo + (int64_t)n * n > f_size)) {
    if (lane == 0) atomicOr(a.flag, kFlagOffsets);
    return;
  }
  if (n == 0) return;
  double* Fi = F + fo;
  if (a.active && !a.active[i]) {
    // not selected: zero blocks, which the factor's ridge makes definite
    const int64_t cnt = blocks ? (int64_t)K * 64 : (int64_t)n * n;
    for (int64_t x = lane; x < cnt; x += 64) Fi[x] = 0.0;
    return;
  }
  if (!blocks)
    for (int64_t x = lane; x < (int64_t)n * n; x += 64) {
      const int r = (int)(x / n), c = (int)(x % n);
      if ((r >> 3) != (c >> 3)) Fi[x] = 0.0;
    }
  const double b = a.beta ? a.beta[i] : 1.0;
  const int ra = lane >> 3, rb = lane & 7;  // the block entry this lane writes
  const int lo = ra < rb ? ra : rb, hi = ra < rb ? rb : ra;
  // the lane holding entry (lo, hi) of the upper triangle after the sums
  const int holder = kSlot36[lo * 8 - lo * (lo - 1) / 2 + (hi - lo)];
  for (int side = a.fd_bridge ? 0 : 1; side < 2; ++side) {
  const FdSide sd = side == 0 ? partner_side(a, tabs, lane) : own_side(a, tabs, lane);
  const double gs = (side == 0 ? 1.0 - b : b) * sd.cnorm * sd.scale * sd.scale * kNs * 0.25;
  const bool first = side == 0 || !a.fd_bridge;
  const LaneGeom g = sd.g;
  for (int k = 0; k < K; ++k) {
    const int row = __builtin_amdgcn_readfirstlane((int)(o0 + k));
    const Src s = src_load(src + (int64_t)row * kSrcWords, sd.qslot);
    const Env e = envelope_amp(s, g);
    double acc[36];
#pragma unroll
    for (int x = 0; x < 36; ++x) acc[x] = 0.0;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      double gr[8], gi[8];
      amp_phase_derivs(s, g, e, c, gr, gi);
      int x = 0;
#pragma unroll
      for (int p = 0; p < 8; ++p)
#pragma unroll
        for (int q = p; q < 8; ++q, ++x) acc[x] = fma(gr[p], gr[q], fma(gi[p], gi[q], acc[x]));
    }
    const double v = __shfl(transposed_sum36(acc, lane), holder);
    double* dst = blocks ? Fi + 64 * k + 8 * ra + rb : Fi + (int64_t)(8 * k + ra) * n + 8 * k + rb;
    *dst = first ? gs * v : *dst + gs * v;
  }
  }
}

// The band spectrum of K sources (out [2][B][2]): one wave.
__global__ __launch_bounds__(64) void fd_spectrum_kernel(PopArgs a, int64_t K, double* out) {
  const int lane = threadIdx.x;
  FdTables tabs;
  stage_tables(tabs, a.fd_table, nullptr);
  const FdSide sd = own_side(a, tabs, lane);
  Resid<4> R;
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) R.re[c][r] = R.im[c][r] = 0.0;
  for (int64_t k = 0; k < K; ++k) {
    const Src s = make_src(a.theta + k * 8, a.fd_T_obs);
    subtract_source<4>(sd, s, sd.g, lane, R, -1.0);
  }
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t b = lane + kNs * r;
      if (b < a.fd_B) {
        out[(c * a.fd_B + b) * 2] = R.re[c][r];
        out[(c * a.fd_B + b) * 2 + 1] = R.im[c][r];
      }
    }
}

// The source rows of the particles the following launch works on (the same
// work items and activity mask): constants with the carrier bins of both
// records (T2 = 0: no partner, word 33 repeats word 32). A group of
// kSrcGroup lanes per particle, one lane per source, four particles to a
// wave: a whole wave per particle left most lanes idle at K <= 10, and one
// thread per particle measured slower in late NUTS leaves, where few
// particles are active. The cost follows the active set.
constexpr int kSrcGroup = 16;

__global__ __launch_bounds__(256) void fd_src_kernel(PopArgs a, double T2) {
  // The rows of a group's particle are contiguous ([K][34] doubles): each
  // lane builds its source's row in registers, and the group writes the
  // rows out through LDS in two halves of 17 words, so that a store of the
  // group covers 128 consecutive bytes instead of one word of each of 16
  // rows. The group's lanes are in one wave, whose LDS accesses complete in
  // order.
  constexpr int kHalf = kSrcWords / 2;
  __shared__ double stage[256 / kSrcGroup][kSrcGroup][kHalf];
  const int sub = threadIdx.x & (kSrcGroup - 1);
  double(*st)[kHalf] = stage[threadIdx.x / kSrcGroup];
  const int64_t n = fd_count(a);
  const int64_t stride = (int64_t)gridDim.x * (blockDim.x / kSrcGroup);
  for (int64_t rank = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kSrcGroup; rank < n;
       rank += stride) {
    FdItem it;
    if (!fd_active_at(a, rank, it)) continue;
    for (int c0 = 0; c0 < it.K; c0 += kSrcGroup) {
      const int rows = it.K - c0 < kSrcGroup ? it.K - c0 : kSrcGroup;
      double w[kSrcWords];
      if (sub < rows) {
        const Src s = make_src(a.theta + (it.m0 + c0 + sub) * 8, a.fd_T_obs);
        src_store(w, s);
        w[kQPartner] = T2 > 0.0 ? __builtin_bit_cast(double, (int64_t)floor(s.f0 * T2)) : w[kQOwn];
      }
      double* out = a.fd_src + (it.m0 + c0) * kSrcWords;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (sub < rows) {
#pragma unroll
          for (int x = 0; x < kHalf; ++x) st[sub][x] = w[h * kHalf + x];
        }
        wave_lds_sync();
        for (int x = sub; x < rows * kHalf; x += kSrcGroup) {
          const int r = x / kHalf, c = x - r * kHalf;
          out[r * kSrcWords + h * kHalf + c] = st[r][c];
        }
        wave_lds_sync();
      }
    }
  }
}

// With a.stride_grid, grids of a fixed size per compute unit whose
// workgroups step through the listed particles: a grid as large as the
// population costs a dispatch per workgroup even when few particles are
// listed (late NUTS doublings). Full passes keep one workgroup per group of
// particles, which the hardware hands out in the K-sorted order.
unsigned fd_grid(const PopArgs& a, int64_t per_block, int64_t blocks_per_cu) {
  const int64_t need = (a.N + per_block - 1) / per_block;
  const int64_t cap = blocks_per_cu * (a.n_cu > 0 ? a.n_cu : 256);
  return (unsigned)std::max<int64_t>(1, a.stride_grid ? std::min(need, cap) : need);
}

hipError_t launch_src_pass(const PopArgs& a, hipStream_t st) {
  if (a.N == 0) return hipSuccess;
  hipLaunchKernelGGL(fd_src_kernel, dim3(fd_grid(a, 256 / kSrcGroup, 8)), dim3(256), 0, st, a,
                     a.fd_bridge ? a.fd2_T_obs : 0.0);
  return hipGetLastError();
}

template <int MODE>
hipError_t launch_fd_mode(const PopArgs& a, hipStream_t st) {
  if (a.N == 0) return hipSuccess;
  if (!a.fd_src_ready) {
    hipError_t e = launch_src_pass(a, st);
    if (e != hipSuccess) return e;
  }
  const dim3 block(256);
  const bool br = a.fd_bridge != 0;
  // two band bins per lane cover up to 128 bins; the wider of two bridged
  // bands decides
  const bool nr2 = a.fd_B <= 2 * kNs && !(br && a.fd2_B > 2 * kNs);
  // LDS bytes: the tables, and for the gradient a residual copy per wave
  const size_t lds2 = 8 * fd_lds_words(br, 4, MODE == 1 ? resid_words<2>() : 0);
  const size_t lds4 = 8 * fd_lds_words(br, 4, MODE == 1 ? resid_words<4>() : 0);
  if (MODE == 1 && a.stride_grid && nr2) {
    // three workgroups fit a compute unit at once: two rounds of them
    hipLaunchKernelGGL((fd_kernel<1, 2, true>), dim3(fd_grid(a, 4, 6)), block, lds2, st, a, a.fd_src);
    return hipGetLastError();
  }
  const dim3 grid((unsigned)((a.N + 3) / 4));
  if (nr2)
    hipLaunchKernelGGL((fd_kernel<MODE, 2, false>), grid, block, lds2, st, a, a.fd_src);
  else
    hipLaunchKernelGGL((fd_kernel<MODE, 4, false>), grid, block, lds4, st, a, a.fd_src);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_fd_src(const PopArgs& a, hipStream_t st) { return launch_src_pass(a, st); }

hipError_t launch_fd(int mode, const PopArgs& a, hipStream_t st) {
  if (a.fd_B < 1 || a.fd_B > 4 * kNs) return hipErrorInvalidValue;
  switch (mode) {
    case 0: return launch_fd_mode<0>(a, st);
    case 1: return launch_fd_mode<1>(a, st);
    case 2: return launch_fd_mode<2>(a, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fd_metric(const PopArgs& a, const int64_t* f_offsets, int64_t f_size, double* F,
                            int blocks, hipStream_t st) {
  if (a.N == 0) return hipSuccess;
  // the metric walks every particle in natural order (no ordering pass ran);
  // a.active (or nullptr) selects the particles it evaluates
  PopArgs all = a;
  all.order = nullptr;
  all.stride_grid = 0;
  hipError_t e = launch_src_pass(all, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(fd_metric_kernel, dim3((unsigned)((a.N + 3) / 4)), dim3(256),
                     8 * fd_lds_words(a.fd_bridge != 0, 4, 0), st, a, a.fd_src, f_offsets, f_size, F,
                     blocks);
  return hipGetLastError();
}

hipError_t launch_fd_spectrum(const PopArgs& a, int64_t K, double* out, hipStream_t st) {
  if (a.fd_B < 1 || a.fd_B > 4 * kNs) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fd_spectrum_kernel, dim3(1), dim3(64), 8 * fd_lds_words(false, 1, 0), st, a, K,
                     out);
  return hipGetLastError();
}

}  // namespace smcx
