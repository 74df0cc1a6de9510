// Batched population kernels for gfx950.
//
// One wave64 owns one work item (particle, chunk of samples). The particle's
// component parameters are turned into per-component FP32/FP64 constants by
// the wave's lanes in parallel and parked in the wave's LDS slice; the wave
// then walks its chunk in tiles of 64*S samples (lane l owns samples
// tile + 64 j + l), keeps the tile's residual in registers, synthesises the
// templates of all components in index order, and reduces.
//
// Precision scheme (the residual and templates are FP32):
//  * Pulses: the pulse centre is split in FP64 into an integer sample index n
//    and a fraction f, so x = (s - n) - f is formed exactly up to one FP32
//    rounding of x itself; the exponent uses one pre-scaled coefficient so
//    the Gaussian is a single hardware exp2.
//    Pulses are truncated where |t - t0| >= sqrt(128 ln 2) w: there the
//    template is below 2^-64 of its peak, far under the FP32 resolution of the
//    residual and the FP64 resolution of the sums it feeds. Each component
//    carries the sample range of its support, and the tile loops skip groups
//    of 64-sample blocks outside it with wave-uniform branches.
//  * Sinusoids: the phase in cycles is a quadratic in the sample index. Per
//    component, lane and tile its value and its per-64-sample step are
//    reduced modulo one cycle in FP64 and carried as 32-bit fixed point
//    (units of 2^-32 cycles, so wrap-around is the modulo); per sample the
//    phase is one integer add plus a small FP32 chirp correction, converted
//    to FP32 revolutions for the hardware sin/cos (they take revolutions).
//  * Sums of r^2 and the birth/death inner products are accumulated per lane
//    in FP64 (products of FP32 values are exact in FP64); gradient sums are
//    FP32 per lane per tile, reduced across the wave in FP32 and accumulated
//    across tiles in FP64.
// All reductions have a fixed order: a particle's results do not depend on
// the other particles in the batch, their order, or the run.
#include "smcx_internal.h"

#include <math.h>

#include <algorithm>
#include <type_traits>

namespace smcx {
namespace {

// sqrt(log2(e) / 2): exp(-x^2 / (2 w^2)) = exp2(-(a x)^2) with a = this / w.
constexpr double kSqrtHalfLog2e = 0.84932180028801904272150283410289;
// Pulse truncation radius in units of z = a x: z^2 = 64 gives exp2(-z^2) = 2^-64,
// i.e. |t - t0| = sqrt(128 ln 2) w.
constexpr double kPulseCutZ = 8.0;
// Bound on sample indices of a pulse support (the data length is at most 2^22).
constexpr double kSampleBound = 16777216.0;
// 1.5 * 2^20: doubles in [2^20, 2^21) have a unit in the last place of 2^-32.
constexpr double kPhaseMagic = 1572864.0;
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kPi = 3.141592653589793238462643383279;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---------------------------------------------------------------- DPP sums
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, ROW_MASK, 0xF, false);
}
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(float, dpp_i<CTRL, ROW_MASK>(__builtin_bit_cast(int, v)));
}
template <int CTRL, int ROW_MASK = 0xF>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = dpp_i<CTRL, ROW_MASK>((int)(b & 0xffffffffll));
  const int hi = dpp_i<CTRL, ROW_MASK>((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes (wave_sum_d); the total is valid in lane 63. The
// steps pair lanes within quads, half rows and rows, then carry row sums up
// with the row broadcasts (rows 1,3 add row 0,2; rows 2,3 add rows 0..1).
//
// Transposed wave sums of four values: one pair stage over lanes (L, L ^ 32)
// takes two values and leaves one (after the row swap, a + b holds a's pair
// sums in lanes 0-31 and b's in lanes 32-63), one over (L, L ^ 16) likewise
// per row pair, then the four row-internal steps (quads, half rows, rows).
// Row r of the result (lanes 16 r .. 16 r + 15) holds the total of value
// row_value(r): 0, 2, 1, 3. Three row swaps and four DPP adds instead of
// four separate six-step sums.
template <int H>
__device__ __forceinline__ float pair_sum_f(float a, float b) {
  const unsigned ua = __builtin_bit_cast(unsigned, a), ub = __builtin_bit_cast(unsigned, b);
  unsigned x, y;
  if constexpr (H == 32) {
    const auto r = __builtin_amdgcn_permlane32_swap(ua, ub, false, false);
    x = r[0];
    y = r[1];
  } else {
    static_assert(H == 16, "row swap span");
    const auto r = __builtin_amdgcn_permlane16_swap(ua, ub, false, false);
    x = r[0];
    y = r[1];
  }
  // An empty asm (no instruction) makes the second result opaque: this
  // compiler folds a float sum of the swap's two results into twice the
  // first (seen in the gfx950 assembly; the FP64 form is not affected).
  asm volatile("" : "+v"(y));
  return __builtin_bit_cast(float, x) + __builtin_bit_cast(float, y);
}
__device__ __forceinline__ float transposed_sum4_f(float v0, float v1, float v2, float v3) {
  float t = pair_sum_f<16>(pair_sum_f<32>(v0, v1), pair_sum_f<32>(v2, v3));
  t += dpp_f<0xB1>(t);   // quad_perm [1,0,3,2]
  t += dpp_f<0x4E>(t);   // quad_perm [2,3,0,1]
  t += dpp_f<0x141>(t);  // row_half_mirror
  t += dpp_f<0x140>(t);  // row_mirror
  return t;
}
// the value whose total row `row` holds after transposed_sum4_f
__device__ __forceinline__ int row_value(int row) { return ((row & 1) << 1) | (row >> 1); }

__device__ __forceinline__ double wave_sum_d(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  v += dpp_d<0x142, 0xA>(v);
  v += dpp_d<0x143, 0xC>(v);
  return v;
}
__device__ __forceinline__ double lane63_d(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(v & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
  return (int64_t)(((unsigned long long)(unsigned int)hi << 32) | (unsigned int)lo);
}

// ---------------------------------------------------------------- models
// Gaussian pulse h = A exp(-(t - t0)^2 / (2 w^2)).
struct PulseC {
  float nf;  // integer part of the centre in samples, as an exact float
  float a;   // sqrt(log2 e / 2) / (w / dt)
  float fa;  // (fractional part of the centre) * a
  float A;
  int lo, hi;  // first and last sample of the truncation support
  unsigned int groups;  // block groups met on the current tile (written per tile)
  int pad;
};
static_assert(sizeof(PulseC) == 32, "pulse constants are 32 bytes");

__device__ __forceinline__ PulseC pulse_make(const double* th, double t_start, double dt) {
  const double A = th[0], t0 = th[1], w = th[2];
  const double c = (t0 - t_start) / dt;
  double n = floor(c);
  n = fmin(fmax(n, -4194304.0), 4194304.0);  // keep s - n exact in FP32
  const double f = c - n;
  const double a = kSqrtHalfLog2e * dt / w;
  PulseC r;
  r.nf = (float)n;
  r.a = (float)a;
  r.fa = (float)(f * a);
  r.A = (float)A;
  // Support |s - c| <= 8 / |a|. Non-finite parameters keep the whole range so
  // that a NaN reaches the particle's outputs.
  double lo = -kSampleBound, hi = kSampleBound;
  const double aa = fabs(a);
  if (isfinite(A) && isfinite(c) && isfinite(aa) && aa > 0.0) {
    const double hw = kPulseCutZ / aa;
    lo = fmin(fmax(ceil(c - hw), -kSampleBound), kSampleBound);
    hi = fmin(fmax(floor(c + hw), -kSampleBound), kSampleBound);
  }
  r.lo = (int)lo;
  r.hi = (int)hi;
  r.groups = 0u;
  r.pad = 0;
  return r;
}

// Blocks of 64 samples are skipped in groups of kPulseGroup.
constexpr int kPulseGroup = 2;

// Bit g set when block group g of the tile starting at sample `tile` meets the
// support of a component (computed by one lane per component at the start of
// each tile, kept with the component's constants and read back by both passes
// as a wave-uniform 32-bit mask, which tests in one scalar instruction).
template <int S>
__device__ __forceinline__ unsigned int pulse_groups(const PulseC& c, int tile) {
  static_assert(S / kPulseGroup <= 32, "one bit per block group");
  // arithmetic shift: floor division by 64
  const int jlo = max((c.lo - tile) >> 6, 0);
  const int jhi = min(((c.hi - tile) >> 6) + 1, S);
  if (jlo >= jhi) return 0u;
  const int glo = jlo / kPulseGroup, n = (jhi - 1) / kPulseGroup - glo + 1;
  return (unsigned int)((n >= 32 ? 0xffffffffu : ((1u << n) - 1u)) << glo);
}

// Chirping sinusoid h = A sin(2 pi (a0 + a1 s + a2 s^2)) in sample index s.
struct GbC {
  double a0m;         // a0 + kPhaseMagic: the phase at s = 0, offset (see gb_tile)
  double a1, a2;      // the phase's linear and quadratic coefficients in cycles
  double p1m;         // 64 a1 + kPhaseMagic: the phase step per 64 samples at s = 0
  double a2x128;      // 128 a2: that step's growth per sample
  float A;
  float c2;  // 4096 a2 in units of 2^-32 cycles: the chirp per (sample step of 64)^2
};
static_assert(sizeof(GbC) == 48, "GB constants are 48 bytes");

__device__ __forceinline__ GbC gb_make(const double* th, double t_start, double dt, int64_t s_lo,
                                       int64_t s_hi, int S, int* flag) {
  const double A = th[0], f0 = th[1], fd = th[2], phi0 = th[3];
  GbC r;
  const double a0 = f0 * t_start + 0.5 * fd * t_start * t_start + phi0 / kTwoPi;
  r.a1 = (f0 + fd * t_start) * dt;
  r.a2 = 0.5 * fd * dt * dt;
  r.a0m = a0 + kPhaseMagic;
  r.p1m = 64.0 * r.a1 + kPhaseMagic;
  r.a2x128 = 128.0 * r.a2;
  r.A = (float)A;
  r.c2 = (float)(4096.0 * r.a2 * 4294967296.0);
  // The phase must stay below 2^19 cycles, so that its offset value stays in
  // the binade whose unit is 2^-32 cycles (gb_tile), and the in-tile chirp
  // correction must stay a small fraction of a cycle.
  const double sh = (double)s_hi;
  const double pmax = fabs(a0) + fabs(r.a1) * sh + fabs(r.a2) * sh * sh;
  const double chirp = fabs(4096.0 * r.a2) * (double)S * S;
  if (!(pmax < 524287.0 && chirp < 0.015625)) {
    if (pmax == pmax && chirp == chirp) atomicOr(flag, kFlagPhase);
    r.A = __builtin_nanf("");
  }
  return r;
}

// Over a lane's S samples of a tile (j = 0 .. S-1) the chirp P2 j^2 departs
// from its chord (S-1) P2 j, moved down by P2 (S-1)^2 / 8, by at most
// |P2| (S-1)^2 / 8. Where that is at most 32 units of 2^-32 cycles (7e-8 rad)
// for every component of a particle, the particle's tiles take the phase as
// linear in j (gb_tile folds the chord into the step), which saves the chirp
// term per sample.
__device__ __forceinline__ bool gb_chord_ok(const GbC& c, int S) {
  return fabs((double)c.c2) * (double)(S - 1) * (double)(S - 1) <= 256.0;
}
// Folds the chord into the constants: the phase at s = 0 moves down by
// 512 (S-1)^2 a2 and the step per 64 samples up by 4096 (S-1) a2, so that
// each tile's P0 and P1 (gb_tile) carry it without further work. The phase
// also gains 2^-24 cycles, half the unit of the 23-bit phase float (gb_rev1),
// which then rounds to nearest (an exact addition at the unit of a0m).
__device__ __forceinline__ void gb_linearize(GbC& c, int S) {
  c.a0m = fma(-512.0 * (double)((S - 1) * (S - 1)), c.a2, c.a0m) + 0x1p-24;
  c.p1m = fma(4096.0 * (double)(S - 1), c.a2, c.p1m);
}

// Low 32 bits of x = y + 1.5*2^20 with |y| < 2^19: x lies in [2^20, 2^21),
// whose unit is 2^-32, so these bits are y mod 1 cycle as a fixed-point
// number in units of 2^-32 cycles (x is rounded to that unit).
__device__ __forceinline__ unsigned int fixed_cycles(double x) {
  return (unsigned int)(__builtin_bit_cast(long long, x) & 0xffffffffll);
}

// Per (component, lane, tile): the lane's samples are s = u + 64 j, so the
// phase is P0 + P1 j + P2 j^2 with P0 = a0 + a1 u + a2 u^2, P1 = 64 a1 +
// 128 a2 u, P2 = 4096 a2. P0 and P1 are reduced modulo one cycle in FP64 and
// carried as 32-bit fixed point (wrap-around is the modulo); P0 + P1 j is an
// exact integer recurrence up to the rounding of P1 to 2^-32 (at most j/2
// units), and P2 j^2 (a tiny chirp correction) is added in FP32.
struct GbTile {
  unsigned int F0;  // P0 mod 1, fixed point
  unsigned int D;   // P1 mod 1, fixed point
  float c2;         // P2 in fixed-point units
};
// With LIN the constants carry the chord (gb_linearize): P2 j^2 is replaced
// by its chord (S-1) P2 j, centred. |P0| and |P1| stay below 2^19 cycles
// (gb_make), and the constant terms carry the offset 1.5*2^20, so that the
// final FMA of each lands in the binade whose bits below the unit are the
// phase modulo one cycle (one rounding to 2^-32 cycles, plus at most half a
// unit from rounding a0 and 64 a1 with the offset).
template <bool LIN, int S>
__device__ __forceinline__ GbTile gb_tile(const GbC& c, double u) {
  GbTile t;
  t.F0 = fixed_cycles(fma(fma(c.a2, u, c.a1), u, c.a0m));
  t.D = fixed_cycles(fma(c.a2x128, u, c.p1m));
  t.c2 = c.c2;
  return t;
}
// With the linear tile phase: the float 1 + F 2^-32 in [1, 2), one revolution
// plus the phase, built from its bits in one funnel shift (the exponent of 1
// above the top 23 bits of F). The sine in revolutions has period one, so
// this is the phase rounded to 2^-23 revolutions (a0m carries the half unit),
// at most 3.7e-7 rad from the fixed-point value, for a shift instead of a
// convert and a multiply per sample.
__device__ __forceinline__ float gb_rev1(unsigned int F) {
  return __builtin_bit_cast(float, __builtin_amdgcn_alignbit(0x7Fu, F, 9u));
}
// Phase of sample j in revolutions (about [-0.5, 0.5)), F = F0 + j D mod 2^32,
// plus the chirp correction unless the tile's phase is linear.
template <int J, bool LIN>
__device__ __forceinline__ float gb_rev(const GbTile& t, unsigned int F) {
  float y = (float)(int)F;
  if (!LIN && J > 0) y = __builtin_fmaf((float)(J * J), t.c2, y);
  return y * 0x1p-32f;
}

// ---------------------------------------------------------------- tile bodies
// Pulse forward over the tile's block groups that meet the support; within a
// group the blocks are independent, so each exp has other work behind it.
// Within a group of blocks the exp argument's base z = a x - (fraction) a
// steps by 64 a (exact: a power-of-two multiple of a) from block to block:
// the group's first block forms z from the sample offset, the next ones add
// the step (one add instead of an add and an FMA). The rounding of z then
// grows by at most one unit of |z| per block.
template <int S, int J, int G>
__device__ __forceinline__ void pulse_fwd_group(const PulseC& c, float a64, float z,
                                                float (&r)[S]) {
  if constexpr (G > 0 && J < S) {
    r[J] = __builtin_fmaf(-c.A, __builtin_amdgcn_exp2f(-(z * z)), r[J]);
    pulse_fwd_group<S, J + 1, G - 1>(c, a64, z + a64, r);
  }
}

template <int S, int J = 0>
__device__ __forceinline__ void pulse_fwd_j(const PulseC& c, float base, float (&r)[S],
                                            unsigned int groups) {
  if constexpr (J < S) {
    if (__builtin_expect((groups >> (J / kPulseGroup)) & 1u, 1u)) {
      const float z = __builtin_fmaf(base + (float)(64 * J), c.a, -c.fa);
      pulse_fwd_group<S, J, kPulseGroup>(c, 64.f * c.a, z, r);
    }
    pulse_fwd_j<S, J + kPulseGroup>(c, base, r, groups);
  }
}

template <int S, int J, int G>
__device__ __forceinline__ void pulse_adj_group(const PulseC& c, float a64, float z,
                                                const float (&r)[S], float& s0, float& s1,
                                                float& s2) {
  if constexpr (G > 0 && J < S) {
    const float nzz = -(z * z);  // the exp argument doubles as the width weight
    const float e = __builtin_amdgcn_exp2f(nzz);
    const float re = r[J] * e;
    s0 += re;
    s1 = __builtin_fmaf(re, z, s1);
    s2 = __builtin_fmaf(re, nzz, s2);
    pulse_adj_group<S, J + 1, G - 1>(c, a64, z + a64, r, s0, s1, s2);
  }
}

template <int S, int J = 0>
__device__ __forceinline__ void pulse_adj_j(const PulseC& c, float base, const float (&r)[S],
                                            float& s0, float& s1, float& s2,
                                            unsigned int groups) {
  if constexpr (J < S) {
    if (__builtin_expect((groups >> (J / kPulseGroup)) & 1u, 1u)) {
      const float z = __builtin_fmaf(base + (float)(64 * J), c.a, -c.fa);
      pulse_adj_group<S, J, kPulseGroup>(c, 64.f * c.a, z, r, s0, s1, s2);
    }
    pulse_adj_j<S, J + kPulseGroup>(c, base, r, s0, s1, s2, groups);
  }
}

// The forward pass with the exact (quadratic) tile phase: a sine per sample.
template <int S, int J = 0>
__device__ __forceinline__ void gb_fwd_exact_j(const GbTile& t, unsigned int F, float A,
                                               float (&r)[S]) {
  if constexpr (J + 1 < S) {
    const unsigned int F1 = F + t.D;
    const float s0 = __builtin_amdgcn_sinf(gb_rev<J, false>(t, F));
    const float s1 = __builtin_amdgcn_sinf(gb_rev<J + 1, false>(t, F1));
    r[J] = __builtin_fmaf(-A, s0, r[J]);
    r[J + 1] = __builtin_fmaf(-A, s1, r[J + 1]);
    gb_fwd_exact_j<S, J + 2>(t, F1 + t.D, A, r);
  } else if constexpr (J < S) {
    r[J] = __builtin_fmaf(-A, __builtin_amdgcn_sinf(gb_rev<J, false>(t, F)), r[J]);
  }
}

// Adjoint sums of one component over a lane's S samples: as = sum r sin, and
// the running sums A_j = sum_{i<=j} r_i cos_i, B_j = sum_{i<=j} A_i,
// C_j = sum_{i<=j} B_i, from which gb_moments takes sum x, sum j x, sum j^2 x
// (x = r cos) with one FMA and two adds per sample instead of a multiply, an
// add and two FMAs.
template <int S, bool LIN, int J = 0>
__device__ __forceinline__ void gb_adj_j(const GbTile& t, unsigned int F, const float (&r)[S],
                                         float& as, float& A, float& B, float& C) {
  if constexpr (J < S) {
    const float ph = gb_rev<J, LIN>(t, F);
    const float s = __builtin_amdgcn_sinf(ph);
    const float c = __builtin_amdgcn_cosf(ph);
    as = __builtin_fmaf(r[J], s, as);
    A = __builtin_fmaf(r[J], c, A);
    B += A;
    C += B;
    gb_adj_j<S, LIN, J + 1>(t, F + t.D, r, as, A, B, C);
  }
}

// The adjoint sums of gb_adj_j with the linear tile phase, the phasor
// z_j = e^{i phase_j} by recurrences in groups of kGbGroup samples. The
// first sample of the tile takes z from the hardware sin and cos; the first
// of each later group is the previous group's first turned by
// w4 = e^{i 2 pi kGbGroup D} (a complex multiply: two multiplies, two FMAs);
// the second of a group is its first turned by w = e^{i 2 pi D}; the others
// follow the three-term recurrence z_{j+1} = 2 cos(2 pi D) z_j - z_{j-1},
// one FMA per part. A rounding error made at step k of the three-term
// recurrence reaches step j multiplied by at most j - k (its propagator is
// sin((j - k) 2 pi D) / sin(2 pi D)), which the short groups keep small;
// over a tile of 32 samples the phasor stays within about 1e-6 of its exact
// value (a few 1e-7 typically). The adjoint only feeds the gradient, whose
// tolerance is 1e-5.
constexpr int kGbGroup = 4;

template <int S, int J = 0>
__device__ __forceinline__ void gb_adj_rot_j(const GbTile& t, float ws, float wc, float wc2,
                                             float w4s, float w4c, const float (&r)[S], float gr,
                                             float gi, float zr, float zi, float pr, float pi,
                                             float& as, float& A, float& B, float& C) {
  if constexpr (J < S) {
    if constexpr (J == 0) {
      const float ph = gb_rev1(t.F0);
      gi = __builtin_amdgcn_sinf(ph);
      gr = __builtin_amdgcn_cosf(ph);
      zr = gr;
      zi = gi;
    } else if constexpr (J % kGbGroup == 0) {
      const float nr = __builtin_fmaf(-gi, w4s, gr * w4c);
      const float ni = __builtin_fmaf(gr, w4s, gi * w4c);
      gr = nr;
      gi = ni;
      zr = gr;
      zi = gi;
    } else if constexpr (J % kGbGroup == 1) {
      const float nr = __builtin_fmaf(-zi, ws, zr * wc);
      const float ni = __builtin_fmaf(zr, ws, zi * wc);
      pr = zr;
      pi = zi;
      zr = nr;
      zi = ni;
    } else {
      const float nr = __builtin_fmaf(wc2, zr, -pr);
      const float ni = __builtin_fmaf(wc2, zi, -pi);
      pr = zr;
      pi = zi;
      zr = nr;
      zi = ni;
    }
    as = __builtin_fmaf(r[J], zi, as);
    A = __builtin_fmaf(r[J], zr, A);
    B += A;
    C += B;
    gb_adj_rot_j<S, J + 1>(t, ws, wc, wc2, w4s, w4c, r, gr, gi, zr, zi, pr, pi, as, A, B, C);
  }
}

// The forward pass with the linear tile phase, in groups of four samples:
// the second and third sines come from the hardware, the first and fourth
// from the three-term relation s_{j+1} + s_{j-1} = 2 cos(2 pi D) s_j
// applied once backwards and once forwards (one FMA each). Each derived
// value is one step from hardware values, so its error stays within about
// three times theirs: 6.6e-7 at most and 1.2e-7 rms against 1.6e-7 and
// 0.7e-7 for the hardware sine alone (FP32 emulation with the hardware's
// error), where two steps from the group's first two sines gave 1.4e-6.
template <int S, int G = 0>
__device__ __forceinline__ void gb_fwd_rec_j(unsigned int F1, unsigned int D, unsigned int D4,
                                             float wc2, float A, float (&r)[S]) {
  static_assert(kGbGroup == 4, "groups of four samples");
  if constexpr (G < S / kGbGroup) {
    constexpr int J = G * kGbGroup;
    const float s1 = __builtin_amdgcn_sinf(gb_rev1(F1));
    const float s2 = __builtin_amdgcn_sinf(gb_rev1(F1 + D));
    const float s0 = __builtin_fmaf(wc2, s1, -s2);
    const float s3 = __builtin_fmaf(wc2, s2, -s1);
    r[J] = __builtin_fmaf(-A, s0, r[J]);
    r[J + 1] = __builtin_fmaf(-A, s1, r[J + 1]);
    r[J + 2] = __builtin_fmaf(-A, s2, r[J + 2]);
    r[J + 3] = __builtin_fmaf(-A, s3, r[J + 3]);
    gb_fwd_rec_j<S, G + 1>(F1 + D4, D, D4, wc2, A, r);
  }
}

// sum x_j, sum j x_j, sum j^2 x_j over j < S from the final running sums:
// B = sum (S - j) x_j and C = sum (S - j)(S - j + 1)/2 x_j.
template <int S>
__device__ __forceinline__ void gb_moments(float A, float B, float C, float& c0, float& c1,
                                           float& c2) {
  c0 = A;
  c1 = __builtin_fmaf((float)S, A, -B);
  c2 = __builtin_fmaf((float)(2 * S + 1), c1, __builtin_fmaf(-(float)(S * S + S), A, 2.f * C));
}

template <int S, bool LIN, int J = 0>
__device__ __forceinline__ void gb_sub2_j(const GbTile& t, unsigned int F, float A, float (&r1)[S],
                                          float (&r2)[S]) {
  if constexpr (J < S) {
    const float s = __builtin_amdgcn_sinf(LIN ? gb_rev1(F) : gb_rev<J, LIN>(t, F));
    r1[J] = __builtin_fmaf(-A, s, r1[J]);
    r2[J] = __builtin_fmaf(-A, s, r2[J]);
    gb_sub2_j<S, LIN, J + 1>(t, F + t.D, A, r1, r2);
  }
}

template <int S, bool LIN, int J = 0>
__device__ __forceinline__ void gb_val_j(const GbTile& t, unsigned int F, float A, float (&h)[S]) {
  if constexpr (J < S) {
    h[J] = A * __builtin_amdgcn_sinf(LIN ? gb_rev1(F) : gb_rev<J, LIN>(t, F));
    gb_val_j<S, LIN, J + 1>(t, F + t.D, A, h);
  }
}

template <int MODEL>
struct Model;

template <>
struct Model<SMCX_PULSE> {
  using C = PulseC;
  static constexpr int P = 3;
  __device__ static C make(const double* th, const PopArgs& a, int /*S*/) {
    return pulse_make(th, a.t_start, a.dt);
  }
  // pulses have one tile path (LIN is ignored)
  __device__ static bool chord_ok(const C&, int) { return true; }
  __device__ static void linearize(C&, int) {}
  // the block groups of the tile that each component meets, one lane per
  // component, for both passes over the tile
  template <int S>
  __device__ static void prepare(C* cst, int K, int64_t tile, int lane) {
    for (int k = lane; k < K; k += 64) cst[k].groups = pulse_groups<S>(cst[k], (int)tile);
    wave_sync();
  }
  template <int S, bool LIN = true>
  __device__ static void forward(const C* cst, int K, int64_t tile, int lane, float (&r)[S]) {
    const float sf0 = (float)(int)(tile + lane);
    for (int k = 0; k < K; ++k) {
      const C c = cst[k];
      // the constants are read together with the mask (one LDS round trip)
      asm volatile("" ::"v"(c.nf), "v"(c.a), "v"(c.fa), "v"(c.A));
      const unsigned int groups = __builtin_amdgcn_readfirstlane(c.groups);
      if (groups == 0) continue;
      pulse_fwd_j<S>(c, sf0 - c.nf, r, groups);
    }
  }
  template <int S, bool LIN = true>
  __device__ static void adjoint(const C* cst, double* acc, int K, int64_t tile, int lane,
                                 const float (&r)[S]) {
    const float sf0 = (float)(int)(tile + lane);
    for (int k = 0; k < K; ++k) {
      const C c = cst[k];
      asm volatile("" ::"v"(c.nf), "v"(c.a), "v"(c.fa));  // one LDS round trip
      const unsigned int groups = __builtin_amdgcn_readfirstlane(c.groups);
      if (groups == 0) continue;  // the component adds nothing on this tile
      float s0 = 0.f, s1 = 0.f, s2 = 0.f;
      pulse_adj_j<S>(c, sf0 - c.nf, r, s0, s1, s2, groups);
      // the first lane of rows 0, 1, 2 adds the total of s0, s2, s1; the
      // accumulator is read before the sum so that the read overlaps it
      // (row 3 reads the next entry, which it does not use)
      double* ap = acc + 3 * k + row_value(lane >> 4);
      double prev = *ap;
      const float tot = transposed_sum4_f(s0, s1, s2, 0.f);
      asm volatile("" : "+v"(prev));  // keeps the read out of the branch below
      if ((lane & 15) == 0 && lane < 48) *ap = prev + (double)tot;
    }
  }
  // Template values of one component on the tile (for birth/death).
  template <int S, bool LIN = true>
  __device__ static void values(const C& c, int64_t tile, int lane, float (&h)[S]) {
    const float base = (float)(int)(tile + lane) - c.nf;
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const float dj = base + (float)(64 * j);
      const float z = __builtin_fmaf(dj, c.a, -c.fa);
      h[j] = c.A * __builtin_amdgcn_exp2f(-(z * z));
    }
  }
  template <int S, bool LIN = true>
  __device__ static void sub2(const C& c, int64_t tile, int lane, float (&r1)[S], float (&r2)[S]) {
    const float base = (float)(int)(tile + lane) - c.nf;
#pragma unroll
    for (int j = 0; j < S; ++j) {
      const float dj = base + (float)(64 * j);
      const float z = __builtin_fmaf(dj, c.a, -c.fa);
      const float e = __builtin_amdgcn_exp2f(-(z * z));
      r1[j] = __builtin_fmaf(-c.A, e, r1[j]);
      r2[j] = __builtin_fmaf(-c.A, e, r2[j]);
    }
  }
  // g = beta/sigma^2 * sum_s r_s dh/dtheta from the accumulated sums
  // S0 = sum r e, S1 = sum r e z, S2 = -sum r e z^2 with z = a x (x in samples).
  __device__ static void scale(const double* th, const double* sums, double bs, const PopArgs& a,
                               double* g) {
    const double A = th[0], w = th[2];
    const double af = (double)pulse_make(th, a.t_start, a.dt).a;
    g[0] = bs * sums[0];
    g[1] = bs * (A * a.dt / (af * w * w)) * sums[1];
    g[2] = -bs * (A * a.dt * a.dt / (af * af * w * w * w)) * sums[2];
  }
};

template <>
struct Model<SMCX_GBSINE> {
  using C = GbC;
  static constexpr int P = 4;
  __device__ static C make(const double* th, const PopArgs& a, int S) {
    return gb_make(th, a.t_start, a.dt, a.s_lo, a.s_hi, S, a.flag);
  }
  // LIN: every component of the particle takes the linear tile phase (gb_chord_ok)
  __device__ static bool chord_ok(const C& c, int S) { return gb_chord_ok(c, S); }
  __device__ static void linearize(C& c, int S) { gb_linearize(c, S); }
  // sinusoids span every tile: nothing to prepare
  template <int S>
  __device__ static void prepare(C*, int, int64_t, int) {}
  template <int S, bool LIN>
  __device__ static void forward(const C* cst, int K, int64_t tile, int lane, float (&r)[S]) {
    const double u = (double)(tile + lane);
    for (int k = 0; k < K; ++k) {
      const C c = cst[k];
      const GbTile t = gb_tile<LIN, S>(c, u);
      if constexpr (LIN) {
        const float wd = (float)(int)t.D * 0x1p-32f;  // step in revolutions
        gb_fwd_rec_j<S>(t.F0 + t.D, t.D, t.D * (unsigned int)kGbGroup,
                        2.f * __builtin_amdgcn_cosf(wd), c.A, r);
      } else {
        gb_fwd_exact_j<S>(t, t.F0, c.A, r);
      }
    }
  }
  template <int S, bool LIN>
  __device__ static void adjoint(const C* cst, double* acc, int K, int64_t tile, int lane,
                                 const float (&r)[S]) {
    const double u = (double)(tile + lane);
    const float uf = (float)(int)(tile + lane);
    for (int k = 0; k < K; ++k) {
      const C c = cst[k];
      const GbTile t = gb_tile<LIN, S>(c, u);
      float as = 0.f, A = 0.f, B = 0.f, Cs = 0.f;
      if constexpr (LIN) {
        const float wd = (float)(int)t.D * 0x1p-32f;  // step in revolutions
        const float wd4 = (float)(int)(t.D * (unsigned int)kGbGroup) * 0x1p-32f;
        const float wc = __builtin_amdgcn_cosf(wd);
        gb_adj_rot_j<S>(t, __builtin_amdgcn_sinf(wd), wc, 2.f * wc, __builtin_amdgcn_sinf(wd4),
                        __builtin_amdgcn_cosf(wd4), r, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, as, A, B, Cs);
      } else {
        gb_adj_j<S, LIN>(t, t.F0, r, as, A, B, Cs);
      }
      float c0, c1, c2;
      gb_moments<S>(A, B, Cs, c0, c1, c2);
      // sample s = u + 64 j:  sum rc s = u c0 + 64 c1,  sum rc s^2 = u^2 c0 + 128 u c1 + 4096 c2
      const float b1 = __builtin_fmaf(uf, c0, 64.f * c1);
      const float b2 = __builtin_fmaf(uf * uf, c0, __builtin_fmaf(128.f * uf, c1, 4096.f * c2));
      // the first lane of each row adds the total of one of as, c0, b1, b2;
      // the accumulator is read before the sum so that the read overlaps it
      double* ap = acc + 4 * k + row_value(lane >> 4);
      double prev = *ap;
      const float tot = transposed_sum4_f(as, c0, b1, b2);
      asm volatile("" : "+v"(prev));  // keeps the read out of the branch below
      if ((lane & 15) == 0) *ap = prev + (double)tot;
    }
  }
  template <int S, bool LIN>
  __device__ static void values(const C& c, int64_t tile, int lane, float (&h)[S]) {
    const GbTile t = gb_tile<LIN, S>(c, (double)(tile + lane));
    gb_val_j<S, LIN>(t, t.F0, c.A, h);
  }
  template <int S, bool LIN>
  __device__ static void sub2(const C& c, int64_t tile, int lane, float (&r1)[S], float (&r2)[S]) {
    const GbTile t = gb_tile<LIN, S>(c, (double)(tile + lane));
    gb_sub2_j<S, LIN>(t, t.F0, c.A, r1, r2);
  }
  // sums: S_sin = sum r sin, C0 = sum r cos, C1 = sum r cos s, C2 = sum r cos s^2.
  __device__ static void scale(const double* th, const double* sums, double bs, const PopArgs& a,
                               double* g) {
    const double A = th[0];
    const double ts = a.t_start, dt = a.dt;
    const double c0 = sums[1], c1 = sums[2], c2 = sums[3];
    g[0] = bs * sums[0];
    g[1] = bs * (kTwoPi * A) * (ts * c0 + dt * c1);
    g[2] = bs * (kPi * A) * (ts * ts * c0 + 2.0 * ts * dt * c1 + dt * dt * c2);
    g[3] = bs * A * c0;
  }
};

__host__ __device__ inline size_t const_bytes(int model) {
  return model == SMCX_PULSE ? sizeof(PulseC) : sizeof(GbC);
}

// LDS of one wave: the component constants, and for gradient passes the
// adjoint accumulators and the particle's theta rows (P doubles each).
__device__ __forceinline__ size_t lds_wave_bytes(int model, int32_t k_max, bool grad) {
  const size_t per = const_bytes(model) + (grad ? 2 * (size_t)n_params(model) * 8 : 0);
  return ((size_t)(k_max + 1) * per + 15) & ~(size_t)15;
}

// ---------------------------------------------------------------- work items
struct Item {
  int i;       // particle
  int c;       // chunk
  int64_t m0;  // first row
  int K;       // components
};

// Map a wave's item index to (particle, chunk). In sorted mode the ordering
// pass has already validated the particles and settled K = 0 ones. In
// particle order the wave validates its own particle: its rows must lie in
// [0, M] and K in [0, k_max] (and a death index in [-1, K)); an invalid
// particle gets NaN outputs and raises the device flag, a particle without
// components gets the precomputed K = 0 value (unless `with_k0`).
// Returns false when the wave has nothing more to do.
__device__ __forceinline__ bool decode_item(const PopArgs& a, int64_t item, int lane, int P,
                                            bool with_k0, Item& it) {
  if (a.order) {
    const int64_t n_items = (int64_t)(*a.n_active) * a.nch;
    if (item >= n_items) return false;
    const int64_t rank = item / a.nch;
    it.c = (int)(item - rank * a.nch);
    it.i = a.order[rank];
    it.m0 = a.offsets[it.i];
    it.K = (int)(a.offsets[it.i + 1] - it.m0);
    return true;
  }
  if (item >= a.N * (int64_t)a.nch) return false;
  const int64_t i = item / a.nch;
  it.c = (int)(item - i * a.nch);
  it.i = (int)i;
  if (item == 0 && lane == 0 && (a.offsets[0] != 0 || a.offsets[a.N] != a.M))
    atomicOr(a.flag, a.offsets[0] != 0 ? kFlagOffsets : kFlagMMax);
  const int64_t o0 = a.offsets[i], o1 = a.offsets[i + 1];
  const bool rows_ok = o0 >= 0 && o1 >= o0 && o1 <= a.M;
  int bad = rows_ok ? 0 : kFlagOffsets;
  if (rows_ok && o1 - o0 > a.k_max) bad |= kFlagKMax;
  if (a.death_idx) {
    const int32_t j = a.death_idx[i];
    if (j < -1 || (int64_t)j >= o1 - o0) bad |= kFlagDeath;
  }
  if (bad) {
    if (it.c == 0) {
      const double nan = __builtin_nan("");
      if (lane == 0) {
        atomicOr(a.flag, bad);
        if (a.logl) a.logl[i] = nan;
        if (a.dlogl_birth) a.dlogl_birth[i] = nan;
        if (a.dlogl_death) a.dlogl_death[i] = nan;
      }
      if (a.grad && rows_ok)
        for (int64_t m = o0 + lane; m < o1; m += 64)
          for (int p = 0; p < P; ++p) a.grad[m * P + p] = nan;
    }
    return false;
  }
  it.m0 = o0;
  it.K = (int)(o1 - o0);
  if (it.K == 0 && !with_k0) {
    if (it.c == 0 && lane == 0 && a.logl)
      a.logl[i] = a.k0_lo + (a.beta ? a.beta[i] : 1.0) * (a.k0_dev ? *a.k0_dev : a.k0);
    return false;
  }
  return true;
}

// Whether the combine pass has work for particle i (natural order): valid
// rows and at least one component (or any valid particle when `with_k0`).
__device__ __forceinline__ bool combine_item(const PopArgs& a, int64_t rank, bool with_k0,
                                             Item& it) {
  if (a.order) {
    if (rank >= *a.n_active) return false;
    it.i = a.order[rank];
  } else {
    if (rank >= a.N) return false;
    it.i = (int)rank;
  }
  const int64_t o0 = a.offsets[it.i], o1 = a.offsets[it.i + 1];
  if (!a.order) {
    if (!(o0 >= 0 && o1 >= o0 && o1 <= a.M && o1 - o0 <= a.k_max)) return false;
    if (a.death_idx) {
      const int32_t j = a.death_idx[it.i];
      if (j < -1 || (int64_t)j >= o1 - o0) return false;
    }
  }
  it.m0 = o0;
  it.K = (int)(o1 - o0);
  it.c = 0;
  return with_k0 || it.K > 0;
}

// ---------------------------------------------------------------- prep
// Ordering pass: validates every particle, settles the ones without work (K = 0
// outside the birth pass, invalid ones) and lists the rest longest-K first
// (a counting sort). Two launches over slices of kPrepSlice particles: the
// count pass writes one K histogram per slice, the scatter pass combines them
// into list positions and places its slice's particles. Each thread loads all
// of its particles of a slice before it uses any, so a pass pays about one
// memory latency. Particles of equal K are listed in no particular order
// (results do not depend on it).
constexpr int kPrepBlock = 256;
constexpr int kPrepUnroll = 8;
constexpr int kPrepSlice = kPrepBlock * kPrepUnroll;

// Work-list key of particle i: K, or -1 when it needs no pass. With `settle`,
// also writes the outputs of invalid and K = 0 particles.
__device__ __forceinline__ int prep_key(const PrepArgs& a, int64_t i, int64_t o0, int64_t o1,
                                        int32_t dj, double beta_i, int bad_global, bool settle) {
  const int64_t K = o1 - o0;
  int bits = 0;
  if (bad_global) bits |= kFlagOffsets;
  if (K < 0) bits |= kFlagOffsets;
  if (K > a.k_max) bits |= kFlagKMax;
  if (a.dlogl_death && a.death_idx && (dj < -1 || (int64_t)dj >= K)) bits |= kFlagDeath;
  if (bits) {
    if (settle) {
      const double nan = __builtin_nan("");
      if (!bad_global) atomicOr(a.flag, bits);
      if (a.logl) a.logl[i] = nan;
      if (a.dlogl_birth) a.dlogl_birth[i] = nan;
      if (a.dlogl_death) a.dlogl_death[i] = nan;
      if (a.grad && !bad_global && K > 0) {
        for (int64_t m = o0 < 0 ? 0 : o0; m < o1 && m < a.M; ++m)
          for (int p = 0; p < a.P; ++p) a.grad[m * a.P + p] = nan;
      }
    }
    return -1;
  }
  if (K == 0 && !a.include_k0) {
    if (settle && a.logl) a.logl[i] = a.k0_lo + beta_i * (a.k0_dev ? *a.k0_dev : a.k0_value);
    return -1;
  }
  return (int)K;
}

// Runs fn(i, key) for every particle of this block's slice. The loads are
// unconditional, on a clamped index, so that they are all in flight together.
template <bool SETTLE, bool DEATH, typename F>
__device__ __forceinline__ void prep_slice(const PrepArgs& a, int bad_global, F fn) {
  const int64_t base = (int64_t)blockIdx.x * kPrepSlice + threadIdx.x;
  int64_t o0[kPrepUnroll], o1[kPrepUnroll];
  int32_t dj[kPrepUnroll];
  double bt[kPrepUnroll];
#pragma unroll
  for (int u = 0; u < kPrepUnroll; ++u) {
    int64_t i = base + (int64_t)u * kPrepBlock;
    i = i < a.N ? i : a.N - 1;
    o0[u] = a.offsets[i];
    o1[u] = a.offsets[i + 1];
    dj[u] = DEATH ? a.death_idx[i] : 0;
    bt[u] = 1.0;
  }
  // the K = 0 outputs are tempered: fetch beta with the rest
  if (SETTLE && a.tempered && a.beta && a.logl) {
#pragma unroll
    for (int u = 0; u < kPrepUnroll; ++u) {
      const int64_t i = base + (int64_t)u * kPrepBlock;
      bt[u] = a.beta[i < a.N ? i : a.N - 1];
    }
  }
#pragma unroll
  for (int u = 0; u < kPrepUnroll; ++u) {
    const int64_t i = base + (int64_t)u * kPrepBlock;
    if (i < a.N) fn(i, prep_key(a, i, o0[u], o1[u], dj[u], bt[u], bad_global, SETTLE));
  }
}

template <bool SETTLE, typename F>
__device__ __forceinline__ void prep_slice(const PrepArgs& a, int bad_global, F fn) {
  if (a.dlogl_death && a.death_idx)
    prep_slice<SETTLE, true>(a, bad_global, fn);
  else
    prep_slice<SETTLE, false>(a, bad_global, fn);
}

// Whether offsets[0] != 0 or offsets[N] != M (every particle is then invalid).
__device__ __forceinline__ int prep_bad_global(const PrepArgs& a, bool raise) {
  __shared__ int bad_global;
  if (threadIdx.x == 0) {
    int bad = 0;
    if (a.N > 0 && (a.offsets[0] != 0 || a.offsets[a.N] != a.M)) bad = 1;
    bad_global = bad;
    if (bad && raise) atomicOr(a.flag, a.offsets[0] != 0 ? kFlagOffsets : kFlagMMax);
  }
  __syncthreads();
  return bad_global;
}

__global__ __launch_bounds__(kPrepBlock) void prep_count_kernel(PrepArgs a) {
  extern __shared__ int hist[];  // [k_max + 1]
  const int nk = a.k_max + 1;
  for (int k = threadIdx.x; k < nk; k += kPrepBlock) hist[k] = 0;
  const int bg = prep_bad_global(a, blockIdx.x == 0);
  prep_slice<true>(a, bg, [&](int64_t, int key) {
    if (key >= 0) atomicAdd(&hist[key], 1);
  });
  __syncthreads();
  for (int k = threadIdx.x; k < nk; k += kPrepBlock) a.block_hist[(size_t)blockIdx.x * nk + k] = hist[k];
}

__global__ __launch_bounds__(kPrepBlock) void prep_scatter_kernel(PrepArgs a) {
  extern __shared__ int sh[];
  const int nk = a.k_max + 1;  // at most 4 * kPrepBlock
  int* tot = sh;               // [nk] particles with K = k, all slices
  int* pos = sh + nk;          // [nk] particles with K = k in earlier slices, then list positions
  __shared__ int scan[kPrepBlock];
  const int tid = threadIdx.x;
  for (int k = tid; k < nk; k += kPrepBlock) tot[k] = pos[k] = 0;
  const int bg = prep_bad_global(a, false);
  // combine the slice histograms (loads batched four at a time)
  const int nh = (int)gridDim.x * nk;
  for (int base = 0; base < nh; base += 4 * kPrepBlock) {
    int c[4], idx[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      idx[q] = base + q * kPrepBlock + tid;
      c[q] = a.block_hist[idx[q] < nh ? idx[q] : nh - 1];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (idx[q] < nh && c[q]) {
        const int b = idx[q] / nk, k = idx[q] - b * nk;
        atomicAdd(&tot[k], c[q]);
        if (b < (int)blockIdx.x) atomicAdd(&pos[k], c[q]);
      }
    }
  }
  __syncthreads();
  // exclusive prefix of tot over K in descending order: 4 entries per thread,
  // then a Hillis-Steele scan over the thread sums
  int loc[4], sum = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = 4 * tid + q;  // j-th K in descending order
    loc[q] = j < nk ? tot[a.k_max - j] : 0;
    sum += loc[q];
  }
  scan[tid] = sum;
  __syncthreads();
  for (int off = 1; off < kPrepBlock; off <<= 1) {
    const int v = tid >= off ? scan[tid - off] : 0;
    __syncthreads();
    scan[tid] += v;
    __syncthreads();
  }
  int run = scan[tid] - sum;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int j = 4 * tid + q;
    if (j < nk) pos[a.k_max - j] += run;
    run += loc[q];
  }
  if (blockIdx.x == 0 && tid == kPrepBlock - 1) *a.n_active = scan[kPrepBlock - 1];
  __syncthreads();
  prep_slice<false>(a, bg, [&](int64_t i, int key) {
    if (key >= 0) a.order[atomicAdd(&pos[key], 1)] = (int32_t)i;
  });
}

// ---------------------------------------------------------------- population kernel
// GRAD = false: logL only (also the data-assimilation segment pass).
// GRAD = true : fused forward + adjoint.
// Occupancy target per tile size: the register file holds 512 VGPRs per lane
// per SIMD, so 8 waves per SIMD leave 64 VGPRs per wave; the residual tile
// alone needs S of them.
template <int MODEL, int S, bool GRAD>
constexpr int pop_waves_per_simd() {
  if (S <= 16) return 8;
  if (S == 32) return (MODEL == SMCX_GBSINE && GRAD) ? 7 : 8;
  return (MODEL == SMCX_GBSINE && GRAD) ? 4 : 5;
}

// The tiles of one work item: forward (and adjoint) over samples [cs, ce);
// returns the tempered (ss) and, with a split, untempered (ss_lo) sums of r^2
// of the lane. LIN selects the sinusoids' linear tile phase.
template <int MODEL, int S, bool GRAD, bool LIN>
__device__ __forceinline__ void pop_tiles(const PopArgs& a, typename Model<MODEL>::C* cst,
                                          double* acc, int K, int lane, int64_t cs, int64_t ce,
                                          bool split, double b, double& ss, double& ss_lo) {
  using M = Model<MODEL>;
  for (int64_t tile = cs; tile < ce; tile += 64 * S) {
    float r[S];
    // d32 is zero-padded by a full 4096-sample tile past T: no load guard
    const float* dp = a.d32 + tile + lane;
#pragma unroll
    for (int j = 0; j < S; ++j) r[j] = dp[64 * j];
    M::template prepare<S>(cst, K, tile, lane);
    M::template forward<S, LIN>(cst, K, tile, lane, r);
    if (tile + 64 * S > ce) {  // ragged tile: samples past the chunk contribute nothing
      const int nv = (int)(ce - tile) - lane;  // lane's samples j with 64 j < nv are inside
#pragma unroll
      for (int j = 0; j < S; ++j) r[j] = 64 * j < nv ? r[j] : 0.f;
    }
    if (!split) {
      // four FP32 chains of S/4 squares, each added to the FP64 sum once per
      // tile: a chain's relative rounding error is at most S/4 units of 2^-24
      // (typically about sqrt(S/4), the roundings falling either way), and
      // the errors of the many chains of a chunk are independent, so that the
      // sum's relative error stays far below that of the FP32 residual
      float q[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int j = 0; j < S; ++j) q[j & 3] = __builtin_fmaf(r[j], r[j], q[j & 3]);
      ss += ((double)q[0] + (double)q[1]) + ((double)q[2] + (double)q[3]);
    } else {
      // samples before the split count untempered; later ones carry beta,
      // which the adjoint then sees through the residual
      const float bf = (float)b;
#pragma unroll
      for (int j = 0; j < S; ++j) {
        const double rd = (double)r[j];
        const bool lo = tile + 64 * j + lane < a.split;
        ss_lo = lo ? fma(rd, rd, ss_lo) : ss_lo;
        ss = lo ? ss : fma(rd, rd, ss);
        if constexpr (GRAD) r[j] = lo ? r[j] : r[j] * bf;
      }
    }
    if constexpr (GRAD) M::template adjoint<S, LIN>(cst, acc, K, tile, lane, r);
  }
}

// One work item of the population kernel (a wave-uniform index).
template <int MODEL, int S, bool GRAD>
__device__ __forceinline__ void pop_item(const PopArgs& a, int64_t item, int lane, int wid,
                                         unsigned char* lds) {
  using M = Model<MODEL>;
  using C = typename M::C;
  constexpr int P = M::P;
  Item it;
  if (!decode_item(a, item, lane, P, false, it)) return;
  // one wave per item: make the item's fields scalar
  const int c = __builtin_amdgcn_readfirstlane(it.c);
  const int i = __builtin_amdgcn_readfirstlane(it.i);
  const int64_t m0 = uniform_i64(it.m0);
  const int K = __builtin_amdgcn_readfirstlane(it.K);
  if (a.active && !a.active[i]) return;

  unsigned char* base = lds + (size_t)wid * lds_wave_bytes(MODEL, a.k_max, GRAD);
  C* cst = reinterpret_cast<C*>(base);
  double* acc = reinterpret_cast<double*>(base + (size_t)(a.k_max + 1) * sizeof(C));
  double* thl = acc + (size_t)(a.k_max + 1) * P;  // the particle's theta rows (GRAD)
  const double* th = a.theta + m0 * P;
  if constexpr (GRAD) {
    // theta in whole lines, kept for the gradient's scaling at the end
    for (int idx = lane; idx < K * P; idx += 64) {
      thl[idx] = th[idx];
      acc[idx] = 0.0;
    }
    wave_sync();
    th = thl;
  }
  bool off_chord = false;  // a component whose chirp needs the exact tile phase
  for (int k = lane; k < K; k += 64) {
    cst[k] = M::make(th + k * P, a, S);
    off_chord |= !M::chord_ok(cst[k], S);
  }
  const bool lin = __builtin_amdgcn_ballot_w64(off_chord) == 0;
  if (lin)  // each lane its own components
    for (int k = lane; k < K; k += 64) M::linearize(cst[k], S);
  wave_sync();

  const int64_t cs = a.s_lo + (int64_t)c * a.chunk_len;
  const int64_t ce = min(cs + a.chunk_len, a.s_hi);
  const bool split = a.split > a.s_lo;  // posterior-start bridge target
  const double b = a.beta ? a.beta[i] : 1.0;
  double ss = 0.0, ss_lo = 0.0;  // tempered and (with a split) untempered sums of r^2
  if constexpr (MODEL != SMCX_GBSINE) {
    pop_tiles<MODEL, S, GRAD, true>(a, cst, acc, K, lane, cs, ce, split, b, ss, ss_lo);
  } else {
    if (lin)
      pop_tiles<MODEL, S, GRAD, true>(a, cst, acc, K, lane, cs, ce, split, b, ss, ss_lo);
    else
      pop_tiles<MODEL, S, GRAD, false>(a, cst, acc, K, lane, cs, ce, split, b, ss, ss_lo);
  }
  ss = lane63_d(wave_sum_d(ss));
  if (split) ss = lane63_d(wave_sum_d(ss_lo)) + b * ss;
  const double outer = split ? 1.0 : b;  // tempering still to apply

  if (a.nch == 1) {
    if (lane == 0 && a.logl) a.logl[i] = outer * (-0.5 * ss * a.inv_sigma2);
    if constexpr (GRAD) {
      wave_sync();
      const double bs = outer * a.inv_sigma2;
      // scale each component's sums in place, then write the rows out in
      // whole lines (lane idx of the particle's K P values)
      for (int k = lane; k < K; k += 64) {
        double g[P];
        M::scale(thl + k * P, acc + k * P, bs, a, g);
        for (int p = 0; p < P; ++p) acc[k * P + p] = g[p];
      }
      wave_sync();
      double* gd = a.grad + m0 * P;
      if (a.p_half) {
        const double he = 0.5 * a.eps * (a.dir ? (double)a.dir[i] : 1.0);
        const double* ph = a.p_half + m0 * P;
        double* po = a.p_out + m0 * P;
        for (int idx = lane; idx < K * P; idx += 64) {
          const double g = acc[idx];
          gd[idx] = g;
          po[idx] = fma(he, g, ph[idx]);
        }
      } else {
        for (int idx = lane; idx < K * P; idx += 64) gd[idx] = acc[idx];
      }
    }
  } else {
    if (lane == 0) a.part[(size_t)c * a.N + i] = ss;
    if constexpr (GRAD) {
      wave_sync();
      double* dst = a.part_g + ((size_t)c * a.m_max + m0) * P;
      for (int idx = lane; idx < K * P; idx += 64) dst[idx] = acc[idx];
    }
  }
}

// The population kernel: one wave per (particle, chunk) work item, or
// (PERSIST) a grid of what the device holds at once whose waves take the
// items at a fixed stride (item w, w + G, ... for wave w of G), which in the
// longest-K-first order hands each wave a similar share of the work. The
// two are separate kernels: the loop's state would otherwise raise the
// register count of the one-item form.
template <int MODEL, int S, bool GRAD, bool PERSIST>
__global__ __launch_bounds__(256, (pop_waves_per_simd<MODEL, S, GRAD>())) void pop_kernel(PopArgs a) {
  extern __shared__ __align__(16) unsigned char lds[];
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wpb = blockDim.x >> 6;
  const int64_t first = (int64_t)blockIdx.x * wpb + wid;
  if constexpr (!PERSIST) {
    pop_item<MODEL, S, GRAD>(a, first, lane, wid, lds);
    return;
  }
  const int64_t n = (a.order ? (int64_t)*a.n_active : a.N) * a.nch;
  const int64_t stride = (int64_t)gridDim.x * wpb;
  for (int64_t item = first; item < n; item += stride) {
    pop_item<MODEL, S, GRAD>(a, item, lane, wid, lds);
    wave_sync();  // the wave's LDS is reused by its next item
  }
}

// Combine chunk partials in chunk order; one wave per particle.
template <int MODEL, bool GRAD>
__global__ __launch_bounds__(256) void finalize_kernel(PopArgs a) {
  using M = Model<MODEL>;
  constexpr int P = M::P;
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t rank = (int64_t)blockIdx.x * (blockDim.x >> 6) + wid;
  Item it;
  if (!combine_item(a, rank, false, it)) return;
  const int i = it.i;
  const int64_t m0 = it.m0;
  const int K = it.K;
  if (a.active && !a.active[i]) return;
  // with a split the chunk partials already carry the per-sample tempering
  const double outer = a.split > a.s_lo ? 1.0 : (a.beta ? a.beta[i] : 1.0);
  if (lane == 0 && a.logl) {
    double ss = 0.0;
    for (int c = 0; c < a.nch; ++c) ss += a.part[(size_t)c * a.N + i];
    a.logl[i] = outer * (-0.5 * ss * a.inv_sigma2);
  }
  if constexpr (GRAD) {
    const double bs = outer * a.inv_sigma2;
    for (int k = lane; k < K; k += 64) {
      double sums[P];
      for (int p = 0; p < P; ++p) sums[p] = 0.0;
      for (int c = 0; c < a.nch; ++c) {
        const double* src = a.part_g + ((size_t)c * a.m_max + m0 + k) * P;
        for (int p = 0; p < P; ++p) sums[p] += src[p];
      }
      double g[P];
      M::scale(a.theta + (m0 + k) * P, sums, bs, a, g);
      for (int p = 0; p < P; ++p) a.grad[(m0 + k) * P + p] = g[p];
      if (a.p_half) {
        const double he = 0.5 * a.eps * (a.dir ? (double)a.dir[i] : 1.0);
        for (int p = 0; p < P; ++p)
          a.p_out[(m0 + k) * P + p] = fma(he, g[p], a.p_half[(m0 + k) * P + p]);
      }
    }
  }
}

// ---------------------------------------------------------------- birth / death
// One pass per (particle, chunk): r (all components) and r_-j (all but j)
// in index order, the templates of the death candidate j and of the birth
// candidate, and four FP64 inner products per lane.
// The tiles of one birth/death work item: the four inner products of the lane.
template <int MODEL, int S, bool LIN>
__device__ __forceinline__ void delta_tiles(const PopArgs& a, const typename Model<MODEL>::C* cst,
                                            int K, int j_death, bool birth, int lane, int64_t cs,
                                            int64_t ce, bool split, double bw, double& xb,
                                            double& yb, double& xd, double& yd) {
  using M = Model<MODEL>;
  using C = typename M::C;
  for (int64_t tile = cs; tile < ce; tile += 64 * S) {
    float rf[S], rn[S], hj[S];
    const float* dp = a.d32 + tile + lane;
#pragma unroll
    for (int jj = 0; jj < S; ++jj) {
      rf[jj] = dp[64 * jj];
      rn[jj] = rf[jj];
      hj[jj] = 0.f;
    }
    for (int k = 0; k < K; ++k) {
      const C cc = cst[k];
      if (k == j_death) {
        M::template values<S, LIN>(cc, tile, lane, hj);
        // r (all components) still subtracts h_j, with the same fma as below
        float dummy[S];
#pragma unroll
        for (int jj = 0; jj < S; ++jj) dummy[jj] = 0.f;
        M::template sub2<S, LIN>(cc, tile, lane, rf, dummy);
      } else {
        M::template sub2<S, LIN>(cc, tile, lane, rf, rn);
      }
    }
    float hn[S];
    if (birth) {
      M::template values<S, LIN>(cst[K], tile, lane, hn);
    } else {
#pragma unroll
      for (int jj = 0; jj < S; ++jj) hn[jj] = 0.f;
    }
    const int nv = (int)min(ce - tile, (int64_t)(64 * S)) - lane;
    if (!split) {
#pragma unroll
      for (int jj = 0; jj < S; ++jj) {
        const bool ok = 64 * jj < nv;
        const double r1 = ok ? (double)rf[jj] : 0.0;
        const double r2 = ok ? (double)rn[jj] : 0.0;
        const double h1 = ok ? (double)hn[jj] : 0.0;
        const double h2 = ok ? (double)hj[jj] : 0.0;
        xb = fma(r1, h1, xb);
        yb = fma(h1, h1, yb);
        xd = fma(r2, h2, xd);
        yd = fma(h2, h2, yd);
      }
    } else {  // per-sample weight: 1 before the split, beta after (products of floats are exact)
#pragma unroll
      for (int jj = 0; jj < S; ++jj) {
        const bool ok = 64 * jj < nv;
        const double r1 = ok ? (double)rf[jj] : 0.0;
        const double r2 = ok ? (double)rn[jj] : 0.0;
        const double h1 = ok ? (double)hn[jj] : 0.0;
        const double h2 = ok ? (double)hj[jj] : 0.0;
        const double ws = tile + 64 * jj + lane < a.split ? 1.0 : bw;
        xb = fma(ws, r1 * h1, xb);
        yb = fma(ws, h1 * h1, yb);
        xd = fma(ws, r2 * h2, xd);
        yd = fma(ws, h2 * h2, yd);
      }
    }
  }
}

template <int MODEL, int S>
__global__ __launch_bounds__(256, (S <= 8 ? 6 : 4)) void delta_kernel(PopArgs a) {
  using M = Model<MODEL>;
  using C = typename M::C;
  constexpr int P = M::P;
  extern __shared__ __align__(16) unsigned char lds[];
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int wpb = blockDim.x >> 6;
  const int64_t item = (int64_t)blockIdx.x * wpb + wid;
  Item it;
  if (!decode_item(a, item, lane, P, true, it)) return;
  const int c = it.c;
  const int i = it.i;
  const int64_t m0 = it.m0;
  const int K = it.K;
  if (a.active && !a.active[i]) return;
  const int j_death = a.death_idx ? a.death_idx[i] : -1;
  const bool birth = a.theta_birth != nullptr;
  if (!birth && j_death < 0) {  // nothing to evaluate: no birth, no death
    if (c == 0 && lane == 0) a.dlogl_death[i] = 0.0;
    return;
  }

  C* cst = reinterpret_cast<C*>(lds + (size_t)wid * lds_wave_bytes(MODEL, a.k_max, false));
  for (int k = lane; k < K; k += 64) cst[k] = M::make(a.theta + (m0 + k) * P, a, S);
  if (birth && lane == 0) cst[K] = M::make(a.theta_birth + (int64_t)i * P, a, S);
  wave_sync();

  const int64_t cs = a.s_lo + (int64_t)c * a.chunk_len;
  const int64_t ce = min(cs + a.chunk_len, a.s_hi);
  const bool split = a.split > a.s_lo;  // posterior-start bridge target
  const double bw = a.beta ? a.beta[i] : 1.0;
  double xb = 0.0, yb = 0.0, xd = 0.0, yd = 0.0;
  // sinusoids take the exact tile phase here, whatever the components: the
  // templates of a birth and of the matching death must not depend on which
  // other components (or candidates) the two calls see
  delta_tiles<MODEL, S, MODEL != SMCX_GBSINE>(a, cst, K, j_death, birth, lane, cs, ce, split, bw,
                                              xb, yb, xd, yd);
  xb = lane63_d(wave_sum_d(xb));
  yb = lane63_d(wave_sum_d(yb));
  xd = lane63_d(wave_sum_d(xd));
  yd = lane63_d(wave_sum_d(yd));
  if (lane != 0) return;
  if (a.nch == 1) {
    const double b = split ? 1.0 : bw;  // tempering still to apply
    if (birth) a.dlogl_birth[i] = b * (xb - 0.5 * yb) * a.inv_sigma2;
    if (a.death_idx) a.dlogl_death[i] = j_death < 0 ? 0.0 : -(b * (xd - 0.5 * yd) * a.inv_sigma2);
  } else {
    double* dst = a.part + ((size_t)c * a.N + i) * 4;
    dst[0] = xb;
    dst[1] = yb;
    dst[2] = xd;
    dst[3] = yd;
  }
}

__global__ __launch_bounds__(256) void delta_finalize_kernel(PopArgs a) {
  const int64_t rank = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  Item it;
  if (!combine_item(a, rank, true, it)) return;
  const int i = it.i;
  if (a.active && !a.active[i]) return;
  if (!a.theta_birth && (!a.death_idx || a.death_idx[i] < 0)) return;  // settled by the main pass
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int c = 0; c < a.nch; ++c) {
    const double* src = a.part + ((size_t)c * a.N + i) * 4;
    for (int q = 0; q < 4; ++q) s[q] += src[q];
  }
  const double b = a.split > a.s_lo ? 1.0 : (a.beta ? a.beta[i] : 1.0);
  if (a.theta_birth) a.dlogl_birth[i] = b * (s[0] - 0.5 * s[1]) * a.inv_sigma2;
  if (a.death_idx) {
    const int j = a.death_idx[i];
    a.dlogl_death[i] = j < 0 ? 0.0 : -(b * (s[2] - 0.5 * s[3]) * a.inv_sigma2);
  }
}

// ---------------------------------------------------------------- reweighting
// Single-block, fixed-order reductions over the population.
__global__ __launch_bounds__(1024) void reweight_kernel(int64_t N, double delta_beta,
                                                        const double* logl_ext,
                                                        const double* logw_prev, double* logw,
                                                        double* w_norm, double* scalars) {
  __shared__ double red[1024];
  __shared__ double red2[1024];
  const int t = threadIdx.x;
  const int nt = blockDim.x;
  const int64_t per = (N + nt - 1) / nt;
  const int64_t lo = min((int64_t)t * per, N), hi = min(lo + per, N);
  auto tree = [&](double v, double v2, bool is_max) {
    red[t] = v;
    red2[t] = v2;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
      if (t < w) {
        red[t] = is_max ? fmax(red[t], red[t + w]) : red[t] + red[t + w];
        red2[t] = red2[t] + red2[t + w];
      }
      __syncthreads();
    }
    double r0 = red[0];
    double r1 = red2[0];
    __syncthreads();
    return make_double2(r0, r1);
  };
  double m = -INFINITY;
  for (int64_t i = lo; i < hi; ++i) {
    const double v = (logw_prev ? logw_prev[i] : 0.0) + delta_beta * logl_ext[i];
    logw[i] = v;
    m = fmax(m, v);
  }
  m = tree(m, 0.0, true).x;
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = lo; i < hi; ++i) {
    const double e = exp(logw[i] - m);
    s1 += e;
    s2 += e * e;
  }
  const double2 S = tree(s1, s2, false);
  for (int64_t i = lo; i < hi; ++i) w_norm[i] = exp(logw[i] - m) / S.x;
  double lse_prev = log((double)N);
  if (logw_prev) {
    double mp = -INFINITY;
    for (int64_t i = lo; i < hi; ++i) mp = fmax(mp, logw_prev[i]);
    mp = tree(mp, 0.0, true).x;
    double sp = 0.0;
    for (int64_t i = lo; i < hi; ++i) sp += exp(logw_prev[i] - mp);
    sp = tree(sp, 0.0, false).x;
    lse_prev = mp + log(sp);
  }
  if (t == 0) {
    if (N == 0) {
      scalars[0] = 0.0;
      scalars[1] = 0.0;
      scalars[2] = -INFINITY;
    } else {
      scalars[0] = S.x * S.x / S.y;
      scalars[1] = m + log(S.x) - lse_prev;
      scalars[2] = m;
    }
  }
}

// The same reductions over many workgroups (three launches): each workgroup
// takes a slice of particles in whole lines; range maxima and sums are
// combined in slice order by every workgroup of the next launch, so all of
// them use the same bits. exp(log w - m) is computed once and kept in w_norm
// until the last launch divides it by the sum.
constexpr int kRwBlock = 256;
constexpr int kRwPer = 4;
constexpr int kRwSlice = kRwBlock * kRwPer;

struct RwArgs {
  int64_t N;
  double delta_beta;
  const double* logl_ext;
  const double* logw_prev;
  double* logw;
  double* w_norm;
  double* scalars;
  double* part;  // [G][5]: max log w, max logw_prev, sum e, sum e^2, sum e_prev
  int G;
};

template <bool MAX>
__device__ __forceinline__ double rw_block(double v, double* sh) {
  for (int o = 32; o >= 1; o >>= 1) {
    const double u = __shfl_xor(v, o);
    v = MAX ? fmax(v, u) : v + u;
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = sh[0];
  for (int w = 1; w < kRwBlock / 64; ++w) r = MAX ? fmax(r, sh[w]) : r + sh[w];
  return r;
}

__global__ __launch_bounds__(kRwBlock) void rw_max_kernel(RwArgs a) {
  __shared__ double sh[kRwBlock / 64];
  const int64_t base = (int64_t)blockIdx.x * kRwSlice;
  double m = -INFINITY, mp = -INFINITY;
#pragma unroll
  for (int u = 0; u < kRwPer; ++u) {
    const int64_t i = base + u * kRwBlock + threadIdx.x;
    if (i < a.N) {
      const double lp = a.logw_prev ? a.logw_prev[i] : 0.0;
      const double v = lp + a.delta_beta * a.logl_ext[i];
      a.logw[i] = v;
      m = fmax(m, v);
      mp = fmax(mp, lp);
    }
  }
  m = rw_block<true>(m, sh);
  mp = rw_block<true>(mp, sh);
  if (threadIdx.x == 0) {
    a.part[5 * blockIdx.x] = m;
    a.part[5 * blockIdx.x + 1] = mp;
  }
}

__global__ __launch_bounds__(kRwBlock) void rw_sum_kernel(RwArgs a) {
  __shared__ double sh[kRwBlock / 64];
  double m = -INFINITY, mp = -INFINITY;
  for (int g = 0; g < a.G; ++g) {
    m = fmax(m, a.part[5 * g]);
    mp = fmax(mp, a.part[5 * g + 1]);
  }
  const int64_t base = (int64_t)blockIdx.x * kRwSlice;
  double s1 = 0.0, s2 = 0.0, sp = 0.0;
#pragma unroll
  for (int u = 0; u < kRwPer; ++u) {
    const int64_t i = base + u * kRwBlock + threadIdx.x;
    if (i < a.N) {
      const double e = exp(a.logw[i] - m);
      a.w_norm[i] = e;
      s1 += e;
      s2 += e * e;
      if (a.logw_prev) sp += exp(a.logw_prev[i] - mp);
    }
  }
  s1 = rw_block<false>(s1, sh);
  s2 = rw_block<false>(s2, sh);
  sp = rw_block<false>(sp, sh);
  if (threadIdx.x == 0) {
    a.part[5 * blockIdx.x + 2] = s1;
    a.part[5 * blockIdx.x + 3] = s2;
    a.part[5 * blockIdx.x + 4] = sp;
  }
}

__global__ __launch_bounds__(kRwBlock) void rw_weights_kernel(RwArgs a) {
  __shared__ double tot[5];
  if (threadIdx.x == 0) {
    double m = -INFINITY, mp = -INFINITY, s1 = 0.0, s2 = 0.0, sp = 0.0;
    for (int g = 0; g < a.G; ++g) {
      m = fmax(m, a.part[5 * g]);
      mp = fmax(mp, a.part[5 * g + 1]);
      s1 += a.part[5 * g + 2];
      s2 += a.part[5 * g + 3];
      sp += a.part[5 * g + 4];
    }
    tot[0] = m;
    tot[1] = mp;
    tot[2] = s1;
    tot[3] = s2;
    tot[4] = sp;
  }
  __syncthreads();
  const double s1 = tot[2];
  const int64_t base = (int64_t)blockIdx.x * kRwSlice;
#pragma unroll
  for (int u = 0; u < kRwPer; ++u) {
    const int64_t i = base + u * kRwBlock + threadIdx.x;
    if (i < a.N) a.w_norm[i] = a.w_norm[i] / s1;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const double lse_prev = a.logw_prev ? tot[1] + log(tot[4]) : log((double)a.N);
    a.scalars[0] = s1 * s1 / tot[3];
    a.scalars[1] = tot[0] + log(s1) - lse_prev;
    a.scalars[2] = tot[0];
  }
}

// ---------------------------------------------------------------- leapfrog drift
// First half of a leapfrog step, one wave per particle over its K*P values:
//   p_half = p + (eps_i/2) g,  q' = q + eps_i p_half;
// inactive particles copy (q, p, g) to the outputs unchanged.
__global__ __launch_bounds__(256) void drift_kernel(int P, int64_t N, int64_t M,
                                                    const int64_t* offsets, double eps,
                                                    const int8_t* dir,
                                                    const uint8_t* active, const double* q_in,
                                                    const double* p_in, const double* g_in,
                                                    double* q_out, double* p_out, double* g_out) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= N) return;
  const int64_t o0 = offsets[i], o1 = offsets[i + 1];
  if (o0 < 0 || o1 < o0 || o1 > M) return;  // invalid particles are reported by the gradient pass
  const bool on = !active || active[i];
  const double e = eps * (dir ? (double)dir[i] : 1.0);
  for (int64_t x = o0 * P + lane; x < o1 * P; x += 64) {
    if (on) {
      const double ph = fma(0.5 * e, g_in[x], p_in[x]);
      p_out[x] = ph;
      q_out[x] = fma(e, ph, q_in[x]);
    } else {
      q_out[x] = q_in[x];
      p_out[x] = p_in[x];
      g_out[x] = g_in[x];
    }
  }
}

// ---------------------------------------------------------------- synthesis
__global__ __launch_bounds__(256) void template_sum_kernel(int model, int64_t K,
                                                           const double* theta, int64_t T,
                                                           double t_start, double dt,
                                                           double* out) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= T) return;
  const double t = t_start + (double)s * dt;
  double acc = 0.0;
  for (int64_t k = 0; k < K; ++k) {
    const double* th = theta + k * n_params(model);
    if (model == SMCX_PULSE) {
      const double x = t - th[1];
      acc += th[0] * exp(-(x * x) / (2.0 * th[2] * th[2]));
    } else {
      acc += th[0] * sin(kTwoPi * th[1] * t + kPi * th[2] * t * t + th[3]);
    }
  }
  out[s] = acc;
}

int waves_per_block(int model, int32_t k_max, bool grad) {
  const size_t per = ((size_t)(k_max + 1) * (const_bytes(model) + (grad ? 2 * n_params(model) * 8 : 0)) +
                      15) & ~(size_t)15;
  int w = 4;
  while (w > 1 && per * w > 65536) --w;
  return w;
}

template <int MODEL, int S, bool GRAD>
const void* pop_fn(bool persist) {
  return persist ? (const void*)pop_kernel<MODEL, S, GRAD, true>
                 : (const void*)pop_kernel<MODEL, S, GRAD, false>;
}

template <int MODEL, bool GRAD>
hipError_t launch_pop_model(const Tiling& t, const PopArgs& a, hipStream_t st) {
  const int wpb = waves_per_block(MODEL, a.k_max, GRAD);
  const size_t lds = pop_lds_bytes_per_wave(MODEL, a.k_max, GRAD) * wpb;
  const int64_t items = a.N * (int64_t)a.nch;
  if (items == 0) return a.prof_stop ? hipEventRecord((hipEvent_t)a.prof_stop, st) : hipSuccess;
  int64_t blocks = (items + wpb - 1) / wpb;
  const void* fn;
  switch (t.S) {
    case 8: fn = pop_fn<MODEL, 8, GRAD>(a.persist); break;
    case 16: fn = pop_fn<MODEL, 16, GRAD>(a.persist); break;
    case 32: fn = pop_fn<MODEL, 32, GRAD>(a.persist); break;
    case 64: fn = pop_fn<MODEL, 64, GRAD>(a.persist); break;
    default: return hipErrorInvalidValue;
  }
  if (a.persist) {
    // the workgroups the device holds at once (at least one per unit)
    int per_cu = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 64 * wpb, lds);
    if (e != hipSuccess) return e;
    blocks = std::min<int64_t>(blocks, (int64_t)std::max(per_cu, 1) * (a.n_cu > 0 ? a.n_cu : 256));
  }
  const dim3 grid((unsigned)blocks);
  const dim3 block(64 * wpb);
  void* args[] = {const_cast<PopArgs*>(&a)};
  hipError_t e = hipLaunchKernel(fn, grid, block, args, lds, st);
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess && a.prof_stop) e = hipEventRecord((hipEvent_t)a.prof_stop, st);
  if (e != hipSuccess || a.nch == 1) return e;
  const dim3 fgrid((unsigned)((a.N + 3) / 4));
  hipLaunchKernelGGL((finalize_kernel<MODEL, GRAD>), fgrid, dim3(256), 0, st, a);
  return hipGetLastError();
}

template <int MODEL>
hipError_t launch_delta_model(const Tiling& t, const PopArgs& a, hipStream_t st) {
  const int wpb = waves_per_block(MODEL, a.k_max, false);
  const size_t lds = pop_lds_bytes_per_wave(MODEL, a.k_max, false) * wpb;
  const int64_t items = a.N * (int64_t)a.nch;
  if (items == 0) return hipSuccess;
  const dim3 grid((unsigned)((items + wpb - 1) / wpb));
  const dim3 block(64 * wpb);
  switch (t.S) {
    case 8: hipLaunchKernelGGL((delta_kernel<MODEL, 8>), grid, block, lds, st, a); break;
    case 16: hipLaunchKernelGGL((delta_kernel<MODEL, 16>), grid, block, lds, st, a); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || a.nch == 1) return e;
  hipLaunchKernelGGL(delta_finalize_kernel, dim3((unsigned)((a.N + 255) / 256)), dim3(256), 0, st,
                     a);
  return hipGetLastError();
}

}  // namespace

size_t pop_lds_bytes_per_wave(int model, int32_t k_max, bool grad) {
  const size_t per = const_bytes(model) + (grad ? 2 * (size_t)n_params(model) * 8 : 0);
  return ((size_t)(k_max + 1) * per + 15) & ~(size_t)15;
}

hipError_t launch_prep(const PrepArgs& a, hipStream_t st) {
  if (a.k_max + 1 > 4 * kPrepBlock) return hipErrorInvalidValue;
  const dim3 grid((unsigned)prep_slices(a.N));
  hipLaunchKernelGGL(prep_count_kernel, grid, dim3(kPrepBlock), (size_t)(a.k_max + 1) * sizeof(int),
                     st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(prep_scatter_kernel, grid, dim3(kPrepBlock),
                     2 * (size_t)(a.k_max + 1) * sizeof(int), st, a);
  return hipGetLastError();
}

int64_t prep_slices(int64_t N) { return N > 0 ? (N + kPrepSlice - 1) / kPrepSlice : 1; }

hipError_t launch_forward(int model, const Tiling& t, const PopArgs& a, hipStream_t st) {
  if (model == SMCX_GBLISA) return launch_fd(0, a, st);
  return model == SMCX_PULSE ? launch_pop_model<SMCX_PULSE, false>(t, a, st)
                             : launch_pop_model<SMCX_GBSINE, false>(t, a, st);
}

hipError_t launch_fused(int model, const Tiling& t, const PopArgs& a, hipStream_t st) {
  if (model == SMCX_GBLISA) return launch_fd(1, a, st);
  return model == SMCX_PULSE ? launch_pop_model<SMCX_PULSE, true>(t, a, st)
                             : launch_pop_model<SMCX_GBSINE, true>(t, a, st);
}

hipError_t launch_delta(int model, const Tiling& t, const PopArgs& a, hipStream_t st) {
  if (model == SMCX_GBLISA) return launch_fd(2, a, st);
  return model == SMCX_PULSE ? launch_delta_model<SMCX_PULSE>(t, a, st)
                             : launch_delta_model<SMCX_GBSINE>(t, a, st);
}

hipError_t launch_reweight_reduce(int64_t N, double delta_beta, const double* logl_ext,
                                  const double* logw_prev, double* logw, double* w_norm,
                                  double* scalars, double* part, size_t part_cap, hipStream_t st) {
  const int64_t G = (N + kRwSlice - 1) / kRwSlice;
  if (N == 0 || !part || part_cap < (size_t)(5 * G)) {
    hipLaunchKernelGGL(reweight_kernel, dim3(1), dim3(1024), 0, st, N, delta_beta, logl_ext,
                       logw_prev, logw, w_norm, scalars);
    return hipGetLastError();
  }
  RwArgs a{N, delta_beta, logl_ext, logw_prev, logw, w_norm, scalars, part, (int)G};
  const dim3 grid((unsigned)G), block(kRwBlock);
  hipLaunchKernelGGL(rw_max_kernel, grid, block, 0, st, a);
  hipLaunchKernelGGL(rw_sum_kernel, grid, block, 0, st, a);
  hipLaunchKernelGGL(rw_weights_kernel, grid, block, 0, st, a);
  return hipGetLastError();
}

hipError_t launch_drift(int model, int64_t N, int64_t M, const int64_t* offsets, double eps,
                        const int8_t* dir, const uint8_t* active, const double* q_in,
                        const double* p_in, const double* g_in, double* q_out, double* p_out,
                        double* g_out, hipStream_t st) {
  if (N == 0) return hipSuccess;
  hipLaunchKernelGGL(drift_kernel, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, st, n_params(model),
                     N, M, offsets, eps, dir, active, q_in, p_in, g_in, q_out, p_out, g_out);
  return hipGetLastError();
}

hipError_t launch_template_sum(int model, int64_t K, const double* theta, int64_t T,
                               double t_start, double dt, double* out, hipStream_t st) {
  if (T == 0) return hipSuccess;
  hipLaunchKernelGGL(template_sum_kernel, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, st,
                     model, K, theta, T, t_start, dt, out);
  return hipGetLastError();
}

}  // namespace smcx
