// Pair arithmetic of the near field (eq. 6 in complex form) shared by the
// single-tree and the batched kernels.
#pragma once

#include "vfmm_device.hpp"

namespace vfmm {

constexpr double kInv2Pi = 0.15915494309189533576888376337251436;

struct Acc32 {
  float s, c;
  __device__ __forceinline__ void add(float x) {  // Knuth TwoSum
    const float t = s + x;
    const float z = t - s;
    c += (s - (t - z)) + (x - z);
    s = t;
  }
  __device__ __forceinline__ double value() const { return double(s) + double(c); }
};

template <typename R> struct P2PMath;

template <> struct P2PMath<double> {
  static constexpr double kFarSigma2 = 76.0;  // exp(-38) < 2^-54
  static constexpr double kSeriesSigma2 = -1.0;  // expm1 is accurate for small r: no series
  // Gamma (1 - exp(r2 kexp)) / r2 with kexp = -1 / (2 sigma^2)
  __device__ __forceinline__ static double near(double g, double r2, double kexp) {
    return g * (-expm1(r2 * kexp) / r2);
  }
  __device__ __forceinline__ static double far(double g, double r2) { return g / r2; }
  // Gamma exp(r2 kexp) / r2: the regularised kernel minus the singular one
  // (up to sign), for the distance cut-off beyond the local list
  __device__ __forceinline__ static double gauss(double g, double r2, double kexp) {
    return g * (exp(r2 * kexp) / r2);
  }
  // the same kernel values without the circulation (symmetric pairs)
  __device__ __forceinline__ static double h_near(double r2, double kexp) {
    return -expm1(r2 * kexp) / r2;
  }
  __device__ __forceinline__ static double h_far(double r2) { return 1.0 / r2; }
};

template <> struct P2PMath<float> {
  static constexpr double kFarSigma2 = 36.0;  // exp(-18) < 2^-25
  // chunks whose box comes closer than sigma / 4 to the target tile take the
  // series form below (a = r^2 / 2 sigma^2 < 1/32 is possible there only)
  static constexpr double kSeriesSigma2 = 1.0 / 16.0;
  __device__ __forceinline__ static float far(float g, float r2) {
    return g * __builtin_amdgcn_rcpf(r2);
  }
  // The regularised forms in units of the Gaussian width
  // (r'^2 = r^2 log2(e) / (2 sigma^2)): exp(-r^2 / 2 sigma^2) = exp2(-r'^2), the
  // exponent argument is a free operand negation; they return Gamma (...) / r'^2,
  // with Gamma (1 - e) computed as one fused op.
  __device__ __forceinline__ static float near_s(float g, float r2) {
    const float e = __builtin_amdgcn_exp2f(-r2);
    return __builtin_fmaf(-g, e, g) * __builtin_amdgcn_rcpf(r2);
  }
  // Close pairs: 1 - e^-a from the hardware exp has an absolute error of
  // ~2^-24, which divided by r'^2 would dominate for r << sigma.  With
  // a = r'^2 ln 2 = r^2 / (2 sigma^2), below a = 1/32 the kernel
  // (1 - e^-a) / r'^2 = ln 2 (1 - a/2 + a^2/6 - a^3/24) is taken as that cubic in
  // r'^2 (truncation < 8e-9 relative), which needs neither the exponential nor
  // the reciprocal; above it the near form.
  static constexpr float kSeriesR2s = 0.045084220027780106f;  // (1/32) / ln 2
  __device__ __forceinline__ static float near_series_s(float g, float r2) {
    const float ser = 0.6931471805599453f +
                      r2 * (-0.2402265069591007f + r2 * (0.05550410866482158f +
                                                         r2 * -0.009618129107628477f));
    const float fn = __builtin_fmaf(-g, __builtin_amdgcn_exp2f(-r2), g) * __builtin_amdgcn_rcpf(r2);
    return r2 < kSeriesR2s ? g * ser : fn;
  }
  __device__ __forceinline__ static float gauss_s(float g, float r2) {
    return g * __builtin_amdgcn_exp2f(-r2) * __builtin_amdgcn_rcpf(r2);
  }
  // the same kernel values without the circulation (symmetric pairs)
  __device__ __forceinline__ static float h_far(float r2) { return __builtin_amdgcn_rcpf(r2); }
  __device__ __forceinline__ static float h_near_s(float r2) {
    const float r = __builtin_amdgcn_rcpf(r2);
    return __builtin_fmaf(-__builtin_amdgcn_exp2f(-r2), r, r);  // (1 - e) / r'^2 in one op
  }
  __device__ __forceinline__ static float h_series_s(float r2) {
    const float ser = 0.6931471805599453f +
                      r2 * (-0.2402265069591007f + r2 * (0.05550410866482158f +
                                                         r2 * -0.009618129107628477f));
    return r2 < kSeriesR2s ? ser : h_near_s(r2);
  }
};


// ------------------------------------------------------- symmetric near field
// Symmetric pairs of two chunks of <= 64 particles (K_sigma is odd, so one
// kernel value serves both directions): one wave holds 64 targets, one per
// lane, and stages the source chunk twice in a row in its own LDS block of 128
// records (entry k holds source (k + 1) mod 64, so that lane l reads source
// (l - s) mod 64 at step s from a fixed offset); per step each lane evaluates
// the kernel of its pair once and adds it to its target with the source's
// circulation and to the source's sums with its own.  The source sums move one
// lane up per step (DPP rotation of the whole wave), so after 64 steps every
// lane holds those of source j0 + lane, which it adds to that particle's
// float64 entry with an atomic addition.
template <typename R> struct __align__(sizeof(R) * 4) SymRec { R x, y, g, pad; };

// The single-tree near field evaluates a pair of chunks both ways at once only
// when they hold at least this many particles together: the 64 steps of a
// symmetric pair cost about what one direction per chunk costs for 96
// particles.
constexpr int kSymMinPair = 96;

__device__ __forceinline__ float lane_up(float v) {  // lane l takes lane l - 1 (mod 64)
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x13C,
                                                            0xF, 0xF, false));
}
__device__ __forceinline__ double lane_up(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = uint32_t(__builtin_amdgcn_mov_dpp(int(uint32_t(b)), 0x13C, 0xF, 0xF, false));
  const uint32_t hi = uint32_t(__builtin_amdgcn_mov_dpp(int(uint32_t(b >> 32)), 0x13C, 0xF, 0xF, false));
  return __builtin_bit_cast(double, (uint64_t(hi) << 32) | lo);
}

// The 64 steps.  FORM: 0 the near form, 1 with the series for close pairs, 2
// the far form; K supplies the circulation-free kernel values hnear, hseries,
// hfar of r'^2.
template <typename R, int FORM, typename K>
__device__ __forceinline__ void sym_steps(const SymRec<R>* __restrict__ rd, R tx, R ty, R tg,
                                          R tiny, const K& pk, R& cu, R& cv, R& su, R& sv) {
#pragma unroll 4
  for (int st = 0; st < 64; ++st) {
    const SymRec<R> q = rd[63 - st];
    const R dx = tx - q.x;
    const R dy = ty - q.y;
    R h;
    if constexpr (FORM == 2) {
      h = pk.hfar(dx * dx + dy * dy);
    } else {
      const R r2 = dx * dx + (dy * dy + tiny);
      h = FORM == 1 ? pk.hseries(r2) : pk.hnear(r2);
    }
    const R a = q.g * h, b = tg * h;
    cu -= a * dy;
    cv += a * dx;
    su += b * dy;
    sv -= b * dx;
    su = lane_up(su);
    sv = lane_up(sv);
  }
}

// One symmetric chunk pair: stage sources part[j0 .. j1) (padding: zero
// circulation at the leaf centre) in buf, run the steps against the lane's
// target (tx, ty, circulation tg; 0 for a padding lane) into (cu, cv), and add
// the source sums times `scale` to react[j0 + lane].
template <typename R, typename Part, typename K>
__device__ __forceinline__ void sym_pair_chunk(SymRec<R>* __restrict__ buf,
                                               const Part* __restrict__ part, int32_t j0,
                                               int32_t j1, int lane, R tx, R ty, R tg, R tiny,
                                               const K& pk, int form, double scale,
                                               double2* __restrict__ react, R& cu, R& cv) {
  SymRec<R> rec{R(0), R(0), R(0), R(0)};
  if (j0 + lane < j1) {
    const auto q = part[j0 + lane];
    rec = SymRec<R>{q.x, q.y, q.g, R(0)};
  }
  // this wave's reads of the previous chunk were consumed before (issued
  // before these writes; LDS operations of a wave are performed in order),
  // and the reads below wait for the writes
  buf[(lane + 63) & 63] = rec;
  buf[64 + ((lane + 63) & 63)] = rec;
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  const SymRec<R>* rd = buf + lane;
  R su = R(0), sv = R(0);
  if (form == 2) sym_steps<R, 2>(rd, tx, ty, tg, tiny, pk, cu, cv, su, sv);
  else if (form == 0) sym_steps<R, 0>(rd, tx, ty, tg, tiny, pk, cu, cv, su, sv);
  else sym_steps<R, 1>(rd, tx, ty, tg, tiny, pk, cu, cv, su, sv);
  if (j0 + lane < j1) {
    double* rj = reinterpret_cast<double*>(react + (j0 + lane));
    unsafeAtomicAdd(rj, double(su) * scale);
    unsafeAtomicAdd(rj + 1, double(sv) * scale);
  }
}

}  // namespace vfmm
