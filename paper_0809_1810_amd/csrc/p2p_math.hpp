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


}  // namespace vfmm
