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
  __device__ __forceinline__ static double near_series(double g, double r2, double kexp, double) {
    return near(g, r2, kexp);
  }
  __device__ __forceinline__ static double far(double g, double r2) { return g / r2; }
  // Gamma exp(r2 kexp) / r2: the regularised kernel minus the singular one
  // (up to sign), for the distance cut-off beyond the local list
  __device__ __forceinline__ static double gauss(double g, double r2, double kexp) {
    return g * (exp(r2 * kexp) / r2);
  }
};

template <> struct P2PMath<float> {
  static constexpr double kFarSigma2 = 36.0;  // exp(-18) < 2^-25
  static constexpr double kSeriesSigma2 = 1.0 / 16.0;  // a = r^2 / 2 sigma^2 < 1/32
  // kexp = -log2(e) / (2 sigma^2); Gamma (1 - e) computed as one fused op
  __device__ __forceinline__ static float near(float g, float r2, float kexp) {
    const float e = __builtin_amdgcn_exp2f(r2 * kexp);
    return __builtin_fmaf(-g, e, g) * __builtin_amdgcn_rcpf(r2);
  }
  // Close pairs: 1 - exp(-a) from the hardware exp has an absolute error of
  // ~2^-24, which divided by r would dominate for r << sigma; below a = 1/32
  // the series a (1 - a/2 + a^2/6 - a^3/24) is used (truncation < 8e-9).
  __device__ __forceinline__ static float near_series(float g, float r2, float kexp, float ka) {
    const float a = r2 * ka;
    const float ser = a * (1.0f - a * (0.5f - a * (1.0f / 6.0f - a * (1.0f / 24.0f))));
    const float e = __builtin_amdgcn_exp2f(r2 * kexp);
    const float om = a < 0.03125f ? ser : 1.0f - e;
    return g * om * __builtin_amdgcn_rcpf(r2);
  }
  __device__ __forceinline__ static float far(float g, float r2) {
    return g * __builtin_amdgcn_rcpf(r2);
  }
  __device__ __forceinline__ static float gauss(float g, float r2, float kexp) {
    return g * __builtin_amdgcn_exp2f(r2 * kexp) * __builtin_amdgcn_rcpf(r2);
  }
  // The same in units of the Gaussian width (r'^2 = r^2 log2(e) / (2 sigma^2)):
  // exp(-r^2 / 2 sigma^2) = exp2(-r'^2), the exponent argument is a free
  // operand negation; the forms return Gamma (...) / r'^2.
  __device__ __forceinline__ static float near_s(float g, float r2) {
    const float e = __builtin_amdgcn_exp2f(-r2);
    return __builtin_fmaf(-g, e, g) * __builtin_amdgcn_rcpf(r2);
  }
  __device__ __forceinline__ static float near_series_s(float g, float r2) {
    const float a = r2 * 0.69314718055994530942f;  // r^2 / (2 sigma^2)
    const float ser = a * (1.0f - a * (0.5f - a * (1.0f / 6.0f - a * (1.0f / 24.0f))));
    const float e = __builtin_amdgcn_exp2f(-r2);
    const float om = a < 0.03125f ? ser : 1.0f - e;
    return g * om * __builtin_amdgcn_rcpf(r2);
  }
  __device__ __forceinline__ static float gauss_s(float g, float r2) {
    return g * __builtin_amdgcn_exp2f(-r2) * __builtin_amdgcn_rcpf(r2);
  }
};


}  // namespace vfmm
