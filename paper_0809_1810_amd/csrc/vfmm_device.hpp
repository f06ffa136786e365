// Small device-side helpers shared by the kernels: complex arithmetic on HIP
// vector types and the per-precision particle / coefficient types.
#pragma once

#include "vfmm_internal.hpp"

namespace vfmm {

template <typename R> struct Types;
template <> struct Types<double> { using C = double2; using Part = Part64; };
template <> struct Types<float> { using C = float2; using Part = Part32; };

template <typename C> __device__ __forceinline__ C cmake(decltype(C::x) r, decltype(C::x) i) {
  C c; c.x = r; c.y = i; return c;
}
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return cmake<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// acc += a * b
template <typename C> __device__ __forceinline__ void cfma(C& acc, C a, C b) {
  acc.x += a.x * b.x - a.y * b.y;
  acc.y += a.x * b.y + a.y * b.x;
}

// Offsets of the interaction list: t = (ox, oy) in [-3,3]^2, table index.
__host__ __device__ __forceinline__ int m2l_index(int ox, int oy) { return (oy + 3) * 7 + (ox + 3); }

// Byte offsets inside the operator-table buffer for expansion order p.
struct OpsLayout {
  size_t m2m64, l2l64, m2l64, m2m32, l2l32, m2l32, mfma32, mfma16, scales, total;
  int mt;        // 32-row output tiles of the real 2p x 2p M2L block
  int ks32;      // K steps of the FP32 matrix instruction (K = 2)
  int ks16;      // K steps of the BF16/FP16 matrix instructions (K = 16)
};
__host__ __device__ inline OpsLayout ops_layout(int p) {
  OpsLayout o;
  const size_t pp = size_t(p) * size_t(p);
  size_t off = 0;
  auto take = [&](size_t b) { size_t r = off; off += (b + 255) & ~size_t(255); return r; };
  o.m2m64 = take(4 * pp * sizeof(double2));
  o.l2l64 = take(4 * pp * sizeof(double2));
  o.m2l64 = take(kM2LOffsets * pp * sizeof(double2));
  o.m2m32 = take(4 * pp * sizeof(float2));
  o.l2l32 = take(4 * pp * sizeof(float2));
  o.m2l32 = take(kM2LOffsets * pp * sizeof(float2));
  // M2L operands packed in matrix-instruction lane order (see m2l_mfma.hip)
  o.mt = (2 * p + 31) / 32;
  o.ks32 = p;
  o.ks16 = (2 * p + 15) / 16;
  o.mfma32 = take(size_t(kM2LOffsets) * o.mt * o.ks32 * 64 * sizeof(float));
  o.mfma16 = take(size_t(kM2LOffsets) * o.mt * o.ks16 * 64 * 8 * sizeof(uint16_t));
  o.scales = take(size_t(kMaxLevels + 1) * sizeof(uint32_t));
  o.total = off;
  return o;
}

}  // namespace vfmm
