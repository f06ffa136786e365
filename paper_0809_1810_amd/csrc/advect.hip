// Advection of the particles with their own velocity (eq. 5, dx_i/dt = u(x_i)):
// the two stages of Heun's explicit Runge-Kutta method,
//   x* = x + dt u(x),   x <- x + (dt / 2) (u(x) + u(x*)),
// elementwise on the caller's float64 arrays (input order).
#include "vfmm_internal.hpp"

namespace vfmm {

namespace {

__global__ void __launch_bounds__(256) k_heun_predict(const double* __restrict__ x,
                                                      const double* __restrict__ y,
                                                      const double* __restrict__ u,
                                                      const double* __restrict__ v, int64_t n,
                                                      double dt, double* __restrict__ xs,
                                                      double* __restrict__ ys) {
  const int64_t i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= n) return;
  xs[i] = x[i] + dt * u[i];
  ys[i] = y[i] + dt * v[i];
}

__global__ void __launch_bounds__(256) k_heun_correct(double* __restrict__ x,
                                                      double* __restrict__ y,
                                                      const double* __restrict__ u1,
                                                      const double* __restrict__ v1,
                                                      const double* __restrict__ u2,
                                                      const double* __restrict__ v2, int64_t n,
                                                      double half_dt) {
  const int64_t i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= n) return;
  x[i] = x[i] + half_dt * (u1[i] + u2[i]);
  y[i] = y[i] + half_dt * (v1[i] + v2[i]);
}

inline unsigned nb(int64_t n) { return unsigned((n + 255) / 256); }

}  // namespace

hipError_t launch_heun_predict(const double* x, const double* y, const double* u, const double* v,
                               int64_t n, double dt, double* xs, double* ys, hipStream_t st) {
  hipLaunchKernelGGL(k_heun_predict, dim3(nb(n)), dim3(256), 0, st, x, y, u, v, n, dt, xs, ys);
  return hipGetLastError();
}

hipError_t launch_heun_correct(double* x, double* y, const double* u1, const double* v1,
                               const double* u2, const double* v2, int64_t n, double dt,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_heun_correct, dim3(nb(n)), dim3(256), 0, st, x, y, u1, v1, u2, v2, n,
                     0.5 * dt);
  return hipGetLastError();
}

}  // namespace vfmm
