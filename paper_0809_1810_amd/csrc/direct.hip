// FP64 direct sum (eq. 7 / eq. 9) and the error metrics used to judge the FMM.
//
// Direct: u(x_i) = sum_{j != i} Gamma_j K_sigma(x_i - x_j) with the regularised
// kernel of eq. 6, evaluated at all particles, at a list of particle indices, or
// at separate evaluation points (eq. 8).
// One thread per target; each block stages 256 sources at a time through LDS,
// so every source is read once per block.  The self pair (and any coincident
// pair) has a zero offset and contributes exactly zero.
//
// Metrics (Section 5.1, errors normalised by the maximum velocity):
// out[0] = max_i |dW_i|, out[1] = sum_i |dW_i|^2, out[2] = max_i |W_ref,i|; and
// the per-point error field log10(|dW_i| / max |W_ref|) behind the paper's
// spatial error maps (Section 5).
#include "vfmm_device.hpp"

namespace vfmm {

namespace {

constexpr double kInv2Pi = 0.15915494309189533576888376337251436;

__global__ void __launch_bounds__(256) k_direct(const double* __restrict__ x,
                                                const double* __restrict__ y,
                                                const double* __restrict__ g, int64_t n,
                                                double kexp, const int64_t* __restrict__ targets,
                                                const double* __restrict__ xt,
                                                const double* __restrict__ yt, int64_t nt,
                                                double* __restrict__ u, double* __restrict__ v) {
  __shared__ double sx[256], sy[256], sg[256];
  const int64_t t = blockIdx.x * 256LL + threadIdx.x;
  const bool valid = t < nt;
  double xi, yi;
  bool in_range = true;
  if (xt) {  // separate evaluation points (eq. 8)
    xi = valid ? xt[t] : 0.0;
    yi = valid ? yt[t] : 0.0;
  } else {
    int64_t i = valid ? (targets ? targets[t] : t) : 0;
    in_range = i >= 0 && i < n;  // out-of-range target indices yield NaN
    if (!in_range) i = 0;
    xi = x[i];
    yi = y[i];
  }
  double au = 0.0, av = 0.0;
  for (int64_t base = 0; base < n; base += 256) {
    const int64_t j = base + threadIdx.x;
    __syncthreads();
    sx[threadIdx.x] = j < n ? x[j] : 0.0;
    sy[threadIdx.x] = j < n ? y[j] : 0.0;
    sg[threadIdx.x] = j < n ? g[j] : 0.0;
    __syncthreads();
    const int cnt = int(n - base < 256 ? n - base : 256);
    for (int k = 0; k < cnt; ++k) {
      const double dx = xi - sx[k];
      const double dy = yi - sy[k];
      const double r2 = dx * dx + dy * dy;
      const double f = r2 > 0.0 ? sg[k] * (-expm1(r2 * kexp) / r2) : 0.0;
      au -= f * dy;
      av += f * dx;
    }
  }
  if (valid) {
    u[t] = in_range ? au * kInv2Pi : __builtin_nan("");
    v[t] = in_range ? av * kInv2Pi : __builtin_nan("");
  }
}

__global__ void __launch_bounds__(256) k_metrics_partial(const double* __restrict__ u,
                                                         const double* __restrict__ v,
                                                         const double* __restrict__ ur,
                                                         const double* __restrict__ vr, int64_t n,
                                                         double* __restrict__ part) {
  __shared__ double s[3][256];
  double mx = 0.0, ss = 0.0, mr = 0.0;
  for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) {
    const double d = hypot(u[i] - ur[i], v[i] - vr[i]);
    mx = fmax(mx, d);
    ss += d * d;
    mr = fmax(mr, hypot(ur[i], vr[i]));
  }
  s[0][threadIdx.x] = mx; s[1][threadIdx.x] = ss; s[2][threadIdx.x] = mr;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (int(threadIdx.x) < st) {
      s[0][threadIdx.x] = fmax(s[0][threadIdx.x], s[0][threadIdx.x + st]);
      s[1][threadIdx.x] += s[1][threadIdx.x + st];
      s[2][threadIdx.x] = fmax(s[2][threadIdx.x], s[2][threadIdx.x + st]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 3) part[blockIdx.x * 3 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ void __launch_bounds__(256) k_metrics_final(const double* __restrict__ part, int nb,
                                                       double* __restrict__ out) {
  __shared__ double s[3][256];
  double mx = 0.0, ss = 0.0, mr = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) {
    mx = fmax(mx, part[3 * b]);
    ss += part[3 * b + 1];
    mr = fmax(mr, part[3 * b + 2]);
  }
  s[0][threadIdx.x] = mx; s[1][threadIdx.x] = ss; s[2][threadIdx.x] = mr;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (int(threadIdx.x) < st) {
      s[0][threadIdx.x] = fmax(s[0][threadIdx.x], s[0][threadIdx.x + st]);
      s[1][threadIdx.x] += s[1][threadIdx.x + st];
      s[2][threadIdx.x] = fmax(s[2][threadIdx.x], s[2][threadIdx.x + st]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 3) out[threadIdx.x] = s[threadIdx.x][0];
}

// log10(|dW_i| / max |W_ref|), floored at 1e-300; NaN propagates.
__global__ void __launch_bounds__(256) k_error_field(const double* __restrict__ u,
                                                     const double* __restrict__ v,
                                                     const double* __restrict__ ur,
                                                     const double* __restrict__ vr, int64_t n,
                                                     const double* __restrict__ metrics,
                                                     double* __restrict__ out) {
  const int64_t i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= n) return;
  const double m = metrics[2];
  const double den = m > 0.0 ? m : 1.0;
  const double d = hypot(u[i] - ur[i], v[i] - vr[i]) / den;
  out[i] = log10(d > 1e-300 ? d : (d == d ? 1e-300 : d));
}

}  // namespace

hipError_t launch_error_field(const double* u, const double* v, const double* ur,
                              const double* vr, int64_t n, const double* metrics, double* out,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_error_field, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, u, v, ur,
                     vr, n, metrics, out);
  return hipGetLastError();
}

hipError_t launch_direct(const double* x, const double* y, const double* g, int64_t n,
                         double sigma, const int64_t* targets, const double* xt,
                         const double* yt, int64_t nt, double* u, double* v, hipStream_t st) {
  const double kexp = -1.0 / (2.0 * sigma * sigma);
  hipLaunchKernelGGL(k_direct, dim3(unsigned((nt + 255) / 256)), dim3(256), 0, st, x, y, g, n,
                     kexp, targets, xt, yt, nt, u, v);
  return hipGetLastError();
}

hipError_t launch_error_metrics(const double* u, const double* v, const double* ur,
                                const double* vr, int64_t n, double* partial, double* out,
                                hipStream_t st) {
  int nb = int((n + 255) / 256);
  if (nb > kReduceBlocks) nb = kReduceBlocks;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_metrics_partial, dim3(nb), dim3(256), 0, st, u, v, ur, vr, n, partial);
  hipLaunchKernelGGL(k_metrics_final, dim3(1), dim3(256), 0, st, partial, nb, out);
  return hipGetLastError();
}

}  // namespace vfmm
