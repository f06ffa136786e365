// FP64 direct sum (eq. 7 / eq. 9) and the error metrics used to judge the FMM.
//
// Direct: u(x_i) = sum_{j != i} Gamma_j K_sigma(x_i - x_j) with the regularised
// kernel of eq. 6, evaluated at all particles, at a list of particle indices, or
// at separate evaluation points (eq. 8).
// 16 targets per workgroup, the sources split over its 16 waves and 4 lanes
// per target, so that a few thousand audit targets still keep several waves
// on every SIMD.  The self pair (and any coincident pair)
// has a zero offset and contributes exactly zero.
//
// Metrics (Section 5.1, errors normalised by the maximum velocity):
// out[0] = max_i |dW_i|, out[1] = sum_i |dW_i|^2, out[2] = max_i |W_ref,i|; and
// the per-point error field log10(|dW_i| / max |W_ref|) behind the paper's
// spatial error maps (Section 5).
#include <cstdio>
#include <mutex>

#include "vfmm_device.hpp"

// Partial sums of vfmm_error_metrics_noalloc: a file-scope device array, one
// copy per GPU, held until the process ends (12 KB).  Host code never passes
// the array's name to a kernel (on the host it is only a stand-in for the
// symbol); it uses the device address hipGetSymbolAddress gives for the
// current device, looked up once per device.
static __device__ __align__(256) double scratch[vfmm::kReduceBlocks * 3];

namespace vfmm {

namespace {

constexpr double kInv2Pi = 0.15915494309189533576888376337251436;

constexpr int kDirectWaves = 16;  // waves per workgroup, each a share of the sources
constexpr int kDirectT = 16;      // targets per workgroup; 4 lanes per target

// 16 targets per workgroup: lane = target (lane % 16) + 16 x sub-stream; wave w
// takes the 64-source chunks w, w + 16, ..., sub-stream s every 4th source of
// a chunk.  The 4 x 16 partial sums of a target are added in a fixed order
// (shuffles, then waves in order through LDS): deterministic.  The FP64 pair
// term is a long dependent chain (exp, division), so the parallelism is spread
// over 4 lanes per target to keep several waves on every SIMD.
__global__ void __launch_bounds__(64 * kDirectWaves) k_direct(
    const double* __restrict__ x, const double* __restrict__ y, const double* __restrict__ g,
    int64_t n, double kexp, const int64_t* __restrict__ targets, const double* __restrict__ xt,
    const double* __restrict__ yt, int64_t nt, double* __restrict__ u, double* __restrict__ v) {
  __shared__ double part[2][kDirectWaves][kDirectT];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tl = lane & (kDirectT - 1), sub = lane / kDirectT;
  const int64_t t = blockIdx.x * int64_t(kDirectT) + tl;
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
  for (int64_t base = int64_t(wv) * 64; base < n; base += 64LL * kDirectWaves) {
    const int64_t end = base + 64 < n ? base + 64 : n;
    for (int64_t j = base + sub; j < end; j += 64 / kDirectT) {
      const double dx = xi - x[j];
      const double dy = yi - y[j];
      const double r2 = dx * dx + dy * dy;
      const double f = r2 > 0.0 ? g[j] * (-expm1(r2 * kexp) / r2) : 0.0;
      au -= f * dy;
      av += f * dx;
    }
  }
  // sub-streams of a target: lanes tl, tl + 16, tl + 32, tl + 48
  for (int o = kDirectT; o < 64; o <<= 1) {
    au += __shfl_xor(au, o, 64);
    av += __shfl_xor(av, o, 64);
  }
  if (sub == 0) {
    part[0][wv][tl] = au;
    part[1][wv][tl] = av;
  }
  __syncthreads();
  if (wv != 0 || sub != 0) return;
  double su = 0.0, sv = 0.0;
#pragma unroll
  for (int w = 0; w < kDirectWaves; ++w) {
    su += part[0][w][tl];
    sv += part[1][w][tl];
  }
  if (valid) {
    u[t] = in_range ? su * kInv2Pi : __builtin_nan("");
    v[t] = in_range ? sv * kInv2Pi : __builtin_nan("");
  }
}

// Maximum that keeps a NaN: fmax would return the other argument and drop it,
// so a NaN velocity would vanish from the error instead of poisoning it.
__device__ __forceinline__ double max_nan(double a, double b) {
  return (a > b || a != a) ? a : b;
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
    mx = max_nan(mx, d);
    ss += d * d;
    mr = max_nan(mr, hypot(ur[i], vr[i]));
  }
  s[0][threadIdx.x] = mx; s[1][threadIdx.x] = ss; s[2][threadIdx.x] = mr;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (int(threadIdx.x) < st) {
      s[0][threadIdx.x] = max_nan(s[0][threadIdx.x], s[0][threadIdx.x + st]);
      s[1][threadIdx.x] += s[1][threadIdx.x + st];
      s[2][threadIdx.x] = max_nan(s[2][threadIdx.x], s[2][threadIdx.x + st]);
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
    mx = max_nan(mx, part[3 * b]);
    ss += part[3 * b + 1];
    mr = max_nan(mr, part[3 * b + 2]);
  }
  s[0][threadIdx.x] = mx; s[1][threadIdx.x] = ss; s[2][threadIdx.x] = mr;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (int(threadIdx.x) < st) {
      s[0][threadIdx.x] = max_nan(s[0][threadIdx.x], s[0][threadIdx.x + st]);
      s[1][threadIdx.x] += s[1][threadIdx.x + st];
      s[2][threadIdx.x] = max_nan(s[2][threadIdx.x], s[2][threadIdx.x + st]);
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

__global__ void k_clear_counter(unsigned long long* c) {
  if (threadIdx.x == 0) c[0] = 0ull;
}

// One atomic per wave: the wave's count of NaN / infinite values.
__global__ void __launch_bounds__(256) k_count_nonfinite(const double* __restrict__ a, int64_t n,
                                                         int64_t stride,
                                                         unsigned long long* __restrict__ c) {
  unsigned long long cnt = 0;
  for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x)
    cnt += __builtin_isfinite(a[i * stride]) ? 0 : 1;
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(c, cnt);
}

}  // namespace

hipError_t launch_clear_counter(unsigned long long* counter, hipStream_t st) {
  hipLaunchKernelGGL(k_clear_counter, dim3(1), dim3(64), 0, st, counter);
  return hipGetLastError();
}

hipError_t launch_count_nonfinite(const double* a, int64_t n, int64_t stride,
                                  unsigned long long* counter, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t nb = (n + 255) / 256;
  if (nb > kReduceBlocks) nb = kReduceBlocks;
  hipLaunchKernelGGL(k_count_nonfinite, dim3(unsigned(nb)), dim3(256), 0, st, a, n, stride,
                     counter);
  return hipGetLastError();
}

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
  hipLaunchKernelGGL(k_direct, dim3(unsigned((nt + kDirectT - 1) / kDirectT)),
                     dim3(64 * kDirectWaves), 0, st, x, y, g, n, kexp, targets, xt, yt, nt, u, v);
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

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device

// Address of this device's copy of `scratch` (looked up on the first call
// made with the device current).
hipError_t scratch_address(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<double*>(g_scratch_ptr[dev]);
  return hipSuccess;
}

}  // namespace

}  // namespace vfmm

extern "C" vfmm_status_t vfmm_error_metrics_noalloc(const double* u, const double* v,
                                                    const double* ur, const double* vr, int64_t n,
                                                    double* out, void* stream) {
  using namespace vfmm;
  // the reduction writes at most kReduceBlocks partial triples, whatever n is
  static_assert(sizeof(scratch) >= size_t(kReduceBlocks) * 3 * sizeof(double),
                "scratch holds the partial sums of every block");
  if (!u || !v || !ur || !vr || !out) {
    set_last_error("vfmm_error_metrics_noalloc: null pointer");
    return VFMM_ERR_INVALID_ARG;
  }
  if (n < 1) {
    set_last_error("vfmm_error_metrics_noalloc: n must be >= 1");
    return VFMM_ERR_INVALID_ARG;
  }
  double* part = nullptr;
  hipError_t e = scratch_address(&part);
  if (e == hipSuccess)
    e = launch_error_metrics(u, v, ur, vr, n, part, out, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) {
    char buf[256];
    snprintf(buf, sizeof(buf), "vfmm_error_metrics_noalloc: %s", hipGetErrorString(e));
    set_last_error(buf);
    return hip_status(e);
  }
  return VFMM_OK;
}
