// (p, levels) selector: particle statistics, features, and the 10 -> 64 -> 64 -> 1
// GELU network with its forward, backward and Adam kernels.
//
// The paper measures how the FMM error depends on N, the levels and the
// expansion order p (Sections 4-5, Figs. 13-23).  Here a small network learns
// log10 of the maximum error (normalised by the maximum velocity, Section 5.1)
// from runs of this library, so that the cheapest (p, levels) meeting a
// tolerance can be chosen before running the method.
//
// Parameters (4929 float32 master values): W1[10][64], b1[64], W2[64][64],
// b2[64], W3[64], b3.  Forward: z1 = x W1 + b1, a1 = gelu(z1), z2 = a1 W2 + b2,
// a2 = gelu(z2), y = a2 . W3 + b3, with the tanh form of GELU.  In BF16 mode the
// weights, inputs and activations are rounded to bfloat16 (RNE) and every
// product is accumulated in float32 (what a bf16 matrix instruction computes);
// gradients, master weights and Adam moments stay float32.
//
// One block of 256 threads handles 32 samples with all weights and
// activations in LDS.  Gradients of each block go to a partial buffer that one
// reduction kernel sums in a fixed order, so training is deterministic.
#include "vfmm_device.hpp"

namespace vfmm {

namespace {

constexpr int kIn = 10, kHid = 64;
constexpr int oW1 = 0, oB1 = oW1 + kIn * kHid, oW2 = oB1 + kHid, oB2 = oW2 + kHid * kHid,
              oW3 = oB2 + kHid, oB3 = oW3 + kHid, kParams = oB3 + 1;
constexpr int kSB = 32;  // samples per block

__device__ __forceinline__ float rnd(float v, bool bf) {
  return bf ? float(__bf16(v)) : v;
}

__device__ __forceinline__ float gelu(float z) {
  const float c = 0.7978845608028654f;
  return 0.5f * z * (1.0f + tanhf(c * (z + 0.044715f * z * z * z)));
}

__device__ __forceinline__ float gelu_grad(float z) {
  const float c = 0.7978845608028654f;
  const float t = tanhf(c * (z + 0.044715f * z * z * z));
  return 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * c * (1.0f + 3.0f * 0.044715f * z * z);
}

template <bool TRAIN, bool BF>
__global__ void __launch_bounds__(256) k_mlp(const float* __restrict__ W, const float* __restrict__ X,
                                             const float* __restrict__ T, int64_t B,
                                             float* __restrict__ Y, float* __restrict__ part,
                                             float* __restrict__ lpart) {
  __shared__ float w[kParams];
  __shared__ float xs[kSB][kIn];
  __shared__ float z1[kSB][kHid], a1[kSB][kHid], z2[kSB][kHid], a2[kSB][kHid];
  __shared__ float dy[kSB];
  const int tid = threadIdx.x;
  const int64_t s0 = int64_t(blockIdx.x) * kSB;
  const int nb = int(B - s0 < kSB ? B - s0 : kSB);
  for (int i = tid; i < kParams; i += 256) w[i] = rnd(W[i], BF);
  for (int i = tid; i < kSB * kIn; i += 256) {
    const int s = i / kIn, k = i % kIn;
    xs[s][k] = s < nb ? rnd(X[(s0 + s) * kIn + k], BF) : 0.f;
  }
  __syncthreads();
  for (int i = tid; i < kSB * kHid; i += 256) {
    const int s = i / kHid, j = i % kHid;
    float z = w[oB1 + j];
    for (int k = 0; k < kIn; ++k) z += xs[s][k] * w[oW1 + k * kHid + j];
    z1[s][j] = z;
    a1[s][j] = rnd(gelu(z), BF);
  }
  __syncthreads();
  for (int i = tid; i < kSB * kHid; i += 256) {
    const int s = i / kHid, j = i % kHid;
    float z = w[oB2 + j];
    for (int k = 0; k < kHid; ++k) z += a1[s][k] * w[oW2 + k * kHid + j];
    z2[s][j] = z;
    a2[s][j] = rnd(gelu(z), BF);
  }
  __syncthreads();
  if (tid < kSB) {
    float yv = w[oB3];
    for (int k = 0; k < kHid; ++k) yv += a2[tid][k] * w[oW3 + k];
    if (tid < nb) Y[s0 + tid] = yv;
    if (TRAIN) {
      const float r = tid < nb ? yv - T[s0 + tid] : 0.f;
      dy[tid] = 2.0f * r / float(B);
      float l2 = r * r;
      for (int o = 16; o > 0; o >>= 1) l2 += __shfl_xor(l2, o, 32);
      if (tid == 0) lpart[blockIdx.x] = l2;
    }
  }
  if (!TRAIN) return;
  __syncthreads();
  float* g = part + int64_t(blockIdx.x) * kParams;
  // output layer and dz2 = dy W3 gelu'(z2)
  if (tid < kHid) {
    float acc = 0.f;
    for (int s = 0; s < kSB; ++s) acc += a2[s][tid] * dy[s];
    g[oW3 + tid] = acc;
  }
  if (tid == kHid) {
    float acc = 0.f;
    for (int s = 0; s < kSB; ++s) acc += dy[s];
    g[oB3] = acc;
  }
  __syncthreads();
  for (int i = tid; i < kSB * kHid; i += 256) {
    const int s = i / kHid, j = i % kHid;
    z2[s][j] = dy[s] * w[oW3 + j] * gelu_grad(z2[s][j]);  // now dz2
  }
  __syncthreads();
  // W2, b2 gradients and dz1 = (dz2 W2^T) gelu'(z1)
  for (int i = tid; i < kHid * kHid; i += 256) {
    const int k = i / kHid, j = i % kHid;
    float acc = 0.f;
    for (int s = 0; s < kSB; ++s) acc += a1[s][k] * z2[s][j];
    g[oW2 + i] = acc;
  }
  if (tid < kHid) {
    float acc = 0.f;
    for (int s = 0; s < kSB; ++s) acc += z2[s][tid];
    g[oB2 + tid] = acc;
  }
  for (int i = tid; i < kSB * kHid; i += 256) {
    const int s = i / kHid, k = i % kHid;
    float acc = 0.f;
    for (int j = 0; j < kHid; ++j) acc += z2[s][j] * w[oW2 + k * kHid + j];
    z1[s][k] = acc * gelu_grad(z1[s][k]);  // now dz1
  }
  __syncthreads();
  for (int i = tid; i < kIn * kHid; i += 256) {
    const int k = i / kHid, j = i % kHid;
    float acc = 0.f;
    for (int s = 0; s < kSB; ++s) acc += xs[s][k] * z1[s][j];
    g[oW1 + i] = acc;
  }
  if (tid < kHid) {
    float acc = 0.f;
    for (int s = 0; s < kSB; ++s) acc += z1[s][tid];
    g[oB1 + tid] = acc;
  }
}

__global__ void __launch_bounds__(256) k_sum_partials(const float* __restrict__ part, int nblk,
                                                      const float* __restrict__ lpart, int64_t B,
                                                      float* __restrict__ grad,
                                                      float* __restrict__ loss) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < kParams) {
    float acc = 0.f;
    for (int b = 0; b < nblk; ++b) acc += part[int64_t(b) * kParams + i];
    grad[i] = acc;
  }
  if (i == 0 && loss) {
    double acc = 0.0;
    for (int b = 0; b < nblk; ++b) acc += lpart[b];
    *loss = float(acc / double(B));
  }
}

__global__ void __launch_bounds__(256) k_adam(float* __restrict__ W, float* __restrict__ m,
                                              float* __restrict__ v, const float* __restrict__ g,
                                              float lr, float b1, float b2, float eps, float c1,
                                              float c2) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= kParams) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  W[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Particle statistics for the features: sum x, sum x^2, sum y, sum y^2,
// sum G, sum G^2, sum |G|, max |G|, min x, max x, min y, max y.
__global__ void __launch_bounds__(256) k_stats_partial(const double* __restrict__ x,
                                                       const double* __restrict__ y,
                                                       const double* __restrict__ g, int64_t n,
                                                       double* __restrict__ part) {
  __shared__ double sh[12][256];
  double a[12] = {0, 0, 0, 0, 0, 0, 0, 0, INFINITY, -INFINITY, INFINITY, -INFINITY};
  for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) {
    const double xi = x[i], yi = y[i], gi = g[i];
    a[0] += xi; a[1] += xi * xi; a[2] += yi; a[3] += yi * yi;
    a[4] += gi; a[5] += gi * gi; a[6] += fabs(gi); a[7] = fmax(a[7], fabs(gi));
    a[8] = fmin(a[8], xi); a[9] = fmax(a[9], xi); a[10] = fmin(a[10], yi); a[11] = fmax(a[11], yi);
  }
  for (int k = 0; k < 12; ++k) sh[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (int(threadIdx.x) < st) {
      const int o = threadIdx.x + st;
      for (int k = 0; k < 7; ++k) sh[k][threadIdx.x] += sh[k][o];
      sh[7][threadIdx.x] = fmax(sh[7][threadIdx.x], sh[7][o]);
      sh[8][threadIdx.x] = fmin(sh[8][threadIdx.x], sh[8][o]);
      sh[9][threadIdx.x] = fmax(sh[9][threadIdx.x], sh[9][o]);
      sh[10][threadIdx.x] = fmin(sh[10][threadIdx.x], sh[10][o]);
      sh[11][threadIdx.x] = fmax(sh[11][threadIdx.x], sh[11][o]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 12) part[blockIdx.x * 12 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void __launch_bounds__(64) k_stats_final(const double* __restrict__ part, int nb,
                                                    double* __restrict__ out) {
  const int k = threadIdx.x;
  if (k >= 12) return;
  double a = k < 7 ? 0.0 : (k == 7 || k == 9 || k == 11 ? -INFINITY : INFINITY);
  for (int b = 0; b < nb; ++b) {
    const double v = part[b * 12 + k];
    if (k < 7) a += v;
    else if (k == 7 || k == 9 || k == 11) a = fmax(a, v);
    else a = fmin(a, v);
  }
  out[k] = a;
}

// Leaf occupancy at level `lev` for the root square given in root[0..2].
__global__ void __launch_bounds__(256) k_leaf_hist(const double* __restrict__ x,
                                                   const double* __restrict__ y, int64_t n,
                                                   double x0, double y0, double S, int lev,
                                                   uint32_t* __restrict__ counts) {
#pragma clang fp contract(off)
  const int64_t i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= n) return;
  const int m = 1 << lev;
  const double fx = floor(((x[i] - x0) / S) * double(m));
  const double fy = floor(((y[i] - y0) / S) * double(m));
  const int ix = !(fx >= 0.0) ? 0 : (fx > double(m - 1) ? m - 1 : int(fx));
  const int iy = !(fy >= 0.0) ? 0 : (fy > double(m - 1) ? m - 1 : int(fy));
  atomicAdd(&counts[int64_t(iy) * m + ix], 1u);
}

}  // namespace

int mlp_param_count() { return kParams; }
int mlp_blocks(int64_t B) { return int((B + kSB - 1) / kSB); }

hipError_t launch_mlp_forward(const float* W, bool bf16, const float* X, int64_t B, float* Y,
                              hipStream_t st) {
  const unsigned nb = unsigned(mlp_blocks(B));
  if (bf16)
    hipLaunchKernelGGL((k_mlp<false, true>), dim3(nb), dim3(256), 0, st, W, X, nullptr, B, Y, nullptr, nullptr);
  else
    hipLaunchKernelGGL((k_mlp<false, false>), dim3(nb), dim3(256), 0, st, W, X, nullptr, B, Y, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_mlp_gradient(const float* W, bool bf16, const float* X, const float* T,
                               int64_t B, float* Y, float* part, float* lpart, float* grad,
                               float* loss, hipStream_t st) {
  const int nb = mlp_blocks(B);
  if (bf16)
    hipLaunchKernelGGL((k_mlp<true, true>), dim3(nb), dim3(256), 0, st, W, X, T, B, Y, part, lpart);
  else
    hipLaunchKernelGGL((k_mlp<true, false>), dim3(nb), dim3(256), 0, st, W, X, T, B, Y, part, lpart);
  hipLaunchKernelGGL(k_sum_partials, dim3((kParams + 255) / 256), dim3(256), 0, st, part, nb, lpart,
                     B, grad, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* W, float* m, float* v, const float* g, int step, float lr,
                       hipStream_t st) {
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = float(1.0 - pow(double(b1), step)), c2 = float(1.0 - pow(double(b2), step));
  hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, st, W, m, v, g, lr, b1, b2,
                     eps, c1, c2);
  return hipGetLastError();
}

hipError_t launch_stats(const double* x, const double* y, const double* g, int64_t n,
                        double* part, double* out, hipStream_t st) {
  int nb = int((n + 255) / 256);
  if (nb > kReduceBlocks) nb = kReduceBlocks;
  hipLaunchKernelGGL(k_stats_partial, dim3(nb), dim3(256), 0, st, x, y, g, n, part);
  hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(64), 0, st, part, nb, out);
  return hipGetLastError();
}

hipError_t launch_leaf_hist(const double* x, const double* y, int64_t n, const double* root3,
                            int lev, uint32_t* counts, hipStream_t st) {
  hipLaunchKernelGGL(k_leaf_hist, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, x, y, n,
                     root3[0], root3[1], root3[2], lev, counts);
  return hipGetLastError();
}

}  // namespace vfmm
