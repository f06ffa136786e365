// Expansion kernels: translation-operator tables, P2M, M2M and the fused
// L2L + M2L downward step (Cruz & Barba 2008, Sections 3.2-3.3).
//
// Scaled coefficients (see vfmm_internal.hpp) make every operator independent
// of the level, so the tables are built once per expansion order p:
//   M2M (Section 3.3.2):  A_c[n][k] = C(n,k) d_c^(n-k) 2^-n,            k <= n
//   L2L (Section 3.3.3):  B_c[n][k] = C(k,n) d_c^(k-n) 2^-(k+1),        k >= n
//   M2L (eq. 22):         T_t[n][k] = (-1)^n C(n+k,k) t^-(n+k+1)
// with the child offset d_c = ((cx&1) - 1/2) + j((cy&1) - 1/2) in units of the
// child side and the interaction offset t in units of the box side.
#include "vfmm_device.hpp"

namespace vfmm {

namespace {

__device__ double binom(int n, int k) {
  if (k < 0 || k > n) return 0.0;
  if (k > n - k) k = n - k;
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * double(n - k + i) / double(i);
  return r;
}

// z^m by binary exponentiation (m >= 0).
__device__ double2 cpow(double2 z, int m) {
  double2 r = make_double2(1.0, 0.0);
  double2 b = z;
  while (m > 0) {
    if (m & 1) r = cmul(r, b);
    b = cmul(b, b);
    m >>= 1;
  }
  return r;
}

__global__ void __launch_bounds__(256) k_build_ops(int p, double2* __restrict__ m2m64,
                                                   double2* __restrict__ l2l64,
                                                   double2* __restrict__ m2l64,
                                                   float2* __restrict__ m2m32,
                                                   float2* __restrict__ l2l32,
                                                   float2* __restrict__ m2l32) {
  const int pp = p * p;
  const int total = (4 + 4 + kM2LOffsets) * pp;
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int tab = e / pp, nk = e % pp, n = nk / p, k = nk % p;
  double2 val = make_double2(0.0, 0.0);
  if (tab < 8) {
    const int c = tab & 3;
    const double2 d = make_double2(double(c & 1) - 0.5, double(c >> 1) - 0.5);
    if (tab < 4) {  // M2M
      if (k <= n) {
        double2 dp = cpow(d, n - k);
        double s = binom(n, k) * ldexp(1.0, -n);
        val = make_double2(s * dp.x, s * dp.y);
      }
      m2m64[c * pp + nk] = val;
      m2m32[c * pp + nk] = make_float2(float(val.x), float(val.y));
    } else {  // L2L
      if (k >= n) {
        double2 dp = cpow(d, k - n);
        double s = binom(k, n) * ldexp(1.0, -(k + 1));
        val = make_double2(s * dp.x, s * dp.y);
      }
      l2l64[c * pp + nk] = val;
      l2l32[c * pp + nk] = make_float2(float(val.x), float(val.y));
    }
  } else {  // M2L
    const int o = tab - 8;
    const int ox = o % 7 - 3, oy = o / 7 - 3;
    if (ox < -1 || ox > 1 || oy < -1 || oy > 1) {
      // t^-(m) = conj(t)^m / |t|^(2m)
      const double2 tc = make_double2(double(ox), -double(oy));
      const int m = n + k + 1;
      double2 num = cpow(tc, m);
      double den = pow(double(ox * ox + oy * oy), -double(m));
      double s = binom(n + k, k) * den * ((n & 1) ? -1.0 : 1.0);
      val = make_double2(s * num.x, s * num.y);
    }
    m2l64[o * pp + nk] = val;
    m2l32[o * pp + nk] = make_float2(float(val.x), float(val.y));
  }
}

// P2M at the leaves: one wave per leaf, lanes stride over the leaf's particles,
// coefficients reduced across lanes through LDS.
template <typename R, int PMAX>
__global__ void __launch_bounds__(64) k_p2m(const typename Types<R>::Part* __restrict__ part,
                                            const int32_t* __restrict__ leaf_start,
                                            int64_t nleaves, const double* __restrict__ root,
                                            int p, typename Types<R>::C* __restrict__ me) {
  using C = typename Types<R>::C;
  __shared__ R red[2 * PMAX][65];
  const int64_t leaf = blockIdx.x;
  if (leaf >= nleaves) return;
  const int lane = threadIdx.x;
  const int32_t s = leaf_start[leaf], e = leaf_start[leaf + 1];
  const R inv_w = R(1.0 / root[3]);
  C acc[PMAX];
#pragma unroll
  for (int k = 0; k < PMAX; ++k) acc[k] = cmake<C>(R(0), R(0));
  for (int32_t i = s + lane; i < e; i += 64) {
    const auto q = part[i];
    const C z = cmake<C>(q.x * inv_w, q.y * inv_w);
    C pw = cmake<C>(q.g, R(0));
#pragma unroll
    for (int k = 0; k < PMAX; ++k) {
      if (k < p) {
        acc[k].x += pw.x;
        acc[k].y += pw.y;
        pw = cmul(pw, z);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < PMAX; ++k) {
    red[2 * k][lane] = acc[k].x;
    red[2 * k + 1][lane] = acc[k].y;
  }
  __syncthreads();
  for (int c = lane; c < 2 * p; c += 64) {
    R t = R(0);
    for (int l = 0; l < 64; ++l) t += red[c][l];
    R* out = reinterpret_cast<R*>(me + leaf * p);
    out[c] = t;
  }
}

// M2M from level l+1 to level l: one thread per (parent box, n).
template <typename R>
__global__ void __launch_bounds__(256) k_m2m(const typename Types<R>::C* __restrict__ child,
                                             typename Types<R>::C* __restrict__ parent, int lev,
                                             int p, const typename Types<R>::C* __restrict__ A) {
  using C = typename Types<R>::C;
  const int64_t t = blockIdx.x * 256LL + threadIdx.x;
  const int64_t nb = int64_t(1) << (2 * lev);
  if (t >= nb * p) return;
  const int64_t box = t / p;
  const int n = int(t % p);
  const int mp = 1 << lev, mc = 2 * mp;
  const int px = int(box & (mp - 1)), py = int(box >> lev);
  C acc = cmake<C>(R(0), R(0));
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int64_t cb = int64_t(2 * py + (c >> 1)) * mc + (2 * px + (c & 1));
    const C* m = child + cb * p;
    const C* a = A + (c * p + n) * p;
    for (int k = 0; k <= n; ++k) cfma(acc, a[k], m[k]);
  }
  parent[box * p + n] = acc;
}

// Downward step at level l: LE = L2L(parent LE) (for l > 2) + sum of M2L over
// the interaction list.  One thread per (box, n).
template <typename R>
__global__ void __launch_bounds__(256) k_m2l_l2l(const typename Types<R>::C* __restrict__ me,
                                                 const typename Types<R>::C* __restrict__ le_par,
                                                 typename Types<R>::C* __restrict__ le, int lev,
                                                 int p, const typename Types<R>::C* __restrict__ T,
                                                 const typename Types<R>::C* __restrict__ B) {
  using C = typename Types<R>::C;
  const int64_t t = blockIdx.x * 256LL + threadIdx.x;
  const int64_t nb = int64_t(1) << (2 * lev);
  if (t >= nb * p) return;
  const int64_t box = t / p;
  const int n = int(t % p);
  const int m = 1 << lev;
  const int bx = int(box & (m - 1)), by = int(box >> lev);
  C acc = cmake<C>(R(0), R(0));
  if (lev > 2) {
    const int64_t pb = int64_t(by >> 1) * (m >> 1) + (bx >> 1);
    const int c = ((by & 1) << 1) | (bx & 1);
    const C* lp = le_par + pb * p;
    const C* b = B + (c * p + n) * p;
    for (int k = n; k < p; ++k) cfma(acc, b[k], lp[k]);
  }
  const int px = bx >> 1, py = by >> 1;
  const int x0 = max(2 * px - 2, 0), x1 = min(2 * px + 3, m - 1);
  const int y0 = max(2 * py - 2, 0), y1 = min(2 * py + 3, m - 1);
  for (int sy = y0; sy <= y1; ++sy) {
    for (int sx = x0; sx <= x1; ++sx) {
      const int ox = bx - sx, oy = by - sy;
      if (ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1) continue;
      const C* ms = me + (int64_t(sy) * m + sx) * p;
      const C* tr = T + (m2l_index(ox, oy) * p + n) * p;
      for (int k = 0; k < p; ++k) cfma(acc, tr[k], ms[k]);
    }
  }
  le[box * p + n] = acc;
}

// float64 coefficients rounded to float32 (count complex values).
__global__ void __launch_bounds__(256) k_narrow(const double2* __restrict__ a, int64_t count,
                                                float2* __restrict__ b) {
  const int64_t i = blockIdx.x * 256LL + threadIdx.x;
  if (i < count) b[i] = make_float2(float(a[i].x), float(a[i].y));
}

// float64 L2L at level l (l > 2 shifts the parent's float64 LE): one thread per
// (box, n); the level's own M2L sum comes in float32 from the matrix cores.
__global__ void __launch_bounds__(256) k_l2l64_add32(const float2* __restrict__ m2l,
                                                     const double2* __restrict__ le_par,
                                                     double2* __restrict__ le, int lev, int p,
                                                     const double2* __restrict__ B) {
  const int64_t t = blockIdx.x * 256LL + threadIdx.x;
  const int64_t nb = int64_t(1) << (2 * lev);
  if (t >= nb * p) return;
  const int64_t box = t / p;
  const int n = int(t % p);
  const float2 own = m2l[box * p + n];
  double2 acc = make_double2(double(own.x), double(own.y));
  if (lev > 2) {
    const int m = 1 << lev;
    const int bx = int(box & (m - 1)), by = int(box >> lev);
    const int64_t pb = int64_t(by >> 1) * (m >> 1) + (bx >> 1);
    const int c = ((by & 1) << 1) | (bx & 1);
    const double2* lp = le_par + pb * p;
    const double2* b = B + (c * p + n) * p;
    for (int k = n; k < p; ++k) cfma(acc, b[k], lp[k]);
  }
  le[box * p + n] = acc;
}

template <typename R, int PMAX>
void launch_p2m_t(const TreeDev& t, int levels, int p, hipStream_t st) {
  using C = typename Types<R>::C;
  const int64_t nl = int64_t(1) << (2 * levels);
  C* me = reinterpret_cast<C*>(t.me) + level_offset(levels) * p;
  const auto* part = reinterpret_cast<const typename Types<R>::Part*>(
      sizeof(R) == 8 ? static_cast<const void*>(t.part64) : static_cast<const void*>(t.part32));
  hipLaunchKernelGGL((k_p2m<R, PMAX>), dim3(unsigned(nl)), dim3(64), 0, st, part, t.leaf_start, nl,
                     t.root, p, me);
}

template <typename R>
hipError_t p2m_t(const TreeDev& t, int levels, int p, hipStream_t st) {
  if (p <= 8) launch_p2m_t<R, 8>(t, levels, p, st);
  else if (p <= 16) launch_p2m_t<R, 16>(t, levels, p, st);
  else if (p <= 24) launch_p2m_t<R, 24>(t, levels, p, st);
  else if (p <= 32) launch_p2m_t<R, 32>(t, levels, p, st);
  else launch_p2m_t<R, 40>(t, levels, p, st);
  return hipGetLastError();
}

template <typename R>
hipError_t m2m_t(const TreeDev& t, int levels, int p, hipStream_t st) {
  using C = typename Types<R>::C;
  const OpsLayout ol = ops_layout(p);
  const C* A = reinterpret_cast<const C*>(static_cast<const char*>(t.ops) +
                                          (sizeof(R) == 8 ? ol.m2m64 : ol.m2m32));
  C* me = reinterpret_cast<C*>(t.me);
  for (int l = levels - 1; l >= 2; --l) {
    const int64_t work = (int64_t(1) << (2 * l)) * p;
    hipLaunchKernelGGL(k_m2m<R>, dim3(unsigned((work + 255) / 256)), dim3(256), 0, st,
                       me + level_offset(l + 1) * p, me + level_offset(l) * p, l, p, A);
  }
  return hipGetLastError();
}

template <typename R>
hipError_t downward_t(const TreeDev& t, int levels, int p, hipStream_t st) {
  using C = typename Types<R>::C;
  const OpsLayout ol = ops_layout(p);
  const char* ops = static_cast<const char*>(t.ops);
  const C* T = reinterpret_cast<const C*>(ops + (sizeof(R) == 8 ? ol.m2l64 : ol.m2l32));
  const C* B = reinterpret_cast<const C*>(ops + (sizeof(R) == 8 ? ol.l2l64 : ol.l2l32));
  const C* me = reinterpret_cast<const C*>(t.me);
  C* le = reinterpret_cast<C*>(t.le);
  for (int l = 2; l <= levels; ++l) {
    const int64_t work = (int64_t(1) << (2 * l)) * p;
    const C* lpar = l > 2 ? le + level_offset(l - 1) * p : nullptr;
    hipLaunchKernelGGL(k_m2l_l2l<R>, dim3(unsigned((work + 255) / 256)), dim3(256), 0, st,
                       me + level_offset(l) * p, lpar, le + level_offset(l) * p, l, p, T, B);
  }
  return hipGetLastError();
}

}  // namespace

size_t ops_bytes(int p) { return ops_layout(p).total; }

hipError_t launch_build_ops(const TreeDev& t, int p, int prec, hipStream_t st) {
  (void)prec;
  const OpsLayout ol = ops_layout(p);
  char* ops = static_cast<char*>(t.ops);
  const int total = (4 + 4 + kM2LOffsets) * p * p;
  hipLaunchKernelGGL(k_build_ops, dim3((total + 255) / 256), dim3(256), 0, st, p,
                     reinterpret_cast<double2*>(ops + ol.m2m64),
                     reinterpret_cast<double2*>(ops + ol.l2l64),
                     reinterpret_cast<double2*>(ops + ol.m2l64),
                     reinterpret_cast<float2*>(ops + ol.m2m32),
                     reinterpret_cast<float2*>(ops + ol.l2l32),
                     reinterpret_cast<float2*>(ops + ol.m2l32));
  return hipGetLastError();
}

hipError_t launch_p2m(const TreeDev& t, int levels, int p, int prec, hipStream_t st) {
  return prec == kFP64 ? p2m_t<double>(t, levels, p, st) : p2m_t<float>(t, levels, p, st);
}

hipError_t launch_m2m(const TreeDev& t, int levels, int p, int prec, hipStream_t st) {
  return prec == kFP64 ? m2m_t<double>(t, levels, p, st) : m2m_t<float>(t, levels, p, st);
}

hipError_t launch_downward_shift64(const TreeDev& t, int levels, int p, int prec,
                                   hipStream_t st) {
  if (levels < 2) return hipSuccess;
  const int64_t count = n_boxes_2_to(levels) * p;
  hipLaunchKernelGGL(k_narrow, dim3(unsigned((count + 255) / 256)), dim3(256), 0, st,
                     static_cast<const double2*>(t.me), count, static_cast<float2*>(t.me32));
  TreeDev t32 = t;
  t32.me = t.me32;
  t32.le = t.le32;
  hipError_t e = launch_downward_mfma(t32, levels, p, prec, st, false);
  if (e != hipSuccess) return e;
  const OpsLayout ol = ops_layout(p);
  const double2* B = reinterpret_cast<const double2*>(static_cast<const char*>(t.ops) + ol.l2l64);
  const float2* m2l = static_cast<const float2*>(t.le32);
  double2* le = static_cast<double2*>(t.le);
  for (int l = 2; l <= levels; ++l) {
    const int64_t work = (int64_t(1) << (2 * l)) * p;
    hipLaunchKernelGGL(k_l2l64_add32, dim3(unsigned((work + 255) / 256)), dim3(256), 0, st,
                       m2l + level_offset(l) * p, l > 2 ? le + level_offset(l - 1) * p : nullptr,
                       le + level_offset(l) * p, l, p, B);
  }
  // every level rounded back (the leaves of an adaptive tree lie at any level)
  hipLaunchKernelGGL(k_narrow, dim3(unsigned((count + 255) / 256)), dim3(256), 0, st, le, count,
                     static_cast<float2*>(t.le32));
  return hipGetLastError();
}

hipError_t launch_downward(const TreeDev& t, int levels, int p, int prec, hipStream_t st) {
  return prec == kFP64 ? downward_t<double>(t, levels, p, st)
                       : downward_t<float>(t, levels, p, st);
}

}  // namespace vfmm
