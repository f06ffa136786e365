// C ABI of the selector network and of the (p, levels) choice.
//
// The choice follows the experiment design of the paper (Section 5: the error
// of an FMM evaluation as a function of N, the number of levels l and the
// truncation p): among candidate (p, L), take the cheapest whose predicted
// log10 max error (normalised by the maximum velocity, Section 5.1), plus a
// safety margin, is within the tolerance; when none qualifies, take the
// conservative choice p = 20 and the deepest level whose leaf side is at
// least 8 sigma (keeping the kernel-substitution error of Section 4.1
// negligible).
#include <algorithm>
#include <cmath>
#include <new>
#include <cstdarg>
#include <cstdio>
#include <vector>

#include "../../include/vfmm.h"
#include "vfmm_device.hpp"

namespace vfmm {
int mlp_param_count();
int mlp_blocks(int64_t B);
hipError_t launch_mlp_forward(const float* W, bool bf16, const float* X, int64_t B, float* Y,
                              hipStream_t st);
hipError_t launch_mlp_gradient(const float* W, bool bf16, const float* X, const float* T,
                               int64_t B, float* Y, float* part, float* lpart, float* grad,
                               float* loss, hipStream_t st);
hipError_t launch_adam(float* W, float* m, float* v, const float* g, int step, float lr,
                       hipStream_t st);
hipError_t launch_stats(const double* x, const double* y, const double* g, int64_t n,
                        double* part, double* out, hipStream_t st);
hipError_t launch_leaf_hist(const double* x, const double* y, int64_t n, const double* root3,
                            int lev, uint32_t* counts, hipStream_t st);
}  // namespace vfmm

using namespace vfmm;

namespace {

vfmm_status_t sfail(vfmm_status_t s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
vfmm_status_t sfail(vfmm_status_t s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  set_last_error(buf);
  return s;
}

inline size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

// max(w_L, a): the distance below which every pair is summed with the
// regularised kernel, w_L the leaf side and a the near radius of the distance
// cut-off clamped to VFMM_NEAR_RINGS_MAX w_L (radius < 0: 6 sigma, the
// automatic radius of a float32 evaluation; 0: the paper's split).
double near_distance(double S, int levels, double sigma, double radius) {
  const double w = S / std::ldexp(1.0, levels);
  if (radius == 0.0) return w;
  const double a = radius < 0.0 ? 6.0 * sigma : radius;
  const double ac = std::fmin(a, VFMM_NEAR_RINGS_MAX * w);
  return std::fmax(w, ac);
}

constexpr int kHistMax = 10;   // finest level of the occupancy histogram
constexpr int kPMin = 4, kPMax = 20;

int hist_level(int64_t n) {
  int l = 2;
  while (l < kHistMax && (int64_t(1) << (2 * (l + 1))) <= 4 * n) ++l;
  return l;
}

// Near-radius options of the candidates: the paper's split, the automatic
// radius and the radius at which one pair's kernel difference equals tol.
constexpr int kNRadii = 3;

size_t select_scratch(int64_t n) {
  const int lh = hist_level(n);
  const int ncand = (kPMax - kPMin + 1) * (lh - 1) * kNRadii;
  return a256(size_t(kReduceBlocks) * 12 * 8) + a256(12 * 8) +
         a256((size_t(1) << (2 * lh)) * 4) + a256(size_t(ncand) * 10 * 4) + a256(size_t(ncand) * 4);
}

double root_side(const double* st) {
  const double ext = std::fmax(st[9] - st[8], st[11] - st[10]);
  return ext > 0.0 ? ext * (1.0 + 0x1p-20) : 1.0;
}

// pairs(L, d) = sum over leaves of n_b * (sum of n_s over the leaves at
// Chebyshev distance <= d): d = 1 is the 3 x 3 local list.
double near_pairs(const std::vector<double>& c, int lev, int d = 1) {
  const int m = 1 << lev;
  double s = 0.0;
  for (int iy = 0; iy < m; ++iy)
    for (int ix = 0; ix < m; ++ix) {
      const double nb = c[size_t(iy) * m + ix];
      if (nb == 0.0) continue;
      double src = 0.0;
      for (int dy = -d; dy <= d; ++dy)
        for (int dx = -d; dx <= d; ++dx) {
          const int jx = ix + dx, jy = iy + dy;
          if (jx >= 0 && jx < m && jy >= 0 && jy < m) src += c[size_t(jy) * m + jx];
        }
      s += nb * src;
    }
  return s;
}

}  // namespace

extern "C" {

size_t vfmm_mlp_scratch_bytes(int64_t batch) {
  if (batch < 1) batch = 1;
  const int nb = mlp_blocks(batch);
  return a256(size_t(nb) * mlp_param_count() * 4) + a256(size_t(nb) * 4) + a256(size_t(batch) * 4);
}

vfmm_status_t vfmm_mlp_forward(const float* params, int32_t bf16, const float* x, int64_t batch,
                               float* y, void* stream) {
  if (!params || !x || !y) return sfail(VFMM_ERR_INVALID_ARG, "null pointer");
  if (batch < 1 || batch > (int64_t(1) << 30)) return sfail(VFMM_ERR_INVALID_ARG, "bad batch");
  hipError_t e = launch_mlp_forward(params, bf16 != 0, x, batch, y, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? VFMM_OK : sfail(hip_status(e), "mlp forward: %s", hipGetErrorString(e));
}

vfmm_status_t vfmm_mlp_gradient(const float* params, int32_t bf16, const float* x,
                                const float* target, int64_t batch, float* grad, float* loss,
                                void* scratch, size_t scratch_bytes, void* stream) {
  if (!params || !x || !target || !grad || !scratch) return sfail(VFMM_ERR_INVALID_ARG, "null pointer");
  if (batch < 1 || batch > (int64_t(1) << 30)) return sfail(VFMM_ERR_INVALID_ARG, "bad batch");
  if (scratch_bytes < vfmm_mlp_scratch_bytes(batch))
    return sfail(VFMM_ERR_WORKSPACE, "scratch too small");
  const int nb = mlp_blocks(batch);
  char* s = static_cast<char*>(scratch);
  float* part = reinterpret_cast<float*>(s);
  float* lpart = reinterpret_cast<float*>(s + a256(size_t(nb) * mlp_param_count() * 4));
  float* yv = reinterpret_cast<float*>(s + a256(size_t(nb) * mlp_param_count() * 4) + a256(size_t(nb) * 4));
  hipError_t e = launch_mlp_gradient(params, bf16 != 0, x, target, batch, yv, part, lpart, grad,
                                     loss, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? VFMM_OK : sfail(hip_status(e), "mlp gradient: %s", hipGetErrorString(e));
}

vfmm_status_t vfmm_mlp_adam(float* params, float* m, float* v, const float* grad, int32_t step,
                            float lr, void* stream) {
  if (!params || !m || !v || !grad) return sfail(VFMM_ERR_INVALID_ARG, "null pointer");
  if (step < 1 || !(lr > 0.f)) return sfail(VFMM_ERR_INVALID_ARG, "step >= 1 and lr > 0 required");
  hipError_t e = launch_adam(params, m, v, grad, step, lr, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? VFMM_OK : sfail(hip_status(e), "adam: %s", hipGetErrorString(e));
}

size_t vfmm_select_scratch_bytes(int64_t n) { return select_scratch(n < 1 ? 1 : n); }

vfmm_status_t vfmm_particle_stats(const double* x, const double* y, const double* gamma, int64_t n,
                                  void* scratch, size_t scratch_bytes, double* stats,
                                  void* stream) {
  if (!x || !y || !gamma || !scratch || !stats) return sfail(VFMM_ERR_INVALID_ARG, "null pointer");
  if (n < 1) return sfail(VFMM_ERR_INVALID_ARG, "n must be >= 1");
  if (scratch_bytes < a256(size_t(kReduceBlocks) * 12 * 8) + a256(12 * 8))
    return sfail(VFMM_ERR_WORKSPACE, "scratch too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* s = static_cast<char*>(scratch);
  double* part = reinterpret_cast<double*>(s);
  double* out = reinterpret_cast<double*>(s + a256(size_t(kReduceBlocks) * 12 * 8));
  hipError_t e = launch_stats(x, y, gamma, n, part, out, st);
  if (e == hipSuccess) e = hipMemcpyAsync(stats, out, 12 * sizeof(double), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e == hipSuccess ? VFMM_OK : sfail(hip_status(e), "stats: %s", hipGetErrorString(e));
}

vfmm_status_t vfmm_selector_features(const double* st, int64_t n, double sigma, int32_t p,
                                     int32_t levels, double near_radius, float* out) {
  if (!st || !out) return sfail(VFMM_ERR_INVALID_ARG, "null pointer");
  if (n < 1 || !(sigma > 0.0)) return sfail(VFMM_ERR_INVALID_ARG, "n >= 1 and sigma > 0 required");
  const double dn = double(n);
  const double S = root_side(st);
  const double h = S / std::sqrt(dn);
  const double mean_g = st[4] / dn, rms = std::sqrt(st[5] / dn);
  const double mx = st[0] / dn, my = st[2] / dn;
  const double sx = std::sqrt(std::fmax(0.0, st[1] / dn - mx * mx));
  const double sy = std::sqrt(std::fmax(0.0, st[3] / dn - my * my));
  const double lg = std::log2(dn);
  out[0] = float(p);
  out[1] = float(levels);
  out[2] = float(lg);
  out[3] = float(lg - 2.0 * levels);
  out[4] = float(std::log2(near_distance(S, levels, sigma, near_radius) / sigma));
  out[5] = float(std::log2(sigma / h));
  out[6] = float(rms > 0.0 ? mean_g / rms : 0.0);
  out[7] = float(st[7] > 0.0 ? std::log10(st[6] / st[7]) : 0.0);
  out[8] = float(sx / S);
  out[9] = float(sy / S);
  return VFMM_OK;
}

static vfmm_status_t vfmm_select_params_impl(const double* x, const double* y, const double* gamma, int64_t n,
                                 double sigma, double tol, const float* params,
                                 const float* feat_mean, const float* feat_std, double margin,
                                 void* scratch, size_t scratch_bytes, int32_t* p_out,
                                 int32_t* levels_out, double* radius_out, double* pred_out,
                                 int32_t* fallback_out, void* stream) {
  if (!x || !y || !gamma || !params || !feat_mean || !feat_std || !scratch || !p_out ||
      !levels_out || !radius_out || !pred_out || !fallback_out)
    return sfail(VFMM_ERR_INVALID_ARG, "null pointer");
  if (n < 1 || !(sigma > 0.0) || !std::isfinite(sigma)) return sfail(VFMM_ERR_INVALID_ARG, "bad n or sigma");
  if (!(tol > 0.0) || !(margin >= 0.0)) return sfail(VFMM_ERR_INVALID_ARG, "tol > 0 and margin >= 0 required");
  if (scratch_bytes < select_scratch(n)) return sfail(VFMM_ERR_WORKSPACE, "scratch too small");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int lh = hist_level(n);
  char* s = static_cast<char*>(scratch);
  size_t off = 0;
  double* part = reinterpret_cast<double*>(s + off); off += a256(size_t(kReduceBlocks) * 12 * 8);
  double* sout = reinterpret_cast<double*>(s + off); off += a256(12 * 8);
  uint32_t* counts = reinterpret_cast<uint32_t*>(s + off); off += a256((size_t(1) << (2 * lh)) * 4);
  const int ncand = (kPMax - kPMin + 1) * (lh - 1) * kNRadii;
  float* xd = reinterpret_cast<float*>(s + off); off += a256(size_t(ncand) * 10 * 4);
  float* yd = reinterpret_cast<float*>(s + off);

  double stats[12];
  hipError_t e = launch_stats(x, y, gamma, n, part, sout, st);
  if (e == hipSuccess) e = hipMemcpyAsync(stats, sout, sizeof(stats), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return sfail(hip_status(e), "select stats: %s", hipGetErrorString(e));
  const double S = root_side(stats);
  const double root3[3] = {0.5 * (stats[8] + stats[9]) - 0.5 * S, 0.5 * (stats[10] + stats[11]) - 0.5 * S, S};
  const size_t nl = size_t(1) << (2 * lh);
  e = hipMemsetAsync(counts, 0, nl * 4, st);
  if (e == hipSuccess) e = launch_leaf_hist(x, y, n, root3, lh, counts, st);
  std::vector<uint32_t> hc(nl);
  if (e == hipSuccess) e = hipMemcpyAsync(hc.data(), counts, nl * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return sfail(hip_status(e), "select histogram: %s", hipGetErrorString(e));

  // occupancy at every level <= lh by 2 x 2 pooling; near-field pair counts
  std::vector<std::vector<double>> occ(lh + 1);
  occ[lh].assign(hc.begin(), hc.end());
  for (int l = lh - 1; l >= 0; --l) {
    const int m = 1 << l;
    occ[l].assign(size_t(m) * m, 0.0);
    for (int iy = 0; iy < 2 * m; ++iy)
      for (int ix = 0; ix < 2 * m; ++ix) occ[l][size_t(iy >> 1) * m + (ix >> 1)] += occ[l + 1][size_t(iy) * 2 * m + ix];
  }
  // candidates (p, L, near radius) and their features (z-scored).  The
  // distance cut-off (Section 4.1's distance a) is a candidate where four leaf
  // sides reach the automatic radius (6 sigma), so that its clamp does not cut it.
  const double radii[kNRadii] = {0.0, VFMM_NEAR_RADIUS_AUTO,
                                 sigma * std::sqrt(2.0 * std::log(1.0 / tol))};
  std::vector<float> X(size_t(ncand) * 10);
  std::vector<int> cp(ncand), cl(ncand), cr(ncand);
  std::vector<char> cok(ncand);
  int c = 0;
  for (int L = 2; L <= lh; ++L)
    for (int r = 0; r < kNRadii; ++r)
      for (int p = kPMin; p <= kPMax; ++p, ++c) {
        float f[10];
        vfmm_selector_features(stats, n, sigma, p, L, radii[r], f);
        for (int k = 0; k < 10; ++k) X[size_t(c) * 10 + k] = (f[k] - feat_mean[k]) / feat_std[k];
        cp[c] = p;
        cl[c] = L;
        cr[c] = r;
        cok[c] = r == 0 || VFMM_NEAR_RINGS_MAX * S / std::ldexp(1.0, L) >= 6.0 * sigma;
      }
  std::vector<float> pred(ncand);
  e = hipMemcpyAsync(xd, X.data(), X.size() * 4, hipMemcpyHostToDevice, st);
  if (e == hipSuccess) e = launch_mlp_forward(params, true, xd, ncand, yd, st);
  if (e == hipSuccess) e = hipMemcpyAsync(pred.data(), yd, size_t(ncand) * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return sfail(hip_status(e), "select network: %s", hipGetErrorString(e));

  // cost model (seconds on one MI355X, FP32 evaluation): local-list pairs;
  // with the cut-off, the pairs of the ring leaves weighted by f^2, f the share
  // of the rings within the radius of the leaf (a ring chunk farther than the
  // radius from the target tile is skipped whole, a closer one costs its
  // tests and the pairs that pass; fitted to the near field measured at
  // L = 7 and 8 on 2^20 clustered particles, within about 30 %); per-particle
  // expansion work, per-box translations, per-level launches
  const double lt = std::log10(tol);
  double best = INFINITY;
  int bi = -1;
  std::vector<double> local(lh + 1, -1.0);
  for (int k = 0; k < ncand; ++k) {
    if (!cok[k] || double(pred[k]) + margin > lt) continue;
    const int L = cl[k], p = cp[k];
    double boxes = 0.0;
    for (int l = 2; l <= L; ++l) boxes += std::ldexp(1.0, 2 * l);
    if (local[L] < 0.0) local[L] = near_pairs(occ[L], L);
    double ring = 0.0;
    if (cr[k] > 0) {
      const double w = S / std::ldexp(1.0, L);
      const double a = std::fmin(radii[cr[k]] < 0.0 ? 6.0 * sigma : radii[cr[k]],
                                 VFMM_NEAR_RINGS_MAX * w);
      int d = 2;
      while (d < VFMM_NEAR_RINGS_MAX && d * w < a) ++d;
      const double f = std::fmin(1.0, std::fmax(0.0, ((w + 2.0 * a) * (w + 2.0 * a) - 9.0 * w * w) /
                                                         (double((2 * d + 1) * (2 * d + 1) - 9) * w * w)));
      ring = (near_pairs(occ[L], L, d) - local[L]) * f * f;
    }
    const double cost = 3.1e-13 * local[L] + 6.4e-13 * ring + 2.0e-11 * double(n) * p +
                        1.2e-10 * boxes * p * p + 2.0e-5 * L;
    if (cost < best) {
      best = cost;
      bi = k;
    }
  }
  if (bi >= 0) {
    *p_out = cp[bi];
    *levels_out = cl[bi];
    *radius_out = radii[cr[bi]];
    *pred_out = double(pred[bi]);
    *fallback_out = 0;
  } else {
    int L = 0;
    while (L + 1 <= kMaxLevels && S / std::ldexp(1.0, L + 1) / sigma >= 8.0 &&
           (int64_t(1) << (2 * (L + 1))) <= 4 * n)
      ++L;
    *p_out = 20;
    *levels_out = L;
    *radius_out = 0.0;
    *pred_out = NAN;
    *fallback_out = 1;
  }
  return VFMM_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Selection with audit (Section 5: the error of an evaluation is measured
// against the direct sum of eq. 7 on sampled targets, normalised by the
// maximum velocity, Section 5.1).

namespace {

// u[targets[k]], v[targets[k]] -> ut[k], vt[k]; an index outside [0, n) gives
// NaN, which fails the audit.
__global__ void __launch_bounds__(256) k_gather_targets(const double* __restrict__ u,
                                                        const double* __restrict__ v,
                                                        const int64_t* __restrict__ tg,
                                                        int64_t nt, int64_t n,
                                                        double* __restrict__ ut,
                                                        double* __restrict__ vt) {
  const int64_t k = blockIdx.x * 256LL + threadIdx.x;
  if (k >= nt) return;
  const int64_t i = tg[k];
  const bool ok = i >= 0 && i < n;
  ut[k] = ok ? u[i] : __builtin_nan("");
  vt[k] = ok ? v[i] : __builtin_nan("");
}

// Deepest level allowed by default: the candidate grid's bound and about four
// particles per leaf.
int default_max_levels(int64_t n) {
  int l = 0;
  while (l < kHistMax && (int64_t(1) << (2 * (l + 1))) <= 4 * n) ++l;
  return l;
}

// The conservative choice: p = 20 and the deepest level whose leaf side is
// at least 8 sigma (the kernel-substitution error of Section 4.1 is then
// negligible), with about four particles per leaf at most.
int conservative_levels(double S, double sigma, int64_t n, int max_levels) {
  int L = 0;
  while (L + 1 <= max_levels && S / std::ldexp(1.0, L + 1) / sigma >= 8.0 &&
         (int64_t(1) << (2 * (L + 1))) <= 4 * n)
    ++L;
  return L;
}

struct AuditWs {
  char* sel;
  size_t sel_bytes;
  char* tree;
  size_t tree_bytes;
  double *u, *v, *ut, *vt, *ur, *vr, *met_scratch, *met;
  size_t total;
};

AuditWs audit_layout(char* base, int64_t n, int64_t nt, int max_levels) {
  AuditWs w{};
  size_t off = 0;
  auto take = [&](size_t b) { size_t r = off; off += a256(b); return base + r; };
  w.sel_bytes = select_scratch(n);
  w.sel = take(w.sel_bytes);
  size_t tb = 0;
  vfmm_workspace_bytes(n, max_levels, kPMax, &tb);
  w.tree_bytes = tb;
  w.tree = take(tb);
  w.u = reinterpret_cast<double*>(take(size_t(n) * 8));
  w.v = reinterpret_cast<double*>(take(size_t(n) * 8));
  w.ut = reinterpret_cast<double*>(take(size_t(nt) * 8));
  w.vt = reinterpret_cast<double*>(take(size_t(nt) * 8));
  w.ur = reinterpret_cast<double*>(take(size_t(nt) * 8));
  w.vr = reinterpret_cast<double*>(take(size_t(nt) * 8));
  w.met_scratch = reinterpret_cast<double*>(take(vfmm_metrics_scratch_bytes()));
  w.met = reinterpret_cast<double*>(take(3 * 8));
  w.total = off;
  return w;
}

struct Auditor {
  const double *x, *y, *g;
  int64_t n;
  double sigma;
  const int64_t* tg;
  int64_t nt;
  const double *ur, *vr;
  AuditWs w;
  int reps;
  hipStream_t st;
  hipEvent_t e0 = nullptr, e1 = nullptr;

  // FMM of (p, L, precision, radius) at all particles, its error on the audit
  // targets and, if `timed`, the median time of `reps` rebuild + evaluation
  // runs (HIP events on the stream).
  vfmm_status_t run(int p, int L, int prec, double radius, bool timed, double& e, double& ms) {
    vfmm_tree_t t = nullptr;
    vfmm_status_t s = vfmm_build_tree(x, y, n, L, nullptr, p, w.tree, w.tree_bytes, st, &t);
    if (s) return s;
    if (!(s = vfmm_tree_set_near_radius(t, radius)))
      s = vfmm_fmm_velocity(t, g, sigma, p, prec, w.u, w.v, st);
    if (!s) {
      hipLaunchKernelGGL(k_gather_targets, dim3(unsigned((nt + 255) / 256)), dim3(256), 0, st,
                         w.u, w.v, tg, nt, n, w.ut, w.vt);
      hipError_t he = hipGetLastError();
      if (he != hipSuccess) s = sfail(hip_status(he), "audit gather: %s", hipGetErrorString(he));
    }
    if (!s) s = vfmm_error_metrics(w.ut, w.vt, ur, vr, nt, w.met_scratch, w.met, st);
    double m[3] = {0.0, 0.0, 0.0};
    if (!s) {
      hipError_t he = hipMemcpyAsync(m, w.met, sizeof(m), hipMemcpyDeviceToHost, st);
      if (he == hipSuccess) he = hipStreamSynchronize(st);
      if (he != hipSuccess) s = sfail(hip_status(he), "audit metrics: %s", hipGetErrorString(he));
    }
    ms = -1.0;
    if (!s && timed) {
      std::vector<float> times;
      for (int r = 0; r < reps && !s; ++r) {
        hipError_t he = hipEventRecord(e0, st);
        if (he != hipSuccess) {
          s = sfail(hip_status(he), "audit timing: %s", hipGetErrorString(he));
          break;
        }
        if ((s = vfmm_tree_rebuild(t, x, y, nullptr, st))) break;
        if ((s = vfmm_fmm_velocity(t, g, sigma, p, prec, w.u, w.v, st))) break;
        he = hipEventRecord(e1, st);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float f = 0.f;
        if (he == hipSuccess) he = hipEventElapsedTime(&f, e0, e1);
        if (he != hipSuccess) s = sfail(hip_status(he), "audit timing: %s", hipGetErrorString(he));
        times.push_back(f);
      }
      if (!s) {
        std::sort(times.begin(), times.end());
        ms = double(times[times.size() / 2]);
      }
    }
    vfmm_tree_destroy(t);
    if (s) return s;
    const double den = m[2] == 0.0 ? 1.0 : m[2];  // a NaN maximum stays NaN
    e = m[0] / den;
    return VFMM_OK;
  }
};

void record(vfmm_selection* out, int p, int L, int prec, double radius, double e, double ms) {
  if (out->n_steps >= VFMM_SELECT_TRAIL_MAX) return;
  vfmm_audit_step& a = out->steps[out->n_steps++];
  a.p = p;
  a.levels = L;
  a.precision = prec;
  a.near_radius = radius;
  a.emax = e;
  a.ms = ms;
}

}  // namespace

extern "C" {

vfmm_status_t vfmm_select_audit_workspace_bytes(int64_t n, int64_t n_audit, int32_t max_levels,
                                                size_t* bytes) {
  if (!bytes) return sfail(VFMM_ERR_INVALID_ARG, "bytes is NULL");
  if (n < 1 || n > 2147483647LL) return sfail(VFMM_ERR_INVALID_ARG, "n out of [1, 2^31-1]");
  if (n_audit < 1 || n_audit > n) return sfail(VFMM_ERR_INVALID_ARG, "n_audit out of [1, n]");
  if (max_levels <= 0) max_levels = default_max_levels(n);
  if (max_levels > kMaxLevels) return sfail(VFMM_ERR_INVALID_ARG, "max_levels > %d", kMaxLevels);
  *bytes = audit_layout(nullptr, n, n_audit, max_levels).total;
  return VFMM_OK;
}

static vfmm_status_t vfmm_select_and_audit_impl(const double* x, const double* y, const double* gamma,
                                    int64_t n, double sigma, double tol, const float* params,
                                    const float* feat_mean, const float* feat_std, double margin,
                                    const int64_t* targets, int64_t n_audit, const double* u_ref,
                                    const double* v_ref, int32_t flags, double slack,
                                    int32_t time_reps, int32_t max_levels, void* workspace,
                                    size_t ws_bytes, vfmm_selection* out, void* stream) {
  if (!x || !y || !gamma || !params || !feat_mean || !feat_std || !out || !workspace)
    return sfail(VFMM_ERR_INVALID_ARG, "null pointer");
  if (n < 1 || n > 2147483647LL) return sfail(VFMM_ERR_INVALID_ARG, "n out of [1, 2^31-1]");
  if (!(sigma > 0.0) || !std::isfinite(sigma)) return sfail(VFMM_ERR_INVALID_ARG, "bad sigma");
  if (!(tol > 0.0) || !(slack > 0.0) || !(slack <= 1.0))
    return sfail(VFMM_ERR_INVALID_ARG, "tol > 0 and 0 < slack <= 1 required");
  if (flags & ~(VFMM_SELECT_AUDIT | VFMM_SELECT_CUTOFF))
    return sfail(VFMM_ERR_INVALID_ARG, "unknown flags 0x%x", unsigned(flags));
  const bool audit = flags & VFMM_SELECT_AUDIT;
  if (audit && (!targets || n_audit < 1 || n_audit > n))
    return sfail(VFMM_ERR_INVALID_ARG, "audit needs 1 <= n_audit <= n targets");
  if (!audit) n_audit = 1;
  if ((u_ref == nullptr) != (v_ref == nullptr))
    return sfail(VFMM_ERR_INVALID_ARG, "give both u_ref and v_ref or neither");
  if (time_reps < 1 || time_reps > 100) return sfail(VFMM_ERR_INVALID_ARG, "time_reps out of [1, 100]");
  if (max_levels <= 0) max_levels = default_max_levels(n);
  if (max_levels > kMaxLevels) return sfail(VFMM_ERR_INVALID_ARG, "max_levels > %d", kMaxLevels);
  if (reinterpret_cast<uintptr_t>(workspace) & 255)
    return sfail(VFMM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  const AuditWs w = audit_layout(static_cast<char*>(workspace), n, n_audit, max_levels);
  if (ws_bytes < w.total)
    return sfail(VFMM_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, w.total);
  hipStream_t st = static_cast<hipStream_t>(stream);
  *out = vfmm_selection{};

  // the network's choice
  int32_t p = 0, L = 0, fb = 0;
  double pred = 0.0, rad = 0.0;
  vfmm_status_t s = vfmm_select_params(x, y, gamma, n, sigma, tol, params, feat_mean, feat_std,
                                       margin, w.sel, w.sel_bytes, &p, &L, &rad, &pred, &fb,
                                       stream);
  if (s) return s;
  if (L > max_levels) L = max_levels;
  if (!(flags & VFMM_SELECT_CUTOFF)) rad = 0.0;
  out->network_p = p;
  out->network_levels = L;
  out->network_radius = rad;
  out->network_fallback = fb;
  out->predicted_log10 = pred;
  out->p = p;
  out->levels = L;
  out->precision = VFMM_FP32;
  out->near_radius = rad;
  out->used_fallback = fb;
  out->audit_emax = NAN;
  if (!audit) return VFMM_OK;

  // the direct-sum reference on the audit targets (eq. 7)
  if (!u_ref) {
    if ((s = vfmm_direct_velocity(x, y, gamma, n, sigma, targets, n_audit, w.ur, w.vr, stream)))
      return s;
    u_ref = w.ur;
    v_ref = w.vr;
  }
  Auditor a{x, y, gamma, n, sigma, targets, n_audit, u_ref, v_ref, w, time_reps, st};
  hipError_t he = hipEventCreate(&a.e0);
  if (he == hipSuccess) he = hipEventCreate(&a.e1);
  if (he != hipSuccess) {
    if (a.e0) (void)hipEventDestroy(a.e0);
    return sfail(hip_status(he), "audit events: %s", hipGetErrorString(he));
  }
  struct Events {
    Auditor& a;
    ~Events() {
      if (a.e0) (void)hipEventDestroy(a.e0);
      if (a.e1) (void)hipEventDestroy(a.e1);
    }
  } release{a};
  const double bar = slack * tol;
  auto pass = [&](double e) { return e <= bar; };  // NaN or infinity fails

  // FP32 at the network's (p, L, radius); p raised by 2 (up to 20) while it fails
  double e = 0.0, ms = 0.0;
  if ((s = a.run(p, L, VFMM_FP32, rad, false, e, ms))) return s;
  record(out, p, L, VFMM_FP32, rad, e, ms);
  while (!pass(e) && p < kPMax) {
    p = p + 2 < kPMax ? p + 2 : kPMax;
    if ((s = a.run(p, L, VFMM_FP32, rad, false, e, ms))) return s;
    record(out, p, L, VFMM_FP32, rad, e, ms);
  }
  out->p = p;
  out->audit_emax = e;
  // root side of the bounding square, for the level conditions below
  double stats[12];
  if ((s = vfmm_particle_stats(x, y, gamma, n, w.sel, w.sel_bytes, stats, stream))) return s;
  const double S = root_side(stats);
  if (!pass(e)) {
    // FP32 cannot meet the tolerance here (its floor, rounding of positions
    // and circulations amplified by cancellation, can exceed it): the
    // conservative choice in FP64
    const int Lc = conservative_levels(S, sigma, n, max_levels);
    if ((s = a.run(kPMax, Lc, VFMM_FP64, 0.0, false, e, ms))) return s;
    record(out, kPMax, Lc, VFMM_FP64, 0.0, e, ms);
    out->p = kPMax;
    out->levels = Lc;
    out->precision = VFMM_FP64;
    out->used_fallback = 1;
    out->audit_emax = e;
    return VFMM_OK;
  }
  if (!(flags & VFMM_SELECT_CUTOFF)) return VFMM_OK;

  // Timed comparison with the neighbours of the accepted choice: the same p
  // at levels L - 1 .. L + 1, each with the paper's split and with the
  // distance cut-off (Section 4.1's distance a) at the automatic radius and
  // at sigma sqrt(2 ln(1/tol)), where one pair's kernel difference falls to
  // the tolerance; the cut-off only where the clamp at VFMM_NEAR_RINGS_MAX
  // leaf sides leaves 6 sigma uncut.  Each is audited; the passing ones are
  // timed, and the fastest replaces the accepted choice only if it is faster
  // by more than kTimeMargin (the spread of repeated timings of one
  // configuration), so that a tie keeps the network's choice.
  const double radii3[3] = {0.0, VFMM_NEAR_RADIUS_AUTO,
                            sigma * std::sqrt(2.0 * std::log(1.0 / tol))};
  int cand_L[9];
  double cand_r[9];
  int nc = 0;
  for (int LL = L - 1; LL <= L + 1; ++LL) {
    if (LL < 2 || LL > max_levels || (int64_t(1) << (2 * LL)) > 4 * n) continue;
    for (double r : radii3) {
      if (LL == L && r == rad) continue;
      if (r != 0.0 && VFMM_NEAR_RINGS_MAX * S / std::ldexp(1.0, LL) < 6.0 * sigma) continue;
      cand_L[nc] = LL;
      cand_r[nc++] = r;
    }
  }
  if (nc == 0) return VFMM_OK;
  double e0 = 0.0, ms0 = 0.0;
  if ((s = a.run(p, L, VFMM_FP32, rad, true, e0, ms0))) return s;
  out->steps[out->n_steps - 1].ms = ms0;  // the accepted step, now timed
  constexpr double kTimeMargin = 0.03;
  double best_ms = ms0 * (1.0 - kTimeMargin), best_e = e, best_r = rad;
  int best_L = L;
  for (int k = 0; k < nc; ++k) {
    double ec = 0.0, msc = 0.0;
    if ((s = a.run(p, cand_L[k], VFMM_FP32, cand_r[k], true, ec, msc))) return s;
    record(out, p, cand_L[k], VFMM_FP32, cand_r[k], ec, msc);
    if (pass(ec) && msc < best_ms) {
      best_ms = msc;
      best_e = ec;
      best_r = cand_r[k];
      best_L = cand_L[k];
    }
  }
  out->levels = best_L;
  out->near_radius = best_r;
  out->audit_emax = best_e;
  return VFMM_OK;
}

// Host allocations inside (std::vector) report running out of memory as a
// status instead of letting the exception cross the C ABI.
vfmm_status_t vfmm_select_params(const double* x, const double* y, const double* gamma, int64_t n,
                                 double sigma, double tol, const float* params,
                                 const float* feat_mean, const float* feat_std, double margin,
                                 void* scratch, size_t scratch_bytes, int32_t* p_out,
                                 int32_t* levels_out, double* radius_out, double* pred_out,
                                 int32_t* fallback_out, void* stream) {
  try {
    return vfmm_select_params_impl(x, y, gamma, n, sigma, tol, params, feat_mean, feat_std, margin, scratch,
                                   scratch_bytes, p_out, levels_out, radius_out, pred_out,
                                   fallback_out, stream);
  } catch (const std::bad_alloc&) {
    return sfail(VFMM_ERR_OUT_OF_MEMORY, "vfmm_select_params: host allocation failed");
  }
}

// Host allocations inside (std::vector) report running out of memory as a
// status instead of letting the exception cross the C ABI.
vfmm_status_t vfmm_select_and_audit(const double* x, const double* y, const double* gamma,
                                    int64_t n, double sigma, double tol, const float* params,
                                    const float* feat_mean, const float* feat_std, double margin,
                                    const int64_t* targets, int64_t n_audit, const double* u_ref,
                                    const double* v_ref, int32_t flags, double slack,
                                    int32_t time_reps, int32_t max_levels, void* workspace,
                                    size_t ws_bytes, vfmm_selection* out, void* stream) {
  try {
    return vfmm_select_and_audit_impl(x, y, gamma, n, sigma, tol, params, feat_mean, feat_std, margin,
                                      targets, n_audit, u_ref, v_ref, flags, slack, time_reps,
                                      max_levels, workspace, ws_bytes, out, stream);
  } catch (const std::bad_alloc&) {
    return sfail(VFMM_ERR_OUT_OF_MEMORY, "vfmm_select_and_audit: host allocation failed");
  }
}

}  // extern "C"
