// Batched evaluation of many independent FMM instances (uneven N, p, levels).
//
// Each phase of the method (Section 3.1, Fig. 3) runs ONCE for all instances:
// bounding squares, one global stable radix sort on (instance, leaf, sub-cell)
// keys, leaf ranges, tiles; then P2M, M2M (one launch per level), M2L and L2L
// (one launch per level) on a second stream while the near field (P2P) runs;
// after both, L2P adds the far field and writes the result.  A work item
// (particle, leaf, box coefficient, tile) finds its instance by binary search
// in a small table of per-instance offsets, so the launch count does not
// depend on the number of instances, and the whole sequence can be captured
// once in a hipGraph (two branches) and replayed.
//
// Arithmetic per instance: P2P in FP32 (as in p2p.hip); expansions in FP32 for
// p <= 16; for p > 16 the shifts (P2M, M2M, L2L) and L2P in FP64 with the M2L
// in FP32 on the matrix cores (the multipoles rounded to float32 copies, the
// M2L sums widened back before the float64 L2L chain); on the scaled,
// level-independent operators of expansions.hip (one table set per p).  The
// M2L (m2l_tile.hpp) takes one launch for the p <= 16 instances and one for the
// p > 16 instances (64-row tiles), each covering all their levels; the L2L
// chain then runs one coefficient per thread, one launch per level.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <new>
#include <vector>

#include "../../include/vfmm.h"
#include "m2l_tile.hpp"
#include "p2p_math.hpp"

namespace vfmm {

// Device descriptor of one instance.
struct BatchInst {
  const double* x;
  const double* y;
  const double* g;
  double* u;
  double* v;
  int64_t n;
  int64_t part_off;  // first particle in the concatenated (sorted) arrays
  int64_t leaf_off;  // first global leaf; leaf_start entries start at leaf_off + index
  int64_t me_off;    // byte offset of the level-2 coefficients in the ME / LE buffers
  int64_t me32_off;  // p > 16: byte offset of their float32 copies in the ME32 / LE32 buffers
  double sigma;
  int32_t p, L, fp64;
  int32_t sym;  // symmetric near field for this instance (see k_b_p2p)
};

constexpr int kBatchMaxLevels = 6;   // leaf index fits 12 key bits
// Inside a leaf, particles are ordered by their cell kBatchSub levels deeper
// (leaves here hold up to about a thousand particles, so 16 cells of tile
// size keep the tiles compact; the single tree's clustered leaves need more)
constexpr int kBatchSub = 2;
constexpr int kBatchKeyInst = 12 + 2 * kBatchSub;  // key = inst << 16 | leaf << 4 | sub-cell
constexpr int kBatchMaxCount = 4096;
constexpr int kBatchP2PWaves = 4;  // near-field waves (tiles) per workgroup
constexpr int kBatchSymMinPPL = 48;  // mean particles per leaf for the symmetric near field
constexpr int kBatchPMax = 24;

namespace {

__device__ __forceinline__ int find_seg(const int64_t* off, int count, int64_t i) {
  // index c with off[c] <= i < off[c + 1] (off has count + 1 entries)
  int lo = 0, hi = count;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= i) lo = mid; else hi = mid;
  }
  return lo;
}

__device__ inline uint32_t spread4b(uint32_t v) {
  v &= 15u;
  v = (v | (v << 2)) & 0x33u;
  v = (v | (v << 1)) & 0x55u;
  return v;
}

__global__ void __launch_bounds__(256) k_b_bbox(const BatchInst* __restrict__ I,
                                                double* __restrict__ roots,
                                                int32_t* __restrict__ nbig) {
#pragma clang fp contract(off)
  __shared__ double s[4][256];
  if (blockIdx.x == 0 && threadIdx.x == 0) *nbig = 0;  // big-leaf list of this run
  const BatchInst in = I[blockIdx.x];
  double a = INFINITY, b = -INFINITY, c = INFINITY, d = -INFINITY;
  // 8 particles per thread and pass: their loads are issued together
  int64_t i = threadIdx.x;
  for (; i + 7 * 256 < in.n; i += 8 * 256) {
    double xs[8], ys[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      xs[k] = in.x[i + k * 256];
      ys[k] = in.y[i + k * 256];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      a = fmin(a, xs[k]); b = fmax(b, xs[k]); c = fmin(c, ys[k]); d = fmax(d, ys[k]);
    }
  }
  for (; i < in.n; i += 256) {
    const double xi = in.x[i], yi = in.y[i];
    a = fmin(a, xi); b = fmax(b, xi); c = fmin(c, yi); d = fmax(d, yi);
  }
  s[0][threadIdx.x] = a; s[1][threadIdx.x] = b; s[2][threadIdx.x] = c; s[3][threadIdx.x] = d;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (int(threadIdx.x) < st) {
      const int o = threadIdx.x + st;
      s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][o]);
      s[1][threadIdx.x] = fmax(s[1][threadIdx.x], s[1][o]);
      s[2][threadIdx.x] = fmin(s[2][threadIdx.x], s[2][o]);
      s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double ext = fmax(s[1][0] - s[0][0], s[3][0] - s[2][0]);
    const double S = ext > 0.0 ? ext * (1.0 + 0x1p-20) : 1.0;
    double* r = roots + 4 * blockIdx.x;
    r[0] = 0.5 * (s[0][0] + s[1][0]) - 0.5 * S;
    r[1] = 0.5 * (s[2][0] + s[3][0]) - 0.5 * S;
    r[2] = S;
    r[3] = S / double(1 << in.L);
  }
}

// Sort keys, the identity permutation, and each particle's record in input
// order (leaf-local position in units of the instance's Gaussian width, as in
// the single tree, and circulation), which k_b_local moves to sorted order.
__global__ void __launch_bounds__(256) k_b_keys(const BatchInst* __restrict__ I,
                                                const int64_t* __restrict__ part_off, int count,
                                                int64_t ntot, const double* __restrict__ roots,
                                                uint32_t* __restrict__ keys,
                                                int32_t* __restrict__ idx,
                                                Part32* __restrict__ raw) {
#pragma clang fp contract(off)
  const int64_t i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= ntot) return;
  const int c = find_seg(part_off, count, i);
  const BatchInst in = I[c];
  const int64_t j = i - in.part_off;
  const double* r = roots + 4 * c;
  const int mf = 1 << (in.L + kBatchSub);
  const double xj = in.x[j], yj = in.y[j];
  const double fx = floor(((xj - r[0]) / r[2]) * double(mf));
  const double fy = floor(((yj - r[1]) / r[2]) * double(mf));
  const int ix = !(fx >= 0.0) ? 0 : (fx > double(mf - 1) ? mf - 1 : int(fx));
  const int iy = !(fy >= 0.0) ? 0 : (fy > double(mf - 1) ? mf - 1 : int(fy));
  const uint32_t leaf = (uint32_t(iy >> kBatchSub) << in.L) | uint32_t(ix >> kBatchSub);
  const uint32_t cm = (1u << kBatchSub) - 1u;
  const uint32_t sub = spread4b(uint32_t(ix) & cm) | (spread4b(uint32_t(iy) & cm) << 1);
  keys[i] = (uint32_t(c) << kBatchKeyInst) | (leaf << (2 * kBatchSub)) | sub;
  idx[i] = int32_t(i);
  const double cx = r[0] + (double(ix >> kBatchSub) + 0.5) * r[3];
  const double cy = r[1] + (double(iy >> kBatchSub) + 0.5) * r[3];
  const double sd = near_scale(in.sigma);
  raw[i] = Part32{float((xj - cx) * sd), float((yj - cy) * sd), float(in.g[j]), 0.0f};
}

// leaf_start[leaf_off + c + k] = first sorted position of leaf k of instance c,
// k = 0 .. 4^L (the last entry ends the instance).
__global__ void __launch_bounds__(256) k_b_leaf_start(const int64_t* __restrict__ ls_off,
                                                      int count, const uint32_t* __restrict__ keys,
                                                      int64_t ntot, int32_t* __restrict__ start) {
  const int64_t q = blockIdx.x * 256LL + threadIdx.x;
  if (q >= ls_off[count]) return;
  const int c = find_seg(ls_off, count, q);
  const int64_t k = q - ls_off[c];
  const uint64_t key = (uint64_t(c) << kBatchKeyInst) + (uint64_t(k) << (2 * kBatchSub));
  int64_t lo = 0, hi = ntot;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (uint64_t(keys[mid]) < key) lo = mid + 1; else hi = mid;
  }
  start[q] = int32_t(lo);
}

// The particles' records in sorted order (one 16-byte record per particle
// through the permutation).
__global__ void __launch_bounds__(256) k_b_local(const Part32* __restrict__ raw,
                                                 const int32_t* __restrict__ perm, int64_t ntot,
                                                 Part32* __restrict__ p32) {
  const int64_t i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= ntot) return;
  p32[i] = raw[perm[i]];
}

__global__ void __launch_bounds__(256) k_b_tile_counts(const int64_t* __restrict__ leaf_off,
                                                       int count,
                                                       const int32_t* __restrict__ start,
                                                       uint32_t* __restrict__ cnt) {
  const int64_t gl = blockIdx.x * 256LL + threadIdx.x;
  const int64_t nl = leaf_off[count];
  if (gl > nl) return;
  if (gl == nl) {
    cnt[gl] = 0u;
    return;
  }
  const int c = find_seg(leaf_off, count, gl);
  const int64_t q = gl + c;
  cnt[gl] = uint32_t((start[q + 1] - start[q] + kTile - 1) / kTile);
}

__global__ void __launch_bounds__(256) k_b_tile_fill(const BatchInst* __restrict__ I,
                                                     const uint32_t* __restrict__ keys,
                                                     const int32_t* __restrict__ start,
                                                     const uint32_t* __restrict__ toff,
                                                     int64_t ntot, int64_t nleaves,
                                                     Tile* __restrict__ tiles,
                                                     int32_t* __restrict__ ntiles) {
  const int64_t i = blockIdx.x * 256LL + threadIdx.x;
  if (i == 0) *ntiles = int32_t(toff[nleaves]);
  if (i >= ntot) return;
  const uint32_t key = keys[i];
  const int c = int(key >> kBatchKeyInst);
  const int64_t gl = I[c].leaf_off + ((key >> (2 * kBatchSub)) & 0xFFFu);
  const int32_t s = start[gl + c], cnt = start[gl + c + 1] - s;
  const int32_t r = int32_t(i) - s;
  if (r % kTile != 0) return;
  const int32_t cc = cnt - r;
  tiles[toff[gl] + r / kTile] = Tile{int32_t(gl), int32_t(i), cc < kTile ? cc : kTile, c};
}

// ------------------------------------------------------------------ expansions

template <typename R>
__device__ __forceinline__ typename Types<R>::C* coef(char* base, const BatchInst& in, int lev) {
  return reinterpret_cast<typename Types<R>::C*>(base + in.me_off) + level_offset(lev) * in.p;
}
// the float32 copies of a p > 16 instance's coefficients (M2L on the matrix cores)
__device__ __forceinline__ float2* coef32(char* base, const BatchInst& in, int lev) {
  return reinterpret_cast<float2*>(base + in.me32_off) + level_offset(lev) * in.p;
}

// Sum of the wave's values when only lanes 0 .. 2^steps - 1 hold non-zeros:
// butterfly within those lanes, then lane 0's total to every lane.
template <typename R>
__device__ __forceinline__ R lanes_sum(R v, int steps) {
  for (int o = 0; o < steps; ++o) v += __shfl_xor(v, 1 << o, 64);
  return __shfl(v, 0, 64);
}

// P2M of one leaf by one wave (eq. 13 on the scaled coefficients): lanes take
// every 64th particle, the partial sums are combined with shuffles (as many
// steps as the leaf's particle count needs), lane c writes component c.
template <typename R>
__device__ void p2m_leaf(const BatchInst& in, const Part32* __restrict__ p32, int32_t s, int32_t e,
                         double w, int leaf, char* me) {
  using C = typename Types<R>::C;
  const int lane = threadIdx.x & 63;
  const R inv_w = R(1.0 / w);
  C acc[kBatchPMax];
#pragma unroll
  for (int k = 0; k < kBatchPMax; ++k) acc[k] = cmake<C>(R(0), R(0));
  for (int32_t i = s + lane; i < e; i += 64) {
    const Part32 q = p32[i];
    const C z = cmake<C>(R(q.x) * inv_w, R(q.y) * inv_w);
    C pw = cmake<C>(R(q.g), R(0));
#pragma unroll
    for (int k = 0; k < kBatchPMax; ++k) {
      if (k < in.p) {
        acc[k].x += pw.x;
        acc[k].y += pw.y;
        pw = cmul(pw, z);
      }
    }
  }
  const int n = e - s;
  int steps = 0;
  while (steps < 6 && (1 << steps) < n) ++steps;
  R mine = R(0);
#pragma unroll
  for (int k = 0; k < kBatchPMax; ++k) {
    if (k < in.p) {
      const R re = lanes_sum(acc[k].x, steps), im = lanes_sum(acc[k].y, steps);
      if (lane == 2 * k) mine = re;
      if (lane == 2 * k + 1) mine = im;
    }
  }
  if (lane < 2 * in.p) reinterpret_cast<R*>(coef<R>(me, in, in.L) + int64_t(leaf) * in.p)[lane] = mine;
}

// P2M of one leaf by one lane: the leaf's particles in order.
template <typename R>
__device__ void p2m_serial(const BatchInst& in, const Part32* __restrict__ p32, int32_t s,
                           int32_t e, double w, int leaf, char* me) {
  using C = typename Types<R>::C;
  const R inv_w = R(1.0 / w);
  C acc[kBatchPMax];
#pragma unroll
  for (int k = 0; k < kBatchPMax; ++k) acc[k] = cmake<C>(R(0), R(0));
  for (int32_t i = s; i < e; ++i) {
    const Part32 q = p32[i];
    const C z = cmake<C>(R(q.x) * inv_w, R(q.y) * inv_w);
    C pw = cmake<C>(R(q.g), R(0));
#pragma unroll
    for (int k = 0; k < kBatchPMax; ++k) {
      if (k < in.p) {
        acc[k].x += pw.x;
        acc[k].y += pw.y;
        pw = cmul(pw, z);
      }
    }
  }
  C* out = coef<R>(me, in, in.L) + int64_t(leaf) * in.p;
#pragma unroll
  for (int k = 0; k < kBatchPMax; ++k)
    if (k < in.p) out[k] = acc[k];
}

// One lane per leaf, 64 consecutive (global) leaves per wave: a leaf of at
// most kTile particles is summed by its lane (empty leaves get zeros); larger
// leaves are appended to big (global leaf, instance) for k_b_p2m_big.
__global__ void __launch_bounds__(256) k_b_p2m(const BatchInst* __restrict__ I,
                                               const int64_t* __restrict__ leaf_off, int count,
                                               const int32_t* __restrict__ start,
                                               const Part32* __restrict__ p32,
                                               const double* __restrict__ roots, char* me,
                                               int2* __restrict__ big, int32_t* __restrict__ nbig) {
  const int lane = threadIdx.x & 63;
  const int64_t base = int64_t(__builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6))) * 64;
  const int64_t nl = leaf_off[count];
  if (base >= nl) return;
  const int64_t gl = base + lane;
  const int c = gl < nl ? find_seg(leaf_off, count, gl) : 0;
  const BatchInst in = I[c];
  const bool mine = gl < nl && in.L >= 2;
  int32_t s = 0, e = 0;
  if (mine) {
    s = start[gl + c];
    e = start[gl + c + 1];
  }
  if (mine && e - s <= kTile) {
    const double w = roots[4 * c + 3] * near_scale(in.sigma);  // leaf side in the particles' units
    const int leaf = int(gl - in.leaf_off);
    if (in.fp64) p2m_serial<double>(in, p32, s, e, w, leaf, me);
    else p2m_serial<float>(in, p32, s, e, w, leaf, me);
  }
  const bool is_big = mine && e - s > kTile;
  const uint64_t bm = __ballot(is_big);
  if (bm) {
    int32_t first = 0;
    if (lane == __builtin_ctzll(bm)) first = atomicAdd(nbig, int32_t(__popcll(bm)));
    first = __shfl(first, __builtin_ctzll(bm), 64);
    if (is_big) big[first + __popcll(bm & ((uint64_t(1) << lane) - 1))] = make_int2(int(gl), c);
  }
}

// The leaves of more than kTile particles: one wave each (grid: an upper bound
// on their number; waves beyond *nbig exit).
__global__ void __launch_bounds__(256) k_b_p2m_big(const BatchInst* __restrict__ I,
                                                   const int32_t* __restrict__ start,
                                                   const Part32* __restrict__ p32,
                                                   const double* __restrict__ roots, char* me,
                                                   const int2* __restrict__ big,
                                                   const int32_t* __restrict__ nbig) {
  const int wid = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (wid >= *nbig) return;
  const int2 b = big[wid];
  const int gl = __builtin_amdgcn_readfirstlane(b.x), c = __builtin_amdgcn_readfirstlane(b.y);
  const BatchInst in = I[c];
  const int32_t s = start[gl + c], e = start[gl + c + 1];
  const int leaf = int(gl - in.leaf_off);
  const double w = roots[4 * c + 3] * near_scale(in.sigma);
  if (in.fp64) p2m_leaf<double>(in, p32, s, e, w, leaf, me);
  else p2m_leaf<float>(in, p32, s, e, w, leaf, me);
}

template <typename R>
__device__ void m2m_item(const BatchInst& in, int lev, int64_t item, char* me, const char* tab,
                         const int64_t* tab_off) {
  using C = typename Types<R>::C;
  const int p = in.p;
  const int64_t box = item / p;
  const int n = int(item % p);
  const int mp = 1 << lev, mc = 2 * mp;
  const int px = int(box & (mp - 1)), py = int(box >> lev);
  const OpsLayout ol = ops_layout(p);
  const C* A = reinterpret_cast<const C*>(tab + tab_off[p] + (sizeof(R) == 8 ? ol.m2m64 : ol.m2m32));
  const C* child = coef<R>(me, in, lev + 1);
  C acc = cmake<C>(R(0), R(0));
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t cb = int64_t(2 * py + (q >> 1)) * mc + (2 * px + (q & 1));
    const C* m = child + cb * p;
    const C* a = A + (q * p + n) * p;
    for (int k = 0; k <= n; ++k) cfma(acc, a[k], m[k]);
  }
  coef<R>(me, in, lev)[box * p + n] = acc;
}

__global__ void __launch_bounds__(256) k_b_m2m(const BatchInst* __restrict__ I,
                                               const int64_t* __restrict__ items, int count,
                                               int lev, char* me, const char* tab,
                                               const int64_t* __restrict__ tab_off) {
  const int64_t t = blockIdx.x * 256LL + threadIdx.x;
  if (t >= items[count]) return;
  const int c = find_seg(items, count, t);
  const BatchInst in = I[c];
  const int64_t item = t - items[c];
  if (in.fp64) m2m_item<double>(in, lev, item, me, tab, tab_off);
  else m2m_item<float>(in, lev, item, me, tab, tab_off);
}

// le[lev] += L2L(le[lev - 1]) (Section 3.3.3), the M2L part of le[lev] being
// already there (lev >= 3); one output coefficient per item.
template <typename R>
__device__ void l2l_item(const BatchInst& in, int lev, int64_t item, char* le, const char* tab,
                         const int64_t* tab_off) {
  using C = typename Types<R>::C;
  const int p = in.p;
  const int64_t box = item / p;
  const int n = int(item % p);
  const int m = 1 << lev;
  const int bx = int(box & (m - 1)), by = int(box >> lev);
  const OpsLayout ol = ops_layout(p);
  const C* B = reinterpret_cast<const C*>(tab + tab_off[p] + (sizeof(R) == 8 ? ol.l2l64 : ol.l2l32));
  const int64_t pb = int64_t(by >> 1) * (m >> 1) + (bx >> 1);
  const int q = ((by & 1) << 1) | (bx & 1);
  const C* lp = coef<R>(le, in, lev - 1) + pb * p;
  const C* b = B + (q * p + n) * p;
  C* out = coef<R>(le, in, lev) + box * p + n;
  C acc = *out;
  for (int k = n; k < p; ++k) cfma(acc, b[k], lp[k]);
  *out = acc;
}

__global__ void __launch_bounds__(256) k_b_l2l(const BatchInst* __restrict__ I,
                                               const int64_t* __restrict__ items, int count,
                                               int lev, char* le, const char* tab,
                                               const int64_t* __restrict__ tab_off) {
  const int64_t t = blockIdx.x * 256LL + threadIdx.x;
  if (t >= items[count]) return;
  const int c = find_seg(items, count, t);
  const BatchInst in = I[c];
  const int64_t item = t - items[c];
  if (in.fp64) l2l_item<double>(in, lev, item, le, tab, tab_off);
  else l2l_item<float>(in, lev, item, le, tab, tab_off);
}

// M2L on the matrix cores in float32: one workgroup per 32-box tile.
// Segment s = one (instance, level) pair, its tiles seg_off[s] .. seg_off[s+1)
// (4 classes x ceil(4^(lev-1) / 32) tiles), seg_il[s] = instance << 8 | level.
// MT = 1: the instances with p <= 16, on their float32 coefficients; MT = 2:
// the instances with p > 16 (2p <= 48 rows in two 32-row tiles), on the float32
// copies of their float64 multipoles (k_b_convert, narrow), into float32
// locals that k_b_convert (widen) adds to the float64 L2L chain.
template <int MT>
__global__ void __launch_bounds__(256) k_b_m2l_mfma(const BatchInst* __restrict__ I,
                                                    const int64_t* __restrict__ seg_off,
                                                    const int32_t* __restrict__ seg_il, int nseg,
                                                    char* me, char* le, const char* tab,
                                                    const int64_t* __restrict__ tab_off) {
  __shared__ M2LTileLds<MT> sh;
  const int64_t tile = blockIdx.x;
  const int s = __builtin_amdgcn_readfirstlane(find_seg(seg_off, nseg, tile));
  const int il = __builtin_amdgcn_readfirstlane(seg_il[s]);
  const int c = il >> 8, lev = il & 255;
  const BatchInst in = I[c];
  const int p = __builtin_amdgcn_readfirstlane(in.p);
  const float* A = reinterpret_cast<const float*>(tab + tab_off[p] + ops_layout(p).mfma32);
  if constexpr (MT == 1)
    m2l_f32_tile<1>(coef<float>(me, in, lev), coef<float>(le, in, lev), lev, p,
                    int(tile - seg_off[s]), A, sh);
  else
    m2l_f32_tile<MT>(coef32(me, in, lev), coef32(le, in, lev), lev, p, int(tile - seg_off[s]),
                     A, sh);
}

// The p > 16 instances: every level's float64 multipoles rounded to float32
// (narrow = true: me -> me32) or every level's float32 M2L sums widened into
// the float64 locals (narrow = false: le32 -> le), before the float64 L2L chain
// adds the shifted parent expansions.  Items: their coefficients of levels
// 2 .. L, instance by instance (items[c] .. items[c + 1]).
__global__ void __launch_bounds__(256) k_b_convert(const BatchInst* __restrict__ I,
                                                   const int64_t* __restrict__ items, int count,
                                                   bool narrow, char* wide, char* thin) {
  const int64_t t = blockIdx.x * 256LL + threadIdx.x;
  if (t >= items[count]) return;
  const int c = find_seg(items, count, t);
  const BatchInst in = I[c];
  const int64_t k = t - items[c];
  double2* w = reinterpret_cast<double2*>(wide + in.me_off) + level_offset(2) * in.p + k;
  float2* f = reinterpret_cast<float2*>(thin + in.me32_off) + level_offset(2) * in.p + k;
  if (narrow) {
    const double2 v = *w;
    *f = make_float2(float(v.x), float(v.y));
  } else {
    const float2 v = *f;
    *w = make_double2(double(v.x), double(v.y));
  }
}

// ------------------------------------------------------------------ near field + evaluation

// zx, zy: leaf-local target in units of the Gaussian width, wsd the leaf side
// in the same units, w in plain units.
template <typename R>
__device__ __forceinline__ void l2p_eval(const BatchInst& in, const char* le, int leaf, float zx,
                                         float zy, double wsd, double w, double& fu, double& fv) {
  using C = typename Types<R>::C;
  const R inv_w = R(1.0 / wsd);
  const C z = cmake<C>(R(zx) * inv_w, R(zy) * inv_w);
  const C* Lc = reinterpret_cast<const C*>(le + in.me_off) + level_offset(in.L) * in.p +
                int64_t(leaf) * in.p;
  C acc = cmake<C>(R(0), R(0));
  for (int k = in.p - 1; k >= 0; --k) {
    const C lk = Lc[k];
    acc = cmul(acc, z);
    acc.x += lk.x;
    acc.y += lk.y;
  }
  const double sc = kInv2Pi / w;
  fu = double(acc.y) * sc;
  fv = double(acc.x) * sc;
}

// Circulation-free kernel values of the symmetric pairs (r'^2 in units of the
// Gaussian width).
struct BatchSymK {
  __device__ __forceinline__ float hnear(float r2) const { return P2PMath<float>::h_near_s(r2); }
  __device__ __forceinline__ float hseries(float r2) const { return P2PMath<float>::h_series_s(r2); }
  __device__ __forceinline__ float hfar(float r2) const { return P2PMath<float>::h_far(r2); }
};

// SYM: the launch holds instances with the symmetric near field
// (p2p_math.hpp; BatchInst::sym): of its 3 x 3 local list a tile of such an
// instance takes the neighbours after its leaf in (row, leaf) order -- E, NW,
// N, NE -- and, in its own leaf, the chunks from its own on; each pair of
// different chunks adds the opposite contributions to react (the other
// neighbours' and the earlier chunks' pairs reach the tile that way).  A
// symmetric chunk pair always takes 64 steps, so only instances with well
// filled leaves use it (set at plan creation).
template <bool SYM>
__global__ void __launch_bounds__(256) k_b_p2p(const BatchInst* __restrict__ I,
                                               const Part32* __restrict__ part,
                                               const int32_t* __restrict__ start,
                                               const Tile* __restrict__ tiles,
                                               const int32_t* __restrict__ ntiles,
                                               const uint32_t* __restrict__ tile_off,
                                               const float4* __restrict__ tile_box,
                                               const double* __restrict__ roots,
                                               double2* __restrict__ nearv,
                                               double2* __restrict__ react) {
  extern __shared__ unsigned char b_p2p_lds[];
  const int wid =
      __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
  if (wid >= *ntiles) return;
  const int lane = threadIdx.x & 63;
  const Tile tile = tiles[wid];
  const int c = __builtin_amdgcn_readfirstlane(tile.pad);
  const BatchInst in = I[c];
  const bool active = lane < tile.count;
  const int32_t i = tile.start + (active ? lane : 0);
  const Part32 tp = part[i];
  const int L = in.L, m = 1 << L;
  const int leaf = int(tile.leaf - in.leaf_off);
  const int bx = leaf & (m - 1), by = leaf >> L;
  const double w = roots[4 * c + 3];
  // positions are in units of the Gaussian width: r'^2 = r^2 log2(e) / (2 sigma^2)
  const double sd = near_scale(in.sigma);
  const double wsd = w * sd;
  const float far2 = float(P2PMath<float>::kFarSigma2 * 1.4426950408889634074 / 2.0);
  const float ser2 = float(P2PMath<float>::kSeriesSigma2 * 1.4426950408889634074 / 2.0);
  const float tiny = float(wsd * wsd * 0x1p-80);
  const float4 tb = tile_box[wid];
  SymRec<float>* const sbuf = reinterpret_cast<SymRec<float>*>(b_p2p_lds) + (threadIdx.x >> 6) * 128;
  const bool sym = SYM && __builtin_amdgcn_readfirstlane(in.sym) != 0;
  const float tg = sym && active ? tp.g : 0.f;
  Acc32 au{0.f, 0.f}, av{0.f, 0.f};
  for (int oy = sym ? 0 : -1; oy <= 1; ++oy) {
    const int sy = by + oy;
    if (sy < 0 || sy >= m) continue;
    for (int ox = sym && oy == 0 ? 0 : -1; ox <= 1; ++ox) {
      const int sx = bx + ox;
      if (sx < 0 || sx >= m) continue;
      const int64_t gsl = in.leaf_off + sy * m + sx;
      const int32_t js = start[gsl + c], je = start[gsl + c + 1];
      const bool self_leaf = ox == 0 && oy == 0;
      const int32_t own = sym && self_leaf ? (tile.start - js) >> 6 : 0;
      const float tx = tp.x - float(double(ox) * wsd);
      const float ty = tp.y - float(double(oy) * wsd);
      const float bx0 = tb.x - float(double(ox) * wsd), bx1 = tb.y - float(double(ox) * wsd);
      const float by0 = tb.z - float(double(oy) * wsd), by1 = tb.w - float(double(oy) * wsd);
      uint32_t ci = tile_off[gsl];
      for (int32_t j0 = js; j0 < je; j0 += 64, ++ci) {
        bool sym_pair = sym && !self_leaf;
        if (sym && self_leaf) {
          const int32_t rel = (j0 - js) >> 6;
          if (rel < own) continue;
          sym_pair = rel > own;
        }
        const int32_t j1 = min(j0 + 64, je);
        const float4 sb = tile_box[ci];
        const float gx = fmaxf(0.f, fmaxf(sb.x - bx1, bx0 - sb.y));
        const float gy = fmaxf(0.f, fmaxf(sb.z - by1, by0 - sb.w));
        const float gap2 = gx * gx + gy * gy;
        float cu = 0.f, cv = 0.f;
        if (sym_pair) {
          sym_pair_chunk(sbuf, part, j0, j1, lane, tx, ty, tg, tiny, BatchSymK{},
                         gap2 > far2 ? 2 : (gap2 > ser2 ? 0 : 1), 1.0, react, cu, cv);
        } else if (gap2 > far2) {
#pragma unroll 8
          for (int32_t j = j0; j < j1; ++j) {
            const Part32 s = part[j];
            const float dx = tx - s.x, dy = ty - s.y;
            const float f = P2PMath<float>::far(s.g, dx * dx + dy * dy);
            cu -= f * dy;
            cv += f * dx;
          }
        } else if (gap2 > ser2) {
#pragma unroll 8
          for (int32_t j = j0; j < j1; ++j) {
            const Part32 s = part[j];
            const float dx = tx - s.x, dy = ty - s.y;
            const float f = P2PMath<float>::near_s(s.g, dx * dx + (dy * dy + tiny));
            cu -= f * dy;
            cv += f * dx;
          }
        } else {
#pragma unroll 4
          for (int32_t j = j0; j < j1; ++j) {
            const Part32 s = part[j];
            const float dx = tx - s.x, dy = ty - s.y;
            const float f = P2PMath<float>::near_series_s(s.g, dx * dx + (dy * dy + tiny));
            cu -= f * dy;
            cv += f * dx;
          }
        }
        au.add(cu);
        av.add(cv);
      }
    }
  }
  // the near sums in the kernel's units (the L2P kernel scales them)
  if (active) nearv[i] = make_double2(au.value(), av.value());
}

__global__ void __launch_bounds__(256) k_b_zero2(double2* __restrict__ a, int64_t n) {
  for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n; i += int64_t(gridDim.x) * 256)
    a[i] = make_double2(0.0, 0.0);
}

// One wave per tile, after the near field and the expansion sweeps: the near
// sums of k_b_p2p scaled to velocities (each pair term is
// Gamma (...) d' / r'^2 = (1 / sd) Gamma (...) d / r^2) plus the far field (L2P),
// in one fused multiply-add, written in the instance's input order.
__device__ __forceinline__ void b_l2p_tile(int wid, int lane, const BatchInst* __restrict__ I,
                                           const Part32* __restrict__ part,
                                           const Tile* __restrict__ tiles,
                                           const double* __restrict__ roots,
                                           const char* __restrict__ le,
                                           const double2* __restrict__ nearv,
                                           const double2* __restrict__ react,
                                           const int32_t* __restrict__ perm) {
  const Tile tile = tiles[wid];
  if (lane >= tile.count) return;
  const int c = __builtin_amdgcn_readfirstlane(tile.pad);
  const BatchInst in = I[c];
  const int32_t i = tile.start + lane;
  double fu = 0.0, fv = 0.0;
  if (in.L >= 2) {
    const Part32 tp = part[i];
    const int leaf = int(tile.leaf - in.leaf_off);
    const double w = roots[4 * c + 3];
    const double wsd = w * near_scale(in.sigma);
    if (in.fp64) l2p_eval<double>(in, le, leaf, tp.x, tp.y, wsd, w, fu, fv);
    else l2p_eval<float>(in, le, leaf, tp.x, tp.y, wsd, w, fu, fv);
  }
  double2 q = nearv[i];
  if (react) {  // the symmetric pairs' contributions to this particle as a source
    const double2 r = react[i];
    q.x += r.x;
    q.y += r.y;
  }
  const double k = kInv2Pi * near_scale(in.sigma);
  const int64_t o = int64_t(perm[i]) - in.part_off;
  in.u[o] = __builtin_fma(q.x, k, fu);
  in.v[o] = __builtin_fma(q.y, k, fv);
}

// b_l2p_tile for every tile, the waves looping over the tiles.
__global__ void __launch_bounds__(256) k_b_l2p(const BatchInst* __restrict__ I,
                                               const Part32* __restrict__ part,
                                               const Tile* __restrict__ tiles,
                                               const int32_t* __restrict__ ntiles,
                                               const double* __restrict__ roots,
                                               const char* __restrict__ le,
                                               const double2* __restrict__ nearv,
                                               const double2* __restrict__ react,
                                               const int32_t* __restrict__ perm) {
  const int nt = *ntiles;
  const int lane = threadIdx.x & 63;
  for (int wid = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6)); wid < nt;
       wid += 4 * gridDim.x)
    b_l2p_tile(wid, lane, I, part, tiles, roots, le, nearv, react, perm);
}

}  // namespace

// ------------------------------------------------------------------ host plan

struct BatchPlanDev {
  BatchInst* inst;
  int64_t *part_off, *leaf_off, *ls_off, *tab_off;
  int64_t* m2m_items;  // [kBatchMaxLevels + 1][count + 1]
  int64_t* l2l_items;
  int64_t* seg_off;  // matrix-core M2L: first tile of each (instance, level), FP32
  int32_t* seg_il;
  int64_t* seg_off64;  // and of the p > 16 instances (two 32-row tiles)
  int32_t* seg_il64;
  double* roots;
  uint32_t *k0, *k1, *counts, *tmp, *toff;
  int32_t *i0, *i1, *start, *ntiles;
  int2* big;      // leaves of more than kTile particles (global leaf, instance)
  int32_t* nbig;  // their number
  Tile* tiles;
  float4* tile_box;
  Part32* p32;
  Part32* raw;  // the records in input order (sort phase)
  char *me, *le, *tab;
  char *me32, *le32;    // float32 copies of the p > 16 instances' coefficients
  int64_t* w64_items;   // [count + 1]: their coefficients of levels 2 .. L, cumulated
  double2* nearv;  // near field of every particle, sorted order
  double2* react;  // symmetric near field (NULL: off): the pairs' sums added to their sources
};

// The sort, leaf ranges and particle records, then the expansion sweeps on the
// side stream sw (after an event recorded on st) while st builds the tiles and
// runs the near field; st waits for the sweeps before L2P.  Captured into a
// graph, the two streams become two branches.
hipError_t batch_launch_all(const BatchPlanDev& d, int count, int64_t ntot, int64_t nleaves,
                            int64_t max_tiles, const int64_t* m2m_tot, const int64_t* l2l_tot,
                            int maxL, int nseg, int64_t mfma_tiles, int nseg64,
                            int64_t mfma_tiles64, int64_t w64_tot, hipStream_t st, hipStream_t sw,
                            hipEvent_t fork, hipEvent_t join) {
  auto nb = [](int64_t n, int b) { return unsigned((n + b - 1) / b); };
  hipLaunchKernelGGL(k_b_bbox, dim3(count), dim3(256), 0, st, d.inst, d.roots, d.nbig);
  hipLaunchKernelGGL(k_b_keys, dim3(nb(ntot, 256)), dim3(256), 0, st, d.inst, d.part_off, count,
                     ntot, d.roots, d.k0, d.i0, d.raw);
  uint32_t* k0 = d.k0; uint32_t* k1 = d.k1;
  int32_t* i0 = d.i0; int32_t* i1 = d.i1;
  int ibits = 1;
  while ((1 << ibits) < count) ++ibits;
  hipError_t e = radix_sort_pairs(k0, k1, i0, i1, ntot, kBatchKeyInst + ibits, d.counts, d.tmp, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_b_leaf_start, dim3(nb(nleaves + count, 256)), dim3(256), 0, st, d.ls_off,
                     count, k0, ntot, d.start);
  hipLaunchKernelGGL(k_b_local, dim3(nb(ntot, 256)), dim3(256), 0, st, d.raw, i0, ntot, d.p32);
  e = hipEventRecord(fork, st);
  if (e == hipSuccess) e = hipStreamWaitEvent(sw, fork, 0);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_b_p2m, dim3(nb(nleaves, 256)), dim3(256), 0, sw, d.inst, d.leaf_off, count,
                     d.start, d.p32, d.roots, d.me, d.big, d.nbig);
  hipLaunchKernelGGL(k_b_p2m_big, dim3(nb(ntot / (kTile + 1) + 1, 4)), dim3(256), 0, sw, d.inst,
                     d.start, d.p32, d.roots, d.me, d.big, d.nbig);
  for (int l = maxL - 1; l >= 2; --l)
    if (m2m_tot[l] > 0)
      hipLaunchKernelGGL(k_b_m2m, dim3(nb(m2m_tot[l], 256)), dim3(256), 0, sw, d.inst,
                         d.m2m_items + int64_t(l) * (count + 1), count, l, d.me, d.tab, d.tab_off);
  if (mfma_tiles > 0)
    hipLaunchKernelGGL(k_b_m2l_mfma<1>, dim3(unsigned(mfma_tiles)), dim3(256), 0, sw, d.inst,
                       d.seg_off, d.seg_il, nseg, d.me, d.le, d.tab, d.tab_off);
  if (mfma_tiles64 > 0) {
    // p > 16: float64 shifts, M2L in float32 on the matrix cores
    hipLaunchKernelGGL(k_b_convert, dim3(nb(w64_tot, 256)), dim3(256), 0, sw, d.inst, d.w64_items,
                       count, true, d.me, d.me32);
    hipLaunchKernelGGL(k_b_m2l_mfma<2>, dim3(unsigned(mfma_tiles64)), dim3(256), 0, sw, d.inst,
                       d.seg_off64, d.seg_il64, nseg64, d.me32, d.le32, d.tab, d.tab_off);
    hipLaunchKernelGGL(k_b_convert, dim3(nb(w64_tot, 256)), dim3(256), 0, sw, d.inst, d.w64_items,
                       count, false, d.le, d.le32);
  }
  for (int l = 3; l <= maxL; ++l)
    if (l2l_tot[l] > 0)
      hipLaunchKernelGGL(k_b_l2l, dim3(nb(l2l_tot[l], 256)), dim3(256), 0, sw, d.inst,
                         d.l2l_items + int64_t(l) * (count + 1), count, l, d.le, d.tab,
                         d.tab_off);
  e = hipEventRecord(join, sw);
  if (e != hipSuccess) return e;
  // the near-field tiles, beside the sweeps
  hipLaunchKernelGGL(k_b_tile_counts, dim3(nb(nleaves + 1, 256)), dim3(256), 0, st, d.leaf_off,
                     count, d.start, d.toff);
  e = scan_exclusive(d.toff, nleaves + 1, d.tmp, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_b_tile_fill, dim3(nb(ntot, 256)), dim3(256), 0, st, d.inst, k0, d.start,
                     d.toff, ntot, nleaves, d.tiles, d.ntiles);
  e = launch_tile_box(d.tiles, d.ntiles, max_tiles, d.p32, d.tile_box, st);
  if (e != hipSuccess) return e;
  if (d.react) {
    hipLaunchKernelGGL(k_b_zero2, dim3(nb(ntot, 256) < 4096 ? nb(ntot, 256) : 4096u), dim3(256), 0,
                       st, d.react, ntot);
    hipLaunchKernelGGL(k_b_p2p<true>, dim3(nb(max_tiles, kBatchP2PWaves)),
                       dim3(64 * kBatchP2PWaves), kBatchP2PWaves * 128 * sizeof(SymRec<float>), st,
                       d.inst, d.p32, d.start, d.tiles, d.ntiles, d.toff, d.tile_box, d.roots,
                       d.nearv, d.react);
  } else {
    hipLaunchKernelGGL(k_b_p2p<false>, dim3(nb(max_tiles, kBatchP2PWaves)),
                       dim3(64 * kBatchP2PWaves), 0, st, d.inst, d.p32, d.start, d.tiles, d.ntiles,
                       d.toff, d.tile_box, d.roots, d.nearv, nullptr);
  }
  e = hipStreamWaitEvent(st, join, 0);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_b_l2p, dim3(tile_loop_blocks(max_tiles)), dim3(256), 0, st, d.inst,
                     d.p32, d.tiles, d.ntiles, d.roots, d.le, d.nearv, d.react, i0);
  return hipGetLastError();
}


}  // namespace vfmm

using namespace vfmm;

struct vfmm_batch_s {
  int count;
  int64_t ntot, nleaves, max_tiles;
  int maxL;
  int64_t m2m_tot[kBatchMaxLevels + 1], l2l_tot[kBatchMaxLevels + 1];
  int nseg, nseg64;              // (instance, level) segments of the matrix-core M2L
  int64_t mfma_tiles, mfma_tiles64;  // their tiles (workgroups), p <= 16 and p > 16
  int64_t w64_tot;               // coefficients of the p > 16 instances (float32 copies)
  std::vector<int> ps;  // distinct expansion orders
  int64_t tab_at[VFMM_MAX_P + 1];  // byte offset of each order's table set
  BatchPlanDev d;
  bool tables_built;
  hipGraph_t graph;
  hipGraphExec_t exec;
  // the expansion sweeps run on `side` (default priority) beside the near field
  hipStream_t side;
  hipEvent_t fork, join;
  // recorded on the caller's stream at the end of every run: the plan is
  // released only once its last run has finished
  hipEvent_t done;
  bool ran;  // a run has been enqueued (the roots of the last one are in d.roots)
  std::vector<double> sigma;  // per instance, for vfmm_batch_substitution_bounds
  std::vector<int> levels;
  ~vfmm_batch_s() {
    if (done) (void)hipEventSynchronize(done);
    if (side) (void)hipStreamSynchronize(side);
    if (done) (void)hipEventDestroy(done);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (side) (void)hipStreamDestroy(side);
  }
};

namespace {

vfmm_status_t bfail(vfmm_status_t s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
vfmm_status_t bfail(vfmm_status_t s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  set_last_error(buf);
  return s;
}

inline size_t al(size_t b) { return (b + 255) & ~size_t(255); }

struct BatchLayout {
  size_t inst, part_off, leaf_off, ls_off, tab_off, m2m_items, l2l_items, seg_off, seg_il,
      seg_off64, seg_il64, roots, k0, k1, i0, i1,
      counts, tmp, toff, start, ntiles, big, nbig, tiles, tile_box, p32, raw, me, le, tab, me32, le32,
      w64_items, nearv, react, total;
  int64_t ntot, nleaves, max_tiles, me_bytes, me32_bytes, tab_bytes;
  int maxL;
  std::vector<int64_t> me_off, me32_off;
  int64_t tab_at[VFMM_MAX_P + 1];
};

vfmm_status_t check_instances(const vfmm_instance* in, int count) {
  static_assert(kBatchMaxCount <= (1 << (32 - kBatchKeyInst)), "instance index must fit the key");
  if (!in || count < 1 || count > kBatchMaxCount)
    return bfail(VFMM_ERR_INVALID_ARG, "count must be in [1, %d]", kBatchMaxCount);
  int64_t ntot = 0;
  for (int c = 0; c < count; ++c) {
    const vfmm_instance& a = in[c];
    if (!a.x || !a.y || !a.gamma || !a.u || !a.v) return bfail(VFMM_ERR_INVALID_ARG, "instance %d: null pointer", c);
    if (a.n < 1) return bfail(VFMM_ERR_INVALID_ARG, "instance %d: n must be >= 1", c);
    if (!(a.sigma > 0.0) || !std::isfinite(a.sigma)) return bfail(VFMM_ERR_INVALID_ARG, "instance %d: bad sigma", c);
    if (a.p < 1 || a.p > kBatchPMax) return bfail(VFMM_ERR_INVALID_ARG, "instance %d: p out of [1, %d]", c, kBatchPMax);
    if (a.levels < 0 || a.levels > kBatchMaxLevels)
      return bfail(VFMM_ERR_INVALID_ARG, "instance %d: levels out of [0, %d]", c, kBatchMaxLevels);
    ntot += a.n;
  }
  if (ntot > 2147483647LL) return bfail(VFMM_ERR_INVALID_ARG, "too many particles in total");
  return VFMM_OK;
}

BatchLayout batch_layout(const vfmm_instance* in, int count) {
  BatchLayout L{};
  L.me_off.resize(count);
  L.me32_off.resize(count);
  int64_t me = 0, me32 = 0;
  bool has_p[VFMM_MAX_P + 1] = {};
  for (int c = 0; c < count; ++c) {
    const vfmm_instance& a = in[c];
    L.ntot += a.n;
    L.nleaves += int64_t(1) << (2 * a.levels);
    L.max_tiles += (a.n + kTile - 1) / kTile + std::min<int64_t>(a.n, int64_t(1) << (2 * a.levels));
    L.maxL = std::max(L.maxL, int(a.levels));
    L.me_off[c] = me;
    me += int64_t(al(size_t(n_boxes_2_to(a.levels)) * a.p * (a.p > 16 ? 16 : 8)));
    L.me32_off[c] = me32;
    if (a.p > 16) me32 += int64_t(al(size_t(n_boxes_2_to(a.levels)) * a.p * 8));
    has_p[a.p] = true;
  }
  L.me_bytes = me;
  L.me32_bytes = me32;
  int64_t tb = 0;
  for (int p = 0; p <= VFMM_MAX_P; ++p) {
    L.tab_at[p] = tb;
    if (has_p[p]) tb += int64_t(al(ops_bytes(p)));
  }
  L.tab_bytes = tb;
  const int64_t sort_blocks = (L.ntot + kSortPerBlock - 1) / kSortPerBlock;
  const int64_t scan_src = std::max<int64_t>(256 * sort_blocks, L.nleaves + 1);
  size_t off = 0;
  auto take = [&](size_t b) { size_t r = off; off += al(b); return r; };
  L.inst = take(sizeof(BatchInst) * count);
  L.part_off = take(8 * (count + 1));
  L.leaf_off = take(8 * (count + 1));
  L.ls_off = take(8 * (count + 1));
  L.tab_off = take(8 * (VFMM_MAX_P + 1));
  L.m2m_items = take(8 * size_t(kBatchMaxLevels + 1) * (count + 1));
  L.l2l_items = take(8 * size_t(kBatchMaxLevels + 1) * (count + 1));
  L.seg_off = take(8 * (size_t(kBatchMaxLevels) * count + 1));
  L.seg_il = take(4 * size_t(kBatchMaxLevels) * count);
  L.seg_off64 = take(8 * (size_t(kBatchMaxLevels) * count + 1));
  L.seg_il64 = take(4 * size_t(kBatchMaxLevels) * count);
  L.roots = take(32 * size_t(count));
  L.k0 = take(4 * L.ntot); L.k1 = take(4 * L.ntot);
  L.i0 = take(4 * L.ntot); L.i1 = take(4 * L.ntot);
  L.counts = take(4 * 256 * size_t(sort_blocks));
  L.tmp = take(4 * size_t((scan_src + kScanPerBlock - 1) / kScanPerBlock + 1));
  L.toff = take(4 * size_t(L.nleaves + 1));
  L.start = take(4 * size_t(L.nleaves + count));
  L.ntiles = take(4);
  L.big = take(sizeof(int2) * size_t(L.ntot / (kTile + 1) + 1));
  L.nbig = take(4);
  L.tiles = take(sizeof(Tile) * size_t(L.max_tiles));
  L.tile_box = take(sizeof(float4) * size_t(L.max_tiles));
  L.p32 = take(sizeof(Part32) * size_t(L.ntot));
  L.raw = take(sizeof(Part32) * size_t(L.ntot));
  L.me = take(size_t(L.me_bytes));
  L.le = take(size_t(L.me_bytes));
  L.tab = take(size_t(L.tab_bytes));
  L.me32 = take(size_t(L.me32_bytes));
  L.le32 = take(size_t(L.me32_bytes));
  L.w64_items = take(8 * size_t(count + 1));
  L.nearv = take(sizeof(double2) * size_t(L.ntot));
  L.react = take(sizeof(double2) * size_t(L.ntot));
  L.total = off;
  return L;
}

}  // namespace

extern "C" {

static vfmm_status_t vfmm_batch_workspace_bytes_impl(const vfmm_instance* inst, int32_t count, size_t* bytes) {
  if (!bytes) return bfail(VFMM_ERR_INVALID_ARG, "bytes is NULL");
  vfmm_status_t s = check_instances(inst, count);
  if (s) return s;
  *bytes = batch_layout(inst, count).total;
  return VFMM_OK;
}

static vfmm_status_t vfmm_batch_create_impl(const vfmm_instance* inst, int32_t count, void* workspace,
                                size_t ws_bytes, vfmm_batch_t* out) {
  if (!out) return bfail(VFMM_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  vfmm_status_t s = check_instances(inst, count);
  if (s) return s;
  if (!workspace) return bfail(VFMM_ERR_INVALID_ARG, "workspace is NULL");
  const BatchLayout L = batch_layout(inst, count);
  if (ws_bytes < L.total) return bfail(VFMM_ERR_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, L.total);
  if (reinterpret_cast<uintptr_t>(workspace) & 255) return bfail(VFMM_ERR_WORKSPACE, "workspace must be 256-byte aligned");
  // host tables
  std::vector<BatchInst> hi(count);
  std::vector<int64_t> part_off(count + 1), leaf_off(count + 1), ls_off(count + 1), tab_off(VFMM_MAX_P + 1);
  std::vector<int64_t> m2m(size_t(kBatchMaxLevels + 1) * (count + 1), 0), l2l(size_t(kBatchMaxLevels + 1) * (count + 1), 0);
  // symmetric near field (VFMM_TUNE_P2P_SYMMETRIC) for the instances with at
  // least kBatchSymMinPPL particles per leaf on average: a symmetric chunk
  // pair takes 64 steps however few particles its chunks hold, while one
  // direction at a time takes one step per particle
  const bool sym = tuning_sym() != 0;
  bool any_sym = false;
  for (int c = 0; c < count; ++c) {
    const vfmm_instance& a = inst[c];
    part_off[c + 1] = part_off[c] + a.n;
    leaf_off[c + 1] = leaf_off[c] + (int64_t(1) << (2 * a.levels));
    ls_off[c] = leaf_off[c] + c;
    const int32_t isym = sym && a.n >= (int64_t(kBatchSymMinPPL) << (2 * a.levels)) ? 1 : 0;
    any_sym = any_sym || isym;
    hi[c] = BatchInst{a.x, a.y, a.gamma, a.u, a.v, a.n, part_off[c], leaf_off[c], L.me_off[c],
                      L.me32_off[c], a.sigma, a.p, a.levels, a.p > 16 ? 1 : 0, isym};
  }
  ls_off[count] = leaf_off[count] + count;
  for (int p = 0; p <= VFMM_MAX_P; ++p) tab_off[p] = L.tab_at[p];
  std::vector<double> sig(count);
  std::vector<int> lev(count);
  for (int c = 0; c < count; ++c) {
    sig[c] = inst[c].sigma;
    lev[c] = inst[c].levels;
  }
  vfmm_batch_s* b = new (std::nothrow) vfmm_batch_s{};
  if (!b) return bfail(VFMM_ERR_OUT_OF_MEMORY, "host allocation failed");
  hipError_t es = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
  if (es == hipSuccess) es = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  if (es == hipSuccess) es = hipEventCreateWithFlags(&b->join, hipEventDisableTiming);
  if (es == hipSuccess) es = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
  if (es != hipSuccess) {
    delete b;
    return bfail(hip_status(es), "batch stream / events: %s", hipGetErrorString(es));
  }
  for (int p = 0; p <= VFMM_MAX_P; ++p) b->tab_at[p] = L.tab_at[p];
  b->count = count;
  b->sigma.swap(sig);
  b->levels.swap(lev);
  b->ntot = L.ntot;
  b->nleaves = L.nleaves;
  b->max_tiles = L.max_tiles;
  b->maxL = L.maxL;
  for (int l = 0; l <= kBatchMaxLevels; ++l) {
    int64_t a = 0, bb = 0;
    for (int c = 0; c < count; ++c) {
      m2m[size_t(l) * (count + 1) + c] = a;
      l2l[size_t(l) * (count + 1) + c] = bb;
      const int64_t items = (int64_t(1) << (2 * l)) * inst[c].p;
      if (l >= 2 && inst[c].levels > l) a += items;
      if (l >= 3 && inst[c].levels >= l) bb += items;
    }
    m2m[size_t(l) * (count + 1) + count] = a;
    l2l[size_t(l) * (count + 1) + count] = bb;
    b->m2m_tot[l] = a;
    b->l2l_tot[l] = bb;
  }
  std::vector<int64_t> seg_off(1, 0), seg_off64(1, 0), w64(count + 1, 0);
  std::vector<int32_t> seg_il, seg_il64;
  for (int c = 0; c < count; ++c) {
    const bool f64 = inst[c].p > 16;
    w64[c + 1] = w64[c] + (f64 ? n_boxes_2_to(inst[c].levels) * inst[c].p : 0);
    const int bw = 32;  // boxes per tile
    std::vector<int64_t>& so = f64 ? seg_off64 : seg_off;
    std::vector<int32_t>& si = f64 ? seg_il64 : seg_il;
    for (int l = 2; l <= inst[c].levels; ++l) {
      si.push_back(int32_t(c) << 8 | l);
      so.push_back(so.back() + 4 * (((int64_t(1) << (2 * (l - 1))) + bw - 1) / bw));
    }
  }
  b->nseg = int(seg_il.size());
  b->mfma_tiles = seg_off.back();
  b->nseg64 = int(seg_il64.size());
  b->mfma_tiles64 = seg_off64.back();
  b->w64_tot = w64[count];
  for (int c = 0; c < count; ++c) {
    bool seen = false;
    for (int q : b->ps) seen |= q == inst[c].p;
    if (!seen) b->ps.push_back(inst[c].p);
  }
  char* ws = static_cast<char*>(workspace);
  BatchPlanDev& d = b->d;
  d.inst = reinterpret_cast<BatchInst*>(ws + L.inst);
  d.part_off = reinterpret_cast<int64_t*>(ws + L.part_off);
  d.leaf_off = reinterpret_cast<int64_t*>(ws + L.leaf_off);
  d.ls_off = reinterpret_cast<int64_t*>(ws + L.ls_off);
  d.tab_off = reinterpret_cast<int64_t*>(ws + L.tab_off);
  d.m2m_items = reinterpret_cast<int64_t*>(ws + L.m2m_items);
  d.l2l_items = reinterpret_cast<int64_t*>(ws + L.l2l_items);
  d.seg_off = reinterpret_cast<int64_t*>(ws + L.seg_off);
  d.seg_il = reinterpret_cast<int32_t*>(ws + L.seg_il);
  d.seg_off64 = reinterpret_cast<int64_t*>(ws + L.seg_off64);
  d.seg_il64 = reinterpret_cast<int32_t*>(ws + L.seg_il64);
  d.roots = reinterpret_cast<double*>(ws + L.roots);
  d.k0 = reinterpret_cast<uint32_t*>(ws + L.k0); d.k1 = reinterpret_cast<uint32_t*>(ws + L.k1);
  d.i0 = reinterpret_cast<int32_t*>(ws + L.i0); d.i1 = reinterpret_cast<int32_t*>(ws + L.i1);
  d.counts = reinterpret_cast<uint32_t*>(ws + L.counts);
  d.tmp = reinterpret_cast<uint32_t*>(ws + L.tmp);
  d.toff = reinterpret_cast<uint32_t*>(ws + L.toff);
  d.start = reinterpret_cast<int32_t*>(ws + L.start);
  d.ntiles = reinterpret_cast<int32_t*>(ws + L.ntiles);
  d.big = reinterpret_cast<int2*>(ws + L.big);
  d.nbig = reinterpret_cast<int32_t*>(ws + L.nbig);
  d.tiles = reinterpret_cast<Tile*>(ws + L.tiles);
  d.tile_box = reinterpret_cast<float4*>(ws + L.tile_box);
  d.p32 = reinterpret_cast<Part32*>(ws + L.p32);
  d.raw = reinterpret_cast<Part32*>(ws + L.raw);
  d.me = ws + L.me;
  d.le = ws + L.le;
  d.tab = ws + L.tab;
  d.me32 = ws + L.me32;
  d.le32 = ws + L.le32;
  d.w64_items = reinterpret_cast<int64_t*>(ws + L.w64_items);
  d.nearv = reinterpret_cast<double2*>(ws + L.nearv);
  d.react = any_sym ? reinterpret_cast<double2*>(ws + L.react) : nullptr;
  hipError_t e = hipMemcpy(d.inst, hi.data(), sizeof(BatchInst) * count, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d.part_off, part_off.data(), 8 * (count + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d.leaf_off, leaf_off.data(), 8 * (count + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d.ls_off, ls_off.data(), 8 * (count + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d.tab_off, tab_off.data(), 8 * (VFMM_MAX_P + 1), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d.m2m_items, m2m.data(), 8 * m2m.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d.l2l_items, l2l.data(), 8 * l2l.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d.seg_off, seg_off.data(), 8 * seg_off.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !seg_il.empty())
    e = hipMemcpy(d.seg_il, seg_il.data(), 4 * seg_il.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d.seg_off64, seg_off64.data(), 8 * seg_off64.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && !seg_il64.empty())
    e = hipMemcpy(d.seg_il64, seg_il64.data(), 4 * seg_il64.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d.w64_items, w64.data(), 8 * w64.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    delete b;
    return bfail(hip_status(e), "batch tables: %s", hipGetErrorString(e));
  }
  *out = b;
  return VFMM_OK;
}

vfmm_status_t vfmm_batch_run(vfmm_batch_t b, int32_t use_graph, void* stream) {
  if (!b) return bfail(VFMM_ERR_INVALID_ARG, "batch is NULL");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (use_graph && !st) return bfail(VFMM_ERR_UNSUPPORTED, "graph replay needs a non-default stream");
  hipError_t e = hipSuccess;
  if (!b->tables_built) {
    for (int p : b->ps) {
      TreeDev t{};
      t.ops = b->d.tab + b->tab_at[p];  // translation tables of order p
      e = launch_build_ops(t, p, kFP64, st);
      if (e == hipSuccess) e = launch_pack_m2l_mfma(t, p, kFP32, st);
      if (e != hipSuccess) break;
    }
    if (e != hipSuccess) return bfail(hip_status(e), "batch tables: %s", hipGetErrorString(e));
    b->tables_built = true;
  }
  if (!use_graph) {
    e = batch_launch_all(b->d, b->count, b->ntot, b->nleaves, b->max_tiles, b->m2m_tot, b->l2l_tot,
                         b->maxL, b->nseg, b->mfma_tiles, b->nseg64, b->mfma_tiles64,
                         b->w64_tot, st, b->side, b->fork, b->join);
    if (e == hipSuccess) e = hipEventRecord(b->done, st);
    if (e == hipSuccess) b->ran = true;
    return e == hipSuccess ? VFMM_OK : bfail(hip_status(e), "batch run: %s", hipGetErrorString(e));
  }
  if (!b->exec) {
    e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return bfail(hip_status(e), "begin capture: %s", hipGetErrorString(e));
    hipError_t le = batch_launch_all(b->d, b->count, b->ntot, b->nleaves, b->max_tiles, b->m2m_tot,
                                     b->l2l_tot, b->maxL, b->nseg, b->mfma_tiles, b->nseg64,
                                     b->mfma_tiles64, b->w64_tot, st, b->side, b->fork, b->join);
    e = hipStreamEndCapture(st, &b->graph);
    if (le != hipSuccess || e != hipSuccess)
      return bfail(hip_status(le != hipSuccess ? le : e), "capture: %s", hipGetErrorString(le != hipSuccess ? le : e));
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return bfail(hip_status(e), "instantiate: %s", hipGetErrorString(e));
  }
  e = hipGraphLaunch(b->exec, st);
  if (e == hipSuccess) e = hipEventRecord(b->done, st);
  if (e == hipSuccess) b->ran = true;
  return e == hipSuccess ? VFMM_OK : bfail(hip_status(e), "graph launch: %s", hipGetErrorString(e));
}

void vfmm_batch_destroy(vfmm_batch_t b) { delete b; }

// Every instance uses the paper's split, so its substitution distance is its
// leaf side, known once the last run has computed the bounding squares.
static vfmm_status_t batch_bounds_impl(vfmm_batch_t b, double* bound) {
  if (!b || !bound) return bfail(VFMM_ERR_INVALID_ARG, "null pointer");
  if (!b->ran) return bfail(VFMM_ERR_INVALID_ARG, "the batch has not run yet");
  hipError_t e = hipEventSynchronize(b->done);
  std::vector<double> r(size_t(b->count) * 4);
  if (e == hipSuccess)
    e = hipMemcpy(r.data(), b->d.roots, r.size() * sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return bfail(hip_status(e), "batch roots: %s", hipGetErrorString(e));
  for (int c = 0; c < b->count; ++c) {
    const vfmm_status_t s =
        vfmm_substitution_bound(r[4 * size_t(c) + 2], b->levels[c], b->sigma[c], 0.0, VFMM_FP32,
                                nullptr, bound + c);
    if (s) return s;
  }
  return VFMM_OK;
}

vfmm_status_t vfmm_batch_substitution_bounds(vfmm_batch_t b, double* bound) {
  try {
    return batch_bounds_impl(b, bound);
  } catch (const std::bad_alloc&) {
    return bfail(VFMM_ERR_OUT_OF_MEMORY, "vfmm_batch_substitution_bounds: host allocation failed");
  }
}

vfmm_status_t vfmm_fmm_velocity_batched(const vfmm_instance* inst, int32_t count, void* workspace,
                                        size_t ws_bytes, void* stream) {
  vfmm_batch_t b = nullptr;
  vfmm_status_t s = vfmm_batch_create(inst, count, workspace, ws_bytes, &b);
  if (s) return s;
  s = vfmm_batch_run(b, 0, stream);
  vfmm_batch_destroy(b);
  return s;
}

// Host allocations inside (std::vector) report running out of memory as a
// status instead of letting the exception cross the C ABI.
vfmm_status_t vfmm_batch_workspace_bytes(const vfmm_instance* inst, int32_t count, size_t* bytes) {
  try {
    return vfmm_batch_workspace_bytes_impl(inst, count, bytes);
  } catch (const std::bad_alloc&) {
    return bfail(VFMM_ERR_OUT_OF_MEMORY, "vfmm_batch_workspace_bytes: host allocation failed");
  }
}

// Host allocations inside (std::vector) report running out of memory as a
// status instead of letting the exception cross the C ABI.
vfmm_status_t vfmm_batch_create(const vfmm_instance* inst, int32_t count, void* workspace, size_t ws_bytes,
                                vfmm_batch_t* out) {
  try {
    return vfmm_batch_create_impl(inst, count, workspace, ws_bytes, out);
  } catch (const std::bad_alloc&) {
    return bfail(VFMM_ERR_OUT_OF_MEMORY, "vfmm_batch_create: host allocation failed");
  }
}

}  // extern "C"
