// Uniform quadtree construction on the GPU (Section 3.3, Fig. 6).
//
// Steps: bounding square of the particles (root box, level 0), sort key of every
// particle, stable LSD radix sort of the keys, leaf ranges by binary search,
// box-local coordinates, and the P2P target tiles (<= 64 consecutive particles
// of one leaf) with their bounding boxes.
//
// Sort key: the row-major leaf index at level L in the high bits, and below it
// the Morton index of the particle's cell at level L + 4 inside the leaf, so a
// leaf's particles are contiguous and a tile of 64 consecutive particles covers
// a compact part of the leaf (ties keep input order).
//
// Leaf convention: ix = clamp(floor(((x - x0) / S) * 2^L), 0, 2^L - 1), the same
// for y; leaf index iy * 2^L + ix.  The root is the bounding square of side
// S = max extent * (1 + 2^-20) centred on the bounding-box midpoint (S = 1 for a
// zero extent), unless the caller gives (x0, y0, S).  These floating-point
// operations are written without contraction so that the integer leaf decision
// is reproducible bit for bit.
#include "vfmm_internal.hpp"

namespace vfmm {

namespace {

__device__ inline double dmin(double a, double b) { return a < b ? a : b; }
__device__ inline double dmax(double a, double b) { return a > b ? a : b; }

__global__ void __launch_bounds__(256) k_bbox_partial(const double* __restrict__ x,
                                                      const double* __restrict__ y, int64_t n,
                                                      double* __restrict__ part) {
  __shared__ double s[4][256];
  double a = INFINITY, b = -INFINITY, c = INFINITY, d = -INFINITY;
  for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x) {
    double xi = x[i], yi = y[i];
    a = dmin(a, xi); b = dmax(b, xi); c = dmin(c, yi); d = dmax(d, yi);
  }
  s[0][threadIdx.x] = a; s[1][threadIdx.x] = b; s[2][threadIdx.x] = c; s[3][threadIdx.x] = d;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (int(threadIdx.x) < st) {
      int o = threadIdx.x + st;
      s[0][threadIdx.x] = dmin(s[0][threadIdx.x], s[0][o]);
      s[1][threadIdx.x] = dmax(s[1][threadIdx.x], s[1][o]);
      s[2][threadIdx.x] = dmin(s[2][threadIdx.x], s[2][o]);
      s[3][threadIdx.x] = dmax(s[3][threadIdx.x], s[3][o]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ void __launch_bounds__(256) k_root(const double* __restrict__ part, int nb,
                                              int has_domain, double dx0, double dy0, double ds,
                                              int levels, double* __restrict__ root) {
#pragma clang fp contract(off)
  __shared__ double s[4][256];
  double a = INFINITY, b = -INFINITY, c = INFINITY, d = -INFINITY;
  for (int i = threadIdx.x; i < nb; i += 256) {
    a = dmin(a, part[4 * i + 0]); b = dmax(b, part[4 * i + 1]);
    c = dmin(c, part[4 * i + 2]); d = dmax(d, part[4 * i + 3]);
  }
  s[0][threadIdx.x] = a; s[1][threadIdx.x] = b; s[2][threadIdx.x] = c; s[3][threadIdx.x] = d;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (int(threadIdx.x) < st) {
      int o = threadIdx.x + st;
      s[0][threadIdx.x] = dmin(s[0][threadIdx.x], s[0][o]);
      s[1][threadIdx.x] = dmax(s[1][threadIdx.x], s[1][o]);
      s[2][threadIdx.x] = dmin(s[2][threadIdx.x], s[2][o]);
      s[3][threadIdx.x] = dmax(s[3][threadIdx.x], s[3][o]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double x0, y0, S;
    if (has_domain) {
      x0 = dx0; y0 = dy0; S = ds;
    } else {
      double xmin = s[0][0], xmax = s[1][0], ymin = s[2][0], ymax = s[3][0];
      double ext = dmax(xmax - xmin, ymax - ymin);
      S = ext > 0.0 ? ext * (1.0 + 0x1p-20) : 1.0;
      x0 = 0.5 * (xmin + xmax) - 0.5 * S;
      y0 = 0.5 * (ymin + ymax) - 0.5 * S;
    }
    root[0] = x0; root[1] = y0; root[2] = S;
    root[3] = S / double(1LL << levels);
  }
}

__device__ inline uint32_t spread4(uint32_t v) {  // bits b3 b2 b1 b0 -> b3 0 b2 0 b1 0 b0
  v &= 15u;
  v = (v | (v << 2)) & 0x33u;
  v = (v | (v << 1)) & 0x55u;
  return v;
}

// Sort key of a point: leaf (row-major) above the Morton index of its cell at
// level L + 4 inside the leaf.
__device__ inline uint32_t point_key(double x, double y, const double* __restrict__ root,
                                     int levels) {
#pragma clang fp contract(off)
  const double x0 = root[0], y0 = root[1], S = root[2];
  const int mf = 1 << (levels + kSubLevels);
  const double scale = double(mf);
  // floor(t 2^(L+4)) >> 4 == floor(t 2^L): the leaf decision is unchanged
  double fx = floor(((x - x0) / S) * scale);
  double fy = floor(((y - y0) / S) * scale);
  // clamped before the conversion; a NaN coordinate goes to cell 0
  const int ix = !(fx >= 0.0) ? 0 : (fx > double(mf - 1) ? mf - 1 : int(fx));
  const int iy = !(fy >= 0.0) ? 0 : (fy > double(mf - 1) ? mf - 1 : int(fy));
  const uint32_t leaf = (uint32_t(iy >> kSubLevels) << levels) | uint32_t(ix >> kSubLevels);
  const uint32_t sub = spread4(uint32_t(ix)) | (spread4(uint32_t(iy)) << 1);
  return (leaf << (2 * kSubLevels)) | sub;
}

// Inside the closed root square (NaN coordinates are outside).
__device__ inline bool in_root(double x, double y, const double* __restrict__ root) {
#pragma clang fp contract(off)
  const double x0 = root[0], y0 = root[1], S = root[2];
  return x >= x0 && x <= x0 + S && y >= y0 && y <= y0 + S;
}

// Sort keys, the identity permutation, and the positions interleaved (one
// 16-byte record per particle, so that the gather after the sort reads one
// record per particle instead of two values from two arrays).
// The sort keys, the identity permutation and the interleaved positions, with
// the first radix pass's digit counts (the key's low 8 bits) of each sort
// block: the workgroups are the sort's (kSortPerBlock consecutive points) and
// the counts go where the counting kernel of that pass would write them.
__global__ void __launch_bounds__(kSortBlock) k_keys(const double* __restrict__ x,
                                                     const double* __restrict__ y, int64_t n,
                                                     const double* __restrict__ root, int levels,
                                                     uint32_t* __restrict__ keys,
                                                     int32_t* __restrict__ idx,
                                                     double2* __restrict__ xy,
                                                     uint32_t* __restrict__ counts, int nblk) {
  __shared__ uint32_t hist[256];
  for (int d = threadIdx.x; d < 256; d += kSortBlock) hist[d] = 0;
  __syncthreads();
  const int64_t base = blockIdx.x * int64_t(kSortPerBlock);
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = base + r * kSortBlock + threadIdx.x;
    if (i < n) {
      const double xi = x[i], yi = y[i];
      const uint32_t k = point_key(xi, yi, root, levels);
      keys[i] = k;
      idx[i] = int32_t(i);
      xy[i] = make_double2(xi, yi);
      atomicAdd(&hist[k & 255u], 1u);
    }
  }
  __syncthreads();
  for (int d = threadIdx.x; d < 256; d += kSortBlock)
    counts[int64_t(d) * nblk + blockIdx.x] = hist[d];
}

// Evaluation points: points outside the root square get key 0 (their
// coordinates become NaN below, so they only produce NaN velocities).
__global__ void __launch_bounds__(256) k_target_keys(const double* __restrict__ x,
                                                     const double* __restrict__ y, int64_t n,
                                                     const double* __restrict__ root, int levels,
                                                     uint32_t* __restrict__ keys,
                                                     int32_t* __restrict__ idx) {
  int64_t i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= n) return;
  const double xi = x[i], yi = y[i];
  keys[i] = in_root(xi, yi, root) ? point_key(xi, yi, root, levels) : 0u;
  idx[i] = int32_t(i);
}

}  // namespace

// ------------------------------------------------------------------ scan
// Exclusive prefix sum of uint32, in place, three phases.

__device__ inline uint32_t wave_incl_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// Block-wide exclusive scan of one value per thread (256 threads); returns the
// exclusive prefix and writes the block total.
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t ws[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t incl = wave_incl_scan(v);
  if (lane == 63) ws[wave] = incl;
  __syncthreads();
  uint32_t pre = 0;
  for (int w = 0; w < wave; ++w) pre += ws[w];
  uint32_t t = ws[0] + ws[1] + ws[2] + ws[3];
  __syncthreads();
  *total = t;
  return pre + incl - v;
}

// Block totals; with gridDim.y = 2 the blocks of row 1 take array a1 and write
// their totals after the nb = gridDim.x of row 0.
__global__ void __launch_bounds__(kScanBlock) k_scan_reduce(const uint32_t* __restrict__ a0,
                                                            const uint32_t* __restrict__ a1,
                                                            int64_t n, uint32_t* __restrict__ tmp) {
  const uint32_t* a = blockIdx.y ? a1 : a0;
  tmp += blockIdx.y * gridDim.x;
  const int64_t base = blockIdx.x * int64_t(kScanPerBlock) + threadIdx.x * int64_t(kScanItems);
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) s += a[base + k];
  uint32_t tot;
  block_excl_scan(s, &tot);
  if (threadIdx.x == 0) tmp[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanBlock) k_scan_tmp(uint32_t* __restrict__ tmp, int64_t nb) {
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nb; base += kScanBlock) {
    int64_t i = base + threadIdx.x;
    uint32_t v = i < nb ? tmp[i] : 0u;
    uint32_t tot;
    uint32_t ex = block_excl_scan(v, &tot);
    uint32_t c = carry;
    if (i < nb) tmp[i] = c + ex;
    __syncthreads();
    if (threadIdx.x == 0) carry = c + tot;
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kScanBlock) k_scan_apply(uint32_t* __restrict__ a, int64_t n,
                                                           const uint32_t* __restrict__ tmp) {
  const int64_t base = blockIdx.x * int64_t(kScanPerBlock) + threadIdx.x * int64_t(kScanItems);
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < n ? a[base + k] : 0u;
    s += v[k];
  }
  uint32_t tot;
  uint32_t ex = block_excl_scan(s, &tot) + tmp[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) a[base + k] = ex;
    ex += v[k];
  }
}

// As k_scan_apply, with tmp holding the block totals themselves: each block
// adds up the totals of the blocks before it (a fixed order, so the result
// equals the three-phase scan's).  For up to kScanFusedBlocks blocks; rows of
// the grid as in k_scan_reduce.
__global__ void __launch_bounds__(kScanBlock) k_scan_apply_totals(uint32_t* __restrict__ a0,
                                                                  uint32_t* __restrict__ a1,
                                                                  int64_t n,
                                                                  const uint32_t* __restrict__ tmp) {
  uint32_t* a = blockIdx.y ? a1 : a0;
  tmp += blockIdx.y * gridDim.x;
  uint32_t before = 0;
  for (int k = threadIdx.x; k < int(blockIdx.x); k += kScanBlock) before += tmp[k];
  uint32_t pre;
  block_excl_scan(before, &pre);
  const int64_t base = blockIdx.x * int64_t(kScanPerBlock) + threadIdx.x * int64_t(kScanItems);
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < n ? a[base + k] : 0u;
    s += v[k];
  }
  uint32_t tot;
  uint32_t ex = block_excl_scan(s, &tot) + pre;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) a[base + k] = ex;
    ex += v[k];
  }
}

// In-place exclusive scan of n elements by one workgroup (blockIdx.y selects
// the array; 16-byte aligned), with a running carry (uniform over the
// workgroup).
__global__ void __launch_bounds__(kScanOneBlock) k_scan_one(uint32_t* __restrict__ a0,
                                                            uint32_t* __restrict__ a1, int64_t n) {
  __shared__ uint32_t ws[kScanOneBlock / 64];
  uint32_t* a = blockIdx.y ? a1 : a0;
  const int64_t me = int64_t(threadIdx.x) * 4;
  uint32_t carry = 0;
  for (int64_t base = 0; base < n; base += kScanOneRound * kScanOneRounds) {
    uint4 q[kScanOneRounds];
#pragma unroll
    for (int r = 0; r < kScanOneRounds; ++r) q[r] = scan_load4(a, base + r * kScanOneRound + me, n);
#pragma unroll
    for (int r = 0; r < kScanOneRounds; ++r) {
      if (base + r * kScanOneRound >= n) break;  // uniform
      uint32_t tot;
      const uint32_t ex =
          block1k_scan_excl(q[r].x + q[r].y + q[r].z + q[r].w, &tot, ws) + carry;
      scan_store4(a, base + r * kScanOneRound + me, n, q[r], ex);
      carry += tot;
    }
  }
}

constexpr int64_t kScanFusedBlocks = 2048;

// Up to kScanOneMax elements: one workgroup (one launch).  Up to
// kScanFusedBlocks blocks of kScanPerBlock elements: block totals, then one
// pass that scans each block after its predecessors' totals (two launches);
// beyond that the three-phase scan.
hipError_t scan_exclusive(uint32_t* a, int64_t n, uint32_t* tmp, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n <= kScanOneMax && (reinterpret_cast<uintptr_t>(a) & 15) == 0) {
    hipLaunchKernelGGL(k_scan_one, dim3(1), dim3(kScanOneBlock), 0, st, a, a, n);
    return hipGetLastError();
  }
  int64_t nb = (n + kScanPerBlock - 1) / kScanPerBlock;
  if (nb <= kScanFusedBlocks) {
    if (nb > 1) hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanBlock), 0, st, a, a, n, tmp);
    hipLaunchKernelGGL(k_scan_apply_totals, dim3(nb), dim3(kScanBlock), 0, st, a, a, n, tmp);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kScanBlock), 0, st, a, a, n, tmp);
  hipLaunchKernelGGL(k_scan_tmp, dim3(1), dim3(kScanBlock), 0, st, tmp, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3(nb), dim3(kScanBlock), 0, st, a, n, tmp);
  return hipGetLastError();
}

// Two arrays of n elements scanned by the same launches (tmp: 2 nb totals);
// beyond kScanFusedBlocks blocks, one after the other.
hipError_t scan_exclusive2(uint32_t* a, uint32_t* b, int64_t n, uint32_t* tmp, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (n <= kScanOneMax && ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15) == 0) {
    hipLaunchKernelGGL(k_scan_one, dim3(1, 2), dim3(kScanOneBlock), 0, st, a, b, n);
    return hipGetLastError();
  }
  int64_t nb = (n + kScanPerBlock - 1) / kScanPerBlock;
  if (nb > kScanFusedBlocks) {
    hipError_t e = scan_exclusive(a, n, tmp, st);
    return e == hipSuccess ? scan_exclusive(b, n, tmp, st) : e;
  }
  if (nb > 1) hipLaunchKernelGGL(k_scan_reduce, dim3(nb, 2), dim3(kScanBlock), 0, st, a, b, n, tmp);
  hipLaunchKernelGGL(k_scan_apply_totals, dim3(nb, 2), dim3(kScanBlock), 0, st, a, b, n, tmp);
  return hipGetLastError();
}

// ------------------------------------------------------------------ radix sort
// Stable LSD counting sort on `bits` (<= 8) key bits per pass.  counts is
// digit-major: counts[d * nblk + b].

constexpr int kSortWaves = kSortBlock / 64;

__global__ void __launch_bounds__(kSortBlock) k_radix_count(const uint32_t* __restrict__ keys,
                                                            int64_t n, int shift, uint32_t mask,
                                                            uint32_t* __restrict__ counts, int nblk) {
  __shared__ uint32_t hist[256];
  for (int d = threadIdx.x; d < 256; d += kSortBlock) hist[d] = 0;
  __syncthreads();
  const int64_t base = blockIdx.x * int64_t(kSortPerBlock);
#pragma unroll
  for (int r = 0; r < kSortItems; ++r) {
    int64_t i = base + r * kSortBlock + threadIdx.x;
    if (i < n) atomicAdd(&hist[(keys[i] >> shift) & mask], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < 256; d += kSortBlock)
    counts[int64_t(d) * nblk + blockIdx.x] = hist[d];
}

// Each round ranks kSortBlock consecutive keys (one per thread): within a
// wave by ballots over the digit's bits, across the waves of the block by the
// per-wave digit counts in wc; run holds each digit's next output position.
__global__ void __launch_bounds__(kSortBlock) k_radix_scatter(
    const uint32_t* __restrict__ kin, const int32_t* __restrict__ iin, int64_t n, int shift,
    uint32_t mask, int bits, const uint32_t* __restrict__ offs, int nblk,
    uint32_t* __restrict__ kout, int32_t* __restrict__ iout) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wc[kSortWaves][256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int d = tid; d < 256; d += kSortBlock) run[d] = offs[int64_t(d) * nblk + blockIdx.x];
  for (int k = tid; k < kSortWaves * 256; k += kSortBlock) wc[k >> 8][k & 255] = 0;
  __syncthreads();
  const int64_t base = blockIdx.x * int64_t(kSortPerBlock);
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < kSortItems; ++r) {
    const int64_t i = base + r * kSortBlock + tid;
    const bool valid = i < n;
    const uint32_t k = valid ? kin[i] : 0u;
    const int32_t ix = valid ? iin[i] : 0;
    const uint32_t d = (k >> shift) & mask;
    uint64_t m = __ballot(valid);
    for (int b = 0; b < bits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    const uint64_t lower = m & below;
    const uint32_t rank_w = __popcll(lower);
    if (valid && lower == 0) wc[wave][d] = __popcll(m);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[d] + rank_w;
      for (int w = 0; w < wave; ++w) pos += wc[w][d];
      kout[pos] = k;
      iout[pos] = ix;
    }
    __syncthreads();
    for (int dd = tid; dd < 256; dd += kSortBlock) {
      uint32_t s = 0;
#pragma unroll
      for (int w = 0; w < kSortWaves; ++w) {
        s += wc[w][dd];
        wc[w][dd] = 0;
      }
      run[dd] += s;
    }
    __syncthreads();
  }
}

namespace {

// Start of leaf k in the sorted keys: the first position whose leaf is >= k.
__device__ __forceinline__ int64_t leaf_start_of(const uint32_t* __restrict__ keys, int64_t n,
                                                 int64_t k) {
  const uint64_t kk = uint64_t(k) << (2 * kSubLevels);
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (uint64_t(keys[mid]) < kk) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__global__ void __launch_bounds__(256) k_leaf_start(const uint32_t* __restrict__ keys, int64_t n,
                                                    int64_t nleaves, int32_t* __restrict__ start) {
  int64_t k = blockIdx.x * 256LL + threadIdx.x;
  if (k > nleaves) return;
  start[k] = int32_t(leaf_start_of(keys, n, k));
}

// Sorted particle i: its position (through the permutation) relative to its
// leaf's centre, in float64 and float32.
__device__ __forceinline__ void local_coords_of(const double2* __restrict__ xy,
                                                const uint32_t* __restrict__ keys,
                                                const int32_t* __restrict__ perm, int64_t i,
                                                const double* __restrict__ root, int levels,
                                                Part64* __restrict__ p64,
                                                Part32* __restrict__ p32) {
#pragma clang fp contract(off)
  const uint32_t leaf = keys[i] >> (2 * kSubLevels);
  const int ix = int(leaf & ((1u << levels) - 1u)), iy = int(leaf >> levels);
  const double w = root[3];
  const double cx = root[0] + (double(ix) + 0.5) * w;
  const double cy = root[1] + (double(iy) + 0.5) * w;
  const double2 q = xy[perm[i]];
  const double lx = q.x - cx, ly = q.y - cy;
  p64[i] = Part64{lx, ly, 0.0, 0.0};
  p32[i] = Part32{float(lx), float(ly), 0.0f, 0.0f};
}

// Waves of the leaf part of k_leaf_coords take 63 leaves each and one more:
// lane l of wave w searches leaf 63 w + l, and lanes 0..62 take their leaf's
// end from the next lane.
constexpr int kLeavesPerWave = 63;

// The leaf starts (nleaves + 1 entries), the tiles per leaf (ceil(count /
// tile); 0 at index nleaves) and the local coordinates in one launch: the
// first leaf_blocks workgroups take the leaves (one binary search per lane,
// latency bound), the rest the particles (a gather through the permutation
// each), so that the two run side by side.
__global__ void __launch_bounds__(256) k_leaf_coords(const double2* __restrict__ xy,
                                                     const uint32_t* __restrict__ keys,
                                                     const int32_t* __restrict__ perm, int64_t n,
                                                     int64_t nleaves, unsigned leaf_blocks,
                                                     int tile, const double* __restrict__ root,
                                                     int levels, int32_t* __restrict__ start,
                                                     uint32_t* __restrict__ tiles_per_leaf,
                                                     Part64* __restrict__ p64,
                                                     Part32* __restrict__ p32) {
  if (blockIdx.x < leaf_blocks) {
    const int lane = int(threadIdx.x) & 63;
    const int64_t k = ((blockIdx.x * 256LL + threadIdx.x) >> 6) * kLeavesPerWave + lane;
    const int64_t s0 = k <= nleaves ? leaf_start_of(keys, n, k) : n;
    const int64_t s1 = __shfl_down(s0, 1, 64);  // the start of leaf k + 1 (lanes 0..62)
    if (lane < kLeavesPerWave && k <= nleaves) {  // lane 63's leaf is the next wave's lane 0's
      start[k] = int32_t(s0);
      tiles_per_leaf[k] = k < nleaves ? uint32_t((s1 - s0 + tile - 1) / tile) : 0u;
    }
  } else {
    const int64_t i = (blockIdx.x - leaf_blocks) * 256LL + threadIdx.x;
    if (i < n) local_coords_of(xy, keys, perm, i, root, levels, p64, p32);
  }
}

__global__ void __launch_bounds__(256) k_target_coords(const double* __restrict__ x,
                                                       const double* __restrict__ y,
                                                       const uint32_t* __restrict__ keys,
                                                       const int32_t* __restrict__ perm, int64_t n,
                                                       const double* __restrict__ root, int levels,
                                                       Part64* __restrict__ p64,
                                                       Part32* __restrict__ p32) {
#pragma clang fp contract(off)
  int64_t i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= n) return;
  const uint32_t leaf = keys[i] >> (2 * kSubLevels);
  const int ix = int(leaf & ((1u << levels) - 1u)), iy = int(leaf >> levels);
  const double w = root[3];
  const double cx = root[0] + (double(ix) + 0.5) * w;
  const double cy = root[1] + (double(iy) + 0.5) * w;
  const int32_t j = perm[i];
  const double xj = x[j], yj = y[j];
  const bool ok = in_root(xj, yj, root);
  const double lx = ok ? xj - cx : NAN, ly = ok ? yj - cy : NAN;
  p64[i] = Part64{lx, ly, 0.0, 0.0};
  p32[i] = Part32{float(lx), float(ly), 0.0f, 0.0f};
}

__global__ void __launch_bounds__(256) k_tile_counts(const int32_t* __restrict__ start,
                                                     int64_t nleaves, int tile,
                                                     uint32_t* __restrict__ cnt) {
  int64_t k = blockIdx.x * 256LL + threadIdx.x;
  if (k > nleaves) return;
  cnt[k] = k < nleaves ? uint32_t((start[k + 1] - start[k] + tile - 1) / tile) : 0u;
}

// One thread per particle: a particle that starts a tile-sized block of its
// leaf writes that tile.
__global__ void __launch_bounds__(256) k_tile_fill(const uint32_t* __restrict__ keys,
                                                   const int32_t* __restrict__ start,
                                                   const uint32_t* __restrict__ off, int64_t n,
                                                   int64_t nleaves, int tile,
                                                   Tile* __restrict__ tiles,
                                                   int32_t* __restrict__ ntiles) {
  const int64_t i = blockIdx.x * 256LL + threadIdx.x;
  if (i == 0) *ntiles = int32_t(off[nleaves]);
  if (i >= n) return;
  const uint32_t leaf = keys[i] >> (2 * kSubLevels);
  const int32_t s = start[leaf], c = start[leaf + 1] - s;
  const int32_t r = int32_t(i) - s;
  if (r % tile != 0) return;
  const int32_t cc = c - r;
  tiles[off[leaf] + r / tile] = Tile{int32_t(leaf), int32_t(i), cc < tile ? cc : tile, 0};
}

// Bounding box of each tile's particles in the leaf's local frame, one wave
// per tile, the waves looping over the tiles.
__global__ void __launch_bounds__(256) k_tile_box(const Tile* __restrict__ tiles,
                                                  const int32_t* __restrict__ ntiles,
                                                  const Part32* __restrict__ p32,
                                                  float4* __restrict__ box) {
  const int nt = *ntiles;
  const int lane = threadIdx.x & 63;
  for (int wid = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6)); wid < nt;
       wid += 4 * gridDim.x) {
    const Tile t = tiles[wid];
    const Part32 q = p32[t.start + (lane < t.count ? lane : 0)];
    float x0 = q.x, x1 = q.x, y0 = q.y, y1 = q.y;
    for (int o = 32; o > 0; o >>= 1) {
      x0 = fminf(x0, __shfl_xor(x0, o, 64));
      x1 = fmaxf(x1, __shfl_xor(x1, o, 64));
      y0 = fminf(y0, __shfl_xor(y0, o, 64));
      y1 = fmaxf(y1, __shfl_xor(y1, o, 64));
    }
    if (lane == 0) box[wid] = make_float4(x0, x1, y0, y1);
  }
}

__global__ void __launch_bounds__(256) k_gather_gamma(const double* __restrict__ gamma,
                                                      const int32_t* __restrict__ perm, int64_t n,
                                                      Part64* __restrict__ p64,
                                                      Part32* __restrict__ p32,
                                                      Part32* __restrict__ p32s, double scale,
                                                      bool with64) {
  int64_t i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= n) return;
  const double g = gamma[perm[i]];
  if (with64) p64[i].g = g;
  p32[i].g = float(g);
  if (scale > 0.0) {
    const Part64 q = p64[i];
    p32s[i] = Part32{float(q.x * scale), float(q.y * scale), float(g), 0.0f};
  }
}

inline unsigned nblocks(int64_t n, int b) { return unsigned((n + b - 1) / b); }

}  // namespace

namespace {

// ------------------------------------------------------------------ adaptive tree
// Particles per box at level l from the counts of level l + 1 (the leaf level's
// come from the leaf ranges).
__global__ void __launch_bounds__(256) k_fine_counts(const int32_t* __restrict__ leaf_start,
                                                     int64_t nleaves, uint32_t* __restrict__ cnt) {
  const int64_t f = blockIdx.x * 256LL + threadIdx.x;
  if (f < nleaves) cnt[f] = uint32_t(leaf_start[f + 1] - leaf_start[f]);
}

__global__ void __launch_bounds__(256) k_coarse_counts(const uint32_t* __restrict__ child, int lev,
                                                       uint32_t* __restrict__ cnt) {
  const int64_t b = blockIdx.x * 256LL + threadIdx.x;
  const int64_t nb = int64_t(1) << (2 * lev);
  if (b >= nb) return;
  const int m = 1 << lev, mc = 2 * m;
  const int bx = int(b & (m - 1)), by = int(b >> lev);
  const int64_t c0 = int64_t(2 * by) * mc + 2 * bx;
  cnt[b] = child[c0] + child[c0 + 1] + child[c0 + mc] + child[c0 + mc + 1];
}

// Level of the adaptive leaf holding each leaf-level box f, as the shift
// k = L - level: the box at level l above f is split while it holds more
// than s particles and l < L.  counts holds the levels 0 .. L one after the
// other (level l at offset (4^l - 1) / 3).
__global__ void __launch_bounds__(256) k_leaf_shift(const uint32_t* __restrict__ counts, int levels,
                                                    int64_t s, uint8_t* __restrict__ shift) {
  const int64_t f = blockIdx.x * 256LL + threadIdx.x;
  const int64_t nl = int64_t(1) << (2 * levels);
  if (f >= nl) return;
  const int fx = int(f & ((1 << levels) - 1)), fy = int(f >> levels);
  int l = 0;
  while (l < levels) {
    const int d = levels - l;
    const int64_t off = ((int64_t(1) << (2 * l)) - 1) / 3;
    const int64_t b = int64_t(fy >> d) * (1 << l) + (fx >> d);
    if (int64_t(counts[off + b]) <= s) break;
    ++l;
  }
  shift[f] = uint8_t(levels - l);
}

// Sort key of a particle (tree order) as a target of the adaptive tree: the
// leaf-level box at the lower-left corner of its adaptive leaf.
__global__ void __launch_bounds__(256) k_adaptive_keys(const uint32_t* __restrict__ tkeys, int64_t n,
                                                       int levels, const uint8_t* __restrict__ shift,
                                                       uint32_t* __restrict__ keys,
                                                       int32_t* __restrict__ idx) {
  const int64_t i = blockIdx.x * 256LL + threadIdx.x;
  if (i >= n) return;
  const uint32_t f = tkeys[i] >> (2 * kSubLevels);
  const int k = shift[f];
  const uint32_t m = 1u << levels;
  const uint32_t fx = (f & (m - 1u)) >> k << k, fy = (f >> levels) >> k << k;
  keys[i] = fy * m + fx;
  idx[i] = int32_t(i);
}

__global__ void __launch_bounds__(256) k_shift_keys(uint32_t* __restrict__ keys, int64_t n) {
  const int64_t i = blockIdx.x * 256LL + threadIdx.x;
  if (i < n) keys[i] <<= 2 * kSubLevels;
}

// Target records of the adaptive set: coordinates relative to the centre of the
// adaptive leaf (the tree's leaf-local coordinates plus the offset of the two
// centres, an exact multiple of half the leaf-level side), for L2P and the tile
// boxes; the tree's own leaf-local record with the leaf-level box in place of
// the circulation (fine64), from which the near field takes its offsets to the
// sources, so that a particle meets itself at offset exactly zero; caller index.
__global__ void __launch_bounds__(256) k_adaptive_coords(const uint32_t* __restrict__ tkeys,
                                                         const int32_t* __restrict__ idx,
                                                         const int32_t* __restrict__ tperm,
                                                         const Part64* __restrict__ tp64, int64_t n,
                                                         const double* __restrict__ root, int levels,
                                                         const uint8_t* __restrict__ shift,
                                                         Part64* __restrict__ p64,
                                                         Part32* __restrict__ p32,
                                                         Part64* __restrict__ fine64,
                                                         int32_t* __restrict__ perm) {
#pragma clang fp contract(off)
  const int64_t j = blockIdx.x * 256LL + threadIdx.x;
  if (j >= n) return;
  const int32_t i = idx[j];
  const uint32_t f = tkeys[i] >> (2 * kSubLevels);
  const int k = shift[f];
  const int fx = int(f & ((1u << levels) - 1u)), fy = int(f >> levels);
  const double w = root[3];
  // (c_f - c_A) / w_L = (fx + 1/2) - (bx + 1/2) 2^k, bx = fx >> k: exact
  const double ox = (double(fx) + 0.5) - (double(fx >> k) + 0.5) * double(1 << k);
  const double oy = (double(fy) + 0.5) - (double(fy >> k) + 0.5) * double(1 << k);
  const Part64 q = tp64[i];
  const double lx = q.x + ox * w, ly = q.y + oy * w;
  p64[j] = Part64{lx, ly, 0.0, 0.0};
  p32[j] = Part32{float(lx), float(ly), 0.0f, 0.0f};
  fine64[j] = Part64{q.x, q.y, double(f), 0.0};
  perm[j] = tperm[i];
}

}  // namespace

hipError_t launch_build_tree(const double* x, const double* y, int64_t n, int levels,
                             const double* domain, const Layout& lay, char* ws, int tile,
                             TreeDev& t, hipStream_t st) {
  double* root = reinterpret_cast<double*>(ws + lay.root);
  double* bbox = reinterpret_cast<double*>(ws + lay.bbox);
  uint32_t* k0 = reinterpret_cast<uint32_t*>(ws + lay.keys0);
  uint32_t* k1 = reinterpret_cast<uint32_t*>(ws + lay.keys1);
  int32_t* i0 = reinterpret_cast<int32_t*>(ws + lay.idx0);
  int32_t* i1 = reinterpret_cast<int32_t*>(ws + lay.idx1);
  uint32_t* counts = reinterpret_cast<uint32_t*>(ws + lay.counts);
  uint32_t* tmp = reinterpret_cast<uint32_t*>(ws + lay.scan_tmp);
  int32_t* lstart = reinterpret_cast<int32_t*>(ws + lay.leaf_start);
  uint32_t* toff = reinterpret_cast<uint32_t*>(ws + lay.tile_off);

  const int nbb = int(nblocks(n, 256) < unsigned(kBBoxBlocks) ? nblocks(n, 256) : kBBoxBlocks);
  hipLaunchKernelGGL(k_bbox_partial, dim3(nbb), dim3(256), 0, st, x, y, n, bbox);
  hipLaunchKernelGGL(k_root, dim3(1), dim3(256), 0, st, bbox, nbb, domain ? 1 : 0,
                     domain ? domain[0] : 0.0, domain ? domain[1] : 0.0,
                     domain ? domain[2] : 1.0, levels, root);
  double2* xy = reinterpret_cast<double2*>(ws + lay.xy);
  const int nblk = int(lay.sort_blocks);
  hipLaunchKernelGGL(k_keys, dim3(nblk), dim3(kSortBlock), 0, st, x, y, n, root, levels, k0, i0,
                     xy, counts, nblk);
  int bits_left = 2 * (levels + kSubLevels), shift = 0;
  static_assert(2 * kSubLevels >= 8, "the first radix pass takes 8 bits");
  while (bits_left > 0) {
    const int bits = bits_left < 8 ? bits_left : 8;
    const uint32_t mask = (1u << bits) - 1u;
    if (shift > 0)  // the first pass's counts come with the keys
      hipLaunchKernelGGL(k_radix_count, dim3(nblk), dim3(kSortBlock), 0, st, k0, n, shift, mask,
                         counts, nblk);
    hipError_t e = scan_exclusive(counts, int64_t(256) * nblk, tmp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(kSortBlock), 0, st, k0, i0, n, shift,
                       mask, bits, counts, nblk, k1, i1);
    uint32_t* tk = k0; k0 = k1; k1 = tk;
    int32_t* ti = i0; i0 = i1; i1 = ti;
    shift += bits;
    bits_left -= bits;
  }
  const int64_t nl = lay.nleaves;
  t.n = n;
  t.root = root;
  t.keys = k0;
  t.perm = i0;
  t.leaf_start = lstart;
  t.tiles = reinterpret_cast<Tile*>(ws + lay.tiles);
  t.ntiles = reinterpret_cast<int32_t*>(ws + lay.ntiles);
  t.part64 = reinterpret_cast<Part64*>(ws + lay.part64);
  t.part32 = reinterpret_cast<Part32*>(ws + lay.part32);
  t.part32s = reinterpret_cast<Part32*>(ws + lay.part32s);
  t.react = reinterpret_cast<double2*>(ws + lay.react);
  t.me = ws + lay.me;
  t.le = ws + lay.le;
  t.me32 = ws + lay.me32;
  t.le32 = ws + lay.le32;
  t.ops = ws + lay.ops;
  t.check = reinterpret_cast<unsigned long long*>(ws + lay.check);
  const unsigned leaf_blocks = nblocks(int64_t(nblocks(nl + 1, kLeavesPerWave)) * 64, 256);
  hipLaunchKernelGGL(k_leaf_coords, dim3(leaf_blocks + nblocks(n, 256)), dim3(256), 0, st, xy, k0,
                     i0, n, nl, leaf_blocks, tile, root, levels, lstart, toff, t.part64,
                     t.part32);
  t.tile = tile;
  hipError_t e = scan_exclusive(toff, nl + 1, tmp, st);
  if (e != hipSuccess) return e;
  t.tile_off = toff;
  t.tile_box = reinterpret_cast<float4*>(ws + lay.tile_box);
  t.sched = P2PSched{reinterpret_cast<uint32_t*>(ws + lay.sched_cnt),
                     reinterpret_cast<uint32_t*>(ws + lay.sched_poff),
                     reinterpret_cast<uint32_t*>(ws + lay.sched_soff),
                     reinterpret_cast<P2PPart*>(ws + lay.sched_parts),
                     reinterpret_cast<double2*>(ws + lay.sched_partial),
                     tmp,
                     reinterpret_cast<double2*>(ws + lay.sched_near)};
  t.max_tiles = lay.max_tiles;
  hipLaunchKernelGGL(k_tile_fill, dim3(nblocks(n, 256)), dim3(256), 0, st, k0, lstart, toff, n, nl,
                     tile, t.tiles, t.ntiles);
  hipLaunchKernelGGL(k_tile_box, dim3(tile_loop_blocks(lay.max_tiles)), dim3(256), 0, st,
                     t.tiles, t.ntiles, t.part32, t.tile_box);
  return hipGetLastError();
}

hipError_t launch_build_targets(const double* xt, const double* yt, int64_t nt, const TreeDev& t,
                                int levels, const TargetLayout& lay, char* ws, TargetsDev& out,
                                hipStream_t st) {
  uint32_t* k0 = reinterpret_cast<uint32_t*>(ws + lay.keys0);
  uint32_t* k1 = reinterpret_cast<uint32_t*>(ws + lay.keys1);
  int32_t* i0 = reinterpret_cast<int32_t*>(ws + lay.idx0);
  int32_t* i1 = reinterpret_cast<int32_t*>(ws + lay.idx1);
  uint32_t* counts = reinterpret_cast<uint32_t*>(ws + lay.counts);
  uint32_t* tmp = reinterpret_cast<uint32_t*>(ws + lay.scan_tmp);
  int32_t* lstart = reinterpret_cast<int32_t*>(ws + lay.leaf_start);
  uint32_t* toff = reinterpret_cast<uint32_t*>(ws + lay.tile_off);
  Tile* tiles = reinterpret_cast<Tile*>(ws + lay.tiles);
  int32_t* ntiles = reinterpret_cast<int32_t*>(ws + lay.ntiles);
  float4* tbox = reinterpret_cast<float4*>(ws + lay.tile_box);
  Part64* p64 = reinterpret_cast<Part64*>(ws + lay.part64);
  Part32* p32 = reinterpret_cast<Part32*>(ws + lay.part32);
  const int64_t nl = lay.nleaves;
  hipLaunchKernelGGL(k_target_keys, dim3(nblocks(nt, 256)), dim3(256), 0, st, xt, yt, nt, t.root,
                     levels, k0, i0);
  hipError_t e = radix_sort_pairs(k0, k1, i0, i1, nt, 2 * (levels + kSubLevels), counts, tmp, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_leaf_start, dim3(nblocks(nl + 1, 256)), dim3(256), 0, st, k0, nt, nl,
                     lstart);
  hipLaunchKernelGGL(k_target_coords, dim3(nblocks(nt, 256)), dim3(256), 0, st, xt, yt, k0, i0,
                     nt, t.root, levels, p64, p32);
  hipLaunchKernelGGL(k_tile_counts, dim3(nblocks(nl + 1, 256)), dim3(256), 0, st, lstart, nl,
                     t.tile, toff);
  e = scan_exclusive(toff, nl + 1, tmp, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tile_fill, dim3(nblocks(nt, 256)), dim3(256), 0, st, k0, lstart, toff, nt,
                     nl, t.tile, tiles, ntiles);
  hipLaunchKernelGGL(k_tile_box, dim3(tile_loop_blocks(lay.max_tiles)), dim3(256), 0, st, tiles,
                     ntiles, p32, tbox);
  const P2PSched sched{reinterpret_cast<uint32_t*>(ws + lay.sched_cnt),
                       reinterpret_cast<uint32_t*>(ws + lay.sched_poff),
                       reinterpret_cast<uint32_t*>(ws + lay.sched_soff),
                       reinterpret_cast<P2PPart*>(ws + lay.sched_parts),
                       reinterpret_cast<double2*>(ws + lay.sched_partial),
                       tmp,
                     reinterpret_cast<double2*>(ws + lay.sched_near)};
  out = TargetsDev{p64, p32, tiles, ntiles, tbox, toff, i0, lay.max_tiles, sched};
  return hipGetLastError();
}

hipError_t radix_sort_pairs(uint32_t*& k0, uint32_t*& k1, int32_t*& i0, int32_t*& i1, int64_t n,
                            int bits, uint32_t* counts, uint32_t* tmp, hipStream_t st) {
  const int nblk = int((n + kSortPerBlock - 1) / kSortPerBlock);
  int shift = 0;
  while (bits > 0) {
    const int b = bits < 8 ? bits : 8;
    const uint32_t mask = (1u << b) - 1u;
    hipLaunchKernelGGL(k_radix_count, dim3(nblk), dim3(kSortBlock), 0, st, k0, n, shift, mask,
                       counts, nblk);
    hipError_t e = scan_exclusive(counts, int64_t(256) * nblk, tmp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(kSortBlock), 0, st, k0, i0, n, shift,
                       mask, b, counts, nblk, k1, i1);
    uint32_t* tk = k0; k0 = k1; k1 = tk;
    int32_t* ti = i0; i0 = i1; i1 = ti;
    shift += b;
    bits -= b;
  }
  return hipGetLastError();
}

hipError_t launch_tile_box(const Tile* tiles, const int32_t* ntiles, int64_t max_tiles,
                           const Part32* p32, float4* box, hipStream_t st) {
  hipLaunchKernelGGL(k_tile_box, dim3(tile_loop_blocks(max_tiles)), dim3(256), 0, st, tiles,
                     ntiles, p32, box);
  return hipGetLastError();
}

hipError_t launch_gather_gamma(const TreeDev& t, const double* gamma, int64_t n, double sigma,
                               bool with64, hipStream_t st) {
  const double scale = sigma > 0.0 ? near_scale(sigma) : 0.0;
  hipLaunchKernelGGL(k_gather_gamma, dim3(nblocks(n, 256)), dim3(256), 0, st, gamma, t.perm, n,
                     t.part64, t.part32, t.part32s, scale, with64);
  return hipGetLastError();
}

hipError_t launch_build_adaptive(const TreeDev& t, int levels, int64_t s, const AdaptiveLayout& lay,
                                 char* ws, TargetsDev& out, hipStream_t st) {
  const TargetLayout& tl = lay.targets;
  const int64_t n = tl.nt, nl = tl.nleaves;
  uint32_t* cnt = reinterpret_cast<uint32_t*>(ws + lay.counts);
  uint8_t* shift = reinterpret_cast<uint8_t*>(ws + lay.shift);
  auto level_counts = [&](int l) { return cnt + ((int64_t(1) << (2 * l)) - 1) / 3; };
  hipLaunchKernelGGL(k_fine_counts, dim3(nblocks(nl, 256)), dim3(256), 0, st, t.leaf_start, nl,
                     level_counts(levels));
  for (int l = levels - 1; l >= 0; --l)
    hipLaunchKernelGGL(k_coarse_counts, dim3(nblocks(int64_t(1) << (2 * l), 256)), dim3(256), 0,
                       st, level_counts(l + 1), l, level_counts(l));
  hipLaunchKernelGGL(k_leaf_shift, dim3(nblocks(nl, 256)), dim3(256), 0, st, cnt, levels, s, shift);
  uint32_t* k0 = reinterpret_cast<uint32_t*>(ws + tl.keys0);
  uint32_t* k1 = reinterpret_cast<uint32_t*>(ws + tl.keys1);
  int32_t* i0 = reinterpret_cast<int32_t*>(ws + tl.idx0);
  int32_t* i1 = reinterpret_cast<int32_t*>(ws + tl.idx1);
  uint32_t* counts = reinterpret_cast<uint32_t*>(ws + tl.counts);
  uint32_t* tmp = reinterpret_cast<uint32_t*>(ws + tl.scan_tmp);
  int32_t* lstart = reinterpret_cast<int32_t*>(ws + tl.leaf_start);
  uint32_t* toff = reinterpret_cast<uint32_t*>(ws + tl.tile_off);
  Tile* tiles = reinterpret_cast<Tile*>(ws + tl.tiles);
  int32_t* ntiles = reinterpret_cast<int32_t*>(ws + tl.ntiles);
  float4* tbox = reinterpret_cast<float4*>(ws + tl.tile_box);
  Part64* p64 = reinterpret_cast<Part64*>(ws + tl.part64);
  Part32* p32 = reinterpret_cast<Part32*>(ws + tl.part32);
  int32_t* perm = reinterpret_cast<int32_t*>(ws + lay.perm);
  Part64* fine64 = reinterpret_cast<Part64*>(ws + lay.fine64);
  hipLaunchKernelGGL(k_adaptive_keys, dim3(nblocks(n, 256)), dim3(256), 0, st, t.keys, n, levels,
                     shift, k0, i0);
  // stable sort on the leaf bits: the tree's order is kept inside each
  // adaptive leaf; then the keys take the usual form (leaf above 2 kSubLevels
  // zero sub-cell bits)
  hipError_t e = radix_sort_pairs(k0, k1, i0, i1, n, 2 * levels, counts, tmp, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_shift_keys, dim3(nblocks(n, 256)), dim3(256), 0, st, k0, n);
  hipLaunchKernelGGL(k_leaf_start, dim3(nblocks(nl + 1, 256)), dim3(256), 0, st, k0, n, nl, lstart);
  hipLaunchKernelGGL(k_adaptive_coords, dim3(nblocks(n, 256)), dim3(256), 0, st, t.keys, i0,
                     t.perm, t.part64, n, t.root, levels, shift, p64, p32, fine64, perm);
  hipLaunchKernelGGL(k_tile_counts, dim3(nblocks(nl + 1, 256)), dim3(256), 0, st, lstart, nl,
                     t.tile, toff);
  e = scan_exclusive(toff, nl + 1, tmp, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tile_fill, dim3(nblocks(n, 256)), dim3(256), 0, st, k0, lstart, toff, n, nl,
                     t.tile, tiles, ntiles);
  hipLaunchKernelGGL(k_tile_box, dim3(tile_loop_blocks(tl.max_tiles)), dim3(256), 0, st, tiles,
                     ntiles, p32, tbox);
  const P2PSched sched{reinterpret_cast<uint32_t*>(ws + tl.sched_cnt),
                       reinterpret_cast<uint32_t*>(ws + tl.sched_poff),
                       reinterpret_cast<uint32_t*>(ws + tl.sched_soff),
                       reinterpret_cast<P2PPart*>(ws + tl.sched_parts),
                       reinterpret_cast<double2*>(ws + tl.sched_partial),
                       tmp,
                       reinterpret_cast<double2*>(ws + tl.sched_near)};
  out = TargetsDev{p64, p32, tiles, ntiles, tbox, toff, perm, tl.max_tiles, sched, shift, fine64};
  return hipGetLastError();
}

}  // namespace vfmm
