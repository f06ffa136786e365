// Near field (P2P) and far-field evaluation (L2P) (Cruz & Barba 2008, eq. 10:
// f = f_near + f_far), at the particles (eq. 9) or at a separate set of
// evaluation points sorted into the same leaves (eq. 8).  Two launches, so
// that the expansion sweeps can run beside the near field: the P2P kernel
// leaves its sums in sorted order (one value per target of a single-part
// tile, one partial sum per part of a split tile); the L2P kernel adds the
// parts of split tiles in part order, adds the far field and writes u, v once,
// in the caller's order.
//
// P2P: for each target, the regularised Biot-Savart sum (eq. 6) over the
// particles of the 3 x 3 local list of its leaf (Section 3.3.1); a source at
// the target itself (the self term) contributes exactly zero because the pair
// offset is (0, 0).
// L2P: W_far = (-j / (2 pi w)) sum_n L_n ((z - c)/w)^n, Horner's rule.
//
// Work decomposition: targets come in tiles of <= T points of one leaf (T = 64,
// 32 or 16 from the tuning; 64 / T lanes per target, each lane taking every
// (64 / T)-th source of a chunk, the lanes of a target summed by shuffles).
// The sources of a tile's local list are the source tiles ("chunks", <= T
// particles of one leaf) of its three rows of leaves; in each row the chunks of
// the three leaves are consecutive.  A schedule cuts every tile's chunk
// sequence into parts of similar size, so that a launch has a set number of
// parts (4 per target tile, 4096 to 65536) whatever the spread of the work: on
// clustered particles, or on a lattice of evaluation points, a few leaves hold
// most of the pairs.  One wave per part; a tile with one part writes its
// result directly, the parts of a split tile write partial sums that a second
// L2P kernel adds in part order (so results do not depend on timing).  The parts
// of the tiles of one leaf are interleaved so that
// neighbouring waves read the same sources.  Workgroups keep the hardware's
// round-robin dealing to the 8 XCDs (contiguous per-XCD ranges, or ordering
// tiles by cost, were measured 1.7-2x slower on clustered inputs).
// With T = 64 the source index is the same for all lanes of the wave, so
// sources are fetched with scalar loads and broadcast (8 per loop trip, so
// several loads are in flight); the part and tile fields are read into scalar
// registers so that the compiler keeps the loop bounds, and the loads, scalar.
// Coordinates are box-local; the target is shifted once per source leaf by the
// exact centre offset.
//
// Distance cut-off (optional; the distance a of Section 4.1): the chunk
// sequence also holds the rings of leaves at Chebyshev distance 2 .. D, whose
// particles the expansions already carry with the singular kernel; a ring
// chunk whose box gap to the target tile is below the radius adds
// Gamma (K_sigma - K') for its pairs closer than the radius
// (Gamma exp(-r^2 / 2 sigma^2) / r^2 in complex form).  A particle outside the
// rings up to D is at least D w_L from every point of the target leaf, so D is
// the smallest number of rings with D w_L >= radius, at most kMaxRings; the
// radius is clamped to kMaxRings w_L.  Every kernel takes D from the leaf side
// on the device, so the schedule and the near field agree.  With one lane per
// target, the
// sources of such a chunk are first tested in parallel (one per lane) against
// the tile's box, and the wave visits only those within the radius (about 45 %
// on clustered particles).
//
// Far chunks: when the bounding boxes of the target tile and of a source chunk
// are more than r_c apart, every pair has exp(-r^2 / 2 sigma^2) below half an
// ulp of 1 (r_c^2 = 36 sigma^2 in FP32, 76 sigma^2 in FP64), so 1 - exp rounds
// to exactly 1 and the chunk is summed with the kernel's far form Gamma / r^2,
// which gives bit-identical results without the exponential.
//
// FP32 variant: per-pair arithmetic in FP32 with the hardware exp2 and
// reciprocal (and a short series for 1 - exp when r < sigma / 4, used only in
// chunks whose bounding box comes that close to the tile); partial sums over
// chunks are added into a compensated (TwoSum) FP32 accumulator, which keeps
// the rounding of long source loops (up to ~1e5 sources per target) near the
// per-term level; the parts of a split tile are added in FP64.
// FP64 variant: plain FP64 with expm1 and division.
#include "p2p_math.hpp"

namespace vfmm {

namespace {

// The chunk sequence of a target leaf (bx, by) is a list of segments, each a
// run of consecutive leaves lo .. hi of one row sy, whose chunks are
// tile_off[sy m + lo] .. tile_off[sy m + hi + 1] - 1:
//   s = 0, 1, 2: the local list, rows by - 1 .. by + 1, leaves bx - 1 .. bx + 1;
//   with the distance cut-off, the rings d = 2 .. D in turn, 4 d segments each:
//   first row by - d, leaves bx - d .. bx + d; then rows by - d + 1 .. by + d - 1,
//   leaf bx - d then leaf bx + d; last row by + d, leaves bx - d .. bx + d;
// all clipped to the level.  Returns false for an empty segment.
__device__ __forceinline__ bool segment(int s, int bx, int by, int m, int& sy, int& lo, int& hi) {
  int d0, d1;
  if (s < 3) {
    sy = by - 1 + s;
    d0 = -1;
    d1 = 1;
  } else {
    int d = 2, base = 3;
    while (s >= base + 4 * d) {
      base += 4 * d;
      ++d;
    }
    const int j = s - base;
    if (j == 0 || j == 4 * d - 1) {
      sy = j == 0 ? by - d : by + d;
      d0 = -d;
      d1 = d;
    } else {
      const int k = j - 1;
      sy = by - d + 1 + (k >> 1);
      d0 = d1 = (k & 1) ? d : -d;
    }
  }
  lo = bx + d0 < 0 ? 0 : bx + d0;
  hi = bx + d1 > m - 1 ? m - 1 : bx + d1;
  return sy >= 0 && sy < m && lo <= hi;
}

constexpr int kSegNear = 3;
constexpr int kMaxRings = 4;  // rings of the distance cut-off: Chebyshev distance 2 .. 4


// Segments of the chunk sequence and the effective cut-off radius^2 for the
// requested radius^2 cut2 (0: the paper's split, no rings) at leaf side w.
struct NearRings {
  int nseg;
  double rc2;
};
__device__ __forceinline__ NearRings near_rings(double cut2, double w) {
  if (cut2 <= 0.0) return NearRings{kSegNear, 0.0};
  int d = 2, nseg = kSegNear + 4 * 2;
  while (d < kMaxRings && cut2 > (d * w) * (d * w)) {
    ++d;
    nseg += 4 * d;
  }
  const double cap = (d * w) * (d * w);
  return NearRings{nseg, cut2 < cap ? cut2 : cap};
}

// The chunk sequence of a target leaf of level L - k (adaptive tree; k = 0 for
// a leaf-level box) in leaf-level terms: segment sg is row sg & (2^k - 1) of the
// 2^k leaf-level rows of the level's segment sg >> k, and spans the 2^k
// leaf-level boxes of every box of that segment.  (bx, by) are the target
// leaf's coordinates at its level, ml = 2^(L - k) the boxes per side there.
__device__ __forceinline__ bool fine_segment(int sg, int k, int bx, int by, int ml, int& sy,
                                             int& lo, int& hi) {
  int syl, lol, hil;
  if (!segment(sg >> k, bx, by, ml, syl, lol, hil)) return false;
  sy = (syl << k) + (sg & ((1 << k) - 1));
  lo = lol << k;
  hi = ((hil + 1) << k) - 1;
  return true;
}

// Level shift k of a target tile's leaf (0 without an adaptive tree).
__device__ __forceinline__ int tile_shift(const uint8_t* __restrict__ leaf_shift, int leaf) {
  return leaf_shift ? int(leaf_shift[leaf]) : 0;
}

// Source chunks in segments first, first + stride, ... of a tile's sequence.
__device__ __forceinline__ uint32_t sequence_chunks(int leaf, int levels, int k, int nseg,
                                                    const uint32_t* __restrict__ tile_off,
                                                    int first, int stride) {
  const int m = 1 << levels;
  const int bx = (leaf & (m - 1)) >> k, by = (leaf >> levels) >> k;
  uint32_t c = 0;
  for (int s = first; s < (nseg << k); s += stride) {
    int sy, lo, hi;
    if (fine_segment(s, k, bx, by, m >> k, sy, lo, hi))
      c += tile_off[sy * m + hi + 1] - tile_off[sy * m + lo];
  }
  return c;
}

// Source chunks per target tile: kSchedLanes lanes per tile (an aligned
// group of a wave) take every kSchedLanes-th segment of its sequence, and the
// group adds up their counts.
constexpr int kSchedLanes = 16;
__global__ void __launch_bounds__(256) k_sched_count(const Tile* __restrict__ ttiles,
                                                     const int32_t* __restrict__ tntiles,
                                                     const uint32_t* __restrict__ tile_off,
                                                     const double* __restrict__ root, int levels,
                                                     double cut2,
                                                     const uint8_t* __restrict__ leaf_shift,
                                                     uint32_t* __restrict__ cnt) {
  const int64_t t = (blockIdx.x * 256LL + threadIdx.x) / kSchedLanes;
  const int sub = int(threadIdx.x) & (kSchedLanes - 1);
  const bool live = t < *tntiles;
  uint32_t c = 0;
  if (live) {
    const int leaf = ttiles[t].leaf;
    const int k = tile_shift(leaf_shift, leaf);
    const int nseg = near_rings(cut2, root[3] * double(1 << k)).nseg;
    c = sequence_chunks(leaf, levels, k, nseg, tile_off, sub, kSchedLanes);
  }
#pragma unroll
  for (int o = kSchedLanes / 2; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if (live && sub == 0) cnt[t] = c;
}

// The schedule's offsets, in one workgroup over the nt = *tntiles tiles:
// first the total of the source chunks (64 bits), hence the part size
// K = max(kP2PMinChunks, ceil(total / P)), P = p2p_parts(max_tiles); then in
// one pass per tile its parts np = max(1, ceil(ch / K)) (ch = cnt[t]), so the
// parts number at most max_tiles + P and those of split tiles at most 2 P, and
// three exclusive prefixes: cnt (source chunks, modulo 2^32), p_off (of np)
// and s_off (of np for split tiles, else 0), with the totals at index nt and,
// for the near-field kernel, p_off[max_tiles].  The arrays are 16-byte
// aligned.
__global__ void __launch_bounds__(kScanOneBlock) k_sched_scan(const int32_t* __restrict__ tntiles,
                                                              int64_t max_tiles,
                                                              uint32_t* __restrict__ cnt,
                                                              uint32_t* __restrict__ p_off,
                                                              uint32_t* __restrict__ s_off) {
  __shared__ uint32_t ws[3 * (kScanOneBlock / 64)];
  __shared__ unsigned long long ws64[kScanOneBlock / 64];
  const int64_t nt = *tntiles;
  const int64_t me = int64_t(threadIdx.x) * 4;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  unsigned long long s64 = 0;
  for (int64_t i = me; i < nt; i += kScanOneRound) {
    const uint4 q = scan_load4(cnt, i, nt);
    s64 += (unsigned long long)q.x + q.y + q.z + q.w;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s64 += __shfl_xor(s64, o, 64);
  if (lane == 0) ws64[wave] = s64;
  __syncthreads();
  unsigned long long total = 0;
#pragma unroll
  for (int w = 0; w < kScanOneBlock / 64; ++w) total += ws64[w];
  const unsigned long long P = (unsigned long long)p2p_parts(max_tiles);
  unsigned long long K = (total + P - 1) / P;
  if (K < kP2PMinChunks) K = kP2PMinChunks;
  // ch < 2^32, so a part size of 2^32 or more gives one part per tile; below
  // it ceil(ch / K) from the float64 quotient, corrected to the exact one
  const bool one_part = K >= (1ull << 32);
  const int64_t K64 = int64_t(K);
  const double rK = 1.0 / double(K);
  uint3 carry = make_uint3(0u, 0u, 0u);
  for (int64_t base = 0; base < nt; base += kScanOneRound * kScanOneRounds) {
    uint4 c[kScanOneRounds];
#pragma unroll
    for (int r = 0; r < kScanOneRounds; ++r) c[r] = scan_load4(cnt, base + r * kScanOneRound + me, nt);
#pragma unroll
    for (int r = 0; r < kScanOneRounds; ++r) {
      const int64_t i = base + r * kScanOneRound + me;
      if (base + r * kScanOneRound >= nt) break;  // uniform
      const uint32_t ch[4] = {c[r].x, c[r].y, c[r].z, c[r].w};
      uint32_t np[4], sp[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        np[j] = 0u;
        if (i + j < nt) {
          if (ch[j] == 0 || one_part) {
            np[j] = 1u;
          } else {
            int64_t q = int64_t(double(ch[j]) * rK);
            int64_t rem = int64_t(ch[j]) - q * K64;
            if (rem < 0) { --q; rem += K64; }
            if (rem >= K64) { ++q; rem -= K64; }
            np[j] = uint32_t(q + (rem > 0 ? 1 : 0));
          }
        }
        sp[j] = np[j] > 1 ? np[j] : 0u;
      }
      uint3 tot;
      uint3 ex = block1k_scan3_excl(make_uint3(c[r].x + c[r].y + c[r].z + c[r].w,
                                               np[0] + np[1] + np[2] + np[3],
                                               sp[0] + sp[1] + sp[2] + sp[3]),
                                    &tot, ws);
      ex.x += carry.x;
      ex.y += carry.y;
      ex.z += carry.z;
      scan_store4(cnt, i, nt, c[r], ex.x);
      scan_store4(p_off, i, nt, make_uint4(np[0], np[1], np[2], np[3]), ex.y);
      scan_store4(s_off, i, nt, make_uint4(sp[0], sp[1], sp[2], sp[3]), ex.z);
      carry.x += tot.x;
      carry.y += tot.y;
      carry.z += tot.z;
    }
  }
  if (threadIdx.x == 0) {
    cnt[nt] = carry.x;
    p_off[nt] = carry.y;
    s_off[nt] = carry.z;
    p_off[max_tiles] = carry.y;
  }
}

// The tiles of one leaf share their local list, hence their chunk count and
// number of parts; their parts are stored part-major (part k of every tile of
// the leaf, then part k + 1), so that neighbouring waves read the same sources.
// The same launch clears react (nreact entries; 0 without the symmetric near
// field).
__global__ void __launch_bounds__(256) k_sched_fill(const Tile* __restrict__ ttiles,
                                                    const int32_t* __restrict__ tntiles,
                                                    const uint32_t* __restrict__ ttile_off,
                                                    const uint32_t* __restrict__ cnt,
                                                    const uint32_t* __restrict__ p_off,
                                                    const uint32_t* __restrict__ s_off,
                                                    P2PPart* __restrict__ parts,
                                                    double2* __restrict__ react, int64_t nreact) {
  const int64_t t = blockIdx.x * 256LL + threadIdx.x;
  // the symmetric near field's float64 sums start at zero
  for (int64_t i = t; i < nreact; i += int64_t(gridDim.x) * 256)
    react[i] = make_double2(0.0, 0.0);
  if (t >= *tntiles) return;
  const int leaf = ttiles[t].leaf;
  const uint32_t t0 = ttile_off[leaf], ntl = ttile_off[leaf + 1] - t0;
  const uint64_t ch = uint32_t(cnt[t + 1] - cnt[t]);
  const uint32_t np = p_off[t + 1] - p_off[t];
  const uint32_t base = p_off[t0], r = uint32_t(t) - t0;
  for (uint32_t k = 0; k < np; ++k)
    parts[base + k * ntl + r] = P2PPart{int32_t(t), int32_t(k * ch / np),
                                        int32_t((k + 1) * ch / np),
                                        np > 1 ? int32_t(s_off[t] + k) : -1};
}

// Far-field evaluation at a target: (-j / (2 pi w)) sum_n L_n (z / w)^n with z
// relative to the leaf centre; returns (u, v) = (Re, -Im).
template <typename R, int PMAX>
__device__ __forceinline__ void l2p(const typename Types<R>::C* __restrict__ L, R x, R y,
                                    double w, int p, double& fu, double& fv) {
  using C = typename Types<R>::C;
  const R inv_w = R(1.0 / w);
  const C z = cmake<C>(x * inv_w, y * inv_w);
  C acc = cmake<C>(R(0), R(0));
#pragma unroll
  for (int k = PMAX - 1; k >= 0; --k) {
    if (k < p) {
      const C lk = L[k];
      acc = cmul(acc, z);
      acc.x += lk.x;
      acc.y += lk.y;
    }
  }
  // (-j/(2 pi w)) (a + j b) = (b - j a)/(2 pi w); u = Re, v = -Im
  const double sc = kInv2Pi / w;
  fu = double(acc.y) * sc;
  fv = double(acc.x) * sc;
}

// Pair arithmetic in the kernel's units: FP32 in units of the Gaussian width
// (sources pre-scaled by the gather kernel), FP64 in plain units.
template <typename R> struct PairK;
template <> struct PairK<float> {
  __device__ __forceinline__ float near(float g, float r2) const { return P2PMath<float>::near_s(g, r2); }
  __device__ __forceinline__ float series(float g, float r2) const {
    return P2PMath<float>::near_series_s(g, r2);
  }
  __device__ __forceinline__ float far(float g, float r2) const { return P2PMath<float>::far(g, r2); }
  __device__ __forceinline__ float gauss(float g, float r2) const { return P2PMath<float>::gauss_s(g, r2); }
  // the kernel value without the circulation, for the symmetric pairs
  __device__ __forceinline__ float hnear(float r2) const { return P2PMath<float>::h_near_s(r2); }
  __device__ __forceinline__ float hseries(float r2) const { return P2PMath<float>::h_series_s(r2); }
  __device__ __forceinline__ float hfar(float r2) const { return P2PMath<float>::h_far(r2); }
};
template <> struct PairK<double> {
  double kexp;
  __device__ __forceinline__ double near(double g, double r2) const {
    return P2PMath<double>::near(g, r2, kexp);
  }
  __device__ __forceinline__ double series(double g, double r2) const { return near(g, r2); }
  __device__ __forceinline__ double far(double g, double r2) const { return P2PMath<double>::far(g, r2); }
  __device__ __forceinline__ double gauss(double g, double r2) const {
    return P2PMath<double>::gauss(g, r2, kexp);
  }
  __device__ __forceinline__ double hnear(double r2) const { return P2PMath<double>::h_near(r2, kexp); }
  __device__ __forceinline__ double hseries(double r2) const { return hnear(r2); }
  __device__ __forceinline__ double hfar(double r2) const { return P2PMath<double>::h_far(r2); }
};

template <typename R, int LPT, bool SYM>
__global__ void __launch_bounds__(512) k_p2p(
    const typename Types<R>::Part* __restrict__ part, const int32_t* __restrict__ leaf_start,
    const uint32_t* __restrict__ tile_off, const float4* __restrict__ tile_box,
    const typename Types<R>::Part* __restrict__ tpart, const Part64* __restrict__ tpart64,
    const Tile* __restrict__ ttiles, const float4* __restrict__ ttile_box,
    const P2PPart* __restrict__ parts, const uint32_t* __restrict__ nparts, double2* __restrict__ partial,
    const double* __restrict__ root, int levels, PairK<R> pk, double sd, float far2, float ser2,
    double cut2, const uint8_t* __restrict__ leaf_shift, const Part64* __restrict__ fine64,
    double2* __restrict__ nearv, double2* __restrict__ react) {
  constexpr int T = 64 / LPT;  // targets per tile = sources per chunk
  // symmetric near field (LPT = 1 only): a block of 128 source records per wave
  extern __shared__ unsigned char p2p_lds[];
  constexpr bool sym = SYM && LPT == 1;
  // FP32: sources and targets in units of the Gaussian width (factor sd);
  // FP64: plain units (sd = 1)
  const int wpb = blockDim.x >> 6;
  const int nwaves = gridDim.x * wpb;
  const int lane = threadIdx.x & 63;
  const int tl = lane % T, grp = lane / T;  // target in tile, source sub-stream
  const int m = 1 << levels;
  const double w = root[3];
  const int np_total = int(*nparts);
  const float sdf = float(sd);
  const double wsd = w * sd;
  for (int pi = __builtin_amdgcn_readfirstlane(blockIdx.x * wpb + (threadIdx.x >> 6));
       pi < np_total; pi += nwaves) {
    // part and tile fields are wave-uniform: keep them in scalar registers so
    // that the source loop bounds, and hence the source loads, stay scalar
    const P2PPart ptv = parts[pi];
    const int pt_tile = __builtin_amdgcn_readfirstlane(ptv.tile);
    const uint32_t v0 = __builtin_amdgcn_readfirstlane(ptv.v0);
    const uint32_t v1 = __builtin_amdgcn_readfirstlane(ptv.v1);
    const int slot = __builtin_amdgcn_readfirstlane(ptv.slot);
    const Tile tv = ttiles[pt_tile];
    const int t_leaf = __builtin_amdgcn_readfirstlane(tv.leaf);
    const int t_start = __builtin_amdgcn_readfirstlane(tv.start);
    const int t_count = __builtin_amdgcn_readfirstlane(tv.count);
    const bool active = tl < t_count;
    const int32_t i = t_start + (active ? tl : 0);
    R tx0, ty0;
    // adaptive tree: each target's own leaf-level box (fx, fy) and its
    // coordinates there, as the tree holds them for the particle as a source
    int fx = 0, fy = 0;
    if (fine64) {
      const Part64 q = fine64[i];
      const int f = int(q.g);
      fx = f & (m - 1);
      fy = f >> levels;
      if constexpr (sizeof(R) == 4) {
        tx0 = float(q.x * sd);
        ty0 = float(q.y * sd);
      } else {
        tx0 = q.x;
        ty0 = q.y;
      }
    } else if constexpr (sizeof(R) == 4) {
      // the same rounding as the gather kernel's, so that a target at a
      // source's position (the self pair) has an offset of exactly zero
      const Part64 q = tpart64[i];
      tx0 = float(q.x * sd);
      ty0 = float(q.y * sd);
    } else {
      const auto q = tpart[i];
      tx0 = q.x;
      ty0 = q.y;
    }
    // the target leaf: level L - k, coordinates (bx, by) there
    const int k = __builtin_amdgcn_readfirstlane(tile_shift(leaf_shift, t_leaf));
    const int bx = (t_leaf & (m - 1)) >> k, by = (t_leaf >> levels) >> k;
    const double half = 0.5 * double(1 << k);  // leaf centre, in leaf-level sides
    // segments of the chunk sequence and the cut-off radius^2, at most (D w_l)^2
    // with D the number of rings searched around the leaf of side w_l
    const NearRings nr = near_rings(cut2, w * double(1 << k));
    const int nseg = nr.nseg << k;
    const double rc2d = nr.rc2;
    const float rc2f = float(rc2d);
    const R rc2 = R(rc2d * sd * sd);
    // symmetric near field: the target's own circulation (the targets are the
    // particles, in the sources' order and units); 0 for the padding lanes
    R tg = R(0);
    if (sym && active) tg = part[i].g;
    SymRec<R>* const sbuf = reinterpret_cast<SymRec<R>*>(p2p_lds) + (threadIdx.x >> 6) * 128;
    const float rc2s = float(rc2d * sd * sd);

    double nu = 0.0, nv = 0.0;
    {
      const R tiny = R(wsd * wsd * 0x1p-80);
      const float4 tb = ttile_box[pt_tile];
      Acc32 au{0.f, 0.f}, av{0.f, 0.f};
      // chunks [v0, v1) of the segment sequence
      uint32_t vb = 0;  // sequence index of the current segment's first chunk
      for (int sg = 0; sg < nseg && vb < v1; ++sg) {
        int sy, lo, hi;
        if (!fine_segment(sg, k, bx, by, m >> k, sy, lo, hi)) continue;
        const bool ring = (sg >> k) >= kSegNear;
        // source row centre minus target leaf centre, in leaf-level sides
        // (sy - by exactly when k = 0); the targets themselves take the offset
        // from their own leaf-level box (equal when k = 0)
        const double oy = (double(sy) + 0.5) - (double(by << k) + half);
        const double oyt = fine64 ? double(sy - fy) : oy;
        const uint32_t ra = tile_off[sy * m + lo], rb = tile_off[sy * m + hi + 1];
        const uint32_t len = rb - ra;
        const uint32_t cl = v0 > vb ? v0 - vb : 0u;
        const uint32_t ch = v1 > vb ? (v1 - vb < len ? v1 - vb : len) : 0u;
        vb += len;
        if (cl >= ch) continue;
        const uint32_t cb = ra + cl, ce = ra + ch;
        const R ty = ty0 - R(oyt * wsd);
        const float by0 = tb.z - float(oy * w), by1 = tb.w - float(oy * w);
        for (int sx = lo; sx <= hi; ++sx) {
          const int sl = sy * m + sx;
          const uint32_t la = tile_off[sl], lb = tile_off[sl + 1];
          const uint32_t qa = la > cb ? la : cb, qb = lb < ce ? lb : ce;
          if (qa >= qb) continue;
          const double ox = (double(sx) + 0.5) - (double(bx << k) + half);
          const double oxt = fine64 ? double(sx - fx) : ox;
          // target relative to the source leaf centre
          const R tx = tx0 - R(oxt * wsd);
          const float bx0 = tb.x - float(ox * w), bx1 = tb.y - float(ox * w);
          const int32_t js = leaf_start[sl], je = leaf_start[sl + 1];
          // symmetric near field: a pair of two different tiles of the local
          // list (a leaf's chunks are its tiles) whose particles number at
          // least kSymMinPair is evaluated once, both directions, by the tile
          // that comes first in (row, leaf, tile) order; the later tile skips
          // it.  Smaller pairs, the tile's own chunk and the rings take one
          // direction per tile.
          const int lrel = sy != by ? sy - by : sx - bx;  // > 0: the leaf comes after
          const int own = sym && lrel == 0 ? (t_start - js) / T : 0;
          for (uint32_t ci = qa; ci < qb; ++ci) {
            const int32_t j0 = js + int32_t(ci - la) * T;
            const int32_t j1 = min(j0 + T, je);
            bool sym_pair = false;
            if (sym && !ring) {
              const int rel = lrel != 0 ? lrel : int(ci - la) - own;
              if (rel != 0 && t_count + (j1 - j0) >= kSymMinPair) {
                if (rel < 0) continue;  // taken by the earlier tile
                sym_pair = true;
              }
            }
            const float4 sb = tile_box[ci];
            const float gx = fmaxf(0.f, fmaxf(sb.x - bx1, bx0 - sb.y));
            const float gy = fmaxf(0.f, fmaxf(sb.z - by1, by0 - sb.w));
            R cu = R(0), cv = R(0);
            const float gap2 = gx * gx + gy * gy;
            if (ring) {
              // beyond the local list: add Gamma (K_sigma - K') for r^2 < rc2
              if (gap2 >= rc2f) continue;
              if constexpr (LPT == 1) {
                // most ring sources are farther than the radius from the whole
                // tile: each lane tests one source against the tile's box and
                // the wave visits only the sources that pass (a uniform mask)
                float d2 = INFINITY;
                if (j0 + lane < j1) {
                  const auto q = part[j0 + lane];
                  const float qx = float(q.x), qy = float(q.y);
                  const float hx = fmaxf(0.f, fmaxf(bx0 * sdf - qx, qx - bx1 * sdf));
                  const float hy = fmaxf(0.f, fmaxf(by0 * sdf - qy, qy - by1 * sdf));
                  d2 = hx * hx + hy * hy;
                }
                uint64_t keep = __ballot(d2 < rc2s);
                while (keep) {
                  const int k = __builtin_ctzll(keep);
                  keep &= keep - 1;
                  const auto s = part[j0 + k];
                  const R dx = tx - s.x;
                  const R dy = ty - s.y;
                  const R r2 = dx * dx + (dy * dy + tiny);
                  const R f = r2 < rc2 ? pk.gauss(s.g, r2) : R(0);
                  cu += f * dy;
                  cv -= f * dx;
                }
              } else {
#pragma unroll 4
                for (int32_t j = j0 + grp; j < j1; j += LPT) {
                  const auto s = part[j];
                  const R dx = tx - s.x;
                  const R dy = ty - s.y;
                  const R r2 = dx * dx + (dy * dy + tiny);
                  const R f = r2 < rc2 ? pk.gauss(s.g, r2) : R(0);
                  cu += f * dy;
                  cv -= f * dx;
                }
              }
            } else if (sym_pair) {
              sym_pair_chunk(sbuf, part, j0, j1, lane, tx, ty, tg, tiny, pk,
                             gap2 > far2 ? 2 : (gap2 > ser2 ? 0 : 1), sd, react, cu, cv);
            } else if (gap2 > far2) {
#pragma unroll 8
              for (int32_t j = j0 + grp; j < j1; j += LPT) {
                const auto s = part[j];
                const R dx = tx - s.x;
                const R dy = ty - s.y;
                const R f = pk.far(s.g, dx * dx + dy * dy);
                cu -= f * dy;
                cv += f * dx;
              }
            } else if (gap2 > ser2) {
#pragma unroll 8
              for (int32_t j = j0 + grp; j < j1; j += LPT) {
                const auto s = part[j];
                const R dx = tx - s.x;
                const R dy = ty - s.y;
                const R r2 = dx * dx + (dy * dy + tiny);
                const R f = pk.near(s.g, r2);
                cu -= f * dy;
                cv += f * dx;
              }
            } else {
#pragma unroll 4
              for (int32_t j = j0 + grp; j < j1; j += LPT) {
                const auto s = part[j];
                const R dx = tx - s.x;
                const R dy = ty - s.y;
                const R r2 = dx * dx + (dy * dy + tiny);
                const R f = pk.series(s.g, r2);
                cu -= f * dy;
                cv += f * dx;
              }
            }
            if constexpr (sizeof(R) == 4) {
              au.add(cu);
              av.add(cv);
            } else {
              nu += cu;
              nv += cv;
            }
          }
        }
      }
      if constexpr (sizeof(R) == 4) {
        nu = au.value();
        nv = av.value();
      }
      // sum the LPT source sub-streams of each target
#pragma unroll
      for (int o = T; o < 64; o <<= 1) {
        nu += __shfl_xor(nu, o, 64);
        nv += __shfl_xor(nv, o, 64);
      }
      nu *= sd;  // back to plain units (Gamma dx / r^2 scales as 1 / sd)
      nv *= sd;
    }

    if (slot >= 0) {
      if (active && grp == 0) partial[int64_t(slot) * kTile + tl] = make_double2(nu, nv);
      continue;
    }
    if (active && grp == 0) nearv[i] = make_double2(nu * kInv2Pi, nv * kInv2Pi);
  }
}

// Result at the targets of one tile (one wave): the near field (near != 0) of
// a single-part tile from nearv, of a split tile the sum of its parts' partial
// sums in part order; plus the far field (L2P, eq. 25 on the scaled LEs of the
// leaves; p = 0: none); written in the caller's order.
template <typename R, int PMAX>
__device__ __forceinline__ void l2p_tile(
    int wid, int lane, const typename Types<R>::Part* __restrict__ tpart,
    const Tile* __restrict__ ttiles, const int32_t* __restrict__ tperm,
    const double* __restrict__ root, int levels, int p,
    const typename Types<R>::C* __restrict__ le_all, const uint8_t* __restrict__ leaf_shift,
    int near, const uint32_t* __restrict__ p_off, const uint32_t* __restrict__ s_off,
    const double2* __restrict__ partial, const double2* __restrict__ nearv,
    const double2* __restrict__ react, double* __restrict__ u, double* __restrict__ v) {
  const Tile tile = ttiles[wid];
  if (lane >= tile.count) return;
  const int32_t i = tile.start + lane;
  double fu = 0.0, fv = 0.0;
  // the target leaf's level l = L - k; levels 0 and 1 have no far field
  const int k = tile_shift(leaf_shift, tile.leaf);
  if (p > 0 && levels - k >= 2) {
    const int l = levels - k, m = 1 << levels;
    const int64_t box = int64_t((tile.leaf >> levels) >> k) * (1 << l) + ((tile.leaf & (m - 1)) >> k);
    const auto tp = tpart[i];  // leaf-local, plain units
    l2p<R, PMAX>(le_all + (level_offset(l) + box) * p, tp.x, tp.y, root[3] * double(1 << k), p,
                 fu, fv);
  }
  const int32_t o = tperm[i];
  if (!near) {
    u[o] = fu;
    v[o] = fv;
    return;
  }
  double nu, nv;
  const uint32_t np = p_off[wid + 1] - p_off[wid];
  if (np > 1) {
    const uint32_t s0 = s_off[wid];
    nu = 0.0;
    nv = 0.0;
    for (uint32_t k = 0; k < np; ++k) {
      const double2 q = partial[int64_t(s0 + k) * kTile + lane];
      nu += q.x;
      nv += q.y;
    }
    nu *= kInv2Pi;
    nv *= kInv2Pi;
  } else {
    const double2 q = nearv[i];
    nu = q.x;
    nv = q.y;
  }
  if (react) {  // the symmetric pairs' contributions to this particle as a source
    const double2 q = react[i];
    nu += q.x * kInv2Pi;
    nv += q.y * kInv2Pi;
  }
  u[o] = p > 0 ? nu + fu : nu;
  v[o] = p > 0 ? nv + fv : nv;
}

// l2p_tile for every target tile, the waves looping over the tiles.
template <typename R, int PMAX>
__global__ void __launch_bounds__(256) k_l2p(
    const typename Types<R>::Part* __restrict__ tpart, const Tile* __restrict__ ttiles,
    const int32_t* __restrict__ tntiles, const int32_t* __restrict__ tperm,
    const double* __restrict__ root, int levels, int p,
    const typename Types<R>::C* __restrict__ le_all, const uint8_t* __restrict__ leaf_shift,
    int near, const uint32_t* __restrict__ p_off, const uint32_t* __restrict__ s_off,
    const double2* __restrict__ partial, const double2* __restrict__ nearv,
    const double2* __restrict__ react, double* __restrict__ u, double* __restrict__ v) {
  const int nt = *tntiles;
  const int lane = threadIdx.x & 63;
  for (int wid = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6)); wid < nt;
       wid += 4 * gridDim.x)
    l2p_tile<R, PMAX>(wid, lane, tpart, ttiles, tperm, root, levels, p, le_all, leaf_shift, near,
                      p_off, s_off, partial, nearv, react, u, v);
}

inline unsigned nblk(int64_t n, int b) { return unsigned((n + b - 1) / b); }

hipError_t build_schedule(const TreeDev& t, const TargetsDev& tg, int levels, double cut2,
                          hipStream_t st) {
  const P2PSched& s = tg.sched;
  const int64_t mt = tg.max_tiles;
  const unsigned cb = nblk(mt * kSchedLanes, 256) > 0 ? nblk(mt * kSchedLanes, 256) : 1u;
  hipLaunchKernelGGL(k_sched_count, dim3(cb), dim3(256), 0, st, tg.tiles, tg.ntiles, t.tile_off,
                     t.root, levels, cut2, tg.leaf_shift, s.cnt);
  hipLaunchKernelGGL(k_sched_scan, dim3(1), dim3(kScanOneBlock), 0, st, tg.ntiles, mt, s.cnt,
                     s.p_off, s.s_off);
  const int64_t nreact = tg.react ? t.n : 0;
  const unsigned fb = nblk(mt, 256) > 0 ? nblk(mt, 256) : 1u;
  hipLaunchKernelGGL(k_sched_fill, dim3(fb), dim3(256), 0, st, tg.tiles, tg.ntiles, tg.tile_off,
                     s.cnt, s.p_off, s.s_off, s.parts, tg.react, nreact);
  return hipGetLastError();
}

template <typename R, int LPT>
void launch_t(const TreeDev& t, const TargetsDev& tg, int levels, double sigma, double cut2,
              hipStream_t st) {
  using Part = typename Types<R>::Part;
  const auto* part = reinterpret_cast<const Part*>(
      sizeof(R) == 8 ? static_cast<const void*>(t.part64) : static_cast<const void*>(t.part32s));
  const auto* tpart = reinterpret_cast<const Part*>(
      sizeof(R) == 8 ? static_cast<const void*>(tg.part64) : static_cast<const void*>(tg.part32));
  PairK<R> pk{};
  double sd = 1.0;
  if constexpr (sizeof(R) == 8) pk.kexp = -1.0 / (2.0 * sigma * sigma);
  else sd = near_scale(sigma);
  const float far2 = float(P2PMath<R>::kFarSigma2 * sigma * sigma);
  const float ser2 = float(P2PMath<R>::kSeriesSigma2 * sigma * sigma);
  const int wpb = t.waves;
  // bound on the number of parts: target tiles + min(P, chunks / K) with
  // chunks <= target tiles x source tiles and K >= kP2PMinChunks
  const int64_t pairs_bound = tg.max_tiles * t.max_tiles / kP2PMinChunks + 1;
  const int64_t P = p2p_parts(tg.max_tiles);
  int64_t waves = tg.max_tiles + (pairs_bound < P ? pairs_bound : P);
  if (waves > kP2PMaxWaves) waves = kP2PMaxWaves;
  const P2PSched& s = tg.sched;
  double2* react = LPT == 1 ? tg.react : nullptr;
  size_t lds = 0;
  if (react) lds = size_t(wpb) * 128 * sizeof(SymRec<R>);  // react cleared by the schedule
  if (react)
    hipLaunchKernelGGL((k_p2p<R, LPT, true>), dim3(nblk(waves, wpb)), dim3(64 * wpb), lds, st,
                       part, t.leaf_start, t.tile_off, t.tile_box, tpart, tg.part64, tg.tiles,
                       tg.tile_box, s.parts, s.p_off + tg.max_tiles, s.partial, t.root, levels, pk,
                       sd, far2, ser2, cut2, tg.leaf_shift, tg.fine64, s.near, react);
  else
    hipLaunchKernelGGL((k_p2p<R, LPT, false>), dim3(nblk(waves, wpb)), dim3(64 * wpb), 0, st,
                       part, t.leaf_start, t.tile_off, t.tile_box, tpart, tg.part64, tg.tiles,
                       tg.tile_box, s.parts, s.p_off + tg.max_tiles, s.partial, t.root, levels, pk,
                       sd, far2, ser2, cut2, tg.leaf_shift, tg.fine64, s.near, nullptr);
}

template <typename R>
void launch_r(const TreeDev& t, const TargetsDev& tg, int levels, double sigma, double radius,
              hipStream_t st) {
  const double cut2 = near_cut2(radius, sigma, sizeof(R) == 8 ? kFP64 : kFP32);
  if (t.tile == 16) launch_t<R, 4>(t, tg, levels, sigma, cut2, st);
  else if (t.tile == 32) launch_t<R, 2>(t, tg, levels, sigma, cut2, st);
  else launch_t<R, 1>(t, tg, levels, sigma, cut2, st);
}

template <typename R, int PMAX>
void launch_l2p_t(const TreeDev& t, const TargetsDev& tg, int levels, int p, int near, double* u,
                  double* v, hipStream_t st) {
  using C = typename Types<R>::C;
  using Part = typename Types<R>::Part;
  const auto* tpart = reinterpret_cast<const Part*>(
      sizeof(R) == 8 ? static_cast<const void*>(tg.part64) : static_cast<const void*>(tg.part32));
  const C* le = reinterpret_cast<const C*>(t.le);  // levels 2 .. L
  hipLaunchKernelGGL((k_l2p<R, PMAX>), dim3(tile_loop_blocks(tg.max_tiles)), dim3(256), 0, st,
                     tpart, tg.tiles, tg.ntiles, tg.perm, t.root, levels, p, le, tg.leaf_shift,
                     near, tg.sched.p_off, tg.sched.s_off, tg.sched.partial, tg.sched.near,
                     near ? tg.react : nullptr, u, v);
}

template <typename R>
void launch_l2p_r(const TreeDev& t, const TargetsDev& tg, int levels, int p, int near, double* u,
                  double* v, hipStream_t st) {
  if (p <= 8) launch_l2p_t<R, 8>(t, tg, levels, p, near, u, v, st);
  else if (p <= 16) launch_l2p_t<R, 16>(t, tg, levels, p, near, u, v, st);
  else if (p <= 24) launch_l2p_t<R, 24>(t, tg, levels, p, near, u, v, st);
  else if (p <= 32) launch_l2p_t<R, 32>(t, tg, levels, p, near, u, v, st);
  else launch_l2p_t<R, 40>(t, tg, levels, p, near, u, v, st);
}

}  // namespace

// Requested cut-off radius^2: 0 for the paper's split (radius 0); for radius
// < 0 the distance beyond which the two kernels agree in this precision; the
// kernels clamp it to (kMaxRings w_L)^2.
double near_cut2(double radius, double sigma, int prec) {
  if (radius == 0.0) return 0.0;
  if (radius > 0.0) return radius * radius;
  return (prec == kFP64 ? P2PMath<double>::kFarSigma2 : P2PMath<float>::kFarSigma2) * sigma * sigma;
}

hipError_t launch_p2p_schedule(const TreeDev& t, const TargetsDev& tg, int levels, int prec,
                               double sigma, double radius, hipStream_t st) {
  return build_schedule(t, tg, levels, near_cut2(radius, sigma, prec), st);
}

hipError_t launch_p2p(const TreeDev& t, const TargetsDev& tg, int levels, int prec, double sigma,
                      double radius, hipStream_t st) {
  if (prec == kFP64) launch_r<double>(t, tg, levels, sigma, radius, st);
  else launch_r<float>(t, tg, levels, sigma, radius, st);
  return hipGetLastError();
}

hipError_t launch_l2p(const TreeDev& t, const TargetsDev& tg, int levels, int p, int prec,
                      int near, double* u, double* v, hipStream_t st) {
  if (prec == kFP64) launch_l2p_r<double>(t, tg, levels, p, near, u, v, st);
  else launch_l2p_r<float>(t, tg, levels, p, near, u, v, st);
  return hipGetLastError();
}

}  // namespace vfmm
