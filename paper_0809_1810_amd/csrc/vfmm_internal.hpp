// Internal declarations of the vortex-particle FMM library (device helpers,
// workspace layout, kernel launchers).  Not part of the public C ABI.
//
// Conventions used by every kernel (Cruz & Barba 2008, Section 3):
//   * complex z = x + j y; the kernels carry the conjugate velocity
//     W = u_x - j u_y, and the velocity of eq. 6 is u = (Re W, -Im W);
//   * level l has 4^l boxes of side w_l = S / 2^l addressed row-major,
//     box = iy * 2^l + ix (Fig. 6);
//   * scaled multipole coefficients M_k = sum_i Gamma_i ((z_i - c)/w)^k
//     (eq. 20 without the -j/2pi factor, divided by w^k);
//   * scaled local coefficients L_n with
//     W(z) = (-j / (2 pi w)) sum_n L_n ((z - c)/w)^n
//     (the LE of Section 3.2.3 multiplied by w^(n+1) and by 2 pi j);
//   * with these scalings every translation operator is level independent:
//       M2M: M'_n = sum_{k<=n} C(n,k) d^(n-k) 2^-n M_k,       d = (c_child - c_parent)/w_child
//       M2L: L_n  = sum_k (-1)^n C(n+k,k) t^-(n+k+1) M_k,      t = (c_target - c_source)/w
//       L2L: L'_n = sum_{k>=n} C(k,n) d^(k-n) 2^-(k+1) L_k,   d = (c_child - c_parent)/w_child
//     where d in {(+-1 +- j)/2} and t is an integer offset in [-3,3]^2 \ [-1,1]^2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/vfmm.h"

namespace vfmm {

// Status of a failed HIP call: running out of device memory is reported as
// such, every other runtime error as VFMM_ERR_HIP.
inline vfmm_status_t hip_status(hipError_t e) {
  return e == hipErrorOutOfMemory ? VFMM_ERR_OUT_OF_MEMORY : VFMM_ERR_HIP;
}
// Message returned by vfmm_last_error() on the calling thread.
void set_last_error(const char* msg);

constexpr int kMaxP = 40;
constexpr int kMaxLevels = 12;
constexpr int kTile = 64;            // P2P targets per wave tile (default; the batched path)
constexpr int kTileMin = 16;         // smallest tunable tile (4 lanes per target)
constexpr int kSubLevels = 4;        // within a leaf, particles are ordered by their cell at level L + 4
constexpr int kSortItems = 2;        // radix-sort elements per thread
constexpr int kSortBlock = 1024;     // radix-sort threads per block (16 waves)
constexpr int kSortPerBlock = kSortItems * kSortBlock;
constexpr int kScanItems = 8;
constexpr int kScanBlock = 256;
constexpr int kScanPerBlock = kScanItems * kScanBlock;
constexpr int kBBoxBlocks = 512;
constexpr int kReduceBlocks = 512;
constexpr int kM2LOffsets = 49;      // 7x7 table indexed by t = (ox, oy) in [-3,3]^2
constexpr int kShift64P = 16;        // reduced precision: P2M, M2M, L2L in float64 above this p
// Near-field schedule: the source chunks of every target tile are cut into
// parts so that a launch has about p2p_parts(max_tiles) parts of similar size
// (4 per target tile, at least 4096, at most 65536: measured on clustered 1M
// particles, 16384 parts left 15 % and 65536 parts under 1 % to gain).
constexpr int64_t kP2PPartsMin = 4096;
constexpr int64_t kP2PPartsMax = 65536;
constexpr int kP2PMinChunks = 8;      // smallest part worth a wave (source chunks)
// Per-tile kernels of uniform cost (tile boxes, L2P) loop over the tiles with
// at most this many workgroups of 4 waves, instead of one wave per tile of
// capacity (most of which would find no tile).
constexpr int kTileLoopBlocks = 4096;
inline unsigned tile_loop_blocks(int64_t max_tiles) {
  const int64_t b = (max_tiles + 3) / 4;
  return unsigned(b < kTileLoopBlocks ? (b > 0 ? b : 1) : kTileLoopBlocks);
}
constexpr int kP2PMaxWaves = 262144;  // near-field grid cap (waves loop over the parts)
inline __host__ __device__ int64_t p2p_parts(int64_t max_tiles) {
  const int64_t t = 4 * max_tiles;
  return t < kP2PPartsMin ? kP2PPartsMin : (t > kP2PPartsMax ? kP2PPartsMax : t);
}

enum Precision : int32_t {
  kFP64 = 0,
  kFP32 = 1,
  kM2L_BF16 = 2,
  kM2L_FP16 = 3,
};

// Particle record in leaf-sorted order: offsets from the leaf centre, circulation.
struct __align__(32) Part64 { double x, y, g, pad; };
struct __align__(16) Part32 { float x, y, g, pad; };

struct Tile { int32_t leaf, start, count, pad; };

// FP32 near field in units of the Gaussian width: with x' = s x,
// s = sqrt(log2(e) / (2 sigma^2)), exp(-r^2 / 2 sigma^2) = exp2(-r'^2).
inline __host__ __device__ double near_scale(double sigma) {
  return sqrt(1.4426950408889634074 / (2.0 * sigma * sigma));
}

// One near-field work part: chunks [v0, v1) of the target tile's sequence of
// source chunks (its local list row by row); slot >= 0 when the tile is split
// and the part writes partial sums instead of the result.
struct P2PPart { int32_t tile, v0, v1, slot; };

struct P2PSched {
  uint32_t* cnt;      // [max_tiles + 1] source chunks per target tile (exclusive scan)
  uint32_t* p_off;    // [max_tiles + 1] first part of each tile; p_off[max_tiles] = parts
  uint32_t* s_off;    // [max_tiles + 1] first partial slot of each split tile
  P2PPart* parts;     // [max_tiles + p2p_parts(max_tiles)]
  double2* partial;   // [2 p2p_parts(max_tiles)][kTile] near-field sums (u, v) of one part
  uint32_t* scan_tmp;
  double2* near;      // [targets] near field (times 1 / 2 pi) of single-part tiles, sorted order
};

inline __host__ __device__ int64_t level_offset(int l) {
  // boxes of levels 2 .. l-1 stored before level l
  int64_t off = 0;
  for (int k = 2; k < l; ++k) off += int64_t(1) << (2 * k);
  return off;
}

inline __host__ __device__ int64_t n_boxes_2_to(int L) {
  return L < 2 ? 0 : level_offset(L + 1);
}

struct Layout {
  size_t root, bbox, keys0, keys1, idx0, idx1, counts, scan_tmp;
  size_t leaf_start, tile_off, tiles, ntiles, tile_box;
  size_t sched_cnt, sched_poff, sched_soff, sched_parts, sched_partial, sched_near;
  size_t part64, part32, part32s, react, xy, me, le, me32, le32, ops, check, total;
  int64_t n, nleaves, max_tiles, sort_blocks, count_len;
  int levels, p_max;
};

Layout make_layout(int64_t n, int levels, int p_max);

// Device tree state: pointers into the caller's workspace.
struct TreeDev {
  int64_t n;             // particles
  double* root;          // [0]=x0 [1]=y0 [2]=S [3]=w_L
  uint32_t* keys;        // sorted leaf keys
  int32_t* perm;         // sorted position -> input index
  int32_t* leaf_start;   // [nleaves + 1]
  int tile;              // particles per P2P tile: 64, 32 or 16 (64 / lanes per target)
  int waves;             // waves per workgroup of the near-field launch: 1, 2, 4 or 8
  int m2l_tile;          // FP32 matrix-core M2L tile for p <= 16: 0 operands in registers,
                         // 1 / 2 sources staged in LDS with 4 / 8 waves per workgroup
  int sym;               // near field at the particles with the leaf pairs of the local list
                         // evaluated once (both directions; 64-particle tiles only)
  int64_t max_tiles;     // capacity of the tile arrays
  Tile* tiles;           // P2P target tiles (<= tile consecutive particles of one leaf)
  int32_t* ntiles;       // device count of tiles
  uint32_t* tile_off;    // [nleaves + 1] first tile of each leaf
  float4* tile_box;      // per tile: (xmin, xmax, ymin, ymax) in its leaf's local frame
  Part64* part64;
  Part32* part32;
  Part32* part32s;       // FP32 near-field sources in units of the Gaussian width (per evaluation)
  void* me;
  void* le;
  void* me32;            // float32 copies for the float64-shift path (p > kShift64P)
  void* le32;
  void* ops;
  unsigned long long* check;  // [2] counters of the opt-in finiteness check
  double2* react;        // [n] sorted order: near-field sums the symmetric pairs add to their
                         // source particles (unscaled, before 1 / 2 pi)
  P2PSched sched;        // near-field schedule of the particles as targets
};

// Evaluation points of the near-field and L2P kernels: the tree's own particles,
// or a separate point set sorted into the tree's leaves (same tile size).
// Points with NaN coordinates produce NaN velocities.
struct TargetsDev {
  const Part64* part64;  // leaf-local coordinates (g unused for separate points)
  const Part32* part32;
  const Tile* tiles;
  const int32_t* ntiles;
  const float4* tile_box;
  const uint32_t* tile_off;  // [nleaves + 1] first tile of each leaf
  const int32_t* perm;   // sorted position -> caller's index
  int64_t max_tiles;
  P2PSched sched;
  // adaptive tree (NULL: every target leaf is a leaf-level box): per
  // leaf-level box f, k = L - level of the adaptive leaf holding it; a tile's
  // leaf is then the leaf-level box at the lower-left corner of its adaptive
  // leaf, which is box (f_x >> k, f_y >> k) of level L - k
  const uint8_t* leaf_shift;
  // adaptive tree: per target the tree's leaf-local record, with the
  // leaf-level box in place of the circulation (offsets to the sources)
  const Part64* fine64;
  // symmetric near field (targets = the tree's particles, uniform tree,
  // 64-particle tiles; NULL otherwise): a pair of two different tiles of the
  // local list with enough particles is evaluated once, by the earlier tile,
  // which also adds the opposite contribution to the source particle's entry
  // here; the later tile skips it
  double2* react;
};

inline TargetsDev self_targets(const TreeDev& t, const Layout& lay) {
  TargetsDev tg{t.part64, t.part32, t.tiles, t.ntiles, t.tile_box, t.tile_off, t.perm,
                lay.max_tiles, t.sched};
  tg.react = t.sym ? t.react : nullptr;
  return tg;
}

// Workspace of a separate evaluation-point set of nt points at leaf level L.
struct TargetLayout {
  size_t keys0, keys1, idx0, idx1, counts, scan_tmp, leaf_start, tile_off, tiles, ntiles,
      tile_box, sched_cnt, sched_poff, sched_soff, sched_parts, sched_partial,
      sched_near, part64,
      part32, total;
  int64_t nt, nleaves, max_tiles, sort_blocks, count_len;
};

TargetLayout make_target_layout(int64_t nt, int levels);

// Workspace of the adaptive target set of a tree of n particles: the target
// layout plus the box counts of levels 0 .. L, the per-box level shift and the
// targets' caller indices.
struct AdaptiveLayout {
  TargetLayout targets;
  size_t counts, shift, perm, fine64, total;
};
AdaptiveLayout make_adaptive_layout(int64_t n, int levels);

// ---------------------------------------------------------------- launchers
// All launchers enqueue on `stream` and return hipSuccess or the launch error.
hipError_t launch_build_tree(const double* x, const double* y, int64_t n, int levels,
                             const double* domain, const Layout& lay, char* ws, int tile,
                             TreeDev& t, hipStream_t stream);
// Tuning parameters (process-wide): the P2P tile size and waves per workgroup
// that trees built from now on take (each tree keeps its own).
int tuning_tile();
int tuning_waves();
int tuning_m2l_tile();
int tuning_sym();
// Circulations into the sorted particle records (part32, and part64 when
// with64: float64 near field or expansions); with sigma > 0 also the FP32
// near-field sources scaled by sqrt(log2(e) / (2 sigma^2)) (part32s).
hipError_t launch_gather_gamma(const TreeDev& t, const double* gamma, int64_t n, double sigma,
                               bool with64, hipStream_t stream);
hipError_t launch_build_ops(const TreeDev& t, int p, int prec, hipStream_t stream);
hipError_t launch_p2m(const TreeDev& t, int levels, int p, int prec, hipStream_t stream);
hipError_t launch_m2m(const TreeDev& t, int levels, int p, int prec, hipStream_t stream);
hipError_t launch_downward(const TreeDev& t, int levels, int p, int prec, hipStream_t stream);
// Reduced-precision downward sweep: M2L of all levels on the matrix cores
// (prec = kFP32, kM2L_BF16 or kM2L_FP16), then the L2L chain.
hipError_t launch_pack_m2l_mfma(const TreeDev& t, int p, int prec, hipStream_t stream);
// with_l2l = false: the M2L of every level only (each level's LE holds its
// interaction-list sum), for a downward sweep whose L2L runs in float64.
hipError_t launch_downward_mfma(const TreeDev& t, int levels, int p, int prec, hipStream_t stream,
                                bool with_l2l = true);
// Reduced-precision evaluation with float64 shifts (p > kShift64P): the
// float64 multipoles of t.me (P2M and M2M in float64) rounded to float32 into
// t.me32, M2L on the matrix cores into t.le32, the L2L chain in float64 into
// t.le (each level: its M2L sum widened plus the shifted parent LE), and every
// level rounded back into t.le32 for the float32 L2P.
hipError_t launch_downward_shift64(const TreeDev& t, int levels, int p, int prec,
                                   hipStream_t stream);
// radius: distance cut-off of the near field (0 = off, < 0 = the distance at
// which the regularised and singular kernels agree in this precision).
// The near-field work schedule of target set tg (launch_p2p_schedule), then
// the near-field kernel over it (launch_p2p, same radius), which leaves its
// sums in the schedule's buffers (tg.sched.near, tg.sched.partial).
hipError_t launch_p2p_schedule(const TreeDev& t, const TargetsDev& tg, int levels, int prec,
                               double sigma, double radius, hipStream_t stream);
// The requested cut-off radius^2 of the kernels (0: the paper's split).
double near_cut2(double radius, double sigma, int prec);
hipError_t launch_p2p(const TreeDev& t, const TargetsDev& tg, int levels, int prec, double sigma,
                      double radius, hipStream_t stream);
// Writes u, v in the caller's order: the near-field sums of launch_p2p
// (near != 0; the parts of split tiles added in part order) plus the far field
// of the leaves' LEs of order p (p = 0: none; with neither, zeros).
hipError_t launch_l2p(const TreeDev& t, const TargetsDev& tg, int levels, int p, int prec,
                      int near, double* u, double* v, hipStream_t stream);
// Sorts nt evaluation points into the leaves of tree t (built with `levels`),
// with leaf-local coordinates (NaN outside the closed root square) and tiles of
// t.tile points.
hipError_t launch_build_targets(const double* xt, const double* yt, int64_t nt, const TreeDev& t,
                                int levels, const TargetLayout& lay, char* ws, TargetsDev& out,
                                hipStream_t stream);
// The tree's particles as targets of the adaptive tree (box split while it
// holds more than s particles, down to the leaf level): each particle sorted
// into its adaptive leaf, coordinates relative to that leaf's centre, tiles of
// t.tile targets of one adaptive leaf.
hipError_t launch_build_adaptive(const TreeDev& t, int levels, int64_t s,
                                 const AdaptiveLayout& lay, char* ws, TargetsDev& out,
                                 hipStream_t stream);
// Per-point log10 of |dW| / max |W_ref| (metrics[2] holds max |W_ref|).
hipError_t launch_error_field(const double* u, const double* v, const double* ur,
                              const double* vr, int64_t n, const double* metrics, double* out,
                              hipStream_t stream);
// Targets: particle indices (targets, or all when NULL and xt is NULL) or
// separate points (xt, yt).
hipError_t launch_direct(const double* x, const double* y, const double* g, int64_t n,
                         double sigma, const int64_t* targets, const double* xt,
                         const double* yt, int64_t nt, double* u, double* v, hipStream_t stream);
// Finiteness check: counter[0] = 0 (a fill kernel, so that the clear can be
// captured in a graph), then counter[0] += number of non-finite values among
// a[k * stride], k < n (one launch per array).
hipError_t launch_clear_counter(unsigned long long* counter, hipStream_t stream);
hipError_t launch_count_nonfinite(const double* a, int64_t n, int64_t stride,
                                  unsigned long long* counter, hipStream_t stream);
hipError_t launch_error_metrics(const double* u, const double* v, const double* ur,
                                const double* vr, int64_t n, double* partial, double* out,
                                hipStream_t stream);
// Heun's method (advect.hip): x* = x + dt u; x += dt/2 (u1 + u2).
hipError_t launch_heun_predict(const double* x, const double* y, const double* u, const double* v,
                               int64_t n, double dt, double* xs, double* ys, hipStream_t stream);
hipError_t launch_heun_correct(double* x, double* y, const double* u1, const double* v1,
                               const double* u2, const double* v2, int64_t n, double dt,
                               hipStream_t stream);
size_t ops_bytes(int p);

// Scans inside one workgroup of kScanOneBlock threads (16 waves): the
// one-launch scans of arrays up to kScanOneMax elements, and the near-field
// schedule's offsets.  A round takes 4 consecutive elements per thread (one
// 16-byte access, so a wave reads 1 KB in one instruction); a pass issues the
// loads of kScanOneRounds rounds before scanning them in order.
constexpr int kScanOneBlock = 1024;
constexpr int kScanOneRounds = 4;
constexpr int64_t kScanOneRound = int64_t(kScanOneBlock) * 4;
constexpr int64_t kScanOneMax = 65536;
// Elements i .. i + 3 of a (zeros at and past n); a 16-byte aligned.
__device__ inline uint4 scan_load4(const uint32_t* a, int64_t i, int64_t n) {
  if (i + 3 < n) return *reinterpret_cast<const uint4*>(a + i);
  uint4 q = make_uint4(0u, 0u, 0u, 0u);
  if (i < n) q.x = a[i];
  if (i + 1 < n) q.y = a[i + 1];
  if (i + 2 < n) q.z = a[i + 2];
  return q;
}
// Writes the exclusive prefixes ex, ex + q.x, ... of elements i .. i + 3 (below n).
__device__ inline void scan_store4(uint32_t* a, int64_t i, int64_t n, uint4 q, uint32_t ex) {
  uint4 o;
  o.x = ex;
  o.y = o.x + q.x;
  o.z = o.y + q.y;
  o.w = o.z + q.z;
  if (i + 3 < n) {
    *reinterpret_cast<uint4*>(a + i) = o;
    return;
  }
  if (i < n) a[i] = o.x;
  if (i + 1 < n) a[i + 1] = o.y;
  if (i + 2 < n) a[i + 2] = o.z;
}
// x plus the DPP-moved x (0 where the move has no source or the row is
// masked), in unsigned (modulo 2^32) arithmetic.
template <int CTRL, int ROW_MASK, bool BOUND>
__device__ __forceinline__ uint32_t dpp_add(uint32_t x) {
  return x + uint32_t(__builtin_amdgcn_update_dpp(0, int(x), CTRL, ROW_MASK, 0xf, BOUND));
}
// Inclusive scan over a wave by DPP: Hillis-Steele within each row of 16
// lanes (row_shr 1, 2, 4, 8, zeros shifted in), then the last lane of row 0
// added to row 1 and of row 2 to row 3 (row_bcast:15), then that of row 1 to
// rows 2 and 3 (row_bcast:31).
__device__ inline uint32_t wave_scan_incl_u32(uint32_t x) {
  x = dpp_add<0x111, 0xf, true>(x);    // row_shr:1
  x = dpp_add<0x112, 0xf, true>(x);    // row_shr:2
  x = dpp_add<0x114, 0xf, true>(x);    // row_shr:4
  x = dpp_add<0x118, 0xf, true>(x);    // row_shr:8
  x = dpp_add<0x142, 0xa, false>(x);   // row_bcast:15, rows 1 and 3
  x = dpp_add<0x143, 0xc, false>(x);   // row_bcast:31, rows 2 and 3
  return x;
}
// Inclusive scan within each row of 16 lanes (row_shr 1, 2, 4, 8).
__device__ inline uint32_t row_scan_incl_u32(uint32_t x) {
  x = dpp_add<0x111, 0xf, true>(x);
  x = dpp_add<0x112, 0xf, true>(x);
  x = dpp_add<0x114, 0xf, true>(x);
  x = dpp_add<0x118, 0xf, true>(x);
  return x;
}
// Exclusive prefix of one value per thread over the workgroup, and the
// workgroup total; ws: 16 entries of LDS.  Every thread must call it.  The
// waves' totals are scanned by the first 16 lanes of each wave (row_shr within
// row 0) and read back with readlane.
__device__ inline uint32_t block1k_scan_excl(uint32_t v, uint32_t* total, uint32_t* ws) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const uint32_t incl = wave_scan_incl_u32(v);
  if (lane == 63) ws[wave] = incl;
  __syncthreads();
  const uint32_t a = row_scan_incl_u32(lane < 16 ? ws[lane] : 0u);
  __syncthreads();
  const uint32_t pre = wave ? uint32_t(__builtin_amdgcn_readlane(int(a), wave - 1)) : 0u;
  *total = uint32_t(__builtin_amdgcn_readlane(int(a), 15));
  return pre + incl - v;
}

// Three exclusive prefixes at once (one value of each of three sequences per
// thread) over the workgroup, with the totals; ws: 3 x 16 entries of LDS.
// Every thread must call it.  Each wave's totals are scanned by its first 16
// lanes (row_shr within row 0) and read back with readlane.
__device__ inline uint3 block1k_scan3_excl(uint3 v, uint3* total, uint32_t* ws) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x >> 6));
  const uint32_t ix = wave_scan_incl_u32(v.x), iy = wave_scan_incl_u32(v.y),
                 iz = wave_scan_incl_u32(v.z);
  if (lane == 63) {
    ws[wave] = ix;
    ws[16 + wave] = iy;
    ws[32 + wave] = iz;
  }
  __syncthreads();
  const uint32_t a = row_scan_incl_u32(lane < 16 ? ws[lane] : 0u);
  const uint32_t b = row_scan_incl_u32(lane < 16 ? ws[16 + lane] : 0u);
  const uint32_t c = row_scan_incl_u32(lane < 16 ? ws[32 + lane] : 0u);
  __syncthreads();
  // lane w of row 0 holds the inclusive sums of the totals of waves 0 .. w
  const uint32_t px = wave ? uint32_t(__builtin_amdgcn_readlane(int(a), wave - 1)) : 0u;
  const uint32_t py = wave ? uint32_t(__builtin_amdgcn_readlane(int(b), wave - 1)) : 0u;
  const uint32_t pz = wave ? uint32_t(__builtin_amdgcn_readlane(int(c), wave - 1)) : 0u;
  *total = make_uint3(uint32_t(__builtin_amdgcn_readlane(int(a), 15)),
                      uint32_t(__builtin_amdgcn_readlane(int(b), 15)),
                      uint32_t(__builtin_amdgcn_readlane(int(c), 15)));
  return make_uint3(px + ix - v.x, py + iy - v.y, pz + iz - v.z);
}

// Shared building blocks (tree.hip).
hipError_t scan_exclusive(uint32_t* a, int64_t n, uint32_t* tmp, hipStream_t st);
// Two arrays of n elements at once; tmp holds 2 ceil(n / kScanPerBlock) entries.
hipError_t scan_exclusive2(uint32_t* a, uint32_t* b, int64_t n, uint32_t* tmp, hipStream_t st);
// Stable LSD radix sort of (key, index) pairs on the low `bits` key bits; on
// return k0/i0 point to the sorted arrays (the other pair is scratch).
hipError_t radix_sort_pairs(uint32_t*& k0, uint32_t*& k1, int32_t*& i0, int32_t*& i1, int64_t n,
                            int bits, uint32_t* counts, uint32_t* tmp, hipStream_t st);
hipError_t launch_tile_box(const Tile* tiles, const int32_t* ntiles, int64_t max_tiles,
                           const Part32* p32, float4* box, hipStream_t st);

}  // namespace vfmm
