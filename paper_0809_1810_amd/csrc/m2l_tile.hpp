// One column tile of the M2L on the matrix cores (eq. 22): 32 boxes in FP32
// (shared by the single-tree kernel in m2l_mfma.hip and the batched kernel in
// batched.hip).
//
// For a target box b of child class c = (bx & 1, by & 1) the 27 interaction
// offsets t are fixed, so l_b = sum_{t in IL(c)} R_t m_{b - t} with R_t the real
// 2p x 2p block form of the complex M2L operator of offset t.  A tile holds 32
// target boxes of one (level, class); the 4 waves of the workgroup take every
// 4th of the 27 offsets, each software-pipelined (the next offset's operands
// are loaded while this offset's v_mfma_f32_32x32x2_f32 instructions run), and
// the 4 partial 32 x 32 tiles are added through LDS.
//
// Lane layout of the 32x32x2 instruction: A[i][k] with i = lane % 32 and
// B[k][j] with j = lane % 32, K-slot k = lane / 32; D[i][j] in 16 registers per
// lane, row i = 8 (r / 4) + 4 (lane / 32) + r % 4, column j = lane % 32.
#pragma once

#include "vfmm_device.hpp"

namespace vfmm {

typedef float v16f __attribute__((ext_vector_type(16)));

// j-th (0..26) interaction offset of a box of child class (cx, cy): the cells
// of [cx - 3, cx + 2] x [cy - 3, cy + 2] outside [-1, 1]^2, row by row.
__device__ __forceinline__ void nth_offset(int j, int cx, int cy, int& ox, int& oy) {
  int c = 0;
  for (int dy = 0; dy < 6; ++dy)
    for (int dx = 0; dx < 6; ++dx) {
      const int x = cx - 3 + dx, y = cy - 3 + dy;
      if (x >= -1 && x <= 1 && y >= -1 && y <= 1) continue;
      if (c == j) {
        ox = x;
        oy = y;
        return;
      }
      ++c;
    }
}

// Operands of one interaction offset: the packed operator column (MT row
// tiles x ks_n K-steps) and the lanes' source vector entries.
template <int MT>
struct OffsetF32 {
  static constexpr int KMAX = 16 * MT;  // ks_n = p <= 16 MT
  float a[MT][KMAX];
  float b[KMAX];
  // src points at a valid box for every lane (a lane without a source box reads
  // box 0 and keeps zeros); k = 2 ks + hi < 2p always, so the loads carry no
  // per-lane condition and need no branch.
  __device__ __forceinline__ void load(const float* __restrict__ A, const float* src, bool sv,
                                       int ks_n, int hi, int lane) {
#pragma unroll
    for (int ks = 0; ks < KMAX; ++ks) {
      if (ks < ks_n) {
        const float v = src[2 * ks + hi];
        b[ks] = sv ? v : 0.f;
#pragma unroll
        for (int t = 0; t < MT; ++t) a[t][ks] = A[(int64_t(t) * ks_n + ks) * 64 + lane];
      }
    }
  }
};

// LDS of one workgroup: partial tiles of waves 1..3.
template <int MT>
struct M2LTileLds {
  float part[3][MT][16][64];
};

// Tile `local` (class-major: local = class * tiles_per_class + column tile) of
// level lev.  me_l / le_l: the level's multipole / local coefficients (4^lev
// boxes x p, row-major box order); packA: the 40 offsets' operators packed in
// lane order (40 x MT x p x 64 floats).  Called by all 256 threads of the
// workgroup (it synchronises once); writes the M2L sum of the tile's boxes.
template <int MT>
__device__ __forceinline__ void m2l_f32_tile(const float2* __restrict__ me_l,
                                             float2* __restrict__ le_l, int lev, int p, int local,
                                             const float* __restrict__ packA, M2LTileLds<MT>& sh) {
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  const int half = 1 << (lev - 1), m = 1 << lev;
  const int per_class = half * half;
  const int tiles_pc = (per_class + 31) / 32;
  const int c = local / tiles_pc, tt = local % tiles_pc;
  const int cx = c & 1, cy = c >> 1;
  const int col = lane & 31, hi = lane >> 5;
  const int q = tt * 32 + col;
  const bool valid = q < per_class;
  const int qq = valid ? q : 0;
  const int bx = 2 * (qq % half) + cx, by = 2 * (qq / half) + cy;
  const int twop = 2 * p;
  const int ks_n = p;

  v16f acc[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[t][r] = 0.f;

  auto src_of = [&](int ox, int oy, bool& sv) {
    const int sx = bx - ox, sy = by - oy;
    sv = valid && sx >= 0 && sx < m && sy >= 0 && sy < m;
    return reinterpret_cast<const float*>(me_l + (sv ? (int64_t(sy) * m + sx) * p : 0));
  };
  auto a_of = [&](int ox, int oy) {
    return packA + int64_t(m2l_index(ox, oy)) * MT * ks_n * 64;
  };
  OffsetF32<MT> cur, nxt;
  int ox, oy;
  bool sv;
  nth_offset(wv, cx, cy, ox, oy);
  cur.load(a_of(ox, oy), src_of(ox, oy, sv), sv, ks_n, hi, lane);
  for (int j = wv; j < 27; j += 4) {
    if (j + 4 < 27) {
      nth_offset(j + 4, cx, cy, ox, oy);
      const float* s2 = src_of(ox, oy, sv);
      nxt.load(a_of(ox, oy), s2, sv, ks_n, hi, lane);
    }
#pragma unroll
    for (int ks = 0; ks < OffsetF32<MT>::KMAX; ++ks) {
      if (ks < ks_n) {
#pragma unroll
        for (int t = 0; t < MT; ++t)
          acc[t] = __builtin_amdgcn_mfma_f32_32x32x2f32(cur.a[t][ks], cur.b[ks], acc[t], 0, 0, 0);
      }
    }
    cur = nxt;
  }
  if (wv > 0) {
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int r = 0; r < 16; ++r) sh.part[wv - 1][t][r][lane] = acc[t][r];
  }
  __syncthreads();
  if (wv > 0 || !valid) return;
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r)
      acc[t][r] += sh.part[0][t][r][lane] + sh.part[1][t][r][lane] + sh.part[2][t][r][lane];
  float* out = reinterpret_cast<float*>(le_l + (int64_t(by) * m + bx) * p);
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = t * 32 + 8 * (r >> 2) + 4 * hi + (r & 3);
      if (i < twop) out[i] = acc[t][r];
    }
}

// ---------------------------------------------------------------- staged FP32 tile
//
// For p <= 16 (one 32-row tile): the multipoles of every source box of the
// tile's 27 offsets are first copied into LDS by the whole workgroup, row by row
// (each row of the source region is contiguous in memory, so the loads are
// coalesced and all in flight at once), then the waves read their B operands
// from LDS.  The region is split by column parity: the 32 sources of one offset
// are every other box of a row, and become consecutive records of stride
// 2p + 1 (odd) floats, so the 32 lanes of a read fall in distinct banks.  The
// operator columns (A) stay in global memory (L2), loaded one offset ahead.
// Source region of a tile: rows 2 r0 - 2 .. 2 r1 + 3 and columns 2 c0 - 2 ..
// 2 c1 + 3 of the level for target class rows r0..r1 and class columns c0..c1,
// clipped.  With half >= 32 a tile is 32 consecutive boxes of one class row
// (6 rows, at most 68 columns: at most 35 boxes per parity plane and row);
// with half <= 16 it spans at most 12 rows of a level at most 32 boxes wide.
// So 2 x rows x (boxes per plane and row) <= 2 x 6 x 35 records.
constexpr int kStageSlots = 2 * 6 * 35;
constexpr int kStageStride = 33;  // 2p + 1 for p = 16, the largest staged order

template <int W>
struct M2LStagedLds {
  float part[W - 1][16][64];
  float src[kStageSlots * kStageStride];
};

template <int W>
__device__ __forceinline__ void m2l_f32_tile_staged(const float2* __restrict__ me_l,
                                                    float2* __restrict__ le_l, int lev, int p,
                                                    int local, const float* __restrict__ packA,
                                                    M2LStagedLds<W>& sh) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int half = 1 << (lev - 1), m = 1 << lev;
  const int per_class = half * half;
  const int tiles_pc = (per_class + 31) / 32;
  const int c = local / tiles_pc, tt = local % tiles_pc;
  const int cx = c & 1, cy = c >> 1;
  const int col = lane & 31, hi = lane >> 5;
  const int q = tt * 32 + col;
  const bool valid = q < per_class;
  const int qq = valid ? q : 0;
  const int bx = 2 * (qq % half) + cx, by = 2 * (qq / half) + cy;
  const int twop = 2 * p;
  const int ks_n = p;
  const int stride = twop + 1;

  // source region: rows of the tile's first and last target, +-(2..3)
  const int q0 = tt * 32, q1 = min(q0 + 31, per_class - 1);
  const int r0 = q0 / half, r1 = q1 / half;  // class rows of the tile
  const int cx0 = r0 == r1 ? q0 % half : 0, cx1 = r0 == r1 ? q1 % half : half - 1;
  const int y0 = max(2 * r0 - 2, 0), y1 = min(2 * r1 + 3, m - 1);
  const int x0 = max(2 * cx0 - 2, 0), x1 = min(2 * cx1 + 3, m - 1);
  const int rows = y1 - y0 + 1;
  const int wp = (x1 >> 1) - (x0 >> 1) + 1;  // boxes per parity plane and row
  const int rowlen = (x1 - x0 + 1) * twop;   // floats of one source row
  const float* gsrc = reinterpret_cast<const float*>(me_l);
  for (int f = tid; f < rows * rowlen; f += 64 * W) {
    const int r = f / rowlen, rem = f - r * rowlen;
    const int bxo = rem / twop, k = rem - bxo * twop;
    const int sx = x0 + bxo;
    const int slot = ((sx & 1) * rows + r) * wp + ((sx >> 1) - (x0 >> 1));
    sh.src[slot * stride + k] = gsrc[(int64_t(y0 + r) * m + x0) * twop + rem];
  }

  v16f acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  auto slot_of = [&](int ox, int oy, bool& sv) {
    const int sx = bx - ox, sy = by - oy;
    sv = valid && sx >= 0 && sx < m && sy >= 0 && sy < m;
    return sv ? (((sx & 1) * rows + (sy - y0)) * wp + ((sx >> 1) - (x0 >> 1))) * stride : 0;
  };
  auto a_of = [&](int ox, int oy) { return packA + int64_t(m2l_index(ox, oy)) * ks_n * 64 + lane; };
  float a_cur[16], a_nxt[16];
  int ox, oy;
  if (wv < 27) {
    nth_offset(wv, cx, cy, ox, oy);
    const float* A = a_of(ox, oy);
#pragma unroll
    for (int ks = 0; ks < 16; ++ks)
      if (ks < ks_n) a_cur[ks] = A[int64_t(ks) * 64];
  }
  __syncthreads();  // the staged sources are complete
  for (int j = wv; j < 27; j += W) {
    nth_offset(j, cx, cy, ox, oy);
    bool sv;
    const int base = slot_of(ox, oy, sv) + hi;
    if (j + W < 27) {
      int ox2, oy2;
      nth_offset(j + W, cx, cy, ox2, oy2);
      const float* A = a_of(ox2, oy2);
#pragma unroll
      for (int ks = 0; ks < 16; ++ks)
        if (ks < ks_n) a_nxt[ks] = A[int64_t(ks) * 64];
    }
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
      if (ks < ks_n) {
        const float b = sv ? sh.src[base + 2 * ks] : 0.f;
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a_cur[ks], b, acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) a_cur[ks] = a_nxt[ks];
  }
  if (wv > 0) {
#pragma unroll
    for (int r = 0; r < 16; ++r) sh.part[wv - 1][r][lane] = acc[r];
  }
  __syncthreads();
  if (wv > 0 || !valid) return;
#pragma unroll
  for (int w = 0; w < W - 1; ++w)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] += sh.part[w][r][lane];
  float* out = reinterpret_cast<float*>(le_l + (int64_t(by) * m + bx) * p);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int i = 8 * (r >> 2) + 4 * hi + (r & 3);
    if (i < twop) out[i] = acc[r];
  }
}

}  // namespace vfmm
