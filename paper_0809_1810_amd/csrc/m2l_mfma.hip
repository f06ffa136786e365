// M2L on the matrix cores (eq. 22), for the FP32 / BF16 / FP16 evaluations.
//
// With scaled coefficients the M2L operator of an interaction offset t depends
// only on t (40 offsets in [-3,3]^2 \ [-1,1]^2).  Written on interleaved real
// vectors m = (Re M_0, Im M_0, Re M_1, ...), each complex p x p operator becomes
// a real 2p x 2p matrix R_t with 2x2 blocks [[Re T, -Im T], [Im T, Re T]].  For a
// target box b of child class c = (bx & 1, by & 1) the 27 interaction offsets
// are fixed, so
//      l_b = sum_{t in IL(c)} R_t m_{b - t}
// is one real GEMM per (level, class): rows = 2p output components, columns =
// target boxes, K = 27 x 2p (source vectors gathered per column).  Every level
// depends only on the multipoles of the upward sweep, so all levels run in one
// launch.  The L2L chain (Section 3.3.3) then adds each parent's LE top-down.
//
// A 32-box column tile is computed with 32 x 32 matrix instructions by the 4
// waves of a workgroup, each taking every 4th of the 27 offsets with the next
// offset's operands loaded while the current ones multiply, the partial tiles
// added through LDS:
//   FP32  v_mfma_f32_32x32x2_f32  (A, B in float32)
//   BF16  v_mfma_f32_32x32x16_bf16 (A, B rounded to bfloat16, RNE)
//   FP16  v_mfma_f32_32x32x16_f16  (A, B rounded to float16, RNE)
// all accumulating in float32.  A 32x32 instruction takes A[i][k] with
// i = lane % 32 and B[k][j] with j = lane % 32 (K-slot given by lane / 32) and
// returns D[i][j] in 16 registers per lane, row
//   i = 8 (r / 4) + 4 (lane / 32) + r % 4,   column j = lane % 32.
// For BF16/FP16 the source vectors of a level are multiplied by a power of two
// 2^-e (e from the largest magnitude of that level's coefficients) so that
// every input lies in [-1, 1]; the result is divided by the same power of two.
#include "m2l_tile.hpp"

namespace vfmm {

namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

enum Mode { kModeF32 = 0, kModeBF16 = 1, kModeF16 = 2 };

struct LevelTiles {
  int first[kMaxLevels + 2];  // first flat tile of each level (levels 2..L), first[L+1] = total
};

__device__ __forceinline__ float real_block(const double2* T, int p, int i, int k) {
  // R[2n + a][2k' + b] from the complex operator T[n][k']
  const int n = i >> 1, a = i & 1, kk = k >> 1, b = k & 1;
  const double2 t = T[n * p + kk];
  double v;
  if (a == 0) v = b == 0 ? t.x : -t.y;
  else v = b == 0 ? t.y : t.x;
  return float(v);
}

__global__ void __launch_bounds__(256) k_pack_f32(const double2* __restrict__ m2l64, int p, int mt,
                                                  float* __restrict__ out) {
  const int ks_n = p;  // K = 2 per instruction
  const int64_t total = int64_t(kM2LOffsets) * mt * ks_n * 64;
  const int64_t e = blockIdx.x * 256LL + threadIdx.x;
  if (e >= total) return;
  const int lane = int(e % 64);
  const int ks = int((e / 64) % ks_n);
  const int t = int((e / (64LL * ks_n)) % mt);
  const int o = int(e / (64LL * ks_n * mt));
  const int i = t * 32 + (lane & 31), k = 2 * ks + (lane >> 5);
  out[e] = (i < 2 * p && k < 2 * p) ? real_block(m2l64 + int64_t(o) * p * p, p, i, k) : 0.f;
}

template <int MODE>
__global__ void __launch_bounds__(256) k_pack_16(const double2* __restrict__ m2l64, int p, int mt,
                                                 uint16_t* __restrict__ out) {
  const int ks_n = (2 * p + 15) / 16;
  const int64_t total = int64_t(kM2LOffsets) * mt * ks_n * 64 * 8;
  const int64_t e = blockIdx.x * 256LL + threadIdx.x;
  if (e >= total) return;
  const int s = int(e % 8);
  const int lane = int((e / 8) % 64);
  const int ks = int((e / 512) % ks_n);
  const int t = int((e / (512LL * ks_n)) % mt);
  const int o = int(e / (512LL * ks_n * mt));
  const int i = t * 32 + (lane & 31), k = 16 * ks + 8 * (lane >> 5) + s;
  const float v = (i < 2 * p && k < 2 * p) ? real_block(m2l64 + int64_t(o) * p * p, p, i, k) : 0.f;
  if (MODE == kModeBF16) {
    const __bf16 h = __bf16(v);
    out[e] = __builtin_bit_cast(uint16_t, h);
  } else {
    const _Float16 h = _Float16(v);
    out[e] = __builtin_bit_cast(uint16_t, h);
  }
}

__global__ void k_zero_u32(uint32_t* __restrict__ a, int n) {
  if (int(threadIdx.x) < n) a[threadIdx.x] = 0u;
}

// Largest |component| of the level's multipoles, as float bits (order-preserving
// for non-negative floats), combined with an integer atomic max.
__global__ void __launch_bounds__(256) k_absmax(const float* __restrict__ a, int64_t n,
                                                uint32_t* __restrict__ slot) {
  float m = 0.f;
  for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x)
    m = fmaxf(m, fabsf(a[i]));
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(slot, __float_as_uint(m));
}

__device__ __forceinline__ float level_scale(const uint32_t* scales, int lev) {
  const float mx = __uint_as_float(scales[lev]);
  if (!(mx > 0.f)) return 1.f;
  int e;
  (void)frexpf(mx, &e);  // mx = f 2^e, f in [0.5, 1)
  return ldexpf(1.f, -e);
}

// FP32: one workgroup per tile (m2l_tile.hpp).
template <int MT>
__global__ void __launch_bounds__(256) k_m2l_mfma_f32(const float2* __restrict__ me,
                                                      float2* __restrict__ le, int levels, int p,
                                                      LevelTiles lt, const float* __restrict__ packA) {
  __shared__ M2LTileLds<MT> sh;
  const int tile = blockIdx.x;
  if (tile >= lt.first[levels + 1]) return;
  int lev = 2;
  while (tile >= lt.first[lev + 1]) ++lev;
  m2l_f32_tile<MT>(me + level_offset(lev) * p, le + level_offset(lev) * p, lev, p,
                   tile - lt.first[lev], packA, sh);
}

// FP32, p <= 16: the tile's source multipoles staged in LDS first (m2l_tile.hpp),
// W waves per workgroup.
template <int W>
__global__ void __launch_bounds__(64 * W) k_m2l_mfma_f32_staged(const float2* __restrict__ me,
                                                               float2* __restrict__ le, int levels,
                                                               int p, LevelTiles lt,
                                                               const float* __restrict__ packA) {
  __shared__ M2LStagedLds<W> sh;
  const int tile = blockIdx.x;
  if (tile >= lt.first[levels + 1]) return;
  int lev = 2;
  while (tile >= lt.first[lev + 1]) ++lev;
  m2l_f32_tile_staged<W>(me + level_offset(lev) * p, le + level_offset(lev) * p, lev, p,
                         tile - lt.first[lev], packA, sh);
}

// 16-bit operands of one interaction offset: the packed operator columns (MT
// row tiles x ks_n K-steps of 8 values per lane) and the lane's 8 source
// entries per K-step, multiplied by the level's power of two and rounded.
template <int MODE, int MT>
struct Offset16 {
  static constexpr int KS = 2 * MT;  // ks_n = ceil(2p / 16) <= 2 MT
  uint4 a[MT][KS];
  uint4 b[KS];
  __device__ __forceinline__ void load(const uint4* __restrict__ A, const float* src, bool sv,
                                       int ks_n, int twop, int hi, int lane, float sc) {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      if (ks < ks_n) {
        const int k0 = 16 * ks + 8 * hi;
        float f[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) {
          const int k = k0 + s;
          const float v = src[k < twop ? k : twop - 1];  // in bounds; zero past 2p
          f[s] = (sv && k < twop) ? v * sc : 0.f;
        }
        if constexpr (MODE == kModeBF16) {
          v8bf h;
#pragma unroll
          for (int s = 0; s < 8; ++s) h[s] = __bf16(f[s]);
          b[ks] = __builtin_bit_cast(uint4, h);
        } else {
          v8h h;
#pragma unroll
          for (int s = 0; s < 8; ++s) h[s] = _Float16(f[s]);
          b[ks] = __builtin_bit_cast(uint4, h);
        }
#pragma unroll
        for (int t = 0; t < MT; ++t) a[t][ks] = A[(int64_t(t) * ks_n + ks) * 64 + lane];
      }
    }
  }
};

// BF16 / FP16: one workgroup per tile, the 27 offsets split over its 4 waves
// (next offset's operands loaded while the current ones multiply), partial
// tiles added through LDS, as the FP32 tile.
template <int MODE, int MT>
__global__ void __launch_bounds__(256) k_m2l_mfma16(const float2* __restrict__ me,
                                                    float2* __restrict__ le, int levels, int p,
                                                    LevelTiles lt, const uint4* __restrict__ packA,
                                                    const uint32_t* __restrict__ scales) {
  __shared__ float part[3][MT][16][64];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int tile = blockIdx.x;
  if (tile >= lt.first[levels + 1]) return;
  int lev = 2;
  while (tile >= lt.first[lev + 1]) ++lev;
  const int half = 1 << (lev - 1), m = 1 << lev;
  const int per_class = half * half;
  const int tiles_pc = (per_class + 31) / 32;
  const int local = tile - lt.first[lev];
  const int c = local / tiles_pc, tt = local % tiles_pc;
  const int cx = c & 1, cy = c >> 1;
  const int col = lane & 31, hi = lane >> 5;
  const int q = tt * 32 + col;
  const bool valid = q < per_class;
  const int qq = valid ? q : 0;
  const int bx = 2 * (qq % half) + cx, by = 2 * (qq / half) + cy;
  const int twop = 2 * p;
  const float2* me_l = me + level_offset(lev) * p;
  const int ks_n = (twop + 15) / 16;
  const float sc = level_scale(scales, lev);

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
  auto a_of = [&](int ox, int oy) { return packA + int64_t(m2l_index(ox, oy)) * MT * ks_n * 64; };
  Offset16<MODE, MT> cur, nxt;
  int ox, oy;
  bool sv;
  nth_offset(wv, cx, cy, ox, oy);
  cur.load(a_of(ox, oy), src_of(ox, oy, sv), sv, ks_n, twop, hi, lane, sc);
  for (int j = wv; j < 27; j += 4) {
    if (j + 4 < 27) {
      nth_offset(j + 4, cx, cy, ox, oy);
      const float* s2 = src_of(ox, oy, sv);
      nxt.load(a_of(ox, oy), s2, sv, ks_n, twop, hi, lane, sc);
    }
#pragma unroll
    for (int ks = 0; ks < Offset16<MODE, MT>::KS; ++ks) {
      if (ks < ks_n) {
#pragma unroll
        for (int t = 0; t < MT; ++t) {
          if constexpr (MODE == kModeBF16)
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(v8bf, cur.a[t][ks]),
                                                             __builtin_bit_cast(v8bf, cur.b[ks]),
                                                             acc[t], 0, 0, 0);
          else
            acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_f16(__builtin_bit_cast(v8h, cur.a[t][ks]),
                                                            __builtin_bit_cast(v8h, cur.b[ks]),
                                                            acc[t], 0, 0, 0);
        }
      }
    }
    cur = nxt;
  }
  if (wv > 0) {
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int r = 0; r < 16; ++r) part[wv - 1][t][r][lane] = acc[t][r];
  }
  __syncthreads();
  if (wv > 0 || !valid) return;
  const float inv = 1.f / sc;
  float* out = reinterpret_cast<float*>(le + level_offset(lev) * p + (int64_t(by) * m + bx) * p);
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int i = t * 32 + 8 * (r >> 2) + 4 * hi + (r & 3);
      const float sum = acc[t][r] + part[0][t][r][lane] + part[1][t][r][lane] + part[2][t][r][lane];
      if (i < twop) out[i] = sum * inv;
    }
}

// le[l] += L2L(le[l-1]) for the levels a .. c (c - a < kL2LSpan; the M2L part
// is already in le[l]), in one launch: one workgroup per level-a box takes
// its parent's local expansion (final before the launch), completes its own
// box, then its 4 children, then their 16 children, each level kept in LDS
// for the next.  Every box of levels a .. c belongs to exactly one workgroup,
// which reads its M2L part and writes its final expansion.  The four shift
// operators (4 p^2 coefficients) are staged in LDS and each thread loads the
// M2L parts of all its outputs first, so that the levels wait on no global
// loads.
constexpr int kL2LSpan = 3;
constexpr int kL2LPer = ((1 << (2 * (kL2LSpan - 1))) * kMaxP + 255) / 256;  // outputs per thread
size_t l2l_span_lds(int p) { return size_t(4 * p * p + 2 * (1 << (2 * (kL2LSpan - 2))) * p) * sizeof(float2); }

__global__ void __launch_bounds__(256) k_l2l_span(float2* __restrict__ le, int a, int c, int p,
                                                  const float2* __restrict__ B) {
  extern __shared__ float2 l2l_sh[];
  float2* Bs = l2l_sh;  // B[(cls p + n) p + k]
  float2* lv[2] = {Bs + 4 * p * p, Bs + 4 * p * p + (1 << (2 * (kL2LSpan - 2))) * p};
  const int ma = 1 << a;
  const int ax = int(blockIdx.x) & (ma - 1), ay = int(blockIdx.x) >> a;
  // the box (level a + d) and coefficient of this thread's output o
  auto where = [&](int d, int o, int& j, int& n, int64_t& g) {
    j = o / p;
    n = o - j * p;
    const int jx = j & ((1 << d) - 1), jy = j >> d;
    g = level_offset(a + d) * p + ((int64_t((ay << d) + jy) << (a + d)) + (ax << d) + jx) * p + n;
  };
  float2 m2l[kL2LSpan][kL2LPer];
#pragma unroll
  for (int d = 0; d < kL2LSpan; ++d)
#pragma unroll
    for (int r = 0; r < kL2LPer; ++r) {
      const int o = int(threadIdx.x) + r * 256;
      if (a + d <= c && o < (p << (2 * d))) {
        int j, n;
        int64_t g;
        where(d, o, j, n, g);
        m2l[d][r] = le[g];
      }
    }
  for (int i = threadIdx.x; i < 4 * p * p; i += 256) Bs[i] = B[i];
  const float2* lp = le + level_offset(a - 1) * p + (int64_t(ay >> 1) * (ma >> 1) + (ax >> 1)) * p;
  for (int k = threadIdx.x; k < p; k += 256) lv[0][k] = lp[k];
  __syncthreads();
#pragma unroll
  for (int d = 0; d < kL2LSpan; ++d) {
    if (a + d > c) break;  // uniform
    const float2* prev = lv[d & 1];
    float2* cur = lv[(d + 1) & 1];
    const int w = 1 << d;
#pragma unroll
    for (int r = 0; r < kL2LPer; ++r) {
      const int o = int(threadIdx.x) + r * 256;
      if (o >= (p << (2 * d))) break;
      int j, n;
      int64_t g;
      where(d, o, j, n, g);
      const int jx = j & (w - 1), jy = j >> d;
      const int cls = (((ay << d) + jy) & 1) << 1 | (((ax << d) + jx) & 1);
      // parent: the subtree's box of the previous level (for d = 0, the one entry)
      const float2* pe = prev + (d == 0 ? 0 : ((jy >> 1) * (w >> 1) + (jx >> 1)) * p);
      const float2* b = Bs + (cls * p + n) * p;
      float2 acc = m2l[d][r];
      for (int k = n; k < p; ++k) cfma(acc, b[k], pe[k]);
      le[g] = acc;
      if (a + d < c) cur[o] = acc;
    }
    __syncthreads();
  }
}

template <int MODE>
void launch_mode(const TreeDev& t, int levels, int p, const LevelTiles& lt, const void* pack,
                 const uint32_t* scales, hipStream_t st) {
  const int mt = (2 * p + 31) / 32;
  const float2* me = static_cast<const float2*>(t.me);
  float2* le = static_cast<float2*>(t.le);
  if constexpr (MODE == kModeF32) {
    const unsigned tiles = unsigned(lt.first[levels + 1]);
    const float* A = static_cast<const float*>(pack);
    if (mt == 1 && t.m2l_tile == 1)
      hipLaunchKernelGGL((k_m2l_mfma_f32_staged<4>), dim3(tiles), dim3(256), 0, st, me, le, levels,
                         p, lt, A);
    else if (mt == 1 && t.m2l_tile == 2)
      hipLaunchKernelGGL((k_m2l_mfma_f32_staged<8>), dim3(tiles), dim3(512), 0, st, me, le, levels,
                         p, lt, A);
    else if (mt == 1)
      hipLaunchKernelGGL((k_m2l_mfma_f32<1>), dim3(tiles), dim3(256), 0, st, me, le, levels, p, lt, A);
    else if (mt == 2)
      hipLaunchKernelGGL((k_m2l_mfma_f32<2>), dim3(tiles), dim3(256), 0, st, me, le, levels, p, lt, A);
    else
      hipLaunchKernelGGL((k_m2l_mfma_f32<3>), dim3(tiles), dim3(256), 0, st, me, le, levels, p, lt, A);
  } else {
    const unsigned tiles = unsigned(lt.first[levels + 1]);
    const uint4* A = static_cast<const uint4*>(pack);
    if (mt == 1)
      hipLaunchKernelGGL((k_m2l_mfma16<MODE, 1>), dim3(tiles), dim3(256), 0, st, me, le, levels, p, lt, A, scales);
    else if (mt == 2)
      hipLaunchKernelGGL((k_m2l_mfma16<MODE, 2>), dim3(tiles), dim3(256), 0, st, me, le, levels, p, lt, A, scales);
    else
      hipLaunchKernelGGL((k_m2l_mfma16<MODE, 3>), dim3(tiles), dim3(256), 0, st, me, le, levels, p, lt, A, scales);
  }
}

}  // namespace

hipError_t launch_pack_m2l_mfma(const TreeDev& t, int p, int prec, hipStream_t st) {
  const OpsLayout ol = ops_layout(p);
  char* ops = static_cast<char*>(t.ops);
  const double2* m2l64 = reinterpret_cast<const double2*>(ops + ol.m2l64);
  if (prec == kFP32) {
    const int64_t total = int64_t(kM2LOffsets) * ol.mt * ol.ks32 * 64;
    hipLaunchKernelGGL(k_pack_f32, dim3(unsigned((total + 255) / 256)), dim3(256), 0, st, m2l64, p,
                       ol.mt, reinterpret_cast<float*>(ops + ol.mfma32));
  } else {
    const int64_t total = int64_t(kM2LOffsets) * ol.mt * ol.ks16 * 64 * 8;
    if (prec == kM2L_BF16)
      hipLaunchKernelGGL(k_pack_16<kModeBF16>, dim3(unsigned((total + 255) / 256)), dim3(256), 0,
                         st, m2l64, p, ol.mt, reinterpret_cast<uint16_t*>(ops + ol.mfma16));
    else
      hipLaunchKernelGGL(k_pack_16<kModeF16>, dim3(unsigned((total + 255) / 256)), dim3(256), 0,
                         st, m2l64, p, ol.mt, reinterpret_cast<uint16_t*>(ops + ol.mfma16));
  }
  return hipGetLastError();
}

hipError_t launch_downward_mfma(const TreeDev& t, int levels, int p, int prec, hipStream_t st,
                                bool with_l2l) {
  if (levels < 2) return hipSuccess;
  const OpsLayout ol = ops_layout(p);
  char* ops = static_cast<char*>(t.ops);
  uint32_t* scales = reinterpret_cast<uint32_t*>(ops + ol.scales);
  LevelTiles lt{};
  int acc = 0;
  for (int l = 2; l <= levels; ++l) {
    lt.first[l] = acc;
    const int64_t per_class = int64_t(1) << (2 * (l - 1));
    acc += int(4 * ((per_class + 31) / 32));
  }
  lt.first[levels + 1] = acc;
  if (prec != kFP32) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, scales, kMaxLevels + 1);
    for (int l = 2; l <= levels; ++l) {
      const int64_t n = (int64_t(1) << (2 * l)) * 2 * p;
      int nb = int((n + 255) / 256);
      if (nb > 1024) nb = 1024;
      hipLaunchKernelGGL(k_absmax, dim3(nb), dim3(256), 0, st,
                         reinterpret_cast<const float*>(static_cast<const float2*>(t.me) + level_offset(l) * p),
                         n, scales + l);
    }
  }
  if (prec == kFP32) launch_mode<kModeF32>(t, levels, p, lt, ops + ol.mfma32, scales, st);
  else if (prec == kM2L_BF16) launch_mode<kModeBF16>(t, levels, p, lt, ops + ol.mfma16, scales, st);
  else launch_mode<kModeF16>(t, levels, p, lt, ops + ol.mfma16, scales, st);
  if (!with_l2l) return hipGetLastError();
  const float2* B = reinterpret_cast<const float2*>(ops + ol.l2l32);
  float2* le = static_cast<float2*>(t.le);
  // spans of kL2LSpan levels from the deepest up, e.g. 3 .. 4 and 5 .. 7 at L = 7
  int spans[kMaxLevels][2], ns = 0;
  for (int c = levels; c >= 3; c -= kL2LSpan) {
    spans[ns][0] = c - kL2LSpan + 1 < 3 ? 3 : c - kL2LSpan + 1;
    spans[ns][1] = c;
    ++ns;
  }
  for (int s = ns - 1; s >= 0; --s)
    hipLaunchKernelGGL(k_l2l_span, dim3(1u << (2 * spans[s][0])), dim3(256), l2l_span_lds(p), st,
                       le, spans[s][0], spans[s][1], p, B);
  return hipGetLastError();
}

}  // namespace vfmm
