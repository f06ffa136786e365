// Near field (P2P) with the far-field evaluation (L2P), the near + far sum and
// the scatter back to the caller's particle order fused into one kernel
// (Cruz & Barba 2008, eq. 10: f = f_near + f_far).
//
// P2P: for each target i, the regularised Biot-Savart sum (eq. 6) over the
// particles of the 3 x 3 local list of its leaf (Section 3.3.1), self term
// excluded; it contributes exactly zero because the pair offset is (0, 0).
// L2P: W_far = (-j / (2 pi w)) sum_n L_n ((z - c)/w)^n, Horner's rule.
//
// Work decomposition: one wave per tile of <= T targets of one leaf (tiles built
// with the tree, in leaf order; T = 64, 32 or 16 from the tuning), 64 / T lanes
// per target, each lane taking every (64 / T)-th source of a chunk, the lanes of a
// target summed by shuffles at the end.  Blocks keep the
// hardware's round-robin dealing to the 8 XCDs, which spreads the heavy tiles of
// dense regions over all XCDs (contiguous per-XCD ranges, or ordering tiles by
// cost, were measured 1.7-2x slower on clustered inputs).
// The source loop runs over the 9 leaf ranges of the local list in chunks of T,
// which are exactly the tiles of the source leaf; with T = 64 the source index
// is the same for all lanes of the wave, so sources are fetched with scalar
// loads and broadcast (8 per loop trip, so several loads are in flight).  Source
// coordinates are box-local; the target is shifted once per neighbour leaf by
// the exact centre offset.
//
// Far chunks: when the bounding boxes of the target tile and of a source chunk
// are more than r_c apart, every pair has exp(-r^2 / 2 sigma^2) below half an
// ulp of 1 (r_c^2 = 36 sigma^2 in FP32, 76 sigma^2 in FP64), so 1 - exp rounds
// to exactly 1 and the chunk is summed with the kernel's far form Gamma / r^2,
// which gives bit-identical results without the exponential.
//
// FP32 variant: per-pair arithmetic in FP32 with the hardware exp2 and
// reciprocal (and a short series for 1 - exp when r < sigma / 4, used only in
// chunks whose bounding box comes that close to the tile); partial sums over chunks of 64 sources are added into a
// compensated (TwoSum) FP32 accumulator, which keeps the rounding of long
// source loops (up to ~1e5 sources per target) near the per-term level.
// FP64 variant: plain FP64 with expm1 and division.
#include "p2p_math.hpp"

namespace vfmm {

namespace {

template <typename R, int PMAX, int LPT>
__global__ void __launch_bounds__(512) k_p2p_l2p(
    const typename Types<R>::Part* __restrict__ part, const int32_t* __restrict__ leaf_start,
    const uint32_t* __restrict__ tile_off, const float4* __restrict__ tile_box,
    const typename Types<R>::Part* __restrict__ tpart, const Tile* __restrict__ ttiles,
    const int32_t* __restrict__ tntiles, const float4* __restrict__ ttile_box,
    const int32_t* __restrict__ tperm, const double* __restrict__ root, int levels, int p,
    const typename Types<R>::C* __restrict__ le_leaf, R kexp, R ka, float far2, float ser2,
    int parts, double* __restrict__ u, double* __restrict__ v) {
  using C = typename Types<R>::C;
  constexpr int T = 64 / LPT;  // targets per tile = sources per chunk
  const int wpb = blockDim.x >> 6;
  const int wid = __builtin_amdgcn_readfirstlane(blockIdx.x * wpb + (threadIdx.x >> 6));
  if (wid >= *tntiles) return;
  const int lane = threadIdx.x & 63;
  const int tl = lane % T, grp = lane / T;  // target in tile, source sub-stream
  const Tile tile = ttiles[wid];
  const bool active = tl < tile.count;
  const int32_t i = tile.start + (active ? tl : 0);
  const auto tp = tpart[i];
  const int m = 1 << levels;
  const int bx = tile.leaf & (m - 1), by = tile.leaf >> levels;
  const double w = root[3];

  double nu = 0.0, nv = 0.0;
  if (parts & 1) {
    const R tiny = R(w * w * 0x1p-80);
    const float4 tb = ttile_box[wid];
    Acc32 au{0.f, 0.f}, av{0.f, 0.f};
    for (int oy = -1; oy <= 1; ++oy) {
      const int sy = by + oy;
      if (sy < 0 || sy >= m) continue;
      for (int ox = -1; ox <= 1; ++ox) {
        const int sx = bx + ox;
        if (sx < 0 || sx >= m) continue;
        const int sl = sy * m + sx;
        const int32_t js = leaf_start[sl], je = leaf_start[sl + 1];
        // target relative to the source leaf centre
        const R tx = tp.x - R(double(ox) * w);
        const R ty = tp.y - R(double(oy) * w);
        const float bx0 = tb.x - float(double(ox) * w), bx1 = tb.y - float(double(ox) * w);
        const float by0 = tb.z - float(double(oy) * w), by1 = tb.w - float(double(oy) * w);
        uint32_t ci = tile_off[sl];
        for (int32_t j0 = js; j0 < je; j0 += T, ++ci) {
          const int32_t j1 = min(j0 + T, je);
          const float4 sb = tile_box[ci];
          const float gx = fmaxf(0.f, fmaxf(sb.x - bx1, bx0 - sb.y));
          const float gy = fmaxf(0.f, fmaxf(sb.z - by1, by0 - sb.w));
          R cu = R(0), cv = R(0);
          const float gap2 = gx * gx + gy * gy;
          if (gap2 > far2) {
#pragma unroll 8
            for (int32_t j = j0 + grp; j < j1; j += LPT) {
              const auto s = part[j];
              const R dx = tx - s.x;
              const R dy = ty - s.y;
              const R f = P2PMath<R>::far(s.g, dx * dx + dy * dy);
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
              const R f = P2PMath<R>::near(s.g, r2, kexp);
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
              const R f = P2PMath<R>::near_series(s.g, r2, kexp, ka);
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
    nu *= kInv2Pi;
    nv *= kInv2Pi;
  }

  double fu = 0.0, fv = 0.0;
  if ((parts & 2) && levels >= 2) {
    const R inv_w = R(1.0 / w);
    const C z = cmake<C>(tp.x * inv_w, tp.y * inv_w);
    const C* L = le_leaf + int64_t(tile.leaf) * p;
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

  if (active && grp == 0) {
    const int32_t o = tperm[i];
    u[o] = nu + fu;
    v[o] = nv + fv;
  }
}

template <typename R, int PMAX, int LPT>
void launch_t(const TreeDev& t, const TargetsDev& tg, int levels, int p, double sigma, int parts,
              double* u, double* v, hipStream_t st) {
  using C = typename Types<R>::C;
  using Part = typename Types<R>::Part;
  const auto* part = reinterpret_cast<const Part*>(
      sizeof(R) == 8 ? static_cast<const void*>(t.part64) : static_cast<const void*>(t.part32));
  const auto* tpart = reinterpret_cast<const Part*>(
      sizeof(R) == 8 ? static_cast<const void*>(tg.part64) : static_cast<const void*>(tg.part32));
  const C* le = reinterpret_cast<const C*>(t.le) + (levels >= 2 ? level_offset(levels) * p : 0);
  const double k64 = -1.0 / (2.0 * sigma * sigma);
  const R kexp = sizeof(R) == 8 ? R(k64) : R(k64 * 1.4426950408889634074);
  const float far2 = float(P2PMath<R>::kFarSigma2 * sigma * sigma);
  const float ser2 = float(P2PMath<R>::kSeriesSigma2 * sigma * sigma);
  const R ka = R(1.0 / (2.0 * sigma * sigma));
  const int wpb = tuning_waves();
  const unsigned blocks = unsigned((tg.max_tiles + wpb - 1) / wpb);
  hipLaunchKernelGGL((k_p2p_l2p<R, PMAX, LPT>), dim3(blocks), dim3(64 * wpb), 0, st, part,
                     t.leaf_start, t.tile_off, t.tile_box, tpart, tg.tiles, tg.ntiles,
                     tg.tile_box, tg.perm, t.root, levels, p, le, kexp, ka, far2, ser2, parts, u,
                     v);
}

template <typename R, int PMAX>
void launch_l(const TreeDev& t, const TargetsDev& tg, int levels, int p, double sigma, int parts,
              double* u, double* v, hipStream_t st) {
  if (t.tile == 16) launch_t<R, PMAX, 4>(t, tg, levels, p, sigma, parts, u, v, st);
  else if (t.tile == 32) launch_t<R, PMAX, 2>(t, tg, levels, p, sigma, parts, u, v, st);
  else launch_t<R, PMAX, 1>(t, tg, levels, p, sigma, parts, u, v, st);
}

template <typename R>
void launch_r(const TreeDev& t, const TargetsDev& tg, int levels, int p, double sigma, int parts,
              double* u, double* v, hipStream_t st) {
  if (p <= 8) launch_l<R, 8>(t, tg, levels, p, sigma, parts, u, v, st);
  else if (p <= 16) launch_l<R, 16>(t, tg, levels, p, sigma, parts, u, v, st);
  else if (p <= 24) launch_l<R, 24>(t, tg, levels, p, sigma, parts, u, v, st);
  else if (p <= 32) launch_l<R, 32>(t, tg, levels, p, sigma, parts, u, v, st);
  else launch_l<R, 40>(t, tg, levels, p, sigma, parts, u, v, st);
}

}  // namespace

hipError_t launch_p2p_l2p(const TreeDev& t, const TargetsDev& tg, int levels, int p, int prec,
                          double sigma, int parts, double* u, double* v, hipStream_t st) {
  if (prec == kFP64) launch_r<double>(t, tg, levels, p, sigma, parts, u, v, st);
  else launch_r<float>(t, tg, levels, p, sigma, parts, u, v, st);
  return hipGetLastError();
}

}  // namespace vfmm
