// Per-tile alpha compositing on gfx950 (the 3D Gaussian splatting rasteriser's
// blending, Sec. 4.4): forward front-to-back with the final transmittance and
// the last contributor saved per pixel, and the reverse walk that turns dL/dI
// into per-Gaussian screen-space gradients.
//
// One workgroup of 256 threads per screen tile, one pixel per thread; each
// 64-lane wavefront owns an 8x8 block of the tile so that a Gaussian whose
// extent box misses that block is skipped by the whole wavefront.  Records of
// the tile's depth-ordered list are staged through LDS in batches.
#include "internal.h"

namespace sixdgs {
namespace {

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

// Staged record: conic pre-scaled so that exp(-q/2) = exp2(p2).
struct Staged {
  float4 a;  // u, v, cA = -log2e/2 Qxx, cB = -log2e Qxy
  float4 b;  // cC = -log2e/2 Qyy, alpha_cond, ex, ey
  float4 c;  // r, g, b, entry id (bits)
};

__device__ __forceinline__ Staged stage(const Rec& r, uint32_t e) {
  Staged s;
  s.a = make_float4(r.a.x, r.a.y, -0.5f * kLog2e * r.a.z, -kLog2e * r.a.w);
  s.b = make_float4(-0.5f * kLog2e * r.b.x, r.b.y, r.b.z, r.b.w);
  s.c = make_float4(r.c.x, r.c.y, r.c.z, __uint_as_float(e));
  return s;
}

// The one evaluation of a Gaussian at a pixel used by both directions, written
// with explicit roundings so that both compile to the same arithmetic.
__device__ __forceinline__ float power2(const float4& A, float cC, float dx, float dy) {
  const float t = __fmaf_rn(A.z, dx, __fmul_rn(A.w, dy));
  return __fmaf_rn(t, dx, __fmul_rn(__fmul_rn(cC, dy), dy));
}

__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }

// Does the extent box (with a one-pixel margin) reach the wavefront's 8x8 block
// of pixel centres [x0, x0 + 7] x [y0, y0 + 7]?
__device__ __forceinline__ bool box_hits(const float4& A, const float4& B, float x0, float y0) {
  return (A.x + B.z >= x0 - 1.0f) && (A.x - B.z <= x0 + 8.0f) && (A.y + B.w >= y0 - 1.0f) &&
         (A.y - B.w <= y0 + 8.0f);
}

__device__ __forceinline__ int find_view(const ViewTable& vt, int tile) {
  int v = 0;
  for (int k = 1; k < vt.nview; k++)
    if (tile >= vt.v[k].tile_base) v = k;
  return v;
}

template <int TW>
struct TileMap {
  static constexpr int TH = 256 / TW;
  static constexpr int BX = TW / 8;  // 8x8 blocks per tile row
  // pixel of this thread inside the tile and the block origin of its wavefront
  __device__ static void pixel(int tid, int& lx, int& ly, int& bx0, int& by0) {
    const int w = tid >> 6, l = tid & 63;
    bx0 = (w % BX) * 8;
    by0 = (w / BX) * 8;
    lx = bx0 + (l & 7);
    ly = by0 + (l >> 3);
  }
};

template <int TW>
__global__ void __launch_bounds__(kBlock) k_blend_fwd(ViewTable vt, DevSettings ds, const Rec* __restrict__ rec,
                                                      const uint2* __restrict__ ranges,
                                                      const uint32_t* __restrict__ pval, BlendState bs, int batch) {
  __shared__ Staged s_rec[kBlock];
  const int tile = blockIdx.x;
  const int vi = find_view(vt, tile);
  const ViewDesc& vd = vt.v[vi];
  const int local = tile - vd.tile_base;
  const int tx = local % vd.ntx, ty = local / vd.ntx;
  int lx, ly, bx0, by0;
  TileMap<TW>::pixel(threadIdx.x, lx, ly, bx0, by0);
  const int px = tx * TW + lx, py = ty * TileMap<TW>::TH + ly;
  const bool inside = px < vd.W && py < vd.H;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  const float wx0 = (float)(tx * TW + bx0) + 0.5f, wy0 = (float)(ty * TileMap<TW>::TH + by0) + 0.5f;

  const uint2 rg = ranges[tile];
  float T = 1.0f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  uint32_t last = 0, cnt = 0;
  bool done = !inside;
  for (uint32_t b0 = rg.x; b0 < rg.y; b0 += batch) {
    if (__syncthreads_count(!done) == 0) break;
    const uint32_t nb = min((uint32_t)batch, rg.y - b0);
    if (threadIdx.x < nb) {
      const uint32_t e = pval[b0 + threadIdx.x];
      s_rec[threadIdx.x] = stage(rec[e], e);
    }
    __syncthreads();
    if (__ballot(!done) != 0) {
      for (uint32_t j = 0; j < nb; j++) {
        const float4 A = s_rec[j].a;
        const float4 B = s_rec[j].b;
        if (!box_hits(A, B, wx0, wy0)) continue;
        if (done) continue;
        const float dx = fx - A.x, dy = fy - A.y;
        const float araw = B.y * exp2_fast(power2(A, B.x, dx, dy));
        const float a = fminf(kAlphaMax, araw);
        if (a < kAlphaMin) continue;
        const float Tn = T * (1.0f - a);
        if (Tn < kTMin) {
          done = true;
          continue;
        }
        const float4 Cc = s_rec[j].c;
        const float wgt = a * T;
        C0 += Cc.x * wgt;
        C1 += Cc.y * wgt;
        C2 += Cc.z * wgt;
        T = Tn;
        last = b0 - rg.x + j + 1;
        cnt++;
      }
    }
    __syncthreads();
  }
  if (inside) {
    const int64_t HW = (int64_t)vd.W * vd.H;
    const int64_t pix = (int64_t)py * vd.W + px;
    vd.img[pix] = C0 + T * ds.bg[0];
    vd.img[HW + pix] = C1 + T * ds.bg[1];
    vd.img[2 * HW + pix] = C2 + T * ds.bg[2];
    bs.T_final[vd.pix_base + pix] = T;
    bs.last[vd.pix_base + pix] = last;
    if (bs.counts) bs.counts[vd.pix_base + pix] = cnt;
  }
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
  return v;
}

template <int TW>
__global__ void __launch_bounds__(kBlock) k_blend_bwd(ViewTable vt, DevSettings ds, const Rec* __restrict__ rec,
                                                      const uint2* __restrict__ ranges,
                                                      const uint32_t* __restrict__ pval, BlendState bs,
                                                      float* __restrict__ g2d, int batch) {
  __shared__ Staged s_rec[kBlock];
  __shared__ uint32_t s_maxlast;
  const int tile = blockIdx.x;
  const int vi = find_view(vt, tile);
  const ViewDesc& vd = vt.v[vi];
  const int local = tile - vd.tile_base;
  const int tx = local % vd.ntx, ty = local / vd.ntx;
  int lx, ly, bx0, by0;
  TileMap<TW>::pixel(threadIdx.x, lx, ly, bx0, by0);
  const int px = tx * TW + lx, py = ty * TileMap<TW>::TH + ly;
  const bool inside = px < vd.W && py < vd.H;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  const float wx0 = (float)(tx * TW + bx0) + 0.5f, wy0 = (float)(ty * TileMap<TW>::TH + by0) + 0.5f;

  float T = 1.f, dC0 = 0.f, dC1 = 0.f, dC2 = 0.f;
  uint32_t last = 0;
  if (inside) {
    const int64_t HW = (int64_t)vd.W * vd.H;
    const int64_t pix = (int64_t)py * vd.W + px;
    T = bs.T_final[vd.pix_base + pix];
    last = bs.last[vd.pix_base + pix];
    dC0 = vd.dimg[pix];
    dC1 = vd.dimg[HW + pix];
    dC2 = vd.dimg[2 * HW + pix];
  }
  // colour behind the current Gaussian, starting with the background seen through T_final
  float S0 = T * ds.bg[0], S1 = T * ds.bg[1], S2 = T * ds.bg[2];
  if (threadIdx.x == 0) s_maxlast = 0;
  __syncthreads();
  const uint32_t wlast = wave_max(last);
  if ((threadIdx.x & 63) == 0) atomicMax(&s_maxlast, wlast);
  __syncthreads();
  const uint2 rg = ranges[tile];
  const uint32_t end = rg.x + s_maxlast;
  const float kq = -0.5f * kLog2e;

  for (uint32_t bend = end; bend > rg.x;) {
    const uint32_t bstart = (bend - rg.x > (uint32_t)batch) ? bend - batch : rg.x;
    const uint32_t nb = bend - bstart;
    if (threadIdx.x < nb) {
      const uint32_t e = pval[bstart + threadIdx.x];
      s_rec[threadIdx.x] = stage(rec[e], e);
    }
    __syncthreads();
    for (int j = (int)nb - 1; j >= 0; j--) {
      const uint32_t pos = bstart - rg.x + j;  // position in the tile's list
      if (pos >= wlast) continue;               // no pixel of this wavefront reached it
      const float4 A = s_rec[j].a;
      const float4 B = s_rec[j].b;
      if (!box_hits(A, B, wx0, wy0)) continue;
      float g[kG2D];
#pragma unroll
      for (int k = 0; k < kG2D; k++) g[k] = 0.f;
      bool contrib = false;
      if (pos < last) {
        const float dx = fx - A.x, dy = fy - A.y;
        const float G = exp2_fast(power2(A, B.x, dx, dy));
        const float araw = B.y * G;
        const float a = fminf(kAlphaMax, araw);
        if (a >= kAlphaMin) {
          contrib = true;
          const float4 Cc = s_rec[j].c;
          const float om = 1.0f - a;
          const float Tb = T / om;  // transmittance in front of this Gaussian
          const float wgt = a * Tb;
          g[6] = dC0 * wgt;
          g[7] = dC1 * wgt;
          g[8] = dC2 * wgt;
          const float dl_da = dC0 * (Cc.x * Tb - S0 / om) + dC1 * (Cc.y * Tb - S1 / om) + dC2 * (Cc.z * Tb - S2 / om);
          S0 += Cc.x * wgt;
          S1 += Cc.y * wgt;
          S2 += Cc.z * wgt;
          T = Tb;
          if (araw <= kAlphaMax) {
            g[5] = dl_da * G;
            const float dl_dp2 = dl_da * araw * kLn2;
            g[0] = -dl_dp2 * (2.f * A.z * dx + A.w * dy);
            g[1] = -dl_dp2 * (A.w * dx + 2.f * B.x * dy);
            g[2] = dl_dp2 * dx * dx;
            g[3] = dl_dp2 * dx * dy;
            g[4] = dl_dp2 * dy * dy;
          }
        }
      }
      if (__ballot(contrib) == 0) continue;
#pragma unroll
      for (int k = 0; k < kG2D; k++) g[k] = wave_sum(g[k]);
      if ((threadIdx.x & 63) == 0) {
        float* dst = g2d + (int64_t)__float_as_uint(s_rec[j].c.w) * kG2D;
        // dp2/d(cA, cB, cC) back to the conic's full-matrix gradient
        unsafeAtomicAdd(dst + 0, g[0]);
        unsafeAtomicAdd(dst + 1, g[1]);
        unsafeAtomicAdd(dst + 2, g[2] * kq);
        unsafeAtomicAdd(dst + 3, g[3] * kq);
        unsafeAtomicAdd(dst + 4, g[4] * kq);
        unsafeAtomicAdd(dst + 5, g[5]);
        unsafeAtomicAdd(dst + 6, g[6]);
        unsafeAtomicAdd(dst + 7, g[7]);
        unsafeAtomicAdd(dst + 8, g[8]);
      }
    }
    __syncthreads();
    bend = bstart;
  }
}

}  // namespace

void launch_blend_fwd(const ViewTable& vt, const DevSettings& s, const Rec* rec, const uint2* ranges,
                      const uint32_t* pval, BlendState bs, int batch, hipStream_t st) {
  if (vt.total_tiles <= 0) return;
  const dim3 grid(vt.total_tiles);
  switch (vt.tile_w) {
    case 8: hipLaunchKernelGGL(k_blend_fwd<8>, grid, dim3(kBlock), 0, st, vt, s, rec, ranges, pval, bs, batch); break;
    case 32: hipLaunchKernelGGL(k_blend_fwd<32>, grid, dim3(kBlock), 0, st, vt, s, rec, ranges, pval, bs, batch); break;
    default: hipLaunchKernelGGL(k_blend_fwd<16>, grid, dim3(kBlock), 0, st, vt, s, rec, ranges, pval, bs, batch); break;
  }
}

void launch_blend_bwd(const ViewTable& vt, const DevSettings& s, const Rec* rec, const uint2* ranges,
                      const uint32_t* pval, BlendState bs, float* g2d, int batch, hipStream_t st) {
  if (vt.total_tiles <= 0) return;
  const dim3 grid(vt.total_tiles);
  switch (vt.tile_w) {
    case 8: hipLaunchKernelGGL(k_blend_bwd<8>, grid, dim3(kBlock), 0, st, vt, s, rec, ranges, pval, bs, g2d, batch); break;
    case 32: hipLaunchKernelGGL(k_blend_bwd<32>, grid, dim3(kBlock), 0, st, vt, s, rec, ranges, pval, bs, g2d, batch); break;
    default: hipLaunchKernelGGL(k_blend_bwd<16>, grid, dim3(kBlock), 0, st, vt, s, rec, ranges, pval, bs, g2d, batch); break;
  }
}

}  // namespace sixdgs
