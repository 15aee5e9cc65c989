// Per-tile alpha compositing on gfx950 (the 3D Gaussian splatting rasteriser's
// blending, Sec. 4.4): forward front-to-back with the final transmittance and
// the last contributor saved per pixel, and the reverse walk that turns dL/dI
// into per-Gaussian screen-space gradients.
//
// One workgroup of 256 threads per screen tile, one pixel per thread; each
// 64-lane wavefront owns an 8x8 block of the tile.  The tile's depth-ordered
// list is staged through LDS in batches; while staging, each Gaussian's
// alpha >= 1/255 ellipse is tested exactly against the four blocks and every
// wavefront gets its own order-preserving list of the Gaussians that can reach
// its pixels, so the per-pixel loop -- the kernels' critical path, since a
// screen this size has fewer wavefronts than the chip can hold -- never
// visits a Gaussian its block cannot see.
#include "internal.h"

namespace sixdgs {
namespace {

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;
constexpr float kLog2AlphaMin = -7.994353436858858f;  // log2(1/255)
constexpr int kWaves = kBlock / 64;

// Staged record: the conic pre-scaled so that alpha exp(-q/2) = exp2(p2 + log2 alpha).
struct Staged {
  float4 a;  // u, v, cA = -log2e/2 Qxx, cB = -log2e Qxy
  float4 b;  // cC = -log2e/2 Qyy, log2(alpha_cond), 1/alpha_cond, entry id (bits)
  float4 c;  // r, g, b, -
};

__device__ __forceinline__ Staged stage(const Rec& r, uint32_t e) {
  Staged s;
  s.a = make_float4(r.a.x, r.a.y, -0.5f * kLog2e * r.a.z, -kLog2e * r.a.w);
  s.b = make_float4(-0.5f * kLog2e * r.b.x, __log2f(r.b.y), 1.0f / r.b.y, __uint_as_float(e));
  s.c = make_float4(r.c.x, r.c.y, r.c.z, 0.f);
  return s;
}

// log2 of the unclamped alpha of a Gaussian at a pixel: the one evaluation both
// directions use, written with explicit roundings so both compile to the same
// arithmetic.
__device__ __forceinline__ float log2_alpha(const float4& A, const float4& B, float dx, float dy) {
  const float t = __fmaf_rn(A.z, dx, __fmul_rn(A.w, dy));
  return __fadd_rn(__fmaf_rn(t, dx, __fmul_rn(__fmul_rn(B.x, dy), dy)), B.y);
}

__device__ __forceinline__ float exp2_fast(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }

// Does the extent box (with a one-pixel margin) reach the 8x8 block of pixel
// centres [x0, x0 + 7] x [y0, y0 + 7]?
__device__ __forceinline__ bool box_hits(const Rec& r, float x0, float y0) {
  return (r.a.x + r.b.z >= x0 - 1.0f) && (r.a.x - r.b.z <= x0 + 8.0f) && (r.a.y + r.b.w >= y0 - 1.0f) &&
         (r.a.y - r.b.w <= y0 + 8.0f);
}

// Can any pixel centre of the 8x8 block reach alpha >= 1/255, i.e. does the
// ellipse q(x) = (x - m)^T Q (x - m) <= q_max = 2 ln(255 alpha_cond) meet the
// block's rectangle of centres?  The minimum of the convex q over the
// rectangle is 0 when the centre m lies inside; otherwise it lies on an edge
// whose line separates m from the rectangle, and along an edge q is a 1D
// quadratic minimised by clamping.  A relative margin keeps the test
// conservative under float32 rounding, so it only skips Gaussians that no
// pixel of the block would take.
__device__ __forceinline__ bool ellipse_hits(const Rec& r, float x0, float y0) {
  if (!box_hits(r, x0, y0)) return false;
  const float qa = r.a.z, qb = r.a.w, qc = r.b.x;
  const float lim = 2.0f * logf(255.0f * r.b.y) * 1.001f + 1e-3f;
  const float xl = x0 - r.a.x, xh = xl + 7.0f;
  const float yl = y0 - r.a.y, yh = yl + 7.0f;
  const bool inx = xl <= 0.f && xh >= 0.f, iny = yl <= 0.f && yh >= 0.f;
  if (inx && iny) return true;
  float best = 3.0e38f;
  if (!inx) {
    const float dx = xl > 0.f ? xl : xh;
    const float dy = fminf(fmaxf(-qb * dx / qc, yl), yh);
    best = fminf(best, qa * dx * dx + 2.0f * qb * dx * dy + qc * dy * dy);
  }
  if (!iny) {
    const float dy = yl > 0.f ? yl : yh;
    const float dx = fminf(fmaxf(-qb * dy / qa, xl), xh);
    best = fminf(best, qa * dx * dx + 2.0f * qb * dx * dy + qc * dy * dy);
  }
  return best <= lim;
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
  __device__ static int bx(int w) { return (w % BX) * 8; }
  __device__ static int by(int w) { return (w / BX) * 8; }
};

// Shared staging state of one batch.
struct BatchLDS {
  Staged rec[kBlock];
  uint8_t list[kWaves][kBlock];  // per wavefront: staged slots in list order
  uint32_t wcnt[kWaves][kWaves];  // [block][staging wave] hits
};

// Stages pairs [b0, b0 + nb) of the tile list and builds the four per-block
// lists.  Returns (through cnt) the list length of this thread's wavefront.
template <int TW>
__device__ __forceinline__ uint32_t stage_batch(BatchLDS& L, const Rec* __restrict__ rec,
                                                const uint32_t* __restrict__ pval, uint32_t b0, uint32_t nb,
                                                float ox, float oy) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  uint32_t mask = 0;
  if ((uint32_t)t < nb) {
    const uint32_t e = pval[b0 + t];
    const Rec r = rec[e];
    L.rec[t] = stage(r, e);
#pragma unroll
    for (int w = 0; w < kWaves; w++)
      if (ellipse_hits(r, ox + TileMap<TW>::bx(w), oy + TileMap<TW>::by(w))) mask |= 1u << w;
  }
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t rank[kWaves];
#pragma unroll
  for (int w = 0; w < kWaves; w++) {
    const uint64_t bal = __ballot((mask >> w) & 1u);
    rank[w] = __popcll(bal & lt);
    if (lane == 0) L.wcnt[w][wv] = __popcll(bal);
  }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < kWaves; w++) {
    if ((mask >> w) & 1u) {
      uint32_t off = rank[w];
      for (int s = 0; s < wv; s++) off += L.wcnt[w][s];
      L.list[w][off] = (uint8_t)t;
    }
  }
  uint32_t cnt = 0;
#pragma unroll
  for (int s = 0; s < kWaves; s++) cnt += L.wcnt[wv][s];
  __syncthreads();
  return cnt;
}

template <int TW>
__global__ void __launch_bounds__(kBlock) k_blend_fwd(ViewTable vt, DevSettings ds, const Rec* __restrict__ rec,
                                                      const uint2* __restrict__ ranges,
                                                      const uint32_t* __restrict__ pval, BlendState bs, int batch) {
  __shared__ BatchLDS L;
  const int tile = blockIdx.x;
  const int vi = find_view(vt, tile);
  const ViewDesc& vd = vt.v[vi];
  const int local = tile - vd.tile_base;
  const int tx = local % vd.ntx, ty = local / vd.ntx;
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  const float ox = (float)(tx * TW) + 0.5f, oy = (float)(ty * TileMap<TW>::TH) + 0.5f;
  const int px = tx * TW + TileMap<TW>::bx(wv) + (l & 7);
  const int py = ty * TileMap<TW>::TH + TileMap<TW>::by(wv) + (l >> 3);
  const bool inside = px < vd.W && py < vd.H;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;

  const uint2 rg = ranges[tile];
  float T = 1.0f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  uint32_t last = 0, cnt = 0;
  bool done = !inside;
  for (uint32_t b0 = rg.x; b0 < rg.y; b0 += batch) {
    if (__syncthreads_count(!done) == 0) break;
    const uint32_t nb = min((uint32_t)batch, rg.y - b0);
    const uint32_t wn = stage_batch<TW>(L, rec, pval, b0, nb, ox, oy);
    const uint32_t pos0 = b0 - rg.x + 1;
    for (uint32_t k = 0; k < wn; k++) {
      if (__ballot(!done) == 0) break;
      const uint32_t j = L.list[wv][k];
      const float4 A = L.rec[j].a;
      const float4 B = L.rec[j].b;
      const float p = log2_alpha(A, B, fx - A.x, fy - A.y);
      if (done || p < kLog2AlphaMin) continue;
      const float a = fminf(kAlphaMax, exp2_fast(p));
      const float Tn = T * (1.0f - a);
      if (Tn < kTMin) {
        done = true;
        continue;
      }
      const float4 Cc = L.rec[j].c;
      const float wgt = a * T;
      C0 += Cc.x * wgt;
      C1 += Cc.y * wgt;
      C2 += Cc.z * wgt;
      T = Tn;
      last = pos0 + j;
      cnt++;
    }
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

// Sum over the 64 lanes of a wavefront, left in lane 63 (DPP row and
// row-broadcast steps, no LDS traffic).
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_move(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xF, false));
}

__device__ __forceinline__ float wave_sum_to_last(float v) {
  v += dpp_move<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x124, 0xF>(v);  // row_ror:4
  v += dpp_move<0x128, 0xF>(v);  // row_ror:8   -> every lane holds its row's sum
  v += dpp_move<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_move<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3 -> lane 63 holds the total
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
  __shared__ BatchLDS L;
  __shared__ float s_g[kG2D][kBlock];  // per staged Gaussian, summed over the four wavefronts
  __shared__ uint32_t s_maxlast;
  const int tile = blockIdx.x;
  const int vi = find_view(vt, tile);
  const ViewDesc& vd = vt.v[vi];
  const int local = tile - vd.tile_base;
  const int tx = local % vd.ntx, ty = local / vd.ntx;
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  const float ox = (float)(tx * TW) + 0.5f, oy = (float)(ty * TileMap<TW>::TH) + 0.5f;
  const int px = tx * TW + TileMap<TW>::bx(wv) + (l & 7);
  const int py = ty * TileMap<TW>::TH + TileMap<TW>::by(wv) + (l >> 3);
  const bool inside = px < vd.W && py < vd.H;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;

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
#pragma unroll
  for (int k = 0; k < kG2D; k++) s_g[k][threadIdx.x] = 0.f;
  __syncthreads();
  const uint32_t wlast = wave_max(last);
  if (l == 0) atomicMax(&s_maxlast, wlast);
  __syncthreads();
  const uint2 rg = ranges[tile];
  const uint32_t end = rg.x + s_maxlast;
  const float kq = -0.5f * kLog2e;

  for (uint32_t bend = end; bend > rg.x;) {
    const uint32_t b0 = (bend - rg.x > (uint32_t)batch) ? bend - batch : rg.x;
    const uint32_t nb = bend - b0;
    const uint32_t wn = stage_batch<TW>(L, rec, pval, b0, nb, ox, oy);
    const uint32_t pos0 = b0 - rg.x;
    for (int k = (int)wn - 1; k >= 0; k--) {
      const uint32_t j = L.list[wv][k];
      if (pos0 + j >= wlast) continue;  // no pixel of this wavefront reached it
      const float4 A = L.rec[j].a;
      const float4 B = L.rec[j].b;
      float g0 = 0.f, g1 = 0.f, g2 = 0.f, g3 = 0.f, g4 = 0.f, g5 = 0.f, g6 = 0.f, g7 = 0.f, g8 = 0.f;
      bool contrib = false;
      if (pos0 + j < last) {
        const float dx = fx - A.x, dy = fy - A.y;
        const float p = log2_alpha(A, B, dx, dy);
        if (p >= kLog2AlphaMin) {
          contrib = true;
          const float araw = exp2_fast(p);
          const float a = fminf(kAlphaMax, araw);
          const float4 Cc = L.rec[j].c;
          const float ro = rcp_fast(1.0f - a);
          const float Tb = T * ro;  // transmittance in front of this Gaussian
          const float wgt = a * Tb;
          g6 = dC0 * wgt;
          g7 = dC1 * wgt;
          g8 = dC2 * wgt;
          const float dl_da = dC0 * (Cc.x * Tb - S0 * ro) + dC1 * (Cc.y * Tb - S1 * ro) + dC2 * (Cc.z * Tb - S2 * ro);
          S0 += Cc.x * wgt;
          S1 += Cc.y * wgt;
          S2 += Cc.z * wgt;
          T = Tb;
          if (araw <= kAlphaMax) {
            const float dl_dp = dl_da * araw;
            g5 = dl_dp * B.z;  // d alpha / d alpha_cond = exp(-q/2) = araw / alpha_cond
            const float dl_dp2 = dl_dp * kLn2;
            g0 = -dl_dp2 * (2.f * A.z * dx + A.w * dy);
            g1 = -dl_dp2 * (A.w * dx + 2.f * B.x * dy);
            g2 = dl_dp2 * dx * dx;
            g3 = dl_dp2 * dx * dy;
            g4 = dl_dp2 * dy * dy;
          }
        }
      }
      if (__ballot(contrib) == 0) continue;
      g0 = wave_sum_to_last(g0);
      g1 = wave_sum_to_last(g1);
      g2 = wave_sum_to_last(g2);
      g3 = wave_sum_to_last(g3);
      g4 = wave_sum_to_last(g4);
      g5 = wave_sum_to_last(g5);
      g6 = wave_sum_to_last(g6);
      g7 = wave_sum_to_last(g7);
      g8 = wave_sum_to_last(g8);
      if (l == 63) {
        atomicAdd(&s_g[0][j], g0);
        atomicAdd(&s_g[1][j], g1);
        atomicAdd(&s_g[2][j], g2);
        atomicAdd(&s_g[3][j], g3);
        atomicAdd(&s_g[4][j], g4);
        atomicAdd(&s_g[5][j], g5);
        atomicAdd(&s_g[6][j], g6);
        atomicAdd(&s_g[7][j], g7);
        atomicAdd(&s_g[8][j], g8);
      }
    }
    __syncthreads();
    // one set of global atomics per (tile, Gaussian), conic gradient converted
    // from the pre-scaled coefficients back to the conic's full-matrix gradient
    if ((uint32_t)threadIdx.x < nb) {
      const int t = threadIdx.x;
      float v[kG2D];
      bool any = false;
#pragma unroll
      for (int k = 0; k < kG2D; k++) {
        v[k] = s_g[k][t];
        s_g[k][t] = 0.f;
        any |= v[k] != 0.f;
      }
      if (any) {
        float* dst = g2d + (int64_t)__float_as_uint(L.rec[t].b.w) * kG2D;
        unsafeAtomicAdd(dst + 0, v[0]);
        unsafeAtomicAdd(dst + 1, v[1]);
        unsafeAtomicAdd(dst + 2, v[2] * kq);
        unsafeAtomicAdd(dst + 3, v[3] * kq);
        unsafeAtomicAdd(dst + 4, v[4] * kq);
        unsafeAtomicAdd(dst + 5, v[5]);
        unsafeAtomicAdd(dst + 6, v[6]);
        unsafeAtomicAdd(dst + 7, v[7]);
        unsafeAtomicAdd(dst + 8, v[8]);
      }
    }
    __syncthreads();
    bend = b0;
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
