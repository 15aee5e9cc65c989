// Per-tile alpha compositing on gfx950 (the 3D Gaussian splatting rasteriser's
// blending, Sec. 4.4): forward front-to-back with the final transmittance and
// the last contributor saved per pixel, and the reverse walk that turns dL/dI
// into per-Gaussian screen-space gradients.
//
// One workgroup of 256 threads per screen tile (forward) or per chunk of a
// tile's list (backward), one pixel per thread; each 64-lane wavefront owns an
// 8x8 block of the tile.  Each Gaussian's alpha >= 1/255 ellipse is tested
// exactly against a block before that block's pixels see it, so the
// per-pixel loop -- the kernels' critical path -- never visits a Gaussian its
// block cannot reach.  The forward's wavefronts walk the list independently
// (a tile's blocks differ in depth complexity, and a shared batch would hold
// every wavefront to the slowest); the backward stages one LDS batch for the
// workgroup and builds the four per-block lists from it.
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
  s.b = make_float4(-0.5f * kLog2e * r.b.x, __log2f(r.b.y), __builtin_amdgcn_rcpf(r.b.y), __uint_as_float(e));
  s.c = make_float4(r.c.x, r.c.y, r.c.z, 0.f);
  return s;
}

// log2 of the unclamped alpha of a Gaussian at a pixel: the one evaluation both
// directions use, written with explicit roundings so both compile to the same
// arithmetic.
__device__ __forceinline__ float log2_alpha(const float4& A, const float4& B, float dx, float dy) {
  const float t = __fmaf_rn(A.z, dx, __fmul_rn(A.w, dy));
  return __fmaf_rn(t, dx, __fmaf_rn(__fmul_rn(B.x, dy), dy, B.y));
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
// pixel of the block would take.  The margins (0.1% and 1e-3) are far wider
// than the errors of the hardware log and reciprocal used here: q_max is off
// by about 1e-7, and an edge minimiser off by a relative 1e-7 moves q by its
// square (q is flat there).
__device__ __forceinline__ bool ellipse_hits(const Rec& r, float x0, float y0) {
  if (!box_hits(r, x0, y0)) return false;
  const float qa = r.a.z, qb = r.a.w, qc = r.b.x;
  const float lim = (2.0f * kLn2) * __builtin_amdgcn_logf(255.0f * r.b.y) * 1.001f + 1e-3f;
  const float xl = x0 - r.a.x, xh = xl + 7.0f;
  const float yl = y0 - r.a.y, yh = yl + 7.0f;
  const bool inx = xl <= 0.f && xh >= 0.f, iny = yl <= 0.f && yh >= 0.f;
  if (inx && iny) return true;
  float best = 3.0e38f;
  if (!inx) {
    const float dx = xl > 0.f ? xl : xh;
    const float dy = fminf(fmaxf(-qb * dx * __builtin_amdgcn_rcpf(qc), yl), yh);
    best = fminf(best, qa * dx * dx + 2.0f * qb * dx * dy + qc * dy * dy);
  }
  if (!iny) {
    const float dy = yl > 0.f ? yl : yh;
    const float dx = fminf(fmaxf(-qb * dy * __builtin_amdgcn_rcpf(qa), xl), xh);
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

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, o, 64));
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
  return __builtin_amdgcn_readfirstlane(cnt);  // uniform over the wavefront
}

// The staged records of four consecutive list slots of a wavefront, as the
// per-pixel loops read them.  The wavefront's list (at most 256 one-byte
// slots) is held one 32-bit word per lane, so a group's slots come from a
// readlane instead of an LDS round trip.
struct Group4 {
  uint32_t j[4];  // staged slots
  float4 a[4];    // u, v, cA, cB
  float2 b[4];    // cC, log2(alpha_cond)
  float3 c[4];    // r, g, b
};

// Slots past the list's length wn take the group's first slot instead: the
// bytes there are left over from earlier use of the LDS, and a record never
// staged may hold infinities or NaNs, which a zero weight does not cancel.
__device__ __forceinline__ void fetch_group(const BatchLDS& L, uint32_t lw, uint32_t g, uint32_t wn, Group4& G) {
  const uint32_t w = (uint32_t)__builtin_amdgcn_readlane((int)lw, (int)g);
#pragma unroll
  for (int u = 0; u < 4; u++) {
    const uint32_t j = (4 * g + u < wn ? w >> (8 * u) : w) & 255u;
    G.j[u] = j;
    G.a[u] = L.rec[j].a;
    G.b[u] = make_float2(L.rec[j].b.x, L.rec[j].b.y);
    G.c[u] = make_float3(L.rec[j].c.x, L.rec[j].c.y, L.rec[j].c.z);
  }
}

// Forward staging: every wavefront walks the tile's list on its own, 64 list
// entries per step, keeps the Gaussians whose alpha >= 1/255 ellipse meets
// its 8x8 block, compacted in its own LDS buffer, and composites them once 64
// have gathered (or at a chunk boundary, or at the list's end).  No wavefront
// waits for another, and the loads of the next step are in flight while the
// current one is tested and blended.
constexpr int kFwdStep = 64;
constexpr int kFwdBuf = 128;  // pending hits stay below 64 before a step adds at most 64
struct FwdWaveLDS {
  float4 a[kFwdBuf];  // u, v, cA, cB
  float2 b[kFwdBuf];  // cC, log2(alpha_cond)
  float4 c[kFwdBuf];  // r, g, b, 1-based list position (bits)
};

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// SAVE = false renders the image only (inference): no chunk boundaries, no
// final transmittance, last contributor or chunk counts for a backward.
// Five wavefronts per SIMD (96 registers, no spills): with tens of thousands
// of tiles the walks' load latency is hidden by the extra wave (eight 1080p
// views of 1M Gaussians: 1.87 -> 1.72 ms).
// COUNTS additionally counts each pixel's contributors (a debug export).
template <int TW, bool SAVE, bool COUNTS>
__global__ void __launch_bounds__(kBlock, 5) k_blend_fwd(ViewTable vt, DevSettings ds, const Rec* __restrict__ rec,
                                                      const uint2* __restrict__ ranges,
                                                      const uint32_t* __restrict__ pval, BlendState bs) {
  __shared__ FwdWaveLDS W[kWaves];
  __shared__ uint32_t s_maxlast, s_ibase;
  __shared__ float s_l1[kWaves];
  const int tile = (int)bs.order[blockIdx.x];
  const int vi = find_view(vt, tile);
  const ViewDesc& vd = vt.v[vi];
  const int local = tile - vd.tile_base;
  const int tx = local % vd.ntx, ty = local / vd.ntx;
  const int wv = threadIdx.x >> 6, l = threadIdx.x & 63;
  const float bx0 = (float)(tx * TW + TileMap<TW>::bx(wv)) + 0.5f;
  const float by0 = (float)(ty * TileMap<TW>::TH + TileMap<TW>::by(wv)) + 0.5f;
  const int px = tx * TW + TileMap<TW>::bx(wv) + (l & 7);
  const int py = ty * TileMap<TW>::TH + TileMap<TW>::by(wv) + (l >> 3);
  const bool inside = px < vd.W && py < vd.H;
  const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
  FwdWaveLDS& B = W[wv];
  const uint64_t lt = (l == 0) ? 0ull : (~0ull >> (64 - l));

  if constexpr (SAVE) {
    if (threadIdx.x == 0) s_maxlast = 0;
    __syncthreads();
  }
  const uint2 rg = ranges[tile];
  const uint32_t n = rg.y - rg.x;
  const uint32_t* pv = pval + rg.x;
  const uint32_t chunk = bs.chunk;
  float T = 1.0f, C0 = 0.f, C1 = 0.f, C2 = 0.f;
  float K0 = 0.f, K1 = 0.f, K2 = 0.f;  // colour of the current chunk alone
  uint32_t last = 0, cnt = 0, nbd = 0;
  bool done = !inside;

  auto composite = [&](uint32_t nh) {
    // the group that ends past nh would read stale slots: fill them with a
    // Gaussian no pixel takes (exponent -1e30) and a zero colour, so that
    // every slot of a group is evaluated alike
    if ((uint32_t)l < ((4u - (nh & 3u)) & 3u)) {
      B.a[nh + l] = make_float4(0.f, 0.f, 0.f, 0.f);
      B.b[nh + l] = make_float2(0.f, -1e30f);
      B.c[nh + l] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    wave_lds_sync();
    for (uint32_t g = 0; 4 * g < nh; g++) {
      if (__ballot(!done) == 0) break;
      float4 A[4], Cc[4];
      float2 Bq[4];
#pragma unroll
      for (int u = 0; u < 4; u++) {
        A[u] = B.a[4 * g + u];
        Bq[u] = B.b[4 * g + u];
        Cc[u] = B.c[4 * g + u];
      }
      // predicated rather than branched, also past the last slot, so the four
      // records are read at once: the lanes of a wavefront rarely agree.  A
      // Gaussian the pixel does not take gets alpha 0, which leaves T exactly
      // as it is; T never falls below 1e-4 (it is only updated when the step
      // does not stop), so such a step never stops either.
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const float p = log2_alpha(A[u], make_float4(Bq[u].x, Bq[u].y, 0.f, 0.f), fx - A[u].x, fy - A[u].y);
        const bool take = !done && p >= kLog2AlphaMin;
        // the clamp doubles as the mask: min(0, .) is 0 whatever the exponent gives
        const float a = fminf(take ? kAlphaMax : 0.f, exp2_fast(p));
        const float Tn = __fmaf_rn(-T, a, T);  // T (1 - a)
        const bool stop = Tn < kTMin;
        done = done || stop;
        const bool took = take && !stop;  // the same as wgt != 0: a >= 1/255 and T >= 1e-4 when taken
        const float wgt = took ? a * T : 0.f;
        C0 += Cc[u].x * wgt;
        C1 += Cc[u].y * wgt;
        C2 += Cc[u].z * wgt;
        T = stop ? T : Tn;
        if constexpr (SAVE) {
          K0 += Cc[u].x * wgt;
          K1 += Cc[u].y * wgt;
          K2 += Cc[u].z * wgt;
          last = took ? __float_as_uint(Cc[u].w) : last;
        }
        if constexpr (COUNTS) cnt += took ? 1u : 0u;
      }
    }
  };

  // software pipeline: entry ids two steps ahead, records one step ahead
  // (past the list the ids stay 0, an entry that exists whenever the list is
  // not empty: every lane loads a record and the ones past the list go
  // unused, which spares zeroing the twelve registers every step)
  uint32_t e_cur = 0, e_nxt = 0;
  if ((uint32_t)l < n) e_cur = pv[l];
  if ((uint32_t)(kFwdStep + l) < n) e_nxt = pv[kFwdStep + l];
  Rec r_cur;
  if (n > 0) r_cur = rec[e_cur];
  uint32_t nh = 0;  // pending hits in B (uniform)
  for (uint32_t s0 = 0; s0 < n; s0 += kFwdStep) {
    if (__ballot(!done) == 0) break;
    const Rec r_nxt = rec[e_nxt];
    uint32_t e_nn = 0;
    if (s0 + 2 * kFwdStep + l < n) e_nn = pv[s0 + 2 * kFwdStep + l];
    if (SAVE && s0 != 0 && (s0 & (chunk - 1)) == 0) {
      // a backward work item starts here: finish the chunk, then keep this
      // pixel's transmittance and the colour of the chunk that ends here
      composite(nh);
      nh = 0;
      const int64_t slot = ((int64_t)rg.x + s0) >> bs.chunk_shift;
      if (slot < bs.nbound) bs.bound[slot * kBlock + threadIdx.x] = make_float4(T, K0, K1, K2);
      K0 = K1 = K2 = 0.f;
      nbd++;
    }
    const bool hit = (s0 + l < n) && ellipse_hits(r_cur, bx0, by0);
    const uint64_t bal = __ballot(hit);
    if (hit) {
      const uint32_t k = nh + (uint32_t)__popcll(bal & lt);
      B.a[k] = make_float4(r_cur.a.x, r_cur.a.y, -0.5f * kLog2e * r_cur.a.z, -kLog2e * r_cur.a.w);
      B.b[k] = make_float2(-0.5f * kLog2e * r_cur.b.x, __log2f(r_cur.b.y));
      B.c[k] = make_float4(r_cur.c.x, r_cur.c.y, r_cur.c.z, __uint_as_float(s0 + l + 1));
    }
    nh += (uint32_t)__popcll(bal);
    wave_lds_sync();
    if (nh >= kFwdStep) {
      composite(nh);
      nh = 0;
      wave_lds_sync();
    }
    r_cur = r_nxt;
    e_nxt = e_nn;
  }
  composite(nh);
  if constexpr (!SAVE) {
    if (inside) {
      const int64_t HW = (int64_t)vd.W * vd.H;
      const int64_t pix = (int64_t)py * vd.W + px;
      vd.img[pix] = C0 + T * ds.bg[0];
      vd.img[HW + pix] = C1 + T * ds.bg[1];
      vd.img[2 * HW + pix] = C2 + T * ds.bg[2];
    }
    return;
  }

  // turn the per-chunk colours into the colour behind each boundary: sums of
  // positive terms from the back, so no cancellation against the total
  float S0 = K0, S1 = K1, S2 = K2;
  for (uint32_t m = nbd; m >= 1; m--) {
    const int64_t slot = ((int64_t)rg.x + (int64_t)m * chunk) >> bs.chunk_shift;
    if (slot >= bs.nbound) continue;
    float4* q = bs.bound + slot * kBlock + threadIdx.x;
    const float4 v = *q;
    *q = make_float4(v.x, S0, S1, S2);
    S0 += v.y;
    S1 += v.z;
    S2 += v.w;
  }
  float l1 = 0.f;  // this pixel's |I - I*| summed over the channels
  if (inside) {
    const int64_t HW = (int64_t)vd.W * vd.H;
    const int64_t pix = (int64_t)py * vd.W + px;
    // the running sum, whose rounding does not depend on where chunks begin
    const float o[3] = {C0 + T * ds.bg[0], C1 + T * ds.bg[1], C2 + T * ds.bg[2]};
#pragma unroll
    for (int c = 0; c < 3; c++) vd.img[c * HW + pix] = o[c];
    bs.T_final[vd.pix_base + pix] = T;
    bs.last[vd.pix_base + pix] = last;
    if constexpr (COUNTS) bs.counts[vd.pix_base + pix] = cnt;
    if (bs.l1_partial) {
      // the L1 loss of the step (Sec. 4.4, Sec. 5.1): dL/dI = sign(I - I*) / count
#pragma unroll
      for (int c = 0; c < 3; c++) {
        const float d = o[c] - vd.tgt[c * HW + pix];
        l1 += fabsf(d);
        vd.dl[c * HW + pix] = (d > 0.f) ? bs.l1_inv : ((d < 0.f) ? -bs.l1_inv : 0.f);
      }
    }
  }
  if (bs.l1_partial) {
    // the tile's sum in a fixed order: lanes, then wavefronts
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) l1 += __shfl_xor(l1, off);
    if (l == 0) s_l1[wv] = l1;
  }
  const uint32_t wlast = wave_max(last);
  if (l == 0) atomicMax(&s_maxlast, wlast);
  __syncthreads();
  // the tile's backward work items (tile, 0 .. nch - 1), appended to the list
  // where the tiles finished so far end (*n_items is zero before the launch)
  const uint32_t nch = (s_maxlast + chunk - 1) >> bs.chunk_shift;
  if (threadIdx.x == 0) {
    bs.tile_nch[tile] = nch;
    s_ibase = nch ? atomicAdd(bs.n_items, nch) : 0u;
    if (bs.l1_partial) {
      float sum = 0.f;
      for (int w = 0; w < kWaves; w++) sum += s_l1[w];
      bs.l1_partial[tile] = sum;
    }
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < nch; k += kBlock) {
    const int64_t slot = (int64_t)s_ibase + k;
    if (slot < bs.items_cap) bs.items[slot] = make_uint2((uint32_t)tile, k);
  }
}

// ------------------------------------------------------------- reductions
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_move(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xF, false));
}

// Sum over the 16 lanes of each row; every lane of the row gets the row total.
__device__ __forceinline__ float row_sum(float v) {
  v += dpp_move<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v += dpp_move<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v += dpp_move<0x124, 0xF>(v);  // row_ror:4
  v += dpp_move<0x128, 0xF>(v);  // row_ror:8
  return v;
}

// a + b after swapping the upper half of a with the lower half of b: lanes
// 0-31 get a[i] + a[i+32], lanes 32-63 get b[i-32] + b[i].
__device__ __forceinline__ float swap32_add(float a, float b) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_int(a), __float_as_int(b), false, false);
  return __int_as_float(r[0]) + __int_as_float(r[1]);
}

// a + b after swapping the odd rows of a with the even rows of b: rows 0, 1,
// 2, 3 get a0 + a1, b0 + b1, a2 + a3, b2 + b3 (rows of 16 lanes).
__device__ __forceinline__ float swap16_add(float a, float b) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_int(a), __float_as_int(b), false, false);
  return __int_as_float(r[0]) + __int_as_float(r[1]);
}

// Sums the nine per-lane values of two Gaussians (slots ja and jb) over the
// wavefront by halving exchanges -- each exchange step halves two values at
// once -- then adds the totals into LDS columns ja and jb of s_g ([9][kBlock]).
// After the two swap stages and the row sums, the rows of k0..k4 hold
// (a0 a2 a1 a3), (a4 a6 a5 a7), (a8 b0 b8 b1), (b2 b4 b3 b5) and (b6 b6 b7 b7).
__device__ __forceinline__ void wave_sum18_to_lds(const float (&a)[kG2D], const float (&b)[kG2D],
                                                  float (*s_g)[kBlock], int ja, int jb, int lane) {
  const float h0 = swap32_add(a[0], a[1]);
  const float h1 = swap32_add(a[2], a[3]);
  const float h2 = swap32_add(a[4], a[5]);
  const float h3 = swap32_add(a[6], a[7]);
  const float h4 = swap32_add(a[8], b[8]);
  const float h5 = swap32_add(b[0], b[1]);
  const float h6 = swap32_add(b[2], b[3]);
  const float h7 = swap32_add(b[4], b[5]);
  const float h8 = swap32_add(b[6], b[7]);
  float k0 = row_sum(swap16_add(h0, h1));
  float k1 = row_sum(swap16_add(h2, h3));
  float k2 = row_sum(swap16_add(h4, h5));
  float k3 = row_sum(swap16_add(h6, h7));
  float k4 = row_sum(swap16_add(h8, h8));
  // the row sums complete on every lane here: left to itself the compiler
  // moves each last add into the branch below, which then needs the rotated
  // value copied out first (three instructions per sum instead of one)
  asm volatile("" : "+v"(k0), "+v"(k1), "+v"(k2), "+v"(k3), "+v"(k4));
  if ((lane & 15) == 0) {
    const int row = lane >> 4;
    const int f0 = (row == 0) ? 0 : (row == 1) ? 2 : (row == 2) ? 1 : 3;
    atomicAdd(&s_g[f0][ja], k0);
    atomicAdd(&s_g[f0 + 4][ja], k1);
    const int f2 = (row == 1) ? 0 : (row == 3) ? 1 : 8;
    atomicAdd(&s_g[f2][row == 0 ? ja : jb], k2);
    atomicAdd(&s_g[f0 + 2][jb], k3);
    if ((row & 1) == 0) atomicAdd(&s_g[6 + (row >> 1)][jb], k4);
  }
}

// One work item = one chunk of `chunk` list positions of one tile, walked
// back to front from the state the forward saved where the next chunk begins
// (or from the pixel's final state for the tile's last chunk).
// Seven wavefronts per SIMD (72 registers, no spills; one 800x800 view of
// 300k Gaussians: 192 -> 190 us).
template <int TW>
__global__ void __launch_bounds__(kBlock, 7) k_blend_bwd(ViewTable vt, DevSettings ds, const Rec* __restrict__ rec,
                                                      const uint2* __restrict__ ranges,
                                                      const uint32_t* __restrict__ pval, BlendState bs,
                                                      float* __restrict__ g2d, int batch) {
  __shared__ BatchLDS L;
  __shared__ float s_g[kG2D][kBlock];  // per staged Gaussian, summed over the four wavefronts
  __shared__ uint32_t s_maxlast;
  // the list holds the items in the order the forward's tiles finished
  // (measured: 5 us faster on c2 than taking it from the back, the long
  // tiles' chunks first)
  const uint32_t ni = (uint32_t)min<int64_t>(*bs.n_items, bs.items_cap);
  if (blockIdx.x >= ni) return;  // uniform
  const uint2 item = bs.items[blockIdx.x];
  const int tile = (int)item.x;
  const uint32_t chunk = bs.chunk;
  const uint32_t cstart = item.y * chunk;  // list positions [cstart, cstart + chunk) of the tile
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
  const uint32_t* list4 = reinterpret_cast<const uint32_t*>(L.list[wv]);

  float Tf = 1.f, dC0 = 0.f, dC1 = 0.f, dC2 = 0.f;
  uint32_t last = 0;
  if (inside) {
    const int64_t HW = (int64_t)vd.W * vd.H;
    const int64_t pix = (int64_t)py * vd.W + px;
    Tf = bs.T_final[vd.pix_base + pix];
    last = bs.last[vd.pix_base + pix];
    dC0 = vd.dimg[pix];
    dC1 = vd.dimg[HW + pix];
    dC2 = vd.dimg[2 * HW + pix];
  }
  if (threadIdx.x == 0) s_maxlast = 0;
#pragma unroll
  for (int k = 0; k < kG2D; k++) s_g[k][threadIdx.x] = 0.f;
  __syncthreads();
  const uint32_t wlast = __builtin_amdgcn_readfirstlane(wave_max(last));
  if (l == 0) atomicMax(&s_maxlast, wlast);
  __syncthreads();
  const uint2 rg = ranges[tile];
  const uint32_t maxlast = s_maxlast;
  // state behind the chunk: transmittance T in front of it and the colour S
  // behind it (background included), carried as D = dL/dC . S
  float T = Tf;
  float S0 = Tf * ds.bg[0], S1 = Tf * ds.bg[1], S2 = Tf * ds.bg[2];
  if (cstart + chunk < last) {
    // the pixel takes Gaussians past this chunk: resume from the state saved
    // where the next chunk begins (otherwise its final state is that state)
    const int64_t slot = ((int64_t)rg.x + cstart + chunk) >> bs.chunk_shift;
    const float4 st = slot < bs.nbound ? bs.bound[slot * kBlock + threadIdx.x] : make_float4(1.f, 0.f, 0.f, 0.f);
    T = st.x;
    S0 += st.y;
    S1 += st.z;
    S2 += st.w;
  }
  float D = dC0 * S0 + dC1 * S1 + dC2 * S2;
  const uint32_t cend = min(cstart + chunk, maxlast);
  const float kq = -0.5f * kLog2e;

  for (uint32_t bend = rg.x + cend; bend > rg.x + cstart;) {
    const uint32_t b0 = (bend - (rg.x + cstart) > (uint32_t)batch) ? bend - batch : rg.x + cstart;
    const uint32_t nb = bend - b0;
    const uint32_t wn = stage_batch<TW>(L, rec, pval, b0, nb, ox, oy);
    const uint32_t pos0 = b0 - rg.x;
    // groups of four list slots, from the back
    const uint32_t lw = list4[l];
    const int ng = (int)((wn + 3) >> 2);
    // A group of four list slots, back to front.  What does not depend on the
    // walk's state -- offsets, exponent, take flag -- is formed for all four
    // first, branch-free; alpha and 1 / (1 - alpha) only for a pair some lane
    // takes (c2 backward 209 -> 206 us); then the reverse steps run in pairs, each pair's
    // 18 per-lane values summed in one straight-line reduction (a Gaussian no
    // lane took adds zeros; a pair no lane took is skipped).  The one
    // reduction for both needs no register copies for the in-place lane
    // swaps, which a choice between a joint and two single reductions did.
    auto grad = [&](const Group4& G, int g) {
      float dxs[4], dys[4], ars[4], as[4], ros[4];  // ars: the exponent until the pair is taken
      bool cs[4];
#pragma unroll
      for (int u = 0; u < 4; u++) {
        const uint32_t pos = pos0 + G.j[u];
        // slots past the list and Gaussians no pixel of this wavefront reached are out
        const bool in = (uint32_t)(4 * g + u) < wn && pos < wlast;
        dxs[u] = fx - G.a[u].x;
        dys[u] = fy - G.a[u].y;
        const float p = log2_alpha(G.a[u], make_float4(G.b[u].x, G.b[u].y, 0.f, 0.f), dxs[u], dys[u]);
        cs[u] = in && pos < last && p >= kLog2AlphaMin;
        ars[u] = p;
      }
      // one reverse step: updates T and D and fills the per-lane values to sum
      auto step = [&](int u, float (&gv)[kG2D]) {
        const bool contrib = cs[u];
        const float a = as[u], ro = ros[u], dx = dxs[u], dy = dys[u];
        const float Tb = T * ro;  // transmittance in front of this Gaussian (T where not taken)
        const float wgt = a * Tb;
        const float dc = dC0 * G.c[u].x + dC1 * G.c[u].y + dC2 * G.c[u].z;
        const float dl_da = Tb * dc - ro * D;  // dL/dC . (c T_front - S_behind / (1 - alpha))
        D += dc * wgt;
        T = Tb;
        // d alpha / d(exponent) = alpha while alpha is below its clamp, zero above
        const float dl_dp = (contrib && ars[u] <= kAlphaMax) ? dl_da * ars[u] : 0.f;
        const float e0 = dl_dp * dx, e1 = dl_dp * dy;
        // moments of dL/d(exponent) over the lanes; the mean and opacity gradients
        // are formed from them once per Gaussian after the reduction
        gv[0] = e0;
        gv[1] = e1;
        gv[2] = e0 * dx;
        gv[3] = e0 * dy;
        gv[4] = e1 * dy;
        gv[5] = dl_dp;
        gv[6] = dC0 * wgt;
        gv[7] = dC1 * wgt;
        gv[8] = dC2 * wgt;
      };
#pragma unroll
      for (int h = 1; h >= 0; h--) {
        if (__ballot(cs[2 * h + 1] || cs[2 * h]) == 0) continue;
#pragma unroll
        for (int u = 2 * h; u < 2 * h + 2; u++) {
          ars[u] = exp2_fast(ars[u]);
          // a lane that does not take the Gaussian gets alpha 0: 1 / (1 - 0) is
          // exactly 1, so its step leaves T and D exactly as they are
          as[u] = fminf(cs[u] ? kAlphaMax : 0.f, ars[u]);
          ros[u] = rcp_fast(1.0f - as[u]);
        }
        float ga[kG2D], gb[kG2D];
        step(2 * h + 1, ga);
        step(2 * h, gb);
        wave_sum18_to_lds(ga, gb, s_g, (int)G.j[2 * h + 1], (int)G.j[2 * h], l);
      }
    };
    for (int g = ng - 1; g >= 0; g--) {
      Group4 X;
      fetch_group(L, lw, (uint32_t)g, wn, X);
      grad(X, g);
    }
    __syncthreads();
    // one set of global atomics per (chunk, Gaussian).  Each staged
    // Gaussian's thread turns its column of sums into the nine components in
    // place (the conic gradient goes from the pre-scaled coefficients back to
    // the conic's full-matrix gradient); the adds then go Gaussian-major, so
    // that consecutive lanes add to consecutive words of one Gaussian's row (a
    // memory request per row instead of one per component), zero components
    // skipped.
    const int t = threadIdx.x;
    static_assert(sizeof(L.list) >= sizeof(uint32_t) * kBlock, "entry ids fit the slot lists");
    uint32_t* s_ent = reinterpret_cast<uint32_t*>(L.list);  // the slot lists are no longer read
    if ((uint32_t)t < nb) {
      float v[kG2D];
#pragma unroll
      for (int k = 0; k < kG2D; k++) v[k] = s_g[k][t];
      // exponent p2 = log2(alpha) = cA dx^2 + cB dx dy + cC dy^2 + log2(alpha_cond), with
      // dx = x - u: dp2/du = -(2 cA dx + cB dy), dp2/dv = -(cB dx + 2 cC dy); and
      // dp2/dcA = dx^2 etc., cA = kq Qxx, cB = 2 kq Qxy, cC = kq Qyy
      const Staged& sr = L.rec[t];
      const float m0 = v[0] * kLn2, m1 = v[1] * kLn2;  // moments of dL/dp2 = dL/dp ln 2
      s_g[0][t] = -(2.f * sr.a.z * m0 + sr.a.w * m1);
      s_g[1][t] = -(sr.a.w * m0 + 2.f * sr.b.x * m1);
      s_g[2][t] = v[2] * (kLn2 * kq);
      s_g[3][t] = v[3] * (kLn2 * kq);
      s_g[4][t] = v[4] * (kLn2 * kq);
      s_g[5][t] = v[5] * sr.b.z;  // d alpha / d alpha_cond = alpha / alpha_cond
      s_ent[t] = __float_as_uint(sr.b.w);
    }
    __syncthreads();
#pragma unroll 1
    for (int r = 0; r < kG2D; r++) {
      const uint32_t idx = (uint32_t)(r * kBlock + t);
      if (idx < nb * kG2D) {
        const uint32_t jg = idx / kG2D, k = idx - jg * kG2D;
        const float val = s_g[k][jg];
        s_g[k][jg] = 0.f;
        if (val != 0.f) unsafeAtomicAdd(g2d + (int64_t)s_ent[jg] * kG2D + k, val);
      }
    }
    __syncthreads();
    bend = b0;
  }
}

}  // namespace

template <bool SAVE, bool COUNTS>
void launch_fwd(const ViewTable& vt, const DevSettings& s, const Rec* rec, const uint2* ranges,
                const uint32_t* pval, const BlendState& bs, hipStream_t st) {
  const dim3 grid(vt.total_tiles);
  switch (vt.tile_w) {
    case 8:
      hipLaunchKernelGGL((k_blend_fwd<8, SAVE, COUNTS>), grid, dim3(kBlock), 0, st, vt, s, rec, ranges, pval, bs);
      break;
    case 32:
      hipLaunchKernelGGL((k_blend_fwd<32, SAVE, COUNTS>), grid, dim3(kBlock), 0, st, vt, s, rec, ranges, pval, bs);
      break;
    default:
      hipLaunchKernelGGL((k_blend_fwd<16, SAVE, COUNTS>), grid, dim3(kBlock), 0, st, vt, s, rec, ranges, pval, bs);
      break;
  }
}

void launch_blend_fwd(const ViewTable& vt, const DevSettings& s, const Rec* rec, const uint2* ranges,
                      const uint32_t* pval, BlendState bs, int batch, bool save, hipStream_t st) {
  if (vt.total_tiles <= 0) return;
  if (!save)
    launch_fwd<false, false>(vt, s, rec, ranges, pval, bs, st);
  else if (bs.counts)
    launch_fwd<true, true>(vt, s, rec, ranges, pval, bs, st);
  else
    launch_fwd<true, false>(vt, s, rec, ranges, pval, bs, st);
}

void launch_blend_bwd(const ViewTable& vt, const DevSettings& s, const Rec* rec, const uint2* ranges,
                      const uint32_t* pval, BlendState bs, float* g2d, int batch, int64_t items, hipStream_t st) {
  if (vt.total_tiles <= 0 || items <= 0) return;
  const dim3 grid((unsigned)items);
  switch (vt.tile_w) {
    case 8: hipLaunchKernelGGL(k_blend_bwd<8>, grid, dim3(kBlock), 0, st, vt, s, rec, ranges, pval, bs, g2d, batch); break;
    case 32: hipLaunchKernelGGL(k_blend_bwd<32>, grid, dim3(kBlock), 0, st, vt, s, rec, ranges, pval, bs, g2d, batch); break;
    default: hipLaunchKernelGGL(k_blend_bwd<16>, grid, dim3(kBlock), 0, st, vt, s, rec, ranges, pval, bs, g2d, batch); break;
  }
}

}  // namespace sixdgs
