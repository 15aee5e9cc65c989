// Internal declarations of the gfx950 renderer: device-side camera table,
// projected record, the settings the kernels see, and the host launchers each
// translation unit provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sixdgs.h"

namespace sixdgs {

constexpr int kRows = 76;
// Inference cache rows per Gaussian (the direction-independent part of the
// slice): Sigma_cond (00 01 02 11 12 22), K = Sigma_pd Sigma_d^-1 (row-major),
// Sigma_d^-1 (00 01 02 11 12 22), alpha.
constexpr int kCacheRows = 22;
constexpr int kRowMuP = 0;
constexpr int kRowMuD = 3;
constexpr int kRowL = 6;
constexpr int kRowSH = 27;
constexpr int kRowOpa = 75;
constexpr int kMaxViews = SIXDGS_MAX_VIEWS;
constexpr int kBlock = 256;  // threads per workgroup for every kernel here

// One camera as the kernels see it (passed by value in kernel arguments).
struct ViewDesc {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  float C[3];        // camera centre -R^T t
  float limx, limy;  // Jacobian guard: 1.3 * tan(half field of view)
  int32_t W, H;
  int32_t ntx, nty;   // tiles per row / column
  int32_t tile_base;  // first global tile id of this view
  int32_t pad0;
  int64_t pix_base;   // offset of this view in the per-pixel state arrays
  float* img;         // [3][H][W] output (forward)
  const float* dimg;  // [3][H][W] upstream gradient (backward)
  const float* tgt;   // [3][H][W] L1 target of a forward with the loss, or nullptr
  float* dl;          // [3][H][W] its dL/dI output
};

struct ViewTable {
  int32_t nview;
  int32_t tile_w, tile_h;
  int32_t tile_shift_x, tile_shift_y;  // log2 of tile_w, tile_h
  int32_t total_tiles;
  int64_t n;  // Gaussians (entry e = view * n + gaussian)
  ViewDesc v[kMaxViews];
};

// Rasteriser constants (the 3D Gaussian splatting ones) and the method's lambda.
struct DevSettings {
  float lambda_opa;
  float z_near;
  float bg[3];
  int32_t rgb_color;        // colour = sigmoid of the SH degree-0 rows (no SH), else the SH expansion
  const float* lambda_raw;  // [n] learnable per-Gaussian lambda = sigmoid(raw), or nullptr: lambda_opa
  float* grad_lambda;       // [n] backward output dL/dlambda_raw, or nullptr
};
constexpr float kDilation = 0.3f;
constexpr float kGuard = 1.3f;
constexpr float kAlphaMax = 0.99f;
constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kTMin = 1e-4f;

// Projected record of one (view, Gaussian) entry, 48 bytes, gathered per pair.
//   a = (u, v, Qxx, Qxy)   b = (Qyy, alpha_cond, ex, ey)   c = (r, g, b, depth)
struct __align__(16) Rec {
  float4 a, b, c;
};

// Screen-space gradient accumulator of one entry:
//   du, dv, dQxx, dQxy, dQyy, dalpha_cond, dr, dg, db  (dQ as full-matrix gradient)
constexpr int kG2D = 9;

// Tile rectangle [x0, x1) x [y0, y1) of an extent box, the one definition used
// by both the projection (to count tiles) and the pair emission (to list them).
__device__ __forceinline__ void tile_rect(float u, float v, float ex, float ey, int shift_x, int shift_y, int ntx,
                                          int nty, int& x0, int& y0, int& x1, int& y1) {
  const float ix = 1.0f / (float)(1 << shift_x);
  const float iy = 1.0f / (float)(1 << shift_y);
  // a subtraction then a multiplication by an exact power of two: no contraction possible
  x0 = (int)floorf(__fmul_rn(__fsub_rn(u, ex), ix));
  x1 = (int)floorf(__fmul_rn(__fadd_rn(u, ex), ix)) + 1;
  y0 = (int)floorf(__fmul_rn(__fsub_rn(v, ey), iy));
  y1 = (int)floorf(__fmul_rn(__fadd_rn(v, ey), iy)) + 1;
  x0 = min(max(x0, 0), ntx);
  x1 = min(max(x1, 0), ntx);
  y0 = min(max(y0, 0), nty);
  y1 = min(max(y1, 0), nty);
}

// One Adam step's constants.  The bias corrections 1 - b^t enter as two
// factors: mhat = m / (1 - b1^t) and sqrt(vhat) = sqrt(v) / sqrt(1 - b2^t), so
// an element takes one square root and one reciprocal (the hardware ones,
// correct to about an ulp).  lb1, lb2 = ln b1, ln b2 (for a step count read
// on the device).
struct AdamArgs {
  float lr[6];  // row groups: mu_p, mu_d, Cholesky, SH degree 0, SH degrees 1-3, opacity
  float b1, b2, eps;
  float inv_bc1;       // 1 / (1 - b1^t)
  float inv_sqrt_bc2;  // 1 / sqrt(1 - b2^t)
  float lb1, lb2;
};
AdamArgs make_adam_args(const float lr[6], float b1, float b2, float eps, int step);

// The bias-correction factors of step t = step_count + 1 (uniform: every lane
// computes the same), with 1 - b^t = -expm1(t ln b), which keeps its relative
// precision where b^t is close to 1.
__device__ __forceinline__ void adam_device_step(AdamArgs& a, int32_t step_count) {
  const float t = (float)(step_count + 1);
  a.inv_bc1 = -1.0f / expm1f(t * a.lb1);
  a.inv_sqrt_bc2 = 1.0f / sqrtf(-expm1f(t * a.lb2));
}

__device__ __forceinline__ int adam_row_group(int r) {
  return r < 3 ? 0 : r < 6 ? 1 : r < 27 ? 2 : r < 30 ? 3 : r < 75 ? 4 : 5;
}

// Bias-corrected Adam update of one parameter:
// p -= lr mhat / (sqrt(vhat) + eps).
__device__ __forceinline__ void adam_update(float& p, float g, float& m, float& v, float lr, const AdamArgs& a) {
  m = a.b1 * m + (1.f - a.b1) * g;
  v = a.b2 * v + (1.f - a.b2) * g * g;
  const float den = __builtin_amdgcn_sqrtf(v) * a.inv_sqrt_bc2 + a.eps;
  p -= (lr * a.inv_bc1) * m * __builtin_amdgcn_rcpf(den);
}

// ----------------------------------------------------------- host launchers
// preprocess.hip
// cache: nullptr, or the inference cache of params (then the slice's
// direction-independent part is read instead of computed)
// The integer stage's preparation -- state words to zero and the tile ranges
// set to (UINT_MAX, 0) -- done by the threads of the launch before the stage
// (thread i takes word i of every region), which saves the stage a launch.
struct BinPrep {
  uint32_t* p[4];
  int64_t n[4];      // words of each region
  uint2* ranges;
  int64_t nranges;
  int64_t threads;   // the largest region: the launch runs at least this many threads
};
__device__ __forceinline__ void bin_prep_at(const BinPrep& bp, int64_t i) {
#pragma unroll
  for (int k = 0; k < 4; k++)
    if (bp.p[k] && i < bp.n[k]) bp.p[k][i] = 0u;
  if (bp.ranges && i < bp.nranges) bp.ranges[i] = make_uint2(0xFFFFFFFFu, 0u);  // merged by min / max
}
// With bp, the launch also does the integer stage's preparation (then the
// return value is true and launch_bin_count is told so).
bool launch_preprocess(const float* params, const float* cache, int64_t n, const ViewTable& vt,
                       const DevSettings& s, Rec* rec, uint32_t* tiles, float* depth, const BinPrep* bp,
                       hipStream_t st);
void launch_build_cache(const float* params, int64_t n, float* cache, hipStream_t st);
void launch_preprocess_bwd(const float* params, int64_t n, const ViewTable& vt, const DevSettings& s,
                           const uint32_t* tiles, const float* g2d, float* grad, float* densify, hipStream_t st);
// The same chain rule with an Adam step applied to params/m/v in place of writing the gradient.
// step_dev: nullptr (the step is in `a`), or the device step count (step = *step_dev + 1); then
// done, if not nullptr, is a zeroed device word with which the last workgroup advances the count.
void launch_preprocess_bwd_adam(float* params, int64_t n, const ViewTable& vt, const DevSettings& s,
                                const uint32_t* tiles, const float* g2d, float* m, float* v, const AdamArgs& a,
                                int32_t* step_dev, uint32_t* done, float* densify, hipStream_t st);

// sort.hip -- the integer stage
constexpr int kMaxPasses = 4;  // radix passes of at most 8 bits over a 32-bit key

struct SortBuffers {
  // entries
  int64_t E;
  uint32_t* tiles;      // [E] tiles touched (input)
  const Rec* rec;       // [E]
  const float* depth;   // [E] camera depth of every binned entry
  uint32_t* dkey[2];    // [E] depth keys (ping-pong)
  uint32_t* dval[2];    // [E] entry ids
  uint32_t* poff;       // [E] exclusive pair offsets of the depth-sorted entries
  // pairs
  int64_t pcap;
  uint32_t* pkey[2];    // [pcap] global tile ids
  uint32_t* pval[2];    // [pcap] entry ids
  uint2* ranges;        // [total_tiles]
  // scratch
  uint32_t* rstate_depth;  // [sort_state_words(E, false)] state of the scans and the depth sort
  uint32_t* rstate_pairs;  // [sort_state_words(pcap, true)] radix state of the tile sort
  uint32_t* blk_start;     // [nblk_start] first sorted entry of each emission block
  int64_t nblk_start;      // sort_block_starts(pcap) when the pair buffers were sized
  int64_t total_tiles;     // tiles of the views being binned
  uint32_t* tile_order;    // [total_tiles] tiles, longest lists first (the compositing order)
  float* g2d;              // [E][kG2D] screen-space gradient accumulators to clear, or nullptr
  uint32_t* order_state;   // [order_state_words()] bucket counts and cursors of the tile order
  uint32_t* n_items;       // the backward work-item count, zeroed here and counted by the forward
  uint32_t* counters;      // [0] binned entries, [1] pairs, [2] overflow flag, [3] sort look-back timeout
  // where the sorted results ended up (index into the ping-pong pairs)
  int dsorted, psorted;
};
// Scratch sizes (32-bit words) of the integer stage for a bound on the items.
int64_t sort_state_words(int64_t bound, bool pairs);
int64_t sort_block_starts(int64_t pcap);
int64_t order_state_words();
// Stage 1: compaction of binned entries and their depth sort, then the pair
// offsets; leaves counters[0] = binned entries, counters[1] = pairs.
// The preparation of the integer stage over b (for launch_preprocess).
BinPrep bin_prep(const SortBuffers& b);
// prepped: bin_prep(b) has been done by an earlier launch on the stream.
void launch_bin_count(SortBuffers& b, bool prepped, hipStream_t st);
// Stage 2: emission of (tile, entry) pairs, their stable tile sort and the
// per-tile ranges; `pairs_hint` bounds the launch sizes (the capacity in
// fixed mode, the exact count otherwise).  `regrown`: the pair buffers and
// the scratch were reallocated after stage 1, so the pair sort's histograms
// and the emission blocks' first entries are set up again.
void launch_bin_emit(SortBuffers& b, const ViewTable& vt, int64_t pairs_hint, bool regrown, hipStream_t st);
// Zero the screen-space gradient accumulators of the binned entries.
void launch_zero_g2d(const SortBuffers& b, float* g2d, hipStream_t st);
// sixdgs_bin's record import: (u, v, ex, ey, depth, alive) -> Rec + tiles.
void launch_import_records(const float* u, const float* v, const float* ex, const float* ey, const float* depth,
                           const int32_t* alive, const ViewTable& vt, Rec* rec, uint32_t* tiles, hipStream_t st);

// blend.hip
// The backward splits each tile's list into work items of `chunk` list
// positions (a power of two and a multiple of the LDS batch); the forward
// saves each tile pixel's transmittance, and the colour behind, where a chunk
// begins.
struct BlendState {
  uint32_t chunk;
  uint32_t chunk_shift;  // log2(chunk)
  float* T_final;      // [pixels]
  uint32_t* last;      // [pixels] 1-based list position of the last contributor (0: none)
  uint32_t* counts;    // [pixels] or nullptr
  float4* bound;       // [nbound][kBlock] per tile pixel at each chunk start after the first: the
                       // transmittance there and the colour of everything behind it (background
                       // excluded); slot = absolute pair position / chunk (unique per boundary)
  int64_t nbound;
  uint32_t* tile_nch;  // [total_tiles] backward work items per tile
  const uint32_t* order;  // [total_tiles] forward workgroup -> tile (longest lists first)
  uint2* items;        // [items_cap] (tile, chunk) backward work items
  int64_t items_cap;
  uint32_t* n_items;   // device count of items
  float* l1_partial;   // [total_tiles] each tile's sum of |I - I*| when the views carry L1 targets, or nullptr
  float l1_inv;        // 1 / (elements of all images): dL/dI = sign(I - I*) * l1_inv
};
// save = false: the image only, none of the state a backward needs
void launch_blend_fwd(const ViewTable& vt, const DevSettings& s, const Rec* rec, const uint2* ranges,
                      const uint32_t* pval, BlendState bs, int batch, bool save, hipStream_t st);
// `grid` bounds the number of backward work items (pairs / chunk + tiles).
void launch_blend_bwd(const ViewTable& vt, const DevSettings& s, const Rec* rec, const uint2* ranges,
                      const uint32_t* pval, BlendState bs, float* g2d, int batch, int64_t grid, hipStream_t st);
// Words of state of launch_count_scan over n counts.
int64_t chunk_scan_words(int64_t n);
// sort.hip: exclusive scan of n counts into off, the sum into *total (device);
// `state` holds chunk_scan_words(n) words (zeroed here).
void launch_count_scan(const uint32_t* cnt, int64_t n, uint32_t* off, uint32_t* total, uint32_t* state,
                       uint32_t* err, hipStream_t st);

// density.hip: rotation and scale of Sigma_cond; the density-control plan
// (decision and output count per Gaussian) and its application.
void launch_decompose(const float* params, int64_t n, float* R, float* S, hipStream_t st);
void launch_density_plan(const float* params, int64_t n, const float* stats, const sixdgs_density_settings& d,
                         uint8_t* dec, uint32_t* cnt, hipStream_t st);
void launch_density_apply(const float* params, const float* m, const float* v, const float* lam, int64_t n,
                          const float* noise, const uint8_t* dec, const uint32_t* off, float* po, float* mo,
                          float* vo, float* lo, int64_t n_out, hipStream_t st);

// train.hip
// Workgroups of the L1 kernel per image at most (one partial sum each).
constexpr int kL1MaxBlocks = 1024;
// The loss from per-tile partial sums of |I - I*| (the forward with the L1 loss): loss = sum * inv.
// scratch: l1_final_scratch(count) floats (none for up to 4,096 partials).
int64_t l1_final_scratch(int64_t count);
void launch_l1_final(const float* partial, int64_t count, float inv, float* loss, float* scratch, hipStream_t st);
void launch_l1(int nimg, const float* const* img, const float* const* tgt, const int64_t* numel,
               float* const* dimg, float* partial, int64_t partial_cap, float* loss, hipStream_t st);
int64_t l1_partial_count(int nimg, const int64_t* numel);
// (1 - lam) L1 + lam (1 - SSIM) over nimg [3][H][W] views: maps holds
// 9 floats per pixel of every view, partial 2 floats per 16x16 tile and channel.
int64_t ssim_blocks(int H, int W);
void launch_l1_dssim(int nimg, const float* const* img, const float* const* tgt, const int32_t* H, const int32_t* W,
                     float lam, float* const* dimg, float* maps, float* partial, float* loss, hipStream_t st);
// Adam over `rows` rows of n floats (rows = 76: the parameter layout, one lr
// per row group; rows = 1: a single vector with lr[0]).  With step_dev the
// step is *step_dev + 1, and the counter is advanced when `advance`.
void launch_adam(float* p, const float* g, float* m, float* v, int rows, int64_t n, const float lr[6], float b1,
                 float b2, float eps, int step, int32_t* step_dev, bool advance, hipStream_t st);

}  // namespace sixdgs
