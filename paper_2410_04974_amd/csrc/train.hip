// Training-step kernels: the L1 photometric loss with its gradient, and a fused
// Adam update over the [76][n] parameter layout (the paper trains with the
// 3DGS losses and Adam, Sec. 4.4 and Sec. 5.1).
#include "internal.h"

namespace sixdgs {
namespace {

constexpr int kL1PerThread = 4;

__device__ __forceinline__ float block_sum(float v) {
  __shared__ float s_w[kBlock / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = v;
  __syncthreads();
  float t = 0.f;
#pragma unroll
  for (int w = 0; w < kBlock / 64; w++) t += s_w[w];
  __syncthreads();
  return t;
}

// The images of one call, one grid row (blockIdx.y) each.
struct L1Images {
  const float* img[kMaxViews];
  const float* tgt[kMaxViews];
  float* dimg[kMaxViews];
  int64_t numel[kMaxViews];
  int64_t off[kMaxViews];  // first partial sum of each image
  int32_t nb[kMaxViews];   // blocks of each image
};

__global__ void __launch_bounds__(kBlock) k_l1(L1Images im, float inv_count, float* __restrict__ partial) {
  const int k = blockIdx.y;
  if ((int)blockIdx.x >= im.nb[k]) return;  // uniform: a smaller image needs fewer blocks
  const float* __restrict__ img = im.img[k];
  const float* __restrict__ tgt = im.tgt[k];
  float* __restrict__ dimg = im.dimg[k];
  const int64_t numel = im.numel[k];
  float acc = 0.f;
  const int64_t stride = (int64_t)im.nb[k] * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < numel; i += stride) {
    const float d = img[i] - tgt[i];
    acc += fabsf(d);
    dimg[i] = (d > 0.f) ? inv_count : ((d < 0.f) ? -inv_count : 0.f);
  }
  const float t = block_sum(acc);
  if (threadIdx.x == 0) partial[im.off[k] + blockIdx.x] = t;
}

// Sum of partial[0, count) by one workgroup, each thread taking kSumRun
// consecutive values per round with as many loads in flight.
constexpr int kSumRun = 16;
constexpr int64_t kSumSpan = (int64_t)kBlock * kSumRun;  // values per round
__device__ __forceinline__ float block_sum_of(const float* __restrict__ partial, int64_t count) {
  float acc[kSumRun];
#pragma unroll
  for (int u = 0; u < kSumRun; u++) acc[u] = 0.f;
  for (int64_t i0 = (int64_t)threadIdx.x * kSumRun; i0 < count; i0 += kSumSpan) {
#pragma unroll
    for (int u = 0; u < kSumRun; u++) acc[u] += i0 + u < count ? partial[i0 + u] : 0.f;
  }
  float a = 0.f;
#pragma unroll
  for (int u = 0; u < kSumRun; u++) a += acc[u];
  return block_sum(a);
}

__global__ void __launch_bounds__(kBlock) k_l1_final(const float* __restrict__ partial, int64_t count,
                                                     float inv_count, float* __restrict__ loss) {
  const float t = block_sum_of(partial, count);
  if (threadIdx.x == 0) *loss = t * inv_count;
}

// First level of a long sum: workgroup b sums partial[b kSumSpan, (b + 1) kSumSpan).
__global__ void __launch_bounds__(kBlock) k_sum_level(const float* __restrict__ partial, int64_t count,
                                                      float* __restrict__ out) {
  const int64_t b0 = (int64_t)blockIdx.x * kSumSpan;
  const float t = block_sum_of(partial + b0, min<int64_t>(kSumSpan, count - b0));
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

int l1_blocks(int64_t numel) {
  int64_t b = (numel + (int64_t)kBlock * kL1PerThread - 1) / ((int64_t)kBlock * kL1PerThread);
  if (b < 1) b = 1;
  return (int)(b < kL1MaxBlocks ? b : kL1MaxBlocks);
}


// ------------------------------------------------------------- D-SSIM
// SSIM (Wang et al. 2004) per channel and pixel under an 11x11 Gaussian window
// (sigma 1.5), zero-padded at the border, C1 = 0.01^2, C2 = 0.03^2; the 3DGS
// loss mixes (1 - lambda) L1 + lambda (1 - mean SSIM), lambda = 0.2 (Sec. 4.4,
// Sec. 5.1: the paper keeps the 3DGS losses).  Tiles of 16x16 outputs with a
// 5-pixel halo in LDS, separable passes (rows, then columns).
constexpr int kSsimTile = 16;
constexpr int kSsimHalo = 5;
constexpr int kSsimSpan = kSsimTile + 2 * kSsimHalo;  // 26
constexpr float kSsimC1 = 0.01f * 0.01f;
constexpr float kSsimC2 = 0.03f * 0.03f;

struct SsimWin {
  float g[2 * kSsimHalo + 1];  // normalised 1D Gaussian
};

// Forward: the five window statistics, SSIM, the partials of SSIM the
// gradient needs (three maps), and per-block sums of SSIM and |x - y|.
__global__ void __launch_bounds__(kBlock) k_ssim_fwd(const float* __restrict__ img, const float* __restrict__ tgt,
                                                     int H, int W, SsimWin win, float* __restrict__ maps,
                                                     float* __restrict__ partial) {
  __shared__ float sx[kSsimSpan][kSsimSpan], sy[kSsimSpan][kSsimSpan];
  __shared__ float hs[5][kSsimSpan][kSsimTile];
  const int t = threadIdx.x, ch = blockIdx.z;
  const int64_t HW = (int64_t)H * W;
  const float* x = img + ch * HW;
  const float* y = tgt + ch * HW;
  const int X0 = blockIdx.x * kSsimTile - kSsimHalo, Y0 = blockIdx.y * kSsimTile - kSsimHalo;
  for (int i = t; i < kSsimSpan * kSsimSpan; i += kBlock) {
    const int r = i / kSsimSpan, c = i % kSsimSpan, gy = Y0 + r, gx = X0 + c;
    const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
    sx[r][c] = in ? x[(int64_t)gy * W + gx] : 0.f;
    sy[r][c] = in ? y[(int64_t)gy * W + gx] : 0.f;
  }
  __syncthreads();
  for (int i = t; i < kSsimSpan * kSsimTile; i += kBlock) {
    const int r = i / kSsimTile, c = i % kSsimTile;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f, a4 = 0.f;
#pragma unroll
    for (int k = 0; k <= 2 * kSsimHalo; k++) {
      const float u = sx[r][c + k], v = sy[r][c + k], w = win.g[k];
      a0 += w * u;
      a1 += w * v;
      a2 += w * u * u;
      a3 += w * v * v;
      a4 += w * u * v;
    }
    hs[0][r][c] = a0;
    hs[1][r][c] = a1;
    hs[2][r][c] = a2;
    hs[3][r][c] = a3;
    hs[4][r][c] = a4;
  }
  __syncthreads();
  const int ty = t / kSsimTile, tx = t % kSsimTile;
  float m[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k <= 2 * kSsimHalo; k++)
#pragma unroll
    for (int q = 0; q < 5; q++) m[q] += win.g[k] * hs[q][ty + k][tx];
  const int px = blockIdx.x * kSsimTile + tx, py = blockIdx.y * kSsimTile + ty;
  float ssim = 0.f, l1 = 0.f;
  if (px < W && py < H) {
    const float mx = m[0], my = m[1];
    const float vx = m[2] - mx * mx, vy = m[3] - my * my, cxy = m[4] - mx * my;
    const float A1 = 2.f * mx * my + kSsimC1, A2 = 2.f * cxy + kSsimC2;
    const float B1 = mx * mx + my * my + kSsimC1, B2 = vx + vy + kSsimC2;
    const float iB = 1.f / (B1 * B2);
    const float S = A1 * A2 * iB;
    const float f_mx = 2.f * my * A2 * iB - S * 2.f * mx / B1;
    const float f_vx = -S / B2;
    const float f_cxy = 2.f * A1 * iB;
    const int64_t pix = (int64_t)py * W + px;
    float* mp = maps + (int64_t)ch * 3 * HW;
    mp[pix] = f_mx - 2.f * mx * f_vx - my * f_cxy;
    mp[HW + pix] = f_vx;
    mp[2 * HW + pix] = f_cxy;
    ssim = S;
    l1 = fabsf(sx[ty + kSsimHalo][tx + kSsimHalo] - sy[ty + kSsimHalo][tx + kSsimHalo]);
  }
  const float bs = block_sum(ssim);
  const float bl = block_sum(l1);
  if (t == 0) {
    const int64_t b = ((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    partial[2 * b] = bs;
    partial[2 * b + 1] = bl;
  }
}

// Backward: dL/dI = (1 - lambda) sign(x - y) / count - lambda / count *
// (w*a + 2 x (w*b) + y (w*c)) from the three maps of the forward.
__global__ void __launch_bounds__(kBlock) k_ssim_bwd(const float* __restrict__ img, const float* __restrict__ tgt,
                                                     int H, int W, SsimWin win, const float* __restrict__ maps,
                                                     float lam, float inv_count, float* __restrict__ dimg) {
  __shared__ float sm[3][kSsimSpan][kSsimSpan];
  __shared__ float hs[3][kSsimSpan][kSsimTile];
  const int t = threadIdx.x, ch = blockIdx.z;
  const int64_t HW = (int64_t)H * W;
  const float* mp = maps + (int64_t)ch * 3 * HW;
  const int X0 = blockIdx.x * kSsimTile - kSsimHalo, Y0 = blockIdx.y * kSsimTile - kSsimHalo;
  for (int i = t; i < kSsimSpan * kSsimSpan; i += kBlock) {
    const int r = i / kSsimSpan, c = i % kSsimSpan, gy = Y0 + r, gx = X0 + c;
    const bool in = gy >= 0 && gy < H && gx >= 0 && gx < W;
    const int64_t pix = (int64_t)gy * W + gx;
#pragma unroll
    for (int q = 0; q < 3; q++) sm[q][r][c] = in ? mp[q * HW + pix] : 0.f;
  }
  __syncthreads();
  for (int i = t; i < kSsimSpan * kSsimTile; i += kBlock) {
    const int r = i / kSsimTile, c = i % kSsimTile;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
#pragma unroll
    for (int k = 0; k <= 2 * kSsimHalo; k++) {
      const float w = win.g[k];
      a0 += w * sm[0][r][c + k];
      a1 += w * sm[1][r][c + k];
      a2 += w * sm[2][r][c + k];
    }
    hs[0][r][c] = a0;
    hs[1][r][c] = a1;
    hs[2][r][c] = a2;
  }
  __syncthreads();
  const int ty = t / kSsimTile, tx = t % kSsimTile;
  const int px = blockIdx.x * kSsimTile + tx, py = blockIdx.y * kSsimTile + ty;
  if (px >= W || py >= H) return;
  float c0 = 0.f, c1 = 0.f, c2 = 0.f;
#pragma unroll
  for (int k = 0; k <= 2 * kSsimHalo; k++) {
    const float w = win.g[k];
    c0 += w * hs[0][ty + k][tx];
    c1 += w * hs[1][ty + k][tx];
    c2 += w * hs[2][ty + k][tx];
  }
  const int64_t pix = ch * HW + (int64_t)py * W + px;
  const float xv = img[pix], yv = tgt[pix], d = xv - yv;
  const float gs = c0 + 2.f * xv * c1 + yv * c2;
  const float g1 = (d > 0.f) ? 1.f : ((d < 0.f) ? -1.f : 0.f);
  dimg[pix] = ((1.f - lam) * g1 - lam * gs) * inv_count;
}

__global__ void __launch_bounds__(kBlock) k_ssim_final(const float* __restrict__ partial, int64_t nblocks,
                                                       float lam, float inv_count, float* __restrict__ loss) {
  float s = 0.f, l = 0.f;
  for (int64_t i = threadIdx.x; i < nblocks; i += kBlock) {
    s += partial[2 * i];
    l += partial[2 * i + 1];
  }
  const float ts = block_sum(s);
  const float tl = block_sum(l);
  if (threadIdx.x == 0) *loss = (1.f - lam) * tl * inv_count + lam * (1.f - ts * inv_count);
}

// With a device step counter the bias corrections are formed on the device
// from the step about to be taken (*step + 1), so a captured graph advances
// the step on every replay; k_step_inc then moves the counter on.
__device__ __forceinline__ void device_bias(AdamArgs& a, const int32_t* step_dev) {
  if (step_dev) adam_device_step(a, *step_dev);
}

__global__ void k_step_inc(int32_t* step_dev) { *step_dev += 1; }

typedef float F4 __attribute__((ext_vector_type(4)));  // a native vector for the non-temporal builtins

// grid.y = parameter row, grid.x covers the row (float4 when n % 4 == 0)
__global__ void __launch_bounds__(kBlock) k_adam4(float4* __restrict__ p, const float4* __restrict__ g,
                                                  float4* __restrict__ m, float4* __restrict__ v, int64_t n4,
                                                  AdamArgs a, const int32_t* step_dev) {
  device_bias(a, step_dev);
  const int r = blockIdx.y;
  const float lr = a.lr[adam_row_group(r)];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n4) return;
  const int64_t k = (int64_t)r * n4 + i;
  // the moments are touched once per step: streamed past the caches, which
  // keep the parameters for the next step's preprocess instead
  const F4 m0 = __builtin_nontemporal_load(reinterpret_cast<const F4*>(m + k));
  const F4 v0 = __builtin_nontemporal_load(reinterpret_cast<const F4*>(v + k));
  float4 pp = p[k], gg = g[k];
  float4 mm = make_float4(m0.x, m0.y, m0.z, m0.w), vv = make_float4(v0.x, v0.y, v0.z, v0.w);
  adam_update(pp.x, gg.x, mm.x, vv.x, lr, a);
  adam_update(pp.y, gg.y, mm.y, vv.y, lr, a);
  adam_update(pp.z, gg.z, mm.z, vv.z, lr, a);
  adam_update(pp.w, gg.w, mm.w, vv.w, lr, a);
  p[k] = pp;
  const F4 m1 = {mm.x, mm.y, mm.z, mm.w}, v1 = {vv.x, vv.y, vv.z, vv.w};
  __builtin_nontemporal_store(m1, reinterpret_cast<F4*>(m + k));
  __builtin_nontemporal_store(v1, reinterpret_cast<F4*>(v + k));
}

__global__ void __launch_bounds__(kBlock) k_adam1(float* __restrict__ p, const float* __restrict__ g,
                                                  float* __restrict__ m, float* __restrict__ v, int64_t n, AdamArgs a,
                                                  const int32_t* step_dev) {
  device_bias(a, step_dev);
  const int r = blockIdx.y;
  const float lr = a.lr[adam_row_group(r)];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  const int64_t k = (int64_t)r * n + i;
  float pp = p[k], mm = __builtin_nontemporal_load(m + k), vv = __builtin_nontemporal_load(v + k);
  adam_update(pp, g[k], mm, vv, lr, a);
  p[k] = pp;
  __builtin_nontemporal_store(mm, m + k);
  __builtin_nontemporal_store(vv, v + k);
}

}  // namespace

int64_t l1_partial_count(int nimg, const int64_t* numel) {
  int64_t c = 0;
  for (int k = 0; k < nimg; k++) c += l1_blocks(numel[k]);
  return c;
}

void launch_l1(int nimg, const float* const* img, const float* const* tgt, const int64_t* numel, float* const* dimg,
               float* partial, int64_t partial_cap, float* loss, hipStream_t st) {
  int64_t total = 0;
  for (int k = 0; k < nimg; k++) total += numel[k];
  const float inv = 1.0f / (float)total;
  // all images in one launch (one grid row each), then the sum of the partials
  L1Images im{};
  int64_t off = 0;
  int nbmax = 1, n = 0;
  for (int k = 0; k < nimg && k < kMaxViews; k++) {
    const int nb = l1_blocks(numel[k]);
    if (off + nb > partial_cap) break;
    im.img[k] = img[k];
    im.tgt[k] = tgt[k];
    im.dimg[k] = dimg[k];
    im.numel[k] = numel[k];
    im.off[k] = off;
    im.nb[k] = nb;
    nbmax = nb > nbmax ? nb : nbmax;
    off += nb;
    n = k + 1;
  }
  if (n > 0) hipLaunchKernelGGL(k_l1, dim3(nbmax, n), dim3(kBlock), 0, st, im, inv, partial);
  hipLaunchKernelGGL(k_l1_final, dim3(1), dim3(kBlock), 0, st, partial, off, inv, loss);
}

int64_t l1_final_scratch(int64_t count) { return count > kSumSpan ? (count + kSumSpan - 1) / kSumSpan : 0; }

void launch_l1_final(const float* partial, int64_t count, float inv, float* loss, float* scratch, hipStream_t st) {
  if (count > kSumSpan) {
    // many tiles (several large views): one level of workgroup sums first
    const int64_t nb = l1_final_scratch(count);
    hipLaunchKernelGGL(k_sum_level, dim3((unsigned)nb), dim3(kBlock), 0, st, partial, count, scratch);
    hipLaunchKernelGGL(k_l1_final, dim3(1), dim3(kBlock), 0, st, (const float*)scratch, nb, inv, loss);
    return;
  }
  hipLaunchKernelGGL(k_l1_final, dim3(1), dim3(kBlock), 0, st, partial, count, inv, loss);
}

int64_t ssim_blocks(int H, int W) {
  return (int64_t)((W + kSsimTile - 1) / kSsimTile) * ((H + kSsimTile - 1) / kSsimTile) * 3;
}

void launch_l1_dssim(int nimg, const float* const* img, const float* const* tgt, const int32_t* H, const int32_t* W,
                     float lam, float* const* dimg, float* maps, float* partial, float* loss, hipStream_t st) {
  SsimWin win;
  double g[2 * kSsimHalo + 1], sum = 0;
  for (int k = 0; k <= 2 * kSsimHalo; k++) {
    const double d = k - kSsimHalo;
    g[k] = __builtin_exp(-d * d / (2.0 * 1.5 * 1.5));
    sum += g[k];
  }
  for (int k = 0; k <= 2 * kSsimHalo; k++) win.g[k] = (float)(g[k] / sum);
  int64_t count = 0;
  for (int k = 0; k < nimg; k++) count += 3 * (int64_t)H[k] * W[k];
  const float inv = 1.0f / (float)count;
  int64_t boff = 0, moff = 0;
  for (int k = 0; k < nimg; k++) {
    const dim3 grid((W[k] + kSsimTile - 1) / kSsimTile, (H[k] + kSsimTile - 1) / kSsimTile, 3);
    hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(kBlock), 0, st, img[k], tgt[k], H[k], W[k], win, maps + moff,
                       partial + 2 * boff);
    hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(kBlock), 0, st, img[k], tgt[k], H[k], W[k], win, maps + moff, lam, inv,
                       dimg[k]);
    boff += ssim_blocks(H[k], W[k]);
    moff += 9 * (int64_t)H[k] * W[k];
  }
  hipLaunchKernelGGL(k_ssim_final, dim3(1), dim3(kBlock), 0, st, partial, boff, lam, inv, loss);
}

AdamArgs make_adam_args(const float lr[6], float b1, float b2, float eps, int step) {
  AdamArgs a;
  for (int k = 0; k < 6; k++) a.lr[k] = lr[k];
  a.b1 = b1;
  a.b2 = b2;
  a.eps = eps;
  a.inv_bc1 = (float)(1.0 / (1.0 - __builtin_pow((double)b1, (double)step)));
  a.inv_sqrt_bc2 = (float)(1.0 / __builtin_sqrt(1.0 - __builtin_pow((double)b2, (double)step)));
  a.lb1 = (float)__builtin_log((double)b1);
  a.lb2 = (float)__builtin_log((double)b2);
  return a;
}

void launch_adam(float* p, const float* g, float* m, float* v, int rows, int64_t n, const float lr[6], float b1,
                 float b2, float eps, int step, int32_t* step_dev, bool advance, hipStream_t st) {
  if (n <= 0 || rows <= 0) return;
  const AdamArgs a = make_adam_args(lr, b1, b2, eps, step_dev ? 1 : step);
  const bool vec = (n % 4 == 0) && ((uintptr_t)p % 16 == 0) && ((uintptr_t)g % 16 == 0) &&
                   ((uintptr_t)m % 16 == 0) && ((uintptr_t)v % 16 == 0);
  if (vec) {
    const int64_t n4 = n / 4;
    const dim3 grid((unsigned)((n4 + kBlock - 1) / kBlock), (unsigned)rows);
    hipLaunchKernelGGL(k_adam4, grid, dim3(kBlock), 0, st, (float4*)p, (const float4*)g, (float4*)m, (float4*)v, n4, a,
                       (const int32_t*)step_dev);
  } else {
    const dim3 grid((unsigned)((n + kBlock - 1) / kBlock), (unsigned)rows);
    hipLaunchKernelGGL(k_adam1, grid, dim3(kBlock), 0, st, p, g, m, v, n, a, (const int32_t*)step_dev);
  }
  if (step_dev && advance) hipLaunchKernelGGL(k_step_inc, dim3(1), dim3(1), 0, st, step_dev);
}

}  // namespace sixdgs
