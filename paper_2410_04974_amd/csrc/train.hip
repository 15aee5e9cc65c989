// Training-step kernels: the L1 photometric loss with its gradient, and a fused
// Adam update over the [76][n] parameter layout (the paper trains with the
// 3DGS losses and Adam, Sec. 4.4 and Sec. 5.1).
#include "internal.h"

namespace sixdgs {
namespace {

constexpr int kL1MaxBlocks = 1024;
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

__global__ void __launch_bounds__(kBlock) k_l1(const float* __restrict__ img, const float* __restrict__ tgt,
                                               float* __restrict__ dimg, int64_t numel, float inv_count,
                                               float* __restrict__ partial) {
  float acc = 0.f;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < numel; i += stride) {
    const float d = img[i] - tgt[i];
    acc += fabsf(d);
    dimg[i] = (d > 0.f) ? inv_count : ((d < 0.f) ? -inv_count : 0.f);
  }
  const float t = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

__global__ void __launch_bounds__(kBlock) k_l1_final(const float* __restrict__ partial, int64_t count,
                                                     float inv_count, float* __restrict__ loss) {
  float acc = 0.f;
  for (int64_t i = threadIdx.x; i < count; i += kBlock) acc += partial[i];
  const float t = block_sum(acc);
  if (threadIdx.x == 0) *loss = t * inv_count;
}

int l1_blocks(int64_t numel) {
  int64_t b = (numel + (int64_t)kBlock * kL1PerThread - 1) / ((int64_t)kBlock * kL1PerThread);
  if (b < 1) b = 1;
  return (int)(b < kL1MaxBlocks ? b : kL1MaxBlocks);
}


// With a device step counter the bias corrections are formed on the device
// from the step about to be taken (*step + 1), so a captured graph advances
// the step on every replay; k_step_inc then moves the counter on.
__device__ __forceinline__ void device_bias(AdamArgs& a, const int32_t* step_dev) {
  if (step_dev) {
    const float t = (float)(*step_dev + 1);
    a.bc1 = 1.0f - powf(a.b1, t);
    a.bc2 = 1.0f - powf(a.b2, t);
  }
}

__global__ void k_step_inc(int32_t* step_dev) { *step_dev += 1; }

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
  float4 pp = p[k], gg = g[k], mm = m[k], vv = v[k];
  adam_update(pp.x, gg.x, mm.x, vv.x, lr, a);
  adam_update(pp.y, gg.y, mm.y, vv.y, lr, a);
  adam_update(pp.z, gg.z, mm.z, vv.z, lr, a);
  adam_update(pp.w, gg.w, mm.w, vv.w, lr, a);
  p[k] = pp;
  m[k] = mm;
  v[k] = vv;
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
  float pp = p[k], mm = m[k], vv = v[k];
  adam_update(pp, g[k], mm, vv, lr, a);
  p[k] = pp;
  m[k] = mm;
  v[k] = vv;
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
  int64_t off = 0;
  for (int k = 0; k < nimg; k++) {
    const int nb = l1_blocks(numel[k]);
    if (off + nb > partial_cap) break;
    hipLaunchKernelGGL(k_l1, dim3(nb), dim3(kBlock), 0, st, img[k], tgt[k], dimg[k], numel[k], inv, partial + off);
    off += nb;
  }
  hipLaunchKernelGGL(k_l1_final, dim3(1), dim3(kBlock), 0, st, partial, off, inv, loss);
}

AdamArgs make_adam_args(const float lr[6], float b1, float b2, float eps, int step) {
  AdamArgs a;
  for (int k = 0; k < 6; k++) a.lr[k] = lr[k];
  a.b1 = b1;
  a.b2 = b2;
  a.eps = eps;
  a.bc1 = (float)(1.0 - __builtin_pow((double)b1, (double)step));
  a.bc2 = (float)(1.0 - __builtin_pow((double)b2, (double)step));
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
