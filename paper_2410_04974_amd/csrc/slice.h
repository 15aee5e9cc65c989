// Direction-independent part of the slice of a 6D Gaussian (Sec. 3.1, Sec. 3.2
// eq:sigma, Algorithm 1 steps 1-3), shared by the per-Gaussian kernels: the
// activated Cholesky factor, the Sigma blocks, A = Sigma_d^-1, K = Sigma_pd A
// and the conditional covariance Sigma_cond.
#pragma once

#include "internal.h"

namespace sixdgs {

__device__ __forceinline__ float sigmoidf(float x) { return 1.0f / (1.0f + expf(-x)); }

// The slice's arithmetic in one of two forms.  Exact: correctly rounded
// division and square root and the library exp, for the forward, whose
// results are held to the decision margins of the float32 analysis.  Fast:
// the hardware reciprocal, square root and exp2 (about an ulp each), for the
// backward, which recomputes those values only as the point at which it
// differentiates, so an ulp there moves a gradient by about an ulp.
template <bool FAST>
struct SliceMath {
  static __device__ __forceinline__ float div(float a, float b) {
    if constexpr (FAST) return a * __builtin_amdgcn_rcpf(b);
    else return a / b;
  }
  static __device__ __forceinline__ float sqrt(float x) {
    if constexpr (FAST) return __builtin_amdgcn_sqrtf(x);
    else return sqrtf(x);
  }
  static __device__ __forceinline__ float exp(float x) {
    if constexpr (FAST) return __builtin_amdgcn_exp2f(x * 1.44269504088896341f);
    else return expf(x);
  }
  static __device__ __forceinline__ float sigmoid(float x) {
    if constexpr (FAST) return __builtin_amdgcn_rcpf(1.0f + exp(-x));
    else return sigmoidf(x);
  }
};

// Index of Cholesky entry (i, j), j <= i, in the packed lower triangle.
__host__ __device__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }
// Entry g of row `row` of a row-major [rows][n] array of 4-byte elements,
// n < 2^30.  The row's base is the same for the whole wavefront and the lane's
// part is a 32-bit byte offset; both pass through empty asm statements that
// keep the compiler from folding them back into one 64-bit vector address per
// row, so each access is issued with a scalar base and the one vector offset
// that every row shares.
__device__ __forceinline__ uint32_t lane_offset(int64_t g) {
  uint32_t o = (uint32_t)g * 4u;
  asm("" : "+v"(o));
  return o;
}
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* row_ptr(T* a, int row, int64_t n, int64_t g) {
  static_assert(sizeof(T) == 4, "4-byte rows");
  typedef __attribute__((address_space(1))) char gbyte;
  gbyte* base = (gbyte*)(a + (int64_t)row * n);
  asm("" : "+s"(base));
  return (__attribute__((address_space(1))) T*)(base + lane_offset(g));
}
template <class T>
__device__ __forceinline__ T row_ld(const T* a, int row, int64_t n, int64_t g) {
  return *row_ptr(a, row, n, g);
}
template <class T>
__device__ __forceinline__ void row_st(T* a, int row, int64_t n, int64_t g, T v) {
  *row_ptr(a, row, n, g) = v;
}

struct Static {
  float L[21];
  float Spd[3][3];
  float A[3][3];
  float K[3][3];
  float Sc[3][3];
  float mu_p[3], mu_d[3];
  float alpha;
};

__device__ __forceinline__ float Lget(const float* L, int i, int j) { return j <= i ? L[tri(i, j)] : 0.0f; }

// The 28 geometry rows of a Gaussian as stored: means, raw Cholesky entries
// and the opacity logit.
struct RawGeom {
  float mu_p[3], mu_d[3], L[21], opa;
};

__device__ __forceinline__ void load_raw_geom(const float* params, int64_t n, int64_t g, RawGeom& r) {
#pragma unroll
  for (int k = 0; k < 3; k++) {
    r.mu_p[k] = row_ld(params, kRowMuP + k, n, g);
    r.mu_d[k] = row_ld(params, kRowMuD + k, n, g);
  }
#pragma unroll
  for (int k = 0; k < 21; k++) r.L[k] = row_ld(params, kRowL + k, n, g);
  r.opa = row_ld(params, kRowOpa, n, g);
}

// The 6D Cholesky factor from its raw entries: exp on the diagonal, 2 sigmoid - 1
// (a value in (-1, 1)) below it.
template <bool FAST = false>
__device__ __forceinline__ void cholesky_from_raw(const float raw[21], float L[21]) {
  using M = SliceMath<FAST>;
#pragma unroll
  for (int i = 0; i < 6; i++)
#pragma unroll
    for (int j = 0; j <= i; j++)
      L[tri(i, j)] = (i == j) ? M::exp(raw[tri(i, j)]) : 2.0f * M::sigmoid(raw[tri(i, j)]) - 1.0f;
}

template <bool FAST = false>
__device__ __forceinline__ void load_cholesky(const float* params, int64_t n, int64_t g, float L[21]) {
  float raw[21];
#pragma unroll
  for (int k = 0; k < 21; k++) raw[k] = row_ld(params, kRowL + k, n, g);
  cholesky_from_raw<FAST>(raw, L);
}

// The direction-independent part of the slice (Sec. 3.2) from the raw rows:
// covariance blocks, A = Sigma_d^-1, K = Sigma_pd A, Sigma_cond, opacity.
template <bool FAST = false>
__device__ __forceinline__ void static_from_raw(const RawGeom& r, Static& s) {
  using M = SliceMath<FAST>;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    s.mu_p[k] = r.mu_p[k];
    s.mu_d[k] = r.mu_d[k];
  }
  cholesky_from_raw<FAST>(r.L, s.L);
  s.alpha = M::sigmoid(r.opa);
  float Sp[3][3], Sd[3][3];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) {
      float sp = 0.f, spd = 0.f, sd = 0.f;
#pragma unroll
      for (int k = 0; k < 6; k++) {
        sp += Lget(s.L, a, k) * Lget(s.L, b, k);
        spd += Lget(s.L, a, k) * Lget(s.L, 3 + b, k);
        sd += Lget(s.L, 3 + a, k) * Lget(s.L, 3 + b, k);
      }
      Sp[a][b] = sp;
      s.Spd[a][b] = spd;
      Sd[a][b] = sd;
    }
  // symmetric 3x3 inverse by the adjugate
  float c00 = Sd[1][1] * Sd[2][2] - Sd[1][2] * Sd[2][1];
  float c01 = Sd[1][2] * Sd[2][0] - Sd[1][0] * Sd[2][2];
  float c02 = Sd[1][0] * Sd[2][1] - Sd[1][1] * Sd[2][0];
  float det = Sd[0][0] * c00 + Sd[0][1] * c01 + Sd[0][2] * c02;
  float id = M::div(1.0f, det);
  s.A[0][0] = c00 * id;
  s.A[0][1] = s.A[1][0] = c01 * id;
  s.A[0][2] = s.A[2][0] = c02 * id;
  s.A[1][1] = (Sd[0][0] * Sd[2][2] - Sd[0][2] * Sd[2][0]) * id;
  s.A[1][2] = s.A[2][1] = (Sd[0][2] * Sd[1][0] - Sd[0][0] * Sd[1][2]) * id;
  s.A[2][2] = (Sd[0][0] * Sd[1][1] - Sd[0][1] * Sd[1][0]) * id;
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) s.K[a][b] = s.Spd[a][0] * s.A[0][b] + s.Spd[a][1] * s.A[1][b] + s.Spd[a][2] * s.A[2][b];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++)
      s.Sc[a][b] = Sp[a][b] - (s.K[a][0] * s.Spd[b][0] + s.K[a][1] * s.Spd[b][1] + s.K[a][2] * s.Spd[b][2]);
  // exact symmetry
  s.Sc[1][0] = s.Sc[0][1];
  s.Sc[2][0] = s.Sc[0][2];
  s.Sc[2][1] = s.Sc[1][2];
}

__device__ __forceinline__ void load_static(const float* params, int64_t n, int64_t g, Static& s) {
  RawGeom r;
  load_raw_geom(params, n, g, r);
  static_from_raw(r, s);
}

// The same from the inference cache (see kCacheRows): only what the forward
// slice uses (mu_p, mu_d, K, Sigma_d^-1, Sigma_cond, alpha).
__device__ __forceinline__ void load_cached(const float* __restrict__ params, const float* __restrict__ cache,
                                            int64_t n, int64_t g, Static& s) {
#pragma unroll
  for (int k = 0; k < 3; k++) {
    s.mu_p[k] = row_ld(params, kRowMuP + k, n, g);
    s.mu_d[k] = row_ld(params, kRowMuD + k, n, g);
  }
  const float c00 = row_ld(cache, 0, n, g), c01 = row_ld(cache, 1, n, g), c02 = row_ld(cache, 2, n, g);
  const float c11 = row_ld(cache, 3, n, g), c12 = row_ld(cache, 4, n, g), c22 = row_ld(cache, 5, n, g);
  s.Sc[0][0] = c00; s.Sc[0][1] = c01; s.Sc[0][2] = c02;
  s.Sc[1][0] = c01; s.Sc[1][1] = c11; s.Sc[1][2] = c12;
  s.Sc[2][0] = c02; s.Sc[2][1] = c12; s.Sc[2][2] = c22;
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) s.K[a][b] = row_ld(cache, 6 + 3 * a + b, n, g);
  const float a00 = row_ld(cache, 15, n, g), a01 = row_ld(cache, 16, n, g), a02 = row_ld(cache, 17, n, g);
  const float a11 = row_ld(cache, 18, n, g), a12 = row_ld(cache, 19, n, g), a22 = row_ld(cache, 20, n, g);
  s.A[0][0] = a00; s.A[0][1] = a01; s.A[0][2] = a02;
  s.A[1][0] = a01; s.A[1][1] = a11; s.A[1][2] = a12;
  s.A[2][0] = a02; s.A[2][1] = a12; s.A[2][2] = a22;
  s.alpha = row_ld(cache, 21, n, g);
}

}  // namespace sixdgs
