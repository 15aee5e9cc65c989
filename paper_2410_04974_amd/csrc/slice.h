// Direction-independent part of the slice of a 6D Gaussian (Sec. 3.1, Sec. 3.2
// eq:sigma, Algorithm 1 steps 1-3), shared by the per-Gaussian kernels: the
// activated Cholesky factor, the Sigma blocks, A = Sigma_d^-1, K = Sigma_pd A
// and the conditional covariance Sigma_cond.
#pragma once

#include "internal.h"

namespace sixdgs {

__device__ __forceinline__ float sigmoidf(float x) { return 1.0f / (1.0f + expf(-x)); }

// Index of Cholesky entry (i, j), j <= i, in the packed lower triangle.
__host__ __device__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

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

__device__ __forceinline__ void load_static(const float* __restrict__ params, int64_t n, int64_t g, Static& s) {
#pragma unroll
  for (int k = 0; k < 3; k++) {
    s.mu_p[k] = params[(kRowMuP + k) * n + g];
    s.mu_d[k] = params[(kRowMuD + k) * n + g];
  }
#pragma unroll
  for (int i = 0; i < 6; i++)
#pragma unroll
    for (int j = 0; j <= i; j++) {
      float raw = params[(kRowL + tri(i, j)) * n + g];
      s.L[tri(i, j)] = (i == j) ? expf(raw) : 2.0f * sigmoidf(raw) - 1.0f;
    }
  s.alpha = sigmoidf(params[kRowOpa * n + g]);
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
  float id = 1.0f / det;
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

// The same from the inference cache (see kCacheRows): only what the forward
// slice uses (mu_p, mu_d, K, Sigma_d^-1, Sigma_cond, alpha).
__device__ __forceinline__ void load_cached(const float* __restrict__ params, const float* __restrict__ cache,
                                            int64_t n, int64_t g, Static& s) {
#pragma unroll
  for (int k = 0; k < 3; k++) {
    s.mu_p[k] = params[(kRowMuP + k) * n + g];
    s.mu_d[k] = params[(kRowMuD + k) * n + g];
  }
  const float c00 = cache[0 * n + g], c01 = cache[1 * n + g], c02 = cache[2 * n + g];
  const float c11 = cache[3 * n + g], c12 = cache[4 * n + g], c22 = cache[5 * n + g];
  s.Sc[0][0] = c00; s.Sc[0][1] = c01; s.Sc[0][2] = c02;
  s.Sc[1][0] = c01; s.Sc[1][1] = c11; s.Sc[1][2] = c12;
  s.Sc[2][0] = c02; s.Sc[2][1] = c12; s.Sc[2][2] = c22;
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) s.K[a][b] = cache[(6 + 3 * a + b) * n + g];
  const float a00 = cache[15 * n + g], a01 = cache[16 * n + g], a02 = cache[17 * n + g];
  const float a11 = cache[18 * n + g], a12 = cache[19 * n + g], a22 = cache[20 * n + g];
  s.A[0][0] = a00; s.A[0][1] = a01; s.A[0][2] = a02;
  s.A[1][0] = a01; s.A[1][1] = a11; s.A[1][2] = a12;
  s.A[2][0] = a02; s.A[2][1] = a12; s.A[2][2] = a22;
  s.alpha = cache[21 * n + g];
}

}  // namespace sixdgs
