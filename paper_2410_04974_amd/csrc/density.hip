// Adaptive density control (Sec. 4.3).  The 3D Gaussian splatting clone /
// split / prune rules need a rotation R and a scale S per Gaussian; they come
// from the SVD of the conditional covariance, Sigma_cond = U D U^T (for this
// symmetric positive definite matrix, its eigendecomposition): R = U with the
// last axis making R proper, S = sqrt(diag D).  Pruning uses the minimum
// opacity 0.01 (Sec. 5.1).
//
// The eigendecomposition is cyclic Jacobi in registers, one thread per
// Gaussian.  A density step is planned (one decision and output count per
// Gaussian, an exclusive scan of the counts) and then applied into new
// parameter / moment arrays whose size the plan reports.
#include "internal.h"
#include "slice.h"

namespace sixdgs {
namespace {

constexpr float kSplitScale = 1.6f;
constexpr int kPrune = 0, kKeep = 1, kClone = 2, kSplit = 3;

// Eigenvalues (diagonal of a on return) and eigenvectors (columns of V) of a
// symmetric 3x3 matrix: each Jacobi rotation in the (p, q) plane zeroes
// a[p][q]; the off-diagonal mass falls quadratically, so a few sweeps reach
// float32 precision.
__device__ void sym_eig3(float a[3][3], float V[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) V[i][j] = (i == j) ? 1.f : 0.f;
  for (int sweep = 0; sweep < 10; sweep++) {
    const float off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const float dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (!(off > 1e-14f * dia)) break;
#pragma unroll
    for (int k = 0; k < 3; k++) {
      const int p = (k == 2) ? 1 : 0, q = (k == 0) ? 1 : 2, r = 3 - p - q;
      const float apq = a[p][q];
      if (apq == 0.f) continue;
      // the smaller root t = tan(theta) of t^2 + 2 tau t - 1 = 0
      const float tau = (a[q][q] - a[p][p]) / (2.f * apq);
      const float t = fabsf(tau) > 1e18f ? 0.5f / tau : copysignf(1.f, tau) / (fabsf(tau) + sqrtf(tau * tau + 1.f));
      const float c = 1.f / sqrtf(t * t + 1.f), s = t * c;
      const float arp = a[r][p], arq = a[r][q];
      a[p][p] -= t * apq;
      a[q][q] += t * apq;
      a[p][q] = a[q][p] = 0.f;
      a[r][p] = a[p][r] = c * arp - s * arq;
      a[r][q] = a[q][r] = s * arp + c * arq;
#pragma unroll
      for (int i = 0; i < 3; i++) {
        const float vp = V[i][p], vq = V[i][q];
        V[i][p] = c * vp - s * vq;
        V[i][q] = s * vp + c * vq;
      }
    }
  }
}

// R (row-major) and S (descending) of Sigma_cond.  Signs: the first two axes
// with their largest component positive, the third their cross product (the
// paper's sign(det R) correction of the last column).
__device__ void rotation_scale(const float Sc[3][3], float R[3][3], float S[3]) {
  float a[3][3], V[3][3];
#pragma unroll
  for (int i = 0; i < 3; i++)
#pragma unroll
    for (int j = 0; j < 3; j++) a[i][j] = Sc[i][j];
  sym_eig3(a, V);
  float w[3] = {a[0][0], a[1][1], a[2][2]};
  int o[3] = {0, 1, 2};
  // sort descending (three compares)
  if (w[o[0]] < w[o[1]]) { const int x = o[0]; o[0] = o[1]; o[1] = x; }
  if (w[o[1]] < w[o[2]]) { const int x = o[1]; o[1] = o[2]; o[2] = x; }
  if (w[o[0]] < w[o[1]]) { const int x = o[0]; o[0] = o[1]; o[1] = x; }
#pragma unroll
  for (int k = 0; k < 2; k++) {
    float col[3] = {V[0][o[k]], V[1][o[k]], V[2][o[k]]};
    int big = 0;
    if (fabsf(col[1]) > fabsf(col[big])) big = 1;
    if (fabsf(col[2]) > fabsf(col[big])) big = 2;
    const float sg = col[big] < 0.f ? -1.f : 1.f;
#pragma unroll
    for (int i = 0; i < 3; i++) R[i][k] = sg * col[i];
    S[k] = sqrtf(fmaxf(w[o[k]], 0.f));
  }
  R[0][2] = R[1][0] * R[2][1] - R[2][0] * R[1][1];
  R[1][2] = R[2][0] * R[0][1] - R[0][0] * R[2][1];
  R[2][2] = R[0][0] * R[1][1] - R[1][0] * R[0][1];
  S[2] = sqrtf(fmaxf(w[o[2]], 0.f));
}

__global__ void __launch_bounds__(kBlock) k_decompose(const float* __restrict__ params, int64_t n,
                                                      float* __restrict__ Rout, float* __restrict__ Sout) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= n) return;
  Static s;
  load_static(params, n, g, s);
  float R[3][3], S[3];
  rotation_scale(s.Sc, R, S);
#pragma unroll
  for (int i = 0; i < 3; i++) {
#pragma unroll
    for (int j = 0; j < 3; j++) Rout[(3 * i + j) * n + g] = R[i][j];
    Sout[i * n + g] = S[i];
  }
}

__device__ __forceinline__ int decide(const float* __restrict__ params, int64_t n, int64_t g,
                                      const float* __restrict__ stats, const sixdgs_density_settings& d, float S0) {
  const float alpha = sigmoidf(params[kRowOpa * n + g]);
  if (alpha < d.min_opacity) return kPrune;
  const float cnt = stats[n + g];
  const float avg = cnt > 0.f ? stats[g] / fmaxf(cnt, 1.f) : 0.f;
  if (!(avg >= d.grad_threshold)) return kKeep;
  return S0 > d.percent_dense * d.extent ? kSplit : kClone;
}

__global__ void __launch_bounds__(kBlock) k_density_plan(const float* __restrict__ params, int64_t n,
                                                         const float* __restrict__ stats,
                                                         sixdgs_density_settings d, uint8_t* __restrict__ dec,
                                                         uint32_t* __restrict__ cnt) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= n) return;
  Static s;
  load_static(params, n, g, s);
  float R[3][3], S[3];
  rotation_scale(s.Sc, R, S);
  const int k = decide(params, n, g, stats, d, S[0]);
  dec[g] = (uint8_t)k;
  cnt[g] = k == kPrune ? 0u : (k == kKeep ? 1u : 2u);
}

__global__ void __launch_bounds__(kBlock) k_density_apply(const float* __restrict__ params,
                                                          const float* __restrict__ m, const float* __restrict__ v,
                                                          const float* __restrict__ lam, int64_t n,
                                                          const float* __restrict__ noise,
                                                          const uint8_t* __restrict__ dec,
                                                          const uint32_t* __restrict__ off, float* __restrict__ po,
                                                          float* __restrict__ mo, float* __restrict__ vo,
                                                          float* __restrict__ lo, int64_t n_out) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= n) return;
  const int k = dec[g];
  if (k == kPrune) return;
  const int outs = (k == kKeep) ? 1 : 2;
  const int64_t o = off[g];
  if (o + outs > n_out) return;  // a plan for other inputs: never write past the arrays
  if (k != kSplit) {
    for (int r = 0; r < kRows; r++) {
      const float x = params[r * n + g];
      po[r * n_out + o] = x;
      if (outs == 2) po[r * n_out + o + 1] = x;
      if (mo) {
        mo[r * n_out + o] = m[r * n + g];
        vo[r * n_out + o] = v[r * n + g];
        if (outs == 2) {
          mo[r * n_out + o + 1] = 0.f;
          vo[r * n_out + o + 1] = 0.f;
        }
      }
    }
  } else {
    Static s;
    load_static(params, n, g, s);
    float R[3][3], S[3];
    rotation_scale(s.Sc, R, S);
    for (int c = 0; c < 2; c++) {
      const int64_t col = o + c;
      for (int r = 0; r < kRows; r++) {
        float x = params[r * n + g];
        if (r >= kRowMuP && r < kRowMuP + 3) {
          // mu_p + R (S * z)
          const int i = r - kRowMuP;
          float acc = 0.f;
#pragma unroll
          for (int j = 0; j < 3; j++) acc += R[i][j] * S[j] * noise[((int64_t)c * 3 + j) * n + g];
          x += acc;
        } else if (r == kRowL + 0 || r == kRowL + 2 || r == kRowL + 5) {
          x -= logf(kSplitScale);  // exp(raw) / 1.6
        } else if (r == kRowL + 1 || r == kRowL + 3 || r == kRowL + 4) {
          const float l = tanhf(0.5f * x) / kSplitScale;  // (2 sigmoid(raw) - 1) / 1.6
          x = logf((1.f + l) / (1.f - l));
        }
        po[r * n_out + col] = x;
        if (mo) {
          mo[r * n_out + col] = 0.f;
          vo[r * n_out + col] = 0.f;
        }
      }
    }
  }
  if (lo)
    for (int c = 0; c < outs; c++) lo[o + c] = lam[g];
}

}  // namespace

void launch_decompose(const float* params, int64_t n, float* R, float* S, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_decompose, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, params, n, R, S);
}

void launch_density_plan(const float* params, int64_t n, const float* stats, const sixdgs_density_settings& d,
                         uint8_t* dec, uint32_t* cnt, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_density_plan, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, params, n,
                     stats, d, dec, cnt);
}

void launch_density_apply(const float* params, const float* m, const float* v, const float* lam, int64_t n,
                          const float* noise, const uint8_t* dec, const uint32_t* off, float* po, float* mo,
                          float* vo, float* lo, int64_t n_out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_density_apply, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, params, m, v,
                     lam, n, noise, dec, off, po, mo, vo, lo, n_out);
}

}  // namespace sixdgs
