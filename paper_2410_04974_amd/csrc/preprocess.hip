// Per-Gaussian stages of the renderer on gfx950: the slice of every 6D Gaussian
// into its view-conditioned 3D Gaussian, SH colour and EWA projection (forward),
// and the chain rule from screen-space gradients back to the 76 raw parameters
// (backward).  One thread per Gaussian, all cameras of the call in registers, so
// the 304 bytes of parameters are read from HBM once per call in coalesced rows.
#include "internal.h"
#include "slice.h"

namespace sixdgs {
namespace {

// The directional-opacity strength of Gaussian g (Sec. 4.2): the setting, or a
// learnable per-Gaussian sigmoid(raw) (trained over an iteration window, Sec. 5.1).
__device__ __forceinline__ float gaussian_lambda(const DevSettings& ds, int64_t g) {
  return ds.lambda_raw ? sigmoidf(ds.lambda_raw[g]) : ds.lambda_opa;
}


// Real SH basis of degree 3 at unit (x, y, z), textbook normalisation, no
// Condon-Shortley phase (Sec. 4.2 colour).
__device__ __forceinline__ void sh_basis(float x, float y, float z, float Y[16]) {
  const float k0 = 0.282094791773878f, k1 = 0.488602511902920f, k2a = 1.092548430592079f,
              k2b = 0.315391565252520f, k2c = 0.546274215296040f, k3a = 0.590043589926644f,
              k3b = 2.890611442640554f, k3c = 0.457045799464466f, k3d = 0.373176332590115f,
              k3e = 1.445305721320277f;
  float xx = x * x, yy = y * y, zz = z * z;
  Y[0] = k0;
  Y[1] = k1 * y;
  Y[2] = k1 * z;
  Y[3] = k1 * x;
  Y[4] = k2a * x * y;
  Y[5] = k2a * y * z;
  Y[6] = k2b * (3.f * zz - 1.f);
  Y[7] = k2a * x * z;
  Y[8] = k2c * (xx - yy);
  Y[9] = k3a * y * (3.f * xx - yy);
  Y[10] = k3b * x * y * z;
  Y[11] = k3c * y * (5.f * zz - 1.f);
  Y[12] = k3d * z * (5.f * zz - 3.f);
  Y[13] = k3c * x * (5.f * zz - 1.f);
  Y[14] = k3e * z * (xx - yy);
  Y[15] = k3a * x * (xx - 3.f * yy);
}

// Gradient of sum_k w_k Y_k w.r.t. (x, y, z), the basis taken as the
// polynomials written in sh_basis.
__device__ __forceinline__ void sh_basis_vjp(float x, float y, float z, const float w[16], float g[3]) {
  const float k1 = 0.488602511902920f, k2a = 1.092548430592079f, k2b = 0.315391565252520f,
              k2c = 0.546274215296040f, k3a = 0.590043589926644f, k3b = 2.890611442640554f,
              k3c = 0.457045799464466f, k3d = 0.373176332590115f, k3e = 1.445305721320277f;
  float xx = x * x, yy = y * y, zz = z * z;
  float gx = k1 * w[3] + k2a * (y * w[4] + z * w[7]) + 2.f * k2c * x * w[8] + 6.f * k3a * x * y * w[9] +
             k3b * y * z * w[10] + k3c * (5.f * zz - 1.f) * w[13] + 2.f * k3e * x * z * w[14] +
             3.f * k3a * (xx - yy) * w[15];
  float gy = k1 * w[1] + k2a * (x * w[4] + z * w[5]) - 2.f * k2c * y * w[8] + 3.f * k3a * (xx - yy) * w[9] +
             k3b * x * z * w[10] + k3c * (5.f * zz - 1.f) * w[11] - 2.f * k3e * y * z * w[14] -
             6.f * k3a * x * y * w[15];
  float gz = k1 * w[2] + k2a * (y * w[5] + x * w[7]) + 6.f * k2b * z * w[6] + k3b * x * y * w[10] +
             10.f * k3c * y * z * w[11] + k3d * (15.f * zz - 3.f) * w[12] + 10.f * k3c * x * z * w[13] +
             k3e * (xx - yy) * w[14];
  g[0] = gx;
  g[1] = gy;
  g[2] = gz;
}

// Everything about one Gaussian in one view that both directions need.
struct ViewState {
  float d[3], nd;     // slice direction and |mu_p - C|
  float x[3], Ax[3];  // d - mu_d, A x
  float mu_c[3];
  float D, f, ac;
  float sdir[3], ns;  // SH direction and |mu_c - C|
  float p[3];
  bool clx, cly;
  float xt, yt;
  float T[2][3];
  float cov[3];  // xx, xy, yy
  float Q[3];
};

// Slice for the view (Sec. 3.2 eq:mu, Sec. 4.2 eq:pdfv2), camera transform and
// EWA projection with the 3DGS guard and dilation.  Returns false when culled.
// The slice at camera centre C (Sec. 3.2): view direction d = (mu_p - C)/|mu_p - C|,
// its offset x = d - mu_d from the direction mean, conditional mean mu_c = mu_p + K x.
template <bool FAST = false>
__device__ __forceinline__ void slice_mean(const Static& s, const ViewDesc& vd, float d[3], float& nd, float x[3],
                                           float mu_c[3]) {
  float nd2 = 0.f;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    d[k] = s.mu_p[k] - vd.C[k];
    nd2 += d[k] * d[k];
  }
  using M = SliceMath<FAST>;
  nd = M::sqrt(nd2);
#pragma unroll
  for (int k = 0; k < 3; k++) {
    d[k] = M::div(d[k], nd);
    x[k] = d[k] - s.mu_d[k];
  }
#pragma unroll
  for (int r = 0; r < 3; r++) mu_c[r] = s.mu_p[r] + (s.K[r][0] * x[0] + s.K[r][1] * x[1] + s.K[r][2] * x[2]);
}

// The SH evaluation direction (mu_c - C)/|mu_c - C| (Sec. 4.2) and the distance.
template <bool FAST = false>
__device__ __forceinline__ void sh_direction(const float mu_c[3], const ViewDesc& vd, float sdir[3], float& ns) {
  float ns2 = 0.f;
#pragma unroll
  for (int k = 0; k < 3; k++) {
    sdir[k] = mu_c[k] - vd.C[k];
    ns2 += sdir[k] * sdir[k];
  }
  using M = SliceMath<FAST>;
  ns = M::sqrt(ns2);
#pragma unroll
  for (int k = 0; k < 3; k++) sdir[k] = M::div(sdir[k], ns);
}

template <bool FAST = false>
__device__ __forceinline__ bool view_state(const Static& s, const ViewDesc& vd, float lambda, float z_near,
                                           ViewState& w) {
  using M = SliceMath<FAST>;
  slice_mean<FAST>(s, vd, w.d, w.nd, w.x, w.mu_c);
#pragma unroll
  for (int r = 0; r < 3; r++) w.Ax[r] = s.A[r][0] * w.x[0] + s.A[r][1] * w.x[1] + s.A[r][2] * w.x[2];
  w.D = w.x[0] * w.Ax[0] + w.x[1] * w.Ax[1] + w.x[2] * w.Ax[2];
  w.f = M::exp(-lambda * w.D);
  w.ac = s.alpha * w.f;
  sh_direction<FAST>(w.mu_c, vd, w.sdir, w.ns);
#pragma unroll
  for (int r = 0; r < 3; r++)
    w.p[r] = vd.R[3 * r] * w.mu_c[0] + vd.R[3 * r + 1] * w.mu_c[1] + vd.R[3 * r + 2] * w.mu_c[2] + vd.t[r];
  if (!(w.p[2] > z_near)) return false;
  const float z = w.p[2];
  const float rx = M::div(w.p[0], z), ry = M::div(w.p[1], z);
  w.clx = (rx < -vd.limx) || (rx > vd.limx);
  w.cly = (ry < -vd.limy) || (ry > vd.limy);
  w.xt = fminf(vd.limx, fmaxf(-vd.limx, rx));
  w.yt = fminf(vd.limy, fmaxf(-vd.limy, ry));
  const float j00 = M::div(vd.fx, z), j02 = M::div(-vd.fx * w.xt, z), j11 = M::div(vd.fy, z),
              j12 = M::div(-vd.fy * w.yt, z);
#pragma unroll
  for (int c = 0; c < 3; c++) {
    w.T[0][c] = j00 * vd.R[c] + j02 * vd.R[6 + c];
    w.T[1][c] = j11 * vd.R[3 + c] + j12 * vd.R[6 + c];
  }
  float TS[2][3];
#pragma unroll
  for (int r = 0; r < 2; r++)
#pragma unroll
    for (int c = 0; c < 3; c++) TS[r][c] = w.T[r][0] * s.Sc[0][c] + w.T[r][1] * s.Sc[1][c] + w.T[r][2] * s.Sc[2][c];
  w.cov[0] = TS[0][0] * w.T[0][0] + TS[0][1] * w.T[0][1] + TS[0][2] * w.T[0][2] + kDilation;
  w.cov[1] = TS[0][0] * w.T[1][0] + TS[0][1] * w.T[1][1] + TS[0][2] * w.T[1][2];
  w.cov[2] = TS[1][0] * w.T[1][0] + TS[1][1] * w.T[1][1] + TS[1][2] * w.T[1][2] + kDilation;
  const float det = w.cov[0] * w.cov[2] - w.cov[1] * w.cov[1];
  if (!(det > 0.f)) return false;
  const float idet = M::div(1.0f, det);
  w.Q[0] = w.cov[2] * idet;
  w.Q[1] = -w.cov[1] * idet;
  w.Q[2] = w.cov[0] * idet;
  return true;
}

template <bool CACHED>
__global__ void __launch_bounds__(kBlock) k_preprocess(const float* __restrict__ params,
                                                       const float* __restrict__ cache, int64_t n, ViewTable vt,
                                                       DevSettings ds, Rec* __restrict__ rec,
                                                       uint32_t* __restrict__ tiles, float* __restrict__ depth,
                                                       BinPrep bp) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  bin_prep_at(bp, g);
  if (g >= n) return;
  Static s;
  if constexpr (CACHED)
    load_cached(params, cache, n, g, s);
  else
    load_static(params, n, g, s);
  // the colour coefficients, issued with the rest of the parameter loads so
  // their latency overlaps the slice (the RGB colour uses the first three)
  float beta[16][3];
#pragma unroll
  for (int k = 0; k < 16; k++)
#pragma unroll
    for (int c = 0; c < 3; c++) beta[k][c] = row_ld(params, kRowSH + 3 * k + c, n, g);
  const float lam = gaussian_lambda(ds, g);
  for (int vi = 0; vi < vt.nview; vi++) {
    const ViewDesc& vd = vt.v[vi];
    const int64_t e = (int64_t)vi * n + g;
    ViewState w;
    uint32_t count = 0;
    if (view_state(s, vd, lam, ds.z_near, w) && w.ac * 255.0f >= 1.0f) {
      const float qmax = 2.0f * logf(255.0f * w.ac);
      const float ex = sqrtf(qmax * w.cov[0]);
      const float ey = sqrtf(qmax * w.cov[2]);
      const float u = vd.fx * w.p[0] / w.p[2] + vd.cx;
      const float v = vd.fy * w.p[1] / w.p[2] + vd.cy;
      int x0, y0, x1, y1;
      tile_rect(u, v, ex, ey, vt.tile_shift_x, vt.tile_shift_y, vd.ntx, vd.nty, x0, y0, x1, y1);
      count = (uint32_t)((x1 - x0) * (y1 - y0));
      if (count > 0) {
        float col[3];
        if (ds.rgb_color) {
          // No-SH colour: sigmoid of the per-Gaussian RGB held in the degree-0 rows
#pragma unroll
          for (int c = 0; c < 3; c++) col[c] = sigmoidf(beta[0][c]);
        } else {
          float Y[16];
          sh_basis(w.sdir[0], w.sdir[1], w.sdir[2], Y);
#pragma unroll
          for (int c = 0; c < 3; c++) {
            float acc = 0.f;
#pragma unroll
            for (int k = 0; k < 16; k++) acc += beta[k][c] * Y[k];
            col[c] = sigmoidf(acc);
          }
        }
        Rec r;
        r.a = make_float4(u, v, w.Q[0], w.Q[1]);
        r.b = make_float4(w.Q[2], w.ac, ex, ey);
        r.c = make_float4(col[0], col[1], col[2], w.p[2]);
        rec[e] = r;
        depth[e] = w.p[2];  // also on its own, for the integer stage's coalesced reads
      }
    }
    tiles[e] = count;
  }
}

// The inference cache: the direction-independent part of the slice (Alg. 1
// caption), computed once so that render-only calls skip it.
__global__ void __launch_bounds__(kBlock) k_build_cache(const float* __restrict__ params, int64_t n,
                                                        float* __restrict__ cache) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= n) return;
  Static s;
  load_static(params, n, g, s);
  const float v[kCacheRows] = {s.Sc[0][0], s.Sc[0][1], s.Sc[0][2], s.Sc[1][1], s.Sc[1][2], s.Sc[2][2],
                               s.K[0][0],  s.K[0][1],  s.K[0][2],  s.K[1][0],  s.K[1][1],  s.K[1][2],
                               s.K[2][0],  s.K[2][1],  s.K[2][2],  s.A[0][0],  s.A[0][1],  s.A[0][2],
                               s.A[1][1],  s.A[1][2],  s.A[2][2],  s.alpha};
#pragma unroll
  for (int k = 0; k < kCacheRows; k++) row_st(cache, k, n, g, v[k]);
}

// ------------------------------------------------------------------ backward
// Where the per-parameter gradient goes: to a gradient buffer, or straight into
// an Adam step on the parameters (the gradient then never reaches memory).
struct GradToBuffer {
  static constexpr bool kAccumulates = false;
  static constexpr bool kColourOut = false;
  float* grad;
  __device__ void put(int row, int64_t n, int64_t g, float v) const { row_st(grad, row, n, g, v); }
  __device__ void add(int, float) const {}
};
// ... or to this wavefront's rows in LDS ([kRows][64]), for an Adam step
// that streams the parameter and moment rows afterwards.  Rows there can also
// be summed in place (the colour rows over the views of a several-view call:
// 48 fewer registers than accumulators).
struct GradToLDS {
  static constexpr bool kAccumulates = true;
  static constexpr bool kColourOut = false;
  float* rows;
  __device__ void put(int row, int64_t, int64_t, float v) const { rows[row * 64 + (threadIdx.x & 63)] = v; }
  __device__ void add(int row, float v) const { rows[row * 64 + (threadIdx.x & 63)] += v; }
};
// ... or, with one view, only the 28 rows that are not colour coefficients to
// LDS ([kGeomRows][64]: rows 0..26, then the opacity): the 48 colour rows are
// the products of three channel terms and the 16 SH basis values of the view
// direction, handed back (kColourOut) for the Adam step to form row by row.
constexpr int kGeomRows = kRowSH + 1;
struct GeomToLDS {
  static constexpr bool kAccumulates = false;
  static constexpr bool kColourOut = true;
  float* rows;
  __device__ void put(int row, int64_t, int64_t, float v) const {
    if (row < kRowSH) rows[row * 64 + (threadIdx.x & 63)] = v;
    else if (row == kRowOpa) rows[kRowSH * 64 + (threadIdx.x & 63)] = v;
  }
  __device__ void add(int, float) const {}
  // the 48 colour coefficients the chain rule read, kept for the update
  // (rows kGeomRows ..): the Adam step does not read them again from memory
  __device__ void keep(int i, float v) const { rows[(kGeomRows + i) * 64 + (threadIdx.x & 63)] = v; }
};

// The chain rule from the screen-space gradients of Gaussian g back to its 76
// parameters, summed over the views, handed to the sink row by row.  params
// may be updated in place after this returns (by the fused Adam step), so it
// is not declared __restrict__.
// With a kColourOut sink (one view), colour_out receives the three channel
// terms of the colour gradient and the view direction (zeros for an invisible
// lane) instead of the 48 colour rows going to the sink.
template <bool ONE_VIEW, class Sink>
__device__ __forceinline__ void bwd_gaussian(const float* params, int64_t n, int64_t g, const ViewTable& vt,
                                             const DevSettings& ds, const uint32_t* __restrict__ tiles,
                                             const float* __restrict__ g2d, const Sink& sink,
                                             float* __restrict__ densify, float* colour_out = nullptr) {
  static_assert(ONE_VIEW || !Sink::kColourOut, "the colour terms are handed back for one view only");
  using M = SliceMath<true>;  // the backward differentiates at recomputed values
  if (g >= n) return;
  // Every load that depends on no other is issued before the first branch, so
  // a wavefront waits for memory once: the 76 parameter rows and the first
  // view's tile count and screen-space gradients.
  RawGeom raw;
  load_raw_geom(params, n, g, raw);
  // the colour coefficients: with one view up front with the rest; with
  // several, read per view (from the cache after the first) rather than held
  // in 48 registers through the whole view loop
  float beta[ONE_VIEW ? 16 : 1][3];
  if constexpr (ONE_VIEW) {
#pragma unroll
    for (int k = 0; k < 16; k++)
#pragma unroll
      for (int c = 0; c < 3; c++) beta[k][c] = row_ld(params, kRowSH + 3 * k + c, n, g);
  }
  auto coef = [&](int k, int c) {
    if constexpr (ONE_VIEW) return beta[k][c];
    else return row_ld(params, kRowSH + 3 * k + c, n, g);
  };
  const uint32_t tiles0 = row_ld(tiles, 0, n, g);
  float gp0[kG2D];
#pragma unroll
  for (int k = 0; k < kG2D; k++) gp0[k] = g2d[g * kG2D + k];
  bool any = tiles0 > 0;
  for (int vi = 1; vi < vt.nview; vi++) any |= row_ld(tiles, vi, n, g) > 0;
  // Only a wavefront with no visible Gaussian leaves early: its lanes store
  // together.  Otherwise invisible lanes run along with zero accumulators
  // (every view is skipped), so each gradient row is written by one store
  // of the whole wavefront instead of two partial ones.
  auto keep_coefs = [&]() {
    if constexpr (Sink::kColourOut) {
#pragma unroll
      for (int k = 0; k < 16; k++)
#pragma unroll
        for (int c = 0; c < 3; c++) sink.keep(3 * k + c, beta[k][c]);
    }
  };
  if (__ballot(any) == 0) {
    for (int r = 0; r < kRows; r++) sink.put(r, n, g, 0.f);
    keep_coefs();
    if (ds.lambda_raw && ds.grad_lambda) ds.grad_lambda[g] = 0.f;
    return;
  }
  Static s;
  static_from_raw<true>(raw, s);
  keep_coefs();

  // an invisible lane's rows are exact zeros whatever its parameters
  auto put = [&](int row, float v) { sink.put(row, n, g, any ? v : 0.f); };
  // accumulators summed over views; with one view the colour gradient is
  // formed at the end from that view's three channel terms and SH direction
  // (or, when the sink sums rows in place, in the sink's colour rows)
  constexpr bool kInSink = !ONE_VIEW && Sink::kAccumulates;
  float g_beta[ONE_VIEW || kInSink ? 1 : 16][3];
#pragma unroll
  for (int k = 0; k < (ONE_VIEW || kInSink ? 1 : 16); k++)
#pragma unroll
    for (int c = 0; c < 3; c++) g_beta[k][c] = 0.f;
  if constexpr (kInSink) {
#pragma unroll
    for (int r = kRowSH; r < kRowSH + 48; r++) sink.put(r, n, g, 0.f);
  }
  float dsc1[3] = {0.f, 0.f, 0.f}, sdir1[3] = {0.f, 0.f, 1.f};
  float g_mup[3] = {0, 0, 0}, g_mud[3] = {0, 0, 0}, g_alpha = 0.f;
  float g_Sc[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};   // dL/dSigma_cond (symmetric)
  float g_Spd_mu[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // mu_cond part of dL/dSigma_pd
  float g_A_mu[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};    // mu_cond and D parts of dL/dA
  float dens_norm = 0.f, dens_cnt = 0.f;
  const float lam = gaussian_lambda(ds, g);
  float g_lam = 0.f;  // dL/dlambda

  for (int vi = 0; vi < vt.nview; vi++) {
    const ViewDesc& vd = vt.v[vi];
    const int64_t e = (int64_t)vi * n + g;
    if ((vi == 0 ? tiles0 : row_ld(tiles, vi, n, g)) == 0) continue;
    float gp[kG2D];
#pragma unroll
    for (int k = 0; k < kG2D; k++) gp[k] = vi == 0 ? gp0[k] : g2d[e * kG2D + k];
    ViewState w;
    view_state<true>(s, vd, lam, ds.z_near, w);
    // colour first (Sec. 4.2): its share of dL/dmu_c, after which the 48
    // coefficients are dead while the geometry's chain rule runs
    float gmu[3] = {0.f, 0.f, 0.f};
    float dsc[3];
    if (ds.rgb_color) {
      // No-SH colour: rgb = sigmoid(c), no dependence on the viewing direction
#pragma unroll
      for (int c = 0; c < 3; c++) {
        const float col = M::sigmoid(coef(0, c));
        dsc[c] = gp[6 + c] * col * (1.f - col);
        if constexpr (kInSink) sink.add(kRowSH + c, dsc[c]);
        else if constexpr (!ONE_VIEW) g_beta[0][c] += dsc[c];
      }
    } else {
      // SH colour: rgb = sigmoid(sum beta Y(s)), s = (mu_c - C)/|mu_c - C|
      float Y[16];
      sh_basis(w.sdir[0], w.sdir[1], w.sdir[2], Y);
      float wsum[16];
#pragma unroll
      for (int k = 0; k < 16; k++) wsum[k] = 0.f;
#pragma unroll
      for (int c = 0; c < 3; c++) {
        float bc[16];
#pragma unroll
        for (int k = 0; k < 16; k++) bc[k] = coef(k, c);
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < 16; k++) acc += bc[k] * Y[k];
        const float col = M::sigmoid(acc);
        dsc[c] = gp[6 + c] * col * (1.f - col);
#pragma unroll
        for (int k = 0; k < 16; k++) {
          if constexpr (kInSink) sink.add(kRowSH + 3 * k + c, dsc[c] * Y[k]);
          else if constexpr (!ONE_VIEW) g_beta[k][c] += dsc[c] * Y[k];
          wsum[k] += dsc[c] * bc[k];
        }
      }
      float gs[3];
      sh_basis_vjp(w.sdir[0], w.sdir[1], w.sdir[2], wsum, gs);
      const float sdot = w.sdir[0] * gs[0] + w.sdir[1] * gs[1] + w.sdir[2] * gs[2];
#pragma unroll
      for (int k = 0; k < 3; k++) gmu[k] = M::div(gs[k] - w.sdir[k] * sdot, w.ns);
    }
    if constexpr (ONE_VIEW) {
#pragma unroll
      for (int c = 0; c < 3; c++) {
        dsc1[c] = dsc[c];
        sdir1[c] = w.sdir[c];
      }
    }
    const float gu = gp[0], gv = gp[1], gqxx = gp[2], gqxy = gp[3], gqyy = gp[4], gac = gp[5];
    const float z = w.p[2], fx = vd.fx, fy = vd.fy;
    dens_norm += M::sqrt((gu * 0.5f * vd.W) * (gu * 0.5f * vd.W) + (gv * 0.5f * vd.H) * (gv * 0.5f * vd.H));
    dens_cnt += 1.f;
    // conic -> 2D covariance: G_S = -Q G_Q Q
    const float Q00 = w.Q[0], Q01 = w.Q[1], Q11 = w.Q[2];
    const float QG00 = Q00 * gqxx + Q01 * gqxy, QG01 = Q00 * gqxy + Q01 * gqyy;
    const float QG10 = Q01 * gqxx + Q11 * gqxy, QG11 = Q01 * gqxy + Q11 * gqyy;
    const float GS00 = -(QG00 * Q00 + QG01 * Q01);
    const float GS01 = -(QG00 * Q01 + QG01 * Q11);
    const float GS11 = -(QG10 * Q01 + QG11 * Q11);
    const float GS[2][2] = {{GS00, GS01}, {GS01, GS11}};
    // Sigma_2D = T Sigma_c T^T + dil I:  dSigma_c = T^T G_S T,  dT = 2 G_S T Sigma_c
    float GT[2][3];
#pragma unroll
    for (int r = 0; r < 2; r++)
#pragma unroll
      for (int c = 0; c < 3; c++) GT[r][c] = GS[r][0] * w.T[0][c] + GS[r][1] * w.T[1][c];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
      for (int b = 0; b < 3; b++) g_Sc[a][b] += w.T[0][a] * GT[0][b] + w.T[1][a] * GT[1][b];
    float dT[2][3];
#pragma unroll
    for (int r = 0; r < 2; r++)
#pragma unroll
      for (int c = 0; c < 3; c++)
        dT[r][c] = 2.f * (GT[r][0] * s.Sc[0][c] + GT[r][1] * s.Sc[1][c] + GT[r][2] * s.Sc[2][c]);
    // T = J R:  dJ = dT R^T (only the non-zero entries of J matter)
    const float dJ00 = dT[0][0] * vd.R[0] + dT[0][1] * vd.R[1] + dT[0][2] * vd.R[2];
    const float dJ02 = dT[0][0] * vd.R[6] + dT[0][1] * vd.R[7] + dT[0][2] * vd.R[8];
    const float dJ11 = dT[1][0] * vd.R[3] + dT[1][1] * vd.R[4] + dT[1][2] * vd.R[5];
    const float dJ12 = dT[1][0] * vd.R[6] + dT[1][1] * vd.R[7] + dT[1][2] * vd.R[8];
    const float iz = M::div(1.0f, z), iz2 = iz * iz;
    float dp0 = 0.f, dp1 = 0.f, dp2 = -(dJ00 * fx + dJ11 * fy) * iz2;
    if (!w.clx) {
      dp0 += -dJ02 * fx * iz2;
      dp2 += dJ02 * 2.f * fx * w.p[0] * iz2 * iz;
    } else {
      dp2 += dJ02 * fx * w.xt * iz2;
    }
    if (!w.cly) {
      dp1 += -dJ12 * fy * iz2;
      dp2 += dJ12 * 2.f * fy * w.p[1] * iz2 * iz;
    } else {
      dp2 += dJ12 * fy * w.yt * iz2;
    }
    // u = fx px/pz + cx, v = fy py/pz + cy
    dp0 += gu * fx * iz;
    dp1 += gv * fy * iz;
    dp2 -= (gu * fx * w.p[0] + gv * fy * w.p[1]) * iz2;
    // p = R mu_c + t
#pragma unroll
    for (int k = 0; k < 3; k++) gmu[k] += vd.R[k] * dp0 + vd.R[3 + k] * dp1 + vd.R[6 + k] * dp2;
    // slice (Sec. 3.2): mu_c = mu_p + K x, D = x^T A x, alpha_c = alpha exp(-lambda D)
    const float dD = -lam * w.ac * gac;
    g_lam -= w.D * w.ac * gac;  // d alpha_c / d lambda = -D alpha_c
    float gx[3];
#pragma unroll
    for (int k = 0; k < 3; k++) gx[k] = s.K[0][k] * gmu[0] + s.K[1][k] * gmu[1] + s.K[2][k] * gmu[2] + 2.f * dD * w.Ax[k];
    const float ddot = w.d[0] * gx[0] + w.d[1] * gx[1] + w.d[2] * gx[2];
#pragma unroll
    for (int k = 0; k < 3; k++) {
      g_mud[k] -= gx[k];
      g_mup[k] += gmu[k] + M::div(gx[k] - w.d[k] * ddot, w.nd);
    }
    g_alpha += gac * w.f;
    float st_g[3];  // Sigma_pd^T gmu
#pragma unroll
    for (int a = 0; a < 3; a++) st_g[a] = s.Spd[0][a] * gmu[0] + s.Spd[1][a] * gmu[1] + s.Spd[2][a] * gmu[2];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
      for (int b = 0; b < 3; b++) {
        g_Spd_mu[a][b] += gmu[a] * w.Ax[b];
        g_A_mu[a][b] += 0.5f * (st_g[a] * w.x[b] + st_g[b] * w.x[a]) + dD * w.x[a] * w.x[b];
      }
  }
  // direction-independent tail: Sigma_cond = Sigma_p - Sigma_pd A Sigma_pd^T
  float GSc[3][3];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) GSc[a][b] = 0.5f * (g_Sc[a][b] + g_Sc[b][a]);
  float GcSpd[3][3];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) GcSpd[a][b] = GSc[a][0] * s.Spd[0][b] + GSc[a][1] * s.Spd[1][b] + GSc[a][2] * s.Spd[2][b];
  float GSpd[3][3], GA[3][3];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) {
      GSpd[a][b] = g_Spd_mu[a][b] - 2.f * (GcSpd[a][0] * s.A[0][b] + GcSpd[a][1] * s.A[1][b] + GcSpd[a][2] * s.A[2][b]);
      GA[a][b] = g_A_mu[a][b] - (s.Spd[0][a] * GcSpd[0][b] + s.Spd[1][a] * GcSpd[1][b] + s.Spd[2][a] * GcSpd[2][b]);
    }
  // A = Sigma_d^-1:  dSigma_d = -A dA A
  float AG[3][3], GSd[3][3];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) AG[a][b] = s.A[a][0] * GA[0][b] + s.A[a][1] * GA[1][b] + s.A[a][2] * GA[2][b];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) GSd[a][b] = -(AG[a][0] * s.A[0][b] + AG[a][1] * s.A[1][b] + AG[a][2] * s.A[2][b]);
  // Sigma = L L^T:  dL = lower(2 G6 L), G6 = [[G_p, G_pd/2], [G_pd^T/2, G_d]]
  float G6[6][6];
#pragma unroll
  for (int a = 0; a < 3; a++)
#pragma unroll
    for (int b = 0; b < 3; b++) {
      G6[a][b] = GSc[a][b];
      G6[3 + a][3 + b] = 0.5f * (GSd[a][b] + GSd[b][a]);
      G6[a][3 + b] = 0.5f * GSpd[a][b];
      G6[3 + b][a] = 0.5f * GSpd[a][b];
    }
  // the factor: kept from the start with one view; with several, formed
  // again from its rows rather than held through the view loop
  float Lt[ONE_VIEW ? 1 : 21];
  if constexpr (!ONE_VIEW) load_cholesky<true>(params, n, g, Lt);
  const float* L = ONE_VIEW ? s.L : Lt;
#pragma unroll
  for (int i = 0; i < 6; i++)
#pragma unroll
    for (int j = 0; j <= i; j++) {
      float acc = 0.f;
#pragma unroll
      for (int k = j; k < 6; k++) acc += G6[i][k] * Lget(L, k, j);
      const float gl = 2.f * acc;
      const float Lij = L[tri(i, j)];
      // exp on the diagonal; 2 sigmoid(r) - 1 elsewhere, whose derivative is (1 - L)(1 + L)/2
      const float graw = (i == j) ? gl * Lij : gl * 0.5f * (1.f - Lij) * (1.f + Lij);
      put(kRowL + tri(i, j), graw);
    }
#pragma unroll
  for (int k = 0; k < 3; k++) {
    put(kRowMuP + k, g_mup[k]);
    put(kRowMuD + k, g_mud[k]);
  }
  if constexpr (Sink::kColourOut) {
#pragma unroll
    for (int c = 0; c < 3; c++) {
      colour_out[c] = any ? dsc1[c] : 0.f;
      colour_out[3 + c] = sdir1[c];
    }
  } else if constexpr (ONE_VIEW) {
    if (ds.rgb_color) {
#pragma unroll
      for (int c = 0; c < 3; c++) put(kRowSH + c, dsc1[c]);
#pragma unroll
      for (int r = kRowSH + 3; r < kRowSH + 48; r++) put(r, 0.f);
    } else {
      float Y[16];
      sh_basis(sdir1[0], sdir1[1], sdir1[2], Y);
#pragma unroll
      for (int k = 0; k < 16; k++)
#pragma unroll
        for (int c = 0; c < 3; c++) put(kRowSH + 3 * k + c, dsc1[c] * Y[k]);
    }
  } else if constexpr (!kInSink) {
#pragma unroll
    for (int k = 0; k < 16; k++)
#pragma unroll
      for (int c = 0; c < 3; c++) put(kRowSH + 3 * k + c, g_beta[k][c]);
  }
  put(kRowOpa, g_alpha * s.alpha * (1.f - s.alpha));
  if (densify) {
    densify[g] += dens_norm;
    densify[n + g] += dens_cnt;
  }
  if (ds.lambda_raw && ds.grad_lambda) ds.grad_lambda[g] = any ? g_lam * lam * (1.f - lam) : 0.f;
}

template <bool ONE_VIEW, class Sink>
__global__ void __launch_bounds__(kBlock) k_preprocess_bwd(const float* params, int64_t n, ViewTable vt,
                                                           DevSettings ds, const uint32_t* __restrict__ tiles,
                                                           const float* __restrict__ g2d, Sink sink,
                                                           float* __restrict__ densify) {
  bwd_gaussian<ONE_VIEW>(params, n, (int64_t)blockIdx.x * kBlock + threadIdx.x, vt, ds, tiles, g2d, sink, densify);
}

// The chain rule with the gradient rows kept in LDS, then one Adam step over
// this wavefront's 64 Gaussians: rows are streamed in groups of 19 (the
// chain rule's registers are free by then), so each lane has 57 loads in
// flight instead of the three of a per-row update.  With step_dev the step is
// *step_dev + 1; with `done` as well, the last workgroup to finish (counted
// in *done, zero before the launch and again after it) moves the counter on,
// once every workgroup has read it.
constexpr int kAdamGroup = 19;  // kRows = 4 groups
template <bool ONE_VIEW>
__global__ void __launch_bounds__(kBlock) k_preprocess_bwd_adam(float* params, int64_t n, ViewTable vt,
                                                                DevSettings ds, const uint32_t* __restrict__ tiles,
                                                                const float* __restrict__ g2d,
                                                                float* __restrict__ m, float* __restrict__ v,
                                                                AdamArgs a, int32_t* step_dev, uint32_t* done,
                                                                float* __restrict__ densify) {
  constexpr int kLdsRows = ONE_VIEW ? kGeomRows + 48 : kRows;
  __shared__ float s_g[kBlock / 64][kLdsRows * 64];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  // one view: the colour rows' gradients are formed during the update from
  // the channel terms and the SH basis of the view direction, so the LDS
  // holds 28 gradient rows per lane, and the 48 colour coefficients the chain
  // rule read, which the update then takes from there instead of memory
  float col[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 1.f};
  if constexpr (ONE_VIEW)
    bwd_gaussian<true>(params, n, g, vt, ds, tiles, g2d, GeomToLDS{s_g[wv]}, densify, col);
  else
    bwd_gaussian<false>(params, n, g, vt, ds, tiles, g2d, GradToLDS{s_g[wv]}, densify);
  if (step_dev) adam_device_step(a, *step_dev);
  // each lane reads back only what it wrote: ordering the wavefront's own LDS
  // accesses is enough
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (g < n) {
    float Y[16];  // colour row 3k + c has gradient col[c] Y[k] (the No-SH colour: Y = (1, 0, ...))
    if constexpr (ONE_VIEW) {
      if (ds.rgb_color) {
#pragma unroll
        for (int k = 0; k < 16; k++) Y[k] = k == 0 ? 1.f : 0.f;
      } else {
        sh_basis(col[3], col[4], col[5], Y);
      }
    }
    auto grad_of = [&](int r) {
      if constexpr (ONE_VIEW) {
        if (r >= kRowSH && r < kRowOpa) return col[(r - kRowSH) % 3] * Y[(r - kRowSH) / 3];
        return s_g[wv][(r == kRowOpa ? kRowSH : r) * 64 + lane];
      } else {
        return s_g[wv][r * 64 + lane];
      }
    };
    static_assert(kRows % kAdamGroup == 0, "row groups");
#pragma unroll
    for (int r0 = 0; r0 < kRows; r0 += kAdamGroup) {
      float pp[kAdamGroup], mm[kAdamGroup], vv[kAdamGroup];
#pragma unroll
      for (int j = 0; j < kAdamGroup; j++) {
        const int r = r0 + j;
        if (ONE_VIEW && r >= kRowSH && r < kRowOpa)
          pp[j] = s_g[wv][(kGeomRows + r - kRowSH) * 64 + lane];  // kept by the chain rule
        else
          pp[j] = row_ld(params, r, n, g);
        // the moments are touched once per step: streamed past the caches,
        // which keep the parameters for the next step's preprocess instead
        mm[j] = __builtin_nontemporal_load(row_ptr(m, r0 + j, n, g));
        vv[j] = __builtin_nontemporal_load(row_ptr(v, r0 + j, n, g));
      }
#pragma unroll
      for (int j = 0; j < kAdamGroup; j++) {
        const int r = r0 + j;
        const int grp = adam_row_group(r);  // selected, not indexed: keeps a.lr out of scratch memory
        const float lr = grp == 0 ? a.lr[0] : grp == 1 ? a.lr[1] : grp == 2 ? a.lr[2] : grp == 3 ? a.lr[3]
                       : grp == 4 ? a.lr[4] : a.lr[5];
        adam_update(pp[j], grad_of(r), mm[j], vv[j], lr, a);
        row_st(params, r, n, g, pp[j]);
        __builtin_nontemporal_store(mm[j], row_ptr(m, r, n, g));
        __builtin_nontemporal_store(vv[j], row_ptr(v, r, n, g));
      }
    }
  }
  if (done) {
    // every thread of this workgroup has used the step count by now
    __syncthreads();
    if (threadIdx.x == 0 && atomicAdd(done, 1u) == gridDim.x - 1) {
      *step_dev += 1;
      *done = 0u;
    }
  }
}

}  // namespace

bool launch_preprocess(const float* params, const float* cache, int64_t n, const ViewTable& vt,
                       const DevSettings& s, Rec* rec, uint32_t* tiles, float* depth, const BinPrep* bp,
                       hipStream_t st) {
  if (n <= 0) return false;
  BinPrep none{};
  const BinPrep& p = bp ? *bp : none;
  const unsigned grid = (unsigned)((std::max<int64_t>(n, p.threads) + kBlock - 1) / kBlock);
  if (cache)
    hipLaunchKernelGGL(k_preprocess<true>, dim3(grid), dim3(kBlock), 0, st, params, cache, n, vt, s, rec, tiles,
                       depth, p);
  else
    hipLaunchKernelGGL(k_preprocess<false>, dim3(grid), dim3(kBlock), 0, st, params, cache, n, vt, s, rec, tiles,
                       depth, p);
  return bp != nullptr;
}

void launch_build_cache(const float* params, int64_t n, float* cache, hipStream_t st) {
  if (n <= 0) return;
  const unsigned grid = (unsigned)((n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_build_cache, dim3(grid), dim3(kBlock), 0, st, params, n, cache);
}

void launch_preprocess_bwd(const float* params, int64_t n, const ViewTable& vt, const DevSettings& s,
                           const uint32_t* tiles, const float* g2d, float* grad, float* densify, hipStream_t st) {
  if (n <= 0) return;
  const unsigned grid = (unsigned)((n + kBlock - 1) / kBlock);
  // one view: the colour gradient needs no accumulators over views
  auto k = vt.nview == 1 ? k_preprocess_bwd<true, GradToBuffer> : k_preprocess_bwd<false, GradToBuffer>;
  hipLaunchKernelGGL(k, dim3(grid), dim3(kBlock), 0, st, params, n, vt, s, tiles, g2d, GradToBuffer{grad}, densify);
}

void launch_preprocess_bwd_adam(float* params, int64_t n, const ViewTable& vt, const DevSettings& s,
                                const uint32_t* tiles, const float* g2d, float* m, float* v, const AdamArgs& a,
                                int32_t* step_dev, uint32_t* done, float* densify, hipStream_t st) {
  if (n <= 0) return;
  const unsigned grid = (unsigned)((n + kBlock - 1) / kBlock);
  auto k = vt.nview == 1 ? k_preprocess_bwd_adam<true> : k_preprocess_bwd_adam<false>;
  hipLaunchKernelGGL(k, dim3(grid), dim3(kBlock), 0, st, params, n, vt, s, tiles, g2d, m, v, a,
                     step_dev, step_dev ? done : nullptr, densify);
}

}  // namespace sixdgs
