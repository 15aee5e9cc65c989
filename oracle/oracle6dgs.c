/*
 * oracle6dgs.c -- plain, slow FP64 CPU reference renderer for view-conditioned
 * 6D Gaussians.  TEST INFRASTRUCTURE ONLY: it exists so that tests, the smoke
 * check and the benchmark's CPU-baseline leg can check and time the GPU path.
 * It shares no code, header, table or constant with the GPU library and must
 * never be called by the product path.
 *
 * What it computes, step by step, and where each step comes from:
 *   - Cholesky parameterisation Sigma = L L^T, exp on the diagonal, a value in
 *     (-1, 1) off the diagonal, read here as 2*sigmoid(r) - 1 (Sec. 3.1);
 *     opacity alpha = sigmoid(logit) (Sec. 3.1 names an opacity; its activation
 *     is not stated and is read as the sigmoid).
 *   - block partition of Sigma into Sigma_p, Sigma_pd, Sigma_d (Sec. 3.2, eq. 1;
 *     Algorithm 1 steps 1-2).
 *   - conditional mean and Schur-complement covariance (Sec. 3.2, eq:mu and
 *     eq:sigma; Algorithm 1 step 3).
 *   - directional opacity f = exp(-lambda (d-mu_d)^T Sigma_d^-1 (d-mu_d)),
 *     alpha_cond = alpha f, with no factor 1/2 as printed (Sec. 4.2 eq:pdfv2,
 *     Sec. 3.2 eq:alpha).  The view direction d is the unit vector from the
 *     camera centre to mu_p.
 *   - colour = sigmoid of a degree-3 real SH expansion with 48 coefficients
 *     (Sec. 4.2), evaluated at the unit vector from the camera centre to
 *     mu_cond; textbook real SH without the Condon-Shortley phase.  The
 *     No-SH ablation of Sec. 5 (a learnable RGB per Gaussian) is the
 *     color_rgb setting: rgb = sigmoid(c), c in the SH degree-0 rows.
 *   - after the slice the renderer is the 3D Gaussian splatting rasteriser
 *     (Sec. 4.4): EWA projection with the 1.3 Jacobian guard and 0.3 screen
 *     dilation, per-pixel front-to-back compositing with alpha clamped at 0.99,
 *     contributions below 1/255 skipped and the walk stopped before the
 *     transmittance would fall below 1e-4.  Here every alive Gaussian is
 *     evaluated at every pixel, in one global (depth, index) order.
 *   - backward: the analytic derivative of the above, written out by hand
 *     (reverse compositing, then projection, SH, slice, Cholesky, activations).
 *
 * Everything is double precision; compile with -O2 -ffp-contract=off and no
 * fast-math.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define NROWS 76
#define ROW_MU_P 0
#define ROW_MU_D 3
#define ROW_L 6
#define ROW_SH 27
#define ROW_OPA 75

/* Record fields (per Gaussian, per camera), double, row length NREC. */
enum {
  F_ALIVE = 0,
  F_MUC = 1,      /* 3: conditional mean */
  F_SIGC = 4,     /* 6: conditional covariance xx, xy, xz, yy, yz, zz */
  F_ALPHA = 10,   /* base opacity sigmoid(logit) */
  F_F = 11,       /* directional factor f */
  F_D = 12,       /* Mahalanobis distance D */
  F_ALPHAC = 13,  /* alpha_cond */
  F_RGB = 14,     /* 3 */
  F_P = 17,       /* 3: camera-space mean */
  F_DEPTH = 20,
  F_U = 21,
  F_V = 22,
  F_COV2D = 23,   /* 3: xx, xy, yy */
  F_CONIC = 26,   /* 3: xx, xy, yy of the inverse 2D covariance */
  F_EX = 29,
  F_EY = 30,
  F_DIR = 31,     /* 3: slice direction d */
  F_SHDIR = 34,   /* 3: SH direction */
  F_NEARCUT = 37, /* 1: culled by alpha_cond < 1/255 within the alpha margin of the cut;
                     2: depth within the depth margin of z_near (see the decision envelope) */
  NREC = 38
};

typedef struct {
  double R[9];
  double t[3];
  double fx, fy, cx, cy;
  int64_t width, height;
} orc_camera;

typedef struct {
  double lambda_opa;
  double z_near;
  double bg[3];
  double jac_guard;  /* 1.3 */
  double dilation;   /* 0.3 */
  double alpha_max;  /* 0.99 */
  double alpha_min;  /* 1/255 */
  double t_min;      /* 1e-4 */
  /* Float32 error bounds of a renderer that takes the walk's decisions on
   * float32 records (test infrastructure: they feed only the decision
   * envelope below, never the rendered values).  A decision whose outcome can
   * change when the record fields move within these bounds is ambiguous. */
  double m_uv;      /* |u_f32 - u|, |v_f32 - v| in pixels */
  double m_conic;   /* |x^T (Q_f32 - Q) x| <= m_conic x^T Q x: the conic's error in its own metric */
  double m_alpha;   /* relative error of alpha_cond */
  double m_depth;   /* relative error of the depth */
  double m_eval;    /* rounding of ln(alpha) evaluated in float32, relative to its terms' magnitudes */
  double m_trel;    /* relative rounding of one float32 operation of the transmittance update */
  int64_t max_leaves; /* outcome states kept per pixel before giving up (flag UNRESOLVED) */
  /* learnable per-Gaussian lambda (Sec. 4.2, trained over a window of
   * iterations per Sec. 5.1): when lambda_raw is not NULL Gaussian i uses
   * lambda = sigmoid(lambda_raw[i]) instead of lambda_opa, and the backward
   * adds dL/dlambda_raw into grad_lambda (when that is not NULL either) */
  const double *lambda_raw;
  double *grad_lambda;
  /* colour model: 0 = sigmoid of the degree-3 SH expansion (Sec. 4.2); 1 = the
   * No-SH ablation of Sec. 5 (a learnable RGB per Gaussian, as in N-DG), read
   * here as rgb = sigmoid(c) with c held in the three rows of the SH degree-0
   * coefficients; the other 45 SH rows are unused and get zero gradient */
  int64_t color_rgb;
} orc_settings;

static double sigm(double x) { return 1.0 / (1.0 + exp(-x)); }

static double lam_of(const orc_settings *s, int64_t i) {
  return s->lambda_raw ? sigm(s->lambda_raw[i]) : s->lambda_opa;
}

/* ---------------------------------------------------------------- algebra */
static void inv3(const double a[3][3], double out[3][3], double *det_out) {
  /* adjugate over determinant */
  double c00 = a[1][1] * a[2][2] - a[1][2] * a[2][1];
  double c01 = a[1][2] * a[2][0] - a[1][0] * a[2][2];
  double c02 = a[1][0] * a[2][1] - a[1][1] * a[2][0];
  double det = a[0][0] * c00 + a[0][1] * c01 + a[0][2] * c02;
  double id = 1.0 / det;
  out[0][0] = c00 * id;
  out[1][0] = c01 * id;
  out[2][0] = c02 * id;
  out[0][1] = (a[0][2] * a[2][1] - a[0][1] * a[2][2]) * id;
  out[1][1] = (a[0][0] * a[2][2] - a[0][2] * a[2][0]) * id;
  out[2][1] = (a[0][1] * a[2][0] - a[0][0] * a[2][1]) * id;
  out[0][2] = (a[0][1] * a[1][2] - a[0][2] * a[1][1]) * id;
  out[1][2] = (a[0][2] * a[1][0] - a[0][0] * a[1][2]) * id;
  out[2][2] = (a[0][0] * a[1][1] - a[0][1] * a[1][0]) * id;
  if (det_out) *det_out = det;
}

static void mm3(const double a[3][3], const double b[3][3], double o[3][3]) {
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double s = 0;
      for (int k = 0; k < 3; k++) s += a[i][k] * b[k][j];
      o[i][j] = s;
    }
}

static void mm3t(const double a[3][3], const double b[3][3], double o[3][3]) { /* a b^T */
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double s = 0;
      for (int k = 0; k < 3; k++) s += a[i][k] * b[j][k];
      o[i][j] = s;
    }
}

static void mtm3(const double a[3][3], const double b[3][3], double o[3][3]) { /* a^T b */
  for (int i = 0; i < 3; i++)
    for (int j = 0; j < 3; j++) {
      double s = 0;
      for (int k = 0; k < 3; k++) s += a[k][i] * b[k][j];
      o[i][j] = s;
    }
}

/* ------------------------------------------------------------ SH (Sec 4.2) */
/* Normalisation constants of the real spherical harmonics, from their closed
 * forms sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!) times the polynomial factors. */
static double SHK[16];
static int sh_ready = 0;
static void sh_init(void) {
  if (sh_ready) return;
  const double pi = 3.14159265358979323846;
  SHK[0] = 0.5 * sqrt(1.0 / pi);
  SHK[1] = SHK[2] = SHK[3] = sqrt(3.0 / (4.0 * pi));
  SHK[4] = 0.5 * sqrt(15.0 / pi);   /* xy */
  SHK[5] = 0.5 * sqrt(15.0 / pi);   /* yz */
  SHK[6] = 0.25 * sqrt(5.0 / pi);   /* 3z^2-1 */
  SHK[7] = 0.5 * sqrt(15.0 / pi);   /* xz */
  SHK[8] = 0.25 * sqrt(15.0 / pi);  /* x^2-y^2 */
  SHK[9] = 0.25 * sqrt(35.0 / (2.0 * pi));   /* y(3x^2-y^2) */
  SHK[10] = 0.5 * sqrt(105.0 / pi);          /* xyz */
  SHK[11] = 0.25 * sqrt(21.0 / (2.0 * pi));  /* y(5z^2-1) */
  SHK[12] = 0.25 * sqrt(7.0 / pi);           /* z(5z^2-3) */
  SHK[13] = 0.25 * sqrt(21.0 / (2.0 * pi));  /* x(5z^2-1) */
  SHK[14] = 0.25 * sqrt(105.0 / pi);         /* z(x^2-y^2) */
  SHK[15] = 0.25 * sqrt(35.0 / (2.0 * pi));  /* x(x^2-3y^2) */
  sh_ready = 1;
}

/* Basis values at unit direction (x, y, z); optional gradient w.r.t. (x, y, z)
 * of the polynomials as written. */
static void sh_eval(const double s[3], double Y[16], double dY[16][3]) {
  double x = s[0], y = s[1], z = s[2];
  const double *K = SHK;
  Y[0] = K[0];
  Y[1] = K[1] * y;
  Y[2] = K[2] * z;
  Y[3] = K[3] * x;
  Y[4] = K[4] * x * y;
  Y[5] = K[5] * y * z;
  Y[6] = K[6] * (3 * z * z - 1);
  Y[7] = K[7] * x * z;
  Y[8] = K[8] * (x * x - y * y);
  Y[9] = K[9] * y * (3 * x * x - y * y);
  Y[10] = K[10] * x * y * z;
  Y[11] = K[11] * y * (5 * z * z - 1);
  Y[12] = K[12] * z * (5 * z * z - 3);
  Y[13] = K[13] * x * (5 * z * z - 1);
  Y[14] = K[14] * z * (x * x - y * y);
  Y[15] = K[15] * x * (x * x - 3 * y * y);
  if (!dY) return;
  memset(dY, 0, sizeof(double) * 48);
  dY[1][1] = K[1];
  dY[2][2] = K[2];
  dY[3][0] = K[3];
  dY[4][0] = K[4] * y; dY[4][1] = K[4] * x;
  dY[5][1] = K[5] * z; dY[5][2] = K[5] * y;
  dY[6][2] = K[6] * 6 * z;
  dY[7][0] = K[7] * z; dY[7][2] = K[7] * x;
  dY[8][0] = K[8] * 2 * x; dY[8][1] = -K[8] * 2 * y;
  dY[9][0] = K[9] * 6 * x * y; dY[9][1] = K[9] * (3 * x * x - 3 * y * y);
  dY[10][0] = K[10] * y * z; dY[10][1] = K[10] * x * z; dY[10][2] = K[10] * x * y;
  dY[11][1] = K[11] * (5 * z * z - 1); dY[11][2] = K[11] * 10 * y * z;
  dY[12][2] = K[12] * (15 * z * z - 3);
  dY[13][0] = K[13] * (5 * z * z - 1); dY[13][2] = K[13] * 10 * x * z;
  dY[14][0] = K[14] * 2 * x * z; dY[14][1] = -K[14] * 2 * y * z; dY[14][2] = K[14] * (x * x - y * y);
  dY[15][0] = K[15] * (3 * x * x - 3 * y * y); dY[15][1] = -K[15] * 6 * x * y;
}

void orc_sh_basis(int64_t m, const double *dirs, double *out) {
  sh_init();
  for (int64_t i = 0; i < m; i++) sh_eval(dirs + 3 * i, out + 16 * i, NULL);
}

/* ----------------------------------------------------------- the 6D model */
typedef struct {
  double L[6][6];
  double Sp[3][3], Spd[3][3], Sd[3][3];
  double A[3][3];  /* Sigma_d^-1 */
  double K[3][3];  /* Sigma_pd A */
  double Sc[3][3]; /* Sigma_cond */
  double mu_p[3], mu_d[3];
  double alpha;
} g6;

static double P(const double *params, int64_t n, int row, int64_t i) { return params[(int64_t)row * n + i]; }

/* Steps 1-2 of Algorithm 1 plus the direction-independent part of step 3. */
static void load_g6(const double *params, int64_t n, int64_t i, g6 *g) {
  memset(g, 0, sizeof(*g));
  for (int r = 0; r < 6; r++)
    for (int c = 0; c <= r; c++) {
      double raw = P(params, n, ROW_L + r * (r + 1) / 2 + c, i);
      g->L[r][c] = (r == c) ? exp(raw) : 2.0 * sigm(raw) - 1.0;
    }
  double S[6][6];
  for (int r = 0; r < 6; r++)
    for (int c = 0; c < 6; c++) {
      double s = 0;
      for (int k = 0; k < 6; k++) s += g->L[r][k] * g->L[c][k];
      S[r][c] = s;
    }
  for (int r = 0; r < 3; r++)
    for (int c = 0; c < 3; c++) {
      g->Sp[r][c] = S[r][c];
      g->Spd[r][c] = S[r][3 + c];
      g->Sd[r][c] = S[3 + r][3 + c];
    }
  inv3(g->Sd, g->A, NULL);
  mm3(g->Spd, g->A, g->K);
  double KSt[3][3];
  mm3t(g->K, g->Spd, KSt);
  for (int r = 0; r < 3; r++)
    for (int c = 0; c < 3; c++) g->Sc[r][c] = g->Sp[r][c] - KSt[r][c];
  for (int k = 0; k < 3; k++) {
    g->mu_p[k] = P(params, n, ROW_MU_P + k, i);
    g->mu_d[k] = P(params, n, ROW_MU_D + k, i);
  }
  g->alpha = sigm(P(params, n, ROW_OPA, i));
}

/* Direction-dependent part of step 3: mu_cond, D, f, alpha_cond for direction d. */
static void slice_dir(const g6 *g, const double d[3], double lambda, double mu_c[3], double x[3],
                      double *D, double *f, double *alpha_c) {
  double Ax[3];
  for (int k = 0; k < 3; k++) x[k] = d[k] - g->mu_d[k];
  for (int r = 0; r < 3; r++) {
    Ax[r] = g->A[r][0] * x[0] + g->A[r][1] * x[1] + g->A[r][2] * x[2];
    mu_c[r] = g->mu_p[r] + g->K[r][0] * x[0] + g->K[r][1] * x[1] + g->K[r][2] * x[2];
  }
  *D = x[0] * Ax[0] + x[1] * Ax[1] + x[2] * Ax[2];
  *f = exp(-lambda * (*D));
  *alpha_c = g->alpha * (*f);
}

/* Slice for arbitrary unit directions: out[i] = mu_cond(3), Sigma_cond(6), D, f, alpha_cond. */
void orc_slice(int64_t n, const double *params, const double *dirs, double lambda, double *out) {
  for (int64_t i = 0; i < n; i++) {
    g6 g;
    load_g6(params, n, i, &g);
    double mu_c[3], x[3], D, f, ac;
    slice_dir(&g, dirs + 3 * i, lambda, mu_c, x, &D, &f, &ac);
    double *o = out + 12 * i;
    o[0] = mu_c[0]; o[1] = mu_c[1]; o[2] = mu_c[2];
    o[3] = g.Sc[0][0]; o[4] = g.Sc[0][1]; o[5] = g.Sc[0][2];
    o[6] = g.Sc[1][1]; o[7] = g.Sc[1][2]; o[8] = g.Sc[2][2];
    o[9] = D; o[10] = f; o[11] = ac;
  }
}

/* The direction-independent part of the slice per Gaussian (what an
 * inference cache holds): out[22 i + k] = Sigma_cond (xx xy xz yy yz zz),
 * K = Sigma_pd Sigma_d^-1 (row-major), Sigma_d^-1 (xx xy xz yy yz zz), alpha. */
void orc_static(int64_t n, const double *params, double *out) {
  for (int64_t i = 0; i < n; i++) {
    g6 g;
    load_g6(params, n, i, &g);
    double *o = out + 22 * i;
    o[0] = g.Sc[0][0]; o[1] = g.Sc[0][1]; o[2] = g.Sc[0][2];
    o[3] = g.Sc[1][1]; o[4] = g.Sc[1][2]; o[5] = g.Sc[2][2];
    for (int r = 0; r < 3; r++)
      for (int c = 0; c < 3; c++) o[6 + 3 * r + c] = g.K[r][c];
    o[15] = g.A[0][0]; o[16] = g.A[0][1]; o[17] = g.A[0][2];
    o[18] = g.A[1][1]; o[19] = g.A[1][2]; o[20] = g.A[2][2];
    o[21] = g.alpha;
  }
}

static void cam_center(const orc_camera *c, double C[3]) {
  for (int k = 0; k < 3; k++) C[k] = -(c->R[0 + k] * c->t[0] + c->R[3 + k] * c->t[1] + c->R[6 + k] * c->t[2]);
}

/* Per-Gaussian record for one camera (the whole pre-rasterisation pipeline). */
static void record_one(const double *params, int64_t n, int64_t i, const orc_camera *cam,
                       const orc_settings *s, double *rec) {
  memset(rec, 0, sizeof(double) * NREC);
  g6 g;
  load_g6(params, n, i, &g);
  double C[3];
  cam_center(cam, C);
  double d[3], nd = 0;
  for (int k = 0; k < 3; k++) { d[k] = g.mu_p[k] - C[k]; nd += d[k] * d[k]; }
  nd = sqrt(nd);
  for (int k = 0; k < 3; k++) d[k] /= nd;
  double mu_c[3], x[3], D, f, ac;
  slice_dir(&g, d, lam_of(s, i), mu_c, x, &D, &f, &ac);
  for (int k = 0; k < 3; k++) { rec[F_MUC + k] = mu_c[k]; rec[F_DIR + k] = d[k]; }
  rec[F_SIGC + 0] = g.Sc[0][0]; rec[F_SIGC + 1] = g.Sc[0][1]; rec[F_SIGC + 2] = g.Sc[0][2];
  rec[F_SIGC + 3] = g.Sc[1][1]; rec[F_SIGC + 4] = g.Sc[1][2]; rec[F_SIGC + 5] = g.Sc[2][2];
  rec[F_ALPHA] = g.alpha; rec[F_F] = f; rec[F_D] = D; rec[F_ALPHAC] = ac;
  /* colour */
  double sdir[3], ns = 0;
  for (int k = 0; k < 3; k++) { sdir[k] = mu_c[k] - C[k]; ns += sdir[k] * sdir[k]; }
  ns = sqrt(ns);
  for (int k = 0; k < 3; k++) { sdir[k] /= ns; rec[F_SHDIR + k] = sdir[k]; }
  if (s->color_rgb) {
    for (int c = 0; c < 3; c++) rec[F_RGB + c] = sigm(P(params, n, ROW_SH + c, i));
  } else {
    double Y[16];
    sh_eval(sdir, Y, NULL);
    for (int c = 0; c < 3; c++) {
      double acc = 0;
      for (int k = 0; k < 16; k++) acc += P(params, n, ROW_SH + 3 * k + c, i) * Y[k];
      rec[F_RGB + c] = sigm(acc);
    }
  }
  /* camera transform and projection */
  double p[3];
  for (int r = 0; r < 3; r++)
    p[r] = cam->R[3 * r] * mu_c[0] + cam->R[3 * r + 1] * mu_c[1] + cam->R[3 * r + 2] * mu_c[2] + cam->t[r];
  for (int k = 0; k < 3; k++) rec[F_P + k] = p[k];
  rec[F_DEPTH] = p[2];
  if (fabs(p[2] - s->z_near) <= s->m_depth * fabs(p[2])) rec[F_NEARCUT] = 2.0;
  if (!(p[2] > s->z_near)) return;
  double z = p[2];
  rec[F_U] = cam->fx * p[0] / z + cam->cx;
  rec[F_V] = cam->fy * p[1] / z + cam->cy;
  double limx = s->jac_guard * (0.5 * (double)cam->width) / cam->fx;
  double limy = s->jac_guard * (0.5 * (double)cam->height) / cam->fy;
  double xt = fmin(limx, fmax(-limx, p[0] / z));
  double yt = fmin(limy, fmax(-limy, p[1] / z));
  double J[2][3] = {{cam->fx / z, 0, -cam->fx * xt / z}, {0, cam->fy / z, -cam->fy * yt / z}};
  double T[2][3];
  for (int r = 0; r < 2; r++)
    for (int c = 0; c < 3; c++) T[r][c] = J[r][0] * cam->R[c] + J[r][1] * cam->R[3 + c] + J[r][2] * cam->R[6 + c];
  double TS[2][3];
  for (int r = 0; r < 2; r++)
    for (int c = 0; c < 3; c++) TS[r][c] = T[r][0] * g.Sc[0][c] + T[r][1] * g.Sc[1][c] + T[r][2] * g.Sc[2][c];
  double cxx = TS[0][0] * T[0][0] + TS[0][1] * T[0][1] + TS[0][2] * T[0][2] + s->dilation;
  double cxy = TS[0][0] * T[1][0] + TS[0][1] * T[1][1] + TS[0][2] * T[1][2];
  double cyy = TS[1][0] * T[1][0] + TS[1][1] * T[1][1] + TS[1][2] * T[1][2] + s->dilation;
  rec[F_COV2D + 0] = cxx; rec[F_COV2D + 1] = cxy; rec[F_COV2D + 2] = cyy;
  double det = cxx * cyy - cxy * cxy;
  if (!(det > 0)) return;
  rec[F_CONIC + 0] = cyy / det;
  rec[F_CONIC + 1] = -cxy / det;
  rec[F_CONIC + 2] = cxx / det;
  if (!(ac * 255.0 >= 1.0)) {
    if (ac * 255.0 * (1.0 + s->m_alpha) >= 1.0 && rec[F_NEARCUT] == 0.0) rec[F_NEARCUT] = 1.0;
    return;
  }
  double qmax = 2.0 * log(255.0 * ac);
  rec[F_EX] = sqrt(qmax * cxx);
  rec[F_EY] = sqrt(qmax * cyy);
  rec[F_ALIVE] = 1.0;
}

void orc_preprocess(int64_t n, const double *params, const orc_camera *cam, const orc_settings *s, double *rec) {
  sh_init();
  for (int64_t i = 0; i < n; i++) record_one(params, n, i, cam, s, rec + NREC * i);
}

/* ------------------------------------------------------- global depth order */
typedef struct { double depth; int64_t idx; } order_item;
static int cmp_order(const void *a, const void *b) {
  const order_item *x = a, *y = b;
  if (x->depth < y->depth) return -1;
  if (x->depth > y->depth) return 1;
  return (x->idx < y->idx) ? -1 : (x->idx > y->idx);
}

/* Gaussians selected by `pick` (alive ones, or alive and near-cut ones),
 * sorted by (depth, index); returns their count. */
static int64_t global_order(int64_t n, const double *rec, int64_t *order, int with_nearcut) {
  order_item *it = malloc(sizeof(order_item) * (n > 0 ? n : 1));
  int64_t m = 0;
  for (int64_t i = 0; i < n; i++) {
    const double *r = rec + NREC * i;
    if (r[F_ALIVE] != 0.0 || (with_nearcut && r[F_NEARCUT] == 1.0)) {
      it[m].depth = r[F_DEPTH];
      it[m].idx = i;
      m++;
    }
  }
  qsort(it, m, sizeof(order_item), cmp_order);
  for (int64_t k = 0; k < m; k++) order[k] = it[k].idx;
  free(it);
  return m;
}

/* Compact view of the sorted records, so the per-pixel walk reads one array. */
typedef struct { double u, v, qa, qb, qc, ac, r, g, b, depth; int live; } sorted_rec;

static sorted_rec *make_sorted(const double *rec, const int64_t *order, int64_t m) {
  sorted_rec *sr = malloc(sizeof(sorted_rec) * (m > 0 ? m : 1));
  for (int64_t k = 0; k < m; k++) {
    const double *r = rec + NREC * order[k];
    sr[k].u = r[F_U]; sr[k].v = r[F_V];
    sr[k].qa = r[F_CONIC]; sr[k].qb = r[F_CONIC + 1]; sr[k].qc = r[F_CONIC + 2];
    sr[k].ac = r[F_ALPHAC];
    sr[k].r = r[F_RGB]; sr[k].g = r[F_RGB + 1]; sr[k].b = r[F_RGB + 2];
    sr[k].depth = r[F_DEPTH];
    sr[k].live = r[F_ALIVE] != 0.0;
  }
  return sr;
}

/* ----------------------------------------------------- per-pixel compositing */
/* Walks one pixel front to back over the alive Gaussians in depth order: the
 * definition of the rendered value.  Fills colour, final T and the contributor
 * count; if clist != NULL stores the contributors' sorted positions, their
 * alpha before the clamp and the transmittance in front of them. */
typedef struct {
  double color[3];
  double T;
  int64_t ncontrib;
} pix_out;

static void walk_pixel(const sorted_rec *sr, int64_t m, double px, double py, const orc_settings *s,
                       pix_out *o, int64_t *clist, double *araw_list, double *T_list) {
  double T = 1.0, C[3] = {0, 0, 0};
  int64_t nc = 0;
  for (int64_t k = 0; k < m; k++) {
    const sorted_rec *g = sr + k;
    double dx = px - g->u, dy = py - g->v;
    double q = g->qa * dx * dx + 2.0 * g->qb * dx * dy + g->qc * dy * dy;
    double araw = g->ac * exp(-0.5 * q);
    double a = fmin(s->alpha_max, araw);
    if (a < s->alpha_min) continue;
    double Tn = T * (1.0 - a);
    if (Tn < s->t_min) break;
    C[0] += g->r * a * T;
    C[1] += g->g * a * T;
    C[2] += g->b * a * T;
    if (clist) { clist[nc] = k; araw_list[nc] = araw; T_list[nc] = T; }
    T = Tn;
    nc++;
  }
  for (int c = 0; c < 3; c++) o->color[c] = C[c] + T * s->bg[c];
  o->T = T;
  o->ncontrib = nc;
}

/* ------------------------------------------------------ decision envelope */
/* Test infrastructure for comparing a float32 renderer with the definition.
 * The walk above takes three kinds of threshold decisions -- skip a Gaussian
 * whose alpha is below 1/255, stop before the transmittance falls below 1e-4,
 * and the front-to-back order of Gaussians at (nearly) equal depth -- and a
 * renderer working on float32 records may legitimately take any of them the
 * other way when the record fields move within the float32 error bounds m_*
 * of the settings.  For one pixel this follows every combination of outcomes
 * of such decisions (each path a walk of the definition with those outcomes
 * forced) and returns the range of colour and final transmittance over all of
 * them.  A pixel with one outcome path is unambiguous, and its range is the
 * single value walk_pixel returns.
 *
 * The paths are followed breadth first over the candidates in depth order.
 * Everything a path decides later depends on its transmittance alone, not on
 * the colour gathered so far, so paths that reach a candidate with the same
 * transmittance are merged into one state that carries the range of their
 * colours.  Candidates whose depths lie within the depth margin of each other
 * form a group that is taken in every order. */
enum { ENV_AMBIGUOUS = 1, ENV_KINK = 2, ENV_UNRESOLVED = 4 };

typedef struct {
  double a;       /* alpha after the clamp */
  double rel;     /* relative uncertainty of a */
  double depth;
  double rgb[3];
  int take_nom;   /* the definition takes it (alpha >= 1/255, alive) */
  int can_flip;   /* the 1/255 decision may go the other way */
  int kink;       /* the 0.99 clamp may go the other way (value continuous, derivative not) */
} cand;

typedef struct {
  double T, Trel;       /* transmittance in front of the next candidate, its relative uncertainty */
  double lo[3], hi[3];  /* range of the colour gathered so far */
} env_state;

typedef struct {
  const orc_settings *s;
  env_state *nxt;       /* states after the current group */
  int64_t nnxt, cap;
  double lo[4], hi[4];  /* colour (3) and final T over the finished paths */
  int64_t leaves;
  int flags;
  double impact;        /* largest local effect of an undecided decision (see pixel_envelope) */
} envelope;

/* Bound on |ln a' - ln a| at pixel offset d = (dx, dy) from the Gaussian's
 * mean when the record moves within the margins: the mean by e = m_uv per
 * axis; the conic Q by E with |x^T E x| <= m_conic x^T Q x for every x (its
 * error in its own metric); alpha_cond by the factor (1 +- m_alpha); plus the
 * float32 evaluation of ln a, whose rounding is m_eval relative to the
 * magnitudes of its terms.  With d' = d - eps,
 *   q' = d'^T (Q + E) d' = (1 + t) d'^T Q d',  |t| <= m_conic,
 *   d'^T Q d' = q - 2 eps^T Q d + eps^T Q eps,
 * |eps^T Q d| <= e (|(Qd)_x| + |(Qd)_y|) and eps^T Q eps <= 2 e^2 (Qxx + Qyy). */
static double ln_alpha_margin(const orc_settings *s, const sorted_rec *g, double dx, double dy) {
  const double e = s->m_uv;
  const double q = g->qa * dx * dx + 2.0 * g->qb * dx * dy + g->qc * dy * dy;
  const double gx = fabs(g->qa * dx + g->qb * dy), gy = fabs(g->qb * dx + g->qc * dy);
  const double shift = 2.0 * e * (gx + gy) + 2.0 * e * e * (g->qa + g->qc);
  const double dq = shift + s->m_conic * (q + shift);
  const double l1 = fabs(dx) + fabs(dy);
  const double terms = 1.0 + fabs(log(g->ac)) + fmax(fabs(g->qa), fabs(g->qc)) * l1 * l1;
  return -log1p(-s->m_alpha) + 0.5 * dq + s->m_eval * terms;
}

/* A finished path: its walk stopped, or ran out of candidates. */
static void env_leaf(envelope *e, double T, const double lo[3], const double hi[3]) {
  const double *bg = e->s->bg;
  const double vl[4] = {lo[0] + T * bg[0], lo[1] + T * bg[1], lo[2] + T * bg[2], T};
  const double vh[4] = {hi[0] + T * bg[0], hi[1] + T * bg[1], hi[2] + T * bg[2], T};
  for (int k = 0; k < 4; k++) {
    if (e->leaves == 0 || vl[k] < e->lo[k]) e->lo[k] = vl[k];
    if (e->leaves == 0 || vh[k] > e->hi[k]) e->hi[k] = vh[k];
  }
  e->leaves++;
}

static void env_push(envelope *e, double T, double Trel, const double lo[3], const double hi[3]) {
  if (e->nnxt == e->cap) { e->flags |= ENV_UNRESOLVED; return; }
  env_state *x = e->nxt + e->nnxt++;
  x->T = T; x->Trel = Trel;
  for (int c = 0; c < 3; c++) { x->lo[c] = lo[c]; x->hi[c] = hi[c]; }
}

/* Members k.. of a group in the order perm: every outcome of each member's
 * decisions; paths that get through the group become states of the next. */
static void env_members(envelope *e, const cand *c, const int64_t *perm, int64_t g, int64_t k, double T, double Trel,
                        const double lo[3], const double hi[3]) {
  if (k == g) { env_push(e, T, Trel, lo, hi); return; }
  const orc_settings *s = e->s;
  const cand *x = c + perm[k];
  if (x->can_flip) {
    e->flags |= ENV_AMBIGUOUS;
    e->impact = fmax(e->impact, T * x->a);
  }
  if (!x->take_nom || x->can_flip) env_members(e, c, perm, g, k + 1, T, Trel, lo, hi); /* skipped */
  if (!x->take_nom && !x->can_flip) return;
  /* taken: T' = T (1 - a) carries the uncertainty of T, of a, and one rounding each of 1 - a and the product */
  const double Tn = T * (1.0 - x->a);
  const double Trel_n = Trel + (x->a * x->rel + s->m_trel) / (1.0 - x->a) + s->m_trel;
  const int may_stop = Tn * (1.0 - Trel_n) < s->t_min;
  const int may_go = Tn * (1.0 + Trel_n) >= s->t_min;
  if (may_stop && may_go) {
    e->flags |= ENV_AMBIGUOUS;
    e->impact = fmax(e->impact, T * x->a);
  }
  if (x->kink) {
    e->flags |= ENV_KINK;
    e->impact = fmax(e->impact, T * x->a);
  }
  if (may_stop) env_leaf(e, T, lo, hi);
  if (may_go) {
    double l2[3], h2[3];
    for (int ch = 0; ch < 3; ch++) {
      l2[ch] = lo[ch] + x->rgb[ch] * x->a * T;
      h2[ch] = hi[ch] + x->rgb[ch] * x->a * T;
    }
    env_members(e, c, perm, g, k + 1, Tn, Trel_n, l2, h2);
  }
}

/* Every order of perm[pos..g) for one incoming state. */
static void env_orders(envelope *e, const cand *c, int64_t *perm, int64_t g, int64_t pos, const env_state *st) {
  if (pos == g) { env_members(e, c, perm, g, 0, st->T, st->Trel, st->lo, st->hi); return; }
  for (int64_t i = pos; i < g; i++) {
    int64_t t = perm[pos]; perm[pos] = perm[i]; perm[i] = t;
    env_orders(e, c, perm, g, pos + 1, st);
    t = perm[pos]; perm[pos] = perm[i]; perm[i] = t;
  }
}

static int cmp_state(const void *a, const void *b) {
  const double x = ((const env_state *)a)->T, y = ((const env_state *)b)->T;
  return (x > y) - (x < y);
}

/* Merges states whose transmittances agree to 1e-12 relative (orders of one
 * group give the same product up to rounding). */
static int64_t env_merge(env_state *st, int64_t n) {
  if (n <= 1) return n;
  qsort(st, n, sizeof(env_state), cmp_state);
  int64_t m = 0;
  for (int64_t i = 1; i < n; i++) {
    env_state *a = st + m, *b = st + i;
    if (b->T - a->T <= 1e-12 * fmax(a->T, b->T)) {
      a->Trel = fmax(a->Trel, b->Trel) + 1e-12;
      for (int c = 0; c < 3; c++) { a->lo[c] = fmin(a->lo[c], b->lo[c]); a->hi[c] = fmax(a->hi[c], b->hi[c]); }
    } else {
      st[++m] = *b;
    }
  }
  return m + 1;
}

/* Largest group of depth-undecided candidates that is permuted (5! orders). */
#define ENV_MAX_GROUP 5

/* Envelope of one pixel over sr (alive and near-cut Gaussians in depth
 * order).  cbuf holds m candidates, sbuf 2 * cap states.  *impact bounds
 * the local effect of the undecided decisions, which is what a gradient
 * comparison must stay clear of: a flipped skip or stop adds or removes one
 * term of size T a; a swap of two Gaussians scales the transmittance in
 * front of one of them by 1 - a of the other, a change of T a_i a_j to its
 * term (the transmittance behind the pair does not depend on their order);
 * a clamp that may go the other way changes the derivative of a term T a. */
static void pixel_envelope(const sorted_rec *sr, int64_t m, double px, double py, const orc_settings *s,
                           cand *cbuf, env_state *sbuf, int64_t cap, double lo[4], double hi[4], int64_t *leaves,
                           int *flags, double *impact) {
  const double ln_min = log(s->alpha_min);
  int64_t nc = 0;
  int fl = 0;
  for (int64_t k = 0; k < m; k++) {
    const sorted_rec *g = sr + k;
    const double dx = px - g->u, dy = py - g->v;
    const double q = g->qa * dx * dx + 2.0 * g->qb * dx * dy + g->qc * dy * dy;
    const double lna = log(g->ac) - 0.5 * q;
    if (lna < ln_min - 0.5) continue; /* far below the cut: no margin here comes near 0.5 */
    const double dl = ln_alpha_margin(s, g, dx, dy);
    if (dl >= 0.5) fl |= ENV_UNRESOLVED;
    if (lna + dl < ln_min) continue;
    const double araw = g->ac * exp(-0.5 * q);
    cand *c = cbuf + nc;
    c->a = fmin(s->alpha_max, araw);
    c->take_nom = g->live && c->a >= s->alpha_min;
    c->can_flip = (araw * exp(-dl) < s->alpha_min) && (araw * exp(dl) >= s->alpha_min);
    const int clamped_lo = araw * exp(-dl) >= s->alpha_max; /* clamped whatever the error */
    c->kink = !clamped_lo && araw * exp(dl) >= s->alpha_max;
    c->rel = clamped_lo ? 0.0 : expm1(dl);
    c->depth = g->depth;
    c->rgb[0] = g->r; c->rgb[1] = g->g; c->rgb[2] = g->b;
    nc++;
  }
  envelope e;
  e.s = s; e.cap = cap; e.leaves = 0; e.flags = fl; e.impact = 0.0;
  env_state *cur = sbuf, *nxt = sbuf + cap;
  int64_t ncur = 1;
  cur[0].T = 1.0; cur[0].Trel = 0.0;
  for (int c = 0; c < 3; c++) cur[0].lo[c] = cur[0].hi[c] = 0.0;
  int64_t perm[ENV_MAX_GROUP];
  for (int64_t j = 0; j < nc && ncur > 0 && !(e.flags & ENV_UNRESOLVED);) {
    /* the group: consecutive candidates whose depths lie within the depth margin */
    int64_t r = j;
    while (r + 1 < nc && fabs(cbuf[r + 1].depth - cbuf[r].depth) <=
                             s->m_depth * (fabs(cbuf[r + 1].depth) + fabs(cbuf[r].depth)))
      r++;
    const int64_t g = r - j + 1;
    if (g > ENV_MAX_GROUP) { e.flags |= ENV_UNRESOLVED; break; }
    if (g > 1) {
      e.flags |= ENV_AMBIGUOUS;
      double tmax = 0.0, a1 = 0.0, a2 = 0.0; /* the largest state T and the two largest alphas */
      for (int64_t i = 0; i < ncur; i++) tmax = fmax(tmax, cur[i].T);
      for (int64_t k = j; k <= r; k++) {
        if (cbuf[k].a > a1) { a2 = a1; a1 = cbuf[k].a; }
        else if (cbuf[k].a > a2) a2 = cbuf[k].a;
      }
      e.impact = fmax(e.impact, tmax * a1 * a2);
    }
    for (int64_t k = 0; k < g; k++) perm[k] = k;
    e.nxt = nxt;
    e.nnxt = 0;
    for (int64_t i = 0; i < ncur; i++) env_orders(&e, cbuf + j, perm, g, 0, cur + i);
    ncur = env_merge(nxt, e.nnxt);
    env_state *t = cur; cur = nxt; nxt = t;
    j = r + 1;
  }
  for (int64_t i = 0; i < ncur; i++) env_leaf(&e, cur[i].T, cur[i].lo, cur[i].hi);
  for (int k = 0; k < 4; k++) { lo[k] = e.lo[k]; hi[k] = e.hi[k]; }
  *leaves = e.leaves;
  *flags = e.flags;
  *impact = e.impact;
}

static int num_threads(int req) {
  if (req > 0) return req;
  long c = sysconf(_SC_NPROCESSORS_ONLN);
  return c > 0 ? (int)c : 1;
}

int orc_num_threads(int req) { return num_threads(req); }

typedef struct {
  const sorted_rec *sr;
  int64_t m;
  const orc_camera *cam;
  const orc_settings *s;
  int64_t npix;
  const int64_t *pix;
  int nthreads, tid;
  /* forward outputs */
  double *color, *Tf;
  int64_t *ncontrib;
  /* decision envelope (NULL: not wanted): the alive and near-cut records */
  const sorted_rec *sr_env;
  int64_t m_env;
  double *env_lo, *env_hi; /* [npix][4] */
  double *env_impact;
  int64_t *env_leaves;
  int32_t *env_flags;
  /* backward */
  const double *dl_dc;   /* [npix][3] */
  const double *rec;     /* sorted positions -> per Gaussian via order */
  const int64_t *order;
  double *g2d;           /* this thread's [n][9] accumulator */
} job;

static void pixel_xy(const job *j, int64_t k, double *px, double *py) {
  int64_t id = j->pix ? j->pix[k] : k;
  int64_t W = j->cam->width;
  *px = (double)(id % W) + 0.5;
  *py = (double)(id / W) + 0.5;
}

static void *fwd_worker(void *arg) {
  job *j = arg;
  const int64_t me = j->m_env > 0 ? j->m_env : 1, cap = j->s->max_leaves > 0 ? j->s->max_leaves : 1;
  cand *cb = j->env_lo ? malloc(sizeof(cand) * me) : NULL;
  env_state *sb = j->env_lo ? malloc(sizeof(env_state) * 2 * cap) : NULL;
  for (int64_t k = j->tid; k < j->npix; k += j->nthreads) {
    double px, py;
    pixel_xy(j, k, &px, &py);
    pix_out o;
    walk_pixel(j->sr, j->m, px, py, j->s, &o, NULL, NULL, NULL);
    for (int c = 0; c < 3; c++) j->color[3 * k + c] = o.color[c];
    j->Tf[k] = o.T;
    j->ncontrib[k] = o.ncontrib;
    if (j->env_lo) {
      int fl;
      pixel_envelope(j->sr_env, j->m_env, px, py, j->s, cb, sb, cap, j->env_lo + 4 * k, j->env_hi + 4 * k,
                     j->env_leaves + k, &fl, j->env_impact + k);
      j->env_flags[k] = fl;
    }
  }
  free(cb);
  free(sb);
  return NULL;
}

/* Shared by the two render entry points: walks the listed pixels (row-major
 * ids j*W+i; all pixels if pix == NULL) over the sorted records; the envelope
 * outputs may be NULL. */
static int render_sorted(const sorted_rec *sr, int64_t m, const sorted_rec *sr_env, int64_t m_env,
                         const orc_camera *cam, const orc_settings *s, int64_t npix, const int64_t *pix,
                         double *color, double *T_final, int64_t *ncontrib, double *env_lo, double *env_hi,
                         double *env_impact, int64_t *env_leaves, int32_t *env_flags, int nthreads_req) {
  int nt = num_threads(nthreads_req);
  pthread_t *th = malloc(sizeof(pthread_t) * nt);
  job *jobs = calloc(nt, sizeof(job));
  if (!th || !jobs) return -1;
  for (int t = 0; t < nt; t++) {
    job *jb = jobs + t;
    jb->sr = sr; jb->m = m; jb->cam = cam; jb->s = s; jb->npix = npix; jb->pix = pix;
    jb->nthreads = nt; jb->tid = t;
    jb->color = color; jb->Tf = T_final; jb->ncontrib = ncontrib;
    jb->sr_env = sr_env; jb->m_env = m_env;
    jb->env_lo = env_lo; jb->env_hi = env_hi; jb->env_impact = env_impact;
    jb->env_leaves = env_leaves; jb->env_flags = env_flags;
    pthread_create(&th[t], NULL, fwd_worker, jb);
  }
  for (int t = 0; t < nt; t++) pthread_join(th[t], NULL);
  free(th);
  free(jobs);
  return 0;
}

/* Render the listed pixels (row-major ids j*W+i; all pixels if pix == NULL).
 * env_* (each NULL, or all given): the decision envelope per pixel, lo / hi
 * [npix][4] (colour, final T), the impact bound, the number of finished
 * outcome paths and the ENV_* flags.  Returns the number of Gaussians whose depth lies within the depth
 * margin of z_near (their culling is a decision no envelope covers), or -1 if
 * memory ran out. */
int orc_render(int64_t n, const double *params, const orc_camera *cam, const orc_settings *s, int64_t npix,
               const int64_t *pix, double *color, double *T_final, int64_t *ncontrib, double *env_lo,
               double *env_hi, double *env_impact, int64_t *env_leaves, int32_t *env_flags, int nthreads_req) {
  sh_init();
  double *rec = malloc(sizeof(double) * NREC * (n > 0 ? n : 1));
  int64_t *order = malloc(sizeof(int64_t) * (n > 0 ? n : 1));
  if (!rec || !order) return -1;
  orc_preprocess(n, params, cam, s, rec);
  int64_t m = global_order(n, rec, order, 0);
  sorted_rec *sr = make_sorted(rec, order, m);
  sorted_rec *sr_env = NULL;
  int64_t m_env = 0, near_z = 0;
  if (env_lo) {
    m_env = global_order(n, rec, order, 1);
    sr_env = make_sorted(rec, order, m_env);
  }
  for (int64_t i = 0; i < n; i++) near_z += rec[NREC * i + F_NEARCUT] == 2.0;
  int rc = render_sorted(sr, m, sr_env, m_env, cam, s, npix, pix, color, T_final, ncontrib, env_lo, env_hi,
                         env_impact, env_leaves, env_flags, nthreads_req);
  free(sr_env); free(sr); free(order); free(rec);
  return rc < 0 ? -1 : (int)near_z;
}

/* Render from given records instead of parameters (m Gaussians, any order;
 * recs [m][11]: u, v, Qxx, Qxy, Qyy, alpha_cond, r, g, b, depth, alive), with
 * the same outputs as orc_render.  Used to check the envelope: records moved
 * within the margins must render inside the envelope of the unmoved ones. */
int orc_render_records(int64_t m, const double *recs, const orc_camera *cam, const orc_settings *s, int64_t npix,
                       const int64_t *pix, double *color, double *T_final, int64_t *ncontrib, double *env_lo,
                       double *env_hi, double *env_impact, int64_t *env_leaves, int32_t *env_flags,
                       int nthreads_req) {
  double *rec = calloc((size_t)NREC * (m > 0 ? m : 1), sizeof(double));
  int64_t *order = malloc(sizeof(int64_t) * (m > 0 ? m : 1));
  if (!rec || !order) return -1;
  for (int64_t i = 0; i < m; i++) {
    const double *x = recs + 11 * i;
    double *r = rec + NREC * i;
    r[F_U] = x[0]; r[F_V] = x[1];
    r[F_CONIC] = x[2]; r[F_CONIC + 1] = x[3]; r[F_CONIC + 2] = x[4];
    r[F_ALPHAC] = x[5];
    r[F_RGB] = x[6]; r[F_RGB + 1] = x[7]; r[F_RGB + 2] = x[8];
    r[F_DEPTH] = x[9];
    r[F_ALIVE] = x[10] != 0.0 && x[5] * 255.0 >= 1.0;
    r[F_NEARCUT] = x[10] != 0.0 && !(x[5] * 255.0 >= 1.0) && x[5] * 255.0 * (1.0 + s->m_alpha) >= 1.0;
  }
  int64_t mm = global_order(m, rec, order, 0);
  sorted_rec *sr = make_sorted(rec, order, mm);
  sorted_rec *sr_env = NULL;
  int64_t m_env = 0;
  if (env_lo) {
    m_env = global_order(m, rec, order, 1);
    sr_env = make_sorted(rec, order, m_env);
  }
  int rc = render_sorted(sr, mm, sr_env, m_env, cam, s, npix, pix, color, T_final, ncontrib, env_lo, env_hi,
                         env_impact, env_leaves, env_flags, nthreads_req);
  free(sr_env); free(sr); free(order); free(rec);
  return rc;
}

/* ----------------------------------------------------- backward: compositing */
/* 2D gradient slots per Gaussian: du, dv, dQxx, dQxy, dQyy, dalpha_c, dr, dg, db.
 * dQ is the full-matrix gradient: dL = dQxx dQ_xx + 2 dQxy dQ_xy + dQyy dQ_yy. */
enum { G_U = 0, G_V, G_QXX, G_QXY, G_QYY, G_AC, G_R, G_G, G_B, NG2D };

static void *bwd_worker(void *arg) {
  job *j = arg;
  int64_t *clist = malloc(sizeof(int64_t) * (j->m > 0 ? j->m : 1));
  double *alist = malloc(sizeof(double) * (j->m > 0 ? j->m : 1));
  double *tlist = malloc(sizeof(double) * (j->m > 0 ? j->m : 1));
  const orc_settings *s = j->s;
  for (int64_t k = j->tid; k < j->npix; k += j->nthreads) {
    double px, py;
    pixel_xy(j, k, &px, &py);
    pix_out o;
    walk_pixel(j->sr, j->m, px, py, s, &o, clist, alist, tlist);
    const double *dc = j->dl_dc + 3 * k;
    /* colour behind the current Gaussian, starting with the background seen through T_final */
    double behind[3] = {o.T * s->bg[0], o.T * s->bg[1], o.T * s->bg[2]};
    for (int64_t c = o.ncontrib - 1; c >= 0; c--) {
      const sorted_rec *g = j->sr + clist[c];
      double araw = alist[c];
      double a = fmin(s->alpha_max, araw);
      double Tk = tlist[c];
      double col[3] = {g->r, g->g, g->b};
      double *acc = j->g2d + NG2D * j->order[clist[c]];
      double dl_da = 0;
      for (int ch = 0; ch < 3; ch++) {
        acc[G_R + ch] += dc[ch] * a * Tk;
        dl_da += dc[ch] * (col[ch] * Tk - behind[ch] / (1.0 - a));
        behind[ch] += col[ch] * a * Tk;
      }
      if (araw > s->alpha_max) continue; /* clamped: a does not depend on alpha_c or q */
      double G = exp(-0.5 * (g->qa * (px - g->u) * (px - g->u) + 2.0 * g->qb * (px - g->u) * (py - g->v) +
                             g->qc * (py - g->v) * (py - g->v)));
      acc[G_AC] += dl_da * G;
      double dl_dq = dl_da * (-0.5 * araw);
      double dx = px - g->u, dy = py - g->v;
      acc[G_U] += dl_dq * (-2.0) * (g->qa * dx + g->qb * dy);
      acc[G_V] += dl_dq * (-2.0) * (g->qb * dx + g->qc * dy);
      acc[G_QXX] += dl_dq * dx * dx;
      acc[G_QXY] += dl_dq * dx * dy;
      acc[G_QYY] += dl_dq * dy * dy;
    }
  }
  free(clist); free(alist); free(tlist);
  return NULL;
}

/* ------------------------------------------- backward: per-Gaussian chain rule */
/* Vector-Jacobian product of one Gaussian's record (u, v, conic, alpha_c, rgb)
 * with respect to its 76 raw parameters; adds into grad ([76][n]). */
static void record_vjp(const double *params, int64_t n, int64_t i, const orc_camera *cam, const orc_settings *s,
                       const double *g2, double *grad) {
  double rec[NREC];
  record_one(params, n, i, cam, s, rec);
  if (rec[F_ALIVE] == 0.0) return;
  g6 g;
  load_g6(params, n, i, &g);
  double C[3];
  cam_center(cam, C);
  double z = rec[F_P + 2], px = rec[F_P], py = rec[F_P + 1];
  double fx = cam->fx, fy = cam->fy;
  const double *R = cam->R;
  /* conic -> 2D covariance: G_S = -Q G_Q Q */
  double Q[2][2] = {{rec[F_CONIC], rec[F_CONIC + 1]}, {rec[F_CONIC + 1], rec[F_CONIC + 2]}};
  double GQ[2][2] = {{g2[G_QXX], g2[G_QXY]}, {g2[G_QXY], g2[G_QYY]}};
  double QG[2][2], GS[2][2];
  for (int r = 0; r < 2; r++)
    for (int c = 0; c < 2; c++) QG[r][c] = Q[r][0] * GQ[0][c] + Q[r][1] * GQ[1][c];
  for (int r = 0; r < 2; r++)
    for (int c = 0; c < 2; c++) GS[r][c] = -(QG[r][0] * Q[0][c] + QG[r][1] * Q[1][c]);
  /* Sigma2D = T Sigma_c T^T + dil I, T = J R */
  double limx = s->jac_guard * (0.5 * (double)cam->width) / fx;
  double limy = s->jac_guard * (0.5 * (double)cam->height) / fy;
  double rx = px / z, ry = py / z;
  int clx = (rx < -limx) || (rx > limx);
  int cly = (ry < -limy) || (ry > limy);
  double xt = fmin(limx, fmax(-limx, rx));
  double yt = fmin(limy, fmax(-limy, ry));
  double J[2][3] = {{fx / z, 0, -fx * xt / z}, {0, fy / z, -fy * yt / z}};
  double T[2][3];
  for (int r = 0; r < 2; r++)
    for (int c = 0; c < 3; c++) T[r][c] = J[r][0] * R[c] + J[r][1] * R[3 + c] + J[r][2] * R[6 + c];
  double Gc[3][3]; /* T^T G_S T */
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) {
      double acc = 0;
      for (int r = 0; r < 2; r++)
        for (int c = 0; c < 2; c++) acc += T[r][a] * GS[r][c] * T[c][b];
      Gc[a][b] = acc;
    }
  double dT[2][3]; /* 2 G_S T Sigma_c */
  for (int r = 0; r < 2; r++)
    for (int c = 0; c < 3; c++) {
      double acc = 0;
      for (int k = 0; k < 2; k++)
        for (int m = 0; m < 3; m++) acc += GS[r][k] * T[k][m] * g.Sc[m][c];
      dT[r][c] = 2.0 * acc;
    }
  double dJ[2][3]; /* dT R^T */
  for (int r = 0; r < 2; r++)
    for (int c = 0; c < 3; c++) dJ[r][c] = dT[r][0] * R[3 * c] + dT[r][1] * R[3 * c + 1] + dT[r][2] * R[3 * c + 2];
  double dp[3] = {0, 0, 0};
  dp[2] += dJ[0][0] * (-fx / (z * z)) + dJ[1][1] * (-fy / (z * z));
  if (!clx) { dp[0] += dJ[0][2] * (-fx / (z * z)); dp[2] += dJ[0][2] * (2.0 * fx * px / (z * z * z)); }
  else { dp[2] += dJ[0][2] * (fx * xt / (z * z)); }
  if (!cly) { dp[1] += dJ[1][2] * (-fy / (z * z)); dp[2] += dJ[1][2] * (2.0 * fy * py / (z * z * z)); }
  else { dp[2] += dJ[1][2] * (fy * yt / (z * z)); }
  /* u, v */
  dp[0] += g2[G_U] * fx / z;
  dp[1] += g2[G_V] * fy / z;
  dp[2] += -g2[G_U] * fx * px / (z * z) - g2[G_V] * fy * py / (z * z);
  /* p = R mu_c + t */
  double gmu[3];
  for (int k = 0; k < 3; k++) gmu[k] = R[k] * dp[0] + R[3 + k] * dp[1] + R[6 + k] * dp[2];
  /* SH colour */
  double sv[3], ns = 0;
  for (int k = 0; k < 3; k++) { sv[k] = rec[F_MUC + k] - C[k]; ns += sv[k] * sv[k]; }
  ns = sqrt(ns);
  double sh[3] = {sv[0] / ns, sv[1] / ns, sv[2] / ns};
  double gs[3] = {0, 0, 0};
  if (s->color_rgb) {
    /* rgb = sigmoid(c): no dependence on the viewing direction */
    for (int c = 0; c < 3; c++) {
      double rgb = rec[F_RGB + c];
      grad[(int64_t)(ROW_SH + c) * n + i] += g2[G_R + c] * rgb * (1.0 - rgb);
    }
  } else {
    double Y[16], dY[16][3];
    sh_eval(sh, Y, dY);
    for (int c = 0; c < 3; c++) {
      double rgb = rec[F_RGB + c];
      double dsc = g2[G_R + c] * rgb * (1.0 - rgb);
      for (int k = 0; k < 16; k++) {
        grad[(int64_t)(ROW_SH + 3 * k + c) * n + i] += dsc * Y[k];
        double beta = P(params, n, ROW_SH + 3 * k + c, i);
        for (int m = 0; m < 3; m++) gs[m] += dsc * beta * dY[k][m];
      }
    }
  }
  double sdot = sh[0] * gs[0] + sh[1] * gs[1] + sh[2] * gs[2];
  for (int k = 0; k < 3; k++) gmu[k] += (gs[k] - sh[k] * sdot) / ns;
  /* slice */
  double x[3], Ax[3];
  for (int k = 0; k < 3; k++) x[k] = rec[F_DIR + k] - g.mu_d[k];
  for (int r = 0; r < 3; r++) Ax[r] = g.A[r][0] * x[0] + g.A[r][1] * x[1] + g.A[r][2] * x[2];
  double ac = rec[F_ALPHAC], gac = g2[G_AC], lam = lam_of(s, i);
  double dD = -lam * ac * gac;
  /* alpha_cond = alpha exp(-lambda D): d alpha_cond / d lambda = -D alpha_cond */
  if (s->lambda_raw && s->grad_lambda) s->grad_lambda[i] += -rec[F_D] * ac * gac * lam * (1.0 - lam);
  double gx[3];
  for (int k = 0; k < 3; k++)
    gx[k] = g.K[0][k] * gmu[0] + g.K[1][k] * gmu[1] + g.K[2][k] * gmu[2] + 2.0 * dD * Ax[k];
  double GSp[3][3], GSpd[3][3], GA[3][3];
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) GSp[a][b] = Gc[a][b];
  double GcSpd[3][3], GcSpdA[3][3];
  mm3(Gc, g.Spd, GcSpd);
  mm3(GcSpd, g.A, GcSpdA);
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) GSpd[a][b] = gmu[a] * Ax[b] - 2.0 * GcSpdA[a][b];
  double SpdTgmu[3];
  for (int a = 0; a < 3; a++) SpdTgmu[a] = g.Spd[0][a] * gmu[0] + g.Spd[1][a] * gmu[1] + g.Spd[2][a] * gmu[2];
  double SpdTGcSpd[3][3];
  mtm3(g.Spd, GcSpd, SpdTGcSpd);
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++)
      GA[a][b] = 0.5 * (SpdTgmu[a] * x[b] + SpdTgmu[b] * x[a]) - SpdTGcSpd[a][b] + dD * x[a] * x[b];
  double AGA[3][3], tmp[3][3], GSd[3][3];
  mm3(g.A, GA, tmp);
  mm3(tmp, g.A, AGA);
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) GSd[a][b] = -AGA[a][b];
  /* mu_d, mu_p (through d = (mu_p - C)/|mu_p - C|), alpha */
  double dv[3], nd = 0;
  for (int k = 0; k < 3; k++) { dv[k] = g.mu_p[k] - C[k]; nd += dv[k] * dv[k]; }
  nd = sqrt(nd);
  double dd[3] = {dv[0] / nd, dv[1] / nd, dv[2] / nd};
  double ddot = dd[0] * gx[0] + dd[1] * gx[1] + dd[2] * gx[2];
  for (int k = 0; k < 3; k++) {
    grad[(int64_t)(ROW_MU_D + k) * n + i] += -gx[k];
    grad[(int64_t)(ROW_MU_P + k) * n + i] += gmu[k] + (gx[k] - dd[k] * ddot) / nd;
  }
  double galpha = gac * rec[F_F];
  grad[(int64_t)ROW_OPA * n + i] += galpha * g.alpha * (1.0 - g.alpha);
  /* Sigma = L L^T: dL/dL = lower(2 G6 L), G6 = [[G_p, H/2], [H^T/2, G_d]] */
  double G6[6][6];
  for (int a = 0; a < 3; a++)
    for (int b = 0; b < 3; b++) {
      G6[a][b] = 0.5 * (GSp[a][b] + GSp[b][a]);
      G6[3 + a][3 + b] = 0.5 * (GSd[a][b] + GSd[b][a]);
      G6[a][3 + b] = 0.5 * GSpd[a][b];
      G6[3 + b][a] = 0.5 * GSpd[a][b];
    }
  for (int r = 0; r < 6; r++)
    for (int c = 0; c <= r; c++) {
      double acc = 0;
      for (int k = 0; k < 6; k++) acc += G6[r][k] * g.L[k][c];
      double gl = 2.0 * acc;
      double raw = P(params, n, ROW_L + r * (r + 1) / 2 + c, i);
      double graw;
      if (r == c) graw = gl * g.L[r][c];
      else { double sg = sigm(raw); graw = gl * 2.0 * sg * (1.0 - sg); }
      grad[(int64_t)(ROW_L + r * (r + 1) / 2 + c) * n + i] += graw;
    }
}

/* Per-Gaussian VJP entry point: g2d is [n][9] (du, dv, dQxx, dQxy, dQyy, dalpha_c, dr, dg, db). */
void orc_record_vjp(int64_t n, const double *params, const orc_camera *cam, const orc_settings *s,
                    const double *g2d, double *grad) {
  sh_init();
  memset(grad, 0, sizeof(double) * NROWS * n);
  for (int64_t i = 0; i < n; i++) {
    int any = 0;
    for (int c = 0; c < NG2D; c++) any |= g2d[NG2D * i + c] != 0.0;
    if (any) record_vjp(params, n, i, cam, s, g2d + NG2D * i, grad); /* else it adds nothing */
  }
}

/* Full backward for the listed pixels with upstream dL/dC ([npix][3]):
 * writes grad ([76][n], overwritten) and, if g2d_out != NULL, the per-Gaussian
 * 2D gradients ([n][9]). */
int orc_backward(int64_t n, const double *params, const orc_camera *cam, const orc_settings *s, int64_t npix,
                 const int64_t *pix, const double *dl_dc, double *grad, double *g2d_out, int nthreads_req) {
  sh_init();
  double *rec = malloc(sizeof(double) * NREC * (n > 0 ? n : 1));
  int64_t *order = malloc(sizeof(int64_t) * (n > 0 ? n : 1));
  if (!rec || !order) return -1;
  orc_preprocess(n, params, cam, s, rec);
  int64_t m = global_order(n, rec, order, 0);
  sorted_rec *sr = make_sorted(rec, order, m);
  int nt = num_threads(nthreads_req);
  pthread_t *th = malloc(sizeof(pthread_t) * nt);
  job *jobs = malloc(sizeof(job) * nt);
  double *acc = calloc((size_t)nt * NG2D * (n > 0 ? n : 1), sizeof(double));
  if (!acc) return -1;
  for (int t = 0; t < nt; t++) {
    job jb;
    memset(&jb, 0, sizeof(jb));
    jb.sr = sr; jb.m = m; jb.cam = cam; jb.s = s; jb.npix = npix; jb.pix = pix; jb.nthreads = nt; jb.tid = t;
    jb.dl_dc = dl_dc; jb.rec = rec; jb.order = order; jb.g2d = acc + (size_t)t * NG2D * n;
    jobs[t] = jb;
    pthread_create(&th[t], NULL, bwd_worker, &jobs[t]);
  }
  for (int t = 0; t < nt; t++) pthread_join(th[t], NULL);
  double *g2 = calloc((size_t)NG2D * (n > 0 ? n : 1), sizeof(double));
  for (int t = 0; t < nt; t++)
    for (int64_t k = 0; k < NG2D * n; k++) g2[k] += acc[(size_t)t * NG2D * n + k];
  memset(grad, 0, sizeof(double) * NROWS * n);
  for (int64_t i = 0; i < n; i++) record_vjp(params, n, i, cam, s, g2 + NG2D * i, grad);
  if (g2d_out) memcpy(g2d_out, g2, sizeof(double) * NG2D * n);
  free(g2); free(acc); free(th); free(jobs); free(sr); free(order); free(rec);
  return 0;
}
