/*
 * sixdgs.h -- C ABI of the MI355X (gfx950) renderer for view-conditioned 6D
 * Gaussians: forward render, its backward, an L1 loss and an Adam step.
 *
 * The method: each 6D Gaussian (position mu_p, direction mu_d, 6x6 covariance
 * Sigma = L L^T, opacity, SH colour; Sec. 3.1 and Sec. 4.2) is sliced for the
 * camera's view direction into a conditional 3D Gaussian (conditional mean,
 * Schur-complement covariance, opacity scaled by
 * exp(-lambda (d-mu_d)^T Sigma_d^-1 (d-mu_d)); Sec. 3.2 eq:mu, eq:sigma,
 * eq:alpha, Sec. 4.2 eq:pdfv2, Algorithm 1) which the 3D Gaussian splatting
 * rasteriser then draws (Sec. 4.4): EWA projection, binning into screen tiles
 * ordered by (tile, depth), and front-to-back alpha compositing.
 *
 * Conventions shared by every entry point
 *   - Parameters are one device buffer of float32 in structure-of-arrays
 *     layout [76][n]: row r of Gaussian i at params[r*n + i].  Rows: 0-2 mu_p,
 *     3-5 mu_d, 6-26 raw lower-triangular Cholesky entries of the 6x6 factor
 *     (entry (i,j), j<=i, at row 6 + i(i+1)/2 + j; the diagonal goes through
 *     exp, the rest through 2*sigmoid(r)-1), 27-74 SH coefficients (basis k,
 *     channel c at row 27 + 3k + c; colour = sigmoid of the expansion), 75 the
 *     opacity logit (opacity = sigmoid).
 *   - Cameras are host structs: world -> camera p = R x + t (R row-major),
 *     OpenCV axes (x right, y down, z forward), pinhole intrinsics; pixel
 *     (i, j) has its centre at (i + 0.5, j + 0.5).
 *   - Images are float32 [3][H][W] in device memory, one buffer per camera,
 *     owned by the caller.
 *   - `stream` is a hipStream_t (NULL = the null stream).  Every call that
 *     takes a stream only enqueues work on it and returns; it does not wait
 *     unless stated.
 *   - Errors: every call returns a status; on failure nothing has been
 *     enqueued (argument checks happen before any launch) unless the status is
 *     SIXDGS_ERR_HIP.  sixdgs_last_error() gives a message.  No C++ exception
 *     crosses this boundary.
 *   - A context is used by one host thread at a time; calls on one context
 *     must be issued on streams ordered with each other.
 */
#ifndef SIXDGS_H
#define SIXDGS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sixdgs_status;
#define SIXDGS_OK 0
#define SIXDGS_ERR_INVALID_ARG 1 /* bad pointer, size, camera or setting */
#define SIXDGS_ERR_OOM 2         /* device allocation failed */
#define SIXDGS_ERR_HIP 3         /* a HIP runtime call failed */
#define SIXDGS_ERR_CAPACITY 4    /* fixed pair capacity was exceeded (output invalid) */
#define SIXDGS_ERR_STATE 5       /* backward without a matching forward, etc. */
#define SIXDGS_ERR_DEBUG 6       /* a debug-mode check failed (SIXDGS_FLAG_DEBUG): a workspace
                                    guard was overwritten or a binning invariant does not hold */

#define SIXDGS_NROWS 76
#define SIXDGS_ROW_MU_P 0
#define SIXDGS_ROW_MU_D 3
#define SIXDGS_ROW_L 6
#define SIXDGS_ROW_SH 27
#define SIXDGS_ROW_OPACITY 75
#define SIXDGS_MAX_VIEWS 16 /* cameras per forward call */

typedef struct sixdgs_ctx sixdgs_ctx;

typedef struct {
  float R[9];   /* world -> camera rotation, row-major */
  float t[3];   /* world -> camera translation */
  float fx, fy; /* focal lengths in pixels */
  float cx, cy; /* principal point in pixels */
  int32_t width, height;
} sixdgs_camera;

typedef struct {
  float lambda_opa;    /* directional opacity strength (Sec. 4.2; paper uses 0.35), in [0, 1] */
  float z_near;        /* camera-space depth below which a Gaussian is culled (0.2) */
  float bg[3];         /* background colour */
  int32_t tile_w;      /* screen tile width in pixels: 8, 16 or 32 */
  int32_t tile_h;      /* screen tile height: tile_w * tile_h must be 256 */
  int32_t batch;       /* Gaussians staged in LDS per backward batch: 64, 128 or 256;
                          0: automatic (128 below 16,384 tiles in the call's
                          views, 256 from there on; never above the chunk) */
  int64_t pair_capacity; /* 0: grow the (tile, Gaussian) pair buffers on demand
                            (sixdgs_forward then waits once on the stream to
                            read the pair count); > 0: fixed capacity, no host
                            waits (capturable), overflow reported as
                            SIXDGS_ERR_CAPACITY by sixdgs_check().  At most
                            2^30 - 1 pairs either way (CAPACITY beyond). */
  int32_t flags;       /* SIXDGS_FLAG_* */
  int32_t chunk;       /* list positions per backward work item: the backward
                          walks each tile's list in chunks of this length in
                          parallel, restarting from state the forward saves at
                          chunk starts.  A power of two, >= batch (and 64),
                          <= 16384; 0: automatic (128 below 16,384 tiles,
                          512 from there on). */
} sixdgs_settings;

#define SIXDGS_FLAG_COUNTS 1 /* forward also stores per-pixel contributor counts (debug export) */
/* No-SH colour (the Sec. 5 ablation): each Gaussian's colour is sigmoid(c) of
 * its own RGB triple c, held in the three SH degree-0 rows (27-29); the 45
 * higher SH rows are ignored and receive zero gradient.  Without the flag the
 * colour is the sigmoid of the degree-3 SH expansion (Sec. 4.2). */
#define SIXDGS_FLAG_RGB_COLOR 2
/* Debug mode, for finding indexing faults without a GPU debugger.  Every
 * workspace buffer the context allocates is padded with 4 KiB guards of a
 * fixed byte before and after it.  After each call on the context that
 * launches work, the host waits for the stream and reads every guard back.
 * After a forward or sixdgs_bin it also checks the integer stage's outputs
 * against sixdgs_debug_check_bins (and, after a forward, each pixel's last
 * contributor and final transmittance against its tile).  A failure returns
 * SIXDGS_ERR_DEBUG with a message that names the buffer or the invariant.
 * Results are bitwise those of the normal mode.  Each call waits for its
 * stream, so the mode is for tests, not for speed.  Turning the flag on or off
 * with sixdgs_set_settings frees the workspace, which drops the state of the
 * last forward. */
#define SIXDGS_FLAG_DEBUG 4

/* Fills `s` with the defaults: lambda 0.35, z_near 0.2, bg 0, 16x16 tiles,
 * batch 0 (automatic), pair_capacity 0, flags 0, chunk 0 (automatic). */
void sixdgs_default_settings(sixdgs_settings* s);

/* Creates a context on the current HIP device.  It owns all scratch memory
 * and the state one forward leaves for the matching backward.  `s` may be
 * NULL (defaults).  Returns INVALID_ARG for unsupported settings. */
sixdgs_status sixdgs_create(sixdgs_ctx** out, const sixdgs_settings* s);

/* Frees the context and its device memory (waits for the device first). */
void sixdgs_destroy(sixdgs_ctx* ctx);

/* Replaces the settings; takes effect at the next forward. */
sixdgs_status sixdgs_set_settings(sixdgs_ctx* ctx, const sixdgs_settings* s);

/* Message for the last failed call on this context (never NULL). */
const char* sixdgs_last_error(const sixdgs_ctx* ctx);

/* Forward render (Sec. 3.2 / Algorithm 1 slice, then the 3DGS rasteriser of
 * Sec. 4.4) of n Gaussians into ncam (1..SIXDGS_MAX_VIEWS) cameras.
 *   params  device [76][n], read only, must stay unchanged until the matching
 *           backward has run.
 *   cams    host array of ncam cameras.
 *   images  host array of ncam device pointers, each [3][H][W], overwritten.
 * n * ncam must stay below 2^30 (INVALID_ARG otherwise).  Keeps, inside ctx, the per-view projected records, the sorted (tile,
 * Gaussian) lists and the per-pixel final transmittance and last-contributor
 * index that the backward consumes; they stay valid until the next forward or
 * sixdgs_bin on this context. */
sixdgs_status sixdgs_forward(sixdgs_ctx* ctx, const float* params, int64_t n, const sixdgs_camera* cams,
                             int32_t ncam, float* const* images, void* stream);

/* sixdgs_forward with the training step's L1 loss (the L1 term of the 3DGS
 * loss that Sec. 4.4 and Sec. 5.1 keep) formed as each pixel is written,
 * instead of by a separate sixdgs_l1_loss over the rendered images:
 * targets[k] (device [3][H][W], read only) are the reference images,
 * dl_dimages[k] (device [3][H][W], overwritten) receive dL/dI = sign(I - I*) /
 * total_count, and the device float `loss` receives mean |I - I*| over every
 * element of every view, the same values sixdgs_l1_loss gives for the
 * rendered images (the loss summed per tile, so its last bits may differ).
 * The state for the backward is kept as by sixdgs_forward.  INVALID_ARG as
 * sixdgs_forward, or for a NULL targets, dl_dimages, loss or per-view
 * pointer. */
sixdgs_status sixdgs_forward_l1(sixdgs_ctx* ctx, const float* params, int64_t n, const sixdgs_camera* cams,
                                int32_t ncam, float* const* images, const float* const* targets,
                                float* const* dl_dimages, float* loss, void* stream);

/* Inference cache (Algorithm 1's caption notes that the slice's
 * direction-independent part can be computed once per Gaussian): writes, for
 * each of the n Gaussians in params (device [76][n]), the rows of
 * cache (device [SIXDGS_CACHE_ROWS][n], caller-owned, overwritten):
 *   0-5   Sigma_cond = Sigma_p - Sigma_pd Sigma_d^-1 Sigma_pd^T (xx xy xz yy yz zz)
 *   6-14  K = Sigma_pd Sigma_d^-1, row-major
 *   15-20 Sigma_d^-1 (xx xy xz yy yz zz)
 *   21    alpha = sigmoid(opacity logit)
 * Asynchronous on `stream`; INVALID_ARG for n < 0 or NULL pointers with n > 0.
 * The cache is a function of the Cholesky and opacity rows only: rebuild it
 * after they change. */
#define SIXDGS_CACHE_ROWS 22
sixdgs_status sixdgs_build_cache(const float* params, int64_t n, float* cache, void* stream);

/* Render-only forward from the inference cache: the images of sixdgs_forward
 * (bit-identical for a cache built from the same params), with the per-view
 * work reduced to the conditional mean, the directional opacity, the colour
 * and the projection, and none of the state a backward needs kept (the next
 * sixdgs_backward on this context returns STATE).  params supplies the mean
 * and colour rows.  Takes the scalar lambda_opa: STATE while a per-Gaussian
 * lambda array is attached. */
sixdgs_status sixdgs_forward_cached(sixdgs_ctx* ctx, const float* params, const float* cache, int64_t n,
                                    const sixdgs_camera* cams, int32_t ncam, float* const* images, void* stream);

/* Backward of the last forward on this context (the derivative of the
 * Sec. 4.4 compositing, then of the projection, the SH colour of Sec. 4.2, the
 * slice of Sec. 3.2 eq:mu / eq:sigma and the directional opacity of Sec. 4.2
 * eq:pdfv2, into the raw parameters of Sec. 3.1): given dL/dI for each of its
 * ncam cameras (host array of ncam device pointers, each [3][H][W] of that
 * camera), writes dL/d params into `grad` (device [76][n], overwritten).
 * `params`, `n` and `ncam` must be those of the forward (STATE for other
 * params / n, INVALID_ARG for another ncam); the dL/dI buffers must hold
 * the forward's image sizes (not checkable here).  If `densify` is not NULL
 * (device [2][n]) it adds, per Gaussian, the norm of its screen-space mean
 * gradient in normalised device units (row 0) and the number of views it was
 * visible in (row 1) -- the statistics the adaptive density control of Sec. 4.3
 * consumes. */
sixdgs_status sixdgs_backward(sixdgs_ctx* ctx, const float* params, int64_t n, int32_t ncam,
                              const float* const* dl_dimages, float* grad, float* densify, void* stream);

/* Backward of the last forward fused with one Adam step: the training step of
 * Sec. 5.1 (the paper trains with Adam, learning rate 1e-2 for the 6D
 * covariance and 1e-3 for the direction mean, 3DGS defaults elsewhere) in the
 * form of sixdgs_backward followed by sixdgs_adam.  The per-Gaussian gradient
 * is applied to params, m and v (device [76][n] each, updated in place) as it
 * is produced and never written to memory.  params must be the pointer the
 * forward rendered (it is modified here, so the forward's saved state is spent:
 * a further backward needs a new forward).  ncam and dl_dimages as in
 * sixdgs_backward; lr, beta1, beta2, eps and step as in sixdgs_adam; densify
 * as in sixdgs_backward. */
sixdgs_status sixdgs_backward_adam(sixdgs_ctx* ctx, float* params, int64_t n, int32_t ncam,
                                   const float* const* dl_dimages, float* m, float* v, const float* lr, float beta1,
                                   float beta2, float eps, int32_t step, float* densify, void* stream);

/* sixdgs_backward_adam with the step count on the device, for training steps
 * captured in a graph (Sec. 5.1 training with Adam): the bias correction uses
 * step = *step_counter + 1 (step_counter: device int32, required).  With
 * advance != 0 the kernel's last workgroup increments *step_counter once every
 * workgroup has read it; with advance = 0 the counter is left for the caller
 * to advance (e.g. after another Adam that shares the step, sixdgs_adam_vec).
 * Other arguments and errors as sixdgs_backward_adam. */
sixdgs_status sixdgs_backward_adam_devstep(sixdgs_ctx* ctx, float* params, int64_t n, int32_t ncam,
                                           const float* const* dl_dimages, float* m, float* v, const float* lr,
                                           float beta1, float beta2, float eps, int32_t* step_counter,
                                           int32_t advance, float* densify, void* stream);

/* Learnable per-Gaussian lambda (Sec. 4.2; the paper trains it over a window
 * of iterations, Sec. 5.1).  lambda_raw: device [n] float32 raw values for the
 * following forwards on this context, Gaussian i using lambda =
 * sigmoid(lambda_raw[i]) in place of settings.lambda_opa; NULL restores the
 * scalar setting.  grad_lambda: device [n], or NULL; each backward (and
 * backward_adam) of a forward that used lambda_raw overwrites it with
 * dL/dlambda_raw.  Both arrays stay owned by the caller, must hold the n of
 * the forwards, and lambda_raw must not change between a forward and its
 * backward.  INVALID_ARG for grad_lambda without lambda_raw. */
sixdgs_status sixdgs_set_lambda(sixdgs_ctx* ctx, const float* lambda_raw, float* grad_lambda);

/* ---- adaptive density control (Sec. 4.3) ------------------------------ */

/* Rotation and scale of every Gaussian from the SVD of its conditional
 * covariance (direction independent): Sigma_cond = R diag(S^2) R^T with S
 * descending, R proper (det +1).  The SVD fixes each axis only up to sign;
 * here the first two axes have their largest component positive and the third
 * is their cross product -- the paper's sign(det R) correction of the last
 * column.  params: device [76][n]; R: device [9][n] (row-major entries),
 * S: device [3][n], both overwritten. */
sixdgs_status sixdgs_decompose(const float* params, int64_t n, float* R, float* S, void* stream);

typedef struct {
  float grad_threshold; /* densify when the mean screen-space gradient norm over the
                           views a Gaussian was visible in reaches this (3DGS: 2e-4) */
  float percent_dense;  /* clone when max(S) <= percent_dense * extent, else split (0.01) */
  float extent;         /* scene extent in world units */
  float min_opacity;    /* prune when sigmoid(opacity logit) < this (Sec. 5.1: 0.01) */
} sixdgs_density_settings;

/* Plans one density-control step: per Gaussian prune (0 outputs), keep (1),
 * clone (the Gaussian and an identical copy) or split (two children whose
 * spatial means are mu_p + R (S * z_k) and whose spatial Cholesky block L_p
 * is divided by 1.6, so S shrinks by 1.6 and R is kept), from stats (device
 * [2][n]: the summed screen-space gradient norm and the visible-view count
 * that sixdgs_backward accumulates into `densify`).  Waits for the stream and
 * writes the number of output Gaussians to *n_out (host).  The plan stays in
 * ctx for the next sixdgs_densify_apply with the same params and n. */
sixdgs_status sixdgs_densify_plan(sixdgs_ctx* ctx, const float* params, int64_t n, const float* stats,
                                  const sixdgs_density_settings* settings, int64_t* n_out, void* stream);

/* Applies the planned step: params_out (device [76][n_out]) receives the
 * outputs in the parents' order, each parent's outputs consecutive.  noise:
 * device [2][3][n] standard normal draws (z_0, z_1 of a split).  m, v (device
 * [76][n], Adam moments) and m_out, v_out: all four or none; moments are kept
 * for kept Gaussians and the first output of a clone and zero for clone copies
 * and split children.  lambda_raw ([n]) / lambda_out ([n_out]): both or
 * neither; copied to every output.  STATE without a matching plan. */
sixdgs_status sixdgs_densify_apply(sixdgs_ctx* ctx, const float* params, const float* m, const float* v,
                                   const float* lambda_raw, int64_t n, const float* noise, float* params_out,
                                   float* m_out, float* v_out, float* lambda_out, int64_t n_out, void* stream);

/* L1 photometric loss (the L1 term of the 3DGS loss that Sec. 4.4 and Sec. 5.1
 * keep) over nimg (1..SIXDGS_MAX_VIEWS) image pairs: loss = mean |I - I*|
 * over every element of every image (written to the device float `loss`),
 * and dL/dI = sign(I - I*) / total_count written to dl_dimages[k] (may alias
 * nothing else).  numel[k] is the element count of image k (host array).
 * INVALID_ARG for nimg out of range, NULL pointers or numel <= 0. */
sixdgs_status sixdgs_l1_loss(sixdgs_ctx* ctx, int32_t nimg, const float* const* images, const float* const* targets,
                             const int64_t* numel, float* const* dl_dimages, float* loss, void* stream);

/* sixdgs_l1_loss without a context and without any allocation, for callers
 * that cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, result and
 * asynchrony as sixdgs_l1_loss.  Its scratch (the per-workgroup partial sums)
 * is a fixed 64 KiB array in device memory of every GPU the library runs on,
 * held until the process ends, sized for the largest call (SIXDGS_MAX_VIEWS
 * images of any size): a call never needs more (it returns
 * SIXDGS_ERR_CAPACITY if it ever would, before any launch).  The array is
 * shared by all calls on one GPU and keeps the last call's contents; calls
 * whose executions overlap on one GPU (different streams, or different host
 * threads, without ordering between them) race on it, so order them.
 * INVALID_ARG as sixdgs_l1_loss; SIXDGS_ERR_HIP if the array's device address
 * cannot be looked up or the launch fails. */
sixdgs_status sixdgs_l1_loss_noalloc(int32_t nimg, const float* const* images, const float* const* targets,
                                     const int64_t* numel, float* const* dl_dimages, float* loss, void* stream);

/* The full 3DGS photometric loss (Sec. 4.4, Sec. 5.1: the paper keeps it):
 * loss = (1 - lambda_dssim) L1 + lambda_dssim (1 - SSIM) over nimg
 * (1..SIXDGS_MAX_VIEWS) views, both terms means over every channel and pixel
 * of every view (3DGS: lambda_dssim = 0.2).  SSIM per channel and pixel under
 * an 11x11 Gaussian window (sigma 1.5) zero-padded at the border, C1 = 1e-4,
 * C2 = 9e-4.  images / targets / dl_dimages: host arrays of device pointers,
 * each [3][heights[k]][widths[k]]; dl_dimages[k] is overwritten with dL/dI;
 * loss is one device float.  Scratch (36 B per pixel) is owned by ctx. */
sixdgs_status sixdgs_l1_dssim_loss(sixdgs_ctx* ctx, int32_t nimg, const float* const* images,
                                   const float* const* targets, const int32_t* heights, const int32_t* widths,
                                   float lambda_dssim, float* const* dl_dimages, float* loss, void* stream);

/* One Adam step (Kingma and Ba, bias-corrected; the optimiser of Sec. 5.1,
 * whose learning rates are 1e-2 for the 6D covariance and 1e-3 for the
 * direction mean, with the 3DGS defaults elsewhere) on params [76][n] in
 * place, with moments m, v (device [76][n], updated in place; zero before
 * step 1).  lr[6] (host) holds the learning rate of the row groups mu_p, mu_d,
 * Cholesky, SH degree 0, SH degree 1-3, opacity.  step counts from 1.
 * INVALID_ARG for NULL pointers with n > 0, step < 1 or betas outside [0, 1). */
sixdgs_status sixdgs_adam(float* params, const float* grad, float* m, float* v, int64_t n, const float* lr,
                          float beta1, float beta2, float eps, int32_t step, void* stream);

/* sixdgs_adam (the Sec. 5.1 optimiser step) with the step count kept on the
 * device: step_counter (device int32, 0 before the first step) holds the
 * number of steps taken; this call takes step *step_counter + 1 and then
 * increments the counter, all on the stream.  Nothing about the step is baked
 * into the launch, so a captured graph of a training step advances Adam on
 * every replay.  Errors as sixdgs_adam. */
sixdgs_status sixdgs_adam_devstep(float* params, const float* grad, float* m, float* v, int64_t n, const float* lr,
                                  float beta1, float beta2, float eps, int32_t* step_counter, void* stream);

/* Adam on one vector of n floats with one learning rate (e.g. the learnable
 * lambda's raw values).  The bias correction uses `step` (from 1), or, when
 * step_counter (device int32) is not NULL, *step_counter + 1 without changing
 * the counter: called before sixdgs_adam_devstep, it shares that training
 * step's count.  p, m, v are updated in place (device [n]). */
sixdgs_status sixdgs_adam_vec(float* p, const float* g, float* m, float* v, int64_t n, float lr, float beta1,
                              float beta2, float eps, int32_t step, const int32_t* step_counter, void* stream);

/* The integer stage alone, on caller-given projected records: bins entries
 * e = view*n + i (arrays of length n*ncam, device) with extents (u +- ex,
 * v +- ey) into the cameras' tile grids, keyed by (tile, float32 depth bits,
 * e), sorts and builds per-tile ranges, exactly as sixdgs_forward does after
 * its projection.  alive[e] != 0 marks entries that take part.  Results are
 * read back with sixdgs_export. */
sixdgs_status sixdgs_bin(sixdgs_ctx* ctx, int64_t n, const sixdgs_camera* cams, int32_t ncam, const float* u,
                         const float* v, const float* ex, const float* ey, const float* depth, const int32_t* alive,
                         void* stream);

/* What sixdgs_export copies out (synchronous: waits for the context's last
 * stream).  Element types and counts:
 *   RECORDS      float  [E][12]: u, v, Qxx, Qxy, Qyy, alpha_cond, ex, ey, r, g, b, depth
 *                (E = n*ncam; rows of entries that are not binned are undefined)
 *   TILES        int32  [E]: tiles touched per entry (0 = culled)
 *   KEYS         uint64 [P]: sorted (global tile << 32 | depth bits)
 *   VALUES       int32  [P]: entry ids in key order
 *   RANGES       int32  [T][2]: per global tile [start, end) into KEYS
 *   T_FINAL      float  [sum H*W]: final transmittance per pixel, views in order
 *   LAST         int32  [sum H*W]: 1 + position (within its tile's range) of the
 *                last contributor, 0 if none
 *   COUNTS       int32  [sum H*W]: contributors per pixel (SIXDGS_FLAG_COUNTS)
 *   SIZES        int64  [7]: E, P, T, number of binned entries, pixels, and
 *                the backward batch depth and chunk the last forward chose */
#define SIXDGS_EXPORT_RECORDS 0
#define SIXDGS_EXPORT_TILES 1
#define SIXDGS_EXPORT_KEYS 2
#define SIXDGS_EXPORT_VALUES 3
#define SIXDGS_EXPORT_RANGES 4
#define SIXDGS_EXPORT_T_FINAL 5
#define SIXDGS_EXPORT_LAST 6
#define SIXDGS_EXPORT_COUNTS 7
#define SIXDGS_EXPORT_SIZES 8
/* Copies item `what` into host memory `dst` of `cap_bytes` bytes; *written
 * receives the byte count.  Returns INVALID_ARG if it does not fit. */
sixdgs_status sixdgs_export(sixdgs_ctx* ctx, int32_t what, void* dst, int64_t cap_bytes, int64_t* written);

/* Host copies of the integer stage's outputs for one binning: E entries
 * (entry e = view * n + gaussian), P (tile, entry) pairs, T global tiles.
 * Rows are as sixdgs_export writes them. */
typedef struct {
  int64_t E, P, T;
  const uint32_t* tiles;   /* [E] tiles each entry touches */
  const float* depth;      /* [E] camera depth of each entry (the depth sort's key) */
  const uint32_t* keys;    /* [P] global tile id of each sorted pair */
  const uint32_t* values;  /* [P] entry id of each sorted pair */
  const uint32_t* ranges;  /* [2T] [start, end) of each tile's run of pairs, (0, 0) if none */
  const uint32_t* order;   /* [T] the compositing order of the tiles, or NULL (not checked) */
  int32_t chunk;           /* the backward's chunk length (with nch and items) */
  const uint32_t* nch;     /* [T] backward chunks per tile, or NULL (no work items) */
  const uint32_t* items;   /* [2 n_items] (tile, chunk) work items */
  int64_t n_items;
} sixdgs_bin_state;

/* Checks the invariants of one binning (the tile binning and (tile, depth)
 * sort of the 3DGS rasteriser, Sec. 4.4, and the backward's chunked work
 * items) on host copies, without a GPU:
 *   - the tile counts sum to P;
 *   - pairs are sorted by tile, and within a tile by (depth, entry id), with
 *     tile ids below T and entry ids below E;
 *   - each entry appears in exactly tiles[e] pairs;
 *   - every range is the exact run of its tile's pairs;
 *   - the order, if given, is a permutation with list lengths of
 *     non-increasing bit length;
 *   - each tile, if nch is given, has at most ceil(run / chunk) chunks, and
 *     the items hold every (t, c) with c < nch[t] exactly once, in any order.
 * Returns SIXDGS_OK, SIXDGS_ERR_DEBUG with the first violation written to
 * msg (NUL-terminated, at most msg_cap bytes, if msg is not NULL), or
 * SIXDGS_ERR_INVALID_ARG for a NULL or inconsistent state.  The debug mode
 * runs it after every binning. */
sixdgs_status sixdgs_debug_check_bins(const sixdgs_bin_state* state, char* msg, int32_t msg_cap);

/* Debug mode only: the device address and byte size of the workspace buffer
 * called `name` (as debug-mode messages name them, e.g. "ranges"), so that a
 * test can check that the guard checks see a write placed just outside it
 * with hipMemcpy.  Returns SIXDGS_ERR_STATE outside the debug mode or before
 * the buffer exists, and INVALID_ARG for an unknown name. */
sixdgs_status sixdgs_debug_buffer(sixdgs_ctx* ctx, const char* name, void** ptr, int64_t* bytes);

/* Waits for the context's last stream and reports a capacity overflow of the
 * fixed-capacity mode (SIXDGS_ERR_CAPACITY), or a sort pass whose bounded
 * wait on an earlier workgroup ran out (SIXDGS_ERR_HIP); the flag is then
 * cleared.  In the debug mode it also checks every workspace guard
 * (SIXDGS_ERR_DEBUG). */
sixdgs_status sixdgs_check(sixdgs_ctx* ctx);

/* Kernel timing with HIP events recorded on the launch stream around the
 * chosen kernels (ids SIXDGS_K_*); off by default.  sixdgs_kernel_time waits
 * for the stream and returns the summed milliseconds and launch count since
 * the last reset. */
#define SIXDGS_K_PREPROCESS 0
#define SIXDGS_K_BLEND_FWD 1
#define SIXDGS_K_BLEND_BWD 2
#define SIXDGS_K_PREPROCESS_BWD 3
#define SIXDGS_K_SORT 4 /* whole integer stage: compaction, both sorts, ranges */
#define SIXDGS_K_COUNT 5
sixdgs_status sixdgs_set_timing(sixdgs_ctx* ctx, int32_t kernel_mask);
sixdgs_status sixdgs_kernel_time(sixdgs_ctx* ctx, int32_t kernel, double* ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* SIXDGS_H */
