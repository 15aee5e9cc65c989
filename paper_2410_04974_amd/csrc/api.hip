// C ABI of the renderer: argument checks, workspace ownership, the order of the
// stages on the caller's stream, and read-back for tests.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "internal.h"

using namespace sixdgs;

namespace {

// Debug mode: guards of kGuardBytes bytes of kGuardByte before and after
// every workspace buffer.
constexpr size_t kGuardBytes = 4096;
constexpr uint8_t kGuardByte = 0xA7;

template <class T>
struct DevBuf {
  T* p = nullptr;
  int64_t cap = 0;
  bool guarded = false;     // allocate with guards (set while the buffer is empty)
  uint8_t* raw = nullptr;   // the allocation: front guard, cap elements, back guard
  // Grows to at least `count` elements (contents are not kept).
  bool ensure(int64_t count, double slack = 1.0) {
    if (count <= cap) return true;
    release();
    int64_t want = (int64_t)std::ceil((double)count * slack);
    if (want < 1) want = 1;
    const size_t bytes = (size_t)want * sizeof(T), pad = guarded ? kGuardBytes : 0;
    if (hipMalloc((void**)&raw, bytes + 2 * pad) != hipSuccess) {
      raw = nullptr;
      return false;
    }
    if (pad && (hipMemset(raw, kGuardByte, pad) != hipSuccess ||
                hipMemset(raw + pad + bytes, kGuardByte, pad) != hipSuccess)) {
      release();
      return false;
    }
    p = (T*)(raw + pad);
    cap = want;
    return true;
  }
  void release() {
    if (raw) (void)hipFree(raw);
    raw = nullptr;
    p = nullptr;
    cap = 0;
  }
  int64_t bytes() const { return cap * (int64_t)sizeof(T); }
  // Reads both guards back (synchronously); "" if they are intact.
  std::string guard_damage(const char* name) const {
    if (!guarded || !raw) return "";
    std::vector<uint8_t> h(kGuardBytes);
    for (int side = 0; side < 2; side++) {
      const uint8_t* src = side == 0 ? raw : raw + kGuardBytes + bytes();
      if (hipMemcpy(h.data(), src, kGuardBytes, hipMemcpyDeviceToHost) != hipSuccess)
        return std::string("guard read-back of ") + name + " failed";
      for (size_t i = 0; i < kGuardBytes; i++)
        if (h[i] != kGuardByte) {
          const int64_t off = side == 0 ? -(int64_t)(kGuardBytes - i) : (int64_t)i;
          return std::string(name) + (side == 0 ? ": written before its start (byte " : ": written past its end (byte ") +
                 std::to_string(off) + (side == 0 ? ")" : " after the end)");
        }
    }
    return "";
  }
};

struct TimedLaunch {
  int kernel;
  hipEvent_t a, b;
};

}  // namespace

struct sixdgs_ctx {
  sixdgs_settings s;
  std::string err;
  // per-entry workspace
  DevBuf<Rec> rec;
  DevBuf<uint32_t> tiles, dkey0, dkey1, dval0, dval1, poff;
  DevBuf<float> depth;                  // [E] camera depth per entry (written by the preprocess)
  const float* bin_depth = nullptr;     // the caller's depth array during sixdgs_bin
  // per-pair workspace
  DevBuf<uint32_t> pkey0, pkey1, pval0, pval1;
  DevBuf<uint2> ranges;
  // per-pixel state
  DevBuf<float> T_final;
  DevBuf<uint32_t> last, counts;
  // backward work items: chunk-boundary state, per-tile chunk counts, (tile, chunk) list
  DevBuf<float4> bound;
  DevBuf<uint32_t> tile_nch;
  DevBuf<uint2> items;
  int64_t bwd_grid = 0;
  int32_t fwd_chunk = 256;   // chunk length the last forward saved its boundary state for
  int32_t fwd_batch = 256;   // LDS batch depth of the last forward's backward
  // learnable per-Gaussian lambda (caller-owned device arrays, sixdgs_set_lambda)
  const float* lambda_raw = nullptr;
  float* grad_lambda = nullptr;
  const float* fwd_lambda = nullptr;  // what the last forward used
  // density control: the last plan (decision, output count and offset per Gaussian)
  DevBuf<uint8_t> dens_dec;
  DevBuf<uint32_t> dens_cnt, dens_off, dens_state;
  const float* dens_params = nullptr;
  int64_t dens_n = -1, dens_total = -1;
  // backward and loss
  DevBuf<float> g2d, l1_partial, ssim_maps, ssim_partial;
  // scratch
  DevBuf<uint32_t> rstate, blk_start, counters, tile_order, order_state;
  uint32_t* host_counters = nullptr;  // pinned
  // state of the last forward
  bool have_fwd = false;
  float* bin_g2d = nullptr;  // the gradient accumulators the binning clears (training forwards)
  bool g2d_clean = false;    // g2d is zero for the binned entries of the last forward
  bool counts_valid = false;
  const float* fwd_params = nullptr;
  int64_t fwd_n = 0;
  int64_t fwd_E = 0;
  int64_t fwd_px = 0;
  ViewTable vt{};
  SortBuffers sb{};
  hipStream_t stream = nullptr;
  // timing
  int32_t timing_mask = 0;
  std::vector<TimedLaunch> pending;
  std::vector<hipEvent_t> free_events;
  double ms[SIXDGS_K_COUNT] = {0};
  int64_t launches[SIXDGS_K_COUNT] = {0};
  bool debug = false;  // SIXDGS_FLAG_DEBUG: guarded workspace, checks after every call
};

namespace {
// Every workspace buffer of the context with the name debug-mode messages use.
template <class F>
void for_each_buf(sixdgs_ctx* c, F f) {
  f(c->rec, "records");
  f(c->tiles, "tiles");
  f(c->dkey0, "depth keys 0");
  f(c->dkey1, "depth keys 1");
  f(c->dval0, "depth values 0");
  f(c->dval1, "depth values 1");
  f(c->poff, "pair offsets");
  f(c->depth, "depth");
  f(c->pkey0, "pair keys 0");
  f(c->pkey1, "pair keys 1");
  f(c->pval0, "pair values 0");
  f(c->pval1, "pair values 1");
  f(c->ranges, "ranges");
  f(c->T_final, "final transmittance");
  f(c->last, "last contributor");
  f(c->counts, "contributor counts");
  f(c->bound, "chunk boundary state");
  f(c->tile_nch, "tile chunk counts");
  f(c->items, "work items");
  f(c->dens_dec, "density decisions");
  f(c->dens_cnt, "density counts");
  f(c->dens_off, "density offsets");
  f(c->dens_state, "density scan state");
  f(c->g2d, "screen-space gradients");
  f(c->l1_partial, "l1 partial sums");
  f(c->ssim_maps, "ssim maps");
  f(c->ssim_partial, "ssim partial sums");
  f(c->rstate, "sort state");
  f(c->blk_start, "emission block starts");
  f(c->counters, "counters");
  f(c->tile_order, "tile order");
  f(c->order_state, "tile order state");
}
}  // namespace

namespace {

sixdgs_status fail(sixdgs_ctx* c, sixdgs_status st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

// counters: [0] binned entries, [1] pairs, [2] pair overflow flag, [3] look-back
// timeout flag, [4] backward work items, [5] density-control outputs, [6] the
// fused backward + Adam's finished workgroups (zero between launches)
constexpr int kCounters = 8;

// Bound on entries and pairs: the radix sort's look-back words hold 30-bit counts.
constexpr int64_t kMaxItems = (1ll << 30) - 1;

bool valid_settings(const sixdgs_settings* s, std::string& why) {
  if (!(s->lambda_opa >= 0.f && s->lambda_opa <= 1.f)) { why = "lambda_opa must lie in [0, 1]"; return false; }
  if (!(s->z_near > 0.f) || !std::isfinite(s->z_near)) { why = "z_near must be positive"; return false; }
  for (int k = 0; k < 3; k++)
    if (!std::isfinite(s->bg[k])) { why = "bg must be finite"; return false; }
  const int tw = s->tile_w, th = s->tile_h;
  if (!((tw == 8 || tw == 16 || tw == 32) && tw * th == 256)) {
    why = "tile shape must be 8x32, 16x16 or 32x8";
    return false;
  }
  if (!(s->batch == 0 || s->batch == 64 || s->batch == 128 || s->batch == 256)) {
    why = "batch must be 0 (automatic), 64, 128 or 256";
    return false;
  }
  if (s->pair_capacity < 0 || s->pair_capacity > kMaxItems) { why = "pair_capacity out of range"; return false; }
  if (s->flags & ~(SIXDGS_FLAG_COUNTS | SIXDGS_FLAG_RGB_COLOR | SIXDGS_FLAG_DEBUG)) {
    why = "unknown flag bits";
    return false;
  }
  if (s->chunk != 0 && (s->chunk < std::max(s->batch, 64) || s->chunk > 16384 || (s->chunk & (s->chunk - 1)) != 0)) {
    why = "chunk must be 0 (automatic) or a power of two between batch (64 at least) and 16384";
    return false;
  }
  return true;
}

int ilog2(int v) {
  int r = 0;
  while ((1 << r) < v) r++;
  return r;
}

// Builds the camera table; returns an empty string or the reason the cameras are rejected.
std::string build_views(const sixdgs_settings& s, int64_t n, const sixdgs_camera* cams, int ncam, ViewTable& vt,
                        int64_t& total_px) {
  if (!cams) return "cams is NULL";
  if (ncam < 1 || ncam > kMaxViews) return "ncam must be in [1, SIXDGS_MAX_VIEWS]";
  std::memset(&vt, 0, sizeof(vt));
  vt.nview = ncam;
  vt.tile_w = s.tile_w;
  vt.tile_h = s.tile_h;
  vt.tile_shift_x = ilog2(s.tile_w);
  vt.tile_shift_y = ilog2(s.tile_h);
  vt.n = n;
  int64_t tiles = 0;
  total_px = 0;
  for (int k = 0; k < ncam; k++) {
    const sixdgs_camera& c = cams[k];
    for (int i = 0; i < 9; i++)
      if (!std::isfinite(c.R[i])) return "camera rotation is not finite";
    for (int i = 0; i < 3; i++)
      if (!std::isfinite(c.t[i])) return "camera translation is not finite";
    if (!(c.fx > 0.f && c.fy > 0.f) || !std::isfinite(c.fx) || !std::isfinite(c.fy) || !std::isfinite(c.cx) ||
        !std::isfinite(c.cy))
      return "camera intrinsics must be finite with positive focal lengths";
    if (c.width <= 0 || c.height <= 0 || c.width > 16384 || c.height > 16384) return "image size out of range";
    ViewDesc& d = vt.v[k];
    for (int i = 0; i < 9; i++) d.R[i] = c.R[i];
    for (int i = 0; i < 3; i++) d.t[i] = c.t[i];
    d.fx = c.fx;
    d.fy = c.fy;
    d.cx = c.cx;
    d.cy = c.cy;
    for (int i = 0; i < 3; i++)
      d.C[i] = (float)(-((double)c.R[i] * c.t[0] + (double)c.R[3 + i] * c.t[1] + (double)c.R[6 + i] * c.t[2]));
    d.limx = (float)(1.3 * (0.5 * (double)c.width) / (double)c.fx);
    d.limy = (float)(1.3 * (0.5 * (double)c.height) / (double)c.fy);
    d.W = c.width;
    d.H = c.height;
    d.ntx = (c.width + s.tile_w - 1) / s.tile_w;
    d.nty = (c.height + s.tile_h - 1) / s.tile_h;
    d.tile_base = (int32_t)tiles;
    d.pix_base = total_px;
    tiles += (int64_t)d.ntx * d.nty;
    total_px += (int64_t)c.width * c.height;
  }
  if (tiles >= (1ll << 24)) return "too many screen tiles";
  vt.total_tiles = (int32_t)tiles;
  if (n < 0) return "n must be >= 0";
  if (n * (int64_t)ncam >= (1ll << 32) - 1) return "n * ncam too large";
  return "";
}

DevSettings dev_settings(const sixdgs_settings& s) {
  DevSettings d;
  d.lambda_opa = s.lambda_opa;
  d.z_near = s.z_near;
  for (int k = 0; k < 3; k++) d.bg[k] = s.bg[k];
  d.rgb_color = (s.flags & SIXDGS_FLAG_RGB_COLOR) != 0;
  d.lambda_raw = nullptr;
  d.grad_lambda = nullptr;
  return d;
}

// from this many tiles on, the automatic backward chunk and batch depth are
// the long ones
constexpr int64_t kAutoTiles = 16384;

bool ensure_entries(sixdgs_ctx* c, int64_t E) {
  const int64_t e1 = E > 0 ? E : 1;
  return c->rec.ensure(e1) && c->tiles.ensure(e1) && c->dkey0.ensure(e1) && c->dkey1.ensure(e1) &&
         c->dval0.ensure(e1) && c->dval1.ensure(e1) && c->poff.ensure(e1) && c->depth.ensure(e1);
}

bool ensure_scratch(sixdgs_ctx* c, int64_t E, int64_t pcap) {
  const int64_t e1 = std::max<int64_t>(E, 1);
  const int64_t p1 = std::max<int64_t>(pcap, 1);
  return c->rstate.ensure(sort_state_words(e1, false) + sort_state_words(p1, true)) &&
         c->blk_start.ensure(sort_block_starts(p1));
}

BlendState blend_state(sixdgs_ctx* c) {
  BlendState bs{};
  bs.chunk = (uint32_t)c->fwd_chunk;
  bs.chunk_shift = (uint32_t)__builtin_ctz((unsigned)c->fwd_chunk);
  bs.T_final = c->T_final.p;
  bs.last = c->last.p;
  bs.counts = nullptr;
  bs.bound = c->bound.p;
  bs.nbound = c->bound.cap / kBlock;
  bs.tile_nch = c->tile_nch.p;
  bs.order = c->tile_order.p;
  bs.items = c->items.p;
  bs.items_cap = c->items.cap;
  bs.n_items = c->counters.p + 4;
  bs.l1_partial = nullptr;
  bs.l1_inv = 0.f;
  return bs;
}

bool ensure_pairs(sixdgs_ctx* c, int64_t P, double slack) {
  const int64_t p1 = P > 0 ? P : 1;
  return c->pkey0.ensure(p1, slack) && c->pkey1.ensure(p1, slack) && c->pval0.ensure(p1, slack) &&
         c->pval1.ensure(p1, slack);
}

void fill_sort_buffers(sixdgs_ctx* c, int64_t E) {
  SortBuffers& b = c->sb;
  b.E = E;
  b.tiles = c->tiles.p;
  b.rec = c->rec.p;
  b.depth = c->bin_depth ? c->bin_depth : c->depth.p;
  b.dkey[0] = c->dkey0.p;
  b.dkey[1] = c->dkey1.p;
  b.dval[0] = c->dval0.p;
  b.dval[1] = c->dval1.p;
  b.poff = c->poff.p;
  b.pcap = std::min(std::min(c->pkey0.cap, c->pkey1.cap), std::min(c->pval0.cap, c->pval1.cap));
  b.pkey[0] = c->pkey0.p;
  b.pkey[1] = c->pkey1.p;
  b.pval[0] = c->pval0.p;
  b.pval[1] = c->pval1.p;
  b.ranges = c->ranges.p;
  b.rstate_depth = c->rstate.p;
  b.rstate_pairs = c->rstate.p + sort_state_words(std::max<int64_t>(E, 1), false);
  b.blk_start = c->blk_start.p;
  b.nblk_start = c->blk_start.cap;
  b.total_tiles = c->vt.total_tiles;
  b.tile_order = c->tile_order.p;
  b.order_state = c->order_state.p;
  b.g2d = c->bin_g2d;
  b.n_items = c->counters.p + 4;
  b.counters = c->counters.p;
}

hipEvent_t get_event(sixdgs_ctx* c) {
  if (!c->free_events.empty()) {
    hipEvent_t e = c->free_events.back();
    c->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

struct Timer {
  sixdgs_ctx* c;
  int k;
  hipStream_t st;
  hipEvent_t a = nullptr;
  Timer(sixdgs_ctx* c_, int k_, hipStream_t st_) : c(c_), k(k_), st(st_) {
    if (c->timing_mask & (1 << k)) {
      a = get_event(c);
      (void)hipEventRecord(a, st);
    }
  }
  ~Timer() {
    if (a) {
      hipEvent_t b = get_event(c);
      (void)hipEventRecord(b, st);
      c->pending.push_back({k, a, b});
    }
  }
};

void collect_timing(sixdgs_ctx* c) {
  for (auto& t : c->pending) {
    (void)hipEventSynchronize(t.b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, t.a, t.b);
    c->ms[t.kernel] += ms;
    c->launches[t.kernel] += 1;
    c->free_events.push_back(t.a);
    c->free_events.push_back(t.b);
  }
  c->pending.clear();
}

sixdgs_status check_launch(sixdgs_ctx* c, const char* where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, SIXDGS_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
  return SIXDGS_OK;
}

// The integer stage's buffers for E entries of the views in c->vt, and its
// buffer table (before the launch that prepares the stage).
sixdgs_status prepare_binning(sixdgs_ctx* c, int64_t E) {
  const bool fixed = c->s.pair_capacity > 0;
  if (fixed) {
    if (!ensure_pairs(c, c->s.pair_capacity, 1.0)) return fail(c, SIXDGS_ERR_OOM, "pair buffers");
  } else if (c->pkey0.cap == 0 && !ensure_pairs(c, 1 << 16, 1.0)) {
    return fail(c, SIXDGS_ERR_OOM, "pair buffers");
  }
  if (!ensure_scratch(c, E, std::max<int64_t>(c->pkey0.cap, fixed ? c->s.pair_capacity : 0)))
    return fail(c, SIXDGS_ERR_OOM, "sort scratch");
  if (!c->ranges.ensure(std::max<int64_t>(c->vt.total_tiles, 1))) return fail(c, SIXDGS_ERR_OOM, "tile ranges");
  if (!c->tile_order.ensure(std::max<int64_t>(c->vt.total_tiles, 1)) || !c->order_state.ensure(order_state_words()))
    return fail(c, SIXDGS_ERR_OOM, "tile order");
  fill_sort_buffers(c, E);
  return SIXDGS_OK;
}

// Integer stage after the records and tile counts of E entries exist
// (prepare_binning first; prepped: bin_prep was done by the launch before).
sixdgs_status run_binning(sixdgs_ctx* c, int64_t E, bool prepped, hipStream_t st) {
  const bool fixed = c->s.pair_capacity > 0;
  Timer t(c, SIXDGS_K_SORT, st);
  launch_bin_count(c->sb, prepped, st);
  int64_t hint = c->sb.pcap;
  bool regrown = false;
  if (!fixed) {
    // read the pair count back, then size the pair buffers exactly (with slack for the next call)
    if (hipMemcpyAsync(c->host_counters, c->counters.p, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return fail(c, SIXDGS_ERR_HIP, "pair count read-back failed");
    const int64_t P = c->host_counters[1];
    if (P > kMaxItems) return fail(c, SIXDGS_ERR_CAPACITY, "more than 2^30 - 1 pairs");
    if (P > c->sb.pcap) {
      if (!ensure_pairs(c, P, 1.25)) return fail(c, SIXDGS_ERR_OOM, "pair buffers");
      if (!ensure_scratch(c, E, c->pkey0.cap)) return fail(c, SIXDGS_ERR_OOM, "sort scratch");
      fill_sort_buffers(c, E);  // keeps dsorted: the depth-sorted entries are untouched
      regrown = true;
    }
    hint = P;
  }
  launch_bin_emit(c->sb, c->vt, hint, regrown, st);
  return check_launch(c, "binning");
}

// Empties the workspace and sets whether it is allocated with guards; the
// state of the last forward, binning and density plan is dropped with it.
void set_debug(sixdgs_ctx* c, bool on) {
  c->debug = on;
  for_each_buf(c, [on](auto& b, const char*) {
    b.release();
    b.guarded = on;
  });
  c->have_fwd = false;
  c->g2d_clean = false;
  c->counts_valid = false;
  c->dens_n = -1;
  c->fwd_E = 0;
  c->fwd_px = 0;
  c->vt = ViewTable{};
  c->sb = SortBuffers{};
}

// The error flags in counters[2..3] are only ever set by kernels and cleared by sixdgs_check.
bool init_counters(sixdgs_ctx* c) {
  return c->counters.ensure(kCounters) && hipMemset(c->counters.p, 0, kCounters * sizeof(uint32_t)) == hipSuccess;
}

template <class T>
bool read_back(std::vector<T>& h, const T* d, int64_t count) {
  h.resize((size_t)std::max<int64_t>(count, 0));
  return count <= 0 || hipMemcpy(h.data(), d, (size_t)count * sizeof(T), hipMemcpyDeviceToHost) == hipSuccess;
}

// The invariants of the last binning (sixdgs_debug_check_bins on host copies
// of its outputs); with `items`, also the backward's work items and each
// pixel's last contributor and final transmittance against its tile.  "" if
// they hold.
std::string debug_check_binning(sixdgs_ctx* c, const float* depth_dev, bool items) {
  uint32_t cnt[kCounters];
  if (hipMemcpy(cnt, c->counters.p, sizeof(cnt), hipMemcpyDeviceToHost) != hipSuccess) return "counter read-back failed";
  const int64_t E = c->sb.E, P = cnt[1], T = c->vt.total_tiles;
  if (P > c->sb.pcap) return "";  // overflow of the fixed capacity: no output to check (sixdgs_check reports it)
  std::vector<uint32_t> tiles, keys, vals, ranges, order, nch, its;
  std::vector<float> depth;
  if (!read_back(tiles, c->tiles.p, E) || !read_back(depth, depth_dev, E) ||
      !read_back(keys, (const uint32_t*)c->sb.pkey[c->sb.psorted], P) ||
      !read_back(vals, (const uint32_t*)c->sb.pval[c->sb.psorted], P) ||
      !read_back(ranges, (const uint32_t*)c->ranges.p, 2 * T) || !read_back(order, (const uint32_t*)c->tile_order.p, T))
    return "binning read-back failed";
  if ((int64_t)cnt[0] > E) return "binned entries " + std::to_string(cnt[0]) + " > " + std::to_string(E);
  sixdgs_bin_state b{};
  b.E = E;
  b.P = P;
  b.T = T;
  b.tiles = tiles.data();
  b.depth = depth.data();
  b.keys = keys.data();
  b.values = vals.data();
  b.ranges = ranges.data();
  b.order = order.data();
  b.chunk = c->fwd_chunk;
  if (items) {
    const int64_t ni = cnt[4];
    if (ni > c->items.cap) return std::to_string(ni) + " work items > capacity " + std::to_string(c->items.cap);
    if (!read_back(nch, (const uint32_t*)c->tile_nch.p, T) || !read_back(its, (const uint32_t*)c->items.p, 2 * ni))
      return "work item read-back failed";
    b.nch = nch.data();
    b.items = its.data();
    b.n_items = ni;
  }
  char msg[512];
  if (sixdgs_debug_check_bins(&b, msg, sizeof(msg)) != SIXDGS_OK) return msg;
  if (!items) return "";
  // per pixel: the last contributor lies in its tile's run, T_final in [kTMin, 1];
  // per tile: chunks = ceil(largest last contributor / chunk)
  std::vector<uint32_t> last;
  std::vector<float> Tf;
  if (!read_back(last, (const uint32_t*)c->last.p, c->fwd_px) || !read_back(Tf, (const float*)c->T_final.p, c->fwd_px))
    return "pixel state read-back failed";
  std::vector<uint32_t> maxlast((size_t)std::max<int64_t>(T, 1), 0u);
  for (int k = 0; k < c->vt.nview; k++) {
    const ViewDesc& vd = c->vt.v[k];
    for (int y = 0; y < vd.H; y++)
      for (int x = 0; x < vd.W; x++) {
        const int64_t pix = vd.pix_base + (int64_t)y * vd.W + x;
        const uint32_t t = (uint32_t)(vd.tile_base + (y >> c->vt.tile_shift_y) * vd.ntx + (x >> c->vt.tile_shift_x));
        const uint32_t run = ranges[2 * t + 1] - ranges[2 * t];
        if (last[pix] > run)
          return "view " + std::to_string(k) + " pixel (" + std::to_string(x) + ", " + std::to_string(y) +
                 "): last contributor " + std::to_string(last[pix]) + " past its tile's " + std::to_string(run) +
                 " pairs";
        if (!(Tf[pix] >= kTMin && Tf[pix] <= 1.0f))
          return "view " + std::to_string(k) + " pixel (" + std::to_string(x) + ", " + std::to_string(y) +
                 "): final transmittance " + std::to_string(Tf[pix]) + " outside [1e-4, 1]";
        maxlast[t] = std::max(maxlast[t], last[pix]);
      }
  }
  for (int64_t t = 0; t < T; t++) {
    const uint32_t want = (uint32_t)(((int64_t)maxlast[t] + c->fwd_chunk - 1) / c->fwd_chunk);
    if (nch[t] != want)
      return "tile " + std::to_string(t) + ": " + std::to_string(nch[t]) + " chunks, its last contributor needs " +
             std::to_string(want);
  }
  return "";
}

// Debug mode: after a call that launched work, waits for it and checks every
// guard; after a binning (bins = 1), or a training forward (bins = 2: with
// the work items and the pixel state), also the invariants of the outputs.
sixdgs_status debug_after(sixdgs_ctx* c, void* stream, sixdgs_status rc, int bins, const float* depth_dev = nullptr) {
  if (!c->debug || rc != SIXDGS_OK) return rc;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
    return fail(c, SIXDGS_ERR_HIP, "stream synchronisation failed");
  std::string why;
  for_each_buf(c, [&](auto& b, const char* name) {
    if (why.empty()) why = b.guard_damage(name);
  });
  if (!why.empty()) return fail(c, SIXDGS_ERR_DEBUG, "debug: guard of " + why);
  if (bins) {
    why = debug_check_binning(c, depth_dev ? depth_dev : c->depth.p, bins == 2);
    if (!why.empty()) return fail(c, SIXDGS_ERR_DEBUG, "debug: " + why);
  }
  return SIXDGS_OK;
}

}  // namespace

extern "C" {

void sixdgs_default_settings(sixdgs_settings* s) {
  if (!s) return;
  std::memset(s, 0, sizeof(*s));
  s->lambda_opa = 0.35f;
  s->z_near = 0.2f;
  s->tile_w = 16;
  s->tile_h = 16;
  s->batch = 0;  // automatic
  s->pair_capacity = 0;
  s->flags = 0;
  s->chunk = 0;  // automatic
}

sixdgs_status sixdgs_create(sixdgs_ctx** out, const sixdgs_settings* s) {
  if (!out) return SIXDGS_ERR_INVALID_ARG;
  *out = nullptr;
  sixdgs_settings def;
  sixdgs_default_settings(&def);
  if (!s) s = &def;
  std::string why;
  if (!valid_settings(s, why)) return SIXDGS_ERR_INVALID_ARG;
  sixdgs_ctx* c = new (std::nothrow) sixdgs_ctx();
  if (!c) return SIXDGS_ERR_OOM;
  c->s = *s;
  if (hipHostMalloc((void**)&c->host_counters, 4 * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
    delete c;
    return SIXDGS_ERR_HIP;
  }
  set_debug(c, (s->flags & SIXDGS_FLAG_DEBUG) != 0);
  if (!init_counters(c)) {
    sixdgs_destroy(c);
    return SIXDGS_ERR_OOM;
  }
  *out = c;
  return SIXDGS_OK;
}

void sixdgs_destroy(sixdgs_ctx* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  collect_timing(c);
  for (hipEvent_t e : c->free_events) (void)hipEventDestroy(e);
  for_each_buf(c, [](auto& b, const char*) { b.release(); });
  if (c->host_counters) (void)hipHostFree(c->host_counters);
  delete c;
}

sixdgs_status sixdgs_set_settings(sixdgs_ctx* c, const sixdgs_settings* s) {
  if (!c || !s) return fail(c, SIXDGS_ERR_INVALID_ARG, "NULL argument");
  std::string why;
  if (!valid_settings(s, why)) return fail(c, SIXDGS_ERR_INVALID_ARG, why);
  const bool debug = (s->flags & SIXDGS_FLAG_DEBUG) != 0;
  c->s = *s;
  if (debug != c->debug) {
    (void)hipDeviceSynchronize();
    set_debug(c, debug);
    if (!init_counters(c)) return fail(c, SIXDGS_ERR_OOM, "counters");
  }
  return SIXDGS_OK;
}

const char* sixdgs_last_error(const sixdgs_ctx* c) {
  if (!c) return "no context";
  return c->err.c_str();
}

}  // extern "C"

namespace {
// The forward; with a cache the slice's direction-independent part is read
// from it, and inference = true renders the images only (no state for a
// backward is kept).
sixdgs_status forward_impl(sixdgs_ctx* c, const float* params, const float* cache, int64_t n,
                           const sixdgs_camera* cams, int32_t ncam, float* const* images, bool inference,
                           void* stream, const float* const* targets = nullptr, float* const* dl_dimages = nullptr,
                           float* loss = nullptr) {
  hipStream_t st = (hipStream_t)stream;
  if (n < 0) return fail(c, SIXDGS_ERR_INVALID_ARG, "n must be >= 0");
  if (n > 0 && !params) return fail(c, SIXDGS_ERR_INVALID_ARG, "params is NULL");
  if (!images) return fail(c, SIXDGS_ERR_INVALID_ARG, "images is NULL");
  ViewTable vt;
  int64_t total_px = 0;
  std::string why = build_views(c->s, n, cams, ncam, vt, total_px);
  if (!why.empty()) return fail(c, SIXDGS_ERR_INVALID_ARG, why);
  for (int k = 0; k < ncam; k++) {
    if (!images[k]) return fail(c, SIXDGS_ERR_INVALID_ARG, "an image pointer is NULL");
    vt.v[k].img = images[k];
  }
  const bool with_l1 = targets != nullptr;
  if (with_l1) {
    if (!dl_dimages || !loss) return fail(c, SIXDGS_ERR_INVALID_ARG, "targets, dl_dimages and loss: all three");
    for (int k = 0; k < ncam; k++) {
      if (!targets[k] || !dl_dimages[k]) return fail(c, SIXDGS_ERR_INVALID_ARG, "a target or dL/dI pointer is NULL");
      vt.v[k].tgt = targets[k];
      vt.v[k].dl = dl_dimages[k];
    }
  }
  const int64_t E = n * ncam;
  if (E > kMaxItems) return fail(c, SIXDGS_ERR_INVALID_ARG, "n * cameras must stay below 2^30");
  c->have_fwd = false;
  if (!ensure_entries(c, E)) return fail(c, SIXDGS_ERR_OOM, "entry buffers");
  if (!c->T_final.ensure(total_px) || !c->last.ensure(total_px)) return fail(c, SIXDGS_ERR_OOM, "pixel state");
  const bool want_counts = (c->s.flags & SIXDGS_FLAG_COUNTS) != 0;
  if (want_counts && !c->counts.ensure(total_px)) return fail(c, SIXDGS_ERR_OOM, "pixel counts");
  c->vt = vt;
  DevSettings ds = dev_settings(c->s);
  ds.lambda_raw = c->lambda_raw;
  c->fwd_lambda = c->lambda_raw;
  c->g2d_clean = false;
  if (!inference && !c->g2d.ensure(E * kG2D)) return fail(c, SIXDGS_ERR_OOM, "gradient accumulators");
  c->bin_g2d = inference ? nullptr : c->g2d.p;  // cleared by the binning for the backward
  sixdgs_status rc = prepare_binning(c, E);
  if (rc != SIXDGS_OK) {
    c->bin_g2d = nullptr;
    return rc;
  }
  bool prepped;
  {
    // the projection also prepares the integer stage
    const BinPrep bp = bin_prep(c->sb);
    Timer t(c, SIXDGS_K_PREPROCESS, st);
    prepped = launch_preprocess(params, cache, n, vt, ds, c->rec.p, c->tiles.p, c->depth.p, &bp, st);
  }
  rc = check_launch(c, "preprocess");
  if (rc == SIXDGS_OK) rc = run_binning(c, E, prepped, st);
  c->bin_g2d = nullptr;
  if (rc != SIXDGS_OK) return rc;
  c->g2d_clean = !inference;
  // the backward's chunk and LDS batch depth: with few tiles, short chunks
  // spread the heavy tiles' walks over many workgroups; with many tiles
  // (several large views) there is parallelism enough and longer chunks save
  // the restarts (measured: 128 / 128 best for one 800x800 view, 256 / 512
  // for eight or sixteen 1080p-class views)
  {
    const bool few = vt.total_tiles < kAutoTiles;
    int chunk = c->s.chunk ? c->s.chunk : (few ? 128 : 512);
    int batch = c->s.batch ? c->s.batch : (few ? 128 : 256);
    if (batch > chunk) batch = chunk;
    c->fwd_chunk = chunk;
    c->fwd_batch = batch;
  }
  // the backward's work items: at most one per `chunk` pairs plus one per tile
  const int64_t nbound = c->sb.pcap / c->fwd_chunk + 1;
  const int64_t grid = nbound + vt.total_tiles;
  if (!c->bound.ensure(nbound * kBlock) ||
      !c->tile_nch.ensure(std::max<int64_t>(vt.total_tiles, 1)) || !c->items.ensure(grid))
    return fail(c, SIXDGS_ERR_OOM, "backward work items");
  c->bwd_grid = grid;
  BlendState bs = blend_state(c);
  bs.counts = want_counts ? c->counts.p : nullptr;
  if (with_l1) {
    // each tile's sum of |I - I*|, then their total
    const int64_t parts = std::max<int64_t>(vt.total_tiles, 1);
    if (!c->l1_partial.ensure(parts + l1_final_scratch(parts))) return fail(c, SIXDGS_ERR_OOM, "loss partials");
    bs.l1_partial = c->l1_partial.p;
    bs.l1_inv = 1.0f / (float)(3 * total_px);
  }
  {
    Timer t(c, SIXDGS_K_BLEND_FWD, st);
    launch_blend_fwd(vt, ds, c->rec.p, c->ranges.p, c->sb.pval[c->sb.psorted], bs, c->fwd_batch, !inference, st);
  }
  if (with_l1) launch_l1_final(c->l1_partial.p, vt.total_tiles, bs.l1_inv, loss, c->l1_partial.p + vt.total_tiles, st);
  if (inference) return check_launch(c, "blend forward");
  rc = check_launch(c, "blend forward");
  if (rc != SIXDGS_OK) return rc;
  c->have_fwd = true;
  c->counts_valid = want_counts;
  c->fwd_params = params;
  c->fwd_n = n;
  c->fwd_E = E;
  c->fwd_px = total_px;
  c->stream = st;
  return SIXDGS_OK;
}
}  // namespace

extern "C" {

sixdgs_status sixdgs_forward(sixdgs_ctx* c, const float* params, int64_t n, const sixdgs_camera* cams, int32_t ncam,
                             float* const* images, void* stream) {
  if (!c) return SIXDGS_ERR_INVALID_ARG;
  return debug_after(c, stream, forward_impl(c, params, nullptr, n, cams, ncam, images, false, stream), 2);
}

sixdgs_status sixdgs_forward_l1(sixdgs_ctx* c, const float* params, int64_t n, const sixdgs_camera* cams,
                                int32_t ncam, float* const* images, const float* const* targets,
                                float* const* dl_dimages, float* loss, void* stream) {
  if (!c) return SIXDGS_ERR_INVALID_ARG;
  if (!targets) return fail(c, SIXDGS_ERR_INVALID_ARG, "targets is NULL");
  return debug_after(c, stream,
                     forward_impl(c, params, nullptr, n, cams, ncam, images, false, stream, targets, dl_dimages, loss),
                     2);
}

sixdgs_status sixdgs_build_cache(const float* params, int64_t n, float* cache, void* stream) {
  if (n < 0 || (n > 0 && (!params || !cache))) return SIXDGS_ERR_INVALID_ARG;
  launch_build_cache(params, n, cache, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? SIXDGS_OK : SIXDGS_ERR_HIP;
}

sixdgs_status sixdgs_forward_cached(sixdgs_ctx* c, const float* params, const float* cache, int64_t n,
                                    const sixdgs_camera* cams, int32_t ncam, float* const* images, void* stream) {
  if (!c) return SIXDGS_ERR_INVALID_ARG;
  if (n > 0 && !cache) return fail(c, SIXDGS_ERR_INVALID_ARG, "cache is NULL");
  if (c->lambda_raw) return fail(c, SIXDGS_ERR_STATE, "a cached forward takes the scalar lambda: detach the array");
  return debug_after(c, stream, forward_impl(c, params, cache, n, cams, ncam, images, true, stream), 1);
}

static sixdgs_status backward_body(sixdgs_ctx* c, const float* params, int64_t n, int32_t ncam,
                                   const float* const* dl_dimages, float* grad, float* densify, void* stream) {
  if (!c) return SIXDGS_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  if (!c->have_fwd) return fail(c, SIXDGS_ERR_STATE, "backward needs a forward on this context first");
  if (params != c->fwd_params || n != c->fwd_n)
    return fail(c, SIXDGS_ERR_STATE, "params / n differ from the last forward");
  if (ncam != c->vt.nview) return fail(c, SIXDGS_ERR_INVALID_ARG, "ncam differs from the last forward's");
  if (!dl_dimages) return fail(c, SIXDGS_ERR_INVALID_ARG, "dl_dimages is NULL");
  if (n > 0 && !grad) return fail(c, SIXDGS_ERR_INVALID_ARG, "grad is NULL");
  ViewTable vt = c->vt;
  for (int k = 0; k < vt.nview; k++) {
    if (!dl_dimages[k]) return fail(c, SIXDGS_ERR_INVALID_ARG, "a dL/dI pointer is NULL");
    vt.v[k].dimg = dl_dimages[k];
  }
  if (n == 0) return SIXDGS_OK;
  if (!c->g2d.ensure(c->fwd_E * kG2D)) return fail(c, SIXDGS_ERR_OOM, "gradient accumulators");
  DevSettings ds = dev_settings(c->s);
  ds.lambda_raw = c->fwd_lambda;
  ds.grad_lambda = c->fwd_lambda ? c->grad_lambda : nullptr;
  if (!c->g2d_clean) launch_zero_g2d(c->sb, c->g2d.p, st);  // a second backward of one forward
  c->g2d_clean = false;
  const BlendState bs = blend_state(c);
  {
    Timer t(c, SIXDGS_K_BLEND_BWD, st);
    launch_blend_bwd(vt, ds, c->rec.p, c->ranges.p, c->sb.pval[c->sb.psorted], bs, c->g2d.p, c->fwd_batch,
                     c->bwd_grid, st);
  }
  sixdgs_status rc = check_launch(c, "blend backward");
  if (rc != SIXDGS_OK) return rc;
  {
    Timer t(c, SIXDGS_K_PREPROCESS_BWD, st);
    launch_preprocess_bwd(params, n, vt, ds, c->tiles.p, c->g2d.p, grad, densify, st);
  }
  return check_launch(c, "preprocess backward");
}

sixdgs_status sixdgs_backward(sixdgs_ctx* c, const float* params, int64_t n, int32_t ncam,
                              const float* const* dl_dimages, float* grad, float* densify, void* stream) {
  if (!c) return SIXDGS_ERR_INVALID_ARG;
  return debug_after(c, stream, backward_body(c, params, n, ncam, dl_dimages, grad, densify, stream), 0);
}

// step >= 1, or step_counter (device) with step = *step_counter + 1, advanced
// after the update when `advance`.
static sixdgs_status backward_adam_body(sixdgs_ctx* c, float* params, int64_t n, int32_t ncam,
                                        const float* const* dl_dimages, float* m, float* v, const float* lr, float beta1,
                                        float beta2, float eps, int32_t step, int32_t* step_counter, bool advance,
                                        float* densify, void* stream) {
  if (!c) return SIXDGS_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  if (!c->have_fwd) return fail(c, SIXDGS_ERR_STATE, "backward needs a forward on this context first");
  if (params != c->fwd_params || n != c->fwd_n)
    return fail(c, SIXDGS_ERR_STATE, "params / n differ from the last forward");
  if (ncam != c->vt.nview) return fail(c, SIXDGS_ERR_INVALID_ARG, "ncam differs from the last forward's");
  if (!dl_dimages || !lr) return fail(c, SIXDGS_ERR_INVALID_ARG, "NULL argument");
  if (n > 0 && (!m || !v)) return fail(c, SIXDGS_ERR_INVALID_ARG, "m or v is NULL");
  if ((!step_counter && step < 1) || !(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f))
    return fail(c, SIXDGS_ERR_INVALID_ARG, "bad Adam hyper-parameters");
  ViewTable vt = c->vt;
  for (int k = 0; k < vt.nview; k++) {
    if (!dl_dimages[k]) return fail(c, SIXDGS_ERR_INVALID_ARG, "a dL/dI pointer is NULL");
    vt.v[k].dimg = dl_dimages[k];
  }
  if (n == 0) return SIXDGS_OK;
  if (!c->g2d.ensure(c->fwd_E * kG2D)) return fail(c, SIXDGS_ERR_OOM, "gradient accumulators");
  DevSettings ds = dev_settings(c->s);
  ds.lambda_raw = c->fwd_lambda;
  ds.grad_lambda = c->fwd_lambda ? c->grad_lambda : nullptr;
  if (!c->g2d_clean) launch_zero_g2d(c->sb, c->g2d.p, st);  // a second backward of one forward
  c->g2d_clean = false;
  const BlendState bs = blend_state(c);
  {
    Timer t(c, SIXDGS_K_BLEND_BWD, st);
    launch_blend_bwd(vt, ds, c->rec.p, c->ranges.p, c->sb.pval[c->sb.psorted], bs, c->g2d.p, c->fwd_batch,
                     c->bwd_grid, st);
  }
  sixdgs_status rc = check_launch(c, "blend backward");
  if (rc != SIXDGS_OK) return rc;
  const AdamArgs a = make_adam_args(lr, beta1, beta2, eps, step_counter ? 1 : step);
  {
    Timer t(c, SIXDGS_K_PREPROCESS_BWD, st);
    // counters[6]: the finished-workgroup count with which the kernel advances the step
    launch_preprocess_bwd_adam(params, n, vt, ds, c->tiles.p, c->g2d.p, m, v, a, step_counter,
                               advance ? c->counters.p + 6 : nullptr, densify, st);
  }
  c->have_fwd = false;  // the parameters moved
  return check_launch(c, "preprocess backward + Adam");
}

sixdgs_status sixdgs_backward_adam(sixdgs_ctx* c, float* params, int64_t n, int32_t ncam,
                                   const float* const* dl_dimages, float* m, float* v, const float* lr, float beta1,
                                   float beta2, float eps, int32_t step, float* densify, void* stream) {
  if (!c) return SIXDGS_ERR_INVALID_ARG;
  return debug_after(c, stream,
                     backward_adam_body(c, params, n, ncam, dl_dimages, m, v, lr, beta1, beta2, eps, step, nullptr,
                                        false, densify, stream),
                     0);
}

sixdgs_status sixdgs_backward_adam_devstep(sixdgs_ctx* c, float* params, int64_t n, int32_t ncam,
                                           const float* const* dl_dimages, float* m, float* v, const float* lr,
                                           float beta1, float beta2, float eps, int32_t* step_counter,
                                           int32_t advance, float* densify, void* stream) {
  if (!c) return SIXDGS_ERR_INVALID_ARG;
  if (!step_counter) return fail(c, SIXDGS_ERR_INVALID_ARG, "step_counter is NULL");
  return debug_after(c, stream,
                     backward_adam_body(c, params, n, ncam, dl_dimages, m, v, lr, beta1, beta2, eps, 1, step_counter,
                                        advance != 0, densify, stream),
                     0);
}

static sixdgs_status l1_loss_body(sixdgs_ctx* c, int32_t nimg, const float* const* images, const float* const* targets,
                                  const int64_t* numel, float* const* dl_dimages, float* loss, void* stream) {
  if (!c) return SIXDGS_ERR_INVALID_ARG;
  if (nimg < 1 || nimg > kMaxViews) return fail(c, SIXDGS_ERR_INVALID_ARG, "nimg out of range");
  if (!images || !targets || !numel || !dl_dimages || !loss) return fail(c, SIXDGS_ERR_INVALID_ARG, "NULL argument");
  for (int k = 0; k < nimg; k++) {
    if (!images[k] || !targets[k] || !dl_dimages[k]) return fail(c, SIXDGS_ERR_INVALID_ARG, "NULL image pointer");
    if (numel[k] <= 0) return fail(c, SIXDGS_ERR_INVALID_ARG, "numel must be positive");
  }
  const int64_t parts = l1_partial_count(nimg, numel);
  if (!c->l1_partial.ensure(parts)) return fail(c, SIXDGS_ERR_OOM, "loss partials");
  launch_l1(nimg, images, targets, numel, dl_dimages, c->l1_partial.p, c->l1_partial.cap, loss, (hipStream_t)stream);
  return check_launch(c, "l1 loss");
}

sixdgs_status sixdgs_l1_loss(sixdgs_ctx* c, int32_t nimg, const float* const* images, const float* const* targets,
                             const int64_t* numel, float* const* dl_dimages, float* loss, void* stream) {
  if (!c) return SIXDGS_ERR_INVALID_ARG;
  return debug_after(c, stream, l1_loss_body(c, nimg, images, targets, numel, dl_dimages, loss, stream), 0);
}

}  // extern "C"

// Scratch of the allocation-free L1 loss: the per-workgroup partial sums of
// k_l1, at most kL1MaxBlocks per image for SIXDGS_MAX_VIEWS images (64 KiB on
// every device the library runs on, held until the process ends).  Its name
// is a host-side stand-in: host code uses only the device address looked up
// for the current device below.
static constexpr int64_t kL1ScratchFloats = (int64_t)kMaxViews * kL1MaxBlocks;
static __device__ __align__(256) float scratch[kL1ScratchFloats];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device; nullptr if the lookup fails.
float* l1_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch_ptr[dev] = static_cast<float*>(ptr);
  }
  return g_scratch_ptr[dev];
}
}  // namespace

extern "C" {

sixdgs_status sixdgs_l1_loss_noalloc(int32_t nimg, const float* const* images, const float* const* targets,
                                     const int64_t* numel, float* const* dl_dimages, float* loss, void* stream) {
  if (nimg < 1 || nimg > kMaxViews) return SIXDGS_ERR_INVALID_ARG;
  if (!images || !targets || !numel || !dl_dimages || !loss) return SIXDGS_ERR_INVALID_ARG;
  for (int k = 0; k < nimg; k++) {
    if (!images[k] || !targets[k] || !dl_dimages[k]) return SIXDGS_ERR_INVALID_ARG;
    if (numel[k] <= 0) return SIXDGS_ERR_INVALID_ARG;
  }
  // every image takes at most kL1MaxBlocks partial sums, so the scratch always suffices
  if (l1_partial_count(nimg, numel) > kL1ScratchFloats) return SIXDGS_ERR_CAPACITY;
  float* partial = l1_scratch();
  if (!partial) return SIXDGS_ERR_HIP;
  // k_l1 writes every partial sum that k_l1_final reads: nothing needs clearing
  launch_l1(nimg, images, targets, numel, dl_dimages, partial, kL1ScratchFloats, loss, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? SIXDGS_OK : SIXDGS_ERR_HIP;
}

static sixdgs_status l1_dssim_loss_body(sixdgs_ctx* c, int32_t nimg, const float* const* images,
                                        const float* const* targets, const int32_t* heights, const int32_t* widths,
                                        float lambda_dssim, float* const* dl_dimages, float* loss, void* stream) {
  if (!c) return SIXDGS_ERR_INVALID_ARG;
  if (nimg < 1 || nimg > kMaxViews) return fail(c, SIXDGS_ERR_INVALID_ARG, "nimg out of range");
  if (!images || !targets || !heights || !widths || !dl_dimages || !loss)
    return fail(c, SIXDGS_ERR_INVALID_ARG, "NULL argument");
  if (!(lambda_dssim >= 0.f && lambda_dssim <= 1.f)) return fail(c, SIXDGS_ERR_INVALID_ARG, "lambda_dssim not in [0, 1]");
  int64_t px = 0, blocks = 0;
  for (int k = 0; k < nimg; k++) {
    if (!images[k] || !targets[k] || !dl_dimages[k]) return fail(c, SIXDGS_ERR_INVALID_ARG, "NULL image pointer");
    if (heights[k] < 1 || widths[k] < 1 || heights[k] > 65535 * 16 || widths[k] > 65535 * 16)
      return fail(c, SIXDGS_ERR_INVALID_ARG, "image size out of range");
    px += (int64_t)heights[k] * widths[k];
    blocks += ssim_blocks(heights[k], widths[k]);
  }
  if (!c->ssim_maps.ensure(9 * px) || !c->ssim_partial.ensure(2 * blocks))
    return fail(c, SIXDGS_ERR_OOM, "ssim scratch");
  launch_l1_dssim(nimg, images, targets, heights, widths, lambda_dssim, dl_dimages, c->ssim_maps.p,
                  c->ssim_partial.p, loss, (hipStream_t)stream);
  return check_launch(c, "l1 + d-ssim loss");
}

sixdgs_status sixdgs_l1_dssim_loss(sixdgs_ctx* c, int32_t nimg, const float* const* images,
                                   const float* const* targets, const int32_t* heights, const int32_t* widths,
                                   float lambda_dssim, float* const* dl_dimages, float* loss, void* stream) {
  if (!c) return SIXDGS_ERR_INVALID_ARG;
  return debug_after(
      c, stream,
      l1_dssim_loss_body(c, nimg, images, targets, heights, widths, lambda_dssim, dl_dimages, loss, stream), 0);
}

sixdgs_status sixdgs_adam(float* params, const float* grad, float* m, float* v, int64_t n, const float* lr,
                          float beta1, float beta2, float eps, int32_t step, void* stream) {
  if (n < 0 || (n > 0 && (!params || !grad || !m || !v)) || !lr || step < 1) return SIXDGS_ERR_INVALID_ARG;
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f)) return SIXDGS_ERR_INVALID_ARG;
  launch_adam(params, grad, m, v, kRows, n, lr, beta1, beta2, eps, step, nullptr, false, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? SIXDGS_OK : SIXDGS_ERR_HIP;
}

sixdgs_status sixdgs_adam_devstep(float* params, const float* grad, float* m, float* v, int64_t n, const float* lr,
                                  float beta1, float beta2, float eps, int32_t* step_counter, void* stream) {
  if (n < 0 || (n > 0 && (!params || !grad || !m || !v)) || !lr || !step_counter) return SIXDGS_ERR_INVALID_ARG;
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f)) return SIXDGS_ERR_INVALID_ARG;
  launch_adam(params, grad, m, v, kRows, n, lr, beta1, beta2, eps, 1, step_counter, true, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? SIXDGS_OK : SIXDGS_ERR_HIP;
}

sixdgs_status sixdgs_adam_vec(float* p, const float* g, float* m, float* v, int64_t n, float lr, float beta1,
                              float beta2, float eps, int32_t step, const int32_t* step_counter, void* stream) {
  if (n < 0 || (n > 0 && (!p || !g || !m || !v)) || (!step_counter && step < 1)) return SIXDGS_ERR_INVALID_ARG;
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps >= 0.f)) return SIXDGS_ERR_INVALID_ARG;
  const float lrs[6] = {lr, lr, lr, lr, lr, lr};
  launch_adam(p, g, m, v, 1, n, lrs, beta1, beta2, eps, step_counter ? 1 : step, const_cast<int32_t*>(step_counter),
              false, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? SIXDGS_OK : SIXDGS_ERR_HIP;
}

sixdgs_status sixdgs_decompose(const float* params, int64_t n, float* R, float* S, void* stream) {
  if (n < 0 || (n > 0 && (!params || !R || !S))) return SIXDGS_ERR_INVALID_ARG;
  launch_decompose(params, n, R, S, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? SIXDGS_OK : SIXDGS_ERR_HIP;
}

static sixdgs_status densify_plan_body(sixdgs_ctx* c, const float* params, int64_t n, const float* stats,
                                       const sixdgs_density_settings* d, int64_t* n_out, void* stream) {
  if (!c) return SIXDGS_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  if (n < 0 || n > kMaxItems) return fail(c, SIXDGS_ERR_INVALID_ARG, "n out of range");
  if (!d || !n_out || (n > 0 && (!params || !stats))) return fail(c, SIXDGS_ERR_INVALID_ARG, "NULL argument");
  if (!(d->grad_threshold > 0.f && d->percent_dense >= 0.f && d->extent > 0.f && d->min_opacity >= 0.f))
    return fail(c, SIXDGS_ERR_INVALID_ARG, "density settings out of range");
  c->dens_n = -1;
  const int64_t n1 = std::max<int64_t>(n, 1);
  if (!c->dens_dec.ensure(n1) || !c->dens_cnt.ensure(n1) || !c->dens_off.ensure(n1) ||
      !c->dens_state.ensure(chunk_scan_words(n1)))
    return fail(c, SIXDGS_ERR_OOM, "density plan buffers");
  launch_density_plan(params, n, stats, *d, c->dens_dec.p, c->dens_cnt.p, st);
  launch_count_scan(c->dens_cnt.p, n, c->dens_off.p, c->counters.p + 5, c->dens_state.p, c->counters.p + 3, st);
  uint32_t total = 0;
  if (hipMemcpyAsync(c->host_counters, c->counters.p + 5, sizeof(uint32_t), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(c, SIXDGS_ERR_HIP, "density plan read-back failed");
  total = c->host_counters[0];
  c->dens_params = params;
  c->dens_n = n;
  c->dens_total = total;
  *n_out = total;
  return check_launch(c, "density plan");
}

sixdgs_status sixdgs_densify_plan(sixdgs_ctx* c, const float* params, int64_t n, const float* stats,
                                  const sixdgs_density_settings* d, int64_t* n_out, void* stream) {
  if (!c) return SIXDGS_ERR_INVALID_ARG;
  return debug_after(c, stream, densify_plan_body(c, params, n, stats, d, n_out, stream), 0);
}

static sixdgs_status densify_apply_body(sixdgs_ctx* c, const float* params, const float* m, const float* v,
                                        const float* lambda_raw, int64_t n, const float* noise, float* params_out,
                                        float* m_out, float* v_out, float* lambda_out, int64_t n_out, void* stream) {
  if (!c) return SIXDGS_ERR_INVALID_ARG;
  if (c->dens_n < 0 || c->dens_n != n || c->dens_params != params || c->dens_total != n_out)
    return fail(c, SIXDGS_ERR_STATE, "no matching sixdgs_densify_plan for these params, n and n_out");
  const bool mom = m || v || m_out || v_out;
  if (mom && !(m && v && m_out && v_out)) return fail(c, SIXDGS_ERR_INVALID_ARG, "m, v, m_out, v_out: all or none");
  if ((lambda_raw != nullptr) != (lambda_out != nullptr))
    return fail(c, SIXDGS_ERR_INVALID_ARG, "lambda_raw and lambda_out: both or neither");
  if (n > 0 && (!noise || (n_out > 0 && !params_out))) return fail(c, SIXDGS_ERR_INVALID_ARG, "NULL argument");
  launch_density_apply(params, m, v, lambda_raw, n, noise, c->dens_dec.p, c->dens_off.p, params_out,
                       mom ? m_out : nullptr, mom ? v_out : nullptr, lambda_out, n_out, (hipStream_t)stream);
  return check_launch(c, "density apply");
}

sixdgs_status sixdgs_densify_apply(sixdgs_ctx* c, const float* params, const float* m, const float* v,
                                   const float* lambda_raw, int64_t n, const float* noise, float* params_out,
                                   float* m_out, float* v_out, float* lambda_out, int64_t n_out, void* stream) {
  if (!c) return SIXDGS_ERR_INVALID_ARG;
  return debug_after(c, stream,
                     densify_apply_body(c, params, m, v, lambda_raw, n, noise, params_out, m_out, v_out, lambda_out,
                                        n_out, stream),
                     0);
}

sixdgs_status sixdgs_set_lambda(sixdgs_ctx* c, const float* lambda_raw, float* grad_lambda) {
  if (!c) return SIXDGS_ERR_INVALID_ARG;
  if (!lambda_raw && grad_lambda) return fail(c, SIXDGS_ERR_INVALID_ARG, "grad_lambda needs lambda_raw");
  c->lambda_raw = lambda_raw;
  c->grad_lambda = grad_lambda;
  return SIXDGS_OK;
}

static sixdgs_status bin_body(sixdgs_ctx* c, int64_t n, const sixdgs_camera* cams, int32_t ncam, const float* u,
                              const float* v, const float* ex, const float* ey, const float* depth, const int32_t* alive,
                              void* stream) {
  if (!c) return SIXDGS_ERR_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  if (n < 0) return fail(c, SIXDGS_ERR_INVALID_ARG, "n must be >= 0");
  if (n > 0 && (!u || !v || !ex || !ey || !depth || !alive)) return fail(c, SIXDGS_ERR_INVALID_ARG, "NULL array");
  ViewTable vt;
  int64_t total_px = 0;
  std::string why = build_views(c->s, n, cams, ncam, vt, total_px);
  if (!why.empty()) return fail(c, SIXDGS_ERR_INVALID_ARG, why);
  const int64_t E = n * ncam;
  if (E > kMaxItems) return fail(c, SIXDGS_ERR_INVALID_ARG, "n * cameras must stay below 2^30");
  c->have_fwd = false;
  if (!ensure_entries(c, E)) return fail(c, SIXDGS_ERR_OOM, "entry buffers");
  c->vt = vt;
  launch_import_records(u, v, ex, ey, depth, alive, vt, c->rec.p, c->tiles.p, st);
  c->bin_depth = depth;
  sixdgs_status rc = prepare_binning(c, E);
  if (rc == SIXDGS_OK) rc = run_binning(c, E, false, st);
  c->bin_depth = nullptr;
  c->fwd_E = E;
  c->fwd_px = 0;
  c->fwd_n = n;
  c->stream = st;
  return rc;
}

sixdgs_status sixdgs_bin(sixdgs_ctx* c, int64_t n, const sixdgs_camera* cams, int32_t ncam, const float* u,
                         const float* v, const float* ex, const float* ey, const float* depth, const int32_t* alive,
                         void* stream) {
  if (!c) return SIXDGS_ERR_INVALID_ARG;
  return debug_after(c, stream, bin_body(c, n, cams, ncam, u, v, ex, ey, depth, alive, stream), 1, depth);
}

sixdgs_status sixdgs_export(sixdgs_ctx* c, int32_t what, void* dst, int64_t cap_bytes, int64_t* written) {
  if (!c || !dst || !written) return fail(c, SIXDGS_ERR_INVALID_ARG, "NULL argument");
  *written = 0;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, SIXDGS_ERR_HIP, "stream synchronisation failed");
  uint32_t cnt[4] = {0, 0, 0, 0};
  if (c->counters.p && hipMemcpy(cnt, c->counters.p, sizeof(cnt), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(c, SIXDGS_ERR_HIP, "counter read-back failed");
  const int64_t E = c->fwd_E;
  const int64_t P = std::min<int64_t>(cnt[1], c->sb.pcap);
  const int64_t T = c->vt.total_tiles;
  auto copy = [&](const void* src, int64_t bytes) -> sixdgs_status {
    if (bytes > cap_bytes) return fail(c, SIXDGS_ERR_INVALID_ARG, "destination too small");
    if (bytes > 0 && hipMemcpy(dst, src, (size_t)bytes, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(c, SIXDGS_ERR_HIP, "read-back failed");
    *written = bytes;
    return SIXDGS_OK;
  };
  switch (what) {
    case SIXDGS_EXPORT_RECORDS: return copy(c->rec.p, E * (int64_t)sizeof(Rec));
    case SIXDGS_EXPORT_TILES: return copy(c->tiles.p, E * 4);
    case SIXDGS_EXPORT_VALUES: return copy(c->sb.pval[c->sb.psorted], P * 4);
    case SIXDGS_EXPORT_RANGES: return copy(c->ranges.p, T * 8);
    case SIXDGS_EXPORT_T_FINAL: return copy(c->T_final.p, c->fwd_px * 4);
    case SIXDGS_EXPORT_LAST: return copy(c->last.p, c->fwd_px * 4);
    case SIXDGS_EXPORT_COUNTS:
      if (!c->counts_valid) return fail(c, SIXDGS_ERR_STATE, "counts need SIXDGS_FLAG_COUNTS at the forward");
      return copy(c->counts.p, c->fwd_px * 4);
    case SIXDGS_EXPORT_KEYS: {
      if (P * 8 > cap_bytes) return fail(c, SIXDGS_ERR_INVALID_ARG, "destination too small");
      std::vector<uint32_t> tk(P), tv(P);
      std::vector<Rec> rec(E);
      if ((P && (hipMemcpy(tk.data(), c->sb.pkey[c->sb.psorted], P * 4, hipMemcpyDeviceToHost) != hipSuccess ||
                 hipMemcpy(tv.data(), c->sb.pval[c->sb.psorted], P * 4, hipMemcpyDeviceToHost) != hipSuccess)) ||
          (E && hipMemcpy(rec.data(), c->rec.p, E * sizeof(Rec), hipMemcpyDeviceToHost) != hipSuccess))
        return fail(c, SIXDGS_ERR_HIP, "read-back failed");
      uint64_t* o = (uint64_t*)dst;
      for (int64_t i = 0; i < P; i++) {
        uint32_t bits;
        std::memcpy(&bits, &rec[tv[i]].c.w, 4);
        o[i] = ((uint64_t)tk[i] << 32) | bits;
      }
      *written = P * 8;
      return SIXDGS_OK;
    }
    case SIXDGS_EXPORT_SIZES: {
      if (cap_bytes < 56) return fail(c, SIXDGS_ERR_INVALID_ARG, "destination too small");
      int64_t* o = (int64_t*)dst;
      o[0] = E;
      o[1] = cnt[1];
      o[2] = T;
      o[3] = cnt[0];
      o[4] = c->fwd_px;
      o[5] = c->fwd_batch;
      o[6] = c->fwd_chunk;
      *written = 56;
      return SIXDGS_OK;
    }
    default: return fail(c, SIXDGS_ERR_INVALID_ARG, "unknown export item");
  }
}

sixdgs_status sixdgs_check(sixdgs_ctx* c) {
  if (!c) return SIXDGS_ERR_INVALID_ARG;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, SIXDGS_ERR_HIP, "stream synchronisation failed");
  const sixdgs_status rc = debug_after(c, c->stream, SIXDGS_OK, 0);
  if (rc != SIXDGS_OK) return rc;
  if (!c->counters.p) return SIXDGS_OK;
  uint32_t cnt[4];
  if (hipMemcpy(cnt, c->counters.p, sizeof(cnt), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(c, SIXDGS_ERR_HIP, "counter read-back failed");
  if (cnt[3]) {
    const uint32_t zero = 0;
    (void)hipMemcpy(c->counters.p + 3, &zero, 4, hipMemcpyHostToDevice);
    return fail(c, SIXDGS_ERR_HIP, "radix sort look-back wait timed out (output invalid)");
  }
  if (cnt[2]) {
    const uint32_t zero = 0;
    (void)hipMemcpy(c->counters.p + 2, &zero, 4, hipMemcpyHostToDevice);
    return fail(c, SIXDGS_ERR_CAPACITY,
                "pair capacity exceeded: " + std::to_string(cnt[1]) + " pairs > " + std::to_string(c->sb.pcap));
  }
  return SIXDGS_OK;
}

sixdgs_status sixdgs_debug_buffer(sixdgs_ctx* c, const char* name, void** ptr, int64_t* bytes) {
  if (!c || !name || !ptr || !bytes) return fail(c, SIXDGS_ERR_INVALID_ARG, "NULL argument");
  *ptr = nullptr;
  *bytes = 0;
  if (!c->debug) return fail(c, SIXDGS_ERR_STATE, "not in the debug mode");
  bool known = false;
  for_each_buf(c, [&](auto& b, const char* nm) {
    if (std::strcmp(nm, name) == 0) {
      known = true;
      *ptr = b.p;
      *bytes = b.bytes();
    }
  });
  if (!known) return fail(c, SIXDGS_ERR_INVALID_ARG, std::string("no workspace buffer called ") + name);
  if (!*ptr) return fail(c, SIXDGS_ERR_STATE, std::string(name) + " is not allocated");
  return SIXDGS_OK;
}

sixdgs_status sixdgs_set_timing(sixdgs_ctx* c, int32_t mask) {
  if (!c) return SIXDGS_ERR_INVALID_ARG;
  collect_timing(c);
  c->timing_mask = mask;
  for (int k = 0; k < SIXDGS_K_COUNT; k++) {
    c->ms[k] = 0;
    c->launches[k] = 0;
  }
  return SIXDGS_OK;
}

sixdgs_status sixdgs_kernel_time(sixdgs_ctx* c, int32_t kernel, double* ms, int64_t* launches) {
  if (!c || !ms || !launches || kernel < 0 || kernel >= SIXDGS_K_COUNT)
    return fail(c, SIXDGS_ERR_INVALID_ARG, "bad argument");
  collect_timing(c);
  *ms = c->ms[kernel];
  *launches = c->launches[kernel];
  return SIXDGS_OK;
}

}  // extern "C"
