// Integer stage of the rasteriser on gfx950: compaction of the binned entries,
// an LSD radix sort of their float32 depths, emission of one (tile, entry) pair
// per covered tile in depth order, a stable LSD radix sort of the pairs by
// global tile id and the per-tile [start, end) ranges.  Sorting depth before
// duplication makes the two-key (tile, depth) order cost 4 passes over the
// binned entries plus ceil(tile bits / 8) passes over the pairs, instead of a
// 64-bit sort of the pairs.
//
// Every kernel reads its element count from device memory and takes a grid
// sized by a host-side upper bound, so the stage needs no host round trip
// (and can be captured) when the pair capacity is fixed.
#include "internal.h"

namespace sixdgs {
namespace {

constexpr int kItems = 8;                     // items per thread
constexpr int kChunk = kBlock * kItems;       // items per workgroup (2048)
constexpr int kWaves = kBlock / 64;

__device__ __forceinline__ uint32_t load_count(const uint32_t* ptr, uint32_t fixed, uint32_t cap) {
  uint32_t c = ptr ? *ptr : fixed;
  return c < cap ? c : cap;
}

// Inclusive scan over a 64-lane wavefront.
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  return x;
}

// Exclusive scan of one value per thread over the workgroup; returns the
// exclusive prefix and the workgroup total.
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t x, uint32_t& total) {
  __shared__ uint32_t s_w[kWaves];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t inc = wave_scan_incl(x);
  if (lane == 63) s_w[wv] = inc;
  __syncthreads();
  uint32_t before = 0;
  total = 0;
#pragma unroll
  for (int w = 0; w < kWaves; w++) {
    const uint32_t s = s_w[w];
    before += (w < wv) ? s : 0u;
    total += s;
  }
  __syncthreads();
  return before + inc - x;
}

// ---------------------------------------------------------- generic scan
// Phase 1: per-workgroup sums of f(i) over i < count.
template <class F>
__global__ void __launch_bounds__(kBlock) k_scan_reduce(F f, const uint32_t* count_ptr, uint32_t fixed, uint32_t cap,
                                                        uint32_t* __restrict__ block_sums) {
  const uint32_t count = load_count(count_ptr, fixed, cap);
  const int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)threadIdx.x * kItems;
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kItems; k++)
    if (base + k < count) s += f(base + k);
  uint32_t total;
  block_scan_excl(s, total);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// Phase 2: one workgroup scans the block sums in place (exclusive) and writes the total.
__global__ void __launch_bounds__(kBlock) k_scan_top(uint32_t* __restrict__ block_sums, uint32_t nblocks,
                                                     uint32_t* __restrict__ total_out) {
  uint32_t carry = 0;
  for (uint32_t base = 0; base < nblocks; base += kChunk) {
    uint32_t v[kItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kItems; k++) {
      const uint32_t i = base + threadIdx.x * kItems + k;
      v[k] = i < nblocks ? block_sums[i] : 0u;
      s += v[k];
    }
    uint32_t total;
    uint32_t pre = block_scan_excl(s, total) + carry;
#pragma unroll
    for (int k = 0; k < kItems; k++) {
      const uint32_t i = base + threadIdx.x * kItems + k;
      if (i < nblocks) block_sums[i] = pre;
      pre += v[k];
    }
    carry += total;
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

// Phase 3: exclusive prefix of f(i) handed to g(i, prefix, value).
template <class F, class G>
__global__ void __launch_bounds__(kBlock) k_scan_apply(F f, G g, const uint32_t* count_ptr, uint32_t fixed,
                                                       uint32_t cap, const uint32_t* __restrict__ block_sums) {
  const uint32_t count = load_count(count_ptr, fixed, cap);
  const int64_t base = (int64_t)blockIdx.x * kChunk + (int64_t)threadIdx.x * kItems;
  uint32_t v[kItems];
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kItems; k++) {
    v[k] = (base + k < count) ? f(base + k) : 0u;
    s += v[k];
  }
  uint32_t total;
  uint32_t pre = block_scan_excl(s, total) + block_sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kItems; k++) {
    if (base + k < count) g(base + k, pre, v[k]);
    pre += v[k];
  }
}

template <class F, class G>
void scan(F f, G g, const uint32_t* count_ptr, uint32_t fixed, uint32_t cap, int64_t bound, uint32_t* block_sums,
          uint32_t* total_out, hipStream_t st) {
  const uint32_t nb = (uint32_t)((bound + kChunk - 1) / kChunk);
  if (nb == 0) return;
  hipLaunchKernelGGL((k_scan_reduce<F>), dim3(nb), dim3(kBlock), 0, st, f, count_ptr, fixed, cap, block_sums);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kBlock), 0, st, block_sums, nb, total_out);
  hipLaunchKernelGGL((k_scan_apply<F, G>), dim3(nb), dim3(kBlock), 0, st, f, g, count_ptr, fixed, cap, block_sums);
}

// ------------------------------------------------------------ radix sort
__global__ void __launch_bounds__(kBlock) k_radix_hist(const uint32_t* __restrict__ keys, const uint32_t* count_ptr,
                                                       uint32_t cap, int shift, uint32_t* __restrict__ hist,
                                                       uint32_t nblocks) {
  __shared__ uint32_t s_h[256];
  s_h[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t count = load_count(count_ptr, cap, cap);
  const int64_t base = (int64_t)blockIdx.x * kChunk;
#pragma unroll
  for (int r = 0; r < kItems; r++) {
    const int64_t i = base + r * kBlock + threadIdx.x;
    if (i < count) atomicAdd(&s_h[(keys[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)threadIdx.x * nblocks + blockIdx.x] = s_h[threadIdx.x];
}

// Stable scatter: items are ranked in index order within the workgroup (256
// consecutive items per round; within a wavefront equal digits are matched
// with 8 ballots), then placed after all smaller digits and all earlier
// workgroups' items of the same digit.
__global__ void __launch_bounds__(kBlock) k_radix_scatter(const uint32_t* __restrict__ kin,
                                                          const uint32_t* __restrict__ vin,
                                                          uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                          const uint32_t* count_ptr, uint32_t cap, int shift,
                                                          const uint32_t* __restrict__ hist, uint32_t nblocks) {
  __shared__ uint32_t s_off[256];
  __shared__ uint32_t s_cnt[kWaves][256];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const uint32_t count = load_count(count_ptr, cap, cap);
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  if (base >= count) return;  // uniform over the workgroup
  s_off[t] = hist[(int64_t)t * nblocks + blockIdx.x];
#pragma unroll
  for (int w = 0; w < kWaves; w++) s_cnt[w][t] = 0;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int r = 0; r < kItems; r++) {
    const int64_t i = base + r * kBlock + t;
    if (base + r * kBlock >= count) break;  // uniform
    const bool valid = i < count;
    const uint32_t key = valid ? kin[i] : 0u;
    const uint32_t val = valid ? vin[i] : 0u;
    const uint32_t dig = (key >> shift) & 255u;
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      const bool bit = (dig >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    const uint32_t rank = __popcll(m & lt);
    if (valid && rank == 0) s_cnt[wv][dig] = __popcll(m);
    __syncthreads();
    if (valid) {
      uint32_t off = s_off[dig] + rank;
      for (int w = 0; w < wv; w++) off += s_cnt[w][dig];
      kout[off] = key;
      vout[off] = val;
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int w = 0; w < kWaves; w++) {
      add += s_cnt[w][t];
      s_cnt[w][t] = 0;
    }
    s_off[t] += add;
    __syncthreads();
  }
}

struct HistVal {
  const uint32_t* h;
  __device__ uint32_t operator()(int64_t i) const { return h[i]; }
};
struct HistStore {
  uint32_t* h;
  __device__ void operator()(int64_t i, uint32_t pre, uint32_t) const { h[i] = pre; }
};

// Sorts (keys, vals) of length *count_ptr (<= bound) by the low `bits` bits;
// returns which buffer of the ping-pong pair holds the result.
int radix_sort(uint32_t* keys[2], uint32_t* vals[2], const uint32_t* count_ptr, int64_t bound, int bits,
               uint32_t* hist, uint32_t* scan_blocks, hipStream_t st) {
  const uint32_t nb = (uint32_t)((bound + kChunk - 1) / kChunk);
  int cur = 0;
  if (nb == 0) return cur;
  const uint32_t cap = (uint32_t)bound;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(kBlock), 0, st, keys[cur], count_ptr, cap, shift, hist, nb);
    scan(HistVal{hist}, HistStore{hist}, nullptr, 256u * nb, 256u * nb, (int64_t)256 * nb, scan_blocks, nullptr, st);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(kBlock), 0, st, keys[cur], vals[cur], keys[cur ^ 1],
                       vals[cur ^ 1], count_ptr, cap, shift, hist, nb);
    cur ^= 1;
  }
  return cur;
}

// ------------------------------------------------------------ the stage
struct BinnedFlag {
  const uint32_t* tiles;
  __device__ uint32_t operator()(int64_t i) const { return tiles[i] > 0 ? 1u : 0u; }
};
struct CompactDepth {
  const Rec* rec;
  uint32_t* dkey;
  uint32_t* dval;
  __device__ void operator()(int64_t i, uint32_t pre, uint32_t v) const {
    if (v) {
      // depths of binned entries exceed z_near > 0, so their bit patterns order as the values
      dkey[pre] = __float_as_uint(rec[i].c.w);
      dval[pre] = (uint32_t)i;
    }
  }
};
struct SortedTiles {
  const uint32_t* tiles;
  const uint32_t* dval;
  __device__ uint32_t operator()(int64_t i) const { return tiles[dval[i]]; }
};
struct StoreOffset {
  uint32_t* poff;
  __device__ void operator()(int64_t i, uint32_t pre, uint32_t) const { poff[i] = pre; }
};

__global__ void __launch_bounds__(kBlock) k_emit(ViewTable vt, const Rec* __restrict__ rec,
                                                 const uint32_t* __restrict__ tiles,
                                                 const uint32_t* __restrict__ dval, const uint32_t* __restrict__ poff,
                                                 uint32_t* __restrict__ counters, uint32_t pcap,
                                                 uint32_t* __restrict__ pkey, uint32_t* __restrict__ pval) {
  const uint32_t nb = counters[0];
  const uint32_t P = counters[1];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (P > pcap) {
    if (i == 0) counters[2] = 1u;
    return;
  }
  if (i >= nb) return;
  const uint32_t e = dval[i];
  const int view = (int)(e / (uint64_t)vt.n);
  const ViewDesc& vd = vt.v[view];
  const Rec r = rec[e];
  int x0, y0, x1, y1;
  tile_rect(r.a.x, r.a.y, r.b.z, r.b.w, vt.tile_shift_x, vt.tile_shift_y, vd.ntx, vd.nty, x0, y0, x1, y1);
  uint32_t o = poff[i];
  // the rectangle is the one the tile count came from; the bound only guards the buffers
  const uint32_t stop = min(o + tiles[e], P);
  for (int ty = y0; ty < y1; ty++)
    for (int tx = x0; tx < x1; tx++) {
      if (o >= stop) return;
      pkey[o] = (uint32_t)(vd.tile_base + ty * vd.ntx + tx);
      pval[o] = e;
      o++;
    }
}

__global__ void __launch_bounds__(kBlock) k_fill_u2(uint2* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = make_uint2(0u, 0u);
}

__global__ void __launch_bounds__(kBlock) k_ranges(const uint32_t* __restrict__ pkey, const uint32_t* counters,
                                                   uint32_t pcap, uint32_t total_tiles, uint2* __restrict__ ranges) {
  const uint32_t P = counters[1];
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (P > pcap || i >= P) return;  // on overflow the pair lists were not written: leave every range empty
  const uint32_t k = pkey[i];
  if (k >= total_tiles) return;
  if (i == 0 || pkey[i - 1] != k) ranges[k].x = (uint32_t)i;
  if (i == (int64_t)P - 1 || pkey[i + 1] != k) ranges[k].y = (uint32_t)(i + 1);
}

__global__ void __launch_bounds__(kBlock) k_zero_g2d(const uint32_t* __restrict__ dval, const uint32_t* counters,
                                                     float* __restrict__ g2d) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= counters[0]) return;
  float* p = g2d + (int64_t)dval[i] * kG2D;
#pragma unroll
  for (int k = 0; k < kG2D; k++) p[k] = 0.f;
}

__global__ void __launch_bounds__(kBlock) k_import(const float* __restrict__ u, const float* __restrict__ v,
                                                   const float* __restrict__ ex, const float* __restrict__ ey,
                                                   const float* __restrict__ depth,
                                                   const int32_t* __restrict__ alive, ViewTable vt,
                                                   Rec* __restrict__ rec, uint32_t* __restrict__ tiles) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t E = vt.n * vt.nview;
  if (e >= E) return;
  uint32_t count = 0;
  if (alive[e]) {
    const ViewDesc& vd = vt.v[e / vt.n];
    int x0, y0, x1, y1;
    tile_rect(u[e], v[e], ex[e], ey[e], vt.tile_shift_x, vt.tile_shift_y, vd.ntx, vd.nty, x0, y0, x1, y1);
    count = (uint32_t)((x1 - x0) * (y1 - y0));
    Rec r;
    r.a = make_float4(u[e], v[e], 0.f, 0.f);
    r.b = make_float4(0.f, 0.f, ex[e], ey[e]);
    r.c = make_float4(0.f, 0.f, 0.f, depth[e]);
    rec[e] = r;
  }
  tiles[e] = count;
}

}  // namespace

void launch_bin_count(SortBuffers& b, hipStream_t st) {
  const uint32_t E = (uint32_t)b.E;
  // compaction of the binned entries with their depth keys
  scan(BinnedFlag{b.tiles}, CompactDepth{b.rec, b.dkey[0], b.dval[0]}, nullptr, E, E, b.E, b.scan_blocks,
       &b.counters[0], st);
  // depth order (stable: equal depths keep entry order)
  b.dsorted = radix_sort(b.dkey, b.dval, &b.counters[0], b.E, 32, b.hist, b.scan_blocks, st);
  // pair offsets in depth order
  scan(SortedTiles{b.tiles, b.dval[b.dsorted]}, StoreOffset{b.poff}, &b.counters[0], 0u, E, b.E, b.scan_blocks,
       &b.counters[1], st);
}

void launch_bin_emit(SortBuffers& b, const ViewTable& vt, int64_t pairs_hint, hipStream_t st) {
  const unsigned ge = (unsigned)((b.E + kBlock - 1) / kBlock);
  if (ge)
    hipLaunchKernelGGL(k_emit, dim3(ge), dim3(kBlock), 0, st, vt, b.rec, b.tiles, b.dval[b.dsorted], b.poff, b.counters,
                       (uint32_t)b.pcap, b.pkey[0], b.pval[0]);
  int bits = 1;
  while ((1ll << bits) < (int64_t)vt.total_tiles) bits++;
  const int64_t bound = pairs_hint < b.pcap ? pairs_hint : b.pcap;
  b.psorted = radix_sort(b.pkey, b.pval, &b.counters[1], bound, bits, b.hist, b.scan_blocks, st);
  const unsigned gt = (unsigned)((vt.total_tiles + kBlock - 1) / kBlock);
  if (gt) hipLaunchKernelGGL(k_fill_u2, dim3(gt), dim3(kBlock), 0, st, b.ranges, (int64_t)vt.total_tiles);
  const unsigned gp = (unsigned)((bound + kBlock - 1) / kBlock);
  if (gp)
    hipLaunchKernelGGL(k_ranges, dim3(gp), dim3(kBlock), 0, st, b.pkey[b.psorted], b.counters, (uint32_t)b.pcap,
                       (uint32_t)vt.total_tiles, b.ranges);
}

void launch_zero_g2d(const SortBuffers& b, float* g2d, hipStream_t st) {
  const unsigned g = (unsigned)((b.E + kBlock - 1) / kBlock);
  if (g) hipLaunchKernelGGL(k_zero_g2d, dim3(g), dim3(kBlock), 0, st, b.dval[b.dsorted], b.counters, g2d);
}

void launch_import_records(const float* u, const float* v, const float* ex, const float* ey, const float* depth,
                           const int32_t* alive, const ViewTable& vt, Rec* rec, uint32_t* tiles, hipStream_t st) {
  const int64_t E = vt.n * vt.nview;
  const unsigned g = (unsigned)((E + kBlock - 1) / kBlock);
  if (g) hipLaunchKernelGGL(k_import, dim3(g), dim3(kBlock), 0, st, u, v, ex, ey, depth, alive, vt, rec, tiles);
}

}  // namespace sixdgs
