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

// ------------------------------------------------------------ radix sort
// The depth order's passes (the pair sort's are further below): one kernel
// per pass, where each workgroup takes the next 4096 items in ticket
// order, ranks them stably by digit in LDS, and finds where its items of each
// digit go by looking back over the per-digit counts that earlier workgroups
// publish (a status word per digit: aggregate of that workgroup alone, or
// inclusive prefix through it).  The global digit offsets come from a
// histogram of every pass taken before the first pass, so each pass reads and
// writes the data once.  Tickets make a workgroup wait only on workgroups that
// are already running; the wait is bounded and reports a timeout in the error
// word instead of spinning forever.
constexpr int kRItems = 16;
constexpr int kRItemsSmall = 8;           // short sorts: 2048 items per workgroup, 2x the workgroups
constexpr int64_t kLargeSort = 1 << 20;    // from this many entries the depth sort uses kRItems
constexpr int64_t kLargePairs = 1 << 24;   // from this pair capacity on the pair sort uses kRItems
// Items per thread of the pair sort's workgroups (and pairs per emission
// block: kBlock times this).  Measured: 2,048-pair blocks 5 us faster on one
// 800x800 view (3.2M pairs), 4,096 6% faster on eight 1080p views.
inline int pair_items(int64_t pcap) { return pcap >= kLargePairs ? kRItems : kRItemsSmall; }
constexpr uint32_t kStAgg = 1u << 30;
constexpr uint32_t kStIncl = 2u << 30;
constexpr uint32_t kStVal = kStAgg - 1u;
constexpr int kMaxSpin = 1 << 20;

// The global digit histograms are kept as kGhCopies copies that workgroups
// add into by workgroup index: every workgroup adds its counts of every digit
// at its end, and atomics on one word serialise (about 17 ns apart on MI355X:
// 800 workgroups adding into 128 words took 16 us, 14 of them waiting), so
// the copies cut each word's queue; readers sum the copies.
constexpr int kGhCopies = 16;
constexpr int kGhStride = kMaxPasses * 256;  // words from one copy to the next

__device__ __forceinline__ uint32_t* ghist_copy(uint32_t* ghist, int64_t blk) {
  return ghist + (blk % kGhCopies) * kGhStride;
}
// Total count of digit d in the histogram at g (one pass's row of copy 0).
__device__ __forceinline__ uint32_t ghist_total(const uint32_t* g, int d) {
  uint32_t s = 0;
#pragma unroll
  for (int c = 0; c < kGhCopies; c++) s += g[c * kGhStride + d];
  return s;
}

// Radix state of one sort: global digit histograms, tickets and look-back
// status words, laid out in one buffer.
struct RadixState {
  uint32_t* ghist;        // [kGhCopies][kMaxPasses][256]
  uint32_t* tickets;      // [kMaxPasses] passes, then [2] scans (padded to 256 words)
  uint32_t* status;       // [kMaxPasses][nblk][256]: look-back words (depth sort), chunk tables (pair sort)
  uint64_t* scan_status;  // [2][nscan] look-back words of the two scans over entries
  int64_t nblk, nscan;
  int items;              // items per thread of the passes
  __host__ __device__ int64_t words() const {
    return (int64_t)kMaxPasses * 256 * (nblk + 1 + kGhCopies) + 4 * nscan;
  }
};

inline int64_t radix_blocks(int64_t bound, int items) {
  const int64_t chunk = (int64_t)kBlock * items;
  return (bound + chunk - 1) / chunk;
}

RadixState radix_state(uint32_t* base, int64_t bound, int items, bool with_scans) {
  RadixState r;
  r.items = items;
  r.nblk = radix_blocks(bound, items);
  r.nscan = with_scans ? (bound + kChunk - 1) / kChunk : 0;
  r.ghist = base;
  r.tickets = base + kGhCopies * kGhStride;
  r.status = base + (kGhCopies + 1) * kGhStride;
  r.scan_status = reinterpret_cast<uint64_t*>(r.status + (int64_t)kMaxPasses * r.nblk * 256);
  return r;
}

// Pass layout of a key with `bits` significant bits: ceil(bits / 8) passes of
// equal digit width (fewer buckets per pass when the key is short).
struct RadixPlan {
  int npass, dbits;
};
RadixPlan radix_plan(int bits) {
  RadixPlan p;
  p.npass = (bits + 7) / 8;
  if (p.npass < 1) p.npass = 1;
  p.dbits = (bits + p.npass - 1) / p.npass;
  if (p.dbits < 1) p.dbits = 1;
  return p;
}

__device__ __forceinline__ uint32_t st_load(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_store(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive prefix over earlier workgroups from their 64-bit look-back words
// (flag in the high half, a 32-bit sum in the low half); bounded wait.
constexpr uint64_t kSc64Agg = 1ull << 32;
constexpr uint64_t kSc64Incl = 2ull << 32;

__device__ __forceinline__ uint64_t st_load64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_store64(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive prefix over workgroups [0, blk) from their look-back words at
// status[j * stride] (an aggregate of workgroup j alone, or an inclusive
// prefix through it).  A window of predecessors is read per round trip and
// summed nearest first until an inclusive word; a word not yet published is
// waited on, boundedly (a timeout sets *err and gives up).
constexpr int kLookWin = 4;

__device__ __forceinline__ bool lb_incl(uint32_t s) { return (s & kStIncl) != 0; }
__device__ __forceinline__ uint32_t lb_val(uint32_t s) { return s & kStVal; }
__device__ __forceinline__ uint32_t lb_load(const uint32_t* p) { return st_load(p); }
__device__ __forceinline__ bool lb_incl(uint64_t s) { return (s & kSc64Incl) != 0; }
__device__ __forceinline__ uint32_t lb_val(uint64_t s) { return (uint32_t)s; }
__device__ __forceinline__ uint64_t lb_load(const uint64_t* p) { return st_load64(p); }

template <class W>
__device__ uint32_t look_back(const W* status, int64_t stride, int64_t blk, uint32_t* err) {
  uint32_t excl = 0;
  for (int64_t j = blk - 1; j >= 0; j -= kLookWin) {
    W s[kLookWin];
#pragma unroll
    for (int k = 0; k < kLookWin; k++) s[k] = (j - k >= 0) ? lb_load(status + (j - k) * stride) : W(0);
#pragma unroll
    for (int k = 0; k < kLookWin; k++) {
      if (j - k < 0) return excl;  // not reached: the first workgroup publishes an inclusive word
      W v = s[k];
      for (int spin = 0; !v && spin < kMaxSpin; spin++) {
        __builtin_amdgcn_s_sleep(1);
        v = lb_load(status + (j - k) * stride);
      }
      if (!v) {
        atomicOr(err, 1u);
        return excl;
      }
      excl += lb_val(v);
      if (lb_incl(v)) return excl;
    }
  }
  return excl;
}

// Single-pass exclusive scan of f(i) over i < count, handing (i, prefix,
// value) to g.  Workgroups take 2048 items each in ticket order and chain
// their prefixes through look-back words; the workgroup holding the last item
// writes the total.  With HIST, g.key(i) of every item with a non-zero value
// also enters the digit histograms of a 4-pass, 8-bit radix sort.
template <class F, class G, bool HIST>
__global__ void __launch_bounds__(kBlock) k_scan1(F f, G g, const uint32_t* count_ptr, uint32_t fixed, uint32_t cap,
                                                  uint32_t* ticket, uint64_t* status, uint32_t* total_out,
                                                  uint32_t* ghist, uint32_t* err) {
  __shared__ uint32_t s_blk, s_pre;
  __shared__ uint32_t s_h[HIST ? kMaxPasses : 1][256];
  const int t = threadIdx.x;
  if (t == 0) s_blk = atomicAdd(ticket, 1u);
  if (HIST) {
#pragma unroll
    for (int p = 0; p < kMaxPasses; p++) s_h[p][t] = 0;
  }
  __syncthreads();
  const int64_t blk = s_blk;
  const uint32_t count = load_count(count_ptr, fixed, cap);
  const int64_t start = blk * kChunk;
  if (start >= count) {  // uniform
    if (blk == 0 && t == 0 && total_out) *total_out = 0u;
    return;
  }
  const int64_t base = start + (int64_t)t * kItems;
  uint32_t v[kItems];
  uint32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kItems; k++) {
    v[k] = (base + k < count) ? f(base + k) : 0u;
    sum += v[k];
  }
  uint32_t total;
  uint32_t pre = block_scan_excl(sum, total);
  if (t == 0) {
    uint64_t* my = status + blk;
    uint32_t excl = 0;
    if (blk == 0) {
      st_store64(my, kSc64Incl | total);
    } else {
      st_store64(my, kSc64Agg | total);
      excl = look_back(status, 1, blk, err);
      st_store64(my, kSc64Incl | (uint32_t)(excl + total));
    }
    s_pre = excl;
    if (start + kChunk >= count && total_out) *total_out = excl + total;
  }
  __syncthreads();
  pre += s_pre;
#pragma unroll
  for (int k = 0; k < kItems; k++) {
    if (base + k < count) {
      g(base + k, pre, v[k]);
      if constexpr (HIST) {
        if (v[k]) {
          const uint32_t key = g.key(base + k);
#pragma unroll
          for (int p = 0; p < kMaxPasses; p++) atomicAdd(&s_h[p][(key >> (8 * p)) & 255u], 1u);
        }
      }
    }
    pre += v[k];
  }
  if (HIST) {
    __syncthreads();
    uint32_t* gh = ghist_copy(ghist, blk);
#pragma unroll
    for (int p = 0; p < kMaxPasses; p++)
      if (s_h[p][t]) atomicAdd(&gh[p * 256 + t], s_h[p][t]);
  }
}

template <bool HIST, class F, class G>
void scan1(F f, G g, const uint32_t* count_ptr, uint32_t fixed, uint32_t cap, int64_t bound, uint32_t* ticket,
           uint64_t* status, uint32_t* total_out, uint32_t* ghist, uint32_t* err, hipStream_t st) {
  int64_t nb = (bound + kChunk - 1) / kChunk;
  if (nb < 1) nb = 1;  // one workgroup writes a zero total
  hipLaunchKernelGGL((k_scan1<F, G, HIST>), dim3((unsigned)nb), dim3(kBlock), 0, st, f, g, count_ptr, fixed, cap,
                     ticket, status, total_out, ghist, err);
}

// Up to four word ranges a preparation kernel zeroes.
struct ZeroList {
  uint32_t* p[4];
  int64_t n[4];
};

// Zeroes the first zero_words words of a radix state, the regions of z and
// the tile ranges; when given the depth-sorted entries, records for every
// emission block the sorted entry whose pairs contain the block's first pair
// (normally the pair-offset scan records them; this is for pair buffers that
// were regrown after it).
__global__ void __launch_bounds__(kBlock) k_stage_prep(RadixState rs, int64_t zero_words, ZeroList z,
                                                       uint2* __restrict__ ranges, int64_t nranges,
                                                       const uint32_t* __restrict__ counters,
                                                       const uint32_t* __restrict__ tiles,
                                                       const uint32_t* __restrict__ dval,
                                                       const uint32_t* __restrict__ poff, uint32_t pcap,
                                                       uint32_t* __restrict__ blk_start, int64_t nblk_start,
                                                       uint32_t chunk) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < zero_words / 4) reinterpret_cast<uint4*>(rs.ghist)[i] = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
  for (int k = 0; k < 4; k++)
    if (z.p[k] && i < z.n[k]) z.p[k][i] = 0u;
  if (ranges && i < nranges) ranges[i] = make_uint2(0xFFFFFFFFu, 0u);  // merged by min / max
  if (blk_start && i < (int64_t)counters[0] && counters[1] <= pcap) {
    const uint32_t o = poff[i];
    const uint32_t end = o + tiles[dval[i]];
    for (uint32_t b = (o + chunk - 1) / chunk; (int64_t)b * chunk < end && b < nblk_start; b++)
      blk_start[b] = (uint32_t)i;
  }
}

// One stable pass over the digit at `shift` (width dbits) of keys[0, count).
template <int ITEMS>
__global__ void __launch_bounds__(kBlock) k_onesweep(const uint32_t* __restrict__ kin,
                                                     const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
                                                     uint32_t* __restrict__ vout, const uint32_t* count_ptr,
                                                     uint32_t cap, int shift, int dbits,
                                                     const uint32_t* __restrict__ ghist, uint32_t* ticket,
                                                     uint32_t* status, uint32_t* err) {
  constexpr int kChunkI = kBlock * ITEMS;
  constexpr int kWaveItems = kChunkI / kWaves;
  __shared__ uint32_t s_key[kChunkI];
  __shared__ uint32_t s_val[kChunkI];
  __shared__ uint32_t s_wc[kWaves][256];  // per-wave digit counts, then exclusive prefixes over waves
  __shared__ uint32_t s_lex[256];         // exclusive digit offsets inside the workgroup
  __shared__ uint32_t s_gb[256];          // output position of LDS slot 0 of each digit
  __shared__ uint32_t s_blk;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  if (t == 0) s_blk = atomicAdd(ticket, 1u);
#pragma unroll
  for (int w = 0; w < kWaves; w++) s_wc[w][t] = 0;
  __syncthreads();
  const int64_t blk = s_blk;
  const uint32_t count = load_count(count_ptr, cap, cap);
  const int64_t base = blk * kChunkI;
  if (base >= count) return;  // uniform; no later workgroup has items, so none waits on this one
  const uint32_t mask = (1u << dbits) - 1u;
  const bool own = (uint32_t)t <= mask;
  const uint32_t gh = own ? ghist_total(ghist, t) : 0u;  // issued early: used after the look-back
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t wbase = base + (int64_t)wv * kWaveItems;  // each wavefront ranks consecutive items
  uint32_t key[ITEMS], val[ITEMS], loc[ITEMS];
#pragma unroll
  for (int r = 0; r < ITEMS; r++) {
    const int64_t i = wbase + r * 64 + lane;
    key[r] = i < count ? kin[i] : 0u;
    val[r] = i < count ? vin[i] : 0u;
  }
  // every key has the same digit in this pass (e.g. the exponent byte of
  // depths within one octave): the stable order is the input order, so the
  // pass is a copy (decided while the loads are in flight)
  if (__syncthreads_or(own && gh == count)) {
#pragma unroll
    for (int r = 0; r < ITEMS; r++) {
      const int64_t i = wbase + r * 64 + lane;
      if (i < count) {
        kout[i] = key[r];
        vout[i] = val[r];
      }
    }
    return;
  }
#pragma unroll
  for (int r = 0; r < ITEMS; r++) {
    const bool valid = wbase + r * 64 + lane < count;
    const uint32_t d = (key[r] >> shift) & mask;
    uint64_t m = __ballot(valid);
    for (int b = 0; b < dbits; b++) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    const uint32_t rank = __popcll(m & lt);
    // every lane of a digit group reads the running count before its first lane moves it on
    const uint32_t pre = s_wc[wv][d];
    if (valid && rank == 0) s_wc[wv][d] = pre + (uint32_t)__popcll(m);
    loc[r] = valid ? ((pre + rank) << 8 | d) : 0xFFFFFFFFu;
  }
  __syncthreads();
  uint32_t tot = 0;
#pragma unroll
  for (int w = 0; w < kWaves; w++) {
    const uint32_t c = s_wc[w][t];
    s_wc[w][t] = tot;
    tot += c;
  }
  uint32_t* my = status + blk * 256 + t;
  if (own) st_store(my, (blk == 0 ? kStIncl : kStAgg) | tot);
  uint32_t total;
  const uint32_t lex = block_scan_excl(tot, total);
  s_lex[t] = lex;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < ITEMS; r++) {
    if (loc[r] != 0xFFFFFFFFu) {
      const uint32_t d = loc[r] & 255u;
      const uint32_t pos = s_lex[d] + s_wc[wv][d] + (loc[r] >> 8);
      if (pos < (uint32_t)kChunkI) {  // always true; guards LDS against inconsistent counts
        s_key[pos] = key[r];
        s_val[pos] = val[r];
      }
    }
  }
  // exclusive prefix of this digit over the earlier workgroups
  uint32_t excl = 0;
  if (own && blk > 0) {
    excl = look_back(status + t, 256, blk, err);
    st_store(my, kStIncl | (excl + tot));
  }
  const uint32_t gex = block_scan_excl(gh, total);
  s_gb[t] = gex + excl - lex;  // modular: adding an LDS slot of this digit lands in range
  __syncthreads();
  const int64_t left = (int64_t)count - base;
  const int nvalid = left < kChunkI ? (int)left : kChunkI;
#pragma unroll
  for (int r = 0; r < ITEMS; r++) {
    const int k = r * kBlock + t;
    if (k < nvalid) {
      const uint32_t kk = s_key[k];
      const uint32_t o = s_gb[(kk >> shift) & mask] + (uint32_t)k;
      if (o < count) {  // always true for a consistent histogram; guards the buffers
        kout[o] = kk;
        vout[o] = s_val[k];
      }
    }
  }
}

// ---------------------------------------------------- reduce-then-scan passes
// The pair sort's passes in three launches with no chain between workgroups
// (the wait on earlier workgroups' counts dominated the one-kernel passes at
// a few thousand workgroups, and the emission counts the first pass's chunks
// for free):
// each chunk's digit counts (2,048 or 4,096 items, pair_items; k_digit_count;
// for the first pass the emission writes them), one scan per digit over the
// chunks, offset by the
// counts of the smaller digits (k_digit_scan), and the stable scatter
// (k_digit_scatter), where chunk b's items of digit d start at the scanned
// table entry (d, b).  The tables are [digit][chunk]; chunks past the item
// count are read as zero.

// Stable ranks of the workgroup's items by digit, each wavefront over its
// consecutive items (ballot matching): loc[r] = (rank in the wavefront << 8) |
// digit, or ~0 past the count; on return wc[w][d] holds the count of digit d in
// the wavefronts before w, and the return value is the workgroup's count of
// digit threadIdx.x.
template <int ITEMS>
__device__ __forceinline__ uint32_t rank_chunk(uint32_t (*wc)[256], const uint32_t (&key)[ITEMS], int64_t wbase,
                                               uint32_t count, int shift, int dbits, uint32_t (&loc)[ITEMS]) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const uint32_t mask = (1u << dbits) - 1u;
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
  for (int r = 0; r < ITEMS; r++) {
    const bool valid = wbase + r * 64 + lane < count;
    const uint32_t d = (key[r] >> shift) & mask;
    uint64_t m = __ballot(valid);
    for (int b = 0; b < dbits; b++) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    const uint32_t rank = __popcll(m & lt);
    // every lane of a digit group reads the running count before its first lane moves it on
    const uint32_t pre = wc[wv][d];
    if (valid && rank == 0) wc[wv][d] = pre + (uint32_t)__popcll(m);
    loc[r] = valid ? ((pre + rank) << 8 | d) : 0xFFFFFFFFu;
  }
  __syncthreads();
  uint32_t tot = 0;
#pragma unroll
  for (int w = 0; w < kWaves; w++) {
    const uint32_t c = wc[w][t];
    wc[w][t] = tot;
    tot += c;
  }
  return tot;
}

template <int ITEMS>
__global__ void __launch_bounds__(kBlock) k_digit_count(const uint32_t* __restrict__ kin, const uint32_t* count_ptr,
                                                        uint32_t cap, int shift, int dbits,
                                                        uint32_t* __restrict__ table, int64_t nblk) {
  constexpr int kChunkI = kBlock * ITEMS;
  __shared__ uint32_t s_wc[kWaves][256];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t blk = blockIdx.x;
  const uint32_t count = load_count(count_ptr, cap, cap);
  const int64_t base = blk * kChunkI;
  if (base >= count) return;  // uniform
#pragma unroll
  for (int w = 0; w < kWaves; w++) s_wc[w][t] = 0;
  __syncthreads();
  const int64_t wbase = base + (int64_t)wv * (kChunkI / kWaves);
  uint32_t key[ITEMS], loc[ITEMS];
#pragma unroll
  for (int r = 0; r < ITEMS; r++) {
    const int64_t i = wbase + r * 64 + lane;
    key[r] = i < count ? kin[i] : 0u;
  }
  const uint32_t tot = rank_chunk<ITEMS>(s_wc, key, wbase, count, shift, dbits, loc);
  if ((uint32_t)t < (1u << dbits)) table[(int64_t)t * nblk + blk] = tot;
}

// One workgroup per digit d: table[d][b] <- (items of digits < d) + (items of
// digit d in chunks < b), over the chunks that hold items.
__global__ void __launch_bounds__(kBlock) k_digit_scan(uint32_t* __restrict__ table, int64_t nblk,
                                                       const uint32_t* count_ptr, uint32_t cap, int chunk_items,
                                                       const uint32_t* __restrict__ ghist) {
  const int d = blockIdx.x, t = threadIdx.x;
  const uint32_t count = load_count(count_ptr, cap, cap);
  const int64_t used = ((int64_t)count + chunk_items - 1) / chunk_items;
  uint32_t dbase;  // items of the digits below d: the total of this scan
  block_scan_excl((uint32_t)t < (uint32_t)d ? ghist_total(ghist, t) : 0u, dbase);
  uint32_t* row = table + (int64_t)d * nblk;
  const int64_t per = (used + kBlock - 1) / kBlock;
  const int64_t b0 = min<int64_t>((int64_t)t * per, used), b1 = min<int64_t>(b0 + per, used);
  uint32_t sum = 0;
  for (int64_t b = b0; b < b1; b++) sum += row[b];
  uint32_t all;
  uint32_t pre = dbase + block_scan_excl(sum, all);
  for (int64_t b = b0; b < b1; b++) {
    const uint32_t c = row[b];
    row[b] = pre;
    pre += c;
  }
}

template <int ITEMS>
__global__ void __launch_bounds__(kBlock) k_digit_scatter(const uint32_t* __restrict__ kin,
                                                          const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
                                                          uint32_t* __restrict__ vout, const uint32_t* count_ptr,
                                                          uint32_t cap, int shift, int dbits,
                                                          const uint32_t* __restrict__ table, int64_t nblk,
                                                          uint2* __restrict__ ranges, uint32_t total_tiles,
                                                          const uint32_t* __restrict__ counters, uint32_t pcap) {
  constexpr int kChunkI = kBlock * ITEMS;
  __shared__ uint32_t s_key[kChunkI];
  __shared__ uint32_t s_val[kChunkI];
  __shared__ uint32_t s_wc[kWaves][256];
  __shared__ uint32_t s_lex[256];
  __shared__ uint32_t s_gb[256];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t blk = blockIdx.x;
  const uint32_t count = load_count(count_ptr, cap, cap);
  const int64_t base = blk * kChunkI;
  if (base >= count) return;  // uniform
  const uint32_t mask = (1u << dbits) - 1u;
  const bool own = (uint32_t)t <= mask;
  const uint32_t gstart = own ? table[(int64_t)t * nblk + blk] : 0u;  // issued early
#pragma unroll
  for (int w = 0; w < kWaves; w++) s_wc[w][t] = 0;
  __syncthreads();
  const int64_t wbase = base + (int64_t)wv * (kChunkI / kWaves);
  uint32_t key[ITEMS], val[ITEMS], loc[ITEMS];
#pragma unroll
  for (int r = 0; r < ITEMS; r++) {
    const int64_t i = wbase + r * 64 + lane;
    key[r] = i < count ? kin[i] : 0u;
    val[r] = i < count ? vin[i] : 0u;
  }
  const uint32_t tot = rank_chunk<ITEMS>(s_wc, key, wbase, count, shift, dbits, loc);
  uint32_t total;
  const uint32_t lex = block_scan_excl(tot, total);
  s_lex[t] = lex;
  s_gb[t] = gstart - lex;  // modular: adding an LDS slot of this digit lands in range
  __syncthreads();
#pragma unroll
  for (int r = 0; r < ITEMS; r++) {
    if (loc[r] != 0xFFFFFFFFu) {
      const uint32_t d = loc[r] & 255u;
      const uint32_t pos = s_lex[d] + s_wc[wv][d] + (loc[r] >> 8);
      if (pos < (uint32_t)kChunkI) {  // always true; guards LDS against inconsistent counts
        s_key[pos] = key[r];
        s_val[pos] = val[r];
      }
    }
  }
  __syncthreads();
  const int64_t left = (int64_t)count - base;
  const int nvalid = left < kChunkI ? (int)left : kChunkI;
  // the last pass also finds the tiles' ranges: the workgroup's digit runs
  // are sorted by the whole key, so where the key changes inside a run is
  // where the output changes key; a run's ends meet other workgroups' items,
  // so every end is merged with a device min / max (ranges start at
  // (UINT_MAX, 0); the tile order turns the untouched ones into (0, 0)).
  // Skipped when the pairs overflowed: every range then stays empty.
  const bool with_ranges = ranges && counters[1] <= pcap;
#pragma unroll
  for (int r = 0; r < ITEMS; r++) {
    const int k = r * kBlock + t;
    if (k < nvalid) {
      const uint32_t kk = s_key[k];
      const uint32_t o = s_gb[(kk >> shift) & mask] + (uint32_t)k;
      if (o < count) {  // always true for consistent tables; guards the buffers
        kout[o] = kk;
        vout[o] = s_val[k];
        if (with_ranges && kk < total_tiles) {
          if (k == 0 || s_key[k - 1] != kk) atomicMin(&ranges[kk].x, o);
          if (k == nvalid - 1 || s_key[k + 1] != kk) atomicMax(&ranges[kk].y, o + 1u);
        }
      }
    }
  }
}

// Sorts (keys, vals) of length *count_ptr (<= bound) over plan.npass digits
// whose histograms are already in rs.ghist; returns which buffer of the
// ping-pong pair holds the result.
int radix_sort(uint32_t* keys[2], uint32_t* vals[2], const uint32_t* count_ptr, int64_t bound, RadixPlan plan,
               const RadixState& rs, uint32_t* err, hipStream_t st) {
  const int64_t nb = rs.nblk;
  int cur = 0;
  if (nb == 0) return cur;
  for (int p = 0; p < plan.npass; p++) {
    auto k = rs.items == kRItems ? k_onesweep<kRItems> : k_onesweep<kRItemsSmall>;
    hipLaunchKernelGGL(k, dim3((unsigned)nb), dim3(kBlock), 0, st, keys[cur], vals[cur], keys[cur ^ 1],
                       vals[cur ^ 1], count_ptr, (uint32_t)bound, p * plan.dbits, plan.dbits, rs.ghist + p * 256,
                       rs.tickets + p, rs.status + (int64_t)p * rs.nblk * 256, err);
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
  const float* depth;
  uint32_t* dkey;
  uint32_t* dval;
  // depths of binned entries exceed z_near > 0, so their bit patterns order as the values
  __device__ uint32_t key(int64_t i) const { return __float_as_uint(depth[i]); }
  __device__ void operator()(int64_t i, uint32_t pre, uint32_t v) const {
    if (v) {
      dkey[pre] = key(i);
      dval[pre] = (uint32_t)i;
    }
  }
};
struct SortedTiles {
  const uint32_t* tiles;
  const uint32_t* dval;
  __device__ uint32_t operator()(int64_t i) const { return tiles[dval[i]]; }
};
// The pair offset of each depth-sorted entry, and for every emission block
// that starts inside the entry's pairs, the entry.
struct StoreOffset {
  uint32_t* poff;
  uint32_t* blk_start;
  int64_t nblk_start;
  int64_t chunk;  // pairs per emission block
  __device__ void operator()(int64_t i, uint32_t pre, uint32_t n) const {
    poff[i] = pre;
    for (int64_t b = ((int64_t)pre + chunk - 1) / chunk; b * chunk < (int64_t)pre + n && b < nblk_start; b++)
      blk_start[b] = (uint32_t)i;
  }
};

// Load-balanced pair emission: workgroup b writes pairs [chunk b, chunk (b + 1))
// in depth order.  It walks the depth-sorted entries from the one holding its
// first pair, 256 entries per step; each thread finds the entry of a pair by
// binary search over the entries' pair offsets in LDS and the pair's tile from
// its index in the entry's tile rectangle (row-major, the order the count
// came from), so consecutive threads write consecutive pairs whatever the
// entries' sizes.  The digit histograms of every pass of the tile sort are
// accumulated on the way.
__global__ void __launch_bounds__(kBlock) k_emit(ViewTable vt, const Rec* __restrict__ rec,
                                                 const uint32_t* __restrict__ dval, const uint32_t* __restrict__ poff,
                                                 const uint32_t* __restrict__ blk_start,
                                                 uint32_t* __restrict__ counters, uint32_t pcap, int npass, int dbits,
                                                 uint32_t* __restrict__ ghist, uint32_t* __restrict__ pkey,
                                                 uint32_t* __restrict__ pval, uint32_t* __restrict__ table0,
                                                 uint32_t chunk) {
  __shared__ uint32_t s_o[kBlock + 1];  // pair offset of each entry of the step; [kBlock]: the next step's
  __shared__ uint32_t s_e[kBlock];      // entry id
  __shared__ uint32_t s_base[kBlock];   // global id of the rectangle's first tile
  __shared__ uint32_t s_w[kBlock];      // rectangle width in tiles
  __shared__ uint32_t s_ntx[kBlock];    // tiles per row of the entry's view
  __shared__ uint32_t s_h[kMaxPasses][256];
  const int t = threadIdx.x;
  // blk_start holds an entry for every workgroup of the grid: read with the
  // counts, not after them
  uint32_t ib = blk_start[blockIdx.x];
  const uint32_t nb = counters[0];
  const uint32_t P = counters[1];
  if (P > pcap) {
    if (blockIdx.x == 0 && t == 0) counters[2] = 1u;
    return;
  }
  const int64_t p0 = (int64_t)blockIdx.x * chunk;
  if (p0 >= P) return;  // uniform
  const uint32_t p1 = (uint32_t)min<int64_t>(p0 + chunk, (int64_t)P);
  const uint32_t mask = (1u << dbits) - 1u;
#pragma unroll
  for (int p = 0; p < kMaxPasses; p++) s_h[p][t] = 0;
  for (;;) {
    const uint32_t i = ib + t;
    if (i < nb) {
      const uint32_t o = poff[i];
      s_o[t] = o;
      // an entry whose pairs start past this block is never chosen by the
      // search below: its record is not read (a block of 2,048 pairs needs
      // about a hundred of the step's entries)
      if (o < p1) {
        const uint32_t e = dval[i];
        const ViewDesc& vd = vt.v[e / (uint64_t)vt.n];
        const float4 ra = rec[e].a, rb = rec[e].b;
        int x0, y0, x1, y1;
        tile_rect(ra.x, ra.y, rb.z, rb.w, vt.tile_shift_x, vt.tile_shift_y, vd.ntx, vd.nty, x0, y0, x1, y1);
        s_e[t] = e;
        s_base[t] = (uint32_t)(vd.tile_base + y0 * vd.ntx + x0);
        s_w[t] = (uint32_t)(x1 - x0);
        s_ntx[t] = (uint32_t)vd.ntx;
      }
    } else {
      s_o[t] = P;  // past the last entry: never chosen by the search below
    }
    if (t == 0) s_o[kBlock] = (uint64_t)ib + kBlock < nb ? poff[ib + kBlock] : P;
    __syncthreads();
    const uint32_t lo = max((uint32_t)p0, s_o[0]);
    const uint32_t hi = min(p1, s_o[kBlock]);
    for (uint32_t q = lo + t; q < hi; q += kBlock) {
      int j = 0;  // last entry of the step whose pairs start at or before q
#pragma unroll
      for (int step = kBlock / 2; step > 0; step >>= 1)
        if (s_o[j + step] <= q) j += step;
      const uint32_t local = q - s_o[j];
      const uint32_t w = s_w[j];
      const uint32_t ty = local / w;
      const uint32_t key = s_base[j] + ty * s_ntx[j] + (local - ty * w);
      pkey[q] = key;
      pval[q] = s_e[j];
      // Lanes whose digit equals the first active lane's add as one: the
      // tiles of one wide Gaussian share their high digits, and same-address
      // shared-memory atomics from one wavefront serialise.
      const uint64_t act = __ballot(1);
      const bool leader = __lane_id() == (unsigned)(__ffsll((unsigned long long)act) - 1);
      for (int p = 0; p < npass; p++) {
        const uint32_t d = (key >> (p * dbits)) & mask;
        const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
        const uint64_t same = __ballot(d == d0);
        if (d != d0)
          atomicAdd(&s_h[p][d], 1u);
        else if (leader)
          atomicAdd(&s_h[p][d0], (uint32_t)__popcll(same));
      }
    }
    const bool done = s_o[kBlock] >= p1;
    __syncthreads();
    if (done) break;
    ib += kBlock;
  }
  uint32_t* gh = ghist_copy(ghist, blockIdx.x);
  for (int p = 0; p < npass; p++)
    if (s_h[p][t]) atomicAdd(&gh[p * 256 + t], s_h[p][t]);
  // this chunk's counts of the first pass's digits (the chunk is the pass's)
  if ((uint32_t)t <= mask) table0[(int64_t)t * gridDim.x + blockIdx.x] = s_h[0][t];
}

// Order in which the compositing kernels take the tiles: longest lists first
// (buckets of log2 of the pair count, heaviest bucket first), so the tiles
// whose per-pixel walks are longest start before the light ones and the
// kernels' tails shrink (LPT scheduling); the order inside a bucket is
// arbitrary.  Up to kOrderOneGroup tiles one workgroup of 1024 threads takes
// the bucket histogram, its scan and the scatter; beyond, k_order_count and
// k_order_place split the same over many workgroups, which reserve their
// places inside each bucket with one device atomic per bucket.  Workgroups
// past the ordering ones zero the screen-space gradient accumulators of the
// binned entries (when g2d is given) for the backward that may follow.
constexpr int kOrderThreads = 1024;
constexpr int kOrderBuckets = 33;
constexpr int kOrderU = 8;                                   // tiles per thread and round
constexpr uint32_t kOrderGroupTiles = kOrderThreads * kOrderU;
constexpr uint32_t kOrderOneGroup = 2 * kOrderGroupTiles;    // one workgroup orders up to this many tiles
constexpr int kOrderStateWords = 2 * kOrderBuckets;          // bucket counts, then bucket cursors

// the bucket of tile k (heaviest first: slot 0 holds 2^31 pairs and more, the
// last slot the empty tiles), -1 past the last tile
// FIX: also turn a range the sort left untouched ((UINT_MAX, 0): a tile
// without pairs) into (0, 0), the form every later reader expects.
template <bool FIX>
__device__ __forceinline__ int order_slot(uint2* __restrict__ ranges, uint32_t total_tiles, uint32_t k) {
  if (k >= total_tiles) return -1;
  const uint2 r = ranges[k];
  uint32_t c = r.y - r.x;
  if (r.x >= r.y) {
    c = 0;
    if (FIX && (r.x | r.y)) ranges[k] = make_uint2(0u, 0u);
  }
  return kOrderBuckets - 1 - (c ? 32 - __clz(c) : 0);
}

// Zeroes the gradient-accumulator row of entry i if it is binned (a tile
// count above zero).  Taken in entry order, consecutive threads write
// consecutive rows (the binned entries in depth order would scatter them),
// and the unbinned ones cost a 4-byte read.
__device__ __forceinline__ void zero_g2d_entry(int64_t i, const uint32_t* __restrict__ tiles, int64_t E,
                                               float* __restrict__ g2d) {
  if (i < E && tiles[i] > 0) {
    float* p = g2d + i * kG2D;
#pragma unroll
    for (int k = 0; k < kG2D; k++) p[k] = 0.f;
  }
}

// exclusive scan of the kOrderBuckets counts in s (one thread; tiny)
__device__ __forceinline__ void scan_buckets(uint32_t* s) {
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int b = 0; b < kOrderBuckets; b++) {
      const uint32_t c = s[b];
      s[b] = acc;
      acc += c;
    }
  }
}

__global__ void __launch_bounds__(kOrderThreads) k_tile_order(uint2* __restrict__ ranges, uint32_t total_tiles,
                                                              uint32_t* __restrict__ order,
                                                              const uint32_t* __restrict__ tiles, int64_t E,
                                                              float* __restrict__ g2d) {
  __shared__ uint32_t s_h[kOrderBuckets];
  const int t = threadIdx.x;
  if (blockIdx.x > 0) {
    zero_g2d_entry((int64_t)(blockIdx.x - 1) * kOrderThreads + t, tiles, E, g2d);
    return;
  }
  if (t < kOrderBuckets) s_h[t] = 0;
  __syncthreads();
  const uint32_t span = (total_tiles + kOrderGroupTiles - 1) / kOrderGroupTiles * kOrderGroupTiles;
  for (uint32_t k0 = t; k0 < span; k0 += kOrderGroupTiles) {
    int b[kOrderU];
#pragma unroll
    for (int u = 0; u < kOrderU; u++) b[u] = order_slot<true>(ranges, total_tiles, k0 + u * kOrderThreads);
#pragma unroll
    for (int u = 0; u < kOrderU; u++)
      if (b[u] >= 0) atomicAdd(&s_h[b[u]], 1u);
  }
  __syncthreads();
  scan_buckets(s_h);
  __syncthreads();
  for (uint32_t k0 = t; k0 < span; k0 += kOrderGroupTiles) {
    int b[kOrderU];
#pragma unroll
    for (int u = 0; u < kOrderU; u++) b[u] = order_slot<false>(ranges, total_tiles, k0 + u * kOrderThreads);
#pragma unroll
    for (int u = 0; u < kOrderU; u++) {
      const uint32_t pos = b[u] >= 0 ? atomicAdd(&s_h[b[u]], 1u) : 0u;
      if (b[u] >= 0 && pos < total_tiles) order[pos] = k0 + u * kOrderThreads;
    }
  }
}

// Many tiles, first half: bucket counts of kOrderGroupTiles tiles per
// workgroup, added into state[0, kOrderBuckets) (zeroed beforehand).
__global__ void __launch_bounds__(kOrderThreads) k_order_count(uint2* __restrict__ ranges, uint32_t total_tiles,
                                                               uint32_t ngroups, uint32_t* __restrict__ state,
                                                               const uint32_t* __restrict__ tiles, int64_t E,
                                                               float* __restrict__ g2d) {
  __shared__ uint32_t s_h[kOrderBuckets];
  const int t = threadIdx.x;
  if (blockIdx.x >= ngroups) {
    zero_g2d_entry((int64_t)(blockIdx.x - ngroups) * kOrderThreads + t, tiles, E, g2d);
    return;
  }
  if (t < kOrderBuckets) s_h[t] = 0;
  __syncthreads();
  const uint32_t k0 = blockIdx.x * kOrderGroupTiles + t;
  int b[kOrderU];
#pragma unroll
  for (int u = 0; u < kOrderU; u++) b[u] = order_slot<true>(ranges, total_tiles, k0 + u * kOrderThreads);
#pragma unroll
  for (int u = 0; u < kOrderU; u++)
    if (b[u] >= 0) atomicAdd(&s_h[b[u]], 1u);
  __syncthreads();
  if (t < kOrderBuckets && s_h[t]) atomicAdd(&state[t], s_h[t]);
}

// Second half: each workgroup ranks its tiles inside their buckets, reserves
// a run of places per bucket (device atomics on state[kOrderBuckets + b]) and
// writes the tiles there.
__global__ void __launch_bounds__(kOrderThreads) k_order_place(uint2* __restrict__ ranges, uint32_t total_tiles,
                                                               uint32_t* __restrict__ state,
                                                               uint32_t* __restrict__ order) {
  __shared__ uint32_t s_off[kOrderBuckets];   // first place of each bucket
  __shared__ uint32_t s_loc[kOrderBuckets];   // this workgroup's count per bucket, then its reserved base
  const int t = threadIdx.x;
  if (t < kOrderBuckets) {
    s_off[t] = state[t];
    s_loc[t] = 0;
  }
  __syncthreads();
  scan_buckets(s_off);
  const uint32_t k0 = blockIdx.x * kOrderGroupTiles + t;
  int b[kOrderU];
  uint32_t rank[kOrderU];
#pragma unroll
  for (int u = 0; u < kOrderU; u++) b[u] = order_slot<false>(ranges, total_tiles, k0 + u * kOrderThreads);
#pragma unroll
  for (int u = 0; u < kOrderU; u++) rank[u] = b[u] >= 0 ? atomicAdd(&s_loc[b[u]], 1u) : 0u;
  __syncthreads();
  if (t < kOrderBuckets && s_loc[t]) s_loc[t] = atomicAdd(&state[kOrderBuckets + t], s_loc[t]);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kOrderU; u++) {
    if (b[u] < 0) continue;
    const uint32_t pos = s_off[b[u]] + s_loc[b[u]] + rank[u];
    if (pos < total_tiles) order[pos] = k0 + u * kOrderThreads;
  }
}

__global__ void __launch_bounds__(kBlock) k_zero_g2d(const uint32_t* __restrict__ tiles, int64_t E,
                                                     float* __restrict__ g2d) {
  zero_g2d_entry((int64_t)blockIdx.x * kBlock + threadIdx.x, tiles, E, g2d);
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

namespace {
RadixState depth_state(const SortBuffers& b) {
  // short sorts take small workgroups (more of them in flight); long ones the pairs' size
  return radix_state(b.rstate_depth, b.E, b.E >= kLargeSort ? kRItems : kRItemsSmall, true);
}
}  // namespace

// One preparation for the whole stage: the depth sort's state, the pair
// sort's histograms, the tile ranges, the tile order's counts and the
// backward work-item count.
BinPrep bin_prep(const SortBuffers& b) {
  const RadixState rs = depth_state(b);
  BinPrep bp{{b.rstate_depth, b.order_state, b.n_items, b.rstate_pairs},
             {rs.words(), (int64_t)kOrderStateWords, 1, (kGhCopies + 1) * kGhStride},
             b.ranges,
             b.total_tiles,
             0};
  bp.threads = bp.nranges;
  for (int k = 0; k < 4; k++) bp.threads = std::max(bp.threads, bp.n[k]);
  return bp;
}

void launch_bin_count(SortBuffers& b, bool prepped, hipStream_t st) {
  const uint32_t E = (uint32_t)b.E;
  const RadixState rs = depth_state(b);
  const RadixPlan plan{4, 8};
  if (!prepped) {
    const ZeroList z{{b.order_state, b.n_items, b.rstate_pairs, nullptr},
                     {(int64_t)kOrderStateWords, 1, (kGhCopies + 1) * kGhStride, 0}};
    int64_t prep = rs.words() / 4;
    for (int k = 0; k < 3; k++) prep = std::max(prep, z.n[k]);
    prep = std::max(prep, b.total_tiles);
    hipLaunchKernelGGL(k_stage_prep, dim3((unsigned)((prep + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, rs,
                       rs.words(), z, b.ranges, b.total_tiles, (const uint32_t*)b.counters,
                       (const uint32_t*)nullptr, (const uint32_t*)nullptr, (const uint32_t*)nullptr, 0u,
                       (uint32_t*)nullptr, (int64_t)0, 0u);
  }
  // compaction of the binned entries with their depth keys, and the depth keys' digit histograms
  scan1<true>(BinnedFlag{b.tiles}, CompactDepth{b.depth, b.dkey[0], b.dval[0]}, nullptr, E, E, b.E,
              rs.tickets + kMaxPasses, rs.scan_status, &b.counters[0], rs.ghist, &b.counters[3], st);
  // depth order (stable: equal depths keep entry order)
  b.dsorted = radix_sort(b.dkey, b.dval, &b.counters[0], b.E, plan, rs, &b.counters[3], st);
  // pair offsets in depth order
  scan1<false>(SortedTiles{b.tiles, b.dval[b.dsorted]},
               StoreOffset{b.poff, b.blk_start, b.nblk_start, (int64_t)kBlock * pair_items(b.pcap)},
               &b.counters[0], 0u, E, b.E,
               rs.tickets + kMaxPasses + 1, rs.scan_status + rs.nscan, &b.counters[1], (uint32_t*)nullptr,
               &b.counters[3], st);
}

void launch_bin_emit(SortBuffers& b, const ViewTable& vt, int64_t pairs_hint, bool regrown, hipStream_t st) {
  int bits = 1;
  while ((1ll << bits) < (int64_t)vt.total_tiles) bits++;
  const RadixPlan plan = radix_plan(bits);
  const int64_t bound = pairs_hint < b.pcap ? pairs_hint : b.pcap;
  const int items = pair_items(b.pcap);
  const uint32_t chunk = (uint32_t)(kBlock * items);
  const RadixState rs = radix_state(b.rstate_pairs, bound, items, false);
  if (regrown) {
    // the passes write every table entry they read: only the histograms (and
    // the unused tickets) start from zero
    const int64_t zero_words = (kGhCopies + 1) * kGhStride;
    const ZeroList z{{nullptr, nullptr, nullptr, nullptr}, {0, 0, 0, 0}};
    const int64_t prep = std::max<int64_t>(zero_words / 4, b.E);
    hipLaunchKernelGGL(k_stage_prep, dim3((unsigned)((prep + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, rs,
                       zero_words, z, (uint2*)nullptr, (int64_t)0, (const uint32_t*)b.counters,
                       (const uint32_t*)b.tiles, (const uint32_t*)b.dval[b.dsorted], (const uint32_t*)b.poff,
                       (uint32_t)b.pcap, b.blk_start, rs.nblk, chunk);
  }
  // the pairs, with every pass's digit histogram and the first pass's per-chunk
  // counts; then the passes, each a scan of the chunk counts and a scatter
  // (the chunk counts of later passes taken from their input)
  int cur = 0;
  if (rs.nblk) {
    const int64_t nb = rs.nblk;
    const uint32_t cap = (uint32_t)bound;
    hipLaunchKernelGGL(k_emit, dim3((unsigned)nb), dim3(kBlock), 0, st, vt, b.rec, b.dval[b.dsorted], b.poff,
                       b.blk_start, b.counters, (uint32_t)b.pcap, plan.npass, plan.dbits, rs.ghist, b.pkey[0],
                       b.pval[0], rs.status, chunk);
    for (int p = 0; p < plan.npass; p++) {
      uint32_t* table = rs.status + (int64_t)p * nb * 256;
      const int shift = p * plan.dbits;
      if (p > 0)
        hipLaunchKernelGGL(items == kRItems ? k_digit_count<kRItems> : k_digit_count<kRItemsSmall>, dim3((unsigned)nb),
                           dim3(kBlock), 0, st, b.pkey[cur],
                           (const uint32_t*)&b.counters[1], cap, shift, plan.dbits, table, nb);
      hipLaunchKernelGGL(k_digit_scan, dim3(1u << plan.dbits), dim3(kBlock), 0, st, table, nb,
                         (const uint32_t*)&b.counters[1], cap, (int)chunk, (const uint32_t*)(rs.ghist + p * 256));
      const bool last = p == plan.npass - 1;
      hipLaunchKernelGGL(items == kRItems ? k_digit_scatter<kRItems> : k_digit_scatter<kRItemsSmall>,
                         dim3((unsigned)nb), dim3(kBlock), 0, st, b.pkey[cur],
                         b.pval[cur], b.pkey[cur ^ 1], b.pval[cur ^ 1], (const uint32_t*)&b.counters[1], cap, shift,
                         plan.dbits, (const uint32_t*)table, nb, last ? b.ranges : nullptr,
                         (uint32_t)vt.total_tiles, (const uint32_t*)b.counters, (uint32_t)b.pcap);
      cur ^= 1;
    }
  }
  b.psorted = cur;
  // the tile order, and the gradient accumulators cleared for a backward
  const unsigned gz = b.g2d ? (unsigned)((b.E + kOrderThreads - 1) / kOrderThreads) : 0u;
  const uint32_t T = (uint32_t)vt.total_tiles;
  if (T <= kOrderOneGroup) {
    if (T > 0 || gz)
      hipLaunchKernelGGL(k_tile_order, dim3(1 + gz), dim3(kOrderThreads), 0, st, b.ranges, T,
                         b.tile_order, (const uint32_t*)b.tiles, b.E, b.g2d);
  } else {
    const uint32_t ng = (T + kOrderGroupTiles - 1) / kOrderGroupTiles;
    hipLaunchKernelGGL(k_order_count, dim3(ng + gz), dim3(kOrderThreads), 0, st, b.ranges, T, ng,
                       b.order_state, (const uint32_t*)b.tiles, b.E, b.g2d);
    hipLaunchKernelGGL(k_order_place, dim3(ng), dim3(kOrderThreads), 0, st, b.ranges, T,
                       b.order_state, b.tile_order);
  }
}

int64_t chunk_scan_words(int64_t n) { return 2 + 2 * ((n + kChunk - 1) / kChunk + 1); }

namespace {
struct CountVal {
  const uint32_t* c;
  __device__ uint32_t operator()(int64_t i) const { return c[i]; }
};
struct CountOffset {
  uint32_t* off;
  __device__ void operator()(int64_t i, uint32_t pre, uint32_t) const { off[i] = pre; }
};
__global__ void __launch_bounds__(kBlock) k_zero_words(uint32_t* __restrict__ p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = 0u;
}
}  // namespace

void launch_count_scan(const uint32_t* cnt, int64_t n, uint32_t* off, uint32_t* total, uint32_t* state,
                       uint32_t* err, hipStream_t st) {
  const int64_t words = chunk_scan_words(n);
  hipLaunchKernelGGL(k_zero_words, dim3((unsigned)((words + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, state, words);
  const uint32_t N = (uint32_t)n;
  scan1<false>(CountVal{cnt}, CountOffset{off}, nullptr, N, N, n, state, reinterpret_cast<uint64_t*>(state + 2), total,
               (uint32_t*)nullptr, err, st);
}

int64_t sort_state_words(int64_t bound, bool pairs) {
  // the pair state sized for the smaller blocks, whichever pair_items picks
  return radix_state(nullptr, bound, kRItemsSmall, !pairs).words();
}
int64_t sort_block_starts(int64_t pcap) { return radix_blocks(pcap, kRItemsSmall) + 1; }
int64_t order_state_words() { return kOrderStateWords; }

void launch_zero_g2d(const SortBuffers& b, float* g2d, hipStream_t st) {
  const unsigned g = (unsigned)((b.E + kBlock - 1) / kBlock);
  if (g) hipLaunchKernelGGL(k_zero_g2d, dim3(g), dim3(kBlock), 0, st, (const uint32_t*)b.tiles, b.E, g2d);
}

void launch_import_records(const float* u, const float* v, const float* ex, const float* ey, const float* depth,
                           const int32_t* alive, const ViewTable& vt, Rec* rec, uint32_t* tiles, hipStream_t st) {
  const int64_t E = vt.n * vt.nview;
  const unsigned g = (unsigned)((E + kBlock - 1) / kBlock);
  if (g) hipLaunchKernelGGL(k_import, dim3(g), dim3(kBlock), 0, st, u, v, ex, ey, depth, alive, vt, rec, tiles);
}

}  // namespace sixdgs
