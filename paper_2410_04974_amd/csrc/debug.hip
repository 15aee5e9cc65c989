// Host-side invariants of one binning, for the debug mode and for tests that
// run without a GPU: the tile counts, the (tile, depth, entry) order of the
// sorted pairs, the tile ranges, the compositing order and the backward's
// chunked work items, all checked on host copies.
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

namespace {

std::string at(const char* what, int64_t i) { return std::string(what) + " " + std::to_string(i); }

int bit_length(uint32_t v) {
  int b = 0;
  while (v) {
    b++;
    v >>= 1;
  }
  return b;
}

// The first violated invariant, or "" if there is none.
std::string check(const sixdgs_bin_state& s) {
  const int64_t E = s.E, P = s.P, T = s.T;
  // tile counts
  uint64_t sum = 0;
  for (int64_t e = 0; e < E; e++) sum += s.tiles[e];
  if (sum != (uint64_t)P)
    return "the tile counts sum to " + std::to_string(sum) + ", not to the " + std::to_string(P) + " pairs";
  // the pairs: tile ids, entry ids, order, and each entry's multiplicity
  std::vector<uint32_t> seen(E > 0 ? E : 1, 0u);
  for (int64_t i = 0; i < P; i++) {
    const uint32_t t = s.keys[i], e = s.values[i];
    if ((int64_t)t >= T) return at("pair", i) + ": tile id " + std::to_string(t) + " >= " + std::to_string(T);
    if ((int64_t)e >= E) return at("pair", i) + ": entry id " + std::to_string(e) + " >= " + std::to_string(E);
    if (++seen[e] > s.tiles[e]) return at("entry", e) + " appears in more pairs than its " +
                                       std::to_string(s.tiles[e]) + " tiles";
    if (i > 0) {
      const uint32_t tp = s.keys[i - 1], ep = s.values[i - 1];
      if (t < tp) return at("pair", i) + ": tile ids decrease";
      if (t == tp) {
        const float d = s.depth[e], dp = s.depth[ep];
        if (d < dp || (d == dp && e <= ep))
          return at("pair", i) + ": not after pair " + std::to_string(i - 1) + " in (depth, entry) order within tile " +
                 std::to_string(t);
      }
    }
  }
  for (int64_t e = 0; e < E; e++)
    if (seen[e] != s.tiles[e]) return at("entry", e) + " appears in fewer pairs than its tiles";
  // ranges: the exact run of each tile
  std::vector<int64_t> first(T > 0 ? T : 1, -1), end(T > 0 ? T : 1, -1);
  for (int64_t i = 0; i < P; i++) {
    const uint32_t t = s.keys[i];
    if (first[t] < 0) first[t] = i;
    end[t] = i + 1;
  }
  for (int64_t t = 0; t < T; t++) {
    const uint32_t b = s.ranges[2 * t], en = s.ranges[2 * t + 1];
    if (first[t] < 0) {
      if (b != 0u || en != 0u) return at("tile", t) + " has no pairs but range [" + std::to_string(b) + ", " +
                                      std::to_string(en) + ")";
    } else if ((int64_t)b != first[t] || (int64_t)en != end[t]) {
      return at("tile", t) + ": range [" + std::to_string(b) + ", " + std::to_string(en) + ") but its pairs are [" +
             std::to_string(first[t]) + ", " + std::to_string(end[t]) + ")";
    }
  }
  auto run = [&](uint32_t t) { return s.ranges[2 * t + 1] - s.ranges[2 * t]; };
  // the compositing order: a permutation, heavier bit lengths first
  if (s.order) {
    std::vector<uint8_t> hit(T > 0 ? T : 1, 0);
    for (int64_t i = 0; i < T; i++) {
      const uint32_t t = s.order[i];
      if ((int64_t)t >= T) return at("order position", i) + ": tile id " + std::to_string(t) + " out of range";
      if (hit[t]++) return at("order position", i) + ": tile " + std::to_string(t) + " listed twice";
      if (i > 0 && bit_length(run(t)) > bit_length(run(s.order[i - 1])))
        return at("order position", i) + ": a longer list after a shorter one";
    }
  }
  // the backward's work items: every (t, c) with c < nch[t] exactly once, in any order
  if (s.nch) {
    if (s.chunk < 1) return "chunk must be positive";
    std::vector<int64_t> item0(T + 1, 0);  // first item of each tile
    for (int64_t t = 0; t < T; t++) {
      const int64_t most = ((int64_t)run((uint32_t)t) + s.chunk - 1) / s.chunk;
      if ((int64_t)s.nch[t] > most)
        return at("tile", t) + ": " + std::to_string(s.nch[t]) + " chunks for a run of " +
               std::to_string(run((uint32_t)t)) + " pairs";
      item0[t + 1] = item0[t] + s.nch[t];
    }
    if (item0[T] != s.n_items)
      return std::to_string(s.n_items) + " work items, but the tiles' chunks add up to " + std::to_string(item0[T]);
    std::vector<uint8_t> hit((size_t)std::max<int64_t>(item0[T], 1), 0);
    for (int64_t k = 0; k < s.n_items; k++) {
      const uint32_t t = s.items[2 * k], c = s.items[2 * k + 1];
      if ((int64_t)t >= T) return at("work item", k) + ": tile id " + std::to_string(t) + " out of range";
      if (c >= s.nch[t])
        return at("work item", k) + ": chunk " + std::to_string(c) + " of tile " + std::to_string(t) + ", which has " +
               std::to_string(s.nch[t]);
      if (hit[item0[t] + c]++)
        return at("work item", k) + ": (" + std::to_string(t) + ", " + std::to_string(c) + ") listed twice";
    }
  }
  return "";
}

}  // namespace

extern "C" sixdgs_status sixdgs_debug_check_bins(const sixdgs_bin_state* s, char* msg, int32_t msg_cap) {
  auto put = [&](const std::string& m) {
    if (msg && msg_cap > 0) std::snprintf(msg, (size_t)msg_cap, "%s", m.c_str());
  };
  if (!s || s->E < 0 || s->P < 0 || s->T < 0 || s->n_items < 0) {
    put("bad state");
    return SIXDGS_ERR_INVALID_ARG;
  }
  if ((s->E > 0 && (!s->tiles || !s->depth)) || (s->P > 0 && (!s->keys || !s->values)) || (s->T > 0 && !s->ranges) ||
      (s->n_items > 0 && !s->items)) {
    put("NULL array");
    return SIXDGS_ERR_INVALID_ARG;
  }
  const std::string why = check(*s);
  put(why);
  return why.empty() ? SIXDGS_OK : SIXDGS_ERR_DEBUG;
}
