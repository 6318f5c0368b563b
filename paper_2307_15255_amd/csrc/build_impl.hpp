// build_impl.hpp - how a build reaches the keys it inserts (Sec. 3.2 of the
// paper: the outgoing half of the filter transformation inserts the key of
// every row that survived the table's probes). Shared by the build and
// partitioned-build translation units.
//
// A wave takes a segment of bitmap words; a sparse segment is walked lane
// by lane (each lane pops the set bits of its own word), a dense one word
// by word (lanes = rows, coalesced key loads), whichever needs fewer steps.
// When the table's probe appended its survivors' keys, the build reads
// those instead (contiguous), except for regions the probe marked as
// overflowed, whose bitmap words are walked.
#pragma once

#include "pt_common.hpp"

namespace pt {

constexpr int kWalkBatch = 8;

// Calls f(rows, ok) for the selected rows of segments seg_first,
// seg_first + seg_step, ... (seg_words words each), U rows per lane at a
// time: rows[u] is valid where bit u of ok is set. A batch of U rows lets
// the caller issue U key loads before it waits.
template <int U, typename F>
__device__ __forceinline__ void walk_rows(uint64_t seg_first, uint64_t seg_step, uint32_t seg_words,
                                          uint64_t n_rows, const uint64_t *bitmap, F &&f) {
  const uint32_t lane = lane_id();
  const uint64_t n_words = (n_rows + 63) / 64;
  // lane l holds word l of a segment of seg_words (1..64) words
  for (uint64_t seg = seg_first; seg * seg_words < n_words; seg += seg_step) {
    const uint64_t w = seg * seg_words + lane;
    uint64_t word = lane < seg_words ? tail_mask(w, n_words, n_rows) : 0;
    if (bitmap && lane < seg_words && w < n_words) word &= bitmap[w];
    const uint64_t nonzero = __ballot(word != 0);
    if (nonzero == 0) continue;
    // Sparse steps load 64 scattered rows at once; dense steps load 64
    // consecutive rows (one coalesced access). Walk sparsely only when that
    // needs clearly fewer steps.
    const uint32_t steps_sparse = wave_max(__popcll(word));
    const uint32_t steps_dense = __popcll(nonzero);
    if (4 * steps_sparse < steps_dense) {
      while (__ballot(word != 0)) {
        uint64_t rows[U];
        uint32_t ok = 0;
#pragma unroll
        for (int u = 0; u < U; u++) {
          rows[u] = 0;
          if (word) {
            rows[u] = w * 64 + (__ffsll(static_cast<unsigned long long>(word)) - 1);
            word &= word - 1;
            ok |= 1u << u;
          }
        }
        f(rows, ok);
      }
    } else {
      uint64_t todo = nonzero;
      while (todo) {
        uint64_t rows[U];
        uint32_t ok = 0;
#pragma unroll
        for (int u = 0; u < U; u++) {
          rows[u] = 0;
          if (todo) {
            const uint32_t j = __ffsll(static_cast<unsigned long long>(todo)) - 1;
            todo &= todo - 1;
            const uint64_t wj = __shfl(word, j);
            rows[u] = (seg * seg_words + j) * 64 + lane;
            if ((wj >> lane) & 1) ok |= 1u << u;
          }
        }
        f(rows, ok);
      }
    }
  }
}

// Filter hashes of the keys of up to U rows (those set in ok) of a key
// column; the loads are issued together.
template <int U>
__device__ __forceinline__ void hash_rows(const void *keys, uint32_t key64, const uint64_t (&row)[U], uint32_t ok,
                                          uint32_t (&h1)[U], uint32_t (&h2)[U]) {
  if (key64) {
    uint64_t x[U];
#pragma unroll
    for (int u = 0; u < U; u++) x[u] = (ok >> u) & 1 ? static_cast<const uint64_t *>(keys)[row[u]] : 0;
#pragma unroll
    for (int u = 0; u < U; u++) hash_key(x[u], h1[u], h2[u]);
  } else {
    uint32_t x[U];
#pragma unroll
    for (int u = 0; u < U; u++) x[u] = (ok >> u) & 1 ? static_cast<const uint32_t *>(keys)[row[u]] : 0;
#pragma unroll
    for (int u = 0; u < U; u++) hash_key32(x[u], h1[u], h2[u]);
  }
}

struct NoHook {
  __device__ void operator()() const {}
};

// Calls g(h1, h2) for the key of every selected row in the key column of
// filter f. Without appended keys (APP false, or f.app == 0) the grid's
// waves walk the bitmap; with them each wave takes whole regions, reading
// their appended keys (contiguous) or, for a region that overflowed,
// walking the bitmap words of the probe groups it covers. after() runs with
// every lane of the wave after each key a lane may have passed to g.
template <bool APP, typename G, typename H = NoHook>
__device__ __forceinline__ void for_each_key(const FilterRef &f, const AppendSet &app, uint64_t n_rows,
                                             const uint64_t *bitmap, uint32_t seg_words, const VGrid &vg, G &&g,
                                             H &&after = H{}) {
  constexpr int U = kWalkBatch;
  const void *keys = f.keys;
  const uint32_t key64 = f.key64;
  auto from_rows = [&](const uint64_t (&row)[U], uint32_t ok) {
    uint32_t h1[U], h2[U];
    hash_rows<U>(keys, key64, row, ok, h1, h2);
#pragma unroll
    for (int u = 0; u < U; u++) {
      if ((ok >> u) & 1) g(h1[u], h2[u]);
      after();
    }
  };
  if (!APP || app.n_cols == 0 || f.app == 0) {
    walk_rows<U>(global_wave(vg), wave_count(vg), seg_words, n_rows, bitmap, from_rows);
    return;
  }
  const uint32_t c = f.app - 1;
  const void *col = app.dst[c];
  const uint32_t col64 = app.key64[c];
  const uint32_t lane = lane_id();
  for (uint64_t r = global_wave(vg); r < app.n_regions; r += wave_count(vg)) {
    const uint32_t n = __builtin_amdgcn_readfirstlane(app.counts[r]);
    if (n > app.region_cap) {
      walk_rows<U>(r, app.n_regions, app.group_words, n_rows, bitmap, from_rows);
      continue;
    }
    const uint64_t base = r * app.region_cap;
    for (uint32_t j0 = 0; j0 < n; j0 += U * kWave) {
      uint64_t idx[U];
      uint32_t ok = 0;
#pragma unroll
      for (int u = 0; u < U; u++) {
        const uint32_t j = j0 + u * kWave + lane;
        idx[u] = base + j;
        if (j < n) ok |= 1u << u;
      }
      uint32_t h1[U], h2[U];
      hash_rows<U>(col, col64, idx, ok, h1, h2);
#pragma unroll
      for (int u = 0; u < U; u++) {
        if ((ok >> u) & 1) g(h1[u], h2[u]);
        after();
      }
    }
  }
}

}  // namespace pt

namespace pt {

// ------------------------------------------------------- the size step
//
// A build kernel sizes its filters itself from the builder's selected count
// (n_rows when count is NULL): nb = max(1, ceil(n_sel * bpk / B)), at most
// the capacity. Returns false when the set is pruned (a non-empty builder
// that kept every row). `lead`, one thread of the grid, records each
// filter's block count (0 for a pruned set) and raises an overflow.
__device__ __forceinline__ bool size_step(const FilterSet &fs, uint32_t lg, uint32_t bits_per_key,
                                          const uint64_t *count, uint64_t n_rows, bool lead, uint32_t *status,
                                          uint64_t &n_sel) {
  n_sel = count ? *count : n_rows;
  const bool pruned = fs.prune && count && n_rows > 0 && n_sel == n_rows;
  if (lead)
    for (uint32_t i = 0; i < fs.n; i++)
      *fs.f[i].nb = pruned ? 0 : blocks_needed(n_sel, 1u << lg, bits_per_key, fs.f[i].cap_words >> (lg - 5), status);
  return !pruned;
}

// Filter f's block count for n_sel selected keys (as the size step records it).
__device__ __forceinline__ uint32_t sized_blocks(const FilterRef &f, uint32_t lg, uint32_t bits_per_key,
                                                 uint64_t n_sel) {
  return static_cast<uint32_t>(blocks_needed(n_sel, 1u << lg, bits_per_key, f.cap_words >> (lg - 5), nullptr));
}

// ---------------------------------------------------- partitioned builds
//
// Filters too large for LDS are built tile by tile: each filter's blocks are
// cut into tiles of tile_blocks blocks (at most 128 KB) and every (filter,
// tile) pair is a bucket; filter i's buckets follow those of filters < i.
// The plan fits when the buckets fit the bucket table and every key of
// every filter fits the entry buffer (entries_cap entries).
struct PartGeo {
  uint32_t tile_blocks;
  uint32_t buckets;
  uint64_t n_sel;
  bool ok;
};

// Blocks of filter f in a partitioned build: from the selected count when
// the filter is being sized, else as recorded in f.nb.
__device__ __forceinline__ uint32_t part_blocks(const FilterRef &f, uint32_t lg, uint32_t bits_per_key,
                                                uint64_t n_sel, bool from_count) {
  const uint64_t cap_blocks = f.cap_words >> (lg - 5);
  if (from_count) return static_cast<uint32_t>(blocks_needed(n_sel, 1u << lg, bits_per_key, cap_blocks, nullptr));
  return clamp_blocks(*f.nb, cap_blocks, nullptr);
}

// target_buckets: how many (filter, tile) buckets the build aims for - many
// for one large build that must fill the device by itself, few for the
// builds of a batch, which fill it together (fewer, larger tiles).
// min_tile_blocks: the smallest tile (fewer, larger buckets for a small
// build: less to scan, more entries per fill workgroup).
__device__ __forceinline__ PartGeo part_geo(const FilterSet &fs, uint32_t lg, uint32_t bits_per_key,
                                            const uint64_t *count, uint64_t n_rows, uint64_t entries_cap,
                                            bool from_count, uint32_t target_buckets = kTargetBuckets,
                                            uint32_t min_tile_blocks = 1) {
  PartGeo g{};
  g.n_sel = count ? *count : n_rows;
  uint64_t all_blocks = 0;
  for (uint32_t i = 0; i < fs.n; i++) all_blocks += part_blocks(fs.f[i], lg, bits_per_key, g.n_sel, from_count);
  // Tiles of at most 128 KB, small enough that the group has about
  // target_buckets of them (the fill step runs one workgroup per tile).
  uint64_t tb = (all_blocks + target_buckets - 1) / target_buckets;
  if (tb < min_tile_blocks) tb = min_tile_blocks;
  const uint64_t max_tb = kTileWords >> (lg - 5);
  g.tile_blocks = static_cast<uint32_t>(tb < 1 ? 1 : (tb > max_tb ? max_tb : tb));
  uint64_t buckets = 0;
  for (uint32_t i = 0; i < fs.n; i++)
    buckets += (part_blocks(fs.f[i], lg, bits_per_key, g.n_sel, from_count) + g.tile_blocks - 1) / g.tile_blocks;
  g.buckets = static_cast<uint32_t>(buckets < kMaxBuckets ? buckets : kMaxBuckets);
  g.ok = entries_cap > 0 && buckets <= kMaxBuckets && g.n_sel * fs.n <= entries_cap;
  return g;
}

}  // namespace pt
