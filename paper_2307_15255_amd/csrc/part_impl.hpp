// part_impl.hpp - bodies of the partitioned build of Bloom filters too
// large for LDS (Sec. 2.1 and Sec. 3.2 of the paper: the outgoing filters of
// a table receive the keys of its selected rows), over a (virtual) grid:
// shared by the partitioned-build kernels and the batch kernel.
//
// Each filter's blocks are cut into tiles of at most 128 KB, and every
// (filter, tile) pair is a bucket (buckets of filter i follow those of
// filters < i).
//   count    each workgroup walks its rows and histograms their bucket
//            in LDS, then stores its histogram row;
//   scan     per bucket, an exclusive scan over the workgroups' counts, then
//            one scan over the bucket totals (in the single-build kernels
//            every scatter workgroup does this one itself): every
//            (workgroup, bucket) gets its own range of the entry buffer;
//   scatter  the same walk again (same grid, so the same rows per
//            workgroup) writes each entry - block within the tile and H2 -
//            at its range's next slot (LDS cursors); when the plan does not
//            fit, this kernel inserts in place with global atomics instead;
//   fill     one workgroup per bucket sets the bits of its entries in an LDS
//            tile and stores the whole tile (every block of the filter is
//            written exactly once).
#pragma once

#include "build_impl.hpp"

namespace pt {

// An entry is 32 bits: the block within its tile above the top 2 log2(B)
// bits of H2, the only bits of H2 the bit positions use. Tiles hold at most
// 128 KB, so the block index fits (15 bits for B = 32, 10 for B = 1024).
__device__ __forceinline__ uint32_t pack_entry(uint32_t blk_in_tile, uint32_t h2, uint32_t lg) {
  return (blk_in_tile << (2 * lg)) | (h2 >> (32 - 2 * lg));
}
__device__ __forceinline__ uint32_t entry_block(uint32_t v, uint32_t lg) { return v >> (2 * lg); }
__device__ __forceinline__ uint32_t entry_h2(uint32_t v, uint32_t lg) { return v << (32 - 2 * lg); }

// Adds n to counter[b] for every active lane: the lanes whose b equals the
// first active lane's add together with one atomic (keys with few distinct
// values, a skewed foreign key, would otherwise serialise on one counter),
// the others one by one. Returns each lane's previous count plus its rank
// among the lanes that added to the same counter together.
template <typename T>
__device__ __forceinline__ T wave_counter_add(T *counter, uint32_t b) {
  const uint32_t b0 = __builtin_amdgcn_readfirstlane(b);
  const uint64_t same = __ballot(b == b0);
  if (b != b0) return atomicAdd(&counter[b], T(1));
  const uint32_t rank = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(same >> 32),
                                                  __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(same), 0));
  T base = 0;
  if (rank == 0) base = atomicAdd(&counter[b0], static_cast<T>(__popcll(same)));
  // the first active lane of this branch is the rank-0 lane
  if constexpr (sizeof(T) == 8)
    base = (static_cast<T>(__builtin_amdgcn_readfirstlane(static_cast<uint32_t>(base >> 32))) << 32) |
           static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<uint32_t>(base)));
  else
    base = static_cast<T>(__builtin_amdgcn_readfirstlane(static_cast<uint32_t>(base)));
  return base + rank;
}

// Histogram of this workgroup's keys over the buckets, stored to hist_row.
template <bool APP>
__device__ __forceinline__ void part_count_body(const FilterSet &fs, const AppendSet &app, uint32_t lg,
                                                uint32_t bits_per_key, const uint64_t *count, uint64_t n_rows,
                                                const uint64_t *bitmap, uint32_t seg_words, uint64_t entries_cap,
                                                uint32_t *hist_row, bool from_count, uint32_t target,
                                                const VGrid &vg, uint32_t min_tile = 1) {
  extern __shared__ __align__(16) uint32_t s_hist[];
  const PartGeo geo = part_geo(fs, lg, bits_per_key, count, n_rows, entries_cap, from_count, target, min_tile);
  if (!geo.ok) return;
  for (uint32_t b = threadIdx.x; b < geo.buckets; b += blockDim.x) s_hist[b] = 0;
  __syncthreads();
  const uint32_t tb = geo.tile_blocks;
  uint32_t base = 0;
  for (uint32_t i = 0; i < fs.n; i++) {
    const FilterRef &f = fs.f[i];
    const uint32_t nb = part_blocks(f, lg, bits_per_key, geo.n_sel, from_count);
    uint32_t *mine = s_hist + base;
    for_each_key<APP>(f, app, n_rows, bitmap, seg_words, vg,
                      [&](uint32_t h1, uint32_t) { wave_counter_add(mine, block_of(h1, nb) / tb); });
    base += (nb + tb - 1) / tb;
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < geo.buckets; b += blockDim.x) hist_row[b] = s_hist[b];
}

// Entries a bucket gathers in LDS before they are stored as one run.
constexpr uint32_t kStageEntries = 32;
// LDS bytes per bucket of a staged scatter: cursor, claim and write counts,
// the staged entries.
constexpr uint32_t kStagedBucketBytes = 8 + 4 + 4 + 4 * kStageEntries;
// Fewer buckets than this are not staged: each wave's stores to one bucket
// already form runs, and the workgroup's claims would crowd a few counters.
constexpr uint32_t kStageMinBuckets = 64;

// Writes this workgroup's entries at its ranges (hist_row: its exclusive
// offsets within each bucket, starts: the buckets' first entries, or NULL
// when the caller left them in the cursor array s_cur). When the
// plan does not fit the entry buffer, inserts in place with global atomics
// instead (the filters were zeroed in that case).
//
// With many buckets and room in lds_bytes for every bucket's stage, entries
// are not stored one by one (thousands of buckets take one 4-byte store
// each, and the partial cache lines cost several times the bytes in
// write-backs): a lane claims a slot of its bucket's stage in LDS and
// writes the entry there; the lane whose write fills the stage marks it,
// and right after that key its wave stores the stage as one coalesced run
// at the bucket's cursor and empties it. A claim beyond a full stage that
// is not emptied yet stores its entry directly. What is left in the stages
// is stored at the end. Every entry is stored exactly once, at the
// workgroup's range of its bucket.
template <bool APP, int K>
__device__ __forceinline__ void part_scatter_body(const FilterSet &fs, const AppendSet &app, uint32_t k, uint32_t lg,
                                                  uint32_t bits_per_key, const uint64_t *count, uint64_t n_rows,
                                                  const uint64_t *bitmap, uint32_t seg_words, uint64_t entries_cap,
                                                  const uint32_t *hist_row, const uint64_t *starts,
                                                  uint32_t *entries, uint32_t *status, bool from_count,
                                                  uint32_t target, const VGrid &vg, uint64_t lds_bytes = 0,
                                                  uint32_t min_tile = 1) {
  extern __shared__ __align__(16) uint64_t s_cur[];
  const PartGeo geo = part_geo(fs, lg, bits_per_key, count, n_rows, entries_cap, from_count, target, min_tile);
  if (!geo.ok) {
    for (uint32_t i = 0; i < fs.n; i++) {
      const FilterRef &f = fs.f[i];
      const uint32_t nb = part_blocks(f, lg, bits_per_key, geo.n_sel, from_count);
      uint32_t *words = f.words;
      for_each_key<APP>(f, app, n_rows, bitmap, seg_words, vg,
                        [&](uint32_t h1, uint32_t h2) { insert_bits<K>(words, nb, k, h1, h2, lg); });
    }
    return;
  }
  // s_cur[b]: the next entry slot of this workgroup in bucket b
  const uint32_t nbk = geo.buckets;
  const bool staged = nbk >= kStageMinBuckets && static_cast<uint64_t>(nbk) * kStagedBucketBytes <= lds_bytes;
  uint32_t *s_claim = reinterpret_cast<uint32_t *>(s_cur + nbk);  // [nbk]: slots claimed
  uint32_t *s_wrote = s_claim + nbk;                               // [nbk]: slots written
  uint32_t *s_stage = s_wrote + nbk;                               // [nbk][kStageEntries]
  for (uint32_t b = threadIdx.x; b < nbk; b += blockDim.x) {
    s_cur[b] = (starts ? starts[b] : s_cur[b]) + hist_row[b];
    if (staged) s_claim[b] = s_wrote[b] = 0;
  }
  __syncthreads();
  const uint32_t tb = geo.tile_blocks;
  const uint32_t lane = lane_id();
  auto store = [&](uint64_t pos, uint32_t e) {
    if (pos < entries_cap)  // always true while *count is the bitmap's popcount
      entries[pos] = e;
    else
      raise_status(status, PT_STATUS_ENTRIES_OVERFLOW);
  };
  uint32_t base = 0;
  for (uint32_t i = 0; i < fs.n; i++) {
    const FilterRef &f = fs.f[i];
    const uint32_t nb = part_blocks(f, lg, bits_per_key, geo.n_sel, from_count);
    unsigned long long *cur = reinterpret_cast<unsigned long long *>(s_cur);
    if (!staged) {
      for_each_key<APP>(f, app, n_rows, bitmap, seg_words, vg, [&](uint32_t h1, uint32_t h2) {
        const uint32_t blk = block_of(h1, nb);
        store(wave_counter_add(cur + base, blk / tb), pack_entry(blk % tb, h2, lg));
      });
    } else {
      constexpr uint32_t kNone = 0xFFFFFFFFu;
      uint32_t full = kNone;  // this lane filled the stage of bucket `full`
      auto put = [&](uint32_t h1, uint32_t h2) {
        const uint32_t blk = block_of(h1, nb);
        const uint32_t b = base + blk / tb;
        const uint32_t e = pack_entry(blk % tb, h2, lg);
        const uint32_t slot = atomicAdd(&s_claim[b], 1u);
        if (slot >= kStageEntries) {  // the stage is full and not emptied yet
          store(atomicAdd(&cur[b], 1ull), e);
          return;
        }
        s_stage[b * kStageEntries + slot] = e;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        if (atomicAdd(&s_wrote[b], 1u) == kStageEntries - 1) full = b;
      };
      auto flush = [&]() {
        // every lane takes part: kStageEntries lanes store one full stage at a time
        for (uint64_t m = __ballot(full != kNone); m; m &= m - 1) {
          const uint32_t src = __builtin_amdgcn_readlane(full, __builtin_ctzll(m));
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
          uint64_t at = 0;
          if (lane == 0) at = atomicAdd(&cur[src], static_cast<unsigned long long>(kStageEntries));
          at = (static_cast<uint64_t>(__builtin_amdgcn_readlane(static_cast<uint32_t>(at >> 32), 0)) << 32) |
               static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<uint32_t>(at), 0));
          if (lane < kStageEntries) store(at + lane, s_stage[src * kStageEntries + lane]);
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // the stage's reads come first
          // the stage is read: reopen it (the write count first, so that new
          // claims start from a zero count)
          if (lane == 0) {
            atomicExch(&s_wrote[src], 0u);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            atomicExch(&s_claim[src], 0u);
          }
        }
        full = kNone;
      };
      for_each_key<APP>(f, app, n_rows, bitmap, seg_words, vg, put, flush);
    }
    base += (nb + tb - 1) / tb;
  }
  if (!staged) return;
  // what is left in the stages (fewer than 16 entries each)
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < nbk; b += blockDim.x) {
    const uint32_t n = min(s_wrote[b], kStageEntries);
    for (uint32_t j = 0; j < n; j++) store(s_cur[b] + j, s_stage[b * kStageEntries + j]);
  }
}

// Buckets b_first, b_first + b_step, ...: each tile built in LDS from its
// entries and stored once. Entry ranges are clamped to the buffer, so
// nothing is read outside it whatever the starts hold.
template <int K>
__device__ __forceinline__ void part_fill_body(const FilterSet &fs, uint32_t k, uint32_t lg, uint32_t bits_per_key,
                                               const uint64_t *count, uint64_t n_rows, uint64_t entries_cap,
                                               const uint64_t *starts, const uint32_t *entries, uint32_t b_first,
                                               uint32_t b_step, bool from_count, uint32_t target,
                                               uint32_t min_tile = 1) {
  extern __shared__ __align__(16) uint32_t tile[];
  const uint32_t W = 1u << (lg - 5);
  const PartGeo geo = part_geo(fs, lg, bits_per_key, count, n_rows, entries_cap, from_count, target, min_tile);
  if (!geo.ok) return;
  const uint32_t tb = geo.tile_blocks;
  for (uint32_t b = b_first; b < geo.buckets; b += b_step) {
    // the filter the bucket belongs to, and the tile within it
    uint32_t f = 0, base = 0, nb = 0;
    for (uint32_t i = 0; i < fs.n; i++) {
      nb = part_blocks(fs.f[i], lg, bits_per_key, geo.n_sel, from_count);
      const uint32_t tiles = (nb + tb - 1) / tb;
      f = i;
      if (b < base + tiles) break;
      base += tiles;
    }
    const uint32_t t = b - base;
    const uint32_t first = t * tb;
    const uint32_t n_blocks = min(tb, nb - first);
    for (uint32_t j = threadIdx.x; j < n_blocks * W; j += blockDim.x) tile[j] = 0;
    __syncthreads();
    const uint64_t e0 = min(starts[b], entries_cap), e1 = min(starts[b + 1], entries_cap);
    // the entry names its block inside the tile; with nb = 1 and h1 = 0,
    // insert_lds sets the key's k bits in the block it is pointed at
    auto insert = [&](uint32_t v) {
      const uint32_t blk = min(entry_block(v, lg), n_blocks - 1);
      insert_lds<K>(tile + blk * W, 1, k, 0, entry_h2(v, lg), lg);
    };
    // eight entries per thread in flight (a bucket can hold millions); the
    // last round's loads are clamped to the bucket's last entry rather than
    // skipped, so that they too are issued together
    constexpr int kFillBatch = 8;
    for (uint64_t e = e0 + threadIdx.x; e < e1; e += static_cast<uint64_t>(kFillBatch) * blockDim.x) {
      uint32_t v[kFillBatch];
#pragma unroll
      for (int q = 0; q < kFillBatch; q++) {
        const uint64_t i = e + static_cast<uint64_t>(q) * blockDim.x;
        v[q] = entries[i < e1 ? i : e1 - 1];
      }
#pragma unroll
      for (int q = 0; q < kFillBatch; q++)
        if (e + static_cast<uint64_t>(q) * blockDim.x < e1) insert(v[q]);
    }
    __syncthreads();
    uint32_t *out = fs.f[f].words + static_cast<uint64_t>(first) * W;
    for (uint32_t j = threadIdx.x; j < n_blocks * W; j += blockDim.x) out[j] = tile[j];
    __syncthreads();
  }
}

}  // namespace pt
