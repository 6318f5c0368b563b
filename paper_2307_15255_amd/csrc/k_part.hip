// k_part.hip - partitioned build of Bloom filters too large for LDS.
//
// Each filter's blocks are cut into tiles of at most 64 KB, and every
// (filter, tile) pair is a bucket.
//   count    each workgroup walks its rows and histograms their bucket
//            in LDS, then stores its histogram row;
//   scan     per bucket, an exclusive scan over the workgroups' counts, then
//            one scan over the bucket totals: every (workgroup, bucket) gets
//            its own range of the entry buffer;
//   scatter  the same walk again (same grid, so the same rows per
//            workgroup) writes each entry - block within the tile and H2 -
//            at its range's next slot (LDS cursors); when the plan does not
//            fit, this kernel inserts in place with global atomics instead;
//   fill     one workgroup per bucket sets the bits of its entries in an LDS
//            tile and stores the whole tile (every block of the filter is
//            written exactly once).
// No step needs a global atomic: device-scope atomics bypass the per-XCD L2
// on this chip, while every tile here is written by one workgroup.
#include "build_impl.hpp"

namespace pt {

namespace {

// An entry is 32 bits: the block within its tile above the top 2 log2(B)
// bits of H2, the only bits of H2 the bit positions use. Tiles hold at most
// 64 KB, so the block index fits (14 bits for B = 32, 9 for B = 1024).
__device__ __forceinline__ uint32_t pack_entry(uint32_t blk_in_tile, uint32_t h2, uint32_t lg) {
  return (blk_in_tile << (2 * lg)) | (h2 >> (32 - 2 * lg));
}
__device__ __forceinline__ uint32_t entry_block(uint32_t v, uint32_t lg) { return v >> (2 * lg); }
__device__ __forceinline__ uint32_t entry_h2(uint32_t v, uint32_t lg) { return v << (32 - 2 * lg); }

template <int B>
__global__ void __launch_bounds__(kWideThreads)
    k_part_count(FilterSet fs, AppendSet app, uint32_t lg_rt, uint32_t bits_per_key, const uint64_t *count,
                 uint64_t n_rows, const uint64_t *__restrict__ bitmap, uint32_t seg_words, uint64_t entries_cap,
                 uint32_t *__restrict__ hist) {
  extern __shared__ __align__(16) uint32_t s_hist[];
  const uint32_t lg = block_log2<B>(lg_rt);
  const PartGeo geo = part_geo(fs, lg, bits_per_key, count, n_rows, entries_cap, false);
  if (!geo.ok) return;
  for (uint32_t b = threadIdx.x; b < geo.buckets; b += blockDim.x) s_hist[b] = 0;
  __syncthreads();
  const uint32_t tb = geo.tile_blocks;
  uint32_t base = 0;
  for (uint32_t i = 0; i < fs.n; i++) {
    const FilterRef &f = fs.f[i];
    const uint32_t nb = part_blocks(f, lg, bits_per_key, geo.n_sel, false);
    uint32_t *mine = s_hist + base;
    for_each_key<true>(f, app, n_rows, bitmap, seg_words, whole_grid(),
                       [&](uint32_t h1, uint32_t) { atomicAdd(&mine[block_of(h1, nb) / tb], 1u); });
    base += (nb + tb - 1) / tb;
  }
  __syncthreads();
  uint32_t *row_out = hist + static_cast<uint64_t>(blockIdx.x) * kMaxBuckets;
  for (uint32_t b = threadIdx.x; b < geo.buckets; b += blockDim.x) row_out[b] = s_hist[b];
}

// Bucket b (blockIdx.x): exclusive scan of hist[g][b] over the n_groups
// workgroups, in place; the bucket's total goes to totals[b].
__global__ void __launch_bounds__(kWideThreads)
    k_part_scan_groups(FilterSet fs, uint32_t lg, uint32_t bits_per_key, const uint64_t *count, uint64_t n_rows,
                       uint64_t entries_cap, uint32_t *__restrict__ hist, uint32_t n_groups,
                       uint64_t *__restrict__ totals) {
  __shared__ uint64_t s[kWideThreads];
  const PartGeo geo = part_geo(fs, lg, bits_per_key, count, n_rows, entries_cap, false);
  if (!geo.ok) return;
  for (uint32_t b = blockIdx.x; b < geo.buckets; b += gridDim.x) {
    const uint32_t g = threadIdx.x;
    const uint64_t v = g < n_groups ? hist[static_cast<uint64_t>(g) * kMaxBuckets + b] : 0;
    uint64_t total;
    const uint64_t ex = block_exclusive_scan(v, s, total);
    if (g < n_groups) hist[static_cast<uint64_t>(g) * kMaxBuckets + b] = static_cast<uint32_t>(ex);
    if (g == 0) totals[b] = total;
  }
}

// starts[b] = sum of totals[0..b) for every bucket, starts[buckets] = all.
__global__ void __launch_bounds__(kWideThreads)
    k_part_scan_buckets(FilterSet fs, uint32_t lg, uint32_t bits_per_key, const uint64_t *count, uint64_t n_rows,
                        uint64_t entries_cap, const uint64_t *__restrict__ totals, uint64_t *__restrict__ starts) {
  __shared__ uint64_t s[kWideThreads];
  const PartGeo geo = part_geo(fs, lg, bits_per_key, count, n_rows, entries_cap, false);
  if (!geo.ok) return;
  uint64_t carry = 0;
  for (uint32_t base = 0; base < geo.buckets; base += blockDim.x) {
    const uint32_t b = base + threadIdx.x;
    const uint64_t v = b < geo.buckets ? totals[b] : 0;
    uint64_t total;
    const uint64_t ex = block_exclusive_scan(v, s, total);
    if (b < geo.buckets) starts[b] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) starts[geo.buckets] = carry;
}

template <int B, int K>
__global__ void __launch_bounds__(kWideThreads)
    k_part_scatter(FilterSet fs, AppendSet app, uint32_t k, uint32_t lg_rt, uint32_t bits_per_key,
                   const uint64_t *count, uint64_t n_rows, const uint64_t *__restrict__ bitmap, uint32_t seg_words,
                   uint64_t entries_cap, const uint32_t *__restrict__ hist, const uint64_t *__restrict__ starts,
                   uint32_t *__restrict__ entries, uint32_t *status) {
  extern __shared__ __align__(16) uint64_t s_cur[];
  const uint32_t lg = block_log2<B>(lg_rt);
  const PartGeo geo = part_geo(fs, lg, bits_per_key, count, n_rows, entries_cap, false);
  if (!geo.ok) {
    // The plan does not fit: insert in place with global atomics (the size
    // kernel zeroed the filters in this case).
    for (uint32_t i = 0; i < fs.n; i++) {
      const FilterRef &f = fs.f[i];
      const uint32_t nb = part_blocks(f, lg, bits_per_key, geo.n_sel, false);
      uint32_t *words = f.words;
      for_each_key<true>(f, app, n_rows, bitmap, seg_words, whole_grid(),
                         [&](uint32_t h1, uint32_t h2) { insert_bits<K>(words, nb, k, h1, h2, lg); });
    }
    return;
  }
  const uint32_t *my = hist + static_cast<uint64_t>(blockIdx.x) * kMaxBuckets;
  // s_cur[b]: the next entry slot of this workgroup in bucket b
  for (uint32_t b = threadIdx.x; b < geo.buckets; b += blockDim.x) s_cur[b] = starts[b] + my[b];
  __syncthreads();
  const uint32_t tb = geo.tile_blocks;
  uint32_t base = 0;
  for (uint32_t i = 0; i < fs.n; i++) {
    const FilterRef &f = fs.f[i];
    const uint32_t nb = part_blocks(f, lg, bits_per_key, geo.n_sel, false);
    unsigned long long *cur = reinterpret_cast<unsigned long long *>(s_cur) + base;
    for_each_key<true>(f, app, n_rows, bitmap, seg_words, whole_grid(), [&](uint32_t h1, uint32_t h2) {
      const uint32_t blk = block_of(h1, nb);
      const uint64_t pos = atomicAdd(&cur[blk / tb], 1ull);
      if (pos < entries_cap)  // always true while *count is the bitmap's popcount
        entries[pos] = pack_entry(blk % tb, h2, lg);
      else
        raise_status(status, PT_STATUS_ENTRIES_OVERFLOW);
    });
    base += (nb + tb - 1) / tb;
  }
}

template <int B, int K>
__global__ void __launch_bounds__(kWideThreads)
    k_part_fill(FilterSet fs, uint32_t k, uint32_t lg_rt, uint32_t bits_per_key, const uint64_t *count,
                uint64_t n_rows, uint64_t entries_cap, const uint64_t *__restrict__ starts,
                const uint32_t *__restrict__ entries) {
  extern __shared__ __align__(16) uint32_t tile[];
  const uint32_t lg = block_log2<B>(lg_rt);
  const uint32_t W = 1u << (lg - 5);
  const PartGeo geo = part_geo(fs, lg, bits_per_key, count, n_rows, entries_cap, false);
  if (!geo.ok) return;
  const uint32_t tb = geo.tile_blocks;
  for (uint32_t b = blockIdx.x; b < geo.buckets; b += gridDim.x) {
    // the filter the bucket belongs to, and the tile within it
    uint32_t f = 0, base = 0, nb = 0;
    for (uint32_t i = 0; i < fs.n; i++) {
      nb = part_blocks(fs.f[i], lg, bits_per_key, geo.n_sel, false);
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
    for (uint64_t e = starts[b] + threadIdx.x; e < starts[b + 1]; e += blockDim.x) {
      const uint32_t v = entries[e];
      // the entry names its block inside the tile; with nb = 1 and h1 = 0,
      // insert_lds sets the key's k bits in the block it is pointed at
      insert_lds<K>(tile + entry_block(v, lg) * W, 1, k, 0, entry_h2(v, lg), lg);
    }
    __syncthreads();
    uint32_t *out = fs.f[f].words + static_cast<uint64_t>(first) * W;
    for (uint32_t j = threadIdx.x; j < n_blocks * W; j += blockDim.x) out[j] = tile[j];
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_part_build(uint32_t block_bits, uint32_t k, uint32_t bits_per_key, const FilterSet &fs,
                             uint64_t n_rows, const uint64_t *bitmap, const uint64_t *count,
                             const BuildScratch &scratch, const AppendSet &a, uint32_t seg_words, uint32_t *status,
                             hipStream_t s) {
  const uint32_t lg = log2_of(static_cast<int>(block_bits));
  if (lg == 0) return hipErrorInvalidValue;
  const uint64_t n_words = (n_rows + 63) / 64;
  const uint64_t entries_cap = scratch.entries_cap;
  // The count and scatter kernels use the same grid, so each workgroup walks
  // the same rows in both.
  uint64_t groups = (n_words + seg_words * 16 - 1) / (seg_words * 16);
  if (groups > scratch.hist_groups) groups = scratch.hist_groups;
  if (groups == 0) groups = 1;
  const uint32_t n_groups = static_cast<uint32_t>(groups);
  const uint32_t W = block_bits / 32;
  // Upper bound of the device's bucket count: kTargetBuckets plus one
  // partial tile per filter, or the 64 KB tiles of the largest filters.
  uint64_t max_buckets = kTargetBuckets + fs.n;
  {
    uint64_t big = 0;
    for (uint32_t i = 0; i < fs.n; i++) big += (fs.f[i].cap_words / W + kTileWords / W - 1) / (kTileWords / W);
    if (big > max_buckets) max_buckets = big;
  }
  if (max_buckets > kMaxBuckets) max_buckets = kMaxBuckets;
  const uint32_t scan_grid = static_cast<uint32_t>(max_buckets < 2048 ? max_buckets : 2048);
  uint64_t fill_grid = static_cast<uint64_t>(device_info().n_cu) * 2;
  if (fill_grid > max_buckets) fill_grid = max_buckets;
  const bool spec = block_bits == 512 && k == 3;
  auto count_k = spec ? k_part_count<512> : k_part_count<0>;
  auto scatter_k = spec ? k_part_scatter<512, 3> : k_part_scatter<0, 0>;
  auto fill_k = spec ? k_part_fill<512, 3> : k_part_fill<0, 0>;
  const uint64_t hist_bytes = max_buckets * 4;
  const uint64_t cursor_bytes = max_buckets * 8;
  const uint64_t tile_bytes = static_cast<uint64_t>(kTileWords) * 4;
  hipError_t e = allow_lds(reinterpret_cast<const void *>(count_k), hist_bytes);
  if (e == hipSuccess) e = allow_lds(reinterpret_cast<const void *>(scatter_k), cursor_bytes);
  if (e == hipSuccess) e = allow_lds(reinterpret_cast<const void *>(fill_k), tile_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(count_k, dim3(n_groups), dim3(kWideThreads), hist_bytes, s, fs, a, lg, bits_per_key, count,
                     n_rows, bitmap, seg_words, entries_cap, scratch.hist);
  hipLaunchKernelGGL(k_part_scan_groups, dim3(scan_grid ? scan_grid : 1), dim3(kWideThreads), 0, s, fs, lg,
                     bits_per_key, count, n_rows, entries_cap, scratch.hist, n_groups, scratch.totals);
  hipLaunchKernelGGL(k_part_scan_buckets, dim3(1), dim3(kWideThreads), 0, s, fs, lg, bits_per_key, count, n_rows,
                     entries_cap, scratch.totals, scratch.starts);
  hipLaunchKernelGGL(scatter_k, dim3(n_groups), dim3(kWideThreads), cursor_bytes, s, fs, a, k, lg, bits_per_key,
                     count, n_rows, bitmap, seg_words, entries_cap, scratch.hist, scratch.starts, scratch.entries,
                     status);
  hipLaunchKernelGGL(fill_k, dim3(static_cast<uint32_t>(fill_grid ? fill_grid : 1)), dim3(kWideThreads), tile_bytes,
                     s, fs, k, lg, bits_per_key, count, n_rows, entries_cap, scratch.starts, scratch.entries);
  return hipGetLastError();
}

}  // namespace pt
