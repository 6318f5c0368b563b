// k_part.hip - partitioned build of Bloom filters too large for LDS: the
// count (with the size step), scan, scatter and fill kernels of one table's
// build (their bodies and the scheme are in part_impl.hpp). No step needs a
// global atomic: device-scope atomics bypass the per-XCD L2 on this chip,
// while every tile here is written by one workgroup.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "part_impl.hpp"

namespace pt {

namespace {

// Smallest tile of a single build: 8 KB.
constexpr uint32_t kMinTileWords = 2048;
// A single build whose filters would take tiles of at most 32 KB at
// kTargetBuckets aims for 256 buckets instead, one fill workgroup per CU
// (the star's 3 MB of backward filters: 256 tiles of 12 KB rather than 372
// of 8 KB, two rounds of fill workgroups); larger ones keep kTargetBuckets
// (a 75 MB filter measured slower with 572 tiles of 128 KB than with 1024
// of 73 KB).
constexpr uint32_t kSmallBuildBuckets = 256;
constexpr uint32_t kSmallBuildTileWords = 8192;

// The bucket target of a single build, from its filters' block counts (as
// sized from the selected count, or as recorded): the same in every kernel
// of the build.
__device__ __forceinline__ uint32_t single_target(const FilterSet &fs, uint32_t lg, uint32_t bits_per_key,
                                                  uint64_t n_sel, bool from_count) {
  uint64_t all = 0;
  for (uint32_t i = 0; i < fs.n; i++) all += part_blocks(fs.f[i], lg, bits_per_key, n_sel, from_count);
  return all <= static_cast<uint64_t>(kSmallBuildBuckets) * (kSmallBuildTileWords >> (lg - 5)) ? kSmallBuildBuckets
                                                                                              : kTargetBuckets;
}

// LDS words of the private copies a partitioned build falls back to when
// its filters turn out small: 64 KB, so that two count workgroups still fit
// on a CU.
constexpr uint32_t kCopyWords = 16384;

// Filters sized for a partitioned build (the capacity of a large table)
// may turn out small once the selected count is known. When the recorded
// sizes fit in copy_words together (0: no room for copies), the build runs
// as private LDS copies instead: the count kernel sets each workgroup's
// rows' bits in its copy, the scan kernel ORs the copies into the filters,
// and the scatter and fill kernels have nothing to do. Returns the words
// of the filters in that case, else 0.
__device__ __forceinline__ uint32_t copies_total(const FilterSet &fs, uint32_t lg, uint32_t copy_words) {
  if (copy_words == 0) return 0;
  uint64_t t = 0;
  for (uint32_t i = 0; i < fs.n; i++)
    t += static_cast<uint64_t>(clamp_blocks(*fs.f[i].nb, fs.f[i].cap_words >> (lg - 5), nullptr)) << (lg - 5);
  return t <= copy_words ? static_cast<uint32_t>(t) : 0;
}

// The count kernel also does the size step: workgroup 0 records the
// pruned marker or each filter's block count (from the selected count) and
// the overflow status. Small filters are built as LDS copies (see
// copies_total). When the plan does not fit, the filters are cleared here
// instead of counted: the scatter then inserts in place with global
// atomics.
template <int B, int K>
__global__ void __launch_bounds__(kWideThreads)
    k_part_count(FilterSet fs, AppendSet app, uint32_t k, uint32_t lg_rt, uint32_t bits_per_key,
                 const uint64_t *count, uint64_t n_rows, const uint64_t *__restrict__ bitmap, uint32_t seg_words,
                 uint64_t entries_cap, uint32_t *__restrict__ hist, uint32_t *__restrict__ copies,
                 uint32_t copy_words, uint32_t *status) {
  extern __shared__ __align__(16) uint32_t s_copy[];
  const uint32_t lg = block_log2<B>(lg_rt);
  uint64_t n_sel;
  if (!size_step(fs, lg, bits_per_key, count, n_rows, blockIdx.x == 0 && threadIdx.x == 0, status, n_sel)) return;
  if (copy_words) {
    // the sizes workgroup 0 records, computed here (they are not stored yet)
    uint64_t total = 0;
    for (uint32_t i = 0; i < fs.n; i++) total += static_cast<uint64_t>(sized_blocks(fs.f[i], lg, bits_per_key, n_sel))
                                                 << (lg - 5);
    if (total <= copy_words) {
      for (uint32_t j = threadIdx.x; j < total; j += blockDim.x) s_copy[j] = 0;
      __syncthreads();
      uint32_t off = 0;
      for (uint32_t i = 0; i < fs.n; i++) {
        const FilterRef &f = fs.f[i];
        const uint32_t nb = sized_blocks(f, lg, bits_per_key, n_sel);
        uint32_t *mine = s_copy + off;
        for_each_key<true>(f, app, n_rows, bitmap, seg_words, whole_grid(),
                           [&](uint32_t h1, uint32_t h2) { insert_lds<K>(mine, nb, k, h1, h2, lg); });
        off += nb << (lg - 5);
      }
      __syncthreads();
      uint32_t *out = copies + static_cast<uint64_t>(blockIdx.x) * copy_words;
      for (uint32_t j = threadIdx.x; j < total; j += blockDim.x) out[j] = s_copy[j];
      return;
    }
  }
  const uint32_t target = single_target(fs, lg, bits_per_key, n_sel, true);
  const PartGeo geo = part_geo(fs, lg, bits_per_key, count, n_rows, entries_cap, true, target,
                               kMinTileWords >> (lg - 5));
  if (!geo.ok) {
    for (uint32_t i = 0; i < fs.n; i++) {
      const FilterRef &f = fs.f[i];
      const uint64_t n = static_cast<uint64_t>(sized_blocks(f, lg, bits_per_key, n_sel)) << (lg - 5);
      for (uint64_t j = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; j < n;
           j += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        f.words[j] = 0;
    }
    return;
  }
  part_count_body<true>(fs, app, lg, bits_per_key, count, n_rows, bitmap, seg_words, entries_cap,
                        hist + static_cast<uint64_t>(blockIdx.x) * kMaxBuckets, true, target, whole_grid(),
                        kMinTileWords >> (lg - 5));
}

// Exclusive scan of hist[g][b] over the n_groups workgroups for every
// bucket b, in place; bucket b's total goes to totals[b]. A workgroup takes
// 64 buckets at a time (lane = bucket, so every read covers 64 consecutive
// counters); wave w sums its share of the groups, the waves' sums are
// combined in LDS, and each wave rewrites its share as running offsets.
// When the filters were built as copies, it ORs the n_groups copies into
// them instead, 64 words per workgroup step (wave w ORs every 16th copy,
// the waves' results are combined in LDS).
__global__ void __launch_bounds__(kWideThreads)
    k_part_scan_groups(FilterSet fs, uint32_t lg, uint32_t bits_per_key, const uint64_t *count, uint64_t n_rows,
                       uint64_t entries_cap, uint32_t *__restrict__ hist, uint32_t n_groups,
                       uint64_t *__restrict__ totals, const uint32_t *__restrict__ copies, uint32_t copy_words) {
  constexpr uint32_t kWaves = kWideThreads / kWave;
  __shared__ uint64_t s_part[kWaves][kWave];
  if (build_pruned(fs)) return;
  const uint32_t lane = lane_id();
  const uint32_t wv = threadIdx.x / kWave;
  const uint32_t total = copies_total(fs, lg, copy_words);
  if (total) {
    for (uint32_t base = blockIdx.x * kWave; base < total; base += gridDim.x * kWave) {
      const uint32_t w = base + lane;
      uint32_t v = 0;
      if (w < total) {
#pragma unroll 8
        for (uint32_t g = wv; g < n_groups; g += kWaves) v |= copies[static_cast<uint64_t>(g) * copy_words + w];
      }
      s_part[wv][lane] = v;
      __syncthreads();
      if (wv == 0 && w < total) {
        uint32_t r = 0;
#pragma unroll
        for (uint32_t q = 0; q < kWaves; q++) r |= static_cast<uint32_t>(s_part[q][lane]);
        // word w of the concatenated filters
        uint32_t off = 0;
        for (uint32_t i = 0; i < fs.n; i++) {
          const uint32_t n = clamp_blocks(*fs.f[i].nb, fs.f[i].cap_words >> (lg - 5), nullptr) << (lg - 5);
          if (w >= off && w < off + n) fs.f[i].words[w - off] = r;
          off += n;
        }
      }
      __syncthreads();
    }
    return;
  }
  const uint32_t target = single_target(fs, lg, bits_per_key, 0, false);
  const PartGeo geo = part_geo(fs, lg, bits_per_key, count, n_rows, entries_cap, false, target,
                               kMinTileWords >> (lg - 5));
  if (!geo.ok) return;
  const uint32_t per = (n_groups + kWaves - 1) / kWaves;
  const uint32_t g0 = min(wv * per, n_groups), g1 = min(g0 + per, n_groups);
  // A wave's first kRegGroups counters stay in registers between the sum
  // and the rewrite (one round of loads, issued together: the addresses
  // are clamped into the table, the values of lanes or groups outside it
  // zeroed); groups beyond that (more than 16 x 16 workgroups) are read
  // again.
  constexpr uint32_t kRegGroups = 16;
  for (uint32_t b0 = blockIdx.x * kWave; b0 < geo.buckets; b0 += gridDim.x * kWave) {
    const uint32_t b = b0 + lane;
    const bool in = b < geo.buckets;
    const uint32_t bc = in ? b : geo.buckets - 1;
    uint32_t v[kRegGroups];
    uint64_t sum = 0;
    if (g1 > g0) {
#pragma unroll
      for (uint32_t j = 0; j < kRegGroups; j++) {
        const uint32_t g = g0 + j;
        const uint32_t x = hist[(g < g1 ? g : g1 - 1) * kMaxBuckets + bc];  // < 2^32: groups <= 2^18
        v[j] = in && g < g1 ? x : 0;
      }
#pragma unroll
      for (uint32_t j = 0; j < kRegGroups; j++) sum += v[j];
      for (uint32_t g = g0 + kRegGroups; g < g1; g++) sum += in ? hist[static_cast<uint64_t>(g) * kMaxBuckets + b] : 0;
    }
    s_part[wv][lane] = sum;
    __syncthreads();
    uint64_t run = 0;
    for (uint32_t w = 0; w < wv; w++) run += s_part[w][lane];
    if (wv == kWaves - 1 && in) totals[b] = run + sum;
    if (in) {
#pragma unroll
      for (uint32_t j = 0; j < kRegGroups; j++) {
        const uint32_t g = g0 + j;
        if (g < g1) hist[g * kMaxBuckets + b] = static_cast<uint32_t>(run);
        run += v[j];
      }
      for (uint32_t g = g0 + kRegGroups; g < g1; g++) {
        uint32_t *h = hist + static_cast<uint64_t>(g) * kMaxBuckets + b;
        const uint32_t x = *h;
        *h = static_cast<uint32_t>(run);
        run += x;
      }
    }
    __syncthreads();
  }
}

// Every workgroup first turns the bucket totals into the buckets' first
// entries itself (an exclusive scan, 1024 buckets per round: lane shuffles
// within a wave, the wave sums through LDS) and keeps them as its cursors;
// workgroup 0 also stores them, with starts[buckets] = all, for the fill.
// Redoing the scan in each workgroup costs less than a launch of its own.
template <int B, int K>
__global__ void __launch_bounds__(kWideThreads)
    k_part_scatter(FilterSet fs, AppendSet app, uint32_t k, uint32_t lg_rt, uint32_t bits_per_key,
                   const uint64_t *count, uint64_t n_rows, const uint64_t *__restrict__ bitmap, uint32_t seg_words,
                   uint64_t entries_cap, const uint32_t *__restrict__ hist, const uint64_t *__restrict__ totals,
                   uint64_t *__restrict__ starts, uint32_t *__restrict__ entries, uint32_t *status,
                   uint64_t lds_bytes, uint32_t copy_words) {
  constexpr uint32_t kWaves = kWideThreads / kWave;
  extern __shared__ __align__(16) uint64_t s_cur[];
  __shared__ uint64_t s_wsum[kWaves];
  const uint32_t lg = block_log2<B>(lg_rt);
  if (build_pruned(fs) || copies_total(fs, lg, copy_words)) return;
  const uint32_t target = single_target(fs, lg, bits_per_key, 0, false);
  const PartGeo geo = part_geo(fs, lg, bits_per_key, count, n_rows, entries_cap, false, target,
                               kMinTileWords >> (lg - 5));
  if (geo.ok) {
    const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
    uint64_t carry = 0;
    for (uint32_t base = 0; base < geo.buckets; base += blockDim.x) {
      const uint32_t b = base + threadIdx.x;
      const uint64_t v = b < geo.buckets ? totals[b] : 0;
      uint64_t incl = v;
#pragma unroll
      for (uint32_t d = 1; d < kWave; d <<= 1) {
        const uint64_t t = __shfl_up(static_cast<unsigned long long>(incl), d, kWave);
        if (lane >= d) incl += t;
      }
      if (lane == kWave - 1) s_wsum[wv] = incl;
      __syncthreads();
      uint64_t before = 0, all = 0;
      for (uint32_t w = 0; w < kWaves; w++) {
        const uint64_t ws = s_wsum[w];
        before += w < wv ? ws : 0;
        all += ws;
      }
      if (b < geo.buckets) {
        const uint64_t ex = carry + before + incl - v;
        s_cur[b] = ex;
        if (blockIdx.x == 0) starts[b] = ex;
      }
      carry += all;
      __syncthreads();
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) starts[geo.buckets] = carry;
  }
  part_scatter_body<true, K>(fs, app, k, lg, bits_per_key, count, n_rows, bitmap, seg_words, entries_cap,
                             hist + static_cast<uint64_t>(blockIdx.x) * kMaxBuckets, nullptr, entries, status, false,
                             target, whole_grid(), lds_bytes, kMinTileWords >> (lg - 5));
}

template <int B, int K>
__global__ void __launch_bounds__(kWideThreads)
    k_part_fill(FilterSet fs, uint32_t k, uint32_t lg_rt, uint32_t bits_per_key, const uint64_t *count,
                uint64_t n_rows, uint64_t entries_cap, const uint64_t *__restrict__ starts,
                const uint32_t *__restrict__ entries, uint32_t copy_words) {
  const uint32_t lg = block_log2<B>(lg_rt);
  if (build_pruned(fs) || copies_total(fs, lg, copy_words)) return;
  part_fill_body<K>(fs, k, lg, bits_per_key, count, n_rows, entries_cap, starts, entries, blockIdx.x, gridDim.x,
                    false, single_target(fs, lg, bits_per_key, 0, false), kMinTileWords >> (lg - 5));
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
  // partial tile per filter, or the 128 KB tiles of the largest filters.
  uint64_t max_buckets = kTargetBuckets + fs.n;
  {
    uint64_t big = 0;
    for (uint32_t i = 0; i < fs.n; i++) big += (fs.f[i].cap_words / W + kTileWords / W - 1) / (kTileWords / W);
    if (big > max_buckets) max_buckets = big;
  }
  if (max_buckets > kMaxBuckets) max_buckets = kMaxBuckets;
  const uint32_t scan_grid = static_cast<uint32_t>((max_buckets + kWave - 1) / kWave);
  uint64_t fill_grid = static_cast<uint64_t>(device_info().n_cu) * 2;
  if (fill_grid > max_buckets) fill_grid = max_buckets;
  const bool spec = block_bits == 512 && k == 3;
  auto count_k = spec ? k_part_count<512, 3> : k_part_count<0, 0>;
  // Room for the small-filter copies: kCopyWords per count workgroup
  // (PT_BUILD_PATH=part, for testing: always partition).
  const char *force = std::getenv("PT_BUILD_PATH");
  const bool force_part = force && std::strcmp(force, "part") == 0;
  const uint32_t copy_words =
      !force_part && scratch.copies && scratch.copies_words >= static_cast<uint64_t>(n_groups) * kCopyWords
          ? kCopyWords
          : 0;
  auto scatter_k = spec ? k_part_scatter<512, 3> : k_part_scatter<0, 0>;
  auto fill_k = spec ? k_part_fill<512, 3> : k_part_fill<0, 0>;
  const uint64_t hist_bytes = max_buckets * 4;
  // the scatter stages entries per bucket in LDS when every bucket's stage fits
  const uint64_t lds_avail = static_cast<uint64_t>(device_info().max_lds_block) - 2048;
  const uint64_t staged_bytes = max_buckets * kStagedBucketBytes;
  const uint64_t cursor_bytes = staged_bytes <= lds_avail ? staged_bytes : max_buckets * 8;
  const uint64_t tile_bytes = static_cast<uint64_t>(kTileWords) * 4;
  const uint64_t count_bytes = std::max<uint64_t>(hist_bytes, static_cast<uint64_t>(copy_words) * 4);
  // the scan kernel ORs up to copy_words words of copies, 64 per workgroup
  const uint32_t scan_blocks = std::max<uint32_t>(scan_grid, copy_words / kWave);
  hipError_t e = allow_lds(reinterpret_cast<const void *>(count_k), count_bytes);
  if (e == hipSuccess) e = allow_lds(reinterpret_cast<const void *>(scatter_k), cursor_bytes);
  if (e == hipSuccess) e = allow_lds(reinterpret_cast<const void *>(fill_k), tile_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(count_k, dim3(n_groups), dim3(kWideThreads), count_bytes, s, fs, a, k, lg, bits_per_key, count,
                     n_rows, bitmap, seg_words, entries_cap, scratch.hist, scratch.copies, copy_words, status);
  hipLaunchKernelGGL(k_part_scan_groups, dim3(scan_blocks ? scan_blocks : 1), dim3(kWideThreads), 0, s, fs, lg,
                     bits_per_key, count, n_rows, entries_cap, scratch.hist, n_groups, scratch.totals, scratch.copies,
                     copy_words);
  hipLaunchKernelGGL(scatter_k, dim3(n_groups), dim3(kWideThreads), cursor_bytes, s, fs, a, k, lg, bits_per_key,
                     count, n_rows, bitmap, seg_words, entries_cap, scratch.hist, scratch.totals, scratch.starts,
                     scratch.entries, status, cursor_bytes, copy_words);
  hipLaunchKernelGGL(fill_k, dim3(static_cast<uint32_t>(fill_grid ? fill_grid : 1)), dim3(kWideThreads), tile_bytes,
                     s, fs, k, lg, bits_per_key, count, n_rows, entries_cap, scratch.starts, scratch.entries,
                     copy_words);
  return hipGetLastError();
}

}  // namespace pt
