// k_build.hip - Bloom build (Sec. 2.1 of the paper; Sec. 3.2, the outgoing
// half of the filter transformation): every selected row's key is inserted
// into each outgoing filter by OR, which is order-free, so the filter bits do
// not depend on scheduling.
//
// Filters that fit in LDS together are built without global atomics. A
// small table's are built by one workgroup in one launch: it sizes them
// from the selected count, sets the bits in LDS and stores every word.
// Otherwise each workgroup sets the bits of its rows in private LDS copies
// (LDS atomics), writes the copies to scratch memory, and a second kernel
// ORs the copies word by word into the filters. Larger filters go to the
// partitioned build
// (k_part.hip) when the caller gave its scratch, else they are built in
// place with global atomic OR, skipped when a read already shows the bit set.
#include <cstdlib>
#include <cstring>

#include "build_impl.hpp"

namespace pt {

namespace {

// Tables of at most this many bitmap words (4096 rows) whose filters fit in
// LDS are built by one workgroup: its 16 waves then walk a few words each
// (10 k rows took one workgroup longer than the three launches of the
// copies path).
constexpr uint64_t kOneGroupWords = 64;

// Block count of filter f as recorded by its size step, in [1, capacity].
__device__ __forceinline__ uint32_t filter_blocks(const FilterRef &f, uint32_t lg, uint32_t *status) {
  return clamp_blocks(*f.nb, f.cap_words >> (lg - 5), status);
}

template <int B, int K>
__global__ void __launch_bounds__(kThreads)
    k_build(FilterSet fs, AppendSet app, uint32_t k, uint32_t lg_rt, uint64_t n_rows,
            const uint64_t *__restrict__ bitmap, uint32_t seg_words, uint32_t *status) {
  if (build_pruned(fs)) return;
  const uint32_t lg = block_log2<B>(lg_rt);
  for (uint32_t i = 0; i < fs.n; i++) {
    const FilterRef &f = fs.f[i];
    const uint32_t nb = filter_blocks(f, lg, status);
    uint32_t *words = f.words;
    for_each_key<true>(f, app, n_rows, bitmap, seg_words, whole_grid(),
                       [&](uint32_t h1, uint32_t h2) { insert_bits<K>(words, nb, k, h1, h2, lg); });
  }
}

// Words of LDS all private copies of a filter set take (filter i's copy
// starts where filter i - 1's ends), or 0 when they exceed lds_words.
__device__ __forceinline__ uint32_t lds_total(const FilterSet &fs, uint32_t lg, uint32_t lds_words) {
  uint64_t total = 0;
  for (uint32_t i = 0; i < fs.n; i++) total += static_cast<uint64_t>(filter_blocks(fs.f[i], lg, nullptr)) << (lg - 5);
  return total <= lds_words ? static_cast<uint32_t>(total) : 0;
}

// Private LDS copies: each workgroup sizes the filters (the size step;
// workgroup 0 records the counts), sets the bits of its rows in its copies
// and stores them at partials + blockIdx.x * copy_words. The launch makes
// sure every filter's capacity fits in copy_words together.
template <int B, int K>
__global__ void __launch_bounds__(kWideThreads)
    k_build_lds(FilterSet fs, AppendSet app, uint32_t k, uint32_t lg_rt, uint32_t bits_per_key,
                const uint64_t *count, uint64_t n_rows, const uint64_t *__restrict__ bitmap, uint32_t seg_words,
                uint32_t *__restrict__ partials, uint32_t copy_words, uint32_t *status) {
  extern __shared__ __align__(16) uint32_t lds[];
  const uint32_t lg = block_log2<B>(lg_rt);
  uint64_t n_sel;
  if (!size_step(fs, lg, bits_per_key, count, n_rows, blockIdx.x == 0 && threadIdx.x == 0, status, n_sel)) return;
  uint32_t total = 0;
  for (uint32_t i = 0; i < fs.n; i++) total += sized_blocks(fs.f[i], lg, bits_per_key, n_sel) << (lg - 5);
  for (uint32_t j = threadIdx.x; j < total; j += blockDim.x) lds[j] = 0;
  __syncthreads();
  uint32_t off = 0;
  for (uint32_t i = 0; i < fs.n; i++) {
    const FilterRef &f = fs.f[i];
    const uint32_t nb = sized_blocks(f, lg, bits_per_key, n_sel);
    uint32_t *mine = lds + off;
    for_each_key<true>(f, app, n_rows, bitmap, seg_words, whole_grid(),
                       [&](uint32_t h1, uint32_t h2) { insert_lds<K>(mine, nb, k, h1, h2, lg); });
    off += nb << (lg - 5);
  }
  __syncthreads();
  uint32_t *out = partials + static_cast<uint64_t>(blockIdx.x) * copy_words;
  for (uint32_t j = threadIdx.x; j < total; j += blockDim.x) out[j] = lds[j];
}

// Filter i (blockIdx.y) = OR over the n_parts private copies. A workgroup
// takes 64 consecutive words: its 16 waves each OR every 16th copy (loads
// issued together, coalesced across the 64 lanes), then one wave combines
// the 16 partial results through LDS.
__global__ void __launch_bounds__(kWideThreads)
    k_build_reduce(FilterSet fs, uint32_t lg, const uint32_t *__restrict__ partials, uint32_t n_parts,
                   uint32_t lds_words) {
  constexpr int kGroups = kWideThreads / kWave;
  __shared__ uint32_t s_or[kGroups][kWave];
  if (build_pruned(fs) || lds_total(fs, lg, lds_words) == 0) return;
  const uint32_t i = blockIdx.y;
  uint32_t off = 0;
  for (uint32_t j = 0; j < i; j++) off += filter_blocks(fs.f[j], lg, nullptr) << (lg - 5);
  const FilterRef &f = fs.f[i];
  uint32_t *words = f.words;
  const uint32_t n = filter_blocks(f, lg, nullptr) << (lg - 5);
  const uint32_t lane = lane_id();
  const uint32_t g = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  for (uint32_t base = blockIdx.x * kWave; base < n; base += gridDim.x * kWave) {
    const uint32_t w = base + lane;
    uint32_t v = 0;
    if (w < n) {
#pragma unroll 8
      for (uint32_t p = g; p < n_parts; p += kGroups) v |= partials[static_cast<uint64_t>(p) * lds_words + off + w];
    }
    s_or[g][lane] = v;
    __syncthreads();
    if (g == 0 && w < n) {
      uint32_t r = 0;
#pragma unroll
      for (int q = 0; q < kGroups; q++) r |= s_or[q][lane];
      words[w] = r;
    }
    __syncthreads();
  }
}

}  // namespace

uint64_t build_lds_words() {
  // LDS of one build workgroup: the private filter copies.
  return (static_cast<uint64_t>(device_info().max_lds_block) - 1024) / 4;
}

// The one-launch build of a small table: the size step's work (the pruned
// marker, each filter's block count from the selected count, the overflow
// status), then every filter built in LDS (their capacities fit) and stored
// whole, so nothing has to be cleared first.
template <int B, int K>
__global__ void __launch_bounds__(kWideThreads)
    k_build_one(FilterSet fs, AppendSet app, uint32_t k, uint32_t lg_rt, uint32_t bits_per_key,
                const uint64_t *count, uint64_t n_rows, const uint64_t *__restrict__ bitmap, uint32_t seg_words,
                uint32_t *status) {
  extern __shared__ __align__(16) uint32_t lds[];
  const uint32_t lg = block_log2<B>(lg_rt);
  uint64_t n_sel;
  if (!size_step(fs, lg, bits_per_key, count, n_rows, threadIdx.x == 0, status, n_sel)) return;
  uint32_t total = 0;
  for (uint32_t i = 0; i < fs.n; i++) total += sized_blocks(fs.f[i], lg, bits_per_key, n_sel) << (lg - 5);
  for (uint32_t j = threadIdx.x; j < total; j += blockDim.x) lds[j] = 0;
  __syncthreads();
  uint32_t off = 0;
  for (uint32_t i = 0; i < fs.n; i++) {
    const FilterRef &f = fs.f[i];
    const uint32_t nb = sized_blocks(f, lg, bits_per_key, n_sel);
    uint32_t *mine = lds + off;
    for_each_key<true>(f, app, n_rows, bitmap, seg_words, whole_grid(),
                       [&](uint32_t h1, uint32_t h2) { insert_lds<K>(mine, nb, k, h1, h2, lg); });
    off += nb << (lg - 5);
  }
  __syncthreads();
  off = 0;
  for (uint32_t i = 0; i < fs.n; i++) {
    const FilterRef &f = fs.f[i];
    const uint32_t n = sized_blocks(f, lg, bits_per_key, n_sel) << (lg - 5);
    uint32_t *words = f.words;
    for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) words[j] = lds[off + j];
    off += n;
  }
}

hipError_t launch_build(uint32_t block_bits, uint32_t k, uint32_t bits_per_key, const FilterSet &fs,
                        uint64_t n_rows, const uint64_t *bitmap, const uint64_t *count, const BuildScratch *scratch,
                        const AppendSet *app, uint32_t *status, hipStream_t s) {
  if (fs.n == 0) return hipSuccess;
  const uint32_t lg = log2_of(static_cast<int>(block_bits));
  if (lg == 0) return hipErrorInvalidValue;
  // Appended keys are used only when every filter names one of them.
  AppendSet a{};
  if (app && app->n_cols > 0 && app->n_cols <= static_cast<uint32_t>(kMaxAppend)) {
    bool all = true;
    for (uint32_t i = 0; i < fs.n; i++) all = all && fs.f[i].app >= 1 && fs.f[i].app <= app->n_cols;
    if (all) a = *app;
  }
  const uint64_t n_words = (n_rows + 63) / 64;
  const uint32_t seg_words = segment_words(n_words ? n_words : 1);
  const uint64_t lds_words = build_lds_words();
  uint64_t cap_words = 0;
  for (uint32_t i = 0; i < fs.n; i++) cap_words += fs.f[i].cap_words;
  // Which path: when all filters surely fit in LDS, one workgroup for a
  // small table, else private LDS copies; the partitioned build when the
  // caller gave its buffers; else atomics.
  enum { kOne, kLds, kPart, kAtomic } path = kAtomic;
  if (cap_words <= lds_words && n_words <= kOneGroupWords) path = kOne;
  else if (scratch && scratch->copies && cap_words <= lds_words) path = kLds;
  else if (scratch && scratch->entries && scratch->entries_cap) path = kPart;
  // PT_BUILD_PATH=atomic|lds|part (testing): take that path where it is allowed.
  if (const char *force = std::getenv("PT_BUILD_PATH")) {
    if (std::strcmp(force, "atomic") == 0) path = kAtomic;
    else if (std::strcmp(force, "lds") == 0 && scratch && scratch->copies && cap_words <= lds_words) path = kLds;
    else if (std::strcmp(force, "part") == 0 && scratch && scratch->entries && scratch->entries_cap) path = kPart;
  }

  hipError_t e = hipSuccess;
  if (path == kOne) {
    auto kern = (block_bits == 512 && k == 3) ? k_build_one<512, 3> : k_build_one<0, 0>;
    e = allow_lds(reinterpret_cast<const void *>(kern), cap_words * 4);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(1), dim3(kWideThreads), cap_words * 4, s, fs, a, k, lg, bits_per_key, count,
                       n_rows, bitmap, seg_words, status);
    return hipGetLastError();
  }
  // The partitioned and LDS-copy builds do the size step in their first
  // kernel.
  if (path == kAtomic || n_words == 0) {
    e = launch_size(block_bits, bits_per_key, fs, count, n_rows, path == kPart ? scratch->entries_cap : 0, status,
                    s);
    if (e != hipSuccess || n_words == 0) return e;
  }

  if (path == kPart)
    return launch_part_build(block_bits, k, bits_per_key, fs, n_rows, bitmap, count, *scratch, a, seg_words, status,
                             s);

  if (path == kAtomic) {
    const uint32_t grid = grid_for((n_words + seg_words - 1) / seg_words, kThreads, 8);
    if (block_bits == 512 && k == 3)
      hipLaunchKernelGGL((k_build<512, 3>), dim3(grid), dim3(kThreads), 0, s, fs, a, k, lg, n_rows, bitmap,
                         seg_words, status);
    else
      hipLaunchKernelGGL((k_build<0, 0>), dim3(grid), dim3(kThreads), 0, s, fs, a, k, lg, n_rows, bitmap,
                         seg_words, status);
    return hipGetLastError();
  }

  const uint64_t copy_words = cap_words;
  uint64_t parts = scratch->copies_words / copy_words;
  const uint64_t work_parts = (n_words + seg_words * 16 - 1) / (seg_words * 16);
  if (parts > static_cast<uint64_t>(device_info().n_cu)) parts = device_info().n_cu;
  if (parts > work_parts) parts = work_parts;
  if (parts == 0) parts = 1;
  const uint32_t cw = static_cast<uint32_t>(copy_words);
  const uint32_t n_parts = static_cast<uint32_t>(parts);
  auto kern = (block_bits == 512 && k == 3) ? k_build_lds<512, 3> : k_build_lds<0, 0>;
  e = allow_lds(reinterpret_cast<const void *>(kern), copy_words * 4);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(n_parts), dim3(kWideThreads), copy_words * 4, s, fs, a, k, lg, bits_per_key, count,
                     n_rows, bitmap, seg_words, scratch->copies, cw, status);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  uint64_t gx = (copy_words + kWave - 1) / kWave;
  if (gx > 1024) gx = 1024;
  hipLaunchKernelGGL(k_build_reduce, dim3(static_cast<uint32_t>(gx), fs.n), dim3(kWideThreads), 0, s, fs, lg,
                     scratch->copies, n_parts, cw);
  return hipGetLastError();
}

}  // namespace pt
