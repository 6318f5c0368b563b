// k_misc.hip - the small steps of the transfer phase: local filters (Sec.
// 3.2: inherent filters applied during the scan; Sec. 3.4: predicates on
// base tables), filter sizing, ordered compaction (the reduced row sets
// handed to the join phase, Sec. 3.3), counters, and the launch helpers the
// other kernel units share.
#include <algorithm>
#include <map>
#include <mutex>

#include "build_impl.hpp"
#include "local_impl.hpp"

namespace pt {

namespace {

__global__ void __launch_bounds__(kThreads) k_zero_u64(uint64_t *p, uint64_t n) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    p[i] = 0;
}

// All rows selected: the bitmap of a table without predicates.
__global__ void __launch_bounds__(kThreads) k_fill_all(uint64_t *bitmap, uint64_t n_rows, uint64_t *count) {
  const uint64_t n_words = (n_rows + 63) / 64;
  for (uint64_t w = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; w < n_words;
       w += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    bitmap[w] = tail_mask(w, n_words, n_rows);
  if (count && blockIdx.x == 0 && threadIdx.x == 0) *count = n_rows;
}

__global__ void __launch_bounds__(kWideThreads)
    k_local(PredSet ps, uint64_t n_rows, uint64_t *__restrict__ bitmap, unsigned long long *count,
            uint32_t seg_words) {
  local_body(ps, n_rows, bitmap, count, seg_words, whole_grid());
}

// --------------------------------------------------------- size and zero
//
// Filter i (blockIdx.y) gets nb = max(1, ceil(count * bits_per_key / B))
// blocks, read from the device counter so the launch sequence never waits
// for the host. Its first nb blocks are zeroed unless the partitioned build
// (which writes every block) will run. A pruned build set gets nb = 0.

__global__ void __launch_bounds__(kThreads)
    k_size_zero(FilterSet fs, uint32_t lg, uint32_t bits_per_key, const uint64_t *count, uint64_t n_rows,
                uint64_t entries_cap, uint32_t *status) {
  const FilterRef &f = fs.f[blockIdx.y];
  const uint64_t W = 1u << (lg - 5);
  if (fs.prune && count && n_rows > 0 && *count == n_rows) {  // pruned: no filter
    if (blockIdx.x == 0 && threadIdx.x == 0) *f.nb = 0;
    return;
  }
  const uint64_t nb = blocks_needed(count ? *count : n_rows, 1u << lg, bits_per_key, f.cap_words / W,
                                    blockIdx.x == 0 && threadIdx.x == 0 ? status : nullptr);
  if (blockIdx.x == 0 && threadIdx.x == 0) *f.nb = nb;
  if (entries_cap && part_geo(fs, lg, bits_per_key, count, n_rows, entries_cap, true).ok) return;
  const uint64_t n = nb * W;
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    f.words[i] = 0;
}

// ------------------------------------------------------------- counters

struct SlotTable {
  uint32_t slot[64];
};

__global__ void k_copy_counts(const uint64_t *src, SlotTable t, uint32_t n, uint64_t *dst) {
  const uint32_t i = threadIdx.x;
  if (i < n) dst[i] = src[t.slot[i]];
}

// -------------------------------------------------------------- compact
//
// Ordered compaction in three steps: per-workgroup popcounts of 1024 bitmap
// words, one exclusive scan over the workgroup totals, then each workgroup
// rescans its words and writes the set rows' ids in ascending order.

constexpr uint64_t kCompactWordsPerBlock = 1024;  // 4 words per thread

__global__ void __launch_bounds__(kThreads)
    k_compact_count(const uint64_t *__restrict__ bitmap, uint64_t n_words, uint64_t n_rows, uint64_t *partials) {
  __shared__ unsigned long long s_cnt;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  const uint64_t base = blockIdx.x * kCompactWordsPerBlock + threadIdx.x * 4;
  uint64_t c = 0;
#pragma unroll
  for (int j = 0; j < 4; j++)
    if (base + j < n_words) c += __popcll(bitmap[base + j] & tail_mask(base + j, n_words, n_rows));
  atomicAdd(&s_cnt, static_cast<unsigned long long>(c));
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = s_cnt;
}

__global__ void __launch_bounds__(1024) k_compact_scan(uint64_t *partials, uint64_t n_parts, uint64_t *count) {
  __shared__ uint64_t s[1024];
  uint64_t carry = 0;
  for (uint64_t base = 0; base < n_parts; base += blockDim.x) {
    const uint64_t i = base + threadIdx.x;
    const uint64_t v = i < n_parts ? partials[i] : 0;
    uint64_t total;
    const uint64_t ex = block_exclusive_scan(v, s, total);
    if (i < n_parts) partials[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) *count = carry;
}

__global__ void __launch_bounds__(kThreads)
    k_compact_write(const uint64_t *__restrict__ bitmap, uint64_t n_words, uint64_t n_rows,
                    const uint64_t *partials, uint32_t *__restrict__ idx) {
  __shared__ uint64_t s[kThreads];
  const uint64_t base = blockIdx.x * kCompactWordsPerBlock + threadIdx.x * 4;
  uint64_t words[4];
  uint64_t c = 0;
#pragma unroll
  for (int j = 0; j < 4; j++) {
    words[j] = base + j < n_words ? bitmap[base + j] & tail_mask(base + j, n_words, n_rows) : 0;
    c += __popcll(words[j]);
  }
  uint64_t total;
  uint64_t pos = partials[blockIdx.x] + block_exclusive_scan(c, s, total);
#pragma unroll
  for (int j = 0; j < 4; j++) {
    uint64_t m = words[j];
    while (m) {
      const uint32_t b = __ffsll(static_cast<unsigned long long>(m)) - 1;
      idx[pos++] = static_cast<uint32_t>((base + j) * 64 + b);
      m &= m - 1;
    }
  }
}

// The allocation-free compaction keeps its partial counts here: one array
// per GPU, alive until the process ends. In host code `scratch` only names
// the symbol; its device address comes from hipGetSymbolAddress.
static_assert(kStaticCompactRows % (64 * kCompactWordsPerBlock) == 0, "whole partials");
constexpr uint64_t kStaticCompactPartials = kStaticCompactRows / 64 / kCompactWordsPerBlock;
static __device__ __align__(256) uint64_t scratch[kStaticCompactPartials];

}  // namespace

hipError_t static_compact_scratch(uint64_t **out) {
  static std::mutex mu;
  static uint64_t *addr[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[dev]) {
    // once per device, with that device current: its own copy of the array
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = static_cast<uint64_t *>(p);
  }
  *out = addr[dev];
  return hipSuccess;
}

// ------------------------------------------------------------- helpers

hipError_t allow_lds(const void *kern, uint64_t bytes) {
  static std::mutex mu;
  static std::map<std::pair<int, const void *>, uint64_t> granted;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  std::lock_guard<std::mutex> lock(mu);
  uint64_t &g = granted[{dev, kern}];
  if (bytes <= g) return hipSuccess;
  // as much as the kernel's static LDS leaves (set once per kernel)
  hipFuncAttributes attr{};
  uint64_t static_bytes = 1024;
  if (hipFuncGetAttributes(&attr, kern) == hipSuccess) static_bytes = std::max<uint64_t>(attr.sharedSizeBytes, 256);
  const uint64_t want = static_cast<uint64_t>(device_info().max_lds_block) - ((static_bytes + 255) & ~uint64_t(255));
  hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     static_cast<int>(bytes > want ? bytes : want));
  if (e == hipSuccess) g = bytes > want ? bytes : want;
  return e;
}

uint32_t segment_words(uint64_t n_words) {
  const uint64_t target_waves = static_cast<uint64_t>(device_info().n_cu) * 32;
  uint64_t seg = (n_words + target_waves - 1) / target_waves;
  return static_cast<uint32_t>(seg < 1 ? 1 : (seg > 64 ? 64 : seg));
}

uint32_t grid_for(uint64_t waves_of_work, uint32_t threads, uint32_t per_cu) {
  const uint64_t blocks = (waves_of_work * kWave + threads - 1) / threads;
  const uint64_t cap = static_cast<uint64_t>(device_info().n_cu) * per_cu;
  const uint64_t g = blocks < cap ? blocks : cap;
  return static_cast<uint32_t>(g == 0 ? 1 : g);
}

// ------------------------------------------------------------ launchers

hipError_t launch_zero_u64(uint64_t *p, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint32_t grid = grid_for((n + 63) / 64, kThreads, 4);
  hipLaunchKernelGGL(k_zero_u64, dim3(grid), dim3(kThreads), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_fill_all(uint64_t *bitmap, uint64_t n_rows, uint64_t *count, hipStream_t s) {
  const uint64_t n_words = (n_rows + 63) / 64;
  const uint32_t grid = grid_for((n_words + 63) / 64, kThreads, 8);
  hipLaunchKernelGGL(k_fill_all, dim3(grid), dim3(kThreads), 0, s, n_words ? bitmap : nullptr, n_rows, count);
  return hipGetLastError();
}

hipError_t launch_local_filter(const PredSet &preds, uint64_t n_rows, uint64_t *bitmap, uint64_t *count,
                               hipStream_t s) {
  const uint64_t n_words = (n_rows + 63) / 64;
  if (n_words == 0) return hipSuccess;
  const uint32_t seg_words = segment_words(n_words);
  const uint32_t grid = grid_for((n_words + seg_words - 1) / seg_words, kWideThreads, 1);
  hipLaunchKernelGGL(k_local, dim3(grid), dim3(kWideThreads), 0, s, preds, n_rows, bitmap,
                     reinterpret_cast<unsigned long long *>(count), seg_words);
  return hipGetLastError();
}

hipError_t launch_size(uint32_t block_bits, uint32_t bits_per_key, const FilterSet &fs, const uint64_t *count,
                       uint64_t n_rows, uint64_t entries_cap, uint32_t *status, hipStream_t s) {
  if (fs.n == 0) return hipSuccess;
  const uint32_t lg = log2_of(static_cast<int>(block_bits));
  if (lg == 0) return hipErrorInvalidValue;
  uint64_t max_cap_words = 0;
  for (uint32_t i = 0; i < fs.n; i++) max_cap_words = fs.f[i].cap_words > max_cap_words ? fs.f[i].cap_words : max_cap_words;
  uint64_t gx = (max_cap_words + kThreads * 4 - 1) / (kThreads * 4);
  const uint64_t cap = static_cast<uint64_t>(device_info().n_cu) * 2;
  gx = gx > cap ? cap : (gx == 0 ? 1 : gx);
  hipLaunchKernelGGL(k_size_zero, dim3(static_cast<uint32_t>(gx), fs.n), dim3(kThreads), 0, s, fs, lg, bits_per_key,
                     count, n_rows, entries_cap, status);
  return hipGetLastError();
}

hipError_t launch_copy_counts(const uint64_t *src, const uint32_t *slot, uint32_t n, uint64_t *dst, hipStream_t s) {
  if (n == 0) return hipSuccess;
  SlotTable t{};
  for (uint32_t i = 0; i < n && i < 64; i++) t.slot[i] = slot[i];
  hipLaunchKernelGGL(k_copy_counts, dim3(1), dim3(64), 0, s, src, t, n, dst);
  return hipGetLastError();
}

uint64_t compact_partials(uint64_t n_rows) {
  const uint64_t n_words = (n_rows + 63) / 64;
  return (n_words + kCompactWordsPerBlock - 1) / kCompactWordsPerBlock;
}

hipError_t launch_compact(const uint64_t *bitmap, uint64_t n_rows, uint32_t *idx, uint64_t *count,
                          uint64_t *partials, hipStream_t s) {
  const uint64_t n_words = (n_rows + 63) / 64;
  const uint64_t n_parts = compact_partials(n_rows);
  if (n_parts == 0) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, count, 1);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_compact_count, dim3(static_cast<uint32_t>(n_parts)), dim3(kThreads), 0, s, bitmap, n_words,
                     n_rows, partials);
  hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(1024), 0, s, partials, n_parts, count);
  hipLaunchKernelGGL(k_compact_write, dim3(static_cast<uint32_t>(n_parts)), dim3(kThreads), 0, s, bitmap, n_words,
                     n_rows, partials, idx);
  return hipGetLastError();
}

}  // namespace pt
