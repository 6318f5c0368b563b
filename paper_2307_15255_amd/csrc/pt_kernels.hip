// pt_kernels.hip - gfx950 kernels of the predicate-transfer phase.
//
// Every kernel works on 64-row groups: one wave64 owns one 64-bit bitmap
// word at a time (lane l holds row 64 * w + l), so a wave's ballot is the
// word and each word has exactly one writer. Rows are streamed with
// coalesced 256-byte (int32) or 512-byte (int64) loads per wave.
#include "pt_internal.hpp"

namespace pt {

namespace {

constexpr int kThreads = 256;        // local filter, build, size, compact
constexpr int kProbeThreads = 1024;  // probe: one or two workgroups per CU

__device__ __forceinline__ uint64_t lane_id() { return threadIdx.x & (kWave - 1); }

__device__ __forceinline__ uint64_t global_wave() {
  return (static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / kWave;
}

__device__ __forceinline__ uint64_t wave_count() {
  return static_cast<uint64_t>(gridDim.x) * blockDim.x / kWave;
}

// Adds a per-wave count (held by lane 0) into *out with one atomic per
// workgroup.
__device__ __forceinline__ void block_count_add(uint64_t wave_cnt, unsigned long long *s_cnt,
                                                unsigned long long *out) {
  if (lane_id() == 0 && wave_cnt) atomicAdd(s_cnt, static_cast<unsigned long long>(wave_cnt));
  __syncthreads();
  if (threadIdx.x == 0 && out && *s_cnt) atomicAdd(out, *s_cnt);
}

// A filter's block count as read from device memory, kept inside [1, cap]
// so that no address computed from it leaves the filter's buffer.
__device__ __forceinline__ uint32_t clamp_blocks(uint64_t nb, uint64_t cap_blocks) {
  if (nb > cap_blocks) nb = cap_blocks;
  return static_cast<uint32_t>(nb == 0 ? 1 : nb);
}

// Selects filter i of a set without a dynamically indexed kernel argument.
__device__ __forceinline__ FilterRef pick(const FilterSet &fs, uint32_t i) {
  FilterRef r = fs.f[0];
#pragma unroll
  for (int j = 1; j < kMaxFilters; j++)
    if (i == static_cast<uint32_t>(j)) r = fs.f[j];
  return r;
}

// ------------------------------------------------------------------ zero

__global__ void __launch_bounds__(kThreads) k_zero_u64(uint64_t *p, uint64_t n) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    p[i] = 0;
}

// ---------------------------------------------------------- local filter

__device__ __forceinline__ bool pred_holds(uint32_t op, int64_t v, int64_t lo, int64_t hi) {
  switch (op) {
    case 0: return v < lo;
    case 1: return v <= lo;
    case 2: return v > lo;
    case 3: return v >= lo;
    case 4: return v == lo;
    case 5: return v != lo;
    default: return lo <= v && v <= hi;
  }
}

__global__ void __launch_bounds__(kThreads)
    k_local(PredSet ps, uint64_t n_rows, uint64_t *__restrict__ bitmap,
            unsigned long long *count) {
  __shared__ unsigned long long s_cnt;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  const uint64_t lane = lane_id();
  const uint64_t n_words = (n_rows + 63) / 64;
  uint64_t cnt = 0;
  for (uint64_t w = global_wave(); w < n_words; w += wave_count()) {
    const uint64_t row = w * 64 + lane;
    bool keep = row < n_rows;
    if (ps.and_into) keep = keep && ((bitmap[w] >> lane) & 1);
#pragma unroll
    for (int i = 0; i < kMaxPreds; i++) {
      if (i < static_cast<int>(ps.n) && keep) {
        const PredRef &p = ps.p[i];
        const int64_t v = static_cast<int64_t>(load_key(p.col, p.col64, row));
        keep = pred_holds(p.op, v, p.lo, p.hi);
      }
    }
    const uint64_t word = __ballot(keep);
    if (lane == 0) bitmap[w] = word;
    cnt += __popcll(word);
  }
  block_count_add(cnt, &s_cnt, count);
}

// ------------------------------------------------------------------ probe
//
// One scan of the table probes every incoming filter (the incoming half of
// the filter transformation). Each workgroup first copies the filters that
// fit into its LDS (in filter order, by their current size), then streams
// U bitmap words per wave per iteration: all key columns of the alive rows
// are loaded before any test so every load of the iteration is in flight at
// once.

template <int B, int K, bool ANY64>
__global__ void __launch_bounds__(kProbeThreads)
    k_probe(FilterSet fs, uint32_t k, uint64_t n_rows, uint64_t *__restrict__ bitmap,
            unsigned long long *count, uint32_t lds_cap_words) {
  extern __shared__ uint32_t lds[];
  constexpr int W = BlockShape<B>::kWords;
  constexpr int U = ANY64 ? 4 : 8;
  __shared__ uint32_t s_nb[kMaxProbe];
  __shared__ uint32_t s_off[kMaxProbe];
  __shared__ uint32_t s_staged[kMaxProbe];
  __shared__ unsigned long long s_cnt;

  if (threadIdx.x == 0) {
    uint64_t off = 0;
#pragma unroll
    for (int i = 0; i < kMaxProbe; i++) {
      if (i < static_cast<int>(fs.n)) {
        const uint32_t nb = clamp_blocks(*fs.f[i].nb, fs.f[i].cap_words / W);
        const uint64_t need = static_cast<uint64_t>(nb) * W;
        const bool st = off + need <= lds_cap_words;
        s_nb[i] = nb;
        s_off[i] = static_cast<uint32_t>(off);
        s_staged[i] = st;
        if (st) off += need;
      }
    }
    s_cnt = 0;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kMaxProbe; i++) {
    if (i < static_cast<int>(fs.n) && s_staged[i]) {
      const uint32_t n = s_nb[i] * W;
      const uint32_t *src = fs.f[i].words;
      uint32_t *dst = lds + s_off[i];
      for (uint32_t j = threadIdx.x; j < n; j += blockDim.x) dst[j] = src[j];
    }
  }
  __syncthreads();

  uint32_t nb[kMaxProbe], off[kMaxProbe];
  bool staged[kMaxProbe];
#pragma unroll
  for (int i = 0; i < kMaxProbe; i++) {
    nb[i] = i < static_cast<int>(fs.n) ? s_nb[i] : 0;
    off[i] = i < static_cast<int>(fs.n) ? s_off[i] : 0;
    staged[i] = i < static_cast<int>(fs.n) ? s_staged[i] != 0 : false;
  }

  const uint64_t lane = lane_id();
  const uint64_t n_words = (n_rows + 63) / 64;
  const uint64_t stride = wave_count() * U;
  uint64_t cnt = 0;
  for (uint64_t w0 = global_wave() * U; w0 < n_words; w0 += stride) {
    uint64_t word[U];
    bool alive[U];
    uint64_t any = 0;
#pragma unroll
    for (int u = 0; u < U; u++) {
      const uint64_t w = w0 + u;
      word[u] = w < n_words ? bitmap[w] : 0;
      alive[u] = ((word[u] >> lane) & 1) && (w * 64 + lane) < n_rows;
      any |= word[u];
    }
    if (any == 0) continue;

    uint32_t lo[kMaxProbe][U];
    uint32_t hi[ANY64 ? kMaxProbe : 1][U];
#pragma unroll
    for (int i = 0; i < kMaxProbe; i++) {
      if (i < static_cast<int>(fs.n)) {
#pragma unroll
        for (int u = 0; u < U; u++) {
          if (alive[u]) {
            const uint64_t row = (w0 + u) * 64 + lane;
            if (ANY64 && fs.f[i].key64) {
              const uint64_t x = static_cast<const uint64_t *>(fs.f[i].keys)[row];
              lo[i][u] = static_cast<uint32_t>(x);
              hi[ANY64 ? i : 0][u] = static_cast<uint32_t>(x >> 32);
            } else {
              const int32_t x = static_cast<const int32_t *>(fs.f[i].keys)[row];
              lo[i][u] = static_cast<uint32_t>(x);
              if (ANY64) hi[ANY64 ? i : 0][u] = static_cast<uint32_t>(x >> 31);
            }
          }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kMaxProbe; i++) {
      if (i < static_cast<int>(fs.n)) {
#pragma unroll
        for (int u = 0; u < U; u++) {
          if (alive[u]) {
            uint64_t x;
            if (ANY64)
              x = (static_cast<uint64_t>(hi[ANY64 ? i : 0][u]) << 32) | lo[i][u];
            else
              x = static_cast<uint64_t>(static_cast<int64_t>(static_cast<int32_t>(lo[i][u])));
            uint32_t h1, h2;
            hash_key(x, h1, h2);
            const uint32_t blk = block_of(h1, nb[i]);
            if (staged[i])
              alive[u] = block_has<B, K>(lds + off[i] + blk * W, h2, k);
            else
              alive[u] = block_has<B, K>(fs.f[i].words + static_cast<uint64_t>(blk) * W, h2, k);
          }
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const uint64_t out = __ballot(alive[u]);
      if (lane == 0 && w0 + u < n_words) bitmap[w0 + u] = out;
      cnt += __popcll(out);
    }
  }
  block_count_add(cnt, &s_cnt, count);
}

// --------------------------------------------------------- size and zero
//
// Filter i (blockIdx.y) gets nb = max(1, ceil(count * bits_per_key / B))
// blocks, read from the device counter so the launch sequence never waits
// for the host; its first nb blocks are zeroed.

__global__ void __launch_bounds__(kThreads)
    k_size_zero(FilterSet fs, uint32_t block_bits, uint32_t bits_per_key, const uint64_t *count,
                uint64_t n_rows) {
  const FilterRef f = pick(fs, blockIdx.y);
  const uint64_t n_sel = count ? *count : n_rows;
  const uint64_t words_per_block = block_bits / 32;
  uint64_t nb = (n_sel * bits_per_key + block_bits - 1) / block_bits;
  if (nb == 0) nb = 1;
  const uint64_t cap_blocks = f.cap_words / words_per_block;
  if (nb > cap_blocks) nb = cap_blocks;  // unreachable when the capacity was checked
  if (blockIdx.x == 0 && threadIdx.x == 0) *f.nb = nb;
  const uint64_t n = nb * words_per_block;
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    f.words[i] = 0;
}

// ------------------------------------------------------------------ build
//
// The outgoing half of the filter transformation: every selected row's key
// is inserted into each outgoing filter by atomic OR (order-free, so the
// filter bits do not depend on scheduling).

template <int B, int K>
__global__ void __launch_bounds__(kThreads)
    k_build(FilterSet fs, uint32_t k, uint64_t n_rows, const uint64_t *__restrict__ bitmap) {
  uint32_t nb[kMaxFilters];
#pragma unroll
  for (int i = 0; i < kMaxFilters; i++)
    nb[i] = i < static_cast<int>(fs.n)
                ? clamp_blocks(*fs.f[i].nb, fs.f[i].cap_words / BlockShape<B>::kWords)
                : 0;
  const uint64_t lane = lane_id();
  const uint64_t n_words = (n_rows + 63) / 64;
  for (uint64_t w = global_wave(); w < n_words; w += wave_count()) {
    const uint64_t row = w * 64 + lane;
    const uint64_t word = bitmap ? bitmap[w] : ~0ull;
    if (word == 0) continue;
    if (!(((word >> lane) & 1) && row < n_rows)) continue;
#pragma unroll
    for (int i = 0; i < kMaxFilters; i++) {
      if (i < static_cast<int>(fs.n))
        insert_global<B, K>(fs.f[i].words, nb[i], k, load_key(fs.f[i].keys, fs.f[i].key64, row));
    }
  }
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

// Bits of word w that belong to rows below n_rows.
__device__ __forceinline__ uint64_t tail_mask(uint64_t w, uint64_t n_words, uint64_t n_rows) {
  return (w + 1 == n_words && (n_rows & 63)) ? (1ull << (n_rows & 63)) - 1 : ~0ull;
}

__device__ __forceinline__ uint64_t block_exclusive_scan(uint64_t v, uint64_t *s, uint64_t &total) {
  const uint32_t t = threadIdx.x;
  s[t] = v;
  __syncthreads();
  for (uint32_t d = 1; d < blockDim.x; d <<= 1) {
    const uint64_t add = t >= d ? s[t - d] : 0;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  total = s[blockDim.x - 1];
  const uint64_t incl = s[t];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(kThreads)
    k_compact_count(const uint64_t *__restrict__ bitmap, uint64_t n_words, uint64_t n_rows,
                    uint64_t *partials) {
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

__global__ void __launch_bounds__(1024) k_compact_scan(uint64_t *partials, uint64_t n_parts,
                                                       uint64_t *count) {
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

// ------------------------------------------------------------ dispatch

template <typename F>
hipError_t by_block_bits(uint32_t block_bits, F &&f) {
  switch (block_bits) {
    case 32: return f(std::integral_constant<int, 32>{});
    case 64: return f(std::integral_constant<int, 64>{});
    case 128: return f(std::integral_constant<int, 128>{});
    case 256: return f(std::integral_constant<int, 256>{});
    case 512: return f(std::integral_constant<int, 512>{});
    case 1024: return f(std::integral_constant<int, 1024>{});
    default: return hipErrorInvalidValue;
  }
}

uint32_t grid_for(uint64_t waves_of_work, uint32_t threads, uint32_t per_cu) {
  const uint64_t blocks = (waves_of_work * kWave + threads - 1) / threads;
  const uint64_t cap = static_cast<uint64_t>(device_info().n_cu) * per_cu;
  uint64_t g = blocks < cap ? blocks : cap;
  return static_cast<uint32_t>(g == 0 ? 1 : g);
}

}  // namespace

hipError_t launch_zero_u64(uint64_t *p, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint32_t grid = grid_for((n + 63) / 64, kThreads, 4);
  hipLaunchKernelGGL(k_zero_u64, dim3(grid), dim3(kThreads), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_local_filter(const PredSet &preds, uint64_t n_rows, uint64_t *bitmap,
                               uint64_t *count, hipStream_t s) {
  const uint64_t n_words = (n_rows + 63) / 64;
  if (n_words == 0) return hipSuccess;
  const uint32_t grid = grid_for(n_words, kThreads, 8);
  hipLaunchKernelGGL(k_local, dim3(grid), dim3(kThreads), 0, s, preds, n_rows, bitmap,
                     reinterpret_cast<unsigned long long *>(count));
  return hipGetLastError();
}

hipError_t launch_probe(uint32_t block_bits, uint32_t k, const FilterSet &fs, uint64_t n_rows,
                        uint64_t *bitmap, uint64_t *count, hipStream_t s) {
  const uint64_t n_words = (n_rows + 63) / 64;
  if (n_words == 0) return hipSuccess;
  bool any64 = false;
  uint64_t want_words = 0;
  for (uint32_t i = 0; i < fs.n; i++) {
    any64 = any64 || fs.f[i].key64;
    want_words += fs.f[i].cap_words;
  }
  const DeviceInfo &di = device_info();
  // Leave room for the kernel's own static LDS (a few dozen bytes).
  const uint64_t budget = static_cast<uint64_t>(di.max_lds_block) - 1024;
  uint64_t lds_bytes = want_words * 4;
  if (lds_bytes > budget) lds_bytes = budget;
  const uint32_t per_cu = lds_bytes * 2 <= budget ? 2 : 1;
  const int U = any64 ? 4 : 8;
  const uint32_t grid = grid_for((n_words + U - 1) / U, kProbeThreads, per_cu);
  const uint32_t cap_words = static_cast<uint32_t>(lds_bytes / 4);
  auto *cnt = reinterpret_cast<unsigned long long *>(count);
  return by_block_bits(block_bits, [&](auto bb) -> hipError_t {
    constexpr int B = decltype(bb)::value;
    auto launch = [&](auto kern) -> hipError_t {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kern),
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         static_cast<int>(lds_bytes));
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(kern, dim3(grid), dim3(kProbeThreads), lds_bytes, s, fs, k, n_rows,
                         bitmap, cnt, cap_words);
      return hipGetLastError();
    };
    if (k == 3) return any64 ? launch(k_probe<B, 3, true>) : launch(k_probe<B, 3, false>);
    return any64 ? launch(k_probe<B, 0, true>) : launch(k_probe<B, 0, false>);
  });
}

hipError_t launch_size_zero(uint32_t block_bits, uint32_t bits_per_key, const FilterSet &fs,
                            const uint64_t *count, uint64_t n_rows, hipStream_t s) {
  if (fs.n == 0) return hipSuccess;
  uint64_t max_words = 0;
  for (uint32_t i = 0; i < fs.n; i++) max_words = fs.f[i].cap_words > max_words ? fs.f[i].cap_words : max_words;
  uint64_t gx = (max_words + kThreads * 4 - 1) / (kThreads * 4);
  const uint64_t cap = static_cast<uint64_t>(device_info().n_cu) * 2;
  if (gx > cap) gx = cap;
  if (gx == 0) gx = 1;
  hipLaunchKernelGGL(k_size_zero, dim3(static_cast<uint32_t>(gx), fs.n), dim3(kThreads), 0, s, fs,
                     block_bits, bits_per_key, count, n_rows);
  return hipGetLastError();
}

hipError_t launch_build(uint32_t block_bits, uint32_t k, const FilterSet &fs, uint64_t n_rows,
                        const uint64_t *bitmap, hipStream_t s) {
  const uint64_t n_words = (n_rows + 63) / 64;
  if (n_words == 0 || fs.n == 0) return hipSuccess;
  const uint32_t grid = grid_for(n_words, kThreads, 8);
  return by_block_bits(block_bits, [&](auto bb) -> hipError_t {
    constexpr int B = decltype(bb)::value;
    if (k == 3)
      hipLaunchKernelGGL((k_build<B, 3>), dim3(grid), dim3(kThreads), 0, s, fs, k, n_rows, bitmap);
    else
      hipLaunchKernelGGL((k_build<B, 0>), dim3(grid), dim3(kThreads), 0, s, fs, k, n_rows, bitmap);
    return hipGetLastError();
  });
}

hipError_t launch_copy_counts(const uint64_t *src, const uint32_t *slot, uint32_t n, uint64_t *dst,
                              hipStream_t s) {
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
  hipLaunchKernelGGL(k_compact_count, dim3(static_cast<uint32_t>(n_parts)), dim3(kThreads), 0, s,
                     bitmap, n_words, n_rows, partials);
  hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(1024), 0, s, partials, n_parts, count);
  hipLaunchKernelGGL(k_compact_write, dim3(static_cast<uint32_t>(n_parts)), dim3(kThreads), 0, s,
                     bitmap, n_words, n_rows, partials, idx);
  return hipGetLastError();
}

}  // namespace pt
