// k_exact.hip - transfer with exact filters (Sec. 3.2, "Filter Type": with
// a precise filter instead of a Bloom filter the transfer phase is a series
// of semi-joins, as in the semi-join phase of Yannakakis, Sec. 2.2). A
// filter is the set of distinct keys of the builder's selected rows, held
// in an open-addressing hash table of int64 keys in device memory and sized
// on the device from the builder's selected rows; a probe keeps a row when
// its key is in every incoming set.
#include "pt_common.hpp"

namespace pt {

namespace {

constexpr unsigned long long kSetEmpty = 0x8000000000000000ull;  // INT64_MIN marks a free slot

__device__ __forceinline__ uint64_t thread_index() {
  return static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
}

__device__ __forceinline__ uint64_t set_slot(unsigned long long key, uint32_t lg) {
  return static_cast<uint64_t>(key * kHashMul) >> (64 - lg);  // multiply-shift
}

// Whether `key` is in the set (lg: log2 of the slots in use).
__device__ __forceinline__ bool set_has(const SetRef &f, uint32_t lg, unsigned long long key) {
  if (key == kSetEmpty) return f.keys[1ull << f.lg_cap] != 0;
  const uint64_t mask = (1ull << lg) - 1;
  for (uint64_t s = set_slot(key, lg);; s = (s + 1) & mask) {
    const unsigned long long k2 = f.keys[s];
    if (k2 == key) return true;
    if (k2 == kSetEmpty) return false;
  }
}

// Sizes the set from the builder's selected rows (twice that many slots,
// rounded up to a power of two, within [64, 2^lg_cap]) and clears it. With
// prune, a non-empty builder that still holds every row leaves lg = 0: no
// set.
__global__ void __launch_bounds__(kThreads)
    k_set_clear(SetRef f, const uint64_t *count, uint64_t n_rows, uint32_t prune) {
  uint64_t n = count ? *count : n_rows;
  if (prune && count && n_rows > 0 && n == n_rows) {
    if (thread_index() == 0) *f.lg = 0;
    return;
  }
  if (n > n_rows) n = n_rows;
  uint32_t lg = 6;
  while (lg < f.lg_cap && (1ull << lg) < 2 * n) lg++;
  if (thread_index() == 0) {
    *f.lg = lg;
    f.keys[1ull << f.lg_cap] = 0;  // INT64_MIN not present
  }
  for (uint64_t i = thread_index(); i < (1ull << lg); i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    f.keys[i] = kSetEmpty;
}

// Inserts the key of every selected row (bitmap NULL: every row). The slots
// in use are at least twice the selected rows, so a free slot is reached.
__global__ void __launch_bounds__(kThreads) k_set_build(SetRef f, uint64_t n_rows, const uint64_t *bitmap) {
  const uint32_t lg = static_cast<uint32_t>(*f.lg);
  if (lg == 0) return;  // pruned
  const uint64_t mask = (1ull << lg) - 1;
  const uint64_t n_words = (n_rows + 63) / 64;
  const uint32_t lane = lane_id();
  const uint64_t n_waves = static_cast<uint64_t>(gridDim.x) * (blockDim.x / kWave);
  for (uint64_t w = thread_index() / kWave; w < n_words; w += n_waves) {
    const uint64_t bits = bitmap ? bitmap[w] : ~0ull;
    const uint64_t r = w * 64 + lane;
    if (r >= n_rows || !((bits >> lane) & 1)) continue;
    const unsigned long long key = load_key(f.col, f.key64, r);
    if (key == kSetEmpty) {
      f.keys[1ull << f.lg_cap] = 1;
      continue;
    }
    for (uint64_t s = set_slot(key, lg);; s = (s + 1) & mask) {
      const unsigned long long prev = atomicCAS(&f.keys[s], kSetEmpty, key);
      if (prev == kSetEmpty || prev == key) break;
    }
  }
}

// One scan of a table: a row stays when its key is in every incoming set.
// Each wave takes bitmap words; lane l holds row 64 w + l.
__global__ void __launch_bounds__(kThreads)
    k_set_probe(SetProbe sp, uint64_t n_rows, uint64_t *bitmap, unsigned long long *count, uint32_t input_all) {
  __shared__ unsigned long long s_cnt;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  uint32_t lg[kMaxProbe];
#pragma unroll
  for (int j = 0; j < kMaxProbe; j++) lg[j] = j < static_cast<int>(sp.n) ? static_cast<uint32_t>(*sp.f[j].lg) : 6;
  const uint64_t n_words = (n_rows + 63) / 64;
  const uint32_t lane = lane_id();
  const uint64_t n_waves = static_cast<uint64_t>(gridDim.x) * (blockDim.x / kWave);
  uint64_t cnt = 0;
  for (uint64_t w = thread_index() / kWave; w < n_words; w += n_waves) {
    const uint64_t word = tail_mask(w, n_words, n_rows) & (input_all ? ~0ull : bitmap[w]);
    const uint64_t r = w * 64 + lane;
    bool keep = (word >> lane) & 1;
#pragma unroll
    for (int j = 0; j < kMaxProbe; j++) {
      if (j < static_cast<int>(sp.n) && keep && lg[j] != 0)  // lg 0: a pruned set
        keep = set_has(sp.f[j], lg[j], load_key(sp.f[j].col, sp.f[j].key64, r));
    }
    const uint64_t m = __ballot(keep);
    if (lane == 0) {
      bitmap[w] = m;
      cnt += __popcll(m);
    }
  }
  if (lane_id() == 0 && cnt) atomicAdd(&s_cnt, static_cast<unsigned long long>(cnt));
  __syncthreads();
  if (threadIdx.x == 0 && count && s_cnt) atomicAdd(count, s_cnt);
}

}  // namespace

hipError_t launch_set_build(const SetRef &f, uint64_t n_rows, const uint64_t *bitmap, const uint64_t *count,
                            bool prune, hipStream_t s) {
  hipLaunchKernelGGL(k_set_clear, dim3(grid_for((1ull << f.lg_cap) / 64, kThreads, 8)), dim3(kThreads), 0, s, f,
                     count, n_rows, prune ? 1u : 0u);
  if (n_rows)
    hipLaunchKernelGGL(k_set_build, dim3(grid_for((n_rows + 63) / 64, kThreads, 8)), dim3(kThreads), 0, s, f,
                       n_rows, bitmap);
  return hipGetLastError();
}

hipError_t launch_set_probe(const SetProbe &sp, uint64_t n_rows, uint64_t *bitmap, uint64_t *count, bool input_all,
                            hipStream_t s) {
  if (n_rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_probe, dim3(grid_for((n_rows + 63) / 64, kThreads, 8)), dim3(kThreads), 0, s, sp, n_rows,
                     bitmap, reinterpret_cast<unsigned long long *>(count), input_all ? 1u : 0u);
  return hipGetLastError();
}

}  // namespace pt
