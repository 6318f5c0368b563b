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

// Sizes the set from the builder's selected rows (four times that many
// slots, rounded up to a power of two, within [64, 2^lg_cap]; the capacity
// holds twice the builder's rows, so the table is at most half full) and
// clears it. Most probes look up an absent key, whose linear probe ends at
// the first free slot: a quarter-full table keeps those chains short. With
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
  while (lg < f.lg_cap && (1ull << lg) < 4 * n) lg++;
  if (thread_index() == 0) {
    *f.lg = lg;
    f.keys[1ull << f.lg_cap] = 0;  // INT64_MIN not present
  }
  for (uint64_t i = thread_index(); i < (1ull << lg); i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    f.keys[i] = kSetEmpty;
}

// Rows a wave takes per step in the set kernels: kSetWords bitmap words, one
// row of each per lane, so that every lane has several reads in flight.
constexpr int kSetWords = 4;

// Keys of rows base + 64 u + lane (u < kSetWords) of a column, as int64
// images, for the lanes whose bit u of `live` is set (0 elsewhere). Every
// lane loads (the others from row 0, one cache line for all of them), and
// the width test is outside the loads, so they are issued together.
__device__ __forceinline__ void set_keys(const void *col, uint32_t key64, uint64_t base, uint32_t live,
                                        unsigned long long (&key)[kSetWords]) {
  const uint32_t lane = lane_id();
  uint64_t row[kSetWords];
#pragma unroll
  for (int u = 0; u < kSetWords; u++) row[u] = (live >> u) & 1 ? base + u * 64 + lane : 0;
  if (key64) {
#pragma unroll
    for (int u = 0; u < kSetWords; u++) key[u] = static_cast<const unsigned long long *>(col)[row[u]];
  } else {
    uint32_t x[kSetWords];
#pragma unroll
    for (int u = 0; u < kSetWords; u++) x[u] = static_cast<const uint32_t *>(col)[row[u]];
#pragma unroll
    for (int u = 0; u < kSetWords; u++)
      key[u] = static_cast<unsigned long long>(static_cast<int64_t>(static_cast<int32_t>(x[u])));
  }
#pragma unroll
  for (int u = 0; u < kSetWords; u++)
    if (!((live >> u) & 1)) key[u] = 0;
}

// Inserts the key of every selected row (bitmap NULL: every row). The slots
// in use are at least twice the selected rows, so a free slot is reached.
// A wave reads 64 bitmap words per step (one per lane) and takes the words
// that hold selected rows kSetWords at a time: the keys of their selected
// rows are read together, then inserted one word after the other.
__global__ void __launch_bounds__(kThreads) k_set_build(SetRef f, uint64_t n_rows, const uint64_t *bitmap) {
  constexpr int U = kSetWords;
  const uint32_t lg = static_cast<uint32_t>(*f.lg);
  if (lg == 0) return;  // pruned
  const uint64_t mask = (1ull << lg) - 1;
  const uint64_t n_words = (n_rows + 63) / 64;
  const uint32_t lane = lane_id();
  const uint64_t n_waves = static_cast<uint64_t>(gridDim.x) * (blockDim.x / kWave);
  for (uint64_t w0 = thread_index() / kWave * kWave; w0 < n_words; w0 += n_waves * kWave) {
    // lane l: word w0 + l
    const uint64_t wl = w0 + lane;
    uint64_t mine = wl < n_words ? tail_mask(wl, n_words, n_rows) : 0;
    if (bitmap) mine &= bitmap[min(wl, n_words - 1)];
    for (uint64_t todo = __ballot(mine != 0); todo;) {
      // up to U of the words that hold selected rows
      uint32_t live = 0;
      uint64_t base[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        base[u] = 0;
        if (todo) {
          const uint32_t j = __builtin_ctzll(todo);
          todo &= todo - 1;
          const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(mine), j);
          const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(mine >> 32), j);
          const uint64_t word = (static_cast<uint64_t>(hi) << 32) | lo;
          base[u] = (w0 + j) * 64;
          live |= static_cast<uint32_t>((word >> lane) & 1) << u;
        }
      }
      unsigned long long key[U];
      {
        // the rows of word u start at base[u]: one load per word
        uint64_t row[U];
#pragma unroll
        for (int u = 0; u < U; u++) row[u] = (live >> u) & 1 ? base[u] + lane : 0;
        if (f.key64) {
#pragma unroll
          for (int u = 0; u < U; u++) key[u] = static_cast<const unsigned long long *>(f.col)[row[u]];
        } else {
          uint32_t x[U];
#pragma unroll
          for (int u = 0; u < U; u++) x[u] = static_cast<const uint32_t *>(f.col)[row[u]];
#pragma unroll
          for (int u = 0; u < U; u++)
            key[u] = static_cast<unsigned long long>(static_cast<int64_t>(static_cast<int32_t>(x[u])));
        }
      }
#pragma unroll
      for (int u = 0; u < U; u++) {
        if (!((live >> u) & 1)) continue;
        if (key[u] == kSetEmpty) {
          f.keys[1ull << f.lg_cap] = 1;
          continue;
        }
        for (uint64_t s = set_slot(key[u], lg);; s = (s + 1) & mask) {
          const unsigned long long prev = atomicCAS(&f.keys[s], kSetEmpty, key[u]);
          if (prev == kSetEmpty || prev == key[u]) break;
        }
      }
    }
  }
}

// One scan of a table: a row stays when its key is in every incoming set.
// A wave takes kSetWords words per step (lane l holds row 64 w + l of
// each); set by set, it reads the keys of the rows still selected and
// issues the first slot read of every one of them before it resolves any.
__global__ void __launch_bounds__(kThreads)
    k_set_probe(SetProbe sp, uint64_t n_rows, uint64_t *bitmap, unsigned long long *count, uint32_t input_all) {
  constexpr int U = kSetWords;
  __shared__ unsigned long long s_cnt;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  uint32_t lg[kMaxProbe];
#pragma unroll
  for (int j = 0; j < kMaxProbe; j++) lg[j] = j < static_cast<int>(sp.n) ? static_cast<uint32_t>(*sp.f[j].lg) : 0;
  const uint64_t n_words = (n_rows + 63) / 64;
  const uint32_t lane = lane_id();
  const uint64_t n_waves = static_cast<uint64_t>(gridDim.x) * (blockDim.x / kWave);
  uint64_t cnt = 0;
  for (uint64_t w0 = thread_index() / kWave * U; w0 < n_words; w0 += n_waves * U) {
    uint32_t live = 0;
    uint64_t bits[U];  // (clamped reads, all issued together)
#pragma unroll
    for (int u = 0; u < U; u++) bits[u] = input_all ? ~0ull : bitmap[min(w0 + u, n_words - 1)];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const uint64_t w = w0 + u;
      const uint64_t word = w < n_words ? tail_mask(w, n_words, n_rows) & bits[u] : 0;
      live |= static_cast<uint32_t>((word >> lane) & 1) << u;
    }
#pragma unroll
    for (int j = 0; j < kMaxProbe; j++) {
      if (j >= static_cast<int>(sp.n) || lg[j] == 0) continue;  // lg 0: a pruned set
      if (__ballot(live != 0) == 0) break;
      const SetRef &f = sp.f[j];
      unsigned long long key[U];
      set_keys(f.col, f.key64, w0 * 64, live, key);
      const uint64_t mask = (1ull << lg[j]) - 1;
      uint64_t slot[U];
      unsigned long long v[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        // every lane reads (dead lanes slot 0), so the reads go out together
        const bool go = ((live >> u) & 1) && key[u] != kSetEmpty;
        slot[u] = set_slot(key[u], lg[j]);
        v[u] = f.keys[go ? slot[u] : 0];
        if (!go) v[u] = kSetEmpty;
      }
#pragma unroll
      for (int u = 0; u < U; u++) {
        if (!((live >> u) & 1)) continue;
        bool has;
        if (key[u] == kSetEmpty) {
          has = f.keys[1ull << f.lg_cap] != 0;
        } else {
          while (v[u] != key[u] && v[u] != kSetEmpty) {
            slot[u] = (slot[u] + 1) & mask;
            v[u] = f.keys[slot[u]];
          }
          has = v[u] == key[u];
        }
        if (!has) live &= ~(1u << u);
      }
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const uint64_t m = __ballot((live >> u) & 1);
      if (w0 + u < n_words) {
        if (lane == 0) bitmap[w0 + u] = m;
        cnt += __popcll(m);
      }
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
