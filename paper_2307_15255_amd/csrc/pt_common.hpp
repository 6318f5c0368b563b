// pt_common.hpp - device-side building blocks shared by the gfx950 kernels
// of the predicate-transfer phase: wave and workgroup helpers, the filter
// hash, block addressing, and the bit tests and inserts of a blocked Bloom
// filter (Sec. 2.1 of the paper: no false negatives, possible false
// positives; the filter specification itself is stated in include/pt.h).
//
// A wave64 owns 64-row groups: lane l holds row 64 * w + l of bitmap word w,
// so a wave's ballot is the word. Every branch in the streaming loops is
// wave-uniform; per-lane work that does not matter (rows already removed,
// rows past the end) is computed anyway on clamped, in-bounds addresses and
// masked out, which keeps the exec mask full and the code straight-line.
//
// Block geometry. A kernel specialised for one block size B passes
// log2(B) as a constant; the generic kernels pass it at run time. Every
// helper below is force-inlined, so the constant folds into the shifts.
#pragma once

#include "pt_internal.hpp"

namespace pt {

constexpr uint64_t kHashMul = 0x9E3779B97F4A7C15ull;  // multiply-shift multiplier
constexpr uint32_t kMixMul = 0x85EBCA6Bu;             // second-stage 32-bit multiplier

constexpr int kThreads = 256;        // local filter, build, size, compact
constexpr int kProbeThreads = 1024;  // probe: sixteen waves per workgroup
constexpr int kWideThreads = 1024;   // kernels that count: one workgroup (one atomic) per CU
constexpr int kProbeWaves = kProbeThreads / kWave;

// log2 of the block bits: the compile-time value of a specialised kernel
// (B > 0), else the run-time argument.
template <int B>
__device__ __forceinline__ uint32_t block_log2(uint32_t lg_rt) {
  if constexpr (B > 0) {
    static_assert(log2_of(B) != 0, "block bits");
    return log2_of(B);
  } else {
    return lg_rt;
  }
}

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & (kWave - 1); }

// The wave's index in the grid, as a wave-uniform (scalar) value: the
// compiler cannot tell on its own that threadIdx.x / 64 is the same for
// every lane, and would otherwise keep loop counters derived from it in
// vector registers and turn every uniform branch into an exec-mask branch.
//
// A batched launch runs many tasks in one grid: each task owns a range of
// its workgroups, and sees them as a grid of its own (VGrid: this
// workgroup's index in the task, and the task's workgroup count).
struct VGrid {
  uint32_t block;
  uint32_t blocks;
};

__device__ __forceinline__ VGrid whole_grid() { return VGrid{blockIdx.x, gridDim.x}; }

__device__ __forceinline__ uint64_t global_wave(const VGrid &g) {
  const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  return static_cast<uint64_t>(g.block) * (blockDim.x / kWave) + w;
}

__device__ __forceinline__ uint64_t wave_count(const VGrid &g) {
  return static_cast<uint64_t>(g.blocks) * blockDim.x / kWave;
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, static_cast<uint32_t>(__shfl_xor(v, off)));
  return v;
}

// Adds a wave-uniform count into *out with one global atomic per workgroup.
__device__ __forceinline__ void block_count_add(int64_t wave_cnt, unsigned long long *s_cnt,
                                                unsigned long long *out) {
  if (lane_id() == 0 && wave_cnt) atomicAdd(s_cnt, static_cast<unsigned long long>(wave_cnt));
  __syncthreads();
  if (threadIdx.x == 0 && out && *s_cnt) atomicAdd(out, *s_cnt);
}

// Records a condition in a call's status word (NULL: not reported). Only
// taken on the error path, so the atomic costs nothing in normal runs.
__device__ __forceinline__ void raise_status(uint32_t *status, uint32_t bit) {
  if (status) atomicOr(status, bit);
}

// Whether a build set was pruned: its size step found the builder holding
// every row and recorded a block count of zero (the set's filters share
// their builder, so the first one tells).
__device__ __forceinline__ bool build_pruned(const FilterSet &fs) {
  return fs.prune && fs.n > 0 && *fs.f[0].nb == 0;
}

// A filter's block count as read from device memory, kept inside [1, cap]
// so that no address computed from it leaves the filter's buffer. A count
// above the capacity is reported as an overflow.
__device__ __forceinline__ uint32_t clamp_blocks(uint64_t nb, uint64_t cap_blocks, uint32_t *status) {
  if (nb > cap_blocks) {
    raise_status(status, PT_STATUS_FILTER_OVERFLOW);
    nb = cap_blocks;
  }
  return static_cast<uint32_t>(nb == 0 ? 1 : nb);
}

// Blocks of a filter over n_sel keys (at least one), clamped to the
// capacity; a clamp is reported as an overflow.
__device__ __forceinline__ uint64_t blocks_needed(uint64_t n_sel, uint32_t block_bits, uint32_t bits_per_key,
                                                  uint64_t cap_blocks, uint32_t *status) {
  uint64_t nb = (n_sel * bits_per_key + block_bits - 1) / block_bits;
  if (nb == 0) nb = 1;
  if (nb > cap_blocks) {
    raise_status(status, PT_STATUS_FILTER_OVERFLOW);
    nb = cap_blocks;
  }
  return nb;
}

// Bits of word w that belong to rows below n_rows.
__device__ __forceinline__ uint64_t tail_mask(uint64_t w, uint64_t n_words, uint64_t n_rows) {
  if (w >= n_words) return 0;
  return (w + 1 == n_words && (n_rows & 63)) ? (1ull << (n_rows & 63)) - 1 : ~0ull;
}

// Exclusive prefix sum of v over the workgroup (blockDim.x entries of s).
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

// ------------------------------------------------------------------- hash

// H1 selects the block; H2 supplies the in-block bit positions.
__device__ __forceinline__ void hash_key(uint64_t x, uint32_t &h1, uint32_t &h2) {
  const uint64_t p = x * kHashMul;
  const uint32_t hi = static_cast<uint32_t>(p >> 32);
  uint32_t t = static_cast<uint32_t>(p) ^ hi;
  t ^= t >> 16;
  h1 = hi;
  h2 = t * kMixMul;
}

// The filter hash of an int32 key: the same value as hash_key on its
// sign-extended image x. With A = A_hi * 2^32 + A_lo and A_lo < 2^31, the
// signed product x * A_lo is exact in 64 bits, and x * A mod 2^64 has
// high word hi(x * A_lo) + lo * A_hi mod 2^32 (x and lo agree mod 2^32):
// one signed and one unsigned multiply-add instead of three multiplies and a
// sign correction.
__device__ __forceinline__ void hash_key32(uint32_t lo, uint32_t &h1, uint32_t &h2) {
  constexpr uint32_t a_lo = static_cast<uint32_t>(kHashMul);
  constexpr uint32_t a_hi = static_cast<uint32_t>(kHashMul >> 32);
  static_assert(a_lo < 0x80000000u, "the low word of the multiplier must be a positive int32");
  const int64_t p = static_cast<int64_t>(static_cast<int32_t>(lo)) * static_cast<int64_t>(a_lo);
  const uint32_t hi = static_cast<uint32_t>(static_cast<uint64_t>(p) >> 32) + lo * a_hi;
  uint32_t t = static_cast<uint32_t>(p) ^ hi;
  t ^= t >> 16;
  h1 = hi;
  h2 = t * kMixMul;
}

__device__ __forceinline__ void hash_parts(uint32_t lo, uint32_t hi, bool key64, uint32_t &h1, uint32_t &h2) {
  if (key64)
    hash_key((static_cast<uint64_t>(hi) << 32) | lo, h1, h2);
  else
    hash_key32(lo, h1, h2);
}

// Key of row r of a column, as the uint64 image of its int64 value.
__device__ __forceinline__ uint64_t load_key(const void *col, uint32_t key64, uint64_t r) {
  if (key64) return static_cast<uint64_t>(static_cast<const int64_t *>(col)[r]);
  return static_cast<uint64_t>(static_cast<int64_t>(static_cast<const int32_t *>(col)[r]));
}

// ---------------------------------------------------------- block access

// Index of the block a key lands in (multiply-high range reduction).
__device__ __forceinline__ uint32_t block_of(uint32_t h1, uint32_t nb) { return __umulhi(h1, nb); }

// The two double-hashing terms of a key's in-block positions.
__device__ __forceinline__ void probe_terms(uint32_t h2, uint32_t lg, uint32_t &g1, uint32_t &g2) {
  g1 = h2 >> (32 - lg);
  g2 = ((h2 >> (32 - 2 * lg)) & ((1u << lg) - 1)) | 1u;
}

// All k bits of a key set? `blk` points at the first word of its block (in
// LDS or in global memory). K > 0 fixes k at compile time; K == 0 reads k at
// run time.
template <int K>
__device__ __forceinline__ bool block_has(const uint32_t *blk, uint32_t h2, uint32_t k, uint32_t lg) {
  uint32_t g1, g2;
  probe_terms(h2, lg, g1, g2);
  const uint32_t mask = (1u << lg) - 1;
  uint32_t pos = g1;
  uint32_t all = 1;
  if constexpr (K > 0) {
#pragma unroll
    for (int i = 0; i < K; i++) {
      const uint32_t p = pos & mask;
      all &= blk[p >> 5] >> (p & 31);
      pos += g2;
    }
  } else {
    for (uint32_t i = 0; i < k; i++) {
      const uint32_t p = pos & mask;
      all &= blk[p >> 5] >> (p & 31);
      pos += g2;
    }
  }
  return (all & 1u) != 0;
}

// Sets the k bits of (h1, h2) in a filter in global memory with atomic OR;
// each bit is first read with a device-coherent load and written only if it
// is not already set. Bits only go from 0 to 1 during a build, so a stale
// read can only cost an extra atomic, never a lost bit.
template <int K>
__device__ __forceinline__ void insert_bits(uint32_t *words, uint32_t nb, uint32_t k, uint32_t h1, uint32_t h2,
                                            uint32_t lg) {
  uint32_t *blk = words + (static_cast<uint64_t>(block_of(h1, nb)) << (lg - 5));
  uint32_t g1, g2;
  probe_terms(h2, lg, g1, g2);
  const uint32_t mask = (1u << lg) - 1;
  uint32_t pos = g1;
  const uint32_t kk = K > 0 ? static_cast<uint32_t>(K) : k;
#pragma unroll
  for (uint32_t i = 0; i < kk; i++) {
    const uint32_t p = pos & mask;
    const uint32_t bit = 1u << (p & 31);
    uint32_t *w = blk + (p >> 5);
    if ((__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & bit) == 0) atomicOr(w, bit);
    pos += g2;
  }
}

// The same in a filter held in LDS (32-bit offsets).
template <int K>
__device__ __forceinline__ void insert_lds(uint32_t *filter, uint32_t nb, uint32_t k, uint32_t h1, uint32_t h2,
                                           uint32_t lg) {
  uint32_t *blk = filter + (block_of(h1, nb) << (lg - 5));
  uint32_t g1, g2;
  probe_terms(h2, lg, g1, g2);
  const uint32_t mask = (1u << lg) - 1;
  uint32_t pos = g1;
  const uint32_t kk = K > 0 ? static_cast<uint32_t>(K) : k;
#pragma unroll
  for (uint32_t i = 0; i < kk; i++) {
    const uint32_t p = pos & mask;
    // A bit already set needs no atomic: repeated keys (a foreign key with
    // few distinct values) would otherwise serialise on one LDS word.
    const uint32_t bit = 1u << (p & 31);
    if (!(blk[p >> 5] & bit)) atomicOr(blk + (p >> 5), bit);
    pos += g2;
  }
}

}  // namespace pt
