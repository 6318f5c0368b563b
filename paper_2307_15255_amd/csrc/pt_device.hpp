// pt_device.hpp - device-side building blocks of the predicate-transfer
// kernels for gfx950 (wave64): the filter hash, block addressing, and the
// bit tests and inserts of a blocked Bloom filter.
//
// The filter specification is stated in include/pt.h. Bloom filters: no false
// negatives, possible false positives (Sec. 2.1 of the paper).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pt {

constexpr uint64_t kHashMul = 0x9E3779B97F4A7C15ull;  // multiply-shift multiplier
constexpr uint32_t kMixMul = 0x85EBCA6Bu;             // second-stage 32-bit multiplier

constexpr int kWave = 64;
constexpr int kMaxFilters = 8;  // filters handled by one build launch
constexpr int kMaxProbe = 4;    // filters handled by one probe launch (their keys stay in registers)
constexpr int kMaxPreds = 8;    // predicates handled by one local-filter launch

template <int B>
struct BlockShape {
  static_assert(B >= 32 && B <= 1024 && (B & (B - 1)) == 0, "block bits");
  static constexpr int kBits = B;
  static constexpr int kWords = B / 32;
  static constexpr int kLog2 = (B == 32) ? 5 : (B == 64) ? 6 : (B == 128) ? 7 : (B == 256) ? 8
                               : (B == 512) ? 9 : 10;
};

// H1 selects the block; H2 supplies the in-block bit positions.
__device__ __forceinline__ void hash_key(uint64_t x, uint32_t &h1, uint32_t &h2) {
  const uint64_t p = x * kHashMul;
  const uint32_t hi = static_cast<uint32_t>(p >> 32);
  uint32_t t = static_cast<uint32_t>(p) ^ hi;
  t ^= t >> 16;
  h1 = hi;
  h2 = t * kMixMul;
}

// Key of row r of a column, as the uint64 image of its int64 value.
__device__ __forceinline__ uint64_t load_key(const void *col, uint32_t key64, uint64_t r) {
  if (key64) return static_cast<uint64_t>(static_cast<const int64_t *>(col)[r]);
  return static_cast<uint64_t>(static_cast<int64_t>(static_cast<const int32_t *>(col)[r]));
}

// Word index (within the filter) of block blk.
__device__ __forceinline__ uint32_t block_of(uint32_t h1, uint32_t nb) { return __umulhi(h1, nb); }

// All k bits of a key set? `blk` points at the first word of its block (in
// LDS or in global memory). K > 0 fixes k at compile time; K == 0 reads k at
// run time.
template <int B, int K>
__device__ __forceinline__ bool block_has(const uint32_t *blk, uint32_t h2, uint32_t k) {
  using S = BlockShape<B>;
  const uint32_t g1 = h2 >> (32 - S::kLog2);
  const uint32_t g2 = ((h2 >> (32 - 2 * S::kLog2)) & (B - 1)) | 1u;
  uint32_t pos = g1;
  uint32_t all = 1;
  if constexpr (K > 0) {
#pragma unroll
    for (int i = 0; i < K; i++) {
      const uint32_t p = pos & (B - 1);
      all &= blk[p >> 5] >> (p & 31);
      pos += g2;
    }
  } else {
    for (uint32_t i = 0; i < k; i++) {
      const uint32_t p = pos & (B - 1);
      all &= blk[p >> 5] >> (p & 31);
      pos += g2;
    }
  }
  return (all & 1u) != 0;
}

// Set the k bits of a key in a filter in global memory. A bit is only
// written by an atomic OR when a plain read does not already show it set;
// bits only go from 0 to 1 during a build, so a stale read can only cost an
// extra atomic, never a lost bit.
template <int B, int K>
__device__ __forceinline__ void insert_global(uint32_t *words, uint32_t nb, uint32_t k,
                                              uint64_t x) {
  using S = BlockShape<B>;
  uint32_t h1, h2;
  hash_key(x, h1, h2);
  uint32_t *blk = words + static_cast<uint64_t>(block_of(h1, nb)) * S::kWords;
  const uint32_t g1 = h2 >> (32 - S::kLog2);
  const uint32_t g2 = ((h2 >> (32 - 2 * S::kLog2)) & (B - 1)) | 1u;
  uint32_t pos = g1;
  const uint32_t kk = K > 0 ? static_cast<uint32_t>(K) : k;
#pragma unroll
  for (uint32_t i = 0; i < (K > 0 ? static_cast<uint32_t>(K) : kk); i++) {
    const uint32_t p = pos & (B - 1);
    const uint32_t bit = 1u << (p & 31);
    uint32_t *w = blk + (p >> 5);
    if ((*w & bit) == 0) atomicOr(w, bit);
    pos += g2;
  }
}

}  // namespace pt
