// pt_internal.hpp - launch descriptors shared by the host API and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "pt_device.hpp"

namespace pt {

// One filter as a probe or build launch sees it.
struct FilterRef {
  const void *keys;   // key column of the scanned table
  uint32_t *words;    // filter words (device)
  uint64_t *nb;       // device: number of blocks in use
  uint64_t cap_words; // capacity of `words`
  uint32_t key64;     // key column is int64
  uint32_t pad;
  // Probe order hint: the builder kept *sel of its `rows` rows (NULL or 0:
  // unknown). Filters with the smallest ratio are tested first.
  const uint64_t *sel;
  uint64_t rows;
};

struct FilterSet {
  uint32_t n;
  uint32_t pad;
  FilterRef f[kMaxFilters];
};

struct PredRef {
  const void *col;
  uint32_t col64;
  uint32_t op;
  int64_t lo, hi;
};

struct PredSet {
  uint32_t n;
  uint32_t and_into;  // AND into the existing bitmap instead of overwriting it
  PredRef p[kMaxPreds];
};

struct DeviceInfo {
  int device = -1;
  int n_cu = 0;
  int max_lds_block = 0;  // bytes of LDS one workgroup may allocate
};

const DeviceInfo &device_info();

// Launchers (pt_kernels.hip). Each returns hipSuccess or the launch error.
hipError_t launch_zero_u64(uint64_t *p, uint64_t n, hipStream_t s);
hipError_t launch_local_filter(const PredSet &preds, uint64_t n_rows, uint64_t *bitmap,
                               uint64_t *count, hipStream_t s);
hipError_t launch_fill_all(uint64_t *bitmap, uint64_t n_rows, uint64_t *count, hipStream_t s);
// input_all: every row starts selected (the bitmap is not read, only written).
hipError_t launch_probe(uint32_t block_bits, uint32_t k, const FilterSet &fs, uint64_t n_rows,
                        uint64_t *bitmap, uint64_t *count, bool input_all, hipStream_t s);
constexpr uint32_t kTileWords = 16384;   // 64 KB of filter per partitioned-build tile
constexpr uint32_t kMaxBuckets = 16384;  // (filter, tile) buckets of one partitioned build

// Device buffers a build may use. copies: private per-workgroup LDS copies
// (filters that fit in LDS); hist / totals / starts / entries: the
// partitioned build (hist_groups x kMaxBuckets counters, kMaxBuckets totals,
// kMaxBuckets + 1 starts, entries_cap entries). Any part may be absent.
struct BuildScratch {
  uint32_t *copies = nullptr;
  uint64_t copies_words = 0;
  uint32_t *hist = nullptr;
  uint32_t hist_groups = 0;
  uint64_t *totals = nullptr;
  uint64_t *starts = nullptr;
  uint64_t *entries = nullptr;
  uint64_t entries_cap = 0;
};

// Sizes filters from *count (n_rows when count is NULL) and builds them
// from the selected rows (bitmap NULL: all rows).
hipError_t launch_build(uint32_t block_bits, uint32_t k, uint32_t bits_per_key, const FilterSet &fs,
                        uint64_t n_rows, const uint64_t *bitmap, const uint64_t *count,
                        const BuildScratch *scratch, hipStream_t s);
// Words of LDS one build workgroup uses for its private filter copies.
uint64_t build_lds_words();
hipError_t launch_copy_counts(const uint64_t *src, const uint32_t *slot, uint32_t n,
                              uint64_t *dst, hipStream_t s);
hipError_t launch_compact(const uint64_t *bitmap, uint64_t n_rows, uint32_t *idx, uint64_t *count,
                          uint64_t *partials, hipStream_t s);
uint64_t compact_partials(uint64_t n_rows);

}  // namespace pt
