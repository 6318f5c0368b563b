// pt_internal.hpp - launch descriptors shared by the host API and the kernel
// translation units, and the launchers each of those units exports.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pt.h"

namespace pt {

constexpr int kWave = 64;
constexpr int kMaxFilters = 8;  // filters handled by one build launch
constexpr int kMaxProbe = 4;    // filters handled by one probe launch (their keys stay in registers)
constexpr int kMaxPreds = 8;    // predicates handled by one local-filter launch

// One filter as a probe or build launch sees it.
struct FilterRef {
  const void *keys;   // key column of the scanned table
  uint32_t *words;    // filter words (device)
  uint64_t *nb;       // device: number of blocks in use
  uint64_t cap_words; // capacity of `words`
  uint32_t key64;     // key column is int64
  uint32_t app;       // build: 1 + the appended column holding the keys (0: none)
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

// Survivor keys a probe appends for the builds that follow it (the
// transformation scans the table once). Region r belongs to wave r of the
// probe grid and holds, in its first counts[r] slots, the keys of the rows
// that survived in that wave's word groups (groups r, r + n_regions, ... of
// group_words words). A region whose survivors exceed region_cap, or with a
// word group of more than 64 survivors of the probe's first filter, is
// marked by a count above region_cap; builds walk that region's bitmap words
// instead.
constexpr int kMaxAppend = 4;
struct AppendSet {
  uint32_t n_cols = 0;         // 0: nothing appended
  uint32_t n_regions = 0;
  uint32_t region_cap = 0;     // entries per region and column
  uint32_t group_words = 0;
  uint32_t *counts = nullptr;  // [n_regions]
  const void *src[kMaxAppend] = {};
  void *dst[kMaxAppend] = {};  // [n_regions * region_cap] keys of src's width
  uint32_t key64[kMaxAppend] = {};
};
// Upper bound of a probe grid's waves (regions of an AppendSet).
constexpr uint32_t kMaxRegions = 65536;

// Launch options of a probe that come from the caller's parameters.
struct ProbeOpts {
  uint64_t lds_budget = 0;  // bytes of LDS to stage filters in (0: as much as the device allows)
  bool keep_order = false;  // test the filters in the given order (no selectivity ordering)
};

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
  uint32_t *entries = nullptr;
  uint64_t entries_cap = 0;
};

// ------------------------------------------------------------ launchers
//
// Each returns hipSuccess or the launch error. `status` (may be NULL) is the
// call's device status word: kernels OR PT_STATUS_* bits into it.

// k_misc.hip
hipError_t launch_zero_u64(uint64_t *p, uint64_t n, hipStream_t s);
hipError_t launch_local_filter(const PredSet &preds, uint64_t n_rows, uint64_t *bitmap, uint64_t *count,
                               hipStream_t s);
hipError_t launch_fill_all(uint64_t *bitmap, uint64_t n_rows, uint64_t *count, hipStream_t s);
hipError_t launch_copy_counts(const uint64_t *src, const uint32_t *slot, uint32_t n, uint64_t *dst,
                              hipStream_t s);
hipError_t launch_compact(const uint64_t *bitmap, uint64_t n_rows, uint32_t *idx, uint64_t *count,
                          uint64_t *partials, hipStream_t s);
uint64_t compact_partials(uint64_t n_rows);
// Rows the allocation-free compaction takes at most, and the device address
// of its partial counts on the current device (a static device array, found
// once per device).
constexpr uint64_t kStaticCompactRows = 1ull << 31;
hipError_t static_compact_scratch(uint64_t **out);
// Sizes filters from *count (n_rows when count is NULL) and zeroes their
// blocks, except when a partitioned build with entries_cap entries (0:
// none) will write every block: that is decided on the device from *count.
hipError_t launch_size(uint32_t block_bits, uint32_t bits_per_key, const FilterSet &fs, const uint64_t *count,
                       uint64_t n_rows, uint64_t entries_cap, uint32_t *status, hipStream_t s);

// Raises a kernel's dynamic-LDS limit once per device (to the largest
// request seen); later launches that fit skip the call.
hipError_t allow_lds(const void *kern, uint64_t bytes);
// Bitmap words per wave for the word-segment kernels: enough waves to cover
// the device several times over, at most one word per lane.
uint32_t segment_words(uint64_t n_words);
uint32_t grid_for(uint64_t waves_of_work, uint32_t threads, uint32_t per_cu);

// k_probe*.hip
// input_all: every row starts selected (the bitmap is not read, only written).
// app (optional, in/out): columns to append (n_cols, src, dst, key64,
// counts) and the capacity of each dst in entries (capacity); the launch
// fills in its region geometry, or sets n_cols = 0 when it appends nothing.
hipError_t launch_probe(uint32_t block_bits, uint32_t k, const FilterSet &fs, uint64_t n_rows, uint64_t *bitmap,
                        uint64_t *count, bool input_all, AppendSet *app, uint64_t capacity,
                        const ProbeOpts &opt, uint32_t *status, hipStream_t s);

// Arguments of one probe kernel launch (built by launch_probe).
struct ProbeLaunch {
  FilterSet fs;
  uint32_t k, lg;
  uint64_t n_rows;
  uint64_t *bitmap;
  unsigned long long *count;
  uint32_t lds_filter_words;
  uint32_t input_all;
  uint32_t keep_order;
  uint32_t *status;
  AppendSet app;
  uint32_t grid;
  uint64_t lds_bytes;
};
// One probe kernel, specialised for B = 512 and k = 3 (k_probe_512.hip) or
// generic in B and k (k_probe_gen.hip).
hipError_t launch_probe_512_k3(const ProbeLaunch &pl, hipStream_t s);
hipError_t launch_probe_generic(const ProbeLaunch &pl, hipStream_t s);

// k_build.hip / k_part.hip
// Sizes filters from *count (n_rows when count is NULL) and builds them
// from the selected rows (bitmap NULL: all rows). With app (the AppendSet
// of the probe that produced the bitmap, every filter's `app` set), the
// keys are read from the appended columns.
hipError_t launch_build(uint32_t block_bits, uint32_t k, uint32_t bits_per_key, const FilterSet &fs,
                        uint64_t n_rows, const uint64_t *bitmap, const uint64_t *count,
                        const BuildScratch *scratch, const AppendSet *app, uint32_t *status, hipStream_t s);
// Words of LDS one build workgroup uses for its private filter copies.
uint64_t build_lds_words();
// Partitioned build of filters too large for LDS (sized and not zeroed
// beforehand by launch_size); falls back to global atomics in place when
// the plan does not fit the scratch (then the filters must be zeroed).
hipError_t launch_part_build(uint32_t block_bits, uint32_t k, uint32_t bits_per_key, const FilterSet &fs,
                             uint64_t n_rows, const uint64_t *bitmap, const uint64_t *count,
                             const BuildScratch &scratch, const AppendSet &app, uint32_t seg_words,
                             uint32_t *status, hipStream_t s);
// Buckets a partitioned build aims for: its fill kernel runs one workgroup
// per (filter, tile) bucket.
constexpr uint64_t kTargetBuckets = 1024;

// ------------------------------------------------------------ batched steps
//
// A batched launch runs the same step for many tables of many problems. Its
// tasks live in device memory; task i owns workgroups [first[i], first[i+1])
// of the launch (first has n + 1 entries, first[n] = the grid size, then
// one entry per workgroup: the task it belongs to).

// Local predicates of one table (no predicates: every row).
struct LocalTask {
  PredSet ps;
  uint64_t n_rows;
  uint64_t *bitmap;
  uint64_t *count;
  uint32_t seg_words;
  uint32_t pad;
};

// Size one filter from its builder's count and zero its blocks.
struct SizeTask {
  FilterRef f;
  const uint64_t *count;
  uint64_t n_rows;
  uint32_t block_bits;
  uint32_t bits_per_key;
};

// Build up to kMaxProbe filters of one table from its selected rows.
struct BuildTask {
  FilterSet fs;
  uint64_t n_rows;
  const uint64_t *bitmap;
  uint32_t seg_words;
  uint32_t pad;
};

// Probe up to kMaxProbe filters on one table.
struct ProbeTask {
  FilterSet fs;
  uint64_t n_rows;
  uint64_t *bitmap;
  uint64_t *count;
  uint32_t input_all;
  uint32_t pad;
};

struct CopyPair {
  const uint64_t *src;
  uint64_t *dst;
};

constexpr int kBatchThreads = 1024;  // every batched kernel: sixteen waves per workgroup

hipError_t launch_local_batch(const LocalTask *tasks, const uint32_t *first, uint32_t n, uint32_t grid,
                              hipStream_t s);
hipError_t launch_size_batch(const SizeTask *tasks, const uint32_t *first, uint32_t n, uint32_t grid,
                             uint32_t *status, hipStream_t s);
// lds_words: LDS words per workgroup for private filter copies (a task whose
// filters need more inserts with global atomics).
hipError_t launch_build_batch(uint32_t block_bits, uint32_t k, const BuildTask *tasks, const uint32_t *first,
                              uint32_t n, uint32_t grid, uint32_t lds_words, uint32_t *status, hipStream_t s);
// lds_filter_words: LDS words per workgroup for staged filters.
hipError_t launch_probe_batch(uint32_t block_bits, uint32_t k, const ProbeTask *tasks,
                              const uint32_t *first, uint32_t n, uint32_t grid, uint32_t lds_filter_words,
                              uint32_t *status, hipStream_t s);
hipError_t launch_copy_pairs(const CopyPair *pairs, uint32_t n, hipStream_t s);
// Bytes of LDS a probe workgroup needs besides its staged filters.
uint64_t probe_queue_bytes();
// Kernels whose LDS limit must be raised before a batch is captured.
hipError_t prepare_batch_kernels(uint32_t block_bits, uint32_t k);
hipError_t prepare_probe_batch_kernel(uint32_t block_bits, uint32_t k);
hipError_t prepare_build_batch_kernel(uint32_t block_bits, uint32_t k);

}  // namespace pt
