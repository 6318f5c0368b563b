// pt_internal.hpp - launch descriptors shared by the host API and the kernel
// translation units, and the launchers each of those units exports.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/pt.h"

namespace pt {

constexpr int kWave = 64;

// log2 of a filter's block bits (0 for a size the filter does not allow).
constexpr uint32_t log2_of(int b) {
  return b == 32 ? 5 : b == 64 ? 6 : b == 128 ? 7 : b == 256 ? 8 : b == 512 ? 9 : b == 1024 ? 10 : 0;
}
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
  // Transfer path pruning: a build whose non-empty builder still holds
  // every row (*count == n_rows) builds nothing and records a block count
  // of zero;
  // a probe skips every filter whose block count is zero. The filters of
  // one build set share their builder.
  uint32_t prune;
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

constexpr uint32_t kTileWords = 32768;   // 128 KB of filter per partitioned-build tile (fits LDS)
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
  uint32_t threads;  // per workgroup: kProbeThreads, or fewer for a small table
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
// Partitioned build of filters too large for LDS. Its count kernel sizes
// the filters from *count (the size step); when the plan does not fit the
// scratch it clears them instead, and the scatter inserts in place with
// global atomics.
hipError_t launch_part_build(uint32_t block_bits, uint32_t k, uint32_t bits_per_key, const FilterSet &fs,
                             uint64_t n_rows, const uint64_t *bitmap, const uint64_t *count,
                             const BuildScratch &scratch, const AppendSet &app, uint32_t seg_words,
                             uint32_t *status, hipStream_t s);
// Buckets a partitioned build aims for: its fill kernel runs one workgroup
// per (filter, tile) bucket.
constexpr uint64_t kTargetBuckets = 1024;
// The same for the builds of a batch: few and large tiles, since many builds
// share the device.
constexpr uint32_t kBatchTargetBuckets = 16;

// ---------------------------------------------------------------- batches
//
// A batch of independent transfer problems runs as one persistent kernel
// over a list of tasks: one task is one step of one table of one problem
// (local filter, probe, build, ...), split into work items of one workgroup
// each. A task's phase is its depth in the dependency graph (one more than
// the deepest task it depends on), and the list is ordered by phase.
// Workgroups take items in list order from a device counter; the first
// item a workgroup takes in a phase waits until every item of the previous
// phase has finished (per-phase completion counters), so each task runs
// after all the tasks it depends on.

enum BatchKind : uint32_t {
  kBLocal = 0,  // local predicates of a table (every row when it has none)
  kBProbe,      // probe up to kMaxProbe filters on a table
  kBBuild,      // private LDS copies of a table's outgoing filters (small filters)
  kBReduce,     // OR of those copies into the filters
  kBZero,       // zero filters a partitioned build may fill with atomics
  kBCount,      // partitioned build: bucket histogram of a row tile
  kBScan,       // partitioned build: entry ranges of every (tile, bucket)
  kBScatter,    // partitioned build: entries of a row tile
  kBFill,       // partitioned build: one filter tile per item
  kBCopy,       // final counts to the caller's arrays
  kBShared,     // one scan of a table probed by several problems (shared scan)
};

struct BTask {
  uint32_t kind;        // BatchKind
  uint32_t n_items;     // work items, one workgroup each
  uint32_t first_item;  // global index of item 0
  uint32_t phase;       // depth in the dependency graph
  uint32_t arg;         // index into the argument array of the kind
  uint32_t n_arg;       // kBCopy: number of count pairs
};

struct BLocal {
  PredSet ps;
  uint64_t n_rows;
  uint64_t *bitmap;
  uint64_t *count;
  uint32_t seg_words;
  uint32_t pad;
};

struct BProbe {
  FilterSet fs;
  uint64_t n_rows;
  uint64_t *bitmap;
  uint64_t *count;  // NULL except for the last probe of the table in its pass
  uint32_t k, lg;
};

// The outgoing filters of one table in one pass (at most kMaxFilters),
// with the scratch of whichever build they take.
struct BBuild {
  FilterSet fs;  // keys: the builder's columns
  uint64_t n_rows;
  const uint64_t *bitmap;
  const uint64_t *count;  // the builder's selected rows after this pass's probes
  uint32_t k, lg, bits_per_key, seg_words;
  // LDS build: n_parts private copies of copy_words words each
  uint32_t *copies;
  uint32_t copy_words, n_parts;
  // partitioned build: hist_rows x hist_cols counters, totals, starts, entries
  uint32_t *hist;
  uint32_t hist_cols, hist_rows;
  uint64_t *totals;
  uint64_t *starts;
  uint32_t *entries;
  uint64_t entries_cap;
};

struct CopyPair {
  const uint64_t *src;
  uint64_t *dst;
};

// A shared scan: the probes of several problems over one table of the same
// rows (a resident table that every problem joins). Each row group's keys
// are read once per column of the union (at most four columns) and hashed
// once; every member's filters are then tested on them and every member
// writes its own bitmap.
constexpr int kMaxSharedMembers = 16;
constexpr int kMaxSharedCols = 4;
constexpr uint64_t kSharedMinRows = 1ull << 20;  // smaller tables are probed one problem at a time
struct BShared {
  uint64_t n_rows;
  uint32_t n_members;
  uint32_t n_cols;
  uint32_t first_probe;  // members: probes[first_probe, first_probe + n_members)
  uint32_t pad;
  const void *cols[kMaxSharedCols];
  uint32_t key64[kMaxSharedCols];
  uint8_t col_of[kMaxSharedMembers][kMaxProbe];  // member m's filter j reads cols[col_of[m][j]]
};

struct BatchArgs {
  const BTask *tasks;
  const uint32_t *item_task;    // task of every item
  const uint32_t *phase_items;  // items of every phase
  const BLocal *locals;
  const BProbe *probes;
  const BBuild *builds;
  const CopyPair *pairs;
  const BShared *shared;
  uint32_t *head;        // next item to take
  uint32_t *phase_done;  // finished items of every phase
  uint32_t *status;      // the batch's status word
  uint32_t n_items;
  uint32_t n_phases;
  uint32_t lds_filter_words;  // probe: LDS words for staged filters
  uint32_t lds_bytes;         // dynamic LDS of a workgroup
  uint64_t spin_limit;        // longest wait for a phase, in wall-clock ticks
  uint64_t *timeline;         // NULL, or the start and end (wall clock) of every item
};

constexpr int kBatchThreads = 1024;    // the batch kernel: sixteen waves per workgroup
constexpr uint32_t kReduceWords = 16384;   // filter words one reduce item of a batch covers
constexpr uint32_t kZeroWords = 1u << 20;  // filter words one zero item covers (usually it has nothing to do)

// k_batch*.hip: the persistent kernel for B = 512 and k = 3 or 2, or generic.
// grid: workgroups (all resident); lds_bytes: dynamic LDS per workgroup.
hipError_t launch_batch_512_k3(const BatchArgs &a, uint32_t grid, uint64_t lds_bytes, hipStream_t s);
hipError_t launch_batch_512_k2(const BatchArgs &a, uint32_t grid, uint64_t lds_bytes, hipStream_t s);
hipError_t launch_batch_generic(const BatchArgs &a, uint32_t grid, uint64_t lds_bytes, hipStream_t s);
// Raise the batch kernels' LDS limit (before a capture).
hipError_t prepare_batch_kernels();
hipError_t prepare_batch_512();
// Bytes of LDS a probe workgroup needs besides its staged filters.
uint64_t probe_queue_bytes();

// ---------------------------------------------------------- exact filters
// (k_exact.hip) The precise filter of Sec. 3.2: the distinct keys of the
// builder's selected rows in a device hash table.
struct SetRef {
  unsigned long long *keys;  // 2^lg_cap slots, then one word: INT64_MIN present
  uint64_t *lg;              // device: log2 of the slots in use (set by the build)
  const void *col;           // key column of the table the launch scans
  uint32_t key64;
  uint32_t lg_cap;
};
struct SetProbe {
  uint32_t n;
  uint32_t pad;
  SetRef f[kMaxProbe];
};
// Sizes the set from *count (n_rows when NULL), clears it, and inserts the
// keys of f.col's selected rows (bitmap NULL: every row). With prune, a
// non-empty builder that still holds every row (*count == n_rows) builds
// nothing and the set's *lg is 0 (a pruned set).
hipError_t launch_set_build(const SetRef &f, uint64_t n_rows, const uint64_t *bitmap, const uint64_t *count,
                            bool prune, hipStream_t s);
// Clears the bitmap bit of every row whose key misses one of the sets
// (input_all: the bitmap is not read, every row starts selected); adds the
// rows left to *count (NULL: not counted). A pruned set (*lg == 0) lets
// every key through.
hipError_t launch_set_probe(const SetProbe &sp, uint64_t n_rows, uint64_t *bitmap, uint64_t *count, bool input_all,
                            hipStream_t s);

// ---------------------------------------------------------- join phase
// (k_join.hip) Hash joins on the reduced tables: each table added to the
// join gets a hash table over its selected rows; the tuples built so far
// probe it and are extended by every match.

constexpr uint32_t kMaxJoinWidth = 32;  // tables in one join
constexpr uint32_t kMaxJoinChecks = 8;  // edges checked per added table besides the lookup edge
constexpr uint32_t kJoinNone = 0xFFFFFFFFu;

// Hash table of one table's selected rows: open addressing on the keys,
// each key's rows chained through `next`. Its used size follows the number
// of selected rows (twice that, rounded up to a power of two, at least 64,
// at most the capacity 2^lg_cap).
struct JoinHash {
  unsigned long long *keys;  // 2^lg_cap + 1 slots; the last one belongs to kJoinEmptyKey
  uint32_t *heads;           // 2^lg_cap + 1: first entry of the slot's chain, kJoinNone if none
  uint32_t *next;            // one per selected row: next entry with the same key, kJoinNone at the end
  const uint32_t *ids;       // the table's selected row ids
  const uint64_t *count;     // their number
  const void *key;           // the key column the table is looked up by
  uint32_t key64;
  uint32_t lg_cap;
  uint64_t n_rows;           // the table's rows (bounds *count and next[])
};

// One more edge between the added table and a table already joined.
struct JoinCheck {
  const void *v_col;  // the added table's column
  const void *p_col;  // the joined table's column
  uint32_t v64, p64;
  uint32_t pos;  // the joined table's place in the tuples
  uint32_t pad;
};

// One join step: tuples of `width` row ids (columns in[0..width)) probe the
// hash table of the added table by the key of the joined table at place
// u_pos; every match that passes the checks becomes a tuple of width + 1
// ids in out[0..width] (the added table's id last).
struct JoinStep {
  JoinHash h;
  const void *u_key;
  uint32_t u64;
  uint32_t u_pos;
  uint32_t width;
  uint32_t n_checks;
  JoinCheck checks[kMaxJoinChecks];
  const uint32_t *in[kMaxJoinWidth];
  uint32_t *out[kMaxJoinWidth];
  const uint64_t *n_in;  // tuples in (at most in_cap are read)
  uint64_t *n_out;       // tuples produced (only the first cap are written)
  uint64_t in_cap;
  uint64_t cap;
  uint32_t *status;
};

constexpr unsigned long long kJoinEmptyKey = 0x8000000000000000ull;  // INT64_MIN marks a free slot

hipError_t launch_join_ids(const uint64_t *bitmap, uint64_t n_rows, uint32_t *ids, uint64_t *count,
                           uint64_t *partials, hipStream_t s);
hipError_t launch_join_build(const JoinHash &h, hipStream_t s);
hipError_t launch_join_step(const JoinStep &st, hipStream_t s);
// *n_out = the largest of step_counts[0..n_steps) and *n_out when one of
// step_counts exceeds cap (an intermediate step overflowed).
hipError_t launch_join_finish(const uint64_t *step_counts, uint32_t n_steps, uint64_t cap, uint64_t *n_out,
                              hipStream_t s);
// dst[i] = src[i] for i < min(*n, cap); *n_out = *n (a one-table join).
hipError_t launch_join_copy(const uint32_t *src, const uint64_t *n, uint64_t cap, uint32_t *dst, uint64_t *n_out,
                            uint32_t *status, hipStream_t s);

}  // namespace pt
