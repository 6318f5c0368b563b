/*
 * pt.h - C ABI of the MI355X (gfx950) predicate-transfer library, libpt_hip.so.
 *
 * Predicate transfer (Yang, Zhao, Yu, Koutris, "Predicate Transfer: Efficient
 * Pre-Filtering on Multi-Join Queries", CIDR 2024) pre-filters every table of
 * a multi-join query before any join runs:
 *   - Sec. 3.1: the query is a join graph, one vertex per table and one edge
 *     per equi-join; phase 1 transfers filters along it, phase 2 joins.
 *   - Sec. 3.2: local predicates become filters; at each table a single scan
 *     of its join-key columns probes every incoming filter and inserts the
 *     surviving rows' keys into every outgoing filter ("filter
 *     transformation"); edges point from the smaller table to the bigger one
 *     ("predicate transfer graph"); a forward pass visits tables in
 *     topological order, then a backward pass repeats it on the reversed
 *     edges ("transfer schedule").
 *   - Sec. 2.1: the filters are Bloom filters (no false negatives).
 *
 * Every table ends with a selection bitmap; the join phase reads the rows
 * whose bits are set.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.   Pointers named d_* and every column's data are device pointers
 *           (HIP device memory on the current device). Everything else is
 *           host memory, read during the call only. The caller allocates and
 *           owns every buffer and keeps device buffers alive until the work
 *           queued on `stream` has finished. No call allocates device
 *           memory: scratch space is the caller's workspace argument (and
 *           for pt_compact_noalloc, an array the library holds per GPU).
 * Streams.  Work is queued on `stream` (a hipStream_t; NULL is the null
 *           stream) and the call returns without waiting for it.
 * Errors.   Arguments are checked on the host first. A rejected call returns
 *           PT_EINVAL and queues nothing. A failed launch returns
 *           PT_EDEVICE. pt_last_error() gives the calling thread's message
 *           for its last failed call. Nothing is thrown across this ABI.
 * Rows.     A table has fewer than 2^32 rows. Row ids are uint32.
 * Keys.     Columns hold int32 or int64 values. A key is compared as a
 *           signed 64-bit integer, so an int32 column may join an int64 one.
 * Bitmaps.  One bit per row, in uint64 words: row r is bit (r mod 64) of
 *           word r / 64, ceil(n_rows / 64) words. Bits past the last row are
 *           zero on output and must be zero on input.
 *
 * Filter specification (the paper fixes no hash, layout or size; the same
 * rules are implemented independently by the CPU oracle in the tests)
 * -----------------------------------------------------------------------
 *   x   = the key as int64, reinterpreted as uint64
 *   P   = x * 0x9E3779B97F4A7C15 mod 2^64        (multiply-shift hashing)
 *   H1  = P >> 32
 *   t   = (P mod 2^32) xor H1;  t = t xor (t >> 16)
 *   H2  = t * 0x85EBCA6B mod 2^32
 *   B   = block_bits (32..1024, a power of two; 512 = one 64-byte line),
 *         b = log2(B), k = bits per key (1..16)
 *   nb  = max(1, ceil(n_selected * bits_per_key / B)) blocks, nb < 2^32
 *   blk = (H1 * nb) >> 32                        (multiply-high reduction)
 *   g1  = H2 >> (32 - b);  g2 = ((H2 >> (32 - 2b)) mod B) | 1
 *   bit i (i < k) of the key: pos_i = (g1 + i * g2) mod B in block blk,
 *         i.e. bit (pos_i mod 32) of uint32 word blk * B/32 + pos_i / 32
 *   A key is inserted by setting its k bits and passes when all k are set.
 */
#ifndef PT_H
#define PT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pt_status {
  PT_OK = 0,
  PT_EINVAL = 1,       /* an argument was rejected; nothing was queued */
  PT_ENOMEM = 2,       /* a caller-provided workspace is too small */
  PT_EDEVICE = 3,      /* a HIP call or kernel launch failed */
  PT_EUNSUPPORTED = 4, /* a valid request this library does not implement */
  PT_EOVERFLOW = 5     /* pt_check_status: a kernel found a size above a capacity */
} pt_status;

/* Device status word. Kernels OR these bits into a call's status word (a
 * device uint32) when a size read on the device exceeds the room the host
 * set aside; the kernel then clamps and carries on, so nothing is written
 * out of bounds, but the result no longer follows the filter specification.
 * The checks on the host make both impossible inside pt_transfer and the
 * batches; they catch wrong counts or block counts handed to the primitives.
 *   FILTER_OVERFLOW   a filter needed more blocks than cap_words holds, or a
 *                     block count read from d_nb exceeded it (clamped)
 *   ENTRIES_OVERFLOW  a partitioned build met more keys than its count
 *                     said (the extra keys were not inserted)
 * pt_check_status() reads and clears the word. */
#define PT_STATUS_FILTER_OVERFLOW 1u
#define PT_STATUS_ENTRIES_OVERFLOW 2u
/*   WAIT_TIMEOUT      a batch's work item waited longer than its limit for
 *                     the steps it depends on and ran without them (the
 *                     batch's results are then not to be trusted) */
#define PT_STATUS_WAIT_TIMEOUT 4u
/*   JOIN_OVERFLOW     a join produced more tuples than the caller's out_cap
 *                     (pt_join: the tuples are incomplete) */
#define PT_STATUS_JOIN_OVERFLOW 8u

typedef enum pt_dtype { PT_I32 = 0, PT_I64 = 1 } pt_dtype;

/* A hipStream_t. */
typedef void *pt_stream;

/* One column: n_rows values of `dtype` at device address `data` (may be NULL
 * when the table has no rows). */
typedef struct pt_column {
  const void *data;
  uint32_t dtype;    /* pt_dtype */
  uint32_t reserved; /* 0 */
} pt_column;

/* One base table (a vertex of the join graph; the same base table joined
 * twice appears as two vertices). */
typedef struct pt_table {
  uint64_t n_rows;
  uint32_t n_cols;
  uint32_t reserved; /* 0 */
  const pt_column *cols;
} pt_table;

/* One equi-join tables[u].cols[u_col] = tables[v].cols[v_col] (Sec. 3.1).
 * A composite key is several edges between the same tables. flags is the
 * join type (Sec. 3.4): PT_EDGE_INNER, or an outer join, which keeps every
 * row of its preserved side, so no filter may reduce that side through this
 * edge: tables[u] LEFT JOIN tables[v] transfers only u -> v (in whichever
 * pass the edge runs that way), RIGHT only v -> u, FULL not at all. Other
 * values are rejected with PT_EUNSUPPORTED. pt_transfer handles every type;
 * pt_join only inner joins. */
typedef struct pt_edge {
  uint32_t u, u_col, v, v_col;
  uint32_t flags;
} pt_edge;

#define PT_EDGE_INNER 0u
#define PT_EDGE_LEFT_OUTER 1u
#define PT_EDGE_RIGHT_OUTER 2u
#define PT_EDGE_FULL_OUTER 3u

/* The join graph. `orient` is NULL for the paper's rule (Sec. 3.2: each edge
 * points from the table with fewer rows to the one with more; equal sizes
 * point from the lower table index), or one value per edge: +1 for u -> v,
 * -1 for v -> u. The oriented graph must be acyclic. */
typedef struct pt_graph {
  uint32_t n_tables;
  uint32_t n_edges;
  const pt_edge *edges;
  const int8_t *orient;
} pt_graph;

typedef enum pt_cmp {
  PT_LT = 0, PT_LE = 1, PT_GT = 2, PT_GE = 3, PT_EQ = 4, PT_NE = 5,
  PT_BETWEEN = 6 /* lo <= value <= hi */
} pt_cmp;

/* A local predicate "tables[table].cols[col] op lo" (Sec. 3.4: filters over
 * base tables). The predicates of one table form a conjunction; values and
 * bounds compare as int64. */
typedef struct pt_pred {
  uint32_t table, col;
  uint32_t op;       /* pt_cmp */
  uint32_t reserved; /* 0 */
  int64_t lo, hi;
} pt_pred;

/* Filter parameters, one set for every filter of a call. The first three
 * fix the filter bits (with the hash version); the rest only change how the
 * work is laid out on the device, never a bit of any result.
 *   hash_version  0 or 1: the filter specification above; other
 *                 values are rejected with PT_EUNSUPPORTED
 *   lds_budget    bytes of LDS a probe workgroup may stage filters in
 *                 (0: as much as the device allows); filters that do not
 *                 fit together are read from global memory
 *   tile_rows     rows one workgroup of a batch takes per work item: 0 for
 *                 65 536, else a multiple of 4 096 up to 2^24
 *   probe_order   PT_PROBE_SELECTIVE (0): the filter whose builder kept the
 *                 smallest share of its rows is tested first;
 *                 PT_PROBE_GIVEN (1): in edge order */
typedef struct pt_params {
  uint32_t block_bits;   /* B: 32, 64, 128, 256, 512 or 1024 */
  uint32_t k;            /* 1..16 */
  uint32_t bits_per_key; /* 1..64 */
  uint32_t flags;        /* PT_FLAG_* bits */
  uint32_t hash_version;
  uint32_t lds_budget;
  uint32_t tile_rows;
  uint32_t probe_order;
} pt_params;

#define PT_PROBE_SELECTIVE 0u
#define PT_PROBE_GIVEN 1u

/* pt_transfer normally appends the keys of a probe's surviving rows while it
 * scans the table, so that the filters the table then builds read those keys
 * instead of scanning it a second time (Sec. 3.2: the transformation scans
 * a table once). With this flag the builds scan the table's selected rows
 * again and the workspace holds no appended keys. The bits are the same. */
#define PT_FLAG_NO_APPEND 1u

/* In a batch, the probes of problems with this flag that scan tables of the
 * same rows through the same key columns (a resident table they all join)
 * are grouped into shared scans (at most 16 problems and 4 key columns per
 * group): one pass over the table reads each key column once and tests the
 * filters of every grouped problem whose filters fit in LDS with the
 * others', each problem keeping its own bitmap; the other problems of the
 * group are probed one after the other on the same rows. The bits are the
 * same either way. It pays when the key reads dominate (small filters); when
 * filters are read from global memory the separate probes are faster. */
#define PT_FLAG_SHARED_SCAN 2u

/* pt_transfer with precise filters instead of Bloom filters (Sec. 3.2,
 * "Filter Type"): every filter is the set of distinct keys of its builder's
 * selected rows, so each transfer is a semi-join and the reduced tables
 * hold no false positives (Sec. 2.2: with every edge towards one root the
 * two passes are the semi-join phase of Yannakakis). The sets are hash
 * tables in the workspace (16 bytes per builder row at most, sized on the
 * device from the selected rows); block_bits, k and bits_per_key are
 * checked but unused. pt_bloom_*, pt_transfer_filter and batches reject
 * this flag with PT_EUNSUPPORTED. */
#define PT_FLAG_EXACT 4u

/* Transfer path pruning (Sec. 3.2, "Transfer Path Pruning": the paper asks
 * for skipping transfers that cannot make a filter more selective and leaves
 * the rule open). The rule implemented: a non-empty table whose selection
 * still holds every one of its rows sends no filter (such a filter can only
 * remove rows whose key appears nowhere in the whole table), and the tables
 * it would have sent one to are not probed with it. The decision is taken from the
 * exact counts: on the host when the table has no predicate and has not
 * been probed yet (nothing is launched for its filters), otherwise on the
 * device by the build's size step. Every row that joins is still kept, so
 * the join result is the same; with exact filters the reduced tables hold a
 * superset of the rows the full schedule keeps. A pruned filter is left
 * with a block count of zero. Works with PT_FLAG_EXACT and in batches (a
 * problem with this flag takes no part in shared scans). */
#define PT_FLAG_PRUNE 8u

/* A Bloom filter in device memory. `words` holds cap_words uint32 words; the
 * filter in use is its first nb * B/32 words, where nb is the uint64 at
 * device address `d_nb` (written by pt_bloom_build). `d_status` is NULL or
 * a device uint32 status word (PT_STATUS_* bits) that builds and probes of
 * this filter report into; pt_check_status reads it. */
typedef struct pt_bloom {
  uint32_t *words;
  uint64_t cap_words;
  uint64_t *d_nb;
  uint32_t *d_status;
  pt_params params;
} pt_bloom;

/* Per-kernel timing record (see pt_profile_enable). */
typedef struct pt_kernel_time {
  char name[24];   /* "local", "probe", "size", "build", "count", "compact", "batch probe" */
  uint32_t table;  /* table index inside pt_transfer, else 0 */
  uint32_t pass;   /* 0 local, 1 forward, 2 backward; 0 outside pt_transfer */
  uint64_t rows;   /* rows the kernel scanned */
  uint64_t bytes;  /* algorithmic bytes: key and bitmap traffic the step must move */
  float ms;        /* duration between events recorded around the launch */
  uint32_t reserved;
} pt_kernel_time;

/* Library version string. */
const char *pt_version(void);

/* Waits for `stream`, then reads and clears the device status word
 * d_status: a pt_bloom's d_status, or the workspace of pt_transfer or of a
 * batch (its first 4 bytes hold the status of the latest call on it, see
 * the PT_STATUS_* bits above). Returns PT_OK when no bit is set,
 * PT_EOVERFLOW otherwise (pt_last_error names the bits), PT_EINVAL for a
 * NULL pointer, PT_EDEVICE if the copy fails. The paper's schedule ends
 * with every table reduced (Sec. 3.2); this call tells whether the reduced
 * tables are the ones the specification defines. */
pt_status pt_check_status(const void *d_status, pt_stream stream);

/* Message of the calling thread's last failed call ("" if none). */
const char *pt_last_error(void);

/* Local filter (Sec. 3.2, inherent filters applied during the scan; Sec.
 * 3.4). Writes into d_bitmap the rows of `table` that satisfy every one of
 * the n_preds predicates (their `table` field is ignored; all rows if
 * n_preds == 0), and if d_count is not NULL their number into *d_count.
 * d_bitmap: ceil(n_rows/64) words, fully overwritten. */
pt_status pt_local_filter(const pt_table *table, const pt_pred *preds, uint32_t n_preds,
                          uint64_t *d_bitmap, uint64_t *d_count, pt_stream stream);

/* Words a filter needs to hold up to max_keys keys (its cap_words). */
pt_status pt_bloom_capacity(uint64_t max_keys, const pt_params *params, uint64_t *out_words);

/* Bloom build (Sec. 2.1; Sec. 3.2, the outgoing half of the filter
 * transformation). For each of the n_filters filters, sizes it from the
 * number of selected rows (nb above), zeroes its nb blocks, writes nb to
 * *filters[i].d_nb, and inserts keys[i] of every selected row.
 *   keys[i]    key column of this table for filter i (n_rows values)
 *   d_bitmap   selected rows; NULL selects all n_rows rows
 *   d_count    device uint64 holding the number of selected rows (the
 *              popcount of d_bitmap); required when d_bitmap is not NULL
 *   filters[i] cap_words must hold a filter over n_rows keys
 *              (pt_bloom_capacity); all filters share one pt_params value
 * The filters' words must not overlap each other or the inputs. */
pt_status pt_bloom_build(uint32_t n_filters, const pt_column *keys, const pt_bloom *filters,
                         uint64_t n_rows, const uint64_t *d_bitmap, const uint64_t *d_count,
                         pt_stream stream);

/* Bloom probe (Sec. 3.2, the incoming half of the filter transformation).
 * Clears in d_bitmap the bit of every row whose keys[i] fails filters[i],
 * for every i, in one scan of the table; rows already cleared stay cleared.
 * If d_count is not NULL, writes the number of rows left. The order in
 * which the filters are tested does not change the result. */
pt_status pt_bloom_probe(uint32_t n_filters, const pt_column *keys, const pt_bloom *filters,
                         uint64_t n_rows, uint64_t *d_bitmap, uint64_t *d_count,
                         pt_stream stream);

/* Bytes of workspace pt_compact needs for n_rows rows. */
pt_status pt_compact_workspace_size(uint64_t n_rows, size_t *bytes);

/* Compaction: the ids of the set rows of d_bitmap in ascending order into
 * d_idx (room for n_rows ids) and their number into *d_count: the
 * pre-filtered row set handed to the join phase (Sec. 3.3). */
pt_status pt_compact(const uint64_t *d_bitmap, uint64_t n_rows, uint32_t *d_idx,
                     uint64_t *d_count, void *d_ws, size_t ws_bytes, pt_stream stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * compaction as pt_compact, with the same results, but without a workspace.
 * Its partial counts live in a static device array of the library (256 KiB
 * per GPU, held until the process ends), so n_rows is at most 2^31; larger
 * inputs are rejected with PT_EINVAL before anything is queued. It allocates
 * nothing: the array's address is looked up once per device, on the first
 * call there. Every call on one GPU shares that array, so calls that overlap
 * on a GPU (on different streams, or from different threads) race; order
 * them on one stream. */
pt_status pt_compact_noalloc(const uint64_t *d_bitmap, uint64_t n_rows, uint32_t *d_idx,
                             uint64_t *d_count, pt_stream stream);

/* Bytes of workspace pt_transfer needs for this graph, these tables' row
 * counts and these parameters (every filter at its largest possible size,
 * plus counters). */
pt_status pt_transfer_workspace_size(const pt_graph *graph, const pt_table *tables,
                                     const pt_params *params, size_t *bytes);

/* The transfer phase (Sec. 3.2): local predicates, orientation, the forward
 * pass in topological order, then the backward pass on the reversed edges
 * starting from the forward survivors. Without PT_FLAG_PRUNE every edge
 * carries one filter in each pass, and every source of a pass builds its
 * filters whether or not it has a predicate. A filter is sized from the
 * builder's row count after that pass's probes at the builder.
 *   tables     graph->n_tables tables (at most 64)
 *   preds      n_preds predicates, each naming its table
 *   d_ws       workspace of at least pt_transfer_workspace_size bytes,
 *              256-byte aligned; holds every filter after the call
 *   d_bitmaps  d_bitmaps[t] receives table t's final bitmap
 *   d_counts   NULL, or graph->n_tables device uint64: final row counts */
pt_status pt_transfer(const pt_graph *graph, const pt_table *tables, const pt_pred *preds,
                      uint32_t n_preds, const pt_params *params, void *d_ws, size_t ws_bytes,
                      uint64_t *const *d_bitmaps, uint64_t *d_counts, pt_stream stream);

/* Bytes of workspace pt_join needs for the component of `root` in this
 * graph, these tables' row counts and out_cap tuples. */
pt_status pt_join_workspace_size(const pt_graph *graph, const pt_table *tables, uint32_t root,
                                 uint64_t out_cap, size_t *bytes);

/* The join phase (Sec. 3.3): the joins of the query run on the tables as
 * the transfer phase reduced them. Produces every tuple of row ids, one row
 * of each table of root's connected component, whose rows are all selected
 * and whose key columns agree on every edge between tables of the
 * component (keys compared as int64 values). The root is the table the
 * join starts from: the other tables are added one at a time in
 * breadth-first order from it, each through a hash table over its selected
 * rows that the tuples so far probe, so the root is best the largest table
 * (the tables added are the build sides).
 *   d_bitmaps  NULL (every row of every table selected), or graph->n_tables
 *              device pointers: d_bitmaps[t] selects table t's rows (the
 *              bitmaps pt_transfer wrote), NULL for every row of t
 *   d_out      graph->n_tables pointers; for each table t of the component,
 *              d_out[t] has room for out_cap uint32 row ids (others unused)
 *   out_cap    tuples that fit in the d_out columns (and in the workspace's
 *              intermediate tuples)
 *   d_n_out    device uint64: the number of tuples (see overflow below)
 *   d_ws       workspace of at least pt_join_workspace_size bytes, 256-byte
 *              aligned; its first 4 bytes are the call's status word
 * Tuple i is (d_out[t][i] for t in the component). The tuples come out in
 * no particular order (their set is fixed, their order depends on
 * scheduling). When a step produces more than out_cap tuples, only out_cap
 * of them are kept, PT_STATUS_JOIN_OVERFLOW is set in the status word
 * (pt_check_status on d_ws), the result is incomplete and *d_n_out holds
 * the largest number of tuples a step reached (more than out_cap): call
 * again with at least that out_cap (a later step may then need more). Edges with flags other than 0 are rejected with
 * PT_EUNSUPPORTED, as are components of more than 32 tables or a table with
 * more than 9 edges to the tables added before it. */
pt_status pt_join(const pt_graph *graph, const pt_table *tables, uint32_t root,
                  const uint64_t *const *d_bitmaps, uint32_t *const *d_out, uint64_t out_cap,
                  uint64_t *d_n_out, void *d_ws, size_t ws_bytes, pt_stream stream);

/* Where pt_transfer left the filter that `edge` carried in `pass` (1 forward,
 * 2 backward) inside d_ws, and which table built it (*builder); PT_EINVAL
 * when an outer join kept the edge from carrying one in that pass. With
 * PT_FLAG_PRUNE, a filter that pruning left unbuilt has *d_nb == 0. */
pt_status pt_transfer_filter(const pt_graph *graph, const pt_table *tables,
                             const pt_params *params, void *d_ws, uint32_t pass, uint32_t edge,
                             pt_bloom *out, uint32_t *builder);

/* ---------------------------------------------------------------- batches
 *
 * Many independent transfer problems run together (the paper evaluates one
 * query at a time and names parallel execution as future work, Sec. 5).
 * Every step of every problem becomes a task of work items, ordered by its
 * depth in the problems' dependency graphs; one persistent kernel launch
 * takes the items from a device queue and synchronises phase by phase, so
 * the bits equal those of pt_transfer on each problem. A run (a zeroing
 * kernel and the batch kernel) is captured once into a HIP graph that each
 * later run launches with a single call. */

/* One problem of a batch: the arguments of pt_transfer. */
typedef struct pt_problem {
  const pt_graph *graph;
  const pt_table *tables;
  const pt_pred *preds;
  uint32_t n_preds;
  uint32_t reserved;          /* 0 */
  pt_params params;           /* each problem may use its own parameters */
  uint64_t *const *d_bitmaps; /* d_bitmaps[t]: table t's final bitmap */
  uint64_t *d_counts;         /* NULL, or n_tables device uint64 */
} pt_problem;

/* A prepared batch (host object). */
typedef struct pt_batch pt_batch;

/* Bytes of workspace a batch of these problems needs (every filter of both
 * passes of every problem at its largest size, counters and task tables). */
pt_status pt_batch_workspace_size(uint32_t n_problems, const pt_problem *problems, size_t *bytes);

/* Plans the batch: checks every problem as pt_transfer does, writes the
 * task tables of every launch into d_ws (256-byte aligned, at least
 * pt_batch_workspace_size bytes) and returns a handle in *out. Blocking (it
 * copies the tables and synchronizes the device); call it once, then run
 * the batch as often as wanted. The problems' device buffers (columns,
 * bitmaps, counts) and d_ws must stay valid until pt_batch_free. Host
 * arrays in `problems` are only read during this call. */
pt_status pt_batch_prepare(uint32_t n_problems, const pt_problem *problems, void *d_ws,
                           size_t ws_bytes, pt_batch **out);

/* As pt_batch_prepare, but the task tables are copied asynchronously on
 * `stream` (from a host buffer the handle keeps); runs must be ordered after
 * that copy (same stream, or synchronized with it). */
pt_status pt_batch_prepare_async(uint32_t n_problems, const pt_problem *problems, void *d_ws,
                                 size_t ws_bytes, pt_stream stream, pt_batch **out);

/* Runs the batch on `stream`: every problem's bitmaps and counts are
 * written as pt_transfer would write them. flags = 0 launches the captured
 * graph (captured on the first run); PT_BATCH_EAGER enqueues the kernels one
 * by one instead. Runs of one batch on overlapping streams race. */
#define PT_BATCH_EAGER 1u
pt_status pt_batch_run(pt_batch *batch, pt_stream stream, uint32_t flags);

/* Kernel launches in one run of the batch, and rows it probes (the sum
 * over probe steps of the probed table's rows). */
pt_status pt_batch_info(const pt_batch *batch, uint32_t *n_launches, uint64_t *rows_probed);

/* Profiling of a batch prepared while the environment variable
 * PT_BATCH_TIMELINE is 1 (the workspace size query must see it too): after
 * a run, waits for the device and copies up to max_items records of four
 * uint64 each - the item's start and end on the device's wall clock, its
 * task kind and its phase - into `out`, sets *n_items, and the clock's ticks
 * per millisecond into *ticks_per_ms (may be NULL). PT_EUNSUPPORTED for a
 * batch prepared without it. */
pt_status pt_batch_timeline(const pt_batch *batch, uint64_t *out, uint32_t max_items, uint32_t *n_items,
                            uint32_t *ticks_per_ms);

/* Frees the handle and its graph (after the last run has completed). */
void pt_batch_free(pt_batch *batch);

/* Convenience: prepare, run eagerly on `stream`, wait, free. */
pt_status pt_transfer_batch(uint32_t n_problems, const pt_problem *problems, void *d_ws, size_t ws_bytes,
                            pt_stream stream);

/* Kernel timing. While enabled on the calling thread (on = 1: every launch
 * of the calls above; on = 2: probe launches only; 0: off), each launch is
 * bracketed by HIP events recorded on the launch's own stream.
 * pt_profile_read waits for those events, copies up to `max` records into
 * `out`, sets *n to the number copied and clears the list.
 * pt_profile_only narrows recording on the calling thread to the launches
 * whose record would carry this name (compared as stored, at most 23
 * characters), table and pass, so that a timed loop brackets one kernel
 * and leaves the others' launches back to back; NULL or "" records every
 * launch the mode selects again. */
pt_status pt_profile_enable(int on);
pt_status pt_profile_only(const char *name, uint32_t table, uint32_t pass);
pt_status pt_profile_read(pt_kernel_time *out, uint32_t max, uint32_t *n);

#ifdef __cplusplus
}
#endif

#endif /* PT_H */
