/*
 * pt_oracle.h - plain CPU oracle for the predicate-transfer phase.
 *
 * TEST INFRASTRUCTURE ONLY. This library is the slow, obviously correct
 * reference that the GPU path is checked against. Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg load it. It shares no
 * source, header, table or constant with the GPU library: every value here
 * is written out again from the method's description.
 *
 * Method: Yang, Zhao, Yu, Koutris, "Predicate Transfer: Efficient
 * Pre-Filtering on Multi-Join Queries", CIDR 2024.
 *   Sec. 3.1  two phases; the transfer phase works on the join graph
 *   Sec. 3.2  filter transformation, predicate transfer graph (edges point
 *             from the smaller table to the bigger one), transfer schedule
 *             (forward pass in topological order, then a backward pass on
 *             the reversed edges), filter type (precise filter = semi-join)
 *   Sec. 2.1  Bloom filter: no false negatives, possible false positives
 *   Sec. 3.3  join phase: regular joins on the reduced tables
 *
 * The paper fixes no hash function, filter layout or filter size. This
 * oracle implements the filter specification that the GPU library also
 * implements (independently):
 *   key      x  = the key as a signed 64-bit integer (int32 sign-extended),
 *                 reinterpreted as unsigned
 *   hash     P  = x * 0x9E3779B97F4A7C15 mod 2^64 (multiply-shift,
 *                 Dietzfelbinger et al. 1997); H1 = P >> 32;
 *                 t = (P mod 2^32) xor H1; t = t xor (t >> 16);
 *                 H2 = t * 0x85EBCA6B mod 2^32
 *   size     nb = max(1, ceil(n_keys * bits_per_key / B)) blocks of B bits
 *   block    (H1 * nb) >> 32 (multiply-high range reduction, Lemire 2019)
 *   bits     g1 = H2 >> (32 - b), g2 = ((H2 >> (32 - 2b)) & (B - 1)) | 1,
 *            pos_i = (g1 + i * g2) mod B for i < k (double hashing,
 *            Kirsch and Mitzenmacher 2006), b = log2(B)
 *   words    bit pos of block blk is bit (pos mod 32) of 32-bit word
 *            blk * B/32 + pos/32
 *   bitmap   row r is bit (r mod 64) of 64-bit word r/64; bits past the
 *            last row are zero
 */
#ifndef PT_ORACLE_H
#define PT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define PTOR_OK 0
#define PTOR_EINVAL 1
#define PTOR_ENOMEM 2

/* Predicate operators: a row is kept when value OP lo holds
 * (BETWEEN: lo <= value <= hi). Values are compared as int64. */
#define PTOR_LT 0
#define PTOR_LE 1
#define PTOR_GT 2
#define PTOR_GE 3
#define PTOR_EQ 4
#define PTOR_NE 5
#define PTOR_BETWEEN 6

/* Filter kinds (Sec. 3.2, "Filter Type"). */
#define PTOR_BLOOM 0
#define PTOR_EXACT 1

typedef struct {
  const void *data; /* n_rows values, int32 or int64 */
  uint32_t is64;    /* 0: int32, 1: int64 */
  uint32_t pad;
} ptor_column;

typedef struct {
  uint64_t n_rows;
  uint32_t n_cols;
  uint32_t pad;
  const ptor_column *cols;
} ptor_table;

/* One equi-join u.u_col = v.v_col (an undirected join-graph edge) and its
 * join type (Sec. 3.4): an outer join keeps every row of its preserved
 * side, so a filter may cross the edge only towards the other side. */
#define PTOR_INNER 0
#define PTOR_LEFT_OUTER 1  /* u LEFT JOIN v: filters may go u -> v only */
#define PTOR_RIGHT_OUTER 2 /* u RIGHT JOIN v: v -> u only */
#define PTOR_FULL_OUTER 3  /* no filter crosses the edge */
typedef struct {
  uint32_t u, u_col, v, v_col;
  uint32_t flags;
} ptor_edge;

typedef struct {
  uint32_t table, col, op, pad;
  int64_t lo, hi;
} ptor_pred;

typedef struct {
  uint32_t n_tables, n_edges;
  const ptor_table *tables;
  const ptor_edge *edges;
  const int8_t *orient; /* NULL: smaller-to-bigger rule; else per edge +1 (u->v) or -1 (v->u) */
  const ptor_pred *preds;
  uint32_t n_preds, pad;
} ptor_problem;

typedef struct {
  uint32_t block_bits;   /* B: 32 .. 1024, a power of two */
  uint32_t k;            /* bits set per key, 1 .. 16 */
  uint32_t bits_per_key; /* 1 .. 64 */
  uint32_t kind;         /* PTOR_BLOOM or PTOR_EXACT */
  uint32_t n_passes;     /* 1: forward pass only, 2: forward then backward */
  uint32_t variant;      /* bit 0: visit ready nodes largest id first;
                            bit 1: probe incoming filters in reverse edge order.
                            Neither may change any result. */
  uint32_t threads;      /* threads splitting the row scans (0 or 1: one);
                            each takes whole 64-row bitmap words, Bloom builds
                            fill private copies that are OR-ed together, so
                            the result does not depend on the count */
  uint32_t prune;        /* 1: transfer path pruning (Sec. 3.2 leaves the
                            rule open; this is the reading used here): a
                            non-empty table whose selection still holds
                            every one of its rows builds no filter, and the
                            tables it would have sent one to are not probed
                            with it */
} ptor_params;

/* Optional outputs for inspection. Any pointer may be NULL.
 * filter_words[p * n_edges + e] receives the words of the filter carried by
 * edge e in pass p (p = 0 forward, 1 backward), at most filter_cap[...]
 * words; filter_nb[...] receives its block count (0 in exact mode, and 0
 * for a filter that pruning left unbuilt).
 * fwd_bitmaps[t] receives table t's bitmap after the forward pass and
 * fwd_counts[t] its popcount. edge_src[p * n_edges + e] receives the table
 * that built the filter of edge e in pass p. */
typedef struct {
  uint32_t **filter_words;
  const uint64_t *filter_cap;
  uint64_t *filter_nb;
  uint64_t **fwd_bitmaps;
  uint64_t *fwd_counts;
  uint32_t *edge_src;
} ptor_dump;

/* Hash of one key (the specification above). */
void ptor_hash(int64_t key, uint32_t *h1, uint32_t *h2);

/* Number of blocks for a filter over n_keys keys. */
uint64_t ptor_filter_blocks(uint64_t n_keys, uint32_t bits_per_key, uint32_t block_bits);

/* Block index and the k in-block bit positions of one key. */
void ptor_key_slots(int64_t key, uint64_t nb, uint32_t block_bits, uint32_t k,
                    uint64_t *blk, uint32_t *pos);

void ptor_bloom_insert(uint32_t *words, uint64_t nb, uint32_t block_bits, uint32_t k, int64_t key);
int ptor_bloom_contains(const uint32_t *words, uint64_t nb, uint32_t block_bits, uint32_t k,
                        int64_t key);

/* Bitmap of the rows of one table that satisfy every predicate (their
 * `table` field is ignored); all rows when n_preds == 0. */
int ptor_local_filter(const ptor_table *t, const ptor_pred *preds, uint32_t n_preds,
                      uint64_t *bitmap, uint64_t *count);

/* Build a filter over the keys of the selected rows (bitmap NULL: all rows).
 * The filter is sized from the number of selected rows. */
int ptor_bloom_build(const ptor_column *keys, uint64_t n_rows, const uint64_t *bitmap,
                     uint32_t block_bits, uint32_t k, uint32_t bits_per_key,
                     uint32_t *words, uint64_t cap_words, uint64_t *nb_out);

/* Clear the bitmap bit of every row whose key the filter rejects. */
int ptor_bloom_probe(const ptor_column *keys, uint64_t n_rows, const uint32_t *words,
                     uint64_t nb, uint32_t block_bits, uint32_t k, uint64_t *bitmap,
                     uint64_t *count);

/* Ascending row ids of the set bits. */
int ptor_compact(const uint64_t *bitmap, uint64_t n_rows, uint32_t *idx, uint64_t *count);

/* The whole transfer phase (Sec. 3.2): local filters, orientation,
 * forward pass, backward pass. bitmaps[t] receives table t's final bitmap,
 * counts[t] its popcount. */
int ptor_transfer(const ptor_problem *p, const ptor_params *params, uint64_t *const *bitmaps,
                  uint64_t *counts, const ptor_dump *dump);

/* Join phase (Sec. 3.3): the joins run on the tables as the transfer phase
 * reduced them. Returns every tuple of row ids, one row of each table of
 * root's connected component, whose rows are all selected (bitmaps[t] NULL:
 * every row of t) and whose key columns satisfy every edge between tables of
 * the component (keys compared as int64).
 *   comp     receives the component's tables in ascending index order,
 *            *n_comp their number
 *   out      room for cap tuples of *n_comp ids, row-major: the id of table
 *            comp[c] in tuple j is out[j * n_comp + c]; tuples are sorted
 *            ascending, comparing ids in comp order
 *   n_out    the number of tuples; when it exceeds cap only the first cap
 *            are written */
int ptor_join(const ptor_problem *p, uint32_t root, const uint64_t *const *bitmaps, uint32_t *comp,
              uint32_t *n_comp, uint32_t *out, uint64_t cap, uint64_t *n_out);

#ifdef __cplusplus
}
#endif

#endif
