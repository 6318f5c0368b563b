/*
 * pt_oracle.c - plain CPU oracle for the predicate-transfer phase.
 *
 * TEST INFRASTRUCTURE ONLY (see pt_oracle.h). Written for reading, not for
 * speed: one row at a time, one filter at a time, in the order the paper
 * describes the steps (Sec. 3.2). The transfer's row scans can optionally be
 * split over threads by whole bitmap words (params.threads), which changes
 * no result: probes and predicates touch only their own rows' bits, and a
 * Bloom filter is the OR of the copies built from disjoint rows.
 */
#include "pt_oracle.h"

#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Filter specification (the paper leaves hash and layout open; Sec. 4.1
 * only says the prototype reused an existing library's Bloom filter).  */
/* ------------------------------------------------------------------ */

static const uint64_t HASH_MULTIPLIER = 0x9E3779B97F4A7C15ULL;
static const uint32_t MIX_MULTIPLIER = 0x85EBCA6BU;

void ptor_hash(int64_t key, uint32_t *h1, uint32_t *h2) {
  uint64_t x = (uint64_t)key;         /* int32 keys arrive already sign-extended */
  uint64_t p = x * HASH_MULTIPLIER;   /* arithmetic mod 2^64 */
  uint32_t hi = (uint32_t)(p >> 32);
  uint32_t lo = (uint32_t)(p & 0xFFFFFFFFULL);
  uint32_t t = lo ^ hi;               /* the low word alone never sees the key's high word */
  t = t ^ (t >> 16);
  *h1 = hi;
  *h2 = t * MIX_MULTIPLIER;           /* arithmetic mod 2^32 */
}

static uint32_t log2_exact(uint32_t v) {
  uint32_t b = 0;
  while ((1u << b) < v) b++;
  return b;
}

uint64_t ptor_filter_blocks(uint64_t n_keys, uint32_t bits_per_key, uint32_t block_bits) {
  uint64_t bits = n_keys * (uint64_t)bits_per_key;
  uint64_t nb = (bits + block_bits - 1) / block_bits;
  if (nb == 0) nb = 1;
  return nb;
}

void ptor_key_slots(int64_t key, uint64_t nb, uint32_t block_bits, uint32_t k, uint64_t *blk,
                    uint32_t *pos) {
  uint32_t h1, h2;
  ptor_hash(key, &h1, &h2);
  uint32_t b = log2_exact(block_bits);
  *blk = ((uint64_t)h1 * nb) >> 32;
  uint32_t g1 = h2 >> (32 - b);
  uint32_t g2 = ((h2 >> (32 - 2 * b)) & (block_bits - 1)) | 1u;
  for (uint32_t i = 0; i < k; i++) pos[i] = (g1 + i * g2) & (block_bits - 1);
}

void ptor_bloom_insert(uint32_t *words, uint64_t nb, uint32_t block_bits, uint32_t k, int64_t key) {
  uint64_t blk;
  uint32_t pos[16];
  ptor_key_slots(key, nb, block_bits, k, &blk, pos);
  uint64_t words_per_block = block_bits / 32;
  for (uint32_t i = 0; i < k; i++) {
    uint64_t w = blk * words_per_block + pos[i] / 32;
    words[w] |= 1u << (pos[i] % 32);
  }
}

int ptor_bloom_contains(const uint32_t *words, uint64_t nb, uint32_t block_bits, uint32_t k,
                        int64_t key) {
  uint64_t blk;
  uint32_t pos[16];
  ptor_key_slots(key, nb, block_bits, k, &blk, pos);
  uint64_t words_per_block = block_bits / 32;
  for (uint32_t i = 0; i < k; i++) {
    uint64_t w = blk * words_per_block + pos[i] / 32;
    if (((words[w] >> (pos[i] % 32)) & 1u) == 0) return 0;
  }
  return 1;
}

/* ------------------------------------------------------------------ */
/* Columns, bitmaps, predicates                                         */
/* ------------------------------------------------------------------ */

static int64_t column_value(const ptor_column *c, uint64_t r) {
  if (c->is64) return ((const int64_t *)c->data)[r];
  return (int64_t)((const int32_t *)c->data)[r];
}

static uint64_t bitmap_words(uint64_t n_rows) { return (n_rows + 63) / 64; }

static int bit_get(const uint64_t *bm, uint64_t r) { return (int)((bm[r / 64] >> (r % 64)) & 1u); }
static void bit_set(uint64_t *bm, uint64_t r) { bm[r / 64] |= 1ULL << (r % 64); }
static void bit_clear(uint64_t *bm, uint64_t r) { bm[r / 64] &= ~(1ULL << (r % 64)); }

/* One past the last row of bitmap word w. */
static uint64_t row_end(int64_t w, uint64_t n_rows) {
  const uint64_t end = (uint64_t)w * 64 + 64;
  return end < n_rows ? end : n_rows;
}

/* Threads of the row-split scans (params.threads; 0 means one). */
static int n_threads(const ptor_params *pa) { return pa->threads > 1 ? (int)pa->threads : 1; }

static uint64_t bitmap_popcount(const uint64_t *bm, uint64_t n_rows) {
  uint64_t c = 0;
  for (uint64_t r = 0; r < n_rows; r++) c += (uint64_t)bit_get(bm, r);
  return c;
}

static int predicate_holds(const ptor_pred *p, int64_t v) {
  switch (p->op) {
    case PTOR_LT: return v < p->lo;
    case PTOR_LE: return v <= p->lo;
    case PTOR_GT: return v > p->lo;
    case PTOR_GE: return v >= p->lo;
    case PTOR_EQ: return v == p->lo;
    case PTOR_NE: return v != p->lo;
    case PTOR_BETWEEN: return p->lo <= v && v <= p->hi;
    default: return 0;
  }
}

/* Local ("inherent") filters are conjunctions over one base table
 * (Sec. 3.2, filter transformation; Sec. 3.4, filters over base tables). */
int ptor_local_filter(const ptor_table *t, const ptor_pred *preds, uint32_t n_preds,
                      uint64_t *bitmap, uint64_t *count) {
  for (uint32_t i = 0; i < n_preds; i++) {
    if (preds[i].col >= t->n_cols || preds[i].op > PTOR_BETWEEN) return PTOR_EINVAL;
  }
  memset(bitmap, 0, bitmap_words(t->n_rows) * sizeof(uint64_t));
  for (uint64_t r = 0; r < t->n_rows; r++) {
    int keep = 1;
    for (uint32_t i = 0; i < n_preds; i++) {
      if (!predicate_holds(&preds[i], column_value(&t->cols[preds[i].col], r))) keep = 0;
    }
    if (keep) bit_set(bitmap, r);
  }
  if (count) *count = bitmap_popcount(bitmap, t->n_rows);
  return PTOR_OK;
}

static int params_valid(uint32_t block_bits, uint32_t k, uint32_t bits_per_key) {
  if (block_bits < 32 || block_bits > 1024 || (block_bits & (block_bits - 1)) != 0) return 0;
  if (k < 1 || k > 16) return 0;
  if (bits_per_key < 1 || bits_per_key > 64) return 0;
  return 1;
}

int ptor_bloom_build(const ptor_column *keys, uint64_t n_rows, const uint64_t *bitmap,
                     uint32_t block_bits, uint32_t k, uint32_t bits_per_key, uint32_t *words,
                     uint64_t cap_words, uint64_t *nb_out) {
  if (!params_valid(block_bits, k, bits_per_key)) return PTOR_EINVAL;
  uint64_t n_sel = bitmap ? bitmap_popcount(bitmap, n_rows) : n_rows;
  uint64_t nb = ptor_filter_blocks(n_sel, bits_per_key, block_bits);
  uint64_t n_words = nb * (block_bits / 32);
  if (n_words > cap_words) return PTOR_EINVAL;
  memset(words, 0, n_words * sizeof(uint32_t));
  for (uint64_t r = 0; r < n_rows; r++) {
    if (bitmap && !bit_get(bitmap, r)) continue;
    ptor_bloom_insert(words, nb, block_bits, k, column_value(keys, r));
  }
  *nb_out = nb;
  return PTOR_OK;
}

int ptor_bloom_probe(const ptor_column *keys, uint64_t n_rows, const uint32_t *words, uint64_t nb,
                     uint32_t block_bits, uint32_t k, uint64_t *bitmap, uint64_t *count) {
  if (!params_valid(block_bits, k, 1) || nb == 0) return PTOR_EINVAL;
  for (uint64_t r = 0; r < n_rows; r++) {
    if (!bit_get(bitmap, r)) continue;
    if (!ptor_bloom_contains(words, nb, block_bits, k, column_value(keys, r))) bit_clear(bitmap, r);
  }
  if (count) *count = bitmap_popcount(bitmap, n_rows);
  return PTOR_OK;
}

int ptor_compact(const uint64_t *bitmap, uint64_t n_rows, uint32_t *idx, uint64_t *count) {
  uint64_t c = 0;
  for (uint64_t r = 0; r < n_rows; r++) {
    if (bit_get(bitmap, r)) idx[c++] = (uint32_t)r;
  }
  *count = c;
  return PTOR_OK;
}

/* ------------------------------------------------------------------ */
/* Filters carried along the transfer graph                             */
/* ------------------------------------------------------------------ */

/* A transferred filter: a Bloom filter, or (precise filter, Sec. 3.2
 * "Filter Type") the sorted set of distinct keys; `absent` when pruning
 * left it unbuilt (it then lets every key through). */
typedef struct {
  uint32_t kind;
  uint32_t absent;
  uint64_t nb;
  uint32_t *words;
  int64_t *keys;
  uint64_t n_keys;
} filter_t;

static int cmp_i64(const void *a, const void *b) {
  int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
  return (x > y) - (x < y);
}

static int filter_build(filter_t *f, const ptor_params *pa, const ptor_column *col,
                        uint64_t n_rows, const uint64_t *bitmap) {
  memset(f, 0, sizeof(*f));
  f->kind = pa->kind;
  uint64_t n_sel = bitmap_popcount(bitmap, n_rows);
  if (pa->kind == PTOR_BLOOM) {
    f->nb = ptor_filter_blocks(n_sel, pa->bits_per_key, pa->block_bits);
    const uint64_t n_fw = f->nb * (pa->block_bits / 32);
    f->words = (uint32_t *)calloc(n_fw, sizeof(uint32_t));
    if (!f->words) return PTOR_ENOMEM;
    if (n_threads(pa) <= 1) {
      for (uint64_t r = 0; r < n_rows; r++) {
        if (bit_get(bitmap, r))
          ptor_bloom_insert(f->words, f->nb, pa->block_bits, pa->k, column_value(col, r));
      }
      return PTOR_OK;
    }
    /* Row split: each thread inserts its rows into a private copy; OR is
     * order-free, so OR-ing the copies gives the filter bit for bit. */
    const int64_t n_words = (int64_t)bitmap_words(n_rows);
    int failed = 0;
#pragma omp parallel num_threads(n_threads(pa))
    {
      uint32_t *mine = (uint32_t *)calloc(n_fw, sizeof(uint32_t));
#pragma omp for schedule(static)
      for (int64_t w = 0; w < n_words; w++) {
        const uint64_t end = row_end(w, n_rows);
        for (uint64_t r = (uint64_t)w * 64; r < end && mine; r++) {
          if (bit_get(bitmap, r)) ptor_bloom_insert(mine, f->nb, pa->block_bits, pa->k, column_value(col, r));
        }
      }
#pragma omp critical
      {
        if (!mine) failed = 1;
        else
          for (uint64_t i = 0; i < n_fw; i++) f->words[i] |= mine[i];
      }
      free(mine);
    }
    return failed ? PTOR_ENOMEM : PTOR_OK;
  }
  f->keys = (int64_t *)malloc((n_sel ? n_sel : 1) * sizeof(int64_t));
  if (!f->keys) return PTOR_ENOMEM;
  uint64_t c = 0;
  for (uint64_t r = 0; r < n_rows; r++) {
    if (bit_get(bitmap, r)) f->keys[c++] = column_value(col, r);
  }
  qsort(f->keys, c, sizeof(int64_t), cmp_i64);
  uint64_t u = 0;
  for (uint64_t i = 0; i < c; i++) {
    if (u == 0 || f->keys[u - 1] != f->keys[i]) f->keys[u++] = f->keys[i];
  }
  f->n_keys = u;
  return PTOR_OK;
}

static int filter_contains(const filter_t *f, const ptor_params *pa, int64_t key) {
  if (f->absent) return 1;
  if (f->kind == PTOR_BLOOM) return ptor_bloom_contains(f->words, f->nb, pa->block_bits, pa->k, key);
  return bsearch(&key, f->keys, f->n_keys, sizeof(int64_t), cmp_i64) != NULL;
}

static void filter_free(filter_t *f) {
  free(f->words);
  free(f->keys);
  memset(f, 0, sizeof(*f));
}

/* ------------------------------------------------------------------ */
/* Predicate transfer graph and schedule (Sec. 3.2)                     */
/* ------------------------------------------------------------------ */

/* An edge points from the smaller table to the bigger one; equal sizes go
 * from the lower table index. This order on tables is strict and total, so
 * the directed graph has no cycle and no edge is dropped. */
static void orient_edges(const ptor_problem *p, uint32_t *src, uint32_t *dst) {
  for (uint32_t e = 0; e < p->n_edges; e++) {
    uint32_t u = p->edges[e].u, v = p->edges[e].v;
    int u_first;
    if (p->orient) {
      u_first = p->orient[e] > 0;
    } else {
      uint64_t nu = p->tables[u].n_rows, nv = p->tables[v].n_rows;
      u_first = (nu < nv) || (nu == nv && u < v);
    }
    src[e] = u_first ? u : v;
    dst[e] = u_first ? v : u;
  }
}

/* Kahn's algorithm: repeatedly take a table whose incoming edges have all
 * been visited. Returns 0 if the directed graph has a cycle. */
static int topological_order(const ptor_problem *p, const uint32_t *src, const uint32_t *dst,
                             int largest_first, uint32_t *order) {
  uint32_t n = p->n_tables;
  uint32_t *indeg = (uint32_t *)calloc(n ? n : 1, sizeof(uint32_t));
  char *done = (char *)calloc(n ? n : 1, 1);
  int ok = 1;
  for (uint32_t e = 0; e < p->n_edges; e++) indeg[dst[e]]++;
  for (uint32_t i = 0; i < n; i++) {
    int64_t pick = -1;
    for (uint32_t v = 0; v < n; v++) {
      if (done[v] || indeg[v] != 0) continue;
      if (pick < 0 || largest_first) pick = v;
      if (!largest_first) break;
    }
    if (pick < 0) {
      ok = 0;
      break;
    }
    order[i] = (uint32_t)pick;
    done[pick] = 1;
    for (uint32_t e = 0; e < p->n_edges; e++)
      if (src[e] == (uint32_t)pick) indeg[dst[e]]--;
  }
  free(indeg);
  free(done);
  return ok;
}

static const ptor_column *edge_column(const ptor_problem *p, uint32_t e, uint32_t table) {
  const ptor_edge *ed = &p->edges[e];
  uint32_t col = (ed->u == table) ? ed->u_col : ed->v_col;
  return &p->tables[table].cols[col];
}

static void dump_filter(const ptor_dump *d, const ptor_problem *p, uint32_t pass, uint32_t e,
                        const filter_t *f, const ptor_params *pa, uint32_t builder) {
  if (!d) return;
  uint64_t slot = (uint64_t)pass * p->n_edges + e;
  if (d->edge_src) d->edge_src[slot] = builder;
  if (d->filter_nb) d->filter_nb[slot] = (f->kind == PTOR_BLOOM && !f->absent) ? f->nb : 0;
  if (d->filter_words && d->filter_words[slot] && f->kind == PTOR_BLOOM && !f->absent) {
    uint64_t n = f->nb * (pa->block_bits / 32);
    uint64_t cap = d->filter_cap ? d->filter_cap[slot] : n;
    memcpy(d->filter_words[slot], f->words, (n < cap ? n : cap) * sizeof(uint32_t));
  }
}

/* Whether a filter may cross edge e from table `from` to table `to`
 * (Sec. 3.4: an outer join blocks the direction towards its preserved side,
 * a full outer join both). */
static int edge_carries(const ptor_edge *ed, uint32_t from, uint32_t to) {
  switch (ed->flags) {
    case PTOR_INNER: return 1;
    case PTOR_LEFT_OUTER: return from == ed->u && to == ed->v;
    case PTOR_RIGHT_OUTER: return from == ed->v && to == ed->u;
    default: return 0;
  }
}

/* One pass over the predicate transfer graph. A table first collects every
 * incoming filter and probes it on its own join-key column (rows already
 * removed stay removed), then builds one outgoing filter per outgoing edge
 * from the rows that remain. Tables are visited in topological order, so
 * every incoming filter exists before it is probed. */
static int run_pass(const ptor_problem *p, const ptor_params *pa, uint32_t pass,
                    const uint32_t *src, const uint32_t *dst, const uint32_t *order,
                    uint64_t *const *bitmaps, filter_t *filters, const ptor_dump *dump) {
  uint32_t n = p->n_tables, m = p->n_edges;
  int reverse_probe = (pa->variant & 2u) != 0;
  for (uint32_t i = 0; i < n; i++) {
    uint32_t v = order[i];
    const ptor_table *t = &p->tables[v];
    for (uint32_t j = 0; j < m; j++) {
      uint32_t e = reverse_probe ? m - 1 - j : j;
      if (dst[e] != v || !edge_carries(&p->edges[e], src[e], dst[e])) continue;
      const ptor_column *col = edge_column(p, e, v);
      const int64_t n_words = (int64_t)bitmap_words(t->n_rows);
      uint64_t *bm = bitmaps[v];
#pragma omp parallel for num_threads(n_threads(pa)) schedule(static) if (n_threads(pa) > 1)
      for (int64_t w = 0; w < n_words; w++) {
        const uint64_t end = row_end(w, t->n_rows);
        for (uint64_t r = (uint64_t)w * 64; r < end; r++) {
          if (bit_get(bm, r) && !filter_contains(&filters[e], pa, column_value(col, r))) bit_clear(bm, r);
        }
      }
    }
    /* Transfer path pruning: a non-empty table that has lost no row yet
     * would send filters holding every key of its columns; they are not
     * built, and the probes above let every key through them. (An empty
     * table's filter holds no key and removes every row it reaches, so it
     * is always sent.) */
    const int unreduced =
        pa->prune && t->n_rows > 0 && bitmap_popcount(bitmaps[v], t->n_rows) == t->n_rows;
    for (uint32_t e = 0; e < m; e++) {
      if (src[e] != v || !edge_carries(&p->edges[e], src[e], dst[e])) continue;
      if (unreduced) {
        filter_free(&filters[e]);
        filters[e].kind = pa->kind;
        filters[e].absent = 1;
        dump_filter(dump, p, pass, e, &filters[e], pa, v);
        continue;
      }
      int rc = filter_build(&filters[e], pa, edge_column(p, e, v), t->n_rows, bitmaps[v]);
      if (rc != PTOR_OK) return rc;
      dump_filter(dump, p, pass, e, &filters[e], pa, v);
    }
  }
  return PTOR_OK;
}

static int problem_valid(const ptor_problem *p) {
  for (uint32_t e = 0; e < p->n_edges; e++) {
    const ptor_edge *ed = &p->edges[e];
    if (ed->u >= p->n_tables || ed->v >= p->n_tables || ed->u == ed->v) return 0;
    if (ed->flags > PTOR_FULL_OUTER) return 0;
    if (ed->u_col >= p->tables[ed->u].n_cols || ed->v_col >= p->tables[ed->v].n_cols) return 0;
    if (p->orient && p->orient[e] != 1 && p->orient[e] != -1) return 0;
  }
  for (uint32_t i = 0; i < p->n_preds; i++) {
    if (p->preds[i].table >= p->n_tables) return 0;
    if (p->preds[i].col >= p->tables[p->preds[i].table].n_cols) return 0;
    if (p->preds[i].op > PTOR_BETWEEN) return 0;
  }
  return 1;
}

int ptor_transfer(const ptor_problem *p, const ptor_params *pa, uint64_t *const *bitmaps,
                  uint64_t *counts, const ptor_dump *dump) {
  if (!problem_valid(p)) return PTOR_EINVAL;
  if (pa->kind == PTOR_BLOOM && !params_valid(pa->block_bits, pa->k, pa->bits_per_key))
    return PTOR_EINVAL;
  if (pa->kind > PTOR_EXACT || pa->n_passes < 1 || pa->n_passes > 2 || pa->prune > 1) return PTOR_EINVAL;

  uint32_t n = p->n_tables, m = p->n_edges;
  uint32_t *src = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
  uint32_t *dst = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
  uint32_t *order = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
  uint32_t *rev_order = (uint32_t *)malloc((n ? n : 1) * sizeof(uint32_t));
  filter_t *filters = (filter_t *)calloc(m ? m : 1, sizeof(filter_t));
  int rc = PTOR_OK;
  if (!src || !dst || !order || !rev_order || !filters) {
    rc = PTOR_ENOMEM;
    goto out;
  }

  /* Local predicates first: each table starts from its own filtered rows. */
  for (uint32_t t = 0; t < n; t++) {
    const uint64_t n_rows = p->tables[t].n_rows;
    const int64_t n_words = (int64_t)bitmap_words(n_rows);
    uint64_t *bm = bitmaps[t];
    memset(bm, 0, (uint64_t)n_words * sizeof(uint64_t));
#pragma omp parallel for num_threads(n_threads(pa)) schedule(static) if (n_threads(pa) > 1)
    for (int64_t w = 0; w < n_words; w++) {
      const uint64_t end = row_end(w, n_rows);
      for (uint64_t r = (uint64_t)w * 64; r < end; r++) {
        int keep = 1;
        for (uint32_t i = 0; i < p->n_preds; i++) {
          const ptor_pred *pr = &p->preds[i];
          if (pr->table == t && !predicate_holds(pr, column_value(&p->tables[t].cols[pr->col], r)))
            keep = 0;
        }
        if (keep) bit_set(bm, r);
      }
    }
  }

  /* Forward pass on the predicate transfer graph. */
  orient_edges(p, src, dst);
  if (!topological_order(p, src, dst, (pa->variant & 1u) != 0, order)) {
    rc = PTOR_EINVAL;
    goto out;
  }
  rc = run_pass(p, pa, 0, src, dst, order, bitmaps, filters, dump);
  if (rc != PTOR_OK) goto out;
  if (dump) {
    for (uint32_t t = 0; t < n; t++) {
      uint64_t nw = bitmap_words(p->tables[t].n_rows);
      if (dump->fwd_bitmaps && dump->fwd_bitmaps[t])
        memcpy(dump->fwd_bitmaps[t], bitmaps[t], nw * sizeof(uint64_t));
      if (dump->fwd_counts) dump->fwd_counts[t] = bitmap_popcount(bitmaps[t], p->tables[t].n_rows);
    }
  }

  /* Backward pass: every edge reversed, fresh filters, starting from the
   * rows that survived the forward pass. The reverse of a topological order
   * is a topological order of the reversed graph. */
  if (pa->n_passes == 2) {
    for (uint32_t e = 0; e < m; e++) filter_free(&filters[e]);
    for (uint32_t i = 0; i < n; i++) rev_order[i] = order[n - 1 - i];
    rc = run_pass(p, pa, 1, dst, src, rev_order, bitmaps, filters, dump);
    if (rc != PTOR_OK) goto out;
  }

  for (uint32_t t = 0; t < n; t++) counts[t] = bitmap_popcount(bitmaps[t], p->tables[t].n_rows);

out:
  if (filters)
    for (uint32_t e = 0; e < m; e++) filter_free(&filters[e]);
  free(filters);
  free(src);
  free(dst);
  free(order);
  free(rev_order);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Join phase (Sec. 3.3)                                                */
/* ------------------------------------------------------------------ */

/* The join result is defined without reference to any join algorithm: all
 * combinations of selected rows, one per table of the component, that agree
 * on every edge. It is enumerated one table at a time in breadth-first
 * order from the root, so each table joins a prefix it is connected to; the
 * rows of the new table whose key matches one edge to the prefix are found
 * in a key-sorted list of its selected rows, and every edge between the new
 * table and the prefix (the cycle-closing ones and the other halves of a
 * composite key included) is then checked on each candidate. */

typedef struct {
  int64_t key;
  uint32_t row;
} keyed_row;

static int cmp_keyed(const void *a, const void *b) {
  const keyed_row *x = (const keyed_row *)a, *y = (const keyed_row *)b;
  if (x->key != y->key) return (x->key > y->key) - (x->key < y->key);
  return (x->row > y->row) - (x->row < y->row);
}

static _Thread_local uint32_t tuple_width; /* ids per tuple, for cmp_tuple */

static int cmp_tuple(const void *a, const void *b) {
  const uint32_t *x = (const uint32_t *)a, *y = (const uint32_t *)b;
  for (uint32_t c = 0; c < tuple_width; c++)
    if (x[c] != y[c]) return (x[c] > y[c]) - (x[c] < y[c]);
  return 0;
}

static int row_selected(const uint64_t *const *bitmaps, uint32_t t, uint64_t r) {
  return !bitmaps || !bitmaps[t] || bit_get(bitmaps[t], r);
}

int ptor_join(const ptor_problem *p, uint32_t root, const uint64_t *const *bitmaps, uint32_t *comp,
              uint32_t *n_comp, uint32_t *out, uint64_t cap, uint64_t *n_out) {
  if (!p || root >= p->n_tables || !comp || !n_comp || !n_out || (cap && !out)) return PTOR_EINVAL;
  const uint32_t n = p->n_tables, m = p->n_edges;
  for (uint32_t e = 0; e < m; e++) /* a join edge links two different tables */
    if (p->edges[e].u >= n || p->edges[e].v >= n || p->edges[e].u == p->edges[e].v) return PTOR_EINVAL;
  int rc = PTOR_OK;
  uint32_t *order = malloc(n * sizeof(uint32_t));
  int32_t *slot = malloc(n * sizeof(int32_t)); /* position of a table in the tuples, -1: not placed */
  uint32_t *cur = NULL, *next = NULL;
  keyed_row *index = NULL;
  if (!order || !slot) {
    rc = PTOR_ENOMEM;
    goto done;
  }

  /* Breadth-first order of root's component (edges in index order). */
  for (uint32_t t = 0; t < n; t++) slot[t] = -1;
  uint32_t w = 0;
  order[w++] = root;
  slot[root] = 0;
  for (uint32_t head = 0; head < w; head++) {
    const uint32_t t = order[head];
    for (uint32_t e = 0; e < m; e++) {
      const ptor_edge *ed = &p->edges[e];
      uint32_t other;
      if (ed->u == t) other = ed->v;
      else if (ed->v == t) other = ed->u;
      else continue;
      if (slot[other] < 0) {
        slot[other] = (int32_t)w;
        order[w++] = other;
      }
    }
  }

  /* The root's selected rows are the first prefix. */
  uint64_t n_cur = 0;
  const uint64_t root_rows = p->tables[root].n_rows;
  cur = malloc((root_rows ? root_rows : 1) * sizeof(uint32_t));
  if (!cur) {
    rc = PTOR_ENOMEM;
    goto done;
  }
  for (uint64_t r = 0; r < root_rows; r++)
    if (row_selected(bitmaps, root, r)) cur[n_cur++] = (uint32_t)r;

  for (uint32_t i = 1; i < w; i++) {
    const uint32_t v = order[i];
    /* The lowest-indexed edge from v to a table placed before it. */
    uint32_t e0 = m;
    for (uint32_t e = 0; e < m && e0 == m; e++) {
      const ptor_edge *ed = &p->edges[e];
      if ((ed->u == v && (uint32_t)slot[ed->v] < i) || (ed->v == v && (uint32_t)slot[ed->u] < i))
        e0 = e;
    }
    const ptor_edge *ed0 = &p->edges[e0];
    const uint32_t v_col = ed0->u == v ? ed0->u_col : ed0->v_col;
    const uint32_t u = ed0->u == v ? ed0->v : ed0->u;
    const uint32_t u_col = ed0->u == v ? ed0->v_col : ed0->u_col;

    /* v's selected rows sorted by their key on e0. */
    const uint64_t v_rows = p->tables[v].n_rows;
    free(index);
    index = malloc((v_rows ? v_rows : 1) * sizeof(keyed_row));
    if (!index) {
      rc = PTOR_ENOMEM;
      goto done;
    }
    uint64_t n_index = 0;
    for (uint64_t r = 0; r < v_rows; r++) {
      if (!row_selected(bitmaps, v, r)) continue;
      index[n_index].key = column_value(&p->tables[v].cols[v_col], r);
      index[n_index].row = (uint32_t)r;
      n_index++;
    }
    qsort(index, n_index, sizeof(keyed_row), cmp_keyed);

    /* Every prefix tuple extended by every matching row of v. */
    uint64_t n_next = 0, cap_next = n_cur ? n_cur : 1;
    next = malloc(cap_next * (i + 1) * sizeof(uint32_t));
    if (!next) {
      rc = PTOR_ENOMEM;
      goto done;
    }
    for (uint64_t j = 0; j < n_cur; j++) {
      const uint32_t *tup = cur + j * i;
      const int64_t key = column_value(&p->tables[u].cols[u_col], tup[slot[u]]);
      uint64_t lo = 0, hi = n_index; /* first entry with index key >= key */
      while (lo < hi) {
        const uint64_t mid = lo + (hi - lo) / 2;
        if (index[mid].key < key) lo = mid + 1;
        else hi = mid;
      }
      for (uint64_t x = lo; x < n_index && index[x].key == key; x++) {
        const uint32_t r = index[x].row;
        int ok = 1;
        for (uint32_t e = 0; e < m && ok; e++) {
          const ptor_edge *ed = &p->edges[e];
          uint32_t v_c, b_t, b_c; /* v's column; the other table and its column */
          if (ed->u == v) {
            v_c = ed->u_col; b_t = ed->v; b_c = ed->v_col;
          } else if (ed->v == v) {
            v_c = ed->v_col; b_t = ed->u; b_c = ed->u_col;
          } else {
            continue;
          }
          if ((uint32_t)slot[b_t] >= i) continue; /* joined later */
          if (column_value(&p->tables[v].cols[v_c], r) !=
              column_value(&p->tables[b_t].cols[b_c], tup[slot[b_t]]))
            ok = 0;
        }
        if (!ok) continue;
        if (n_next == cap_next) {
          cap_next *= 2;
          uint32_t *grown = realloc(next, cap_next * (i + 1) * sizeof(uint32_t));
          if (!grown) {
            rc = PTOR_ENOMEM;
            goto done;
          }
          next = grown;
        }
        memcpy(next + n_next * (i + 1), tup, i * sizeof(uint32_t));
        next[n_next * (i + 1) + i] = r;
        n_next++;
      }
    }
    free(cur);
    cur = next;
    next = NULL;
    n_cur = n_next;
  }

  /* Columns in ascending table order, tuples sorted. */
  uint32_t c = 0;
  for (uint32_t t = 0; t < n; t++)
    if (slot[t] >= 0) comp[c++] = t;
  *n_comp = w;
  uint32_t *sorted = malloc((n_cur ? n_cur : 1) * w * sizeof(uint32_t));
  if (!sorted) {
    rc = PTOR_ENOMEM;
    goto done;
  }
  for (uint64_t j = 0; j < n_cur; j++)
    for (uint32_t q = 0; q < w; q++) sorted[j * w + q] = cur[j * w + slot[comp[q]]];
  tuple_width = w;
  qsort(sorted, n_cur, w * sizeof(uint32_t), cmp_tuple);
  const uint64_t n_copy = n_cur < cap ? n_cur : cap;
  if (n_copy) memcpy(out, sorted, n_copy * w * sizeof(uint32_t));
  *n_out = n_cur;
  free(sorted);

done:
  free(order);
  free(slot);
  free(cur);
  free(next);
  free(index);
  return rc;
}
