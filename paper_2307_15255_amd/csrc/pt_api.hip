// pt_api.hip - the C ABI (include/pt.h): argument checks, the transfer
// planner and the launch sequence of the transfer phase.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <vector>

#include "pt_internal.hpp"

namespace pt {

// ------------------------------------------------------------- errors

static thread_local std::string g_error;

static pt_status fail(pt_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return st;
}

static pt_status check_hip(hipError_t e, const char *what) {
  if (e == hipSuccess) return PT_OK;
  return fail(PT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// -------------------------------------------------------- device info

const DeviceInfo &device_info() {
  static std::mutex mu;
  static DeviceInfo infos[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) dev = 0;
  std::lock_guard<std::mutex> lock(mu);
  DeviceInfo &di = infos[dev];
  if (di.device < 0) {
    int n_cu = 0, lds = 0, lds_optin = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) n_cu = 256;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) lds = 65536;
    if (hipDeviceGetAttribute(&lds_optin, hipDeviceAttributeSharedMemPerBlockOptin, dev) != hipSuccess) lds_optin = 0;
    di.n_cu = n_cu > 0 ? n_cu : 256;
    di.max_lds_block = std::max(lds, lds_optin);
    if (di.max_lds_block <= 0) di.max_lds_block = 65536;
    di.device = dev;
  }
  return di;
}

// ---------------------------------------------------------- profiling

namespace {

struct ProfRecord {
  pt_kernel_time t;
  hipEvent_t start, stop;
};

thread_local int g_prof_mode = 0;  // 0 off, 1 every launch, 2 probe launches only
// when g_prof_only[0] != 0, only launches of that (name, table, pass) record
thread_local char g_prof_only[sizeof(pt_kernel_time{}.name)] = {};
thread_local uint32_t g_prof_only_table = 0, g_prof_only_pass = 0;
thread_local std::vector<ProfRecord> g_prof;
thread_local std::vector<hipEvent_t> g_event_pool;

hipEvent_t take_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  // timing only: no system-scope fence, so the events add no cache flush
  // (and no bubble) between the launches they bracket
  if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
  return e;
}

// Brackets one launch with events on its stream when profiling is on.
class Timed {
 public:
  Timed(const char *name, uint32_t table, uint32_t pass, uint64_t rows, uint64_t bytes,
        hipStream_t s)
      : s_(s) {
    if (!name || g_prof_mode == 0 || (g_prof_mode == 2 && std::strstr(name, "probe") == nullptr)) return;
    if (g_prof_only[0] && (table != g_prof_only_table || pass != g_prof_only_pass ||
                           std::strncmp(name, g_prof_only, sizeof g_prof_only - 1) != 0))
      return;
    rec_.t = pt_kernel_time{};
    std::snprintf(rec_.t.name, sizeof rec_.t.name, "%s", name);
    rec_.t.table = table;
    rec_.t.pass = pass;
    rec_.t.rows = rows;
    rec_.t.bytes = bytes;
    rec_.start = take_event();
    rec_.stop = take_event();
    if (rec_.start && rec_.stop) {
      active_ = hipEventRecord(rec_.start, s_) == hipSuccess;
    }
  }
  ~Timed() {
    if (!active_) return;
    if (hipEventRecord(rec_.stop, s_) == hipSuccess) g_prof.push_back(rec_);
  }

 private:
  hipStream_t s_;
  ProfRecord rec_{};
  bool active_ = false;
};

// ---------------------------------------------------------- validation

constexpr uint64_t kMaxRows = 0xFFFFFFFFull;  // row ids are uint32
constexpr uint32_t kMaxTables = 64;

pt_status check_params(const pt_params *p) {
  if (!p) return fail(PT_EINVAL, "params is NULL");
  const uint32_t B = p->block_bits;
  if (B < 32 || B > 1024 || (B & (B - 1)) != 0)
    return fail(PT_EINVAL, "block_bits %u is not a power of two in [32, 1024]", B);
  if (p->k < 1 || p->k > 16) return fail(PT_EINVAL, "k %u outside [1, 16]", p->k);
  if (p->bits_per_key < 1 || p->bits_per_key > 64)
    return fail(PT_EINVAL, "bits_per_key %u outside [1, 64]", p->bits_per_key);
  if ((p->flags & ~(PT_FLAG_NO_APPEND | PT_FLAG_SHARED_SCAN | PT_FLAG_EXACT | PT_FLAG_PRUNE)) != 0)
    return fail(PT_EINVAL, "params.flags: unknown bits 0x%x", p->flags);
  if (p->hash_version > 1)
    return fail(PT_EUNSUPPORTED, "hash_version %u (this library implements version 1)", p->hash_version);
  if (p->tile_rows != 0 && (p->tile_rows % 4096 != 0 || p->tile_rows > (1u << 24)))
    return fail(PT_EINVAL, "tile_rows %u is not 0 or a multiple of 4096 up to 2^24", p->tile_rows);
  if (p->probe_order > PT_PROBE_GIVEN) return fail(PT_EINVAL, "probe_order %u", p->probe_order);
  return PT_OK;
}

// The parameters that fix the filter bits: equal for every filter of a call.
bool same_filter(const pt_params &a, const pt_params &b) {
  return a.block_bits == b.block_bits && a.k == b.k && a.bits_per_key == b.bits_per_key &&
         (a.hash_version <= 1) == (b.hash_version <= 1);
}

ProbeOpts probe_opts(const pt_params &p) {
  ProbeOpts o;
  o.lds_budget = p.lds_budget;
  o.keep_order = p.probe_order == PT_PROBE_GIVEN;
  return o;
}

uint64_t blocks_for(uint64_t n_keys, const pt_params &p) {
  uint64_t nb = (n_keys * p.bits_per_key + p.block_bits - 1) / p.block_bits;
  return nb == 0 ? 1 : nb;
}

uint64_t capacity_words(uint64_t n_keys, const pt_params &p) {
  return blocks_for(n_keys, p) * (p.block_bits / 32);
}

pt_status check_column(const pt_column *c, uint64_t n_rows, const char *what) {
  if (!c) return fail(PT_EINVAL, "%s: column is NULL", what);
  if (c->dtype != PT_I32 && c->dtype != PT_I64) return fail(PT_EINVAL, "%s: dtype %u", what, c->dtype);
  if (n_rows > 0 && !c->data) return fail(PT_EINVAL, "%s: data is NULL", what);
  return PT_OK;
}

pt_status check_table(const pt_table *t, uint32_t idx) {
  if (t->n_rows > kMaxRows) return fail(PT_EINVAL, "table %u: %llu rows (limit 2^32 - 1)", idx,
                                        (unsigned long long)t->n_rows);
  if (t->n_cols > 0 && !t->cols) return fail(PT_EINVAL, "table %u: cols is NULL", idx);
  for (uint32_t c = 0; c < t->n_cols; c++) {
    char what[64];
    std::snprintf(what, sizeof what, "table %u column %u", idx, c);
    pt_status st = check_column(&t->cols[c], t->n_rows, what);
    if (st != PT_OK) return st;
  }
  return PT_OK;
}

pt_status check_filter(const pt_bloom &f, const pt_params &p0, uint64_t n_rows, uint32_t i) {
  if (!f.words || !f.d_nb) return fail(PT_EINVAL, "filter %u: words or d_nb is NULL", i);
  pt_status st = check_params(&f.params);
  if (st != PT_OK) return st;
  if (!same_filter(f.params, p0)) return fail(PT_EINVAL, "filter %u: parameters differ from filter 0", i);
  const uint64_t need = capacity_words(n_rows, f.params);
  if (need / (f.params.block_bits / 32) > 0xFFFFFFFFull)
    return fail(PT_EINVAL, "filter %u: %llu blocks exceed 2^32 - 1", i,
                (unsigned long long)(need / (f.params.block_bits / 32)));
  if (f.cap_words < need)
    return fail(PT_EINVAL, "filter %u: cap_words %llu < %llu needed for %llu rows", i,
                (unsigned long long)f.cap_words, (unsigned long long)need,
                (unsigned long long)n_rows);
  return PT_OK;
}

FilterRef make_ref(const pt_column &keys, const pt_bloom &f) {
  FilterRef r{};
  r.keys = keys.data;
  r.words = f.words;
  r.nb = f.d_nb;
  r.cap_words = f.cap_words;
  r.key64 = keys.dtype == PT_I64;
  return r;
}

uint64_t key_bytes(const pt_column &c) { return c.dtype == PT_I64 ? 8 : 4; }

// ------------------------------------------------------------- planner

struct Plan {
  uint32_t n_t = 0, n_e = 0;
  std::vector<uint32_t> src, dst;  // forward orientation of every edge
  // [pass * n_e + e]: edge e carries a filter in that pass (an outer join
  // blocks one direction or both, Sec. 3.4)
  std::vector<uint8_t> active;
  bool sends(uint32_t p, uint32_t e, uint32_t v) const { return active[p * n_e + e] && (p == 0 ? src : dst)[e] == v; }
  bool receives(uint32_t p, uint32_t e, uint32_t v) const {
    return active[p * n_e + e] && (p == 0 ? dst : src)[e] == v;
  }
  std::vector<uint32_t> order;     // forward topological order
  uint64_t off_counts = 0;         // 3 * n_t uint64: local, forward, backward
  uint64_t off_nb = 0;             // 2 * n_e uint64: forward, backward filters
  std::vector<uint64_t> off_filter, cap_words;  // [pass * n_e + e]
  std::vector<uint32_t> set_lg;                 // exact filters: log2 of each set's slot capacity
  bool exact = false;
  uint64_t off_scratch = 0;                     // private filter copies of the builds
  uint64_t scratch_words = 0;
  uint64_t off_hist = 0, off_totals = 0, off_starts = 0, off_entries = 0;  // partitioned builds
  uint32_t hist_groups = 0;
  uint64_t entries_cap = 0;
  uint64_t off_app_counts = 0, off_app = 0;  // appended survivor keys (one probe's at a time)
  uint64_t total = 0;
};

constexpr uint64_t kMaxEntries = 64ull << 20;  // partitioned-build entries (4 bytes each)

uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

pt_status check_preds(const Plan &pl, const pt_table *tables, const pt_pred *preds, uint32_t n_preds) {
  if (n_preds > 0 && !preds) return fail(PT_EINVAL, "preds is NULL");
  for (uint32_t i = 0; i < n_preds; i++) {
    if (preds[i].table >= pl.n_t) return fail(PT_EINVAL, "predicate %u: table out of range", i);
    if (preds[i].col >= tables[preds[i].table].n_cols)
      return fail(PT_EINVAL, "predicate %u: column out of range", i);
    if (preds[i].op > PT_BETWEEN) return fail(PT_EINVAL, "predicate %u: op %u", i, preds[i].op);
  }
  return PT_OK;
}

uint32_t col_at(const pt_graph *g, uint32_t e, uint32_t table) {
  return g->edges[e].u == table ? g->edges[e].u_col : g->edges[e].v_col;
}

// Appended keys (the filter transformation scans a table once, Sec. 3.2):
// the probe of table v in pass p appends its survivors' keys of `cols`, which
// the builds of v in pass `pass` then read, when
//   - v also builds in pass p (cols: its outgoing columns of pass p), or
//   - p is the forward pass, v builds nothing in it and is its last table:
//     v is then the first table of the backward pass, and its backward
//     builds (on the columns of its forward incoming edges) start from the
//     forward survivors.
struct AppendPlan {
  std::vector<uint32_t> cols;  // empty: nothing appended
  uint32_t pass = 0;
};

AppendPlan append_plan(const Plan &pl, const pt_graph *g, const pt_table *tables, const pt_params &params,
                       uint32_t p, uint32_t v) {
  AppendPlan ap;
  if ((params.flags & (PT_FLAG_NO_APPEND | PT_FLAG_EXACT)) || tables[v].n_rows == 0) return ap;
  bool in = false, out = false;
  for (uint32_t e = 0; e < pl.n_e; e++) {
    in = in || pl.receives(p, e, v);
    out = out || pl.sends(p, e, v);
  }
  if (!in) return ap;
  uint32_t q;
  if (out)
    q = p;
  else if (p == 0 && pl.order.back() == v)
    q = 1;
  else
    return ap;
  for (uint32_t e = 0; e < pl.n_e; e++) {
    if (!pl.sends(q, e, v)) continue;
    const uint32_t c = col_at(g, e, v);
    if (std::find(ap.cols.begin(), ap.cols.end(), c) == ap.cols.end()) ap.cols.push_back(c);
  }
  if (ap.cols.empty() || ap.cols.size() > static_cast<size_t>(kMaxAppend)) ap.cols.clear();
  ap.pass = q;
  return ap;
}

// Entries per appended column: a quarter of the rows (a region with more
// survivors is walked instead) plus room for the regions of small tables.
uint64_t append_capacity(uint64_t n_rows) { return (n_rows + 3) / 4 + 65536; }

uint64_t append_bytes(const AppendPlan &ap, const pt_table &t) {
  uint64_t b = 0;
  for (uint32_t c : ap.cols) b += align256(append_capacity(t.n_rows) * key_bytes(t.cols[c]));
  return b;
}


pt_status make_plan(const pt_graph *g, const pt_table *tables, const pt_params *params, Plan &pl) {
  if (!g) return fail(PT_EINVAL, "graph is NULL");
  pt_status st = check_params(params);
  if (st != PT_OK) return st;
  if (g->n_tables > kMaxTables) return fail(PT_EINVAL, "%u tables (limit %u)", g->n_tables, kMaxTables);
  if (g->n_tables > 0 && !tables) return fail(PT_EINVAL, "tables is NULL");
  if (g->n_edges > 0 && !g->edges) return fail(PT_EINVAL, "edges is NULL");
  for (uint32_t t = 0; t < g->n_tables; t++) {
    st = check_table(&tables[t], t);
    if (st != PT_OK) return st;
    const uint64_t nb = blocks_for(tables[t].n_rows, *params);
    if (nb > 0xFFFFFFFFull) return fail(PT_EINVAL, "table %u: filter of %llu blocks exceeds 2^32 - 1", t,
                                        (unsigned long long)nb);
  }
  pl.n_t = g->n_tables;
  pl.n_e = g->n_edges;
  pl.src.assign(pl.n_e, 0);
  pl.dst.assign(pl.n_e, 0);
  pl.active.assign(2ull * pl.n_e, 1);
  for (uint32_t e = 0; e < pl.n_e; e++) {
    const pt_edge &ed = g->edges[e];
    if (ed.u >= pl.n_t || ed.v >= pl.n_t) return fail(PT_EINVAL, "edge %u: table out of range", e);
    if (ed.u == ed.v) return fail(PT_EINVAL, "edge %u joins table %u with itself", e, ed.u);
    if (ed.flags > PT_EDGE_FULL_OUTER)
      return fail(PT_EUNSUPPORTED, "edge %u: flags 0x%x (inner, left, right or full outer join)", e, ed.flags);
    if (ed.u_col >= tables[ed.u].n_cols || ed.v_col >= tables[ed.v].n_cols)
      return fail(PT_EINVAL, "edge %u: column out of range", e);
    bool u_first;
    if (g->orient) {
      if (g->orient[e] != 1 && g->orient[e] != -1)
        return fail(PT_EINVAL, "edge %u: orientation must be +1 or -1", e);
      u_first = g->orient[e] == 1;
    } else {
      // Sec. 3.2: from the smaller table to the bigger one; ties by index.
      const uint64_t nu = tables[ed.u].n_rows, nv = tables[ed.v].n_rows;
      u_first = nu < nv || (nu == nv && ed.u < ed.v);
    }
    pl.src[e] = u_first ? ed.u : ed.v;
    pl.dst[e] = u_first ? ed.v : ed.u;
    // Sec. 3.4: a left outer join keeps every row of its left table, so
    // only the left table's filter may reduce the right one (u -> v); a
    // right outer join the reverse; a full outer join blocks both. The edge
    // then carries a filter only in the pass where it runs that way.
    for (uint32_t p = 0; p < 2; p++) {
      const uint32_t from = p == 0 ? pl.src[e] : pl.dst[e];
      bool ok = true;
      if (ed.flags == PT_EDGE_LEFT_OUTER) ok = from == ed.u;
      else if (ed.flags == PT_EDGE_RIGHT_OUTER) ok = from == ed.v;
      else if (ed.flags == PT_EDGE_FULL_OUTER) ok = false;
      pl.active[p * pl.n_e + e] = ok ? 1 : 0;
    }
  }
  // Kahn's algorithm; the lowest ready index first.
  std::vector<uint32_t> indeg(pl.n_t, 0);
  std::vector<char> done(pl.n_t, 0);
  for (uint32_t e = 0; e < pl.n_e; e++) indeg[pl.dst[e]]++;
  pl.order.clear();
  for (uint32_t i = 0; i < pl.n_t; i++) {
    uint32_t pick = pl.n_t;
    for (uint32_t v = 0; v < pl.n_t; v++)
      if (!done[v] && indeg[v] == 0) {
        pick = v;
        break;
      }
    if (pick == pl.n_t) return fail(PT_EINVAL, "the oriented join graph has a cycle");
    done[pick] = 1;
    pl.order.push_back(pick);
    for (uint32_t e = 0; e < pl.n_e; e++)
      if (pl.src[e] == pick) indeg[pl.dst[e]]--;
  }
  // Workspace layout.
  uint64_t off = 256;
  pl.off_counts = off;
  off = align256(off + 3ull * pl.n_t * 8);
  pl.off_nb = off;
  off = align256(off + 2ull * pl.n_e * 8);
  pl.off_filter.assign(2ull * pl.n_e, 0);
  pl.cap_words.assign(2ull * pl.n_e, 0);
  pl.exact = (params->flags & PT_FLAG_EXACT) != 0;
  pl.set_lg.assign(2ull * pl.n_e, 0);
  for (uint32_t pass = 0; pass < 2; pass++) {
    for (uint32_t e = 0; e < pl.n_e; e++) {
      const uint32_t builder = pass == 0 ? pl.src[e] : pl.dst[e];
      uint64_t cap = capacity_words(tables[builder].n_rows, *params);
      if (pl.exact) {
        // an exact set: int64 slots, at least twice the builder's rows, and
        // one word that records the key INT64_MIN
        uint32_t lg = 6;
        while ((1ull << lg) < 2 * tables[builder].n_rows) lg++;
        pl.set_lg[pass * pl.n_e + e] = lg;
        cap = ((1ull << lg) + 1) * 2;
      }
      pl.off_filter[pass * pl.n_e + e] = off;
      pl.cap_words[pass * pl.n_e + e] = cap;
      off = align256(off + cap * 4);
    }
  }
  // Scratch for the builds' private LDS copies: one copy per CU of the
  // largest group of filters one table builds at once (capped at the LDS).
  uint64_t group_words = 0;
  for (uint32_t pass = 0; pass < 2; pass++) {
    for (uint32_t v = 0; v < pl.n_t; v++) {
      uint64_t w = 0;
      uint32_t in_launch = 0;
      for (uint32_t e = 0; e < pl.n_e; e++) {
        if (!pl.sends(pass, e, v)) continue;
        if (in_launch == kMaxFilters) {
          group_words = std::max(group_words, w);
          w = 0;
          in_launch = 0;
        }
        w += pl.cap_words[pass * pl.n_e + e];
        in_launch++;
      }
      group_words = std::max(group_words, w);
    }
  }
  if (pl.exact) group_words = 0;  // sets are built in place
  const uint64_t copy_words = std::min<uint64_t>(group_words, build_lds_words());
  pl.off_scratch = off;
  pl.scratch_words = copy_words * static_cast<uint64_t>(device_info().n_cu);
  off = align256(off + pl.scratch_words * 4);
  // Partitioned builds (filters larger than LDS): histogram rows, bucket
  // totals and starts, and entries for the largest group (filters x rows of
  // its builder), at most kMaxEntries.
  uint64_t group_entries = 0;
  for (uint32_t pass = 0; pass < 2; pass++) {
    for (uint32_t v = 0; v < pl.n_t; v++) {
      uint32_t f = 0;
      for (uint32_t e = 0; e < pl.n_e; e++)
        if (pl.sends(pass, e, v)) f++;
      group_entries = std::max<uint64_t>(group_entries, static_cast<uint64_t>(std::min<uint32_t>(f, kMaxFilters)) *
                                                            tables[v].n_rows);
    }
  }
  if (pl.exact) group_entries = 0;
  const char *force = std::getenv("PT_BUILD_PATH");
  const bool force_part = force && std::strcmp(force, "part") == 0;
  if ((group_words > build_lds_words() || force_part) && group_entries > 0) {
    pl.hist_groups = static_cast<uint32_t>(device_info().n_cu);
    pl.off_hist = off;
    off = align256(off + static_cast<uint64_t>(pl.hist_groups) * kMaxBuckets * 4);
    pl.off_totals = off;
    off = align256(off + static_cast<uint64_t>(kMaxBuckets) * 8);
    pl.off_starts = off;
    off = align256(off + (static_cast<uint64_t>(kMaxBuckets) + 1) * 8);
    uint64_t max_entries = kMaxEntries;
    // PT_MAX_ENTRIES (testing): a smaller entry buffer, to exercise the
    // in-place fallback of the partitioned build.
    if (const char *env = std::getenv("PT_MAX_ENTRIES")) max_entries = std::strtoull(env, nullptr, 10);
    pl.entries_cap = std::min(group_entries, max_entries);
    pl.off_entries = off;
    off = align256(off + pl.entries_cap * 4);
  }
  // Appended keys: region counts and the largest probe's columns.
  uint64_t app_bytes = 0;
  for (uint32_t p = 0; p < 2; p++)
    for (uint32_t v = 0; v < pl.n_t; v++)
      app_bytes = std::max(app_bytes, append_bytes(append_plan(pl, g, tables, *params, p, v), tables[v]));
  if (app_bytes > 0) {
    pl.off_app_counts = off;
    off = align256(off + static_cast<uint64_t>(kMaxRegions) * 4);
    pl.off_app = off;
    off += app_bytes;
  }
  pl.total = off;
  return PT_OK;
}

}  // namespace
}  // namespace pt

using namespace pt;

extern "C" {

const char *pt_version(void) { return "pt-mi355x 0.1 (gfx950)"; }

const char *pt_last_error(void) { return g_error.c_str(); }

pt_status pt_check_status(const void *d_status, pt_stream stream) {
  if (!d_status) return fail(PT_EINVAL, "d_status is NULL");
  static const uint32_t kZeroWord = 0;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  uint32_t word = 0;
  pt_status st = check_hip(hipMemcpyAsync(&word, d_status, 4, hipMemcpyDeviceToHost, s), "status read");
  if (st == PT_OK)
    st = check_hip(hipMemcpyAsync(const_cast<void *>(d_status), &kZeroWord, 4, hipMemcpyHostToDevice, s),
                   "status clear");
  if (st == PT_OK) st = check_hip(hipStreamSynchronize(s), "status wait");
  if (st != PT_OK) return st;
  if (word == 0) return PT_OK;
  return fail(PT_EOVERFLOW, "device status 0x%x:%s%s%s%s", word,
              (word & PT_STATUS_FILTER_OVERFLOW) ? " a filter needed more blocks than its capacity (clamped)" : "",
              (word & PT_STATUS_ENTRIES_OVERFLOW) ? " a partitioned build met more keys than its count" : "",
              (word & PT_STATUS_WAIT_TIMEOUT) ? " a batch item ran without the steps it waited for" : "",
              (word & PT_STATUS_JOIN_OVERFLOW) ? " a join produced more tuples than out_cap (incomplete)" : "");
}

pt_status pt_profile_enable(int on) {
  if (on < 0 || on > 2) return fail(PT_EINVAL, "pt_profile_enable: mode %d", on);
  g_prof_mode = on;
  return PT_OK;
}

pt_status pt_profile_only(const char *name, uint32_t table, uint32_t pass) {
  if (!name || !name[0]) {
    g_prof_only[0] = 0;
    return PT_OK;
  }
  std::snprintf(g_prof_only, sizeof g_prof_only, "%s", name);
  g_prof_only_table = table;
  g_prof_only_pass = pass;
  return PT_OK;
}

pt_status pt_profile_read(pt_kernel_time *out, uint32_t max, uint32_t *n) {
  if (!n || (max > 0 && !out)) return fail(PT_EINVAL, "pt_profile_read: NULL output");
  uint32_t k = 0;
  pt_status st = PT_OK;
  for (ProfRecord &r : g_prof) {
    if (hipEventSynchronize(r.stop) != hipSuccess) st = fail(PT_EDEVICE, "event synchronize failed");
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.start, r.stop) != hipSuccess) ms = -1.f;
    r.t.ms = ms;
    if (k < max) out[k++] = r.t;
    g_event_pool.push_back(r.start);
    g_event_pool.push_back(r.stop);
  }
  g_prof.clear();
  *n = k;
  return st;
}

pt_status pt_local_filter(const pt_table *table, const pt_pred *preds, uint32_t n_preds,
                          uint64_t *d_bitmap, uint64_t *d_count, pt_stream stream) {
  if (!table) return fail(PT_EINVAL, "table is NULL");
  pt_status st = check_table(table, 0);
  if (st != PT_OK) return st;
  if (n_preds > 0 && !preds) return fail(PT_EINVAL, "preds is NULL");
  if (table->n_rows > 0 && !d_bitmap) return fail(PT_EINVAL, "d_bitmap is NULL");
  for (uint32_t i = 0; i < n_preds; i++) {
    if (preds[i].col >= table->n_cols) return fail(PT_EINVAL, "predicate %u: column out of range", i);
    if (preds[i].op > PT_BETWEEN) return fail(PT_EINVAL, "predicate %u: op %u", i, preds[i].op);
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (d_count) {
    Timed tm("zero", 0, 0, 0, 8, s);
    st = check_hip(launch_zero_u64(d_count, 1, s), "zero count");
    if (st != PT_OK) return st;
  }
  uint32_t done = 0;
  do {
    PredSet ps{};
    ps.and_into = done > 0;
    uint64_t bytes = 0;
    for (; done < n_preds && ps.n < kMaxPreds; done++, ps.n++) {
      const pt_column &c = table->cols[preds[done].col];
      ps.p[ps.n] = PredRef{c.data, c.dtype == PT_I64 ? 1u : 0u, preds[done].op, preds[done].lo,
                           preds[done].hi};
      bytes += table->n_rows * key_bytes(c);
    }
    const bool last = done >= n_preds;
    Timed tm("local", 0, 0, table->n_rows, bytes + (table->n_rows + 63) / 64 * 8, s);
    st = check_hip(launch_local_filter(ps, table->n_rows, d_bitmap, last ? d_count : nullptr, s),
                   "local filter launch");
    if (st != PT_OK) return st;
  } while (done < n_preds);
  return PT_OK;
}

pt_status pt_bloom_capacity(uint64_t max_keys, const pt_params *params, uint64_t *out_words) {
  pt_status st = check_params(params);
  if (st != PT_OK) return st;
  if (!out_words) return fail(PT_EINVAL, "out_words is NULL");
  *out_words = capacity_words(max_keys, *params);
  return PT_OK;
}

// Builds n_filters filters, kMaxFilters per scan. With app, filter i reads
// its keys from appended column app_idx[i] - 1.
static pt_status build_filters(uint32_t n_filters, const pt_column *keys, const pt_bloom *filters,
                               uint64_t n_rows, const uint64_t *d_bitmap, const uint64_t *d_count,
                               const BuildScratch *scratch, const AppendSet *app,
                               const uint32_t *app_idx, uint32_t *status, hipStream_t s, uint32_t table,
                               uint32_t pass, bool prune = false) {
  const pt_params &p = filters[0].params;
  for (uint32_t done = 0; done < n_filters;) {
    FilterSet fs{};
    fs.prune = prune ? 1u : 0u;
    uint64_t bytes = (n_rows + 63) / 64 * 8;
    for (; done < n_filters && fs.n < kMaxFilters; done++, fs.n++) {
      fs.f[fs.n] = make_ref(keys[done], filters[done]);
      if (app) fs.f[fs.n].app = app_idx[done];
      bytes += n_rows * key_bytes(keys[done]);
    }
    Timed tm("build", table, pass, n_rows, bytes, s);
    pt_status st = check_hip(launch_build(p.block_bits, p.k, p.bits_per_key, fs, n_rows, d_bitmap,
                                          d_count, scratch, app, status, s),
                             "build launch");
    if (st != PT_OK) return st;
  }
  return PT_OK;
}

// Probes n_filters filters in one scan per group of kMaxProbe. `sel` and
// `rows` (optional) give each filter's builder count and row total, which
// only order the tests. input_all: the bitmap holds every row and is not
// read by the first launch. count_zeroed: *d_count already holds zero.
// app (optional): the last scan appends the survivors' keys (see
// launch_probe); capacity: entries of each appended column.
static pt_status probe_filters(uint32_t n_filters, const pt_column *keys, const pt_bloom *filters,
                               const uint64_t *const *sel, const uint64_t *rows, uint64_t n_rows,
                               uint64_t *d_bitmap, uint64_t *d_count, bool input_all,
                               bool count_zeroed, AppendSet *app, uint64_t capacity, uint32_t *status,
                               hipStream_t s, uint32_t table, uint32_t pass, bool prune = false) {
  const pt_params &p = filters[0].params;
  if (d_count && !count_zeroed) {
    pt_status st = check_hip(launch_zero_u64(d_count, 1, s), "zero count");
    if (st != PT_OK) return st;
  }
  for (uint32_t done = 0; done < n_filters;) {
    FilterSet fs{};
    fs.prune = prune ? 1u : 0u;
    const bool first = done == 0;
    uint64_t bytes = ((input_all && first) ? 1 : 2) * ((n_rows + 63) / 64 * 8);
    for (; done < n_filters && fs.n < kMaxProbe; done++, fs.n++) {
      fs.f[fs.n] = make_ref(keys[done], filters[done]);
      if (sel && rows) {
        fs.f[fs.n].sel = sel[done];
        fs.f[fs.n].rows = rows[done];
      }
      bytes += n_rows * key_bytes(keys[done]);
    }
    const bool last = done >= n_filters;
    Timed tm("probe", table, pass, n_rows, bytes, s);
    pt_status st = check_hip(launch_probe(p.block_bits, p.k, fs, n_rows, d_bitmap,
                                          last ? d_count : nullptr, input_all && first,
                                          last ? app : nullptr, capacity, probe_opts(p), status, s),
                             "probe launch");
    if (st != PT_OK) return st;
  }
  return PT_OK;
}

// The exact set that edge e carries in pass p, read through table v's key
// column (the builder's when building, the receiver's when probing).
static SetRef set_at(const Plan &pl, const pt_graph *g, const pt_table *tables, char *ws, uint32_t p, uint32_t e,
                     uint32_t v) {
  const uint32_t slot = p * pl.n_e + e;
  const pt_column &c = tables[v].cols[col_at(g, e, v)];
  SetRef f{};
  f.keys = reinterpret_cast<unsigned long long *>(ws + pl.off_filter[slot]);
  f.lg = reinterpret_cast<uint64_t *>(ws + pl.off_nb) + slot;
  f.col = c.data;
  f.key64 = c.dtype == PT_I64 ? 1u : 0u;
  f.lg_cap = pl.set_lg[slot];
  return f;
}

// Probes every set table v receives in pass p, kMaxProbe per scan; the last
// scan counts the rows left into *d_count (which holds zero).
static pt_status probe_sets(const Plan &pl, const pt_graph *g, const pt_table *tables, char *ws, uint32_t p,
                            uint32_t v, uint64_t *d_bitmap, uint64_t *d_count, bool input_all,
                            const std::vector<char> &skipped, hipStream_t s) {
  std::vector<uint32_t> in;
  for (uint32_t e = 0; e < pl.n_e; e++)
    if (pl.receives(p, e, v) && !skipped[p * pl.n_e + e]) in.push_back(e);
  for (size_t c0 = 0; c0 < in.size(); c0 += kMaxProbe) {
    SetProbe sp{};
    uint64_t bytes = (c0 == 0 && input_all ? 1 : 2) * ((tables[v].n_rows + 63) / 64 * 8);
    for (size_t j = c0; j < in.size() && sp.n < static_cast<uint32_t>(kMaxProbe); j++) {
      sp.f[sp.n++] = set_at(pl, g, tables, ws, p, in[j], v);
      bytes += tables[v].n_rows * key_bytes(tables[v].cols[col_at(g, in[j], v)]);
    }
    const bool last = c0 + kMaxProbe >= in.size();
    Timed tm("probe", v, p + 1, tables[v].n_rows, bytes, s);
    pt_status st = check_hip(launch_set_probe(sp, tables[v].n_rows, d_bitmap, last ? d_count : nullptr,
                                              input_all && c0 == 0, s),
                             "set probe launch");
    if (st != PT_OK) return st;
  }
  return PT_OK;
}

pt_status pt_bloom_build(uint32_t n_filters, const pt_column *keys, const pt_bloom *filters,
                         uint64_t n_rows, const uint64_t *d_bitmap, const uint64_t *d_count,
                         pt_stream stream) {
  if (n_filters == 0) return PT_OK;
  if (!keys || !filters) return fail(PT_EINVAL, "keys or filters is NULL");
  if (n_rows > kMaxRows) return fail(PT_EINVAL, "%llu rows (limit 2^32 - 1)", (unsigned long long)n_rows);
  if (d_bitmap && !d_count) return fail(PT_EINVAL, "d_count is required with d_bitmap");
  for (uint32_t i = 0; i < n_filters; i++) {
    pt_status st = check_column(&keys[i], n_rows, "build key");
    if (st != PT_OK) return st;
    st = check_filter(filters[i], filters[0].params, n_rows, i);
    if (st != PT_OK) return st;
  }
  if (filters[0].params.flags & PT_FLAG_EXACT) return fail(PT_EUNSUPPORTED, "a pt_bloom is a Bloom filter (PT_FLAG_EXACT)");
  return build_filters(n_filters, keys, filters, n_rows, d_bitmap, d_bitmap ? d_count : nullptr,
                       nullptr, nullptr, nullptr, filters[0].d_status, reinterpret_cast<hipStream_t>(stream), 0,
                       0);
}

pt_status pt_bloom_probe(uint32_t n_filters, const pt_column *keys, const pt_bloom *filters,
                         uint64_t n_rows, uint64_t *d_bitmap, uint64_t *d_count, pt_stream stream) {
  if (!keys && n_filters > 0) return fail(PT_EINVAL, "keys is NULL");
  if (!filters && n_filters > 0) return fail(PT_EINVAL, "filters is NULL");
  if (n_rows > kMaxRows) return fail(PT_EINVAL, "%llu rows (limit 2^32 - 1)", (unsigned long long)n_rows);
  if (n_rows > 0 && !d_bitmap) return fail(PT_EINVAL, "d_bitmap is NULL");
  for (uint32_t i = 0; i < n_filters; i++) {
    pt_status st = check_column(&keys[i], n_rows, "probe key");
    if (st != PT_OK) return st;
    if (!filters[i].words || !filters[i].d_nb) return fail(PT_EINVAL, "filter %u: NULL pointer", i);
    st = check_params(&filters[i].params);
    if (st != PT_OK) return st;
    if (filters[i].cap_words < filters[i].params.block_bits / 32)
      return fail(PT_EINVAL, "filter %u: cap_words below one block", i);
    if (!same_filter(filters[i].params, filters[0].params))
      return fail(PT_EINVAL, "filter %u: parameters differ from filter 0", i);
    if (filters[i].params.flags & PT_FLAG_EXACT)
      return fail(PT_EUNSUPPORTED, "a pt_bloom is a Bloom filter (PT_FLAG_EXACT)");
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (n_filters == 0) {
    if (!d_count) return PT_OK;
    PredSet ps{};
    ps.and_into = 1;  // no filter: the count of the bitmap as it is
    pt_status st = check_hip(launch_zero_u64(d_count, 1, s), "zero count");
    if (st != PT_OK) return st;
    return check_hip(launch_local_filter(ps, n_rows, d_bitmap, d_count, s), "count launch");
  }
  return probe_filters(n_filters, keys, filters, nullptr, nullptr, n_rows, d_bitmap, d_count, false,
                       false, nullptr, 0, filters[0].d_status, s, 0, 0);
}

pt_status pt_compact_workspace_size(uint64_t n_rows, size_t *bytes) {
  if (!bytes) return fail(PT_EINVAL, "bytes is NULL");
  if (n_rows > kMaxRows) return fail(PT_EINVAL, "%llu rows (limit 2^32 - 1)", (unsigned long long)n_rows);
  *bytes = (compact_partials(n_rows) + 1) * 8;
  return PT_OK;
}

pt_status pt_compact(const uint64_t *d_bitmap, uint64_t n_rows, uint32_t *d_idx, uint64_t *d_count,
                     void *d_ws, size_t ws_bytes, pt_stream stream) {
  if (n_rows > kMaxRows) return fail(PT_EINVAL, "%llu rows (limit 2^32 - 1)", (unsigned long long)n_rows);
  if (!d_count) return fail(PT_EINVAL, "d_count is NULL");
  if (n_rows > 0 && (!d_bitmap || !d_idx)) return fail(PT_EINVAL, "d_bitmap or d_idx is NULL");
  size_t need = 0;
  pt_compact_workspace_size(n_rows, &need);
  if (n_rows > 0 && (!d_ws || ws_bytes < need))
    return fail(PT_ENOMEM, "compact workspace %zu < %zu bytes", ws_bytes, need);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  Timed tm("compact", 0, 0, n_rows, (n_rows + 63) / 64 * 16, s);
  return check_hip(launch_compact(d_bitmap, n_rows, d_idx, d_count, static_cast<uint64_t *>(d_ws), s),
                   "compact launch");
}

pt_status pt_compact_noalloc(const uint64_t *d_bitmap, uint64_t n_rows, uint32_t *d_idx, uint64_t *d_count,
                             pt_stream stream) {
  if (n_rows > kStaticCompactRows)
    return fail(PT_EINVAL,
                "pt_compact_noalloc: %llu rows exceed its static scratch (at most 2^31 rows); "
                "use pt_compact with a workspace",
                (unsigned long long)n_rows);
  if (!d_count) return fail(PT_EINVAL, "d_count is NULL");
  if (n_rows > 0 && (!d_bitmap || !d_idx)) return fail(PT_EINVAL, "d_bitmap or d_idx is NULL");
  uint64_t *partials = nullptr;
  pt_status st = check_hip(static_compact_scratch(&partials), "static scratch address");
  if (st != PT_OK) return st;
  return check_hip(launch_compact(d_bitmap, n_rows, d_idx, d_count, partials, reinterpret_cast<hipStream_t>(stream)),
                   "compact launch");
}

pt_status pt_transfer_workspace_size(const pt_graph *graph, const pt_table *tables,
                                     const pt_params *params, size_t *bytes) {
  if (!bytes) return fail(PT_EINVAL, "bytes is NULL");
  Plan pl;
  pt_status st = make_plan(graph, tables, params, pl);
  if (st != PT_OK) return st;
  *bytes = pl.total;
  return PT_OK;
}

pt_status pt_transfer_filter(const pt_graph *graph, const pt_table *tables, const pt_params *params,
                             void *d_ws, uint32_t pass, uint32_t edge, pt_bloom *out,
                             uint32_t *builder) {
  Plan pl;
  pt_status st = make_plan(graph, tables, params, pl);
  if (st != PT_OK) return st;
  if (!out || !d_ws) return fail(PT_EINVAL, "out or d_ws is NULL");
  if (pass < 1 || pass > 2 || edge >= pl.n_e) return fail(PT_EINVAL, "pass %u / edge %u out of range", pass, edge);
  if (pl.exact) return fail(PT_EUNSUPPORTED, "exact filters are key sets, not pt_bloom filters");
  if (!pl.active[(pass - 1) * pl.n_e + edge])
    return fail(PT_EINVAL, "edge %u carries no filter in pass %u (an outer join blocks that direction)", edge, pass);
  char *ws = static_cast<char *>(d_ws);
  const uint64_t slot = (pass - 1) * pl.n_e + edge;
  out->words = reinterpret_cast<uint32_t *>(ws + pl.off_filter[slot]);
  out->cap_words = pl.cap_words[slot];
  out->d_nb = reinterpret_cast<uint64_t *>(ws + pl.off_nb) + slot;
  out->d_status = reinterpret_cast<uint32_t *>(ws);
  out->params = *params;
  if (builder) *builder = pass == 1 ? pl.src[edge] : pl.dst[edge];
  return PT_OK;
}

pt_status pt_transfer(const pt_graph *graph, const pt_table *tables, const pt_pred *preds,
                      uint32_t n_preds, const pt_params *params, void *d_ws, size_t ws_bytes,
                      uint64_t *const *d_bitmaps, uint64_t *d_counts, pt_stream stream) {
  Plan pl;
  pt_status st = make_plan(graph, tables, params, pl);
  if (st != PT_OK) return st;
  if (!d_ws) return fail(PT_EINVAL, "d_ws is NULL");
  if ((reinterpret_cast<uintptr_t>(d_ws) & 255) != 0) return fail(PT_EINVAL, "d_ws is not 256-byte aligned");
  if (ws_bytes < pl.total)
    return fail(PT_ENOMEM, "workspace %zu < %llu bytes", ws_bytes, (unsigned long long)pl.total);
  if (pl.n_t > 0 && !d_bitmaps) return fail(PT_EINVAL, "d_bitmaps is NULL");
  for (uint32_t t = 0; t < pl.n_t; t++)
    if (tables[t].n_rows > 0 && !d_bitmaps[t]) return fail(PT_EINVAL, "d_bitmaps[%u] is NULL", t);
  st = check_preds(pl, tables, preds, n_preds);
  if (st != PT_OK) return st;

  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char *ws = static_cast<char *>(d_ws);
  uint64_t *counts = reinterpret_cast<uint64_t *>(ws + pl.off_counts);
  uint64_t *nbs = reinterpret_cast<uint64_t *>(ws + pl.off_nb);
  uint32_t *status = reinterpret_cast<uint32_t *>(ws);  // the call's status word
  auto bloom_at = [&](uint32_t slot) {
    pt_bloom b{};
    b.words = reinterpret_cast<uint32_t *>(ws + pl.off_filter[slot]);
    b.cap_words = pl.cap_words[slot];
    b.d_nb = nbs + slot;
    b.d_status = status;
    b.params = *params;
    return b;
  };

  {
    // the status word, the counters and the filters' block counts
    // (everything before off_counts is the workspace header); a filter that
    // pruning leaves unbuilt keeps a block count of zero
    const uint64_t words = (pl.off_nb + 2ull * pl.n_e * 8) / 8;
    Timed tm("zero", 0, 0, 0, words * 8, s);
    st = check_hip(launch_zero_u64(reinterpret_cast<uint64_t *>(ws), words, s), "zero counters");
    if (st != PT_OK) return st;
  }

  // Local predicates: every table starts from its own selected rows. A
  // table without predicates keeps all rows; its bitmap is not materialised
  // until something changes it (its first probe writes every word) or the
  // end of the call.
  std::vector<uint32_t> cur(pl.n_t, 0);  // counter slot (0 local, 1 fwd, 2 bwd) holding t's count
  std::vector<char> all_rows(pl.n_t, 1);
  std::vector<pt_pred> mine;
  for (uint32_t t = 0; t < pl.n_t; t++) {
    mine.clear();
    for (uint32_t i = 0; i < n_preds; i++)
      if (preds[i].table == t) mine.push_back(preds[i]);
    if (mine.empty()) continue;
    all_rows[t] = 0;
    const pt_table &tb = tables[t];
    uint64_t *cnt = counts + t;
    uint32_t done = 0;
    do {
      PredSet ps{};
      ps.and_into = done > 0;
      uint64_t bytes = 0;
      for (; done < mine.size() && ps.n < kMaxPreds; done++, ps.n++) {
        const pt_column &c = tb.cols[mine[done].col];
        ps.p[ps.n] = PredRef{c.data, c.dtype == PT_I64 ? 1u : 0u, mine[done].op, mine[done].lo,
                             mine[done].hi};
        bytes += tb.n_rows * key_bytes(c);
      }
      const bool last = done >= mine.size();
      Timed tm("local", t, 0, tb.n_rows, bytes + (tb.n_rows + 63) / 64 * 8, s);
      st = check_hip(launch_local_filter(ps, tb.n_rows, d_bitmaps[t], last ? cnt : nullptr, s),
                     "local filter launch");
      if (st != PT_OK) return st;
    } while (done < mine.size());
  }

  BuildScratch scratch;
  scratch.copies = reinterpret_cast<uint32_t *>(ws + pl.off_scratch);
  scratch.copies_words = pl.scratch_words;
  if (pl.entries_cap) {
    scratch.hist = reinterpret_cast<uint32_t *>(ws + pl.off_hist);
    scratch.hist_groups = pl.hist_groups;
    scratch.totals = reinterpret_cast<uint64_t *>(ws + pl.off_totals);
    scratch.starts = reinterpret_cast<uint64_t *>(ws + pl.off_starts);
    scratch.entries = reinterpret_cast<uint32_t *>(ws + pl.off_entries);
    scratch.entries_cap = pl.entries_cap;
  }

  // The two passes (Sec. 3.2). In pass p (0 forward, 1 backward) the edge e
  // goes from `from[e]` to `to[e]`; tables are visited in `seq`.
  std::vector<uint32_t> rev(pl.order.rbegin(), pl.order.rend());
  std::vector<pt_column> keys;
  std::vector<pt_bloom> blooms;
  std::vector<const uint64_t *> sel;
  std::vector<uint64_t> rows;
  std::vector<const uint64_t *> built_sel(2ull * pl.n_e, nullptr);  // builder count per filter
  // Transfer path pruning (Sec. 3.2): a non-empty table that still holds
  // every row sends no filter. When the host knows it (no predicate, no probe yet)
  // nothing is launched for the filter and its receivers leave it out
  // (skipped); otherwise the builds' size step decides on the device from
  // the builder's count and the probes skip the filters it pruned.
  const bool prune = (params->flags & PT_FLAG_PRUNE) != 0;
  std::vector<char> skipped(2ull * pl.n_e, 0);
  // The appended keys waiting for their builds: table, pass, columns.
  AppendSet pending{};
  uint32_t pending_table = pl.n_t, pending_pass = 2;
  std::vector<uint32_t> pending_cols, app_idx;
  for (uint32_t p = 0; p < 2; p++) {
    const std::vector<uint32_t> &from = p == 0 ? pl.src : pl.dst;
    const std::vector<uint32_t> &seq = p == 0 ? pl.order : rev;
    for (uint32_t v : seq) {
      const pt_table &tb = tables[v];
      // Incoming filters: probe them all in one scan of v.
      keys.clear();
      blooms.clear();
      sel.clear();
      rows.clear();
      for (uint32_t e = 0; e < pl.n_e; e++) {
        if (!pl.receives(p, e, v) || skipped[p * pl.n_e + e]) continue;
        keys.push_back(tb.cols[col_at(graph, e, v)]);
        blooms.push_back(bloom_at(p * pl.n_e + e));
        sel.push_back(built_sel[p * pl.n_e + e]);
        rows.push_back(tables[from[e]].n_rows);
      }
      if (!keys.empty()) {
        uint64_t *cnt = counts + (p + 1) * pl.n_t + v;
        const AppendPlan ap = append_plan(pl, graph, tables, *params, p, v);
        AppendSet app{};
        if (!ap.cols.empty()) {
          char *dst = ws + pl.off_app;
          app.n_cols = static_cast<uint32_t>(ap.cols.size());
          app.counts = reinterpret_cast<uint32_t *>(ws + pl.off_app_counts);
          for (uint32_t c = 0; c < app.n_cols; c++) {
            const pt_column &col = tb.cols[ap.cols[c]];
            app.src[c] = col.data;
            app.key64[c] = col.dtype == PT_I64;
            app.dst[c] = dst;
            dst += align256(append_capacity(tb.n_rows) * key_bytes(col));
          }
        }
        if (pl.exact)
          st = probe_sets(pl, graph, tables, ws, p, v, d_bitmaps[v], cnt, all_rows[v] != 0, skipped, s);
        else
          st = probe_filters(static_cast<uint32_t>(keys.size()), keys.data(), blooms.data(), sel.data(),
                             rows.data(), tb.n_rows, d_bitmaps[v], cnt, all_rows[v] != 0,
                             /*count_zeroed=*/true, ap.cols.empty() ? nullptr : &app,
                             append_capacity(tb.n_rows), status, s, v, p + 1, prune);
        if (st != PT_OK) return st;
        if (app.n_cols > 0) {
          pending = app;
          pending_table = v;
          pending_pass = ap.pass;
          pending_cols = ap.cols;
        }
        cur[v] = p + 1;
        all_rows[v] = 0;
      }
      // Outgoing filters: sized from v's count after this pass's probes.
      const bool use_app = pending_table == v && pending_pass == p && !all_rows[v];
      keys.clear();
      blooms.clear();
      app_idx.clear();
      for (uint32_t e = 0; e < pl.n_e; e++) {
        if (!pl.sends(p, e, v)) continue;
        if (prune && all_rows[v] && tb.n_rows > 0) {
          skipped[p * pl.n_e + e] = 1;
          continue;
        }
        const uint32_t c = col_at(graph, e, v);
        keys.push_back(tb.cols[c]);
        blooms.push_back(bloom_at(p * pl.n_e + e));
        built_sel[p * pl.n_e + e] = all_rows[v] ? nullptr : counts + cur[v] * pl.n_t + v;
        if (use_app)
          app_idx.push_back(static_cast<uint32_t>(
              std::find(pending_cols.begin(), pending_cols.end(), c) - pending_cols.begin() + 1));
      }
      if (!keys.empty() && pl.exact) {
        const bool all = all_rows[v] != 0;
        for (uint32_t e = 0; e < pl.n_e; e++) {
          if (!pl.sends(p, e, v) || skipped[p * pl.n_e + e]) continue;
          Timed tm("build", v, p + 1, tb.n_rows, tb.n_rows * key_bytes(tb.cols[col_at(graph, e, v)]), s);
          st = check_hip(launch_set_build(set_at(pl, graph, tables, ws, p, e, v), tb.n_rows,
                                          all ? nullptr : d_bitmaps[v], all ? nullptr : counts + cur[v] * pl.n_t + v,
                                          prune, s),
                         "set build launch");
          if (st != PT_OK) return st;
        }
      } else if (!keys.empty()) {
        const bool all = all_rows[v] != 0;
        st = build_filters(static_cast<uint32_t>(keys.size()), keys.data(), blooms.data(), tb.n_rows,
                           all ? nullptr : d_bitmaps[v], all ? nullptr : counts + cur[v] * pl.n_t + v,
                           &scratch, use_app ? &pending : nullptr, app_idx.data(), status, s, v, p + 1, prune);
        if (st != PT_OK) return st;
      }
      if (pending_table == v && pending_pass == p) pending_table = pl.n_t;
    }
  }

  // Tables nothing has filtered keep every row.
  for (uint32_t t = 0; t < pl.n_t; t++) {
    if (!all_rows[t]) continue;
    Timed tm("fill", t, 0, tables[t].n_rows, (tables[t].n_rows + 63) / 64 * 8, s);
    st = check_hip(launch_fill_all(d_bitmaps[t], tables[t].n_rows, counts + t, s), "fill launch");
    if (st != PT_OK) return st;
  }

  if (d_counts) {
    std::vector<uint32_t> slot(pl.n_t);
    for (uint32_t t = 0; t < pl.n_t; t++) slot[t] = cur[t] * pl.n_t + t;
    st = check_hip(launch_copy_counts(counts, slot.data(), pl.n_t, d_counts, s), "count copy");
    if (st != PT_OK) return st;
  }
  return PT_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batches

namespace {

// Longest path from a source of pass p (0: forward edges, 1: reversed) to
// every table: the schedule level. Tables of one level depend only on lower
// levels, so listing every problem's tasks level by level gives one order in
// which every task follows the tasks it depends on.
std::vector<uint32_t> levels(const Plan &pl, uint32_t p) {
  std::vector<uint32_t> lvl(pl.n_t, 0);
  std::vector<uint32_t> seq = pl.order;
  if (p == 1) std::reverse(seq.begin(), seq.end());
  for (uint32_t v : seq)
    for (uint32_t e = 0; e < pl.n_e; e++) {
      const uint32_t from = p == 0 ? pl.src[e] : pl.dst[e];
      const uint32_t to = p == 0 ? pl.dst[e] : pl.src[e];
      if (to == v) lvl[v] = std::max(lvl[v], lvl[from] + 1);
    }
  return lvl;
}

constexpr uint32_t kNoTask = 0xFFFFFFFFu;
constexpr uint32_t kMaxBuildParts = 16;     // private copies of one LDS build
constexpr uint32_t kMaxTileItems = 256;     // row tiles of one partitioned build
constexpr uint32_t kMaxFillItems = 256;     // items of one partitioned fill
constexpr uint64_t kDefaultTileRows = 65536;
constexpr uint32_t kBatchSpinMs = 2000;     // longest wait of an item for its dependencies

enum BatchKernel : uint32_t { kKernelGeneric, kKernel512k3, kKernel512k2 };

// The host image of a batch: its task list, argument arrays and workspace
// layout. Device pointers are ws + offset (offsets alone when ws is NULL).
struct BatchPlan {
  std::vector<Plan> plans;
  std::vector<BTask> tasks;
  std::vector<uint32_t> item_task, phase_items, deps;
  std::vector<std::pair<uint32_t, uint32_t>> dep_range;  // per task (host only)
  std::vector<BLocal> locals;
  std::vector<BProbe> probes;
  std::vector<BBuild> builds;
  std::vector<CopyPair> pairs;
  std::vector<BShared> shared;
  uint64_t off_counts = 0, n_counts = 0, off_done = 0, zero_bytes = 0;
  uint32_t n_items = 0;
  uint64_t off_tables = 0, off_timeline = 0, total = 0;
  uint64_t rows_probed = 0, bytes_moved = 0;
  uint32_t kernel = kKernelGeneric;
};

uint32_t div_up32(uint64_t a, uint64_t b) { return static_cast<uint32_t>((a + b - 1) / b); }

// Upper bound of the buckets a partitioned build of these filters uses (its
// bucket count for the filters' actual sizes never exceeds it).
uint32_t bucket_bound(const FilterSet &fs, uint32_t block_bits) {
  const uint64_t W = block_bits / 32, max_tb = kTileWords / W;
  uint64_t cap_blocks = 0;
  for (uint32_t i = 0; i < fs.n; i++) cap_blocks += fs.f[i].cap_words / W;
  const uint64_t bound = std::max<uint64_t>(kBatchTargetBuckets, (cap_blocks + max_tb - 1) / max_tb) + fs.n;
  return static_cast<uint32_t>(std::min<uint64_t>(bound, kMaxBuckets));
}

pt_status plan_batch(uint32_t n_problems, const pt_problem *probs, char *ws, BatchPlan &bp) {
  if (n_problems > 0 && !probs) return fail(PT_EINVAL, "problems is NULL");
  bp.plans.resize(n_problems);
  uint64_t n_counts = 0;
  bool all_512_3 = n_problems > 0, all_512_2 = n_problems > 0;
  uint64_t tile_rows = kDefaultTileRows;
  for (uint32_t i = 0; i < n_problems; i++) {
    const pt_problem &pr = probs[i];
    Plan &pl = bp.plans[i];
    pt_params params = pr.params;
    if (params.flags & PT_FLAG_EXACT) return fail(PT_EUNSUPPORTED, "problem %u: a batch runs Bloom filters only", i);
    params.flags |= PT_FLAG_NO_APPEND;
    pt_status st = make_plan(pr.graph, pr.tables, &params, pl);
    if (st != PT_OK) return fail(st, "problem %u: %s", i, g_error.c_str());
    st = check_preds(pl, pr.tables, pr.preds, pr.n_preds);
    if (st != PT_OK) return fail(st, "problem %u: %s", i, g_error.c_str());
    if (pr.reserved != 0) return fail(PT_EINVAL, "problem %u: reserved field is not 0", i);
    if (ws) {  // the size query needs no output buffers
      if (pl.n_t > 0 && !pr.d_bitmaps) return fail(PT_EINVAL, "problem %u: d_bitmaps is NULL", i);
      for (uint32_t t = 0; t < pl.n_t; t++)
        if (pr.tables[t].n_rows > 0 && !pr.d_bitmaps[t])
          return fail(PT_EINVAL, "problem %u: d_bitmaps[%u] is NULL", i, t);
    }
    for (uint32_t t = 0; t < pl.n_t; t++) {
      uint32_t n = 0;
      for (uint32_t j = 0; j < pr.n_preds; j++) n += pr.preds[j].table == t;
      if (n > static_cast<uint32_t>(kMaxPreds))
        return fail(PT_EUNSUPPORTED, "problem %u table %u: more than %d predicates in a batch", i, t, kMaxPreds);
    }
    if (i == 0 && pr.params.tile_rows) tile_rows = pr.params.tile_rows;
    all_512_3 = all_512_3 && pr.params.block_bits == 512 && pr.params.k == 3;
    all_512_2 = all_512_2 && pr.params.block_bits == 512 && pr.params.k == 2;
    n_counts += 3ull * pl.n_t;
  }
  bp.kernel = all_512_3 ? kKernel512k3 : all_512_2 ? kKernel512k2 : kKernelGeneric;
  const uint64_t words_per_item = tile_rows / 64;
  const uint64_t dyn_lds = static_cast<uint64_t>(device_info().max_lds_block) - 2048;
  const uint64_t lds_words = dyn_lds / 4;
  const uint64_t lds_filter_words = ((dyn_lds - probe_queue_bytes()) / 4) & ~uint64_t(1);

  // Workspace: header (status word, queue head), counters, completion
  // counts (all zeroed at every run), then the problems' filters and the
  // builds' scratch, then the task tables.
  uint64_t off = 256;
  bp.off_counts = off;
  bp.n_counts = n_counts;
  off = align256(off + n_counts * 8);
  auto ptr = [&](uint64_t o) -> char * { return ws ? ws + o : reinterpret_cast<char *>(o); };
  std::vector<uint64_t> counts_of(n_problems);
  {
    uint64_t c = bp.off_counts;
    for (uint32_t i = 0; i < n_problems; i++) {
      counts_of[i] = c;
      c += 3ull * bp.plans[i].n_t * 8;
    }
  }
  auto count_ptr = [&](uint32_t i, uint32_t slot, uint32_t t) {
    return reinterpret_cast<uint64_t *>(ptr(counts_of[i] + (static_cast<uint64_t>(slot) * bp.plans[i].n_t + t) * 8));
  };
  // The task list is built first (its size fixes the completion counters),
  // with scratch offsets relative to `data`, resolved below.
  struct Pending { uint32_t build; uint64_t copies, hist, totals, starts, entries; };
  std::vector<Pending> scratch;
  uint64_t data = 0;  // bytes of build scratch, laid out after the filters
  std::vector<uint64_t> off_problem(n_problems);

  // Tasks are created in an order where every dependency comes first; their
  // phase (depth in the dependency graph) is computed as they are added.
  std::vector<uint32_t> phase_of;
  auto add_task = [&](uint32_t kind, uint32_t items, const std::vector<uint32_t> &deps, uint32_t arg,
                      uint32_t n_arg = 0) {
    BTask t{};
    t.kind = kind;
    t.n_items = std::max<uint32_t>(items, 1);
    const uint32_t begin = static_cast<uint32_t>(bp.deps.size());
    uint32_t phase = 0;
    for (uint32_t d : deps)
      if (d != kNoTask) {
        bp.deps.push_back(d);
        phase = std::max(phase, phase_of[d] + 1);
      }
    t.phase = phase;
    t.arg = arg;
    t.n_arg = n_arg;
    const uint32_t id = static_cast<uint32_t>(bp.tasks.size());
    bp.tasks.push_back(t);
    bp.dep_range.emplace_back(begin, static_cast<uint32_t>(bp.deps.size()));
    phase_of.push_back(phase);
    return id;
  };

  // Filters of every problem (nb slots and words of both passes, at capacity).
  // Their offsets are known once the completion counters are placed, so
  // they are recorded relative to the start of the filter region.
  uint64_t filters_bytes = 0;
  std::vector<std::vector<uint64_t>> filter_off(n_problems);
  for (uint32_t i = 0; i < n_problems; i++) {
    const Plan &pl = bp.plans[i];
    off_problem[i] = filters_bytes;
    uint64_t o = align256(filters_bytes + 2ull * pl.n_e * 8);
    filter_off[i].resize(2ull * pl.n_e);
    for (uint32_t slot = 0; slot < 2 * pl.n_e; slot++) {
      filter_off[i][slot] = o;
      o = align256(o + pl.cap_words[slot] * 4);
    }
    filters_bytes = o;
  }
  // Completion counters: one per phase, at most one phase per task. The
  // number of tasks is bounded by the plan, so reserve that many counters
  // and place everything else after them.
  // Per problem at most: a local filter per table; per pass, a probe chunk
  // per table plus one per four extra incoming edges (fewer than n_t + n_e),
  // and at most five build steps per group of outgoing filters (fewer than
  // n_t + n_e groups); one count copy.
  uint64_t max_tasks = 0;
  for (uint32_t i = 0; i < n_problems; i++) {
    const Plan &pl = bp.plans[i];
    max_tasks += pl.n_t + 2ull * 6 * (pl.n_t + pl.n_e) + 1;
  }
  bp.off_done = off;
  off = align256(off + max_tasks * 4);
  bp.zero_bytes = off;
  const uint64_t off_filters = off;
  off = align256(off + filters_bytes);
  const uint64_t off_scratch = off;

  auto filter_ref = [&](uint32_t i, uint32_t p, uint32_t e, uint32_t table) {
    const Plan &pl = bp.plans[i];
    const uint32_t slot = p * pl.n_e + e;
    FilterRef r{};
    const pt_column &c = probs[i].tables[table].cols[col_at(probs[i].graph, e, table)];
    r.keys = c.data;
    r.key64 = c.dtype == PT_I64;
    r.words = reinterpret_cast<uint32_t *>(ptr(off_filters + filter_off[i][slot]));
    r.nb = reinterpret_cast<uint64_t *>(ptr(off_filters + off_problem[i] + slot * 8ull));
    r.cap_words = pl.cap_words[slot];
    return r;
  };

  // 1. Local predicates of every table (tables without predicates get
  // every row, so every bitmap is materialised).
  std::vector<std::vector<uint32_t>> writer(n_problems), cur(n_problems);
  std::vector<std::vector<std::vector<uint32_t>>> readers(n_problems);
  std::vector<std::vector<uint32_t>> final_of(n_problems);  // task that finishes filter slot
  for (uint32_t i = 0; i < n_problems; i++) {
    const Plan &pl = bp.plans[i];
    const pt_problem &pr = probs[i];
    writer[i].assign(pl.n_t, kNoTask);
    cur[i].assign(pl.n_t, 0);
    readers[i].assign(pl.n_t, {});
    final_of[i].assign(2ull * pl.n_e, kNoTask);
    for (uint32_t t = 0; t < pl.n_t; t++) {
      const pt_table &tb = pr.tables[t];
      if (tb.n_rows == 0) continue;
      BLocal l{};
      for (uint32_t j = 0; j < pr.n_preds; j++) {
        if (pr.preds[j].table != t) continue;
        const pt_column &c = tb.cols[pr.preds[j].col];
        l.ps.p[l.ps.n++] = PredRef{c.data, c.dtype == PT_I64 ? 1u : 0u, pr.preds[j].op, pr.preds[j].lo,
                                   pr.preds[j].hi};
        bp.bytes_moved += tb.n_rows * key_bytes(c);
      }
      const uint64_t n_words = (tb.n_rows + 63) / 64;
      const uint32_t items = div_up32(n_words, words_per_item);
      l.n_rows = tb.n_rows;
      l.bitmap = ws ? pr.d_bitmaps[t] : nullptr;
      l.count = count_ptr(i, 0, t);
      l.seg_words = std::min<uint32_t>(64, std::max<uint32_t>(1, div_up32(n_words, uint64_t(items) * 16)));
      bp.bytes_moved += n_words * 8;
      writer[i][t] = add_task(kBLocal, items, {}, static_cast<uint32_t>(bp.locals.size()));
      bp.locals.push_back(l);
    }
  }

  // 2. Both passes, level by level over all problems: the probes of a level,
  // then the builds of the filters its tables send.
  bool missing_filter = false;
  std::vector<std::vector<uint32_t>> lvl[2];
  uint32_t max_lvl = 0;
  for (uint32_t p = 0; p < 2; p++) {
    lvl[p].resize(n_problems);
    for (uint32_t i = 0; i < n_problems; i++) {
      lvl[p][i] = levels(bp.plans[i], p);
      for (uint32_t v : lvl[p][i]) max_lvl = std::max(max_lvl, v);
    }
  }
  // Probes whose smallest filter is too large for LDS (per bp.probes
  // entry): their items are cut kCacheProbeSplit times smaller and counted
  // kCacheProbeCost times dearer per row when the items are ordered.
  constexpr uint64_t kCacheProbeSplit = 4;
  constexpr double kCacheProbeCost = 3.0;
  std::vector<char> probe_from_cache;
  // A probe a shared scan may take: the only probe of a large table in its
  // pass (tasks are created once the level's candidates are grouped).
  struct ProbeCand {
    uint32_t i, v;
    BProbe pt;
    std::vector<uint32_t> deps;
    uint64_t n_words, bytes;
  };
  auto emit_probe = [&](const ProbeCand &c) {
    // Every item first copies the filters into its LDS when they fit
    // there: give it at least eight times their size in keys. When even
    // the smallest filter is too large for LDS, every row's test reads
    // the filter from the caches at random, several times slower per row:
    // smaller items keep the phase's last items short.
    uint64_t filter_words = 0, min_words = ~0ull;
    for (uint32_t j = 0; j < c.pt.fs.n; j++) {
      filter_words += c.pt.fs.f[j].cap_words;
      min_words = std::min<uint64_t>(min_words, c.pt.fs.f[j].cap_words);
    }
    const uint64_t staged = filter_words <= lds_filter_words ? filter_words : 0;
    const bool from_cache = min_words > lds_filter_words;
    const uint64_t probe_words = from_cache ? std::max<uint64_t>(64, words_per_item / kCacheProbeSplit)
                                            : std::max<uint64_t>(words_per_item, staged * 4 * 8 / (64 * 4));
    probe_from_cache.push_back(from_cache);
    bp.bytes_moved += c.bytes;
    writer[c.i][c.v] = add_task(kBProbe, div_up32(c.n_words, probe_words), c.deps,
                                static_cast<uint32_t>(bp.probes.size()));
    readers[c.i][c.v].clear();
    bp.probes.push_back(c.pt);
  };
  // Groups probes of one level that scan tables of the same rows with the
  // same filter shape, as long as their key columns (pointer and width)
  // number at most kMaxSharedCols together; a group of one is a plain probe.
  auto emit_shared = [&](std::vector<ProbeCand> &cands) {
    struct Group {
      std::vector<size_t> members;
      std::vector<std::pair<const void *, uint32_t>> cols;
    };
    std::vector<Group> done;
    std::map<std::tuple<uint64_t, uint32_t, uint32_t>, Group> open;
    for (size_t ci = 0; ci < cands.size(); ci++) {
      const ProbeCand &c = cands[ci];
      const auto key = std::make_tuple(c.pt.n_rows, c.pt.k, c.pt.lg);
      Group &g = open[key];
      auto cols = g.cols;
      for (uint32_t j = 0; j < c.pt.fs.n; j++) {
        const auto col = std::make_pair(c.pt.fs.f[j].keys, c.pt.fs.f[j].key64);
        if (std::find(cols.begin(), cols.end(), col) == cols.end()) cols.push_back(col);
      }
      if (!g.members.empty() &&
          (cols.size() > static_cast<size_t>(kMaxSharedCols) || g.members.size() >= static_cast<size_t>(kMaxSharedMembers))) {
        done.push_back(std::move(g));
        g = Group{};
        cols.clear();
        for (uint32_t j = 0; j < c.pt.fs.n; j++) {
          const auto col = std::make_pair(c.pt.fs.f[j].keys, c.pt.fs.f[j].key64);
          if (std::find(cols.begin(), cols.end(), col) == cols.end()) cols.push_back(col);
        }
      }
      g.members.push_back(ci);
      g.cols = std::move(cols);
    }
    for (auto &kv : open)
      if (!kv.second.members.empty()) done.push_back(std::move(kv.second));
    std::sort(done.begin(), done.end(), [](const Group &x, const Group &y) { return x.members[0] < y.members[0]; });
    for (const Group &g : done) {
      if (g.members.size() == 1) {
        emit_probe(cands[g.members[0]]);
        continue;
      }
      BShared sh{};
      const ProbeCand &c0 = cands[g.members[0]];
      sh.n_rows = c0.pt.n_rows;
      sh.n_members = static_cast<uint32_t>(g.members.size());
      sh.n_cols = static_cast<uint32_t>(g.cols.size());
      sh.first_probe = static_cast<uint32_t>(bp.probes.size());
      for (uint32_t c = 0; c < sh.n_cols; c++) {
        sh.cols[c] = g.cols[c].first;
        sh.key64[c] = g.cols[c].second;
        bp.bytes_moved += sh.n_rows * (g.cols[c].second ? 8 : 4);
      }
      std::vector<uint32_t> deps;
      for (uint32_t m = 0; m < sh.n_members; m++) {
        const ProbeCand &c = cands[g.members[m]];
        for (uint32_t j = 0; j < c.pt.fs.n; j++) {
          const auto col = std::make_pair(c.pt.fs.f[j].keys, c.pt.fs.f[j].key64);
          sh.col_of[m][j] = static_cast<uint8_t>(std::find(g.cols.begin(), g.cols.end(), col) - g.cols.begin());
        }
        deps.insert(deps.end(), c.deps.begin(), c.deps.end());
        bp.probes.push_back(c.pt);
        probe_from_cache.push_back(0);
        bp.bytes_moved += 2 * c.n_words * 8;
      }
      const uint32_t id = add_task(kBShared, div_up32(c0.n_words, words_per_item), deps,
                                   static_cast<uint32_t>(bp.shared.size()));
      bp.shared.push_back(sh);
      for (size_t ci : g.members) {
        writer[cands[ci].i][cands[ci].v] = id;
        readers[cands[ci].i][cands[ci].v].clear();
      }
    }
    cands.clear();
  };
  std::vector<ProbeCand> cands;
  for (uint32_t p = 0; p < 2; p++) {
    for (uint32_t L = 0; L <= max_lvl; L++) {
      for (uint32_t i = 0; i < n_problems; i++) {
        const Plan &pl = bp.plans[i];
        const pt_problem &pr = probs[i];
        const uint32_t lg = log2_of(static_cast<int>(pr.params.block_bits));
        for (uint32_t v = 0; v < pl.n_t; v++) {
          if (lvl[p][i][v] != L || pr.tables[v].n_rows == 0) continue;
          std::vector<uint32_t> in;
          for (uint32_t e = 0; e < pl.n_e; e++)
            if (pl.receives(p, e, v)) in.push_back(e);
          if (in.empty()) continue;
          bp.rows_probed += pr.tables[v].n_rows;
          const uint64_t n_rows = pr.tables[v].n_rows, n_words = (n_rows + 63) / 64;
          for (uint32_t c0 = 0; c0 < in.size(); c0 += kMaxProbe) {
            ProbeCand c{i, v, BProbe{}, {writer[i][v]}, n_words, 2 * n_words * 8};
            BProbe &pt = c.pt;
            pt.fs.prune = (pr.params.flags & PT_FLAG_PRUNE) ? 1u : 0u;
            c.deps.insert(c.deps.end(), readers[i][v].begin(), readers[i][v].end());
            for (uint32_t j = c0; j < in.size() && pt.fs.n < static_cast<uint32_t>(kMaxProbe); j++) {
              const uint32_t e = in[j];
              const uint32_t from = p == 0 ? pl.src[e] : pl.dst[e];
              FilterRef r = filter_ref(i, p, e, v);
              if (pr.params.probe_order != PT_PROBE_GIVEN) {
                r.sel = count_ptr(i, cur[i][from], from);
                r.rows = pr.tables[from].n_rows;
              }
              c.bytes += n_rows * (r.key64 ? 8 : 4);
              pt.fs.f[pt.fs.n++] = r;
              missing_filter = missing_filter || final_of[i][p * pl.n_e + e] == kNoTask;
              c.deps.push_back(final_of[i][p * pl.n_e + e]);
            }
            const bool last = c0 + kMaxProbe >= in.size();
            pt.n_rows = n_rows;
            pt.bitmap = ws ? pr.d_bitmaps[v] : nullptr;
            pt.count = last ? count_ptr(i, p + 1, v) : nullptr;
            pt.k = pr.params.k;
            pt.lg = lg;
            // The only probe of a large table may join a shared scan.
            if (in.size() <= static_cast<size_t>(kMaxProbe) && n_rows >= kSharedMinRows &&
                (pr.params.flags & PT_FLAG_SHARED_SCAN) && !(pr.params.flags & PT_FLAG_PRUNE))
              cands.push_back(std::move(c));
            else
              emit_probe(c);
          }
          cur[i][v] = p + 1;
        }
      }
      emit_shared(cands);
      for (uint32_t i = 0; i < n_problems; i++) {
        const Plan &pl = bp.plans[i];
        const pt_problem &pr = probs[i];
        const uint32_t lg = log2_of(static_cast<int>(pr.params.block_bits));
        for (uint32_t v = 0; v < pl.n_t; v++) {
          if (lvl[p][i][v] != L) continue;
          std::vector<uint32_t> out;
          for (uint32_t e = 0; e < pl.n_e; e++)
            if (pl.sends(p, e, v)) out.push_back(e);
          const uint64_t n_rows = pr.tables[v].n_rows, n_words = (n_rows + 63) / 64;
          for (uint32_t c0 = 0; c0 < out.size(); c0 += kMaxFilters) {
            BBuild b{};
            b.fs.prune = (pr.params.flags & PT_FLAG_PRUNE) ? 1u : 0u;
            for (uint32_t j = c0; j < out.size() && b.fs.n < static_cast<uint32_t>(kMaxFilters); j++)
              b.fs.f[b.fs.n++] = filter_ref(i, p, out[j], v);
            b.n_rows = n_rows;
            b.bitmap = (ws && n_rows) ? pr.d_bitmaps[v] : nullptr;
            b.count = count_ptr(i, cur[i][v], v);
            b.k = pr.params.k;
            b.lg = lg;
            b.bits_per_key = pr.params.bits_per_key;
            uint64_t cap_words = 0;
            for (uint32_t j = 0; j < b.fs.n; j++) cap_words += b.fs.f[j].cap_words;
            const uint32_t arg = static_cast<uint32_t>(bp.builds.size());
            Pending sc{arg, 0, 0, 0, 0, 0};
            uint32_t fin;
            if (cap_words <= lds_words) {
              // Small filters: private LDS copies, then an OR of the copies.
              b.n_parts = std::min<uint32_t>(kMaxBuildParts, std::max<uint32_t>(1, div_up32(n_words, words_per_item)));
              b.copy_words = static_cast<uint32_t>(cap_words);
              b.seg_words = std::min<uint32_t>(64, std::max<uint32_t>(1, div_up32(n_words, uint64_t(b.n_parts) * 16)));
              sc.copies = data;
              data = align256(data + uint64_t(b.n_parts) * b.copy_words * 4);
              const uint32_t build = add_task(kBBuild, b.n_parts, {writer[i][v]}, arg);
              fin = add_task(kBReduce, div_up32(cap_words, kReduceWords), {build}, arg);
              readers[i][v].push_back(build);
            } else {
              // Large filters: partitioned build, row tiles then filter tiles.
              const uint32_t tiles = std::min<uint32_t>(kMaxTileItems,
                                                        std::max<uint32_t>(1, div_up32(n_words, words_per_item)));
              b.hist_rows = tiles;
              b.hist_cols = bucket_bound(b.fs, pr.params.block_bits);
              b.seg_words = std::min<uint32_t>(64, std::max<uint32_t>(1, div_up32(n_words, uint64_t(tiles) * 16)));
              b.entries_cap = std::min<uint64_t>(n_rows * b.fs.n, kMaxEntries);
              if (b.entries_cap == 0) b.entries_cap = 1;
              sc.hist = data;
              data = align256(data + uint64_t(b.hist_rows) * b.hist_cols * 4);
              sc.totals = data;
              data = align256(data + uint64_t(b.hist_cols) * 8);
              sc.starts = data;
              data = align256(data + (uint64_t(b.hist_cols) + 1) * 8);
              sc.entries = data;
              data = align256(data + b.entries_cap * 4);
              // The plan may not fit at run time (more keys than entries, or
              // more buckets than the table): the filters are then zeroed
              // and built with atomics.
              uint32_t first_dep = writer[i][v];
              if (n_rows * b.fs.n > b.entries_cap || b.hist_cols >= kMaxBuckets)
                first_dep = add_task(kBZero, div_up32(cap_words, kZeroWords), {writer[i][v]}, arg);
              const uint32_t count = add_task(kBCount, tiles, {writer[i][v], first_dep}, arg);
              const uint32_t scan = add_task(kBScan, 1, {count}, arg);
              const uint32_t scatter = add_task(kBScatter, tiles, {scan}, arg);
              fin = add_task(kBFill, std::min<uint32_t>(kMaxFillItems, b.hist_cols), {scatter}, arg);
              readers[i][v].push_back(count);
              readers[i][v].push_back(scatter);
            }
            for (uint32_t j = c0; j < out.size() && j < c0 + kMaxFilters; j++) final_of[i][p * pl.n_e + out[j]] = fin;
            bp.builds.push_back(b);
            scratch.push_back(sc);
          }
        }
      }
    }
  }
  // 3. Final counts to the callers' arrays.
  for (uint32_t i = 0; i < n_problems; i++) {
    if (ws && !probs[i].d_counts) continue;
    const Plan &pl = bp.plans[i];
    std::vector<uint32_t> deps;
    const uint32_t first = static_cast<uint32_t>(bp.pairs.size());
    for (uint32_t t = 0; t < pl.n_t; t++) {
      bp.pairs.push_back(CopyPair{count_ptr(i, cur[i][t], t), ws ? probs[i].d_counts + t : nullptr});
      deps.push_back(writer[i][t]);
    }
    add_task(kBCopy, 1, deps, first, pl.n_t);
  }
  if (bp.tasks.size() > max_tasks) return fail(PT_EDEVICE, "batch planner: %zu tasks over its bound", bp.tasks.size());
  // The list in phase order (stable): items of a phase follow every item of
  // the phases before it.
  {
    // Within a phase the longest items go first, so that the phase's last
    // items are short and few workgroups wait at its end.
    std::vector<double> cost(bp.tasks.size(), 0.0);
    for (uint32_t t = 0; t < bp.tasks.size(); t++) {
      const BTask &k = bp.tasks[t];
      const double items = k.n_items;
      switch (k.kind) {
        case kBLocal: cost[t] = bp.locals[k.arg].n_rows * (1.0 + bp.locals[k.arg].ps.n) / items; break;
        case kBProbe:
          cost[t] = bp.probes[k.arg].n_rows * (1.0 + bp.probes[k.arg].fs.n) / items *
                    (probe_from_cache[k.arg] ? kCacheProbeCost : 1.0);
          break;
        case kBShared: cost[t] = bp.shared[k.arg].n_rows * (1.0 + bp.shared[k.arg].n_members) / items; break;
        case kBBuild:
        case kBCount:
        case kBScatter:
        case kBFill: cost[t] = bp.builds[k.arg].n_rows * (1.0 + bp.builds[k.arg].fs.n) / items; break;
        case kBScan: cost[t] = 1.0 * bp.builds[k.arg].hist_cols * bp.builds[k.arg].hist_rows; break;
        case kBReduce:
        case kBZero: cost[t] = 4096.0; break;
        default: cost[t] = 0.0;
      }
    }
    std::vector<uint32_t> order(bp.tasks.size());
    for (uint32_t t = 0; t < order.size(); t++) order[t] = t;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
      if (bp.tasks[x].phase != bp.tasks[y].phase) return bp.tasks[x].phase < bp.tasks[y].phase;
      return cost[x] > cost[y];
    });
    std::vector<BTask> sorted;
    sorted.reserve(order.size());
    uint32_t n_phases = 0;
    for (uint32_t t : order) {
      BTask task = bp.tasks[t];
      task.first_item = static_cast<uint32_t>(bp.item_task.size());
      bp.item_task.insert(bp.item_task.end(), task.n_items, static_cast<uint32_t>(sorted.size()));
      n_phases = std::max(n_phases, task.phase + 1);
      sorted.push_back(task);
    }
    bp.phase_items.assign(n_phases, 0);
    for (const BTask &task : sorted) bp.phase_items[task.phase] += task.n_items;
    for (uint32_t t = 0; t < bp.tasks.size(); t++)
      for (uint32_t d = bp.dep_range[t].first; d < bp.dep_range[t].second; d++)
        if (bp.tasks[bp.deps[d]].phase >= bp.tasks[t].phase)
          return fail(PT_EDEVICE, "batch planner: task %u does not follow its dependency", t);
    bp.tasks = std::move(sorted);
    bp.n_items = static_cast<uint32_t>(bp.item_task.size());
  }
  if (missing_filter) return fail(PT_EDEVICE, "batch planner: a probe precedes the build of its filter");

  // Scratch offsets, then the tables.
  for (const Pending &sc : scratch) {
    BBuild &b = bp.builds[sc.build];
    if (b.copy_words) b.copies = reinterpret_cast<uint32_t *>(ptr(off_scratch + sc.copies));
    if (b.hist_rows) {
      b.hist = reinterpret_cast<uint32_t *>(ptr(off_scratch + sc.hist));
      b.totals = reinterpret_cast<uint64_t *>(ptr(off_scratch + sc.totals));
      b.starts = reinterpret_cast<uint64_t *>(ptr(off_scratch + sc.starts));
      b.entries = reinterpret_cast<uint32_t *>(ptr(off_scratch + sc.entries));
    }
  }
  off = align256(off_scratch + data);
  bp.off_tables = off;
  auto table_bytes = [](size_t n, size_t sz) { return align256(static_cast<uint64_t>(n * sz)); };
  off += table_bytes(bp.tasks.size(), sizeof(BTask)) + table_bytes(bp.item_task.size(), 4) +
         table_bytes(bp.phase_items.size(), 4) + table_bytes(bp.locals.size(), sizeof(BLocal)) +
         table_bytes(bp.probes.size(), sizeof(BProbe)) + table_bytes(bp.builds.size(), sizeof(BBuild)) +
         table_bytes(bp.pairs.size(), sizeof(CopyPair)) + table_bytes(bp.shared.size(), sizeof(BShared));
  // PT_BATCH_TIMELINE=1 (profiling): room for every item's start and end.
  if (const char *tl = std::getenv("PT_BATCH_TIMELINE"); tl && std::strcmp(tl, "1") == 0) {
    bp.off_timeline = off;
    off = align256(off + 16ull * bp.n_items);
  }
  bp.total = off;
  return PT_OK;
}

}  // namespace

struct pt_batch {
  int device = 0;
  char *ws = nullptr;
  std::vector<char> staging;  // host image of the task tables
  BatchArgs args{};
  uint32_t kernel = kKernelGeneric;
  uint32_t grid = 0;
  uint64_t lds_bytes = 0, zero_bytes = 0, rows_probed = 0, bytes_moved = 0;
  uint32_t n_tasks = 0, n_phases = 0, rate_khz = 0;
  std::vector<uint32_t> item_kind, item_phase;  // per item, for the timeline
  hipStream_t capture = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static pt_status enqueue_batch(const pt_batch &b, hipStream_t s, bool timed) {
  pt_status st = check_hip(launch_zero_u64(reinterpret_cast<uint64_t *>(b.ws), b.zero_bytes / 8, s), "batch zero");
  if (st != PT_OK) return st;
  Timed tm(timed ? "batch" : nullptr, b.n_tasks, 0, b.rows_probed, b.bytes_moved, s);
  hipError_t e;
  switch (b.kernel) {
    case kKernel512k3: e = launch_batch_512_k3(b.args, b.grid, b.lds_bytes, s); break;
    case kKernel512k2: e = launch_batch_512_k2(b.args, b.grid, b.lds_bytes, s); break;
    default: e = launch_batch_generic(b.args, b.grid, b.lds_bytes, s); break;
  }
  return check_hip(e, "batch launch");
}

extern "C" {

pt_status pt_batch_workspace_size(uint32_t n_problems, const pt_problem *problems, size_t *bytes) {
  if (!bytes) return fail(PT_EINVAL, "bytes is NULL");
  BatchPlan bp;
  pt_status st = plan_batch(n_problems, problems, nullptr, bp);
  if (st != PT_OK) return st;
  *bytes = bp.total;
  return PT_OK;
}

pt_status pt_batch_prepare(uint32_t n_problems, const pt_problem *problems, void *d_ws, size_t ws_bytes,
                           pt_batch **out) {
  pt_status st = pt_batch_prepare_async(n_problems, problems, d_ws, ws_bytes, nullptr, out);
  if (st != PT_OK) return st;
  st = check_hip(hipDeviceSynchronize(), "task table copy");
  if (st != PT_OK) {
    pt_batch_free(*out);
    *out = nullptr;
  }
  return st;
}

pt_status pt_batch_prepare_async(uint32_t n_problems, const pt_problem *problems, void *d_ws, size_t ws_bytes,
                                 pt_stream stream, pt_batch **out) {
  if (!out) return fail(PT_EINVAL, "out is NULL");
  *out = nullptr;
  if (!d_ws) return fail(PT_EINVAL, "d_ws is NULL");
  if ((reinterpret_cast<uintptr_t>(d_ws) & 255) != 0) return fail(PT_EINVAL, "d_ws is not 256-byte aligned");
  BatchPlan bp;
  pt_status st = plan_batch(n_problems, problems, static_cast<char *>(d_ws), bp);
  if (st != PT_OK) return st;
  if (ws_bytes < bp.total)
    return fail(PT_ENOMEM, "workspace %zu < %llu bytes", ws_bytes, (unsigned long long)bp.total);
  // Raise the LDS limits now: the capture must not change kernel attributes.
  st = check_hip(prepare_batch_kernels(), "batch kernel setup");
  if (st != PT_OK) return st;
  char *ws = static_cast<char *>(d_ws);
  auto *b = new pt_batch();
  // The task tables go to the workspace in one asynchronous copy on
  // `stream`, from a host buffer the handle keeps until it is freed.
  b->staging.assign((bp.off_timeline ? bp.off_timeline : bp.total) - bp.off_tables, 0);
  uint64_t o = 0;
  auto put = [&](const void *src, size_t n, size_t sz) {
    const uint64_t at = o;
    if (n) std::memcpy(b->staging.data() + o, src, n * sz);
    o += align256(static_cast<uint64_t>(n * sz));
    return ws + bp.off_tables + at;
  };
  BatchArgs &a = b->args;
  a.tasks = reinterpret_cast<const BTask *>(put(bp.tasks.data(), bp.tasks.size(), sizeof(BTask)));
  a.item_task = reinterpret_cast<const uint32_t *>(put(bp.item_task.data(), bp.item_task.size(), 4));
  a.phase_items = reinterpret_cast<const uint32_t *>(put(bp.phase_items.data(), bp.phase_items.size(), 4));
  a.locals = reinterpret_cast<const BLocal *>(put(bp.locals.data(), bp.locals.size(), sizeof(BLocal)));
  a.probes = reinterpret_cast<const BProbe *>(put(bp.probes.data(), bp.probes.size(), sizeof(BProbe)));
  a.builds = reinterpret_cast<const BBuild *>(put(bp.builds.data(), bp.builds.size(), sizeof(BBuild)));
  a.pairs = reinterpret_cast<const CopyPair *>(put(bp.pairs.data(), bp.pairs.size(), sizeof(CopyPair)));
  a.shared = reinterpret_cast<const BShared *>(put(bp.shared.data(), bp.shared.size(), sizeof(BShared)));
  a.status = reinterpret_cast<uint32_t *>(ws);
  a.head = reinterpret_cast<uint32_t *>(ws + 4);
  a.phase_done = reinterpret_cast<uint32_t *>(ws + bp.off_done);
  a.n_items = bp.n_items;
  a.n_phases = static_cast<uint32_t>(bp.phase_items.size());
  const uint64_t lds_bytes = static_cast<uint64_t>(device_info().max_lds_block) - 2048;
  a.lds_filter_words = static_cast<uint32_t>((lds_bytes - probe_queue_bytes()) / 4) & ~1u;
  a.lds_bytes = static_cast<uint32_t>(lds_bytes);
  int rate_khz = 0;
  if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, device_info().device) != hipSuccess ||
      rate_khz <= 0)
    rate_khz = 100000;
  a.spin_limit = static_cast<uint64_t>(rate_khz) * kBatchSpinMs;
  a.timeline = bp.off_timeline ? reinterpret_cast<uint64_t *>(ws + bp.off_timeline) : nullptr;
  b->rate_khz = static_cast<uint32_t>(rate_khz);
  b->item_kind.resize(bp.n_items);
  b->item_phase.resize(bp.n_items);
  for (const BTask &t : bp.tasks)
    for (uint32_t j = 0; j < t.n_items; j++) {
      b->item_kind[t.first_item + j] = t.kind;
      b->item_phase[t.first_item + j] = t.phase;
    }
  if (!b->staging.empty()) {
    st = check_hip(hipMemcpyAsync(ws + bp.off_tables, b->staging.data(), b->staging.size(), hipMemcpyHostToDevice,
                                  reinterpret_cast<hipStream_t>(stream)),
                   "task table copy");
    if (st != PT_OK) {
      pt_batch_free(b);
      return st;
    }
  }
  if (hipGetDevice(&b->device) != hipSuccess) b->device = 0;
  b->ws = ws;
  b->kernel = bp.kernel;
  b->grid = static_cast<uint32_t>(device_info().n_cu);
  b->lds_bytes = lds_bytes;
  b->zero_bytes = bp.zero_bytes;
  b->rows_probed = bp.rows_probed;
  b->bytes_moved = bp.bytes_moved;
  b->n_tasks = static_cast<uint32_t>(bp.tasks.size());
  b->n_phases = static_cast<uint32_t>(bp.phase_items.size());
  *out = b;
  return PT_OK;
}

pt_status pt_batch_run(pt_batch *b, pt_stream stream, uint32_t flags) {
  if (!b) return fail(PT_EINVAL, "batch is NULL");
  if (flags & ~PT_BATCH_EAGER) return fail(PT_EINVAL, "unknown flags 0x%x", flags);
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (flags & PT_BATCH_EAGER) return enqueue_batch(*b, s, true);
  if (!b->exec) {
    pt_status st = check_hip(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking), "capture stream");
    if (st != PT_OK) return st;
    st = check_hip(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal), "begin capture");
    if (st != PT_OK) return st;
    pt_status enq = enqueue_batch(*b, b->capture, false);
    hipGraph_t g = nullptr;
    st = check_hip(hipStreamEndCapture(b->capture, &g), "end capture");
    if (enq != PT_OK) {
      if (g) (void)hipGraphDestroy(g);
      return enq;
    }
    if (st != PT_OK) return st;
    b->graph = g;
    st = check_hip(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0), "graph instantiate");
    if (st != PT_OK) return st;
  }
  return check_hip(hipGraphLaunch(b->exec, s), "graph launch");
}

pt_status pt_batch_timeline(const pt_batch *b, uint64_t *out, uint32_t max_items, uint32_t *n_items,
                            uint32_t *ticks_per_ms) {
  if (!b || !n_items) return fail(PT_EINVAL, "batch or n_items is NULL");
  if (!b->args.timeline) return fail(PT_EUNSUPPORTED, "the batch was prepared without PT_BATCH_TIMELINE=1");
  const uint32_t n = std::min<uint32_t>(max_items, b->args.n_items);
  if (n > 0 && !out) return fail(PT_EINVAL, "out is NULL");
  std::vector<uint64_t> se(2ull * n);
  pt_status st = check_hip(hipDeviceSynchronize(), "timeline wait");
  if (st == PT_OK && n)
    st = check_hip(hipMemcpy(se.data(), b->args.timeline, se.size() * 8, hipMemcpyDeviceToHost), "timeline read");
  if (st != PT_OK) return st;
  for (uint32_t i = 0; i < n; i++) {
    out[4ull * i] = se[2ull * i];
    out[4ull * i + 1] = se[2ull * i + 1];
    out[4ull * i + 2] = b->item_kind[i];
    out[4ull * i + 3] = b->item_phase[i];
  }
  *n_items = n;
  if (ticks_per_ms) *ticks_per_ms = b->rate_khz;
  return PT_OK;
}

pt_status pt_batch_info(const pt_batch *b, uint32_t *n_launches, uint64_t *rows_probed) {
  if (!b) return fail(PT_EINVAL, "batch is NULL");
  if (n_launches) *n_launches = 2;  // the counter reset and the persistent kernel
  if (rows_probed) *rows_probed = b->rows_probed;
  return PT_OK;
}

void pt_batch_free(pt_batch *b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  delete b;
}

pt_status pt_transfer_batch(uint32_t n_problems, const pt_problem *problems, void *d_ws, size_t ws_bytes,
                            pt_stream stream) {
  pt_batch *b = nullptr;
  pt_status st = pt_batch_prepare(n_problems, problems, d_ws, ws_bytes, &b);
  if (st != PT_OK) return st;
  st = pt_batch_run(b, stream, PT_BATCH_EAGER);
  if (st == PT_OK) st = check_hip(hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream)), "batch wait");
  pt_batch_free(b);
  return st;
}

}  // extern "C"

// ---------------------------------------------------------------- join phase

namespace {

// The join phase's plan: the component's tables in breadth-first order from
// the root, for each added table its lookup edge (the lowest-indexed edge to
// a table added before it) and the other edges to those tables, and the
// workspace layout.
struct JoinPlan {
  std::vector<uint32_t> order;
  std::vector<int> pos;  // place of each table in the tuples, -1 outside the component
  std::vector<uint32_t> lookup;
  std::vector<std::vector<uint32_t>> checks;
  std::vector<uint32_t> lg_cap;
  std::vector<uint64_t> off_ids, off_keys, off_heads, off_next;
  uint64_t off_counts = 0, off_partials = 0, off_tuples[2] = {0, 0}, total = 0;
};

uint32_t ceil_log2(uint64_t x) {
  uint32_t lg = 0;
  while ((1ull << lg) < x) lg++;
  return lg;
}

pt_status make_join_plan(const pt_graph *g, const pt_table *tables, uint32_t root, uint64_t out_cap,
                         JoinPlan &jp) {
  if (!g) return fail(PT_EINVAL, "graph is NULL");
  if (g->n_tables > kMaxTables) return fail(PT_EINVAL, "%u tables (limit %u)", g->n_tables, kMaxTables);
  if (root >= g->n_tables) return fail(PT_EINVAL, "root %u: the graph has %u tables", root, g->n_tables);
  if (!tables) return fail(PT_EINVAL, "tables is NULL");
  if (g->n_edges > 0 && !g->edges) return fail(PT_EINVAL, "edges is NULL");
  if (out_cap > (1ull << 36)) return fail(PT_EINVAL, "out_cap %llu (limit 2^36)", (unsigned long long)out_cap);
  for (uint32_t t = 0; t < g->n_tables; t++) {
    pt_status st = check_table(&tables[t], t);
    if (st != PT_OK) return st;
  }
  for (uint32_t e = 0; e < g->n_edges; e++) {
    const pt_edge &ed = g->edges[e];
    if (ed.u >= g->n_tables || ed.v >= g->n_tables) return fail(PT_EINVAL, "edge %u: table out of range", e);
    if (ed.u == ed.v) return fail(PT_EINVAL, "edge %u joins table %u with itself", e, ed.u);
    if (ed.flags != 0) return fail(PT_EUNSUPPORTED, "edge %u: flags 0x%x (only inner joins, flags = 0)", e, ed.flags);
    if (ed.u_col >= tables[ed.u].n_cols || ed.v_col >= tables[ed.v].n_cols)
      return fail(PT_EINVAL, "edge %u: column out of range", e);
  }
  // Breadth-first order of root's component, edges in index order.
  jp.pos.assign(g->n_tables, -1);
  jp.order.assign(1, root);
  jp.pos[root] = 0;
  for (size_t head = 0; head < jp.order.size(); head++) {
    const uint32_t t = jp.order[head];
    for (uint32_t e = 0; e < g->n_edges; e++) {
      const pt_edge &ed = g->edges[e];
      const uint32_t other = ed.u == t ? ed.v : ed.v == t ? ed.u : t;
      if (other != t && jp.pos[other] < 0) {
        jp.pos[other] = static_cast<int>(jp.order.size());
        jp.order.push_back(other);
      }
    }
  }
  const uint32_t w = static_cast<uint32_t>(jp.order.size());
  if (w > kMaxJoinWidth)
    return fail(PT_EUNSUPPORTED, "root %u's component has %u tables (limit %u)", root, w, kMaxJoinWidth);
  jp.lookup.assign(w, 0);
  jp.checks.assign(w, {});
  for (uint32_t i = 1; i < w; i++) {
    const uint32_t v = jp.order[i];
    bool found = false;
    for (uint32_t e = 0; e < g->n_edges; e++) {
      const pt_edge &ed = g->edges[e];
      if (ed.u != v && ed.v != v) continue;
      const uint32_t other = ed.u == v ? ed.v : ed.u;
      if (static_cast<uint32_t>(jp.pos[other]) >= i) continue;  // added later
      if (!found) {
        jp.lookup[i] = e;
        found = true;
      } else {
        jp.checks[i].push_back(e);
      }
    }
    if (jp.checks[i].size() > kMaxJoinChecks)
      return fail(PT_EUNSUPPORTED, "table %u has %zu edges to the tables joined before it (limit %u)", v,
                  jp.checks[i].size() + 1, kMaxJoinChecks + 1);
  }
  // Workspace: status word, counts (selected rows per table, tuples per
  // step), compaction partials, each table's selected ids, each added
  // table's hash table, two buffers of intermediate tuples.
  uint64_t off = 256;
  jp.off_counts = off;
  off = align256(off + 2ull * w * 8);
  uint64_t max_rows = 0;
  for (uint32_t t : jp.order) max_rows = std::max<uint64_t>(max_rows, tables[t].n_rows);
  jp.off_partials = off;
  off = align256(off + (compact_partials(max_rows) + 1) * 8);
  jp.off_ids.assign(w, 0);
  jp.off_keys.assign(w, 0);
  jp.off_heads.assign(w, 0);
  jp.off_next.assign(w, 0);
  jp.lg_cap.assign(w, 0);
  for (uint32_t i = 0; i < w; i++) {
    const uint64_t n = tables[jp.order[i]].n_rows;
    jp.off_ids[i] = off;
    off = align256(off + std::max<uint64_t>(n, 1) * 4);
    if (i == 0) continue;
    jp.lg_cap[i] = std::max<uint32_t>(6, ceil_log2(2 * n));
    const uint64_t slots = (1ull << jp.lg_cap[i]) + 1;
    jp.off_keys[i] = off;
    off = align256(off + slots * 8);
    jp.off_heads[i] = off;
    off = align256(off + slots * 4);
    jp.off_next[i] = off;
    off = align256(off + std::max<uint64_t>(n, 1) * 4);
  }
  for (int b = 0; b < 2; b++) {
    jp.off_tuples[b] = off;
    if (w >= 3) off = align256(off + static_cast<uint64_t>(w - 1) * out_cap * 4);
  }
  jp.total = off;
  return PT_OK;
}

}  // namespace

extern "C" {

pt_status pt_join_workspace_size(const pt_graph *graph, const pt_table *tables, uint32_t root, uint64_t out_cap,
                                 size_t *bytes) {
  if (!bytes) return fail(PT_EINVAL, "bytes is NULL");
  JoinPlan jp;
  pt_status st = make_join_plan(graph, tables, root, out_cap, jp);
  if (st != PT_OK) return st;
  *bytes = jp.total;
  return PT_OK;
}

pt_status pt_join(const pt_graph *graph, const pt_table *tables, uint32_t root, const uint64_t *const *d_bitmaps,
                  uint32_t *const *d_out, uint64_t out_cap, uint64_t *d_n_out, void *d_ws, size_t ws_bytes,
                  pt_stream stream) {
  JoinPlan jp;
  pt_status st = make_join_plan(graph, tables, root, out_cap, jp);
  if (st != PT_OK) return st;
  if (!d_ws) return fail(PT_EINVAL, "d_ws is NULL");
  if ((reinterpret_cast<uintptr_t>(d_ws) & 255) != 0) return fail(PT_EINVAL, "d_ws is not 256-byte aligned");
  if (ws_bytes < jp.total)
    return fail(PT_ENOMEM, "workspace %zu < %llu bytes", ws_bytes, (unsigned long long)jp.total);
  if (!d_n_out) return fail(PT_EINVAL, "d_n_out is NULL");
  const uint32_t w = static_cast<uint32_t>(jp.order.size());
  if (out_cap > 0) {
    if (!d_out) return fail(PT_EINVAL, "d_out is NULL");
    for (uint32_t t : jp.order)
      if (!d_out[t]) return fail(PT_EINVAL, "d_out[%u] is NULL (table %u is in root's component)", t, t);
  }

  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  char *ws = static_cast<char *>(d_ws);
  uint32_t *status = reinterpret_cast<uint32_t *>(ws);
  uint64_t *counts = reinterpret_cast<uint64_t *>(ws + jp.off_counts);  // [w] selected rows, [w] step tuples
  auto ids_of = [&](uint32_t i) { return reinterpret_cast<uint32_t *>(ws + jp.off_ids[i]); };
  {
    Timed tm("zero", 0, 0, 0, jp.off_counts + 2ull * w * 8, s);
    st = check_hip(launch_zero_u64(reinterpret_cast<uint64_t *>(ws), (jp.off_counts + 2ull * w * 8) / 8, s),
                   "zero counters");
    if (st == PT_OK) st = check_hip(launch_zero_u64(d_n_out, 1, s), "zero count");
    if (st != PT_OK) return st;
  }
  // The selected rows of every table of the component, ascending.
  for (uint32_t i = 0; i < w; i++) {
    const uint32_t t = jp.order[i];
    const uint64_t n = tables[t].n_rows;
    const uint64_t *bm = d_bitmaps ? d_bitmaps[t] : nullptr;
    Timed tm("join ids", t, 0, n, (n + 63) / 64 * 8 + n * 4, s);
    st = check_hip(launch_join_ids(bm, n, ids_of(i), counts + i, reinterpret_cast<uint64_t *>(ws + jp.off_partials),
                                   s),
                   "join ids");
    if (st != PT_OK) return st;
  }
  if (w == 1) {
    Timed tm("join copy", root, 0, tables[root].n_rows, 0, s);
    return check_hip(launch_join_copy(ids_of(0), counts, out_cap, out_cap ? d_out[root] : nullptr, d_n_out, status, s),
                     "join copy");
  }
  auto key_of = [&](uint32_t e, uint32_t t, const void *&data, uint32_t &key64) {
    const pt_column &c = tables[t].cols[col_at(graph, e, t)];
    data = c.data;
    key64 = c.dtype == PT_I64 ? 1u : 0u;
  };
  for (uint32_t i = 1; i < w; i++) {
    const uint32_t v = jp.order[i];
    const uint32_t e0 = jp.lookup[i];
    const pt_edge &ed0 = graph->edges[e0];
    const uint32_t u = ed0.u == v ? ed0.v : ed0.u;
    JoinStep js{};
    JoinHash &h = js.h;
    h.keys = reinterpret_cast<unsigned long long *>(ws + jp.off_keys[i]);
    h.heads = reinterpret_cast<uint32_t *>(ws + jp.off_heads[i]);
    h.next = reinterpret_cast<uint32_t *>(ws + jp.off_next[i]);
    h.ids = ids_of(i);
    h.count = counts + i;
    key_of(e0, v, h.key, h.key64);
    h.lg_cap = jp.lg_cap[i];
    h.n_rows = tables[v].n_rows;
    {
      Timed tm("join build", v, 0, h.n_rows, h.n_rows * 4, s);
      st = check_hip(launch_join_build(h, s), "join build");
      if (st != PT_OK) return st;
    }
    key_of(e0, u, js.u_key, js.u64);
    js.u_pos = static_cast<uint32_t>(jp.pos[u]);
    js.width = i;
    js.n_checks = static_cast<uint32_t>(jp.checks[i].size());
    for (uint32_t c = 0; c < js.n_checks; c++) {
      const uint32_t e = jp.checks[i][c];
      const pt_edge &ed = graph->edges[e];
      const uint32_t other = ed.u == v ? ed.v : ed.u;
      JoinCheck &ck = js.checks[c];
      key_of(e, v, ck.v_col, ck.v64);
      key_of(e, other, ck.p_col, ck.p64);
      ck.pos = static_cast<uint32_t>(jp.pos[other]);
    }
    const bool last = i + 1 == w;
    if (i == 1) {
      js.in[0] = ids_of(0);
      js.n_in = counts;
      js.in_cap = tables[root].n_rows;
    } else {
      const uint32_t *buf = reinterpret_cast<const uint32_t *>(ws + jp.off_tuples[(i - 2) % 2]);
      for (uint32_t c = 0; c < i; c++) js.in[c] = buf + static_cast<uint64_t>(c) * out_cap;
      js.n_in = counts + w + (i - 1);
      js.in_cap = out_cap;
    }
    if (last) {
      for (uint32_t c = 0; c <= i; c++) js.out[c] = out_cap ? d_out[jp.order[c]] : nullptr;
      js.n_out = d_n_out;
    } else {
      uint32_t *buf = reinterpret_cast<uint32_t *>(ws + jp.off_tuples[(i - 1) % 2]);
      for (uint32_t c = 0; c <= i; c++) js.out[c] = buf + static_cast<uint64_t>(c) * out_cap;
      js.n_out = counts + w + i;
    }
    js.cap = out_cap;
    js.status = status;
    Timed tm("join step", v, 0, 0, 0, s);
    st = check_hip(launch_join_step(js, s), "join step");
    if (st != PT_OK) return st;
  }
  if (w >= 3) return check_hip(launch_join_finish(counts + w + 1, w - 2, out_cap, d_n_out, s), "join finish");
  return PT_OK;
}

}  // extern "C"
