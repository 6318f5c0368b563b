// probe_impl.hpp - the Bloom probe (Sec. 3.2 of the paper: the incoming
// half of the filter transformation), shared by the probe translation units
// that instantiate it for particular block sizes and hash counts.
//
// One scan of the table probes every incoming filter, in the order the
// paper describes for a transformation: the first filter is probed with its
// key column on every row, each later filter only on the rows that are
// still alive. At start each workgroup
//   - orders the filters by their estimated pass rate (builder rows kept /
//     builder rows), most selective first - the order cannot change the
//     result, only the work;
//   - copies the filters into its LDS in that order while they fit; the
//     others are read from global memory (L2 / Infinity Cache / HBM).
// Each wave then takes groups of kGroupWords bitmap words (1024 rows):
//   - it streams the first filter's key column for the group (coalesced,
//     the next group's keys already in flight while this one is tested) and
//     tests every row;
//   - when at most 64 rows of the group survive, it compacts them into its
//     LDS slice, one lane each, and gathers only those rows' keys of the
//     other columns, so a selective first filter spares the reads of most
//     of the other columns' cache lines; when more survive, it streams the
//     other columns for the words that still hold rows;
//   - it stores each bitmap word once, from lane u for word u.
#pragma once

#include "pt_common.hpp"

namespace pt {

struct Slot {
  const void *keys;
  const uint32_t *words;
  uint32_t nb;
  uint32_t key64;
};

constexpr int kGroupWords = 16;  // bitmap words (64 rows each) per wave and group

constexpr uint32_t kNotStaged = 0xFFFFFFFFu;  // a slot's filter is read from global memory

template <int K, bool STAGED>
__device__ __forceinline__ bool slot_has(const Slot &s, const uint32_t *lds_filter, uint32_t h1, uint32_t h2,
                                         uint32_t k, uint32_t lg) {
  const uint32_t blk = block_of(h1, s.nb);
  if (STAGED) return block_has<K>(lds_filter + (blk << (lg - 5)), h2, k, lg);
  return block_has<K>(s.words + (static_cast<uint64_t>(blk) << (lg - 5)), h2, k, lg);
}

// A later slot: staged or not is known at run time only (uniform branch).
template <int K>
__device__ __forceinline__ bool slot_has_any(const Slot &s, const uint32_t *lds_filters, uint32_t lds_off,
                                             uint32_t h1, uint32_t h2, uint32_t k, uint32_t lg) {
  if (lds_off != kNotStaged) return slot_has<K, true>(s, lds_filters + lds_off, h1, h2, k, lg);
  return slot_has<K, false>(s, lds_filters, h1, h2, k, lg);
}

// 32-bit words of one wave's LDS slice: the compacted survivors' tags
// (word and lane), their first-column keys (low and high halves), and one
// 64-bit failure mask per word of the group.
constexpr int probe_slice_words() { return kWave * 3 + 2 * kGroupWords; }

// Key of row `row` of a column: the low and high halves of an int64 key, or
// an int32 key in lo (hi is then left as it is: every use of an int32 key
// reads lo alone). Nothing here uses the loaded value, so several gathers
// are in flight together even though the width is only known at run time.
__device__ __forceinline__ void gather_key(const void *col, uint32_t key64, uint64_t row, uint32_t &lo,
                                           uint32_t &hi) {
  if (key64) {
    const uint2 x = static_cast<const uint2 *>(col)[row];
    lo = x.x;
    hi = x.y;
  } else {
    lo = static_cast<const uint32_t *>(col)[row];
  }
}

// The group's first-column keys: lane l gets rows base + 64 u + l (clamped to
// the last row, `last` rows past base), u < kGroupWords.
template <bool KEY64, int G>
__device__ __forceinline__ void load_group(const void *col, uint64_t base, uint32_t last,
                                           uint32_t (&lo)[G], uint32_t (&hi)[KEY64 ? G : 1]) {
  const uint32_t lane = lane_id();
  if constexpr (KEY64) {
    const uint64_t *p = static_cast<const uint64_t *>(col) + base;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const uint64_t x = p[min(static_cast<uint32_t>(u * 64) + lane, last)];
      lo[u] = static_cast<uint32_t>(x);
      hi[u] = static_cast<uint32_t>(x >> 32);
    }
  } else {
    const uint32_t *p = static_cast<const uint32_t *>(col) + base;
#pragma unroll
    for (int u = 0; u < G; u++) lo[u] = p[min(static_cast<uint32_t>(u * 64) + lane, last)];
  }
}

// SPARSE (int32 keys, a bitmap that may hold few rows and a first filter in
// global memory): a row that is not selected reads the same filter words as
// every other such row, so the wave's reads for them fall on one line
// instead of one line each. (The int64 kernels are left without this loop:
// their register allocation, already at the limit, made their other loops
// slower with it.)
template <int K, bool KEY64, bool STAGED, bool APPEND, int G, bool SPARSE = false>
__device__ __forceinline__ int64_t probe_loop(const Slot (&sl)[kMaxProbe], const uint32_t (&lds_off)[kMaxProbe],
                                              uint32_t n_f, uint32_t k, uint32_t lg, uint64_t n_rows,
                                              uint64_t *bitmap, uint32_t input_all, const uint32_t *lds_filters,
                                              uint32_t *slice, const AppendSet &app,
                                              const int (&app_slot)[kMaxAppend], const VGrid &vg) {
  static_assert(G % 4 == 0 && G <= kGroupWords, "group of 4 to kGroupWords words");
  constexpr int U = G;
  uint32_t *q_tag = slice;                                                     // [kWave]
  uint32_t *q_lo = slice + kWave;                                              // [kWave]
  uint32_t *q_hi = slice + 2 * kWave;                                          // [kWave]
  unsigned long long *fail = reinterpret_cast<unsigned long long *>(slice + 3 * kWave);  // [U]
  const uint32_t lane = lane_id();
  const uint64_t n_words = (n_rows + 63) / 64;
  const uint64_t stride = wave_count(vg) * U;
  int64_t cnt = 0;
  uint32_t app_n = 0;  // survivors of this wave's region so far
  const uint64_t app_base = global_wave(vg) * static_cast<uint64_t>(app.region_cap);
  const void *col0 = sl[0].keys;

  // Software pipeline: the keys (and bitmap words) of the group after the
  // current one are requested before the current one's other filters are
  // tested.
  uint64_t w0 = global_wave(vg) * U;
  // One set of key registers: the next group's keys are requested as soon
  // as the first filter has consumed the current group's, so the load is in
  // flight while the current group's other filters are tested.
  uint32_t lo[U], hi[KEY64 ? U : 1];
  uint64_t nbits = 0;
  if (w0 < n_words) {
    const uint64_t left = n_rows - 1 - w0 * 64;
    load_group<KEY64, U>(col0, w0 * 64, left < 0xFFFFFFFFull ? static_cast<uint32_t>(left) : 0xFFFFFFFFu, lo, hi);
    if (!input_all) nbits = bitmap[min(w0 + (lane < U ? lane : 0), n_words - 1)];
  }
  for (; w0 < n_words; w0 += stride) {
    const uint64_t bits = nbits;  // lane u < U: bitmap word w0 + u (unless input_all)
    const uint64_t w_next = w0 + stride;
    const uint64_t base_row = w0 * 64;

    // The first (most selective) filter on every row of the group. The
    // group's words go to lane-parallel form (lane u holds word w0 + u), and
    // the survivors are compacted into the LDS slice as they appear (the
    // first 64 of them: more than that take the dense path below).
    // The filter reads of C words are issued before any of their results is
    // used (they come from L2 or beyond when the filter is not in LDS).
    constexpr int C = STAGED ? 1 : 4;
    uint64_t mine = 0;
    uint32_t total0 = 0;  // survivors of the first filter
#pragma unroll
    for (int u0 = 0; u0 < U; u0 += C) {
      uint64_t word[C];
      bool ok[C];
#pragma unroll
      for (int j = 0; j < C; j++) {
        const int u = u0 + j;
        word[j] = tail_mask(w0 + u, n_words, n_rows);
        if (!input_all) {
          // readlane returns int: widen through uint32_t (no sign extension)
          const uint32_t b_hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(bits >> 32), u);
          const uint32_t b_lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(bits), u);
          word[j] &= (static_cast<uint64_t>(b_hi) << 32) | b_lo;
        }
        ok[j] = false;
        if (word[j]) {
          uint32_t h1, h2;
          if constexpr (KEY64)
            hash_key((static_cast<uint64_t>(hi[u]) << 32) | lo[u], h1, h2);
          else
            hash_key32(lo[u], h1, h2);
          if constexpr (SPARSE) {
            if (!((word[j] >> lane) & 1)) h1 = h2 = 0;
          }
          ok[j] = slot_has<K, STAGED>(sl[0], lds_filters + lds_off[0], h1, h2, k, lg);
        }
      }
#pragma unroll
      for (int j = 0; j < C; j++) {
        const int u = u0 + j;
        if (!word[j]) continue;
        const uint64_t m = __ballot(ok[j]) & word[j];
        mine = lane == u ? m : mine;
        if (m) {
          if ((m >> lane) & 1) {
            const uint32_t pos = total0 + __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                                                    __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0));
            if (pos < kWave) {
              q_tag[pos] = (static_cast<uint32_t>(u) << 6) | lane;
              if (APPEND) {
                q_lo[pos] = lo[u];
                if constexpr (KEY64) q_hi[pos] = hi[u];
              }
            }
          }
          total0 += static_cast<uint32_t>(__popcll(m));
        }
      }
    }
    // The current group's first-column keys are consumed (the survivors'
    // ones are in the slice): request the next group's.
    if (w_next < n_words) {
      const uint64_t left = n_rows - 1 - w_next * 64;
      load_group<KEY64, U>(col0, w_next * 64, left < 0xFFFFFFFFull ? static_cast<uint32_t>(left) : 0xFFFFFFFFu, lo,
                        hi);
      if (!input_all) nbits = bitmap[min(w_next + (lane < U ? lane : 0), n_words - 1)];
    }

    uint32_t total = total0;  // rows left in the group
    bool appended = false;    // the final survivors' keys are stored
    if (total0 > kWave && n_f > 1) {
      // Many survivors: stream the other columns for the words that still
      // hold rows (four words at a time, their loads in flight together),
      // and test them there.
      const uint64_t left = n_rows - 1 - base_row;
      const uint32_t last = left < 0xFFFFFFFFull ? static_cast<uint32_t>(left) : 0xFFFFFFFFu;
#pragma unroll
      for (int s = 1; s < kMaxProbe; s++) {
        if (s < static_cast<int>(n_f)) {
#pragma unroll
          for (int u0 = 0; u0 < U; u0 += 4) {
            uint64_t m[4];
            uint32_t xlo[4], xhi[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
              const uint32_t m_hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(mine >> 32), u0 + j);
              const uint32_t m_lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(mine), u0 + j);
              m[j] = (static_cast<uint64_t>(m_hi) << 32) | m_lo;
              xlo[j] = xhi[j] = 0;
              if (m[j])
                gather_key(sl[s].keys, sl[s].key64, base_row + min(static_cast<uint32_t>((u0 + j) * 64) + lane, last),
                           xlo[j], xhi[j]);
            }
#pragma unroll
            for (int j = 0; j < 4; j++) {
              if (m[j]) {
                uint32_t h1, h2;
                hash_parts(xlo[j], xhi[j], sl[s].key64, h1, h2);
                m[j] &= __ballot(slot_has_any<K>(sl[s], lds_filters, lds_off[s], h1, h2, k, lg));
                mine = lane == u0 + j ? m[j] : mine;
              }
            }
          }
        }
      }
      total = 0;
#pragma unroll
      for (int u = 0; u < U; u++) {
        const uint32_t m_hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(mine >> 32), u);
        const uint32_t m_lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(mine), u);
        total += static_cast<uint32_t>(__popcll((static_cast<uint64_t>(m_hi) << 32) | m_lo));
      }
    }

    if (total0 > 0 && total0 <= kWave && (n_f > 1 || (APPEND && app_n < app.region_cap))) {
      // Few survivors, compacted above, one lane each: gather their keys of
      // the other columns and test those with every lane busy.
      if (lane < U) fail[lane] = 0;
      // The LDS accesses of one wave execute in program order; the wave
      // barrier only keeps the compiler from moving them across.
      __builtin_amdgcn_wave_barrier();
      const bool act = lane < total0;
      const uint32_t idx = act ? lane : 0;
      const uint32_t tag = q_tag[idx];
      const uint64_t row = base_row + (tag >> 6) * 64 + (tag & 63);
      uint32_t klo[kMaxProbe] = {}, khi[kMaxProbe] = {};
      if (APPEND) {
        klo[0] = q_lo[idx];
        khi[0] = KEY64 ? q_hi[idx] : static_cast<uint32_t>(static_cast<int32_t>(klo[0]) >> 31);
      }
      // The second filter's key is read for the survivors of the first,
      // the remaining filters' keys only for the rows that pass the second
      // too (the filters are ordered most selective first, so later
      // columns are read in fewer cache lines; the remaining ones are read
      // together, in one round trip).
      bool ok = act;
      if (n_f > 1) {
        gather_key(sl[1].keys, sl[1].key64, row, klo[1], khi[1]);
        uint32_t h1, h2;
        hash_parts(klo[1], khi[1], sl[1].key64, h1, h2);
        ok = ok && slot_has_any<K>(sl[1], lds_filters, lds_off[1], h1, h2, k, lg);
      }
#pragma unroll
      for (int s = 2; s < kMaxProbe; s++)
        if (s < static_cast<int>(n_f) && ok) gather_key(sl[s].keys, sl[s].key64, row, klo[s], khi[s]);
#pragma unroll
      for (int s = 2; s < kMaxProbe; s++) {
        if (s < static_cast<int>(n_f)) {
          uint32_t h1, h2;
          hash_parts(klo[s], khi[s], sl[s].key64, h1, h2);
          ok = ok && slot_has_any<K>(sl[s], lds_filters, lds_off[s], h1, h2, k, lg);
        }
      }
      const uint64_t failed = __ballot(act && !ok);
      if (failed) {
        if (act && !ok) atomicOr(&fail[tag >> 6], 1ull << (tag & 63));
        __builtin_amdgcn_wave_barrier();
        if (lane < U) mine &= ~fail[lane];
        total -= static_cast<uint32_t>(__popcll(failed));
      }
      if (APPEND) {
        // The final survivors append their keys: one store per column.
        const uint64_t fin = __ballot(ok);
        const uint32_t pos =
            app_n + __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(fin >> 32),
                                              __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(fin), 0));
        if (ok && pos < app.region_cap) {
#pragma unroll
          for (int c = 0; c < kMaxAppend; c++) {
            if (c < static_cast<int>(app.n_cols)) {
              uint32_t alo = 0, ahi = 0;
              bool have = false;
#pragma unroll
              for (int q = 0; q < kMaxProbe; q++)
                if (app_slot[c] == q) {
                  alo = klo[q];
                  ahi = khi[q];
                  have = true;
                }
              if (!have) gather_key(app.src[c], app.key64[c], row, alo, ahi);
              if (app.key64[c])
                static_cast<uint64_t *>(app.dst[c])[app_base + pos] = (static_cast<uint64_t>(ahi) << 32) | alo;
              else
                static_cast<uint32_t *>(app.dst[c])[app_base + pos] = alo;
            }
          }
        }
        app_n += static_cast<uint32_t>(__popcll(fin));
        appended = true;
      }
      __builtin_amdgcn_wave_barrier();
    }

    if (APPEND && !appended && total0 > 0) {
      // Too many first-filter survivors to compact (or a full region): the
      // region is marked as overflowed, and builds walk its bitmap words
      // (dense survivors read coalesced anyway).
      app_n = app.region_cap + 1;
    }

    if (lane < U && w0 + lane < n_words) bitmap[w0 + lane] = mine;
    cnt += total;
  }
  if (APPEND && lane == 0) app.counts[global_wave(vg)] = app_n;
  return cnt;
}

// Key widths a probe kernel is built for: the first filter's key column
// decides on the device which loop runs, and a kernel that only ever meets
// one width (every key column of its filters int32, or every one int64)
// leaves the other loop out, which frees registers.
constexpr int kKeysMixed = 0, kKeys32 = 1, kKeys64 = 2;

template <int B, int K, bool APPEND, int G = kGroupWords, int KW = kKeysMixed>
__device__ __forceinline__ void probe_body(const FilterSet &fs, uint32_t k, uint32_t lg_rt, uint64_t n_rows,
                                           uint64_t *__restrict__ bitmap, unsigned long long *count,
                                           uint32_t lds_filter_words, uint32_t input_all, uint32_t keep_order,
                                           uint32_t *status, const AppendSet &app, const VGrid &vg) {
  extern __shared__ __align__(16) uint32_t lds[];
  const uint32_t lg = block_log2<B>(lg_rt);
  const uint32_t W = 1u << (lg - 5);
  constexpr int kSliceWords = probe_slice_words();
  __shared__ uint32_t s_ord[kMaxProbe];
  __shared__ uint32_t s_nb[kMaxProbe];
  __shared__ uint32_t s_off[kMaxProbe];
  __shared__ unsigned long long s_cnt;

  __shared__ uint64_t s_sel[kMaxProbe];
  __shared__ uint64_t s_nb_raw[kMaxProbe];
  __shared__ uint32_t s_nf;
  const uint32_t n_in = fs.n;
  // Thread i reads filter i's builder count and block count (in parallel).
  if (threadIdx.x < n_in) {
    const FilterRef &f = fs.f[threadIdx.x];
    s_sel[threadIdx.x] = (f.sel && f.rows) ? *f.sel : 1;
    s_nb_raw[threadIdx.x] = *f.nb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t ord[kMaxProbe];
    uint64_t sel[kMaxProbe], rows[kMaxProbe];
    uint32_t n_f = 0;
#pragma unroll
    for (int i = 0; i < kMaxProbe; i++) {
      ord[i] = 0;
      sel[i] = 1;
      rows[i] = 1;
      if (i < static_cast<int>(n_in) && fs.f[i].sel && fs.f[i].rows) {
        sel[i] = s_sel[i];
        rows[i] = fs.f[i].rows;
      }
    }
    // A pruned filter (its builder kept every row, so its size step left a
    // block count of zero) lets every key through: it is not tested.
    for (uint32_t i = 0; i < n_in; i++)
      if (!(fs.prune && s_nb_raw[i] == 0)) ord[n_f++] = i;
    // stable insertion sort by sel / rows (the given order with keep_order)
    for (uint32_t a = 1; a < n_f && !keep_order; a++) {
      for (uint32_t b = a; b > 0; b--) {
        const uint32_t x = ord[b - 1], y = ord[b];
        if (sel[y] * rows[x] < sel[x] * rows[y]) {
          ord[b - 1] = y;
          ord[b] = x;
        } else {
          break;
        }
      }
    }
    // In probe order, every filter that still fits goes to LDS; the rest
    // are read from global memory.
    uint64_t need = 0;
    for (uint32_t j = 0; j < n_f; j++) {
      const FilterRef &f = fs.f[ord[j]];
      const uint32_t nb = clamp_blocks(s_nb_raw[ord[j]], f.cap_words / W, status);
      s_ord[j] = ord[j];
      s_nb[j] = nb;
      const uint64_t words = static_cast<uint64_t>(nb) * W;
      if (need + words <= lds_filter_words) {
        s_off[j] = static_cast<uint32_t>(need);
        need += words;
      } else {
        s_off[j] = kNotStaged;
      }
    }
    s_nf = n_f;
    s_cnt = 0;
  }
  __syncthreads();
  const uint32_t n_f = __builtin_amdgcn_readfirstlane(s_nf);
  if (n_f == 0) {
    // Every filter was pruned: the rows stay as they are.
    const uint64_t n_words = (n_rows + 63) / 64;
    const uint32_t lane = lane_id();
    int64_t cnt = 0;
    for (uint64_t w0 = global_wave(vg) * kWave; w0 < n_words; w0 += wave_count(vg) * kWave) {
      const uint64_t w = w0 + lane;
      uint64_t m = 0;
      if (w < n_words) {
        m = tail_mask(w, n_words, n_rows);
        if (input_all)
          bitmap[w] = m;
        else
          m &= bitmap[w];
      }
      cnt += static_cast<int64_t>(wave_sum(static_cast<uint64_t>(__popcll(m))));
    }
    // builds that would read appended keys walk the bitmap instead
    if (APPEND && lane_id() == 0) app.counts[global_wave(vg)] = app.region_cap + 1;
    block_count_add(cnt, &s_cnt, count);
    return;
  }
  for (uint32_t j = 0; j < n_f; j++) {
    if (s_off[j] == kNotStaged) continue;
    const uint32_t n = s_nb[j] * W;
    const uint32_t *src = fs.f[__builtin_amdgcn_readfirstlane(s_ord[j])].words;
    uint32_t *dst = lds + s_off[j];
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
  }
  __syncthreads();
  const bool staged = s_off[0] != kNotStaged;  // the filter every row is tested against

  // Slot j is filter s_ord[j]; slots past n_f repeat slot 0 (never tested).
  Slot sl[kMaxProbe];
  uint32_t off[kMaxProbe];
#pragma unroll
  for (int j = 0; j < kMaxProbe; j++) {
    const uint32_t jj = j < static_cast<int>(n_f) ? j : 0;
    const FilterRef &f = fs.f[__builtin_amdgcn_readfirstlane(s_ord[jj])];
    sl[j].keys = f.keys;
    sl[j].words = f.words;
    sl[j].nb = __builtin_amdgcn_readfirstlane(s_nb[jj]);
    sl[j].key64 = f.key64;
    off[j] = __builtin_amdgcn_readfirstlane(s_off[jj]);
  }
  // Appended column c comes from slot app_slot[c]'s registers (-1: gathered).
  int app_slot[kMaxAppend];
#pragma unroll
  for (int c = 0; c < kMaxAppend; c++) {
    app_slot[c] = -1;
#pragma unroll
    for (int j = kMaxProbe - 1; j >= 0; j--)
      if (j < static_cast<int>(n_f) && c < static_cast<int>(app.n_cols) && sl[j].keys == app.src[c] &&
          sl[j].key64 == app.key64[c])
        app_slot[c] = j;
  }
  // The per-wave slices follow the filters; lds_filter_words is even, so
  // each slice's 64-bit failure masks stay 8-byte aligned.
  uint32_t *slice = lds + lds_filter_words + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave) * kSliceWords;
  int64_t cnt = 0;
  if (!staged) off[0] = 0;  // slot 0 takes the global path by template
  // (with KW fixed, the host guarantees that every filter's key column has
  // that width, so sl[0].key64 agrees with it)
  const bool key64 = KW == kKeys64 || (KW == kKeysMixed && sl[0].key64);
  if (key64) {
    if constexpr (KW != kKeys32) {
      if (staged)
        cnt = probe_loop<K, true, true, APPEND, G>(sl, off, n_f, k, lg, n_rows, bitmap, input_all, lds, slice, app,
                                                app_slot, vg);
      else
        cnt = probe_loop<K, true, false, APPEND, G>(sl, off, n_f, k, lg, n_rows, bitmap, input_all, lds, slice,
                                                 app, app_slot, vg);
    }
  } else {
    if constexpr (KW != kKeys64) {
      if (staged)
        cnt = probe_loop<K, false, true, APPEND, G>(sl, off, n_f, k, lg, n_rows, bitmap, input_all, lds, slice,
                                                 app, app_slot, vg);
      else if (input_all)
        cnt = probe_loop<K, false, false, APPEND, G>(sl, off, n_f, k, lg, n_rows, bitmap, input_all, lds, slice,
                                                  app, app_slot, vg);
      else
        cnt = probe_loop<K, false, false, APPEND, G, true>(sl, off, n_f, k, lg, n_rows, bitmap, input_all, lds,
                                                        slice, app, app_slot, vg);
    }
  }
  block_count_add(cnt, &s_cnt, count);
}

template <int B, int K, bool APPEND, int KW>
__global__ void __launch_bounds__(kProbeThreads)
    k_probe(FilterSet fs, uint32_t k, uint32_t lg, uint64_t n_rows, uint64_t *__restrict__ bitmap,
            unsigned long long *count, uint32_t lds_filter_words, uint32_t input_all, uint32_t keep_order,
            uint32_t *status, AppendSet app) {
  probe_body<B, K, APPEND, kGroupWords, KW>(fs, k, lg, n_rows, bitmap, count, lds_filter_words, input_all,
                                            keep_order, status, app, whole_grid());
}

// Launches k_probe<B, K, *, *> for one ProbeLaunch: the appending variant
// when it appends, and the one built for its filters' key widths.
template <int B, int K>
hipError_t launch_probe_kernel(const ProbeLaunch &pl, hipStream_t s) {
  auto launch = [&](auto kern) -> hipError_t {
    hipError_t e = allow_lds(reinterpret_cast<const void *>(kern), pl.lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(pl.grid), dim3(pl.threads), pl.lds_bytes, s, pl.fs, pl.k, pl.lg, pl.n_rows,
                       pl.bitmap, pl.count, pl.lds_filter_words, pl.input_all, pl.keep_order, pl.status, pl.app);
    return hipGetLastError();
  };
  uint32_t n64 = 0;
  for (uint32_t i = 0; i < pl.fs.n; i++) n64 += pl.fs.f[i].key64 ? 1u : 0u;
  const int kw = n64 == 0 ? kKeys32 : n64 == pl.fs.n ? kKeys64 : kKeysMixed;
  if (pl.app.n_cols) {
    if (kw == kKeys32) return launch(k_probe<B, K, true, kKeys32>);
    if (kw == kKeys64) return launch(k_probe<B, K, true, kKeys64>);
    return launch(k_probe<B, K, true, kKeysMixed>);
  }
  if (kw == kKeys32) return launch(k_probe<B, K, false, kKeys32>);
  if (kw == kKeys64) return launch(k_probe<B, K, false, kKeys64>);
  return launch(k_probe<B, K, false, kKeysMixed>);
}

}  // namespace pt
