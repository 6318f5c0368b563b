// probe_impl.hpp - the Bloom probe (Sec. 3.2 of the paper: the incoming
// half of the filter transformation), shared by the probe translation units
// that instantiate it for particular block sizes and hash counts.
//
// One scan of the table probes every incoming filter. At start each
// workgroup:
//   - orders the filters by their estimated pass rate (builder rows kept /
//     builder rows), most selective first - the order cannot change the
//     result, only the work;
//   - copies all filters into its LDS when they fit together, else reads
//     all of them from global memory (L2 / Infinity Cache / HBM).
// Each wave then streams U bitmap words per iteration: it loads every key
// column of those rows, tests the first filter on all of them, and, when
// at most 64 rows survive, compacts the survivors (word, lane and
// remaining keys) into its LDS slice so that one fully occupied wave
// instruction stream tests them against the remaining filters. Failures are
// folded back into the group's words through an LDS mask, and every word is
// stored once. Groups with more survivors test the remaining filters on the
// words directly.
#pragma once

#include "pt_common.hpp"

namespace pt {

struct Slot {
  const void *keys;
  const uint32_t *words;
  uint32_t nb;
  uint32_t key64;
};

template <int K, bool STAGED>
__device__ __forceinline__ bool slot_has(const Slot &s, const uint32_t *lds_filter, uint32_t h1, uint32_t h2,
                                         uint32_t k, uint32_t lg) {
  const uint32_t blk = block_of(h1, s.nb);
  if (STAGED) return block_has<K>(lds_filter + (blk << (lg - 5)), h2, k, lg);
  return block_has<K>(s.words + (static_cast<uint64_t>(blk) << (lg - 5)), h2, k, lg);
}

template <bool ANY64>
constexpr int probe_group_words() {
  return ANY64 ? 4 : 8;
}

// 32-bit words of one wave's LDS slice: compacted survivors (word-and-lane
// tag, the keys of every slot) plus one 64-bit failure mask per word of the
// group.
template <bool ANY64>
constexpr int probe_slice_words() {
  return kWave * (1 + kMaxProbe * (ANY64 ? 2 : 1)) + 2 * probe_group_words<ANY64>();
}

// Stores the key of appended column c for a surviving row at region slot
// pos: from the probe's registers (klo/khi of slot app_slot[c]) or, for a
// column the probe did not read, from the table.
template <bool ANY64>
__device__ __forceinline__ void append_key(const AppendSet &app, int c, int slot, const uint32_t (&klo)[kMaxProbe],
                                           const uint32_t (&khi)[kMaxProbe], uint64_t row, uint64_t at) {
  uint32_t lo = 0, hi = 0;
  bool have = false;
#pragma unroll
  for (int q = 0; q < kMaxProbe; q++)
    if (slot == q) {
      lo = klo[q];
      hi = ANY64 ? khi[q] : 0;
      have = true;
    }
  if (app.key64[c]) {
    static_cast<uint64_t *>(app.dst[c])[at] =
        have ? ((static_cast<uint64_t>(hi) << 32) | lo) : static_cast<const uint64_t *>(app.src[c])[row];
  } else {
    static_cast<uint32_t *>(app.dst[c])[at] = have ? lo : static_cast<const uint32_t *>(app.src[c])[row];
  }
}

template <int K, bool ANY64, bool STAGED, bool APPEND>
__device__ __forceinline__ int64_t probe_loop(const Slot (&sl)[kMaxProbe], const uint32_t (&lds_off)[kMaxProbe],
                                              uint32_t n_f, uint32_t k, uint32_t lg, uint64_t n_rows,
                                              uint64_t *bitmap, uint32_t input_all, const uint32_t *lds_filters,
                                              uint32_t *slice, const AppendSet &app,
                                              const int (&app_slot)[kMaxAppend], const VGrid &vg) {
  constexpr int U = probe_group_words<ANY64>();
  uint32_t *q_tag = slice;                                          // [kWave]
  uint32_t *q_lo = slice + kWave;                                   // [kMaxProbe][kWave]
  uint32_t *q_hi = slice + kWave * (1 + kMaxProbe);                 // [kMaxProbe][kWave] (int64)
  unsigned long long *fail_mask = reinterpret_cast<unsigned long long *>(
      slice + kWave * (1 + kMaxProbe * (ANY64 ? 2 : 1)));           // [U]
  const uint32_t lane = lane_id();
  const uint64_t n_words = (n_rows + 63) / 64;
  const uint64_t stride = wave_count(vg) * U;
  int64_t cnt = 0;
  uint32_t app_n = 0;  // survivors of this wave's region so far
  const uint64_t app_base = global_wave(vg) * static_cast<uint64_t>(app.region_cap);

  for (uint64_t w0 = global_wave(vg) * U; w0 < n_words; w0 += stride) {
    // The group's U words: lane u loads word w0 + u (one load), then every
    // lane reads them back as scalars.
    uint64_t mine = 0;
    if (!input_all) {
      const uint64_t wl = w0 + (lane < U ? lane : 0);
      mine = bitmap[wl < n_words ? wl : n_words - 1];
    }
    uint64_t word[U];
    uint64_t any = 0;
#pragma unroll
    for (int u = 0; u < U; u++) {
      const uint64_t m = tail_mask(w0 + u, n_words, n_rows);
      // readlane returns int: widen through uint32_t (no sign extension)
      const uint32_t b_hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(mine >> 32), u);
      const uint32_t b_lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(mine), u);
      const uint64_t b = (static_cast<uint64_t>(b_hi) << 32) | b_lo;
      word[u] = input_all ? m : (b & m);
      any |= word[u];
    }
    if (any == 0) continue;

    // Every key column of the group, for every lane, in straight-line code so
    // that all loads of the group are in flight together. Rows past the end
    // are clamped; slots past n_f read slot 0's column again (cache hits).
    // Offsets are 32-bit from a per-group scalar base.
    const uint64_t base_row = w0 * 64;
    const uint64_t left = n_rows - 1 - base_row;  // rows left after base_row (>= 0)
    const uint32_t last = left < 0xFFFFFFFFull ? static_cast<uint32_t>(left) : 0xFFFFFFFFu;
    uint32_t rel[U];
#pragma unroll
    for (int u = 0; u < U; u++) rel[u] = min(static_cast<uint32_t>(u * 64) + lane, last);
    uint32_t lo[kMaxProbe][U];
    uint32_t hi[ANY64 ? kMaxProbe : 1][U];
#pragma unroll
    for (int s = 0; s < kMaxProbe; s++) {
      if (ANY64 && sl[s].key64) {
        const uint64_t *col = static_cast<const uint64_t *>(sl[s].keys) + base_row;
#pragma unroll
        for (int u = 0; u < U; u++) {
          const uint64_t x = col[rel[u]];
          lo[s][u] = static_cast<uint32_t>(x);
          hi[ANY64 ? s : 0][u] = static_cast<uint32_t>(x >> 32);
        }
      } else {
        const int32_t *col = static_cast<const int32_t *>(sl[s].keys) + base_row;
#pragma unroll
        for (int u = 0; u < U; u++) {
          const int32_t x = col[rel[u]];
          lo[s][u] = static_cast<uint32_t>(x);
          if (ANY64) hi[ANY64 ? s : 0][u] = static_cast<uint32_t>(x >> 31);
        }
      }
    }

    // The first (most selective) filter on every row of the group.
    uint64_t m0[U];
    uint32_t total = 0;
#pragma unroll
    for (int u = 0; u < U; u++) {
      uint32_t h1, h2;
      hash_parts(lo[0][u], ANY64 ? hi[0][u] : 0, ANY64 && sl[0].key64, h1, h2);
      const bool ok = slot_has<K, STAGED>(sl[0], lds_filters + lds_off[0], h1, h2, k, lg);
      m0[u] = __ballot(ok && ((word[u] >> lane) & 1));
      total += __popcll(m0[u]);
    }

    bool appended = false;  // the survivors' keys are stored
    if (n_f > 1 && total > kWave) {
      // Many survivors: test the remaining filters on the words themselves.
#pragma unroll
      for (int s = 1; s < kMaxProbe; s++) {
        if (s < static_cast<int>(n_f)) {
#pragma unroll
          for (int u = 0; u < U; u++) {
            if (m0[u]) {
              uint32_t h1, h2;
              hash_parts(lo[s][u], ANY64 ? hi[ANY64 ? s : 0][u] : 0, ANY64 && sl[s].key64, h1, h2);
              const bool ok = slot_has<K, STAGED>(sl[s], lds_filters + lds_off[s], h1, h2, k, lg);
              m0[u] = __ballot(ok && ((m0[u] >> lane) & 1));
            }
          }
        }
      }
    } else if (total > 0 && total <= kWave && (n_f > 1 || (APPEND && app_n < app.region_cap))) {
      // Few survivors: compact them into the LDS slice, one lane each, and
      // test the remaining filters with every lane busy.
      uint32_t pos0 = 0;
#pragma unroll
      for (int u = 0; u < U; u++) {
        if (lane == 0) fail_mask[u] = 0;
        if ((m0[u] >> lane) & 1) {
          const uint32_t pos = pos0 + __popcll(m0[u] & ((1ull << lane) - 1));
          q_tag[pos] = (static_cast<uint32_t>(u) << 6) | lane;
#pragma unroll
          for (int s = APPEND ? 0 : 1; s < kMaxProbe; s++) {
            if (s < static_cast<int>(n_f)) {
              q_lo[s * kWave + pos] = lo[s][u];
              if (ANY64) q_hi[s * kWave + pos] = hi[ANY64 ? s : 0][u];
            }
          }
        }
        pos0 += __popcll(m0[u]);
      }
      // The LDS accesses of one wave execute in program order; the wave
      // barrier only keeps the compiler from moving them across.
      __builtin_amdgcn_wave_barrier();
      const bool act = lane < total;
      const uint32_t idx = act ? lane : 0;
      bool ok = act;
      uint32_t klo[kMaxProbe] = {}, khi[kMaxProbe] = {};
#pragma unroll
      for (int s = APPEND ? 0 : 1; s < kMaxProbe; s++) {
        if (s < static_cast<int>(n_f)) {
          klo[s] = q_lo[s * kWave + idx];
          khi[s] = ANY64 ? q_hi[s * kWave + idx] : 0;
          if (s > 0) {
            uint32_t h1, h2;
            hash_parts(klo[s], khi[s], ANY64 && sl[s].key64, h1, h2);
            ok = ok && slot_has<K, STAGED>(sl[s], lds_filters + lds_off[s], h1, h2, k, lg);
          }
        }
      }
      const uint32_t tag = q_tag[idx];
      if (act && !ok) atomicOr(&fail_mask[tag >> 6], 1ull << (tag & 63));
      if (APPEND) {
        // The final survivors append their keys: one store per column.
        const uint64_t fin = __ballot(ok);
        const uint32_t pos = app_n + static_cast<uint32_t>(__popcll(fin & ((1ull << lane) - 1)));
        if (ok && pos < app.region_cap) {
          const uint64_t row = base_row + (tag >> 6) * 64 + (tag & 63);
#pragma unroll
          for (int c = 0; c < kMaxAppend; c++)
            if (c < static_cast<int>(app.n_cols)) append_key<ANY64>(app, c, app_slot[c], klo, khi, row, app_base + pos);
        }
        app_n += static_cast<uint32_t>(__popcll(fin));
        appended = true;
      }
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int u = 0; u < U; u++) m0[u] &= ~uniform64(fail_mask[u]);
      __builtin_amdgcn_wave_barrier();
    }

    if (APPEND && !appended && total > 0) {
      // Too many first-filter survivors to compact (or a full region): the
      // region is marked as overflowed, and builds walk its bitmap words
      // (dense survivors read coalesced anyway).
      app_n = app.region_cap + 1;
    }

#pragma unroll
    for (int u = 0; u < U; u++) {
      const uint64_t w = w0 + u;
      if (lane == 0 && w < n_words) bitmap[w] = m0[u];
      cnt += __popcll(m0[u]);
    }
  }
  if (APPEND && lane == 0) app.counts[global_wave(vg)] = app_n;
  return cnt;
}

template <int B, int K, bool ANY64, bool APPEND>
__device__ __forceinline__ void probe_body(const FilterSet &fs, uint32_t k, uint32_t lg_rt, uint64_t n_rows,
                                           uint64_t *__restrict__ bitmap, unsigned long long *count,
                                           uint32_t lds_filter_words, uint32_t input_all, uint32_t keep_order,
                                           uint32_t *status, const AppendSet &app, const VGrid &vg) {
  extern __shared__ __align__(16) uint32_t lds[];
  const uint32_t lg = block_log2<B>(lg_rt);
  const uint32_t W = 1u << (lg - 5);
  constexpr int kSliceWords = probe_slice_words<ANY64>();
  __shared__ uint32_t s_ord[kMaxProbe];
  __shared__ uint32_t s_nb[kMaxProbe];
  __shared__ uint32_t s_off[kMaxProbe];
  __shared__ uint32_t s_staged;
  __shared__ unsigned long long s_cnt;

  __shared__ uint64_t s_sel[kMaxProbe];
  __shared__ uint64_t s_nb_raw[kMaxProbe];
  const uint32_t n_f = fs.n;
  // Thread i reads filter i's builder count and block count (in parallel).
  if (threadIdx.x < n_f) {
    const FilterRef &f = fs.f[threadIdx.x];
    s_sel[threadIdx.x] = (f.sel && f.rows) ? *f.sel : 1;
    s_nb_raw[threadIdx.x] = *f.nb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t ord[kMaxProbe];
    uint64_t sel[kMaxProbe], rows[kMaxProbe];
#pragma unroll
    for (int i = 0; i < kMaxProbe; i++) {
      ord[i] = i;
      sel[i] = 1;
      rows[i] = 1;
      if (i < static_cast<int>(n_f) && fs.f[i].sel && fs.f[i].rows) {
        sel[i] = s_sel[i];
        rows[i] = fs.f[i].rows;
      }
    }
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
    uint64_t need = 0;
    for (uint32_t j = 0; j < n_f; j++) {
      const FilterRef &f = fs.f[ord[j]];
      const uint32_t nb = clamp_blocks(s_nb_raw[ord[j]], f.cap_words / W, status);
      s_ord[j] = ord[j];
      s_nb[j] = nb;
      s_off[j] = static_cast<uint32_t>(need);
      need += static_cast<uint64_t>(nb) * W;
    }
    s_staged = need <= lds_filter_words;
    s_cnt = 0;
  }
  __syncthreads();
  const bool staged = s_staged != 0;
  if (staged) {
    for (uint32_t j = 0; j < n_f; j++) {
      const uint32_t n = s_nb[j] * W;
      const uint32_t *src = fs.f[__builtin_amdgcn_readfirstlane(s_ord[j])].words;
      uint32_t *dst = lds + s_off[j];
      for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
    }
  }
  __syncthreads();

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
  // Appended column c comes from slot app_slot[c]'s registers (-1: loaded).
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
  int64_t cnt;
  if (staged)
    cnt = probe_loop<K, ANY64, true, APPEND>(sl, off, n_f, k, lg, n_rows, bitmap, input_all, lds, slice, app,
                                             app_slot, vg);
  else
    cnt = probe_loop<K, ANY64, false, APPEND>(sl, off, n_f, k, lg, n_rows, bitmap, input_all, lds, slice, app,
                                              app_slot, vg);
  block_count_add(cnt, &s_cnt, count);
}

template <int B, int K, bool ANY64, bool APPEND>
__global__ void __launch_bounds__(kProbeThreads)
    k_probe(FilterSet fs, uint32_t k, uint32_t lg, uint64_t n_rows, uint64_t *__restrict__ bitmap,
            unsigned long long *count, uint32_t lds_filter_words, uint32_t input_all, uint32_t keep_order,
            uint32_t *status, AppendSet app) {
  probe_body<B, K, ANY64, APPEND>(fs, k, lg, n_rows, bitmap, count, lds_filter_words, input_all, keep_order,
                                  status, app, whole_grid());
}

// Launches k_probe<B, K, *, *> for one ProbeLaunch.
template <int B, int K>
hipError_t launch_probe_kernel(const ProbeLaunch &pl, hipStream_t s) {
  auto launch = [&](auto kern) -> hipError_t {
    hipError_t e = allow_lds(reinterpret_cast<const void *>(kern), pl.lds_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(pl.grid), dim3(kProbeThreads), pl.lds_bytes, s, pl.fs, pl.k, pl.lg, pl.n_rows,
                       pl.bitmap, pl.count, pl.lds_filter_words, pl.input_all, pl.keep_order, pl.status, pl.app);
    return hipGetLastError();
  };
  if (pl.app.n_cols)
    return pl.any64 ? launch(k_probe<B, K, true, true>) : launch(k_probe<B, K, false, true>);
  return pl.any64 ? launch(k_probe<B, K, true, false>) : launch(k_probe<B, K, false, false>);
}

}  // namespace pt
