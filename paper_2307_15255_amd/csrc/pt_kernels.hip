// pt_kernels.hip - gfx950 kernels of the predicate-transfer phase.
//
// A wave64 owns 64-row groups: lane l holds row 64 * w + l of bitmap word w,
// so a wave's ballot is the word. Every branch in the streaming loops is
// wave-uniform; per-lane work that does not matter (rows already removed,
// rows past the end) is computed anyway on clamped, in-bounds addresses and
// masked out, which keeps the exec mask full and the code straight-line.
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>

#include "pt_internal.hpp"

namespace pt {

namespace {

constexpr int kThreads = 256;        // local filter, build, size, compact
constexpr int kProbeThreads = 1024;  // probe: sixteen waves per workgroup
constexpr int kWideThreads = 1024;   // kernels that count: one workgroup (one atomic) per CU
constexpr int kProbeWaves = kProbeThreads / kWave;

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & (kWave - 1); }

// The wave's index in the grid, as a wave-uniform (scalar) value: the
// compiler cannot tell on its own that threadIdx.x / 64 is the same for
// every lane, and would otherwise keep loop counters derived from it in
// vector registers and turn every uniform branch into an exec-mask branch.
//
// A batched launch runs many tasks in one grid: each task owns a range of
// its workgroups, and sees them as a grid of its own (VGrid: this
// workgroup's index in the task, and the task's workgroup count).
struct VGrid {
  uint32_t block;
  uint32_t blocks;
};

__device__ __forceinline__ VGrid whole_grid() { return VGrid{blockIdx.x, gridDim.x}; }

__device__ __forceinline__ uint64_t global_wave(const VGrid &g) {
  const uint32_t w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  return static_cast<uint64_t>(g.block) * (blockDim.x / kWave) + w;
}

__device__ __forceinline__ uint64_t wave_count(const VGrid &g) {
  return static_cast<uint64_t>(g.blocks) * blockDim.x / kWave;
}


// The task of this workgroup. `first` holds the n + 1 first workgroups of
// the tasks (first[t] <= blockIdx.x < first[t + 1]) followed by the task of
// every workgroup of the grid, so the lookup is one load and one pair.
__device__ __forceinline__ uint32_t task_of(const uint32_t *first, uint32_t n, VGrid &g) {
  const uint32_t t = __builtin_amdgcn_readfirstlane(first[n + 1 + blockIdx.x]);
  const uint32_t a = __builtin_amdgcn_readfirstlane(first[t]);
  const uint32_t b = __builtin_amdgcn_readfirstlane(first[t + 1]);
  g = VGrid{blockIdx.x - a, b - a};
  return t;
}

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
  const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ uint64_t wave_sum(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = max(v, static_cast<uint32_t>(__shfl_xor(v, off)));
  return v;
}

// Adds a wave-uniform count into *out with one global atomic per workgroup.
__device__ __forceinline__ void block_count_add(int64_t wave_cnt, unsigned long long *s_cnt,
                                                unsigned long long *out) {
  if (lane_id() == 0 && wave_cnt) atomicAdd(s_cnt, static_cast<unsigned long long>(wave_cnt));
  __syncthreads();
  if (threadIdx.x == 0 && out && *s_cnt) atomicAdd(out, *s_cnt);
}

// A filter's block count as read from device memory, kept inside [1, cap]
// so that no address computed from it leaves the filter's buffer.
__device__ __forceinline__ uint32_t clamp_blocks(uint64_t nb, uint64_t cap_blocks) {
  if (nb > cap_blocks) nb = cap_blocks;
  return static_cast<uint32_t>(nb == 0 ? 1 : nb);
}

// Bits of word w that belong to rows below n_rows.
__device__ __forceinline__ uint64_t tail_mask(uint64_t w, uint64_t n_words, uint64_t n_rows) {
  if (w >= n_words) return 0;
  return (w + 1 == n_words && (n_rows & 63)) ? (1ull << (n_rows & 63)) - 1 : ~0ull;
}

// Exclusive prefix sum of v over the workgroup (blockDim.x entries of s).
__device__ __forceinline__ uint64_t block_exclusive_scan(uint64_t v, uint64_t *s, uint64_t &total) {
  const uint32_t t = threadIdx.x;
  s[t] = v;
  __syncthreads();
  for (uint32_t d = 1; d < blockDim.x; d <<= 1) {
    const uint64_t add = t >= d ? s[t - d] : 0;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  total = s[blockDim.x - 1];
  const uint64_t incl = s[t];
  __syncthreads();
  return incl - v;
}

// Selects filter i of a set without a dynamically indexed kernel argument.
__device__ __forceinline__ FilterRef pick(const FilterSet &fs, uint32_t i) {
  FilterRef r = fs.f[0];
#pragma unroll
  for (int j = 1; j < kMaxFilters; j++)
    if (i == static_cast<uint32_t>(j)) r = fs.f[j];
  return r;
}

// The filter hash of an int32 key: the same value as hash_key on its
// sign-extended image, with the sign correction done by a mask instead of
// a second full multiply.
__device__ __forceinline__ void hash_key32(uint32_t lo, uint32_t &h1, uint32_t &h2) {
  constexpr uint32_t a_lo = static_cast<uint32_t>(kHashMul);
  constexpr uint32_t a_hi = static_cast<uint32_t>(kHashMul >> 32);
  const uint64_t p = static_cast<uint64_t>(lo) * a_lo;
  const uint32_t fix = static_cast<uint32_t>(static_cast<int32_t>(lo) >> 31) & (0u - a_lo);
  const uint32_t hi = static_cast<uint32_t>(p >> 32) + lo * a_hi + fix;
  uint32_t t = static_cast<uint32_t>(p) ^ hi;
  t ^= t >> 16;
  h1 = hi;
  h2 = t * kMixMul;
}

__device__ __forceinline__ void hash_parts(uint32_t lo, uint32_t hi, bool key64, uint32_t &h1,
                                           uint32_t &h2) {
  if (key64)
    hash_key((static_cast<uint64_t>(hi) << 32) | lo, h1, h2);
  else
    hash_key32(lo, h1, h2);
}

// Set the k bits of a key. The test read bypasses the per-CU cache so it
// sees bits other workgroups have set; bits only go from 0 to 1 during a
// build, so a stale read costs an extra atomic, never a lost bit.
template <int B, int K>
__device__ __forceinline__ void insert_bits(uint32_t *words, uint32_t nb, uint32_t k, uint32_t h1,
                                            uint32_t h2) {
  using S = BlockShape<B>;
  uint32_t *blk = words + static_cast<uint64_t>(block_of(h1, nb)) * S::kWords;
  const uint32_t g1 = h2 >> (32 - S::kLog2);
  const uint32_t g2 = ((h2 >> (32 - 2 * S::kLog2)) & (B - 1)) | 1u;
  uint32_t pos = g1;
  const uint32_t kk = K > 0 ? static_cast<uint32_t>(K) : k;
#pragma unroll
  for (uint32_t i = 0; i < kk; i++) {
    const uint32_t p = pos & (B - 1);
    const uint32_t bit = 1u << (p & 31);
    uint32_t *w = blk + (p >> 5);
    if ((__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & bit) == 0)
      atomicOr(w, bit);
    pos += g2;
  }
}

// Set the k bits of a key with atomic OR alone (no read first).
template <int B, int K>
__device__ __forceinline__ void or_bits(uint32_t *words, uint32_t nb, uint32_t k, uint32_t h1, uint32_t h2) {
  using S = BlockShape<B>;
  uint32_t *blk = words + static_cast<uint64_t>(block_of(h1, nb)) * S::kWords;
  const uint32_t g1 = h2 >> (32 - S::kLog2);
  const uint32_t g2 = ((h2 >> (32 - 2 * S::kLog2)) & (B - 1)) | 1u;
  uint32_t pos = g1;
  const uint32_t kk = K > 0 ? static_cast<uint32_t>(K) : k;
#pragma unroll
  for (uint32_t i = 0; i < kk; i++) {
    const uint32_t p = pos & (B - 1);
    atomicOr(blk + (p >> 5), 1u << (p & 31));
    pos += g2;
  }
}

// ------------------------------------------------------------------ zero

__global__ void __launch_bounds__(kThreads) k_zero_u64(uint64_t *p, uint64_t n) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    p[i] = 0;
}

// All rows selected: the bitmap of a table without predicates.
__global__ void __launch_bounds__(kThreads)
    k_fill_all(uint64_t *bitmap, uint64_t n_rows, uint64_t *count) {
  const uint64_t n_words = (n_rows + 63) / 64;
  for (uint64_t w = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; w < n_words;
       w += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    bitmap[w] = tail_mask(w, n_words, n_rows);
  if (count && blockIdx.x == 0 && threadIdx.x == 0) *count = n_rows;
}

// ---------------------------------------------------------- local filter
//
// Each wave takes seg_words (1..64) consecutive words, builds word j with the
// ballot of step j, keeps it in lane j, and stores the segment with one
// coalesced store. Eight words are evaluated per step so their loads
// overlap.

__device__ __forceinline__ bool pred_holds(uint32_t op, int64_t v, int64_t lo, int64_t hi) {
  switch (op) {
    case 0: return v < lo;
    case 1: return v <= lo;
    case 2: return v > lo;
    case 3: return v >= lo;
    case 4: return v == lo;
    case 5: return v != lo;
    default: return lo <= v && v <= hi;
  }
}

__device__ __forceinline__ void local_body(const PredSet &ps, uint64_t n_rows, uint64_t *__restrict__ bitmap,
                                           unsigned long long *count, uint32_t seg_words, const VGrid &vg) {
  constexpr int T = 8;
  __shared__ unsigned long long s_cnt;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  const uint32_t lane = lane_id();
  const uint64_t n_words = (n_rows + 63) / 64;
  uint64_t cnt = 0;
  for (uint64_t seg = global_wave(vg); seg * seg_words < n_words; seg += wave_count(vg)) {
    const uint64_t w_base = seg * seg_words;
    const uint32_t n_j = static_cast<uint32_t>(n_words - w_base < seg_words ? n_words - w_base : seg_words);
    uint64_t mine = 0;
    for (uint32_t j0 = 0; j0 < n_j; j0 += T) {
      bool keep[T];
      uint64_t r[T];
#pragma unroll
      for (int t = 0; t < T; t++) {
        const uint64_t row = (w_base + j0 + t) * 64 + lane;
        keep[t] = j0 + t < n_j && row < n_rows;
        r[t] = row < n_rows ? row : n_rows - 1;
        if (ps.and_into && j0 + t < n_j)
          keep[t] = keep[t] && ((uniform64(bitmap[w_base + j0 + t]) >> lane) & 1);
      }
#pragma unroll
      for (int i = 0; i < kMaxPreds; i++) {
        if (i < static_cast<int>(ps.n)) {
          const PredRef &p = ps.p[i];
#pragma unroll
          for (int t = 0; t < T; t++) {
            const int64_t v = static_cast<int64_t>(load_key(p.col, p.col64, r[t]));
            keep[t] = keep[t] && pred_holds(p.op, v, p.lo, p.hi);
          }
        }
      }
#pragma unroll
      for (int t = 0; t < T; t++) {
        const uint64_t m = __ballot(keep[t]);
        if (lane == j0 + t) mine = m;
      }
    }
    if (lane < n_j) bitmap[w_base + lane] = mine;
    cnt += __popcll(mine);
  }
  block_count_add(static_cast<int64_t>(wave_sum(cnt)), &s_cnt, count);
}

__global__ void __launch_bounds__(kWideThreads)
    k_local(PredSet ps, uint64_t n_rows, uint64_t *__restrict__ bitmap,
            unsigned long long *count, uint32_t seg_words) {
  local_body(ps, n_rows, bitmap, count, seg_words, whole_grid());
}

// ------------------------------------------------------------------ probe
//
// One scan of the table probes every incoming filter (the incoming half of
// the filter transformation). At start each workgroup:
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

struct Slot {
  const void *keys;
  const uint32_t *words;
  uint32_t nb;
  uint32_t key64;
};

template <int B, int K, bool STAGED>
__device__ __forceinline__ bool slot_has(const Slot &s, const uint32_t *lds_filter, uint32_t h1,
                                         uint32_t h2, uint32_t k) {
  constexpr int W = BlockShape<B>::kWords;
  const uint32_t blk = block_of(h1, s.nb);
  if (STAGED) return block_has<B, K>(lds_filter + blk * W, h2, k);
  return block_has<B, K>(s.words + static_cast<uint64_t>(blk) * W, h2, k);
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

template <int B, int K, bool ANY64, bool STAGED, bool APPEND>
__device__ __forceinline__ int64_t probe_loop(const Slot (&sl)[kMaxProbe],
                                              const uint32_t (&lds_off)[kMaxProbe], uint32_t n_f,
                                              uint32_t k, uint64_t n_rows, uint64_t *bitmap,
                                              uint32_t input_all, const uint32_t *lds_filters,
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
      const bool ok = slot_has<B, K, STAGED>(sl[0], lds_filters + lds_off[0], h1, h2, k);
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
              const bool ok = slot_has<B, K, STAGED>(sl[s], lds_filters + lds_off[s], h1, h2, k);
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
            ok = ok && slot_has<B, K, STAGED>(sl[s], lds_filters + lds_off[s], h1, h2, k);
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
__device__ __forceinline__ void probe_body(const FilterSet &fs, uint32_t k, uint64_t n_rows,
                                           uint64_t *__restrict__ bitmap, unsigned long long *count,
                                           uint32_t lds_filter_words, uint32_t input_all,
                                           const AppendSet &app, const VGrid &vg) {
  extern __shared__ __align__(16) uint32_t lds[];
  constexpr int W = BlockShape<B>::kWords;
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
    const FilterRef f = pick(fs, threadIdx.x);
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
      if (i < static_cast<int>(n_f)) {
        if (fs.f[i].sel && fs.f[i].rows) {
          sel[i] = s_sel[i];
          rows[i] = fs.f[i].rows;
        }
      }
    }
    // stable insertion sort by sel / rows
    for (uint32_t a = 1; a < n_f; a++) {
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
      const FilterRef f = pick(fs, ord[j]);
      const uint32_t nb = clamp_blocks(s_nb_raw[ord[j]], f.cap_words / W);
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
      const uint32_t *src = pick(fs, s_ord[j]).words;
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
    const FilterRef f = pick(fs, __builtin_amdgcn_readfirstlane(s_ord[jj]));
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
  uint32_t *slice =
      lds + lds_filter_words + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave) * kSliceWords;
  int64_t cnt;
  if (staged)
    cnt = probe_loop<B, K, ANY64, true, APPEND>(sl, off, n_f, k, n_rows, bitmap, input_all, lds, slice,
                                                app, app_slot, vg);
  else
    cnt = probe_loop<B, K, ANY64, false, APPEND>(sl, off, n_f, k, n_rows, bitmap, input_all, lds, slice,
                                                 app, app_slot, vg);
  block_count_add(cnt, &s_cnt, count);
}

template <int B, int K, bool ANY64, bool APPEND>
__global__ void __launch_bounds__(kProbeThreads)
    k_probe(FilterSet fs, uint32_t k, uint64_t n_rows, uint64_t *__restrict__ bitmap,
            unsigned long long *count, uint32_t lds_filter_words, uint32_t input_all, AppendSet app) {
  probe_body<B, K, ANY64, APPEND>(fs, k, n_rows, bitmap, count, lds_filter_words, input_all, app,
                                  whole_grid());
}

// Many probes in one launch (one task each, see VGrid).
template <int B, int K, bool ANY64>
__global__ void __launch_bounds__(kProbeThreads)
    k_probe_batch(const ProbeTask *__restrict__ tasks, const uint32_t *__restrict__ first,
                  uint32_t n_tasks, uint32_t k, uint32_t lds_filter_words) {
  VGrid vg;
  const uint32_t t = task_of(first, n_tasks, vg);
  const ProbeTask &task = tasks[t];
  const AppendSet none{};
  probe_body<B, K, ANY64, false>(task.fs, k, task.n_rows, task.bitmap,
                                 reinterpret_cast<unsigned long long *>(task.count), lds_filter_words,
                                 task.input_all, none, vg);
}

// --------------------------------------------------------- size and zero
//
// Filter i (blockIdx.y) gets nb = max(1, ceil(count * bits_per_key / B))
// blocks, read from the device counter so the launch sequence never waits
// for the host. Its first nb blocks are zeroed unless the partitioned build
// (which writes every block) will run.


__device__ __forceinline__ uint64_t blocks_needed(uint64_t n_sel, uint32_t block_bits,
                                                  uint32_t bits_per_key, uint64_t cap_blocks) {
  uint64_t nb = (n_sel * bits_per_key + block_bits - 1) / block_bits;
  if (nb == 0) nb = 1;
  return nb > cap_blocks ? cap_blocks : nb;  // the cap is unreachable when it was checked
}

// Partitioned-build plan of one group of filters: filter f's tiles are
// buckets [base[f], base[f] + tiles[f]). ok: it fits the bucket table and
// the entry buffer (entries_cap entries).
constexpr uint64_t kTargetBuckets = 1024;

struct PartPlan {
  uint32_t nb[kMaxFilters];
  uint32_t base[kMaxFilters + 1];
  uint32_t tile_blocks;
  uint64_t n_sel;
  bool ok;
};

__device__ __forceinline__ PartPlan part_plan(const FilterSet &fs, uint32_t block_bits,
                                              uint32_t bits_per_key, const uint64_t *count,
                                              uint64_t n_rows, uint64_t entries_cap, bool from_count) {
  PartPlan pl{};
  const uint32_t W = block_bits / 32;
  pl.n_sel = count ? *count : n_rows;
  uint64_t all_blocks = 0;
#pragma unroll
  for (int i = 0; i < kMaxFilters; i++) {
    pl.nb[i] = 1;
    if (i < static_cast<int>(fs.n)) {
      const uint64_t cap_blocks = fs.f[i].cap_words / W;
      pl.nb[i] = from_count ? static_cast<uint32_t>(blocks_needed(pl.n_sel, block_bits, bits_per_key, cap_blocks))
                            : clamp_blocks(*fs.f[i].nb, cap_blocks);
      all_blocks += pl.nb[i];
    }
  }
  // Tiles of at most 64 KB, small enough that the group has about
  // kTargetBuckets of them (the fill kernel runs one workgroup per tile).
  uint64_t tb = (all_blocks + kTargetBuckets - 1) / kTargetBuckets;
  const uint64_t max_tb = kTileWords / W;
  pl.tile_blocks = static_cast<uint32_t>(tb < 1 ? 1 : (tb > max_tb ? max_tb : tb));
  uint64_t buckets = 0;
#pragma unroll
  for (int i = 0; i < kMaxFilters; i++) {
    pl.base[i] = static_cast<uint32_t>(buckets < kMaxBuckets ? buckets : kMaxBuckets);
    if (i < static_cast<int>(fs.n)) buckets += (pl.nb[i] + pl.tile_blocks - 1) / pl.tile_blocks;
  }
  pl.base[kMaxFilters] = static_cast<uint32_t>(buckets < kMaxBuckets ? buckets : kMaxBuckets);
  pl.ok = entries_cap > 0 && buckets <= kMaxBuckets && pl.n_sel * fs.n <= entries_cap;
  return pl;
}

__global__ void __launch_bounds__(kThreads)
    k_size_zero(FilterSet fs, uint32_t block_bits, uint32_t bits_per_key, const uint64_t *count,
                uint64_t n_rows, uint64_t entries_cap) {
  const FilterRef f = pick(fs, blockIdx.y);
  const uint64_t words_per_block = block_bits / 32;
  const uint64_t nb = blocks_needed(count ? *count : n_rows, block_bits, bits_per_key,
                                    f.cap_words / words_per_block);
  if (blockIdx.x == 0 && threadIdx.x == 0) *f.nb = nb;
  if (entries_cap && part_plan(fs, block_bits, bits_per_key, count, n_rows, entries_cap, true).ok)
    return;
  const uint64_t n = nb * words_per_block;
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    f.words[i] = 0;
}

// ------------------------------------------------------------------ build
//
// The outgoing half of the filter transformation: every selected row's key
// is inserted into each outgoing filter by OR (order-free, so the filter
// bits do not depend on scheduling). A wave takes a segment of bitmap words;
// a sparse segment is walked lane by lane (each lane pops the set bits of its
// own word), a dense one word by word (lanes = rows, coalesced key loads),
// whichever needs fewer steps.
//
// Filters that fit in LDS together are built without global atomics: each
// workgroup sets the bits of its rows in private LDS copies (LDS atomics),
// writes the copies to scratch memory, and a second kernel ORs the copies
// word by word into the filters. Larger filters are built in place with
// global atomic OR, skipped when a read already shows the bit set.

// Calls f(rows, ok) for the selected rows of segments seg_first,
// seg_first + seg_step, ... (seg_words words each), U rows per lane at a
// time: rows[u] is valid where bit u of ok is set. A batch of U rows lets
// the caller issue U key loads before it waits.
template <int U, typename F>
__device__ __forceinline__ void walk_rows(uint64_t seg_first, uint64_t seg_step, uint32_t seg_words,
                                          uint64_t n_rows, const uint64_t *bitmap, F &&f) {
  const uint32_t lane = lane_id();
  const uint64_t n_words = (n_rows + 63) / 64;
  // lane l holds word l of a segment of seg_words (1..64) words
  for (uint64_t seg = seg_first; seg * seg_words < n_words; seg += seg_step) {
    const uint64_t w = seg * seg_words + lane;
    uint64_t word = lane < seg_words ? tail_mask(w, n_words, n_rows) : 0;
    if (bitmap && lane < seg_words && w < n_words) word &= bitmap[w];
    const uint64_t nonzero = __ballot(word != 0);
    if (nonzero == 0) continue;
    // Sparse steps load 64 scattered rows at once; dense steps load 64
    // consecutive rows (one coalesced access). Walk sparsely only when that
    // needs clearly fewer steps.
    const uint32_t steps_sparse = wave_max(__popcll(word));
    const uint32_t steps_dense = __popcll(nonzero);
    if (4 * steps_sparse < steps_dense) {
      while (__ballot(word != 0)) {
        uint64_t rows[U];
        uint32_t ok = 0;
#pragma unroll
        for (int u = 0; u < U; u++) {
          rows[u] = 0;
          if (word) {
            rows[u] = w * 64 + (__ffsll(static_cast<unsigned long long>(word)) - 1);
            word &= word - 1;
            ok |= 1u << u;
          }
        }
        f(rows, ok);
      }
    } else {
      uint64_t todo = nonzero;
      while (todo) {
        uint64_t rows[U];
        uint32_t ok = 0;
#pragma unroll
        for (int u = 0; u < U; u++) {
          rows[u] = 0;
          if (todo) {
            const uint32_t j = __ffsll(static_cast<unsigned long long>(todo)) - 1;
            todo &= todo - 1;
            const uint64_t wj = __shfl(word, j);
            rows[u] = (seg * seg_words + j) * 64 + lane;
            if ((wj >> lane) & 1) ok |= 1u << u;
          }
        }
        f(rows, ok);
      }
    }
  }
}

// Filter hashes of the keys of up to U rows (those set in ok) in f's key
// column; the loads are issued together.
template <int U>
__device__ __forceinline__ void hash_rows(const FilterRef &f, const uint64_t (&row)[U], uint32_t ok,
                                          uint32_t (&h1)[U], uint32_t (&h2)[U]) {
  if (f.key64) {
    uint64_t x[U];
#pragma unroll
    for (int u = 0; u < U; u++) x[u] = (ok >> u) & 1 ? static_cast<const uint64_t *>(f.keys)[row[u]] : 0;
#pragma unroll
    for (int u = 0; u < U; u++) hash_key(x[u], h1[u], h2[u]);
  } else {
    uint32_t x[U];
#pragma unroll
    for (int u = 0; u < U; u++) x[u] = (ok >> u) & 1 ? static_cast<const uint32_t *>(f.keys)[row[u]] : 0;
#pragma unroll
    for (int u = 0; u < U; u++) hash_key32(x[u], h1[u], h2[u]);
  }
}

constexpr int kWalkBatch = 8;

// Filter hashes of up to U appended keys (those set in ok): slots
// base + idx[u] of appended column c.
template <int U>
__device__ __forceinline__ void hash_appended(const AppendSet &app, uint32_t c, uint64_t base,
                                              const uint32_t (&idx)[U], uint32_t ok, uint32_t (&h1)[U],
                                              uint32_t (&h2)[U]) {
  const void *col = app.dst[0];
  uint32_t key64 = app.key64[0];
#pragma unroll
  for (int j = 1; j < kMaxAppend; j++)
    if (c == static_cast<uint32_t>(j)) {
      col = app.dst[j];
      key64 = app.key64[j];
    }
  if (key64) {
    const uint64_t *p = static_cast<const uint64_t *>(col) + base;
    uint64_t x[U];
#pragma unroll
    for (int u = 0; u < U; u++) x[u] = (ok >> u) & 1 ? p[idx[u]] : 0;
#pragma unroll
    for (int u = 0; u < U; u++) hash_key(x[u], h1[u], h2[u]);
  } else {
    const uint32_t *p = static_cast<const uint32_t *>(col) + base;
    uint32_t x[U];
#pragma unroll
    for (int u = 0; u < U; u++) x[u] = (ok >> u) & 1 ? p[idx[u]] : 0;
#pragma unroll
    for (int u = 0; u < U; u++) hash_key32(x[u], h1[u], h2[u]);
  }
}

// Calls g(i, h1, h2) for every selected row and every filter i of fs, with
// the hashes of the row's key in filter i's key column. Without appended
// keys the grid's waves walk the bitmap; with them each wave takes whole
// regions, reading their appended keys (contiguous) or, for a region that
// overflowed, walking the bitmap words of the probe groups it covers.
template <typename G>
__device__ __forceinline__ void for_each_key(const FilterSet &fs, const AppendSet &app, uint64_t n_rows,
                                             const uint64_t *bitmap, uint32_t seg_words, const VGrid &vg,
                                             G &&g) {
  constexpr int U = kWalkBatch;
  auto from_rows = [&](const uint64_t (&row)[U], uint32_t ok) {
#pragma unroll
    for (int i = 0; i < kMaxFilters; i++) {
      if (i < static_cast<int>(fs.n)) {
        uint32_t h1[U], h2[U];
        hash_rows<U>(fs.f[i], row, ok, h1, h2);
#pragma unroll
        for (int u = 0; u < U; u++)
          if ((ok >> u) & 1) g(i, h1[u], h2[u]);
      }
    }
  };
  if (app.n_cols == 0) {
    walk_rows<U>(global_wave(vg), wave_count(vg), seg_words, n_rows, bitmap, from_rows);
    return;
  }
  const uint32_t lane = lane_id();
  for (uint64_t r = global_wave(vg); r < app.n_regions; r += wave_count(vg)) {
    const uint32_t n = __builtin_amdgcn_readfirstlane(app.counts[r]);
    if (n > app.region_cap) {
      walk_rows<U>(r, app.n_regions, app.group_words, n_rows, bitmap, from_rows);
      continue;
    }
    const uint64_t base = r * app.region_cap;
    for (uint32_t j0 = 0; j0 < n; j0 += U * kWave) {
      uint32_t idx[U];
      uint32_t ok = 0;
#pragma unroll
      for (int u = 0; u < U; u++) {
        idx[u] = j0 + u * kWave + lane;
        if (idx[u] < n) ok |= 1u << u;
      }
#pragma unroll
      for (int i = 0; i < kMaxFilters; i++) {
        if (i < static_cast<int>(fs.n)) {
          uint32_t h1[U], h2[U];
          hash_appended<U>(app, fs.f[i].app - 1, base, idx, ok, h1, h2);
#pragma unroll
          for (int u = 0; u < U; u++)
            if ((ok >> u) & 1) g(i, h1[u], h2[u]);
        }
      }
    }
  }
}

// Sets the k bits of (h1, h2) in a filter held in LDS.
template <int B, int K>
__device__ __forceinline__ void insert_lds(uint32_t *filter, uint32_t nb, uint32_t k, uint32_t h1,
                                           uint32_t h2) {
  using S = BlockShape<B>;
  uint32_t *blk = filter + block_of(h1, nb) * S::kWords;
  const uint32_t g1 = h2 >> (32 - S::kLog2);
  const uint32_t g2 = ((h2 >> (32 - 2 * S::kLog2)) & (B - 1)) | 1u;
  uint32_t pos = g1;
  const uint32_t kk = K > 0 ? static_cast<uint32_t>(K) : k;
#pragma unroll
  for (uint32_t i = 0; i < kk; i++) {
    const uint32_t p = pos & (B - 1);
    atomicOr(blk + (p >> 5), 1u << (p & 31));
    pos += g2;
  }
}

template <int B, int K>
__global__ void __launch_bounds__(kThreads)
    k_build(FilterSet fs, AppendSet app, uint32_t k, uint64_t n_rows, const uint64_t *__restrict__ bitmap,
            uint32_t seg_words) {
  uint32_t nb[kMaxFilters];
#pragma unroll
  for (int i = 0; i < kMaxFilters; i++)
    nb[i] = i < static_cast<int>(fs.n)
                ? clamp_blocks(*fs.f[i].nb, fs.f[i].cap_words / BlockShape<B>::kWords)
                : 1;
  for_each_key(fs, app, n_rows, bitmap, seg_words, whole_grid(), [&](int i, uint32_t h1, uint32_t h2) {
    insert_bits<B, K>(fs.f[i].words, nb[i], k, h1, h2);
  });
}

// Layout shared by the LDS build and its reduction: filter i's private copy
// starts at word off[i]; `fits` is false when the copies exceed lds_words.
struct LdsPlan {
  uint32_t nb[kMaxFilters];
  uint32_t off[kMaxFilters];
  uint32_t total;
  bool fits;
};

template <int B>
__device__ __forceinline__ LdsPlan lds_plan(const FilterSet &fs, uint32_t lds_words) {
  LdsPlan pl{};
  uint64_t total = 0;
#pragma unroll
  for (int i = 0; i < kMaxFilters; i++) {
    pl.nb[i] = 1;
    pl.off[i] = 0;
    if (i < static_cast<int>(fs.n)) {
      pl.nb[i] = clamp_blocks(*fs.f[i].nb, fs.f[i].cap_words / BlockShape<B>::kWords);
      pl.off[i] = static_cast<uint32_t>(total < 0xFFFFFFFFull ? total : 0);
      total += static_cast<uint64_t>(pl.nb[i]) * BlockShape<B>::kWords;
    }
  }
  pl.fits = total <= lds_words;
  pl.total = pl.fits ? static_cast<uint32_t>(total) : 0;
  return pl;
}

template <int B, int K>
__global__ void __launch_bounds__(kWideThreads)
    k_build_lds(FilterSet fs, AppendSet app, uint32_t k, uint64_t n_rows, const uint64_t *__restrict__ bitmap,
                uint32_t seg_words, uint32_t *__restrict__ partials, uint32_t lds_words) {
  extern __shared__ __align__(16) uint32_t lds[];
  const LdsPlan pl = lds_plan<B>(fs, lds_words);
  if (!pl.fits) {
    // Too large for LDS: insert in place with global atomics.
    for_each_key(fs, app, n_rows, bitmap, seg_words, whole_grid(), [&](int i, uint32_t h1, uint32_t h2) {
      insert_bits<B, K>(fs.f[i].words, pl.nb[i], k, h1, h2);
    });
    return;
  }
  for (uint32_t j = threadIdx.x; j < pl.total; j += blockDim.x) lds[j] = 0;
  __syncthreads();
  for_each_key(fs, app, n_rows, bitmap, seg_words, whole_grid(), [&](int i, uint32_t h1, uint32_t h2) {
    insert_lds<B, K>(lds + pl.off[i], pl.nb[i], k, h1, h2);
  });
  __syncthreads();
  uint32_t *out = partials + static_cast<uint64_t>(blockIdx.x) * lds_words;
  for (uint32_t j = threadIdx.x; j < pl.total; j += blockDim.x) out[j] = lds[j];
}

// filter i (blockIdx.y) = OR over the n_parts private copies. A workgroup
// takes 64 consecutive words: its 16 waves each OR every 16th copy (loads
// issued together, coalesced across the 64 lanes), then one wave combines
// the 16 partial results through LDS.
template <int B>
__global__ void __launch_bounds__(kWideThreads)
    k_build_reduce(FilterSet fs, const uint32_t *__restrict__ partials, uint32_t n_parts,
                   uint32_t lds_words) {
  constexpr int kGroups = kWideThreads / kWave;
  __shared__ uint32_t s_or[kGroups][kWave];
  const LdsPlan pl = lds_plan<B>(fs, lds_words);
  if (!pl.fits) return;
  uint32_t i = 0, off = pl.off[0], nb = pl.nb[0];
#pragma unroll
  for (int j = 1; j < kMaxFilters; j++)
    if (blockIdx.y == static_cast<uint32_t>(j)) {
      i = j;
      off = pl.off[j];
      nb = pl.nb[j];
    }
  uint32_t *words = pick(fs, i).words;
  const uint32_t n = nb * BlockShape<B>::kWords;
  const uint32_t lane = lane_id();
  const uint32_t g = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  for (uint32_t base = blockIdx.x * kWave; base < n; base += gridDim.x * kWave) {
    const uint32_t w = base + lane;
    uint32_t v = 0;
    if (w < n) {
#pragma unroll 8
      for (uint32_t p = g; p < n_parts; p += kGroups)
        v |= partials[static_cast<uint64_t>(p) * lds_words + off + w];
    }
    s_or[g][lane] = v;
    __syncthreads();
    if (g == 0 && w < n) {
      uint32_t r = 0;
#pragma unroll
      for (int q = 0; q < kGroups; q++) r |= s_or[q][lane];
      words[w] = r;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------- partitioned build
//
// Filters too large for LDS are built tile by tile: the filter's blocks are
// cut into 64 KB tiles and every (filter, tile) pair is a bucket.
//   count    each workgroup walks its rows and histograms their bucket
//            in LDS, then stores its histogram row;
//   scan     per bucket, an exclusive scan over the workgroups' counts, then
//            one scan over the bucket totals: every (workgroup, bucket) gets
//            its own range of the entry buffer;
//   scatter  the same walk again (same grid, so the same rows per
//            workgroup) writes each entry - block within the tile and H2 -
//            at its range's next slot (LDS cursors); when the plan does not
//            fit, this kernel inserts in place with global atomics instead;
//   fill     one workgroup per bucket sets the bits of its entries in an LDS
//            tile and stores the whole tile (every block of the filter is
//            written exactly once).
// No step needs a global atomic.

// An entry is 32 bits: the block within its tile above the top 2 log2(B)
// bits of H2, the only bits of H2 the bit positions use. Tiles hold at most
// 64 KB, so the block index fits (14 bits for B = 32, 9 for B = 1024).
template <int B>
__device__ __forceinline__ uint32_t pack_entry(uint32_t blk_in_tile, uint32_t h2) {
  constexpr int L2 = 2 * BlockShape<B>::kLog2;
  return (blk_in_tile << L2) | (h2 >> (32 - L2));
}
template <int B>
__device__ __forceinline__ uint32_t entry_block(uint32_t v) {
  return v >> (2 * BlockShape<B>::kLog2);
}
template <int B>
__device__ __forceinline__ uint32_t entry_h2(uint32_t v) {
  constexpr int L2 = 2 * BlockShape<B>::kLog2;
  return v << (32 - L2);
}

template <int B>
__device__ __forceinline__ uint32_t bucket_of(const PartPlan &pl, int f, uint32_t h1, uint32_t &blk) {
  blk = block_of(h1, pl.nb[f]);
  return pl.base[f] + blk / pl.tile_blocks;
}

template <int B>
__global__ void __launch_bounds__(kWideThreads)
    k_part_count(FilterSet fs, AppendSet app, uint32_t bits_per_key, const uint64_t *count, uint64_t n_rows,
                 const uint64_t *__restrict__ bitmap, uint32_t seg_words, uint64_t entries_cap,
                 uint32_t *__restrict__ hist) {
  extern __shared__ __align__(16) uint32_t s_hist[];
  const PartPlan pl = part_plan(fs, B, bits_per_key, count, n_rows, entries_cap, false);
  if (!pl.ok) return;
  const uint32_t buckets = pl.base[kMaxFilters];
  for (uint32_t b = threadIdx.x; b < buckets; b += blockDim.x) s_hist[b] = 0;
  __syncthreads();
  for_each_key(fs, app, n_rows, bitmap, seg_words, whole_grid(), [&](int i, uint32_t h1, uint32_t h2) {
    uint32_t blk;
    atomicAdd(&s_hist[bucket_of<B>(pl, i, h1, blk)], 1u);
  });
  __syncthreads();
  uint32_t *row_out = hist + static_cast<uint64_t>(blockIdx.x) * kMaxBuckets;
  for (uint32_t b = threadIdx.x; b < buckets; b += blockDim.x) row_out[b] = s_hist[b];
}

// Bucket b (blockIdx.x): exclusive scan of hist[g][b] over the n_groups
// workgroups, in place; the bucket's total goes to totals[b].
__global__ void __launch_bounds__(kWideThreads)
    k_part_scan_groups(FilterSet fs, uint32_t block_bits, uint32_t bits_per_key,
                       const uint64_t *count, uint64_t n_rows, uint64_t entries_cap,
                       uint32_t *__restrict__ hist, uint32_t n_groups, uint64_t *__restrict__ totals) {
  __shared__ uint64_t s[kWideThreads];
  const PartPlan pl = part_plan(fs, block_bits, bits_per_key, count, n_rows, entries_cap, false);
  if (!pl.ok) return;
  for (uint32_t b = blockIdx.x; b < pl.base[kMaxFilters]; b += gridDim.x) {
    const uint32_t g = threadIdx.x;
    const uint64_t v = g < n_groups ? hist[static_cast<uint64_t>(g) * kMaxBuckets + b] : 0;
    uint64_t total;
    const uint64_t ex = block_exclusive_scan(v, s, total);
    if (g < n_groups) hist[static_cast<uint64_t>(g) * kMaxBuckets + b] = static_cast<uint32_t>(ex);
    if (g == 0) totals[b] = total;
  }
}

// starts[b] = sum of totals[0..b) for every bucket, starts[buckets] = all.
__global__ void __launch_bounds__(kWideThreads)
    k_part_scan_buckets(FilterSet fs, uint32_t block_bits, uint32_t bits_per_key,
                        const uint64_t *count, uint64_t n_rows, uint64_t entries_cap,
                        const uint64_t *__restrict__ totals, uint64_t *__restrict__ starts) {
  __shared__ uint64_t s[kWideThreads];
  const PartPlan pl = part_plan(fs, block_bits, bits_per_key, count, n_rows, entries_cap, false);
  if (!pl.ok) return;
  const uint32_t buckets = pl.base[kMaxFilters];
  uint64_t carry = 0;
  for (uint32_t base = 0; base < buckets; base += blockDim.x) {
    const uint32_t b = base + threadIdx.x;
    const uint64_t v = b < buckets ? totals[b] : 0;
    uint64_t total;
    const uint64_t ex = block_exclusive_scan(v, s, total);
    if (b < buckets) starts[b] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) starts[buckets] = carry;
}

template <int B, int K>
__global__ void __launch_bounds__(kWideThreads)
    k_part_scatter(FilterSet fs, AppendSet app, uint32_t k, uint32_t bits_per_key, const uint64_t *count,
                   uint64_t n_rows, const uint64_t *__restrict__ bitmap, uint32_t seg_words,
                   uint64_t entries_cap, const uint32_t *__restrict__ hist,
                   const uint64_t *__restrict__ starts, uint32_t *__restrict__ entries) {
  extern __shared__ __align__(16) uint64_t s_cur[];
  const PartPlan pl = part_plan(fs, B, bits_per_key, count, n_rows, entries_cap, false);
  if (!pl.ok) {
    // The plan does not fit: insert in place with global atomics (the size
    // kernel zeroed the filters in this case).
    for_each_key(fs, app, n_rows, bitmap, seg_words, whole_grid(), [&](int i, uint32_t h1, uint32_t h2) {
      insert_bits<B, K>(fs.f[i].words, pl.nb[i], k, h1, h2);
    });
    return;
  }
  const uint32_t buckets = pl.base[kMaxFilters];
  const uint32_t *my = hist + static_cast<uint64_t>(blockIdx.x) * kMaxBuckets;
  // s_cur[b]: the next entry slot of this workgroup in bucket b
  for (uint32_t b = threadIdx.x; b < buckets; b += blockDim.x) s_cur[b] = starts[b] + my[b];
  __syncthreads();
  for_each_key(fs, app, n_rows, bitmap, seg_words, whole_grid(), [&](int i, uint32_t h1, uint32_t h2) {
    uint32_t blk;
    const uint32_t b = bucket_of<B>(pl, i, h1, blk);
    const uint64_t pos = atomicAdd(&s_cur[b], static_cast<uint64_t>(1));
    if (pos < entries_cap)  // always true while *count is the bitmap's popcount
      entries[pos] = pack_entry<B>(blk % pl.tile_blocks, h2);
  });
}

template <int B, int K>
__global__ void __launch_bounds__(kWideThreads)
    k_part_fill(FilterSet fs, uint32_t k, uint32_t bits_per_key, const uint64_t *count,
                uint64_t n_rows, uint64_t entries_cap, const uint64_t *__restrict__ starts,
                const uint32_t *__restrict__ entries) {
  constexpr int W = BlockShape<B>::kWords;
  extern __shared__ __align__(16) uint32_t tile[];
  const PartPlan pl = part_plan(fs, B, bits_per_key, count, n_rows, entries_cap, false);
  if (!pl.ok) return;
  for (uint32_t b = blockIdx.x; b < pl.base[kMaxFilters]; b += gridDim.x) {
    int f = 0;
#pragma unroll
    for (int i = 1; i < kMaxFilters; i++)
      if (i < static_cast<int>(fs.n) && b >= pl.base[i]) f = i;
    uint32_t nb = pl.nb[0], base = pl.base[0];
#pragma unroll
    for (int i = 1; i < kMaxFilters; i++)
      if (i == f) {
        nb = pl.nb[i];
        base = pl.base[i];
      }
    const uint32_t t = b - base;
    const uint32_t first = t * pl.tile_blocks;
    const uint32_t n_blocks = min(pl.tile_blocks, nb - first);
    for (uint32_t j = threadIdx.x; j < n_blocks * W; j += blockDim.x) tile[j] = 0;
    __syncthreads();
    for (uint64_t e = starts[b] + threadIdx.x; e < starts[b + 1]; e += blockDim.x) {
      const uint32_t v = entries[e];
      // the entry names its block inside the tile; with nb = 1 and h1 = 0,
      // insert_lds sets the key's k bits in the block it is pointed at
      insert_lds<B, K>(tile + entry_block<B>(v) * W, 1, k, 0, entry_h2<B>(v));
    }
    __syncthreads();
    uint32_t *out = pick(fs, f).words + static_cast<uint64_t>(first) * W;
    for (uint32_t j = threadIdx.x; j < n_blocks * W; j += blockDim.x) out[j] = tile[j];
    __syncthreads();
  }
}

// ------------------------------------------------------------- counters

struct SlotTable {
  uint32_t slot[64];
};

__global__ void k_copy_counts(const uint64_t *src, SlotTable t, uint32_t n, uint64_t *dst) {
  const uint32_t i = threadIdx.x;
  if (i < n) dst[i] = src[t.slot[i]];
}

// -------------------------------------------------------------- compact
//
// Ordered compaction in three steps: per-workgroup popcounts of 1024 bitmap
// words, one exclusive scan over the workgroup totals, then each workgroup
// rescans its words and writes the set rows' ids in ascending order.

constexpr uint64_t kCompactWordsPerBlock = 1024;  // 4 words per thread

__global__ void __launch_bounds__(kThreads)
    k_compact_count(const uint64_t *__restrict__ bitmap, uint64_t n_words, uint64_t n_rows,
                    uint64_t *partials) {
  __shared__ unsigned long long s_cnt;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  const uint64_t base = blockIdx.x * kCompactWordsPerBlock + threadIdx.x * 4;
  uint64_t c = 0;
#pragma unroll
  for (int j = 0; j < 4; j++)
    if (base + j < n_words) c += __popcll(bitmap[base + j] & tail_mask(base + j, n_words, n_rows));
  atomicAdd(&s_cnt, static_cast<unsigned long long>(c));
  __syncthreads();
  if (threadIdx.x == 0) partials[blockIdx.x] = s_cnt;
}

__global__ void __launch_bounds__(1024) k_compact_scan(uint64_t *partials, uint64_t n_parts,
                                                       uint64_t *count) {
  __shared__ uint64_t s[1024];
  uint64_t carry = 0;
  for (uint64_t base = 0; base < n_parts; base += blockDim.x) {
    const uint64_t i = base + threadIdx.x;
    const uint64_t v = i < n_parts ? partials[i] : 0;
    uint64_t total;
    const uint64_t ex = block_exclusive_scan(v, s, total);
    if (i < n_parts) partials[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) *count = carry;
}

__global__ void __launch_bounds__(kThreads)
    k_compact_write(const uint64_t *__restrict__ bitmap, uint64_t n_words, uint64_t n_rows,
                    const uint64_t *partials, uint32_t *__restrict__ idx) {
  __shared__ uint64_t s[kThreads];
  const uint64_t base = blockIdx.x * kCompactWordsPerBlock + threadIdx.x * 4;
  uint64_t words[4];
  uint64_t c = 0;
#pragma unroll
  for (int j = 0; j < 4; j++) {
    words[j] = base + j < n_words ? bitmap[base + j] & tail_mask(base + j, n_words, n_rows) : 0;
    c += __popcll(words[j]);
  }
  uint64_t total;
  uint64_t pos = partials[blockIdx.x] + block_exclusive_scan(c, s, total);
#pragma unroll
  for (int j = 0; j < 4; j++) {
    uint64_t m = words[j];
    while (m) {
      const uint32_t b = __ffsll(static_cast<unsigned long long>(m)) - 1;
      idx[pos++] = static_cast<uint32_t>((base + j) * 64 + b);
      m &= m - 1;
    }
  }
}

// ------------------------------------------------------------ dispatch

// ---------------------------------------------------------- batched steps
//
// The same steps for many tables of many problems at once: each workgroup
// finds its task (task_of) and runs the step's body on the task's share of
// the grid.

__global__ void __launch_bounds__(kBatchThreads)
    k_local_batch(const LocalTask *__restrict__ tasks, const uint32_t *__restrict__ first, uint32_t n) {
  VGrid vg;
  const LocalTask &t = tasks[task_of(first, n, vg)];
  local_body(t.ps, t.n_rows, t.bitmap, reinterpret_cast<unsigned long long *>(t.count), t.seg_words, vg);
}

__global__ void __launch_bounds__(kBatchThreads)
    k_size_batch(const SizeTask *__restrict__ tasks, const uint32_t *__restrict__ first, uint32_t n) {
  VGrid vg;
  const SizeTask &t = tasks[task_of(first, n, vg)];
  const uint64_t W = t.block_bits / 32;
  const uint64_t nb = blocks_needed(t.count ? *t.count : t.n_rows, t.block_bits, t.bits_per_key,
                                    t.f.cap_words / W);
  if (vg.block == 0 && threadIdx.x == 0) *t.f.nb = nb;
  const uint64_t words = nb * W;
  for (uint64_t i = static_cast<uint64_t>(vg.block) * blockDim.x + threadIdx.x; i < words;
       i += static_cast<uint64_t>(vg.blocks) * blockDim.x)
    t.f.words[i] = 0;
}

// Filters that fit the launch's LDS are built in private copies and merged
// into the (zeroed) filters: stored when the task has one workgroup, OR-ed
// with atomics otherwise. Larger ones are built with global atomics.
template <int B, int K>
__global__ void __launch_bounds__(kBatchThreads)
    k_build_batch(const BuildTask *__restrict__ tasks, const uint32_t *__restrict__ first, uint32_t n,
                  uint32_t k, uint32_t lds_words) {
  extern __shared__ __align__(16) uint32_t lds[];
  constexpr int W = BlockShape<B>::kWords;
  VGrid vg;
  const BuildTask &t = tasks[task_of(first, n, vg)];
  const FilterSet &fs = t.fs;
  const AppendSet none{};
  const LdsPlan pl = lds_plan<B>(fs, lds_words);
  if (!pl.fits) {
    // atomic OR without a prior read: nothing waits on the result, so a
    // wave's inserts overlap
    for_each_key(fs, none, t.n_rows, t.bitmap, t.seg_words, vg, [&](int i, uint32_t h1, uint32_t h2) {
      or_bits<B, K>(fs.f[i].words, pl.nb[i], k, h1, h2);
    });
    return;
  }
  for (uint32_t j = threadIdx.x; j < pl.total; j += blockDim.x) lds[j] = 0;
  __syncthreads();
  for_each_key(fs, none, t.n_rows, t.bitmap, t.seg_words, vg, [&](int i, uint32_t h1, uint32_t h2) {
    insert_lds<B, K>(lds + pl.off[i], pl.nb[i], k, h1, h2);
  });
  __syncthreads();
  const bool alone = vg.blocks == 1;
#pragma unroll
  for (int i = 0; i < kMaxFilters; i++) {
    if (i < static_cast<int>(fs.n)) {
      uint32_t *words = fs.f[i].words;
      const uint32_t *mine = lds + pl.off[i];
      for (uint32_t j = threadIdx.x; j < pl.nb[i] * W; j += blockDim.x) {
        const uint32_t v = mine[j];
        if (alone) words[j] = v;
        else if (v) atomicOr(words + j, v);
      }
    }
  }
}

__global__ void k_copy_pairs(const CopyPair *__restrict__ pairs, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) *pairs[i].dst = *pairs[i].src;
}

template <typename F>
hipError_t by_block_bits(uint32_t block_bits, F &&f) {
  switch (block_bits) {
    case 32: return f(std::integral_constant<int, 32>{});
    case 64: return f(std::integral_constant<int, 64>{});
    case 128: return f(std::integral_constant<int, 128>{});
    case 256: return f(std::integral_constant<int, 256>{});
    case 512: return f(std::integral_constant<int, 512>{});
    case 1024: return f(std::integral_constant<int, 1024>{});
    default: return hipErrorInvalidValue;
  }
}

// Raises a kernel's dynamic-LDS limit once per device (to the largest
// request seen); later launches that fit skip the call.
hipError_t allow_lds(const void *kern, uint64_t bytes) {
  static std::mutex mu;
  static std::map<std::pair<int, const void *>, uint64_t> granted;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  std::lock_guard<std::mutex> lock(mu);
  uint64_t &g = granted[{dev, kern}];
  if (bytes <= g) return hipSuccess;
  const uint64_t want = static_cast<uint64_t>(device_info().max_lds_block) - 1024;
  hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     static_cast<int>(bytes > want ? bytes : want));
  if (e == hipSuccess) g = bytes > want ? bytes : want;
  return e;
}

// Bitmap words per wave for the word-segment kernels: enough waves to cover
// the device several times over, at most one word per lane.
uint32_t segment_words(uint64_t n_words) {
  const uint64_t target_waves = static_cast<uint64_t>(device_info().n_cu) * 32;
  uint64_t seg = (n_words + target_waves - 1) / target_waves;
  return static_cast<uint32_t>(seg < 1 ? 1 : (seg > 64 ? 64 : seg));
}

uint32_t grid_for(uint64_t waves_of_work, uint32_t threads, uint32_t per_cu) {
  const uint64_t blocks = (waves_of_work * kWave + threads - 1) / threads;
  const uint64_t cap = static_cast<uint64_t>(device_info().n_cu) * per_cu;
  const uint64_t g = blocks < cap ? blocks : cap;
  return static_cast<uint32_t>(g == 0 ? 1 : g);
}

}  // namespace

hipError_t launch_zero_u64(uint64_t *p, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const uint32_t grid = grid_for((n + 63) / 64, kThreads, 4);
  hipLaunchKernelGGL(k_zero_u64, dim3(grid), dim3(kThreads), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_fill_all(uint64_t *bitmap, uint64_t n_rows, uint64_t *count, hipStream_t s) {
  const uint64_t n_words = (n_rows + 63) / 64;
  const uint32_t grid = grid_for((n_words + 63) / 64, kThreads, 8);
  hipLaunchKernelGGL(k_fill_all, dim3(grid), dim3(kThreads), 0, s, n_words ? bitmap : nullptr, n_rows,
                     count);
  return hipGetLastError();
}

hipError_t launch_local_filter(const PredSet &preds, uint64_t n_rows, uint64_t *bitmap,
                               uint64_t *count, hipStream_t s) {
  const uint64_t n_words = (n_rows + 63) / 64;
  if (n_words == 0) return hipSuccess;
  const uint32_t seg_words = segment_words(n_words);
  const uint32_t grid = grid_for((n_words + seg_words - 1) / seg_words, kWideThreads, 1);
  hipLaunchKernelGGL(k_local, dim3(grid), dim3(kWideThreads), 0, s, preds, n_rows, bitmap,
                     reinterpret_cast<unsigned long long *>(count), seg_words);
  return hipGetLastError();
}

hipError_t launch_probe(uint32_t block_bits, uint32_t k, const FilterSet &fs, uint64_t n_rows,
                        uint64_t *bitmap, uint64_t *count, bool input_all, AppendSet *app,
                        uint64_t capacity, hipStream_t s) {
  const uint64_t n_words = (n_rows + 63) / 64;
  if (n_words == 0 || fs.n == 0) {
    if (app) app->n_cols = 0;
    return hipSuccess;
  }
  bool any64 = false;
  uint64_t want_words = 0;
  for (uint32_t i = 0; i < fs.n; i++) {
    any64 = any64 || fs.f[i].key64;
    want_words += fs.f[i].cap_words;
  }
  const DeviceInfo &di = device_info();
  const uint64_t queue_bytes = static_cast<uint64_t>(kProbeWaves) * 4 *
                               (any64 ? probe_slice_words<true>() : probe_slice_words<false>());
  // Leave room for the kernel's own static LDS (a few dozen bytes).
  const uint64_t lds_max = static_cast<uint64_t>(di.max_lds_block) - 1024;
  uint64_t filter_bytes = lds_max > queue_bytes ? lds_max - queue_bytes : 0;
  if (filter_bytes > want_words * 4) filter_bytes = want_words * 4;
  const uint64_t lds_bytes = filter_bytes + queue_bytes;
  const uint32_t per_cu = lds_bytes * 2 <= lds_max ? 2 : 1;
  const int U = any64 ? 4 : 8;
  const uint32_t grid = grid_for((n_words + U - 1) / U, kProbeThreads, per_cu);
  const uint32_t filter_words = static_cast<uint32_t>(filter_bytes / 8) * 2;  // keep slices 8-byte aligned
  auto *cnt = reinterpret_cast<unsigned long long *>(count);
  // Region geometry of the appended keys: one region per wave of the grid,
  // capacity / regions slots each (at most the rows a wave can see).
  AppendSet a{};
  if (app && app->n_cols > 0 && app->n_cols <= static_cast<uint32_t>(kMaxAppend) && app->counts) {
    const uint64_t regions = static_cast<uint64_t>(grid) * kProbeWaves;
    const uint64_t groups = (n_words + U - 1) / U;
    const uint64_t most = (groups + regions - 1) / regions * U * 64;
    uint64_t cap = capacity / regions;
    if (cap > most) cap = most;
    if (regions <= kMaxRegions && cap >= 64) {
      a = *app;
      a.n_regions = static_cast<uint32_t>(regions);
      a.region_cap = static_cast<uint32_t>(cap);
      a.group_words = static_cast<uint32_t>(U);
    }
  }
  if (app) *app = a;
  const uint32_t all = input_all ? 1u : 0u;
  return by_block_bits(block_bits, [&](auto bb) -> hipError_t {
    constexpr int B = decltype(bb)::value;
    auto launch = [&](auto kern) -> hipError_t {
      hipError_t e = allow_lds(reinterpret_cast<const void *>(kern), lds_bytes);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(kern, dim3(grid), dim3(kProbeThreads), lds_bytes, s, fs, k, n_rows,
                         bitmap, cnt, filter_words, all, a);
      return hipGetLastError();
    };
    if (a.n_cols) {
      if (k == 3) return any64 ? launch(k_probe<B, 3, true, true>) : launch(k_probe<B, 3, false, true>);
      return any64 ? launch(k_probe<B, 0, true, true>) : launch(k_probe<B, 0, false, true>);
    }
    if (k == 3) return any64 ? launch(k_probe<B, 3, true, false>) : launch(k_probe<B, 3, false, false>);
    return any64 ? launch(k_probe<B, 0, true, false>) : launch(k_probe<B, 0, false, false>);
  });
}

uint64_t build_lds_words() {
  // LDS of one build workgroup: the private filter copies.
  return (static_cast<uint64_t>(device_info().max_lds_block) - 1024) / 4;
}

hipError_t launch_build(uint32_t block_bits, uint32_t k, uint32_t bits_per_key, const FilterSet &fs,
                        uint64_t n_rows, const uint64_t *bitmap, const uint64_t *count,
                        const BuildScratch *scratch, const AppendSet *app, hipStream_t s) {
  if (fs.n == 0) return hipSuccess;
  // Appended keys are used only when every filter names one of them.
  AppendSet a{};
  if (app && app->n_cols > 0 && app->n_cols <= static_cast<uint32_t>(kMaxAppend)) {
    bool all = true;
    for (uint32_t i = 0; i < fs.n; i++) all = all && fs.f[i].app >= 1 && fs.f[i].app <= app->n_cols;
    if (all) a = *app;
  }
  const uint64_t n_words = (n_rows + 63) / 64;
  const uint32_t seg_words = segment_words(n_words ? n_words : 1);
  const uint64_t lds_words = build_lds_words();
  uint64_t cap_words = 0, max_cap_words = 0;
  for (uint32_t i = 0; i < fs.n; i++) {
    cap_words += fs.f[i].cap_words;
    max_cap_words = fs.f[i].cap_words > max_cap_words ? fs.f[i].cap_words : max_cap_words;
  }
  // Which path: private LDS copies when all filters surely fit in LDS, the
  // partitioned build when the caller gave its buffers, else atomics.
  enum { kLds, kPart, kAtomic } path = kAtomic;
  if (scratch && scratch->copies && cap_words <= lds_words) path = kLds;
  else if (scratch && scratch->entries && scratch->entries_cap) path = kPart;
  // PT_BUILD_PATH=atomic|part (testing): take that path where it is allowed.
  if (const char *force = std::getenv("PT_BUILD_PATH")) {
    if (std::strcmp(force, "atomic") == 0) path = kAtomic;
    else if (std::strcmp(force, "part") == 0 && scratch && scratch->entries && scratch->entries_cap)
      path = kPart;
  }
  const uint64_t entries_cap = path == kPart ? scratch->entries_cap : 0;

  // Size (and zero, when the build writes in place).
  {
    uint64_t gx = (max_cap_words + kThreads * 4 - 1) / (kThreads * 4);
    const uint64_t cap = static_cast<uint64_t>(device_info().n_cu) * 2;
    gx = gx > cap ? cap : (gx == 0 ? 1 : gx);
    hipLaunchKernelGGL(k_size_zero, dim3(static_cast<uint32_t>(gx), fs.n), dim3(kThreads), 0, s, fs,
                       block_bits, bits_per_key, count, n_rows, entries_cap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n_words == 0) return e;
  }

  if (path == kAtomic) {
    const uint32_t grid = grid_for((n_words + seg_words - 1) / seg_words, kThreads, 8);
    return by_block_bits(block_bits, [&](auto bb) -> hipError_t {
      constexpr int B = decltype(bb)::value;
      if (k == 3)
        hipLaunchKernelGGL((k_build<B, 3>), dim3(grid), dim3(kThreads), 0, s, fs, a, k, n_rows, bitmap,
                           seg_words);
      else
        hipLaunchKernelGGL((k_build<B, 0>), dim3(grid), dim3(kThreads), 0, s, fs, a, k, n_rows, bitmap,
                           seg_words);
      return hipGetLastError();
    });
  }

  if (path == kLds) {
    const uint64_t copy_words = cap_words;
    uint64_t parts = scratch->copies_words / copy_words;
    const uint64_t work_parts = (n_words + seg_words * 16 - 1) / (seg_words * 16);
    if (parts > static_cast<uint64_t>(device_info().n_cu)) parts = device_info().n_cu;
    if (parts > work_parts) parts = work_parts;
    if (parts == 0) parts = 1;
    const uint32_t cw = static_cast<uint32_t>(copy_words);
    const uint32_t n_parts = static_cast<uint32_t>(parts);
    return by_block_bits(block_bits, [&](auto bb) -> hipError_t {
      constexpr int B = decltype(bb)::value;
      auto kern = k == 3 ? k_build_lds<B, 3> : k_build_lds<B, 0>;
      hipError_t e = allow_lds(reinterpret_cast<const void *>(kern), copy_words * 4);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(kern, dim3(n_parts), dim3(kWideThreads), copy_words * 4, s, fs, a, k, n_rows,
                         bitmap, seg_words, scratch->copies, cw);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      uint64_t gx = (copy_words + kWave - 1) / kWave;
      if (gx > 1024) gx = 1024;
      hipLaunchKernelGGL((k_build_reduce<B>), dim3(static_cast<uint32_t>(gx), fs.n), dim3(kWideThreads),
                         0, s, fs, scratch->copies, n_parts, cw);
      return hipGetLastError();
    });
  }

  // Partitioned build. The count and scatter kernels use the same grid, so
  // each workgroup walks the same rows in both.
  uint64_t groups = (n_words + seg_words * 16 - 1) / (seg_words * 16);
  if (groups > scratch->hist_groups) groups = scratch->hist_groups;
  if (groups == 0) groups = 1;
  const uint32_t n_groups = static_cast<uint32_t>(groups);
  const uint32_t W = block_bits / 32;
  // Upper bound of the device's bucket count: kTargetBuckets plus one
  // partial tile per filter, or the 64 KB tiles of the largest filters.
  uint64_t max_buckets = kTargetBuckets + fs.n;
  {
    uint64_t big = 0;
    for (uint32_t i = 0; i < fs.n; i++)
      big += (fs.f[i].cap_words / W + kTileWords / W - 1) / (kTileWords / W);
    if (big > max_buckets) max_buckets = big;
  }
  if (max_buckets > kMaxBuckets) max_buckets = kMaxBuckets;
  const uint32_t scan_grid = static_cast<uint32_t>(max_buckets < 2048 ? max_buckets : 2048);
  uint64_t fill_grid = static_cast<uint64_t>(device_info().n_cu) * 2;
  if (fill_grid > max_buckets) fill_grid = max_buckets;
  return by_block_bits(block_bits, [&](auto bb) -> hipError_t {
    constexpr int B = decltype(bb)::value;
    auto count_k = k_part_count<B>;
    auto scatter_k = k == 3 ? k_part_scatter<B, 3> : k_part_scatter<B, 0>;
    auto fill_k = k == 3 ? k_part_fill<B, 3> : k_part_fill<B, 0>;
    const uint64_t hist_bytes = max_buckets * 4;
    const uint64_t cursor_bytes = max_buckets * 8;
    const uint64_t tile_bytes = static_cast<uint64_t>(kTileWords) * 4;
    hipError_t e = allow_lds(reinterpret_cast<const void *>(count_k), hist_bytes);
    if (e == hipSuccess) e = allow_lds(reinterpret_cast<const void *>(scatter_k), cursor_bytes);
    if (e == hipSuccess) e = allow_lds(reinterpret_cast<const void *>(fill_k), tile_bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(count_k, dim3(n_groups), dim3(kWideThreads), hist_bytes, s, fs, a, bits_per_key,
                       count, n_rows, bitmap, seg_words, entries_cap, scratch->hist);
    hipLaunchKernelGGL(k_part_scan_groups, dim3(scan_grid ? scan_grid : 1), dim3(kWideThreads), 0, s, fs,
                       block_bits, bits_per_key, count, n_rows, entries_cap, scratch->hist, n_groups,
                       scratch->totals);
    hipLaunchKernelGGL(k_part_scan_buckets, dim3(1), dim3(kWideThreads), 0, s, fs, block_bits,
                       bits_per_key, count, n_rows, entries_cap, scratch->totals, scratch->starts);
    hipLaunchKernelGGL(scatter_k, dim3(n_groups), dim3(kWideThreads), cursor_bytes, s, fs, a, k, bits_per_key,
                       count, n_rows, bitmap, seg_words, entries_cap, scratch->hist, scratch->starts,
                       scratch->entries);
    hipLaunchKernelGGL(fill_k, dim3(static_cast<uint32_t>(fill_grid ? fill_grid : 1)), dim3(kWideThreads),
                       tile_bytes, s, fs, k, bits_per_key, count, n_rows, entries_cap, scratch->starts,
                       scratch->entries);
    return hipGetLastError();
  });
}

hipError_t launch_copy_counts(const uint64_t *src, const uint32_t *slot, uint32_t n, uint64_t *dst,
                              hipStream_t s) {
  if (n == 0) return hipSuccess;
  SlotTable t{};
  for (uint32_t i = 0; i < n && i < 64; i++) t.slot[i] = slot[i];
  hipLaunchKernelGGL(k_copy_counts, dim3(1), dim3(64), 0, s, src, t, n, dst);
  return hipGetLastError();
}

uint64_t compact_partials(uint64_t n_rows) {
  const uint64_t n_words = (n_rows + 63) / 64;
  return (n_words + kCompactWordsPerBlock - 1) / kCompactWordsPerBlock;
}

hipError_t launch_compact(const uint64_t *bitmap, uint64_t n_rows, uint32_t *idx, uint64_t *count,
                          uint64_t *partials, hipStream_t s) {
  const uint64_t n_words = (n_rows + 63) / 64;
  const uint64_t n_parts = compact_partials(n_rows);
  if (n_parts == 0) {
    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, s, count, 1);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_compact_count, dim3(static_cast<uint32_t>(n_parts)), dim3(kThreads), 0, s,
                     bitmap, n_words, n_rows, partials);
  hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(1024), 0, s, partials, n_parts, count);
  hipLaunchKernelGGL(k_compact_write, dim3(static_cast<uint32_t>(n_parts)), dim3(kThreads), 0, s,
                     bitmap, n_words, n_rows, partials, idx);
  return hipGetLastError();
}

// ------------------------------------------------------- batched launches

hipError_t launch_local_batch(const LocalTask *tasks, const uint32_t *first, uint32_t n, uint32_t grid,
                              hipStream_t s) {
  if (n == 0 || grid == 0) return hipSuccess;
  hipLaunchKernelGGL(k_local_batch, dim3(grid), dim3(kBatchThreads), 0, s, tasks, first, n);
  return hipGetLastError();
}

hipError_t launch_size_batch(const SizeTask *tasks, const uint32_t *first, uint32_t n, uint32_t grid,
                             hipStream_t s) {
  if (n == 0 || grid == 0) return hipSuccess;
  hipLaunchKernelGGL(k_size_batch, dim3(grid), dim3(kBatchThreads), 0, s, tasks, first, n);
  return hipGetLastError();
}

hipError_t launch_build_batch(uint32_t block_bits, uint32_t k, const BuildTask *tasks, const uint32_t *first,
                              uint32_t n, uint32_t grid, uint32_t lds_words, hipStream_t s) {
  if (n == 0 || grid == 0) return hipSuccess;
  return by_block_bits(block_bits, [&](auto bb) -> hipError_t {
    constexpr int B = decltype(bb)::value;
    auto kern = k == 3 ? k_build_batch<B, 3> : k_build_batch<B, 0>;
    hipError_t e = allow_lds(reinterpret_cast<const void *>(kern), static_cast<uint64_t>(lds_words) * 4);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBatchThreads), static_cast<uint64_t>(lds_words) * 4, s, tasks,
                       first, n, k, lds_words);
    return hipGetLastError();
  });
}

uint64_t probe_queue_bytes(bool any64) {
  return static_cast<uint64_t>(kProbeWaves) * 4 *
         (any64 ? probe_slice_words<true>() : probe_slice_words<false>());
}

hipError_t launch_probe_batch(uint32_t block_bits, uint32_t k, bool any64, const ProbeTask *tasks,
                              const uint32_t *first, uint32_t n, uint32_t grid, uint32_t lds_filter_words,
                              hipStream_t s) {
  if (n == 0 || grid == 0) return hipSuccess;
  lds_filter_words &= ~1u;  // keep the slices 8-byte aligned
  const uint64_t lds_bytes = static_cast<uint64_t>(lds_filter_words) * 4 + probe_queue_bytes(any64);
  return by_block_bits(block_bits, [&](auto bb) -> hipError_t {
    constexpr int B = decltype(bb)::value;
    auto launch = [&](auto kern) -> hipError_t {
      hipError_t e = allow_lds(reinterpret_cast<const void *>(kern), lds_bytes);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(kern, dim3(grid), dim3(kProbeThreads), lds_bytes, s, tasks, first, n, k,
                         lds_filter_words);
      return hipGetLastError();
    };
    if (k == 3) return any64 ? launch(k_probe_batch<B, 3, true>) : launch(k_probe_batch<B, 3, false>);
    return any64 ? launch(k_probe_batch<B, 0, true>) : launch(k_probe_batch<B, 0, false>);
  });
}

hipError_t prepare_batch_kernels(uint32_t block_bits, uint32_t k, bool any64) {
  const uint64_t lds_max = static_cast<uint64_t>(device_info().max_lds_block) - 1024;
  return by_block_bits(block_bits, [&](auto bb) -> hipError_t {
    constexpr int B = decltype(bb)::value;
    const void *kerns[] = {
        reinterpret_cast<const void *>(k == 3 ? k_build_batch<B, 3> : k_build_batch<B, 0>),
        reinterpret_cast<const void *>(
            k == 3 ? (any64 ? k_probe_batch<B, 3, true> : k_probe_batch<B, 3, false>)
                   : (any64 ? k_probe_batch<B, 0, true> : k_probe_batch<B, 0, false>))};
    for (const void *kern : kerns) {
      hipError_t e = allow_lds(kern, lds_max);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  });
}

hipError_t launch_copy_pairs(const CopyPair *pairs, uint32_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_pairs, dim3((n + 255) / 256), dim3(256), 0, s, pairs, n);
  return hipGetLastError();
}

}  // namespace pt
