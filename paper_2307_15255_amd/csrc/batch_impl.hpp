// batch_impl.hpp - the persistent kernel of a batch of transfer problems.
//
// Many independent transfer phases (Sec. 3.2 of the paper, one per
// problem) run in one launch. The host lists every step of every problem as
// a task (a local filter, a probe, a build, ...), split into work items of
// one workgroup each, and orders the list by phase: a task's depth in the
// dependency graph. The launch has one resident workgroup per CU; each
// takes the next item from a device counter and runs it on its task's share
// of a virtual grid (VGrid).
//
// Phases, not tasks, are synchronised: the L2 of each XCD is not coherent
// with the others for this memory, so making writes visible device-wide
// means writing back the whole L2 and invalidating the reader's L2. A
// workgroup does that once per phase change: when it takes an item of a
// later phase it waits for its own writes, writes back its XCD's L2 and adds
// the items it finished to the phase's counter (release); then thread 0
// waits until the previous phase's counter is full and invalidates (acquire).
// A workgroup that runs out of items publishes its count before it exits.
//
// Items are taken in list order, and a workgroup publishes everything it
// finished before it waits, so the last unfinished phase always completes:
// the queue drains. The wait is bounded anyway (a timeout is reported in the
// status word, after which nothing waits), so no launch can hang.
#pragma once

#include "local_impl.hpp"
#include "part_impl.hpp"
#include "probe_impl.hpp"

namespace pt {

__device__ __forceinline__ uint64_t load_shared_u64(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Thread 0: waits until every item of `phase` has finished, then acquires
// (invalidates the caches that may hold older data). Once one wait of the
// launch has timed out, no item waits any more, so a launch whose counts were
// wrong ends within about one time limit.
__device__ __forceinline__ void wait_for_phase(const BatchArgs &a, uint32_t phase) {
  const uint32_t need = a.phase_items[phase];
  uint32_t *done = a.phase_done + phase;
  if (__hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
      if (__hip_atomic_load(a.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & PT_STATUS_WAIT_TIMEOUT) break;
      __builtin_amdgcn_s_sleep(4);
      if (wall_clock64() - t0 > a.spin_limit) {
        atomicOr(a.status, PT_STATUS_WAIT_TIMEOUT);
        break;
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// All threads: this workgroup's writes so far become visible device-wide,
// then `items` finished items are added to `phase`'s counter.
__device__ __forceinline__ void publish(const BatchArgs &a, uint32_t phase, uint32_t items) {
  __builtin_amdgcn_s_waitcnt(0);  // every wave: its stores have reached the L2
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // write the L2 back
    __hip_atomic_fetch_add(a.phase_done + phase, items, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// A partitioned build whose buckets would not fit the table the host laid
// out is skipped and reported (the bound the host uses makes this
// unreachable; the check keeps every access inside the scratch).
__device__ __forceinline__ bool part_fits(const BBuild &b, uint32_t lg, uint32_t *status) {
  const PartGeo geo = part_geo(b.fs, lg, b.bits_per_key, b.count, b.n_rows, b.entries_cap, true, kBatchTargetBuckets);
  if (geo.ok && geo.buckets > b.hist_cols) {
    if (threadIdx.x == 0) raise_status(status, PT_STATUS_FILTER_OVERFLOW);
    return false;
  }
  return true;
}

// Words of the filters of b, sized from the builder's count, and filter i's
// offset in their concatenation (s_off: kMaxFilters + 1 entries in LDS,
// written by thread 0).
__device__ __forceinline__ void filter_offsets(const BBuild &b, uint32_t lg, uint64_t n_sel, uint32_t *s_off) {
  if (threadIdx.x == 0) {
    uint32_t off = 0;
    for (uint32_t i = 0; i < b.fs.n; i++) {
      s_off[i] = off;
      off += part_blocks(b.fs.f[i], lg, b.bits_per_key, n_sel, true) << (lg - 5);
    }
    s_off[b.fs.n] = off;
  }
  __syncthreads();
}

// Private LDS copies of the filters of b for this item's rows, stored to
// copy vg.block of the task's scratch.
template <int K>
__device__ __forceinline__ void build_copy_body(const BBuild &b, uint32_t lg, uint32_t *lds, uint32_t *s_off,
                                                uint32_t *status, const VGrid &vg) {
  const uint64_t n_sel = load_shared_u64(b.count);
  filter_offsets(b, lg, n_sel, s_off);
  const uint32_t total = s_off[b.fs.n];
  // The host sizes the copies for every filter at its capacity, so this
  // only guards the LDS and the scratch against a count above the table.
  if (total > b.copy_words) {
    if (threadIdx.x == 0) raise_status(status, PT_STATUS_FILTER_OVERFLOW);
    return;
  }
  for (uint32_t j = threadIdx.x; j < total; j += blockDim.x) lds[j] = 0;
  __syncthreads();
  const AppendSet none{};
  for (uint32_t i = 0; i < b.fs.n; i++) {
    const FilterRef &f = b.fs.f[i];
    const uint32_t nb = part_blocks(f, lg, b.bits_per_key, n_sel, true);
    uint32_t *mine = lds + s_off[i];
    for_each_key<false>(f, none, b.n_rows, b.bitmap, b.seg_words, vg,
                        [&](uint32_t h1, uint32_t h2) { insert_lds<K>(mine, nb, b.k, h1, h2, lg); });
  }
  __syncthreads();
  uint32_t *out = b.copies + static_cast<uint64_t>(vg.block) * b.copy_words;
  for (uint32_t j = threadIdx.x; j < total; j += blockDim.x) out[j] = lds[j];
}

// Filter words [vg.block * kReduceWords, ...) of the concatenation = OR of
// the private copies; item 0 also records every filter's block count.
__device__ __forceinline__ void reduce_body(const BBuild &b, uint32_t lg, uint32_t *s_off, const VGrid &vg) {
  const uint64_t n_sel = load_shared_u64(b.count);
  filter_offsets(b, lg, n_sel, s_off);
  const uint32_t total = min(s_off[b.fs.n], b.copy_words);
  if (vg.block == 0 && threadIdx.x < b.fs.n)
    *b.fs.f[threadIdx.x].nb = part_blocks(b.fs.f[threadIdx.x], lg, b.bits_per_key, n_sel, true);
  const uint64_t w0 = static_cast<uint64_t>(vg.block) * kReduceWords;
  const uint64_t w1 = min(w0 + kReduceWords, static_cast<uint64_t>(total));
  for (uint64_t w = w0 + threadIdx.x; w < w1; w += blockDim.x) {
    uint32_t v = 0;
    for (uint32_t p = 0; p < b.n_parts; p++) v |= b.copies[static_cast<uint64_t>(p) * b.copy_words + w];
    uint32_t i = 0;
    while (i + 1 < b.fs.n && w >= s_off[i + 1]) i++;
    b.fs.f[i].words[w - s_off[i]] = v;
  }
}

// Zeroes the filters of b when its partitioned build will not fit its entry
// buffer (its scatter then inserts with global atomics).
__device__ __forceinline__ void zero_body(const BBuild &b, uint32_t lg, uint32_t *s_off, const VGrid &vg) {
  if (part_geo(b.fs, lg, b.bits_per_key, b.count, b.n_rows, b.entries_cap, true, kBatchTargetBuckets).ok) return;
  const uint64_t n_sel = load_shared_u64(b.count);
  filter_offsets(b, lg, n_sel, s_off);
  const uint64_t w0 = static_cast<uint64_t>(vg.block) * kZeroWords;
  const uint64_t w1 = min(w0 + kZeroWords, static_cast<uint64_t>(s_off[b.fs.n]));
  for (uint64_t w = w0 + threadIdx.x; w < w1; w += blockDim.x) {
    uint32_t i = 0;
    while (i + 1 < b.fs.n && w >= s_off[i + 1]) i++;
    b.fs.f[i].words[w - s_off[i]] = 0;
  }
}

// Entry ranges of a partitioned build: per bucket, an exclusive scan over
// the row tiles' counts (in place), the bucket totals, and their exclusive
// scan (starts, one past the last bucket holding the sum). One item.
__device__ __forceinline__ void scan_body(const BBuild &b, uint32_t lg, uint64_t *s) {
  const PartGeo geo = part_geo(b.fs, lg, b.bits_per_key, b.count, b.n_rows, b.entries_cap, true, kBatchTargetBuckets);
  if (!geo.ok) return;
  const uint32_t buckets = min(geo.buckets, b.hist_cols);
  for (uint32_t j = threadIdx.x; j < buckets; j += blockDim.x) {
    uint64_t run = 0;
    for (uint32_t r = 0; r < b.hist_rows; r++) {
      uint32_t *h = b.hist + static_cast<uint64_t>(r) * b.hist_cols + j;
      const uint32_t v = *h;
      *h = static_cast<uint32_t>(run);
      run += v;
    }
    b.totals[j] = run;
  }
  __syncthreads();
  uint64_t carry = 0;
  for (uint32_t base = 0; base < buckets; base += blockDim.x) {
    const uint32_t j = base + threadIdx.x;
    const uint64_t v = j < buckets ? b.totals[j] : 0;
    uint64_t total;
    const uint64_t ex = block_exclusive_scan(v, s, total);
    if (j < buckets) b.starts[j] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) b.starts[buckets] = carry;
}

// One item of a shared scan. The members whose filters fit in LDS together
// (taken in member order) are staged there and probed in one pass: each
// wave takes groups of four bitmap words (256 rows), loads and hashes the
// rows' keys of every column once, and tests each of those members' filters
// on them (most selective first, only rows still alive). The other members
// are then probed one after the other.
// Bitmap words per wave and group in the batch's probes: fewer than the
// single probe's, so the whole persistent kernel fits its registers.
constexpr int kBatchProbeWords = 8;

static_assert(kMaxSharedMembers * 4 <= kWave, "a shared scan loads every member's bitmap words in one wave load");

template <int B, int K>
__device__ __forceinline__ void shared_probe_body(const BatchArgs &a, const BShared &sh, uint32_t *lds,
                                                  const VGrid &vg) {
  constexpr int U = 4;
  __shared__ uint32_t s_off[kMaxSharedMembers][kMaxProbe];
  __shared__ uint32_t s_nb[kMaxSharedMembers][kMaxProbe];
  __shared__ uint32_t s_ord[kMaxSharedMembers][kMaxProbe];  // member m's j-th filter to test
  __shared__ unsigned long long s_cnt[kMaxSharedMembers];
  const uint32_t n_m = sh.n_members;
  const BProbe *mem = a.probes + sh.first_probe;
  const uint32_t lg = block_log2<B>(mem[0].lg);
  const uint32_t W = 1u << (lg - 5);
  if (threadIdx.x < n_m) {
    // Member m's filters, most selective first (builder rows kept / rows,
    // as in the single probe; the order changes no bit), then staged in
    // that order by thread 0 below.
    const uint32_t m = threadIdx.x;
    const FilterSet &fs = mem[m].fs;
    uint64_t sel[kMaxProbe], rows[kMaxProbe];
    for (uint32_t j = 0; j < fs.n; j++) {
      s_ord[m][j] = j;
      sel[j] = (fs.f[j].sel && fs.f[j].rows) ? *fs.f[j].sel : 1;
      rows[j] = (fs.f[j].sel && fs.f[j].rows) ? fs.f[j].rows : 1;
    }
    for (uint32_t x = 1; x < fs.n; x++) {
      for (uint32_t y = x; y > 0; y--) {
        const uint32_t p = s_ord[m][y - 1], q = s_ord[m][y];
        if (sel[q] * rows[p] < sel[p] * rows[q]) {
          s_ord[m][y - 1] = q;
          s_ord[m][y] = p;
        } else {
          break;
        }
      }
    }
    s_cnt[m] = 0;
  }
  __syncthreads();
  __shared__ uint32_t s_in;  // bit m: member m's filters are all staged (it joins the shared pass)
  if (threadIdx.x == 0) {
    uint32_t used = 0, in = 0;
    for (uint32_t m = 0; m < n_m; m++) {
      uint64_t need = 0;
      for (uint32_t j = 0; j < mem[m].fs.n; j++) {
        const FilterRef &f = mem[m].fs.f[j];
        s_nb[m][j] = clamp_blocks(*f.nb, f.cap_words / W, a.status);
        need += static_cast<uint64_t>(s_nb[m][j]) * W;
      }
      if (used + need > a.lds_filter_words) continue;
      for (uint32_t j = 0; j < mem[m].fs.n; j++) {
        s_off[m][j] = used;
        used += s_nb[m][j] * W;
      }
      in |= 1u << m;
    }
    s_in = in;
  }
  __syncthreads();
  const uint32_t in = __builtin_amdgcn_readfirstlane(s_in);
  for (uint32_t m = 0; m < n_m; m++) {
    if (!((in >> m) & 1)) continue;
    for (uint32_t j = 0; j < mem[m].fs.n; j++) {
      const uint32_t off = s_off[m][j];
      const uint32_t n = s_nb[m][j] * W;
      const uint32_t *src = mem[m].fs.f[j].words;
      for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) lds[off + i] = src[i];
    }
  }
  __syncthreads();

  const uint32_t lane = lane_id();
  const uint64_t n_rows = sh.n_rows;
  const uint64_t n_words = (n_rows + 63) / 64;
  const uint32_t n_cols = sh.n_cols;
  for (uint64_t w0 = global_wave(vg) * U; in && w0 < n_words; w0 += wave_count(vg) * U) {
    // every column's keys of the group, loaded and hashed once
    // (a column's U loads are issued before any is used: a use inside the
    // width branch would wait for each load in turn)
    uint32_t h1[kMaxSharedCols][U], h2[kMaxSharedCols][U];
#pragma unroll
    for (int c = 0; c < kMaxSharedCols; c++) {
      uint64_t x[U];
#pragma unroll
      for (int u = 0; u < U; u++) h1[c][u] = h2[c][u] = 0;
      if (c >= static_cast<int>(n_cols)) continue;
      const bool key64 = sh.key64[c];
      if (key64) {
#pragma unroll
        for (int u = 0; u < U; u++)
          x[u] = static_cast<const uint64_t *>(sh.cols[c])[min(w0 * 64 + u * 64 + lane, n_rows - 1)];
      } else {
#pragma unroll
        for (int u = 0; u < U; u++)
          x[u] = static_cast<const uint32_t *>(sh.cols[c])[min(w0 * 64 + u * 64 + lane, n_rows - 1)];
      }
#pragma unroll
      for (int u = 0; u < U; u++) {
        if (key64)
          hash_key(x[u], h1[c][u], h2[c][u]);
        else
          hash_key32(static_cast<uint32_t>(x[u]), h1[c][u], h2[c][u]);
      }
    }
    // every member's bitmap words of the group in one load: lane 4 m + u
    // holds member m's word w0 + u
    uint64_t all_bits = 0;
    {
      const uint32_t m = lane / U, u = lane % U;
      if (m < n_m && w0 + u < n_words) all_bits = mem[m].bitmap[w0 + u];
    }
    for (uint32_t m = 0; m < n_m; m++) {
      if (!((in >> m) & 1)) continue;
      const BProbe &p = mem[m];
      const uint32_t n_f = p.fs.n;
      uint64_t word[U];
#pragma unroll
      for (int u = 0; u < U; u++) {
        const uint32_t b_hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(all_bits >> 32), m * U + u);
        const uint32_t b_lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(all_bits), m * U + u);
        word[u] = tail_mask(w0 + u, n_words, n_rows) & ((static_cast<uint64_t>(b_hi) << 32) | b_lo);
      }
      // Filter by filter; the four words' filter reads are issued together
      // (they come from L2 or beyond when the filter is not in LDS).
      for (uint32_t jj = 0; jj < n_f; jj++) {
        if ((word[0] | word[1] | word[2] | word[3]) == 0) break;
        const uint32_t j = __builtin_amdgcn_readfirstlane(s_ord[m][jj]);
        const uint32_t c = sh.col_of[m][j];
        const uint32_t nb = __builtin_amdgcn_readfirstlane(s_nb[m][j]);
        const uint32_t off = __builtin_amdgcn_readfirstlane(s_off[m][j]);
        const uint32_t *words = lds + off;  // every filter is staged here
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; u++) {
          uint32_t x1 = h1[0][u], x2 = h2[0][u];
#pragma unroll
          for (int cc = 1; cc < kMaxSharedCols; cc++) {
            if (c == static_cast<uint32_t>(cc)) {
              x1 = h1[cc][u];
              x2 = h2[cc][u];
            }
          }
          // only rows still alive read the filter
          ok[u] = ((word[u] >> lane) & 1) &&
                  block_has<K>(words + (static_cast<uint64_t>(block_of(x1, nb)) << (lg - 5)), x2, p.k, lg);
        }
#pragma unroll
        for (int u = 0; u < U; u++) word[u] &= __ballot(ok[u]);
      }
      uint64_t mine = 0;
      uint32_t cnt = 0;
#pragma unroll
      for (int u = 0; u < U; u++) {
        mine = lane == static_cast<uint32_t>(u) ? word[u] : mine;
        cnt += static_cast<uint32_t>(__popcll(word[u]));
      }
      if (lane < U && w0 + lane < n_words) p.bitmap[w0 + lane] = mine;
      if (lane == 0 && cnt) atomicAdd(&s_cnt[m], static_cast<unsigned long long>(cnt));
    }
  }
  __syncthreads();
  if (threadIdx.x < n_m && ((in >> threadIdx.x) & 1) && mem[threadIdx.x].count && s_cnt[threadIdx.x])
    atomicAdd(reinterpret_cast<unsigned long long *>(mem[threadIdx.x].count), s_cnt[threadIdx.x]);
  // Members whose filters did not fit: their filter reads, not the key
  // reads, are the cost, so each is probed on the item's rows by the
  // single-problem probe (most selective filter first, survivors
  // compacted), which reads the keys again.
  const AppendSet none{};
  for (uint32_t m = 0; m < n_m; m++) {
    if ((in >> m) & 1) continue;
    __syncthreads();
    const BProbe &p = mem[m];
    probe_body<B, K, false, kBatchProbeWords>(p.fs, p.k, p.lg, p.n_rows, p.bitmap,
                                              reinterpret_cast<unsigned long long *>(p.count), a.lds_filter_words, 0,
                                              0, a.status, none, vg);
  }
}

// Transfer path pruning: the (non-empty) builder of b still holds every row, so none
// of its filters is built; the step that records the block counts (the
// reduction, or the fill of a partitioned build) records zero, which the
// probes of the receivers read as "no filter".
__device__ __forceinline__ bool build_item_pruned(const BBuild &b, uint32_t kind, const VGrid &vg) {
  if (!b.fs.prune || b.n_rows == 0 || load_shared_u64(b.count) != b.n_rows) return false;
  if ((kind == kBReduce || kind == kBFill) && vg.block == 0 && threadIdx.x < b.fs.n) *b.fs.f[threadIdx.x].nb = 0;
  return true;
}

template <int B, int K>
__device__ __forceinline__ void run_item(const BatchArgs &a, const BTask &task, const VGrid &vg, uint32_t *lds) {
  __shared__ uint32_t s_off[kMaxFilters + 1];
  switch (task.kind) {
    case kBBuild:
    case kBReduce:
    case kBZero:
    case kBCount:
    case kBScan:
    case kBScatter:
    case kBFill:
      if (build_item_pruned(a.builds[task.arg], task.kind, vg)) return;
      break;
    default:
      break;
  }
  switch (task.kind) {
    case kBLocal: {
      const BLocal &l = a.locals[task.arg];
      local_body(l.ps, l.n_rows, l.bitmap, reinterpret_cast<unsigned long long *>(l.count), l.seg_words, vg);
      break;
    }
    case kBProbe: {
      const BProbe &p = a.probes[task.arg];
      const AppendSet none{};
      probe_body<B, K, false, kBatchProbeWords>(p.fs, p.k, p.lg, p.n_rows, p.bitmap,
                                                reinterpret_cast<unsigned long long *>(p.count), a.lds_filter_words,
                                                0, 0, a.status, none, vg);
      break;
    }
    case kBBuild: {
      const BBuild &b = a.builds[task.arg];
      build_copy_body<K>(b, block_log2<B>(b.lg), lds, s_off, a.status, vg);
      break;
    }
    case kBReduce: {
      const BBuild &b = a.builds[task.arg];
      reduce_body(b, block_log2<B>(b.lg), s_off, vg);
      break;
    }
    case kBZero: {
      const BBuild &b = a.builds[task.arg];
      zero_body(b, block_log2<B>(b.lg), s_off, vg);
      break;
    }
    case kBCount: {
      const BBuild &b = a.builds[task.arg];
      if (!part_fits(b, block_log2<B>(b.lg), a.status)) break;
      const AppendSet none{};
      part_count_body<false>(b.fs, none, block_log2<B>(b.lg), b.bits_per_key, b.count, b.n_rows, b.bitmap,
                             b.seg_words, b.entries_cap, b.hist + static_cast<uint64_t>(vg.block) * b.hist_cols, true,
                             kBatchTargetBuckets, vg);
      break;
    }
    case kBScan: {
      const BBuild &b = a.builds[task.arg];
      if (!part_fits(b, block_log2<B>(b.lg), a.status)) break;
      scan_body(b, block_log2<B>(b.lg), reinterpret_cast<uint64_t *>(lds));
      break;
    }
    case kBScatter: {
      const BBuild &b = a.builds[task.arg];
      if (!part_fits(b, block_log2<B>(b.lg), a.status)) break;
      const AppendSet none{};
      part_scatter_body<false, K>(b.fs, none, b.k, block_log2<B>(b.lg), b.bits_per_key, b.count, b.n_rows, b.bitmap,
                                  b.seg_words, b.entries_cap, b.hist + static_cast<uint64_t>(vg.block) * b.hist_cols,
                                  b.starts, b.entries, a.status, true, kBatchTargetBuckets, vg, a.lds_bytes);
      break;
    }
    case kBFill: {
      const BBuild &b = a.builds[task.arg];
      if (!part_fits(b, block_log2<B>(b.lg), a.status)) break;
      const uint32_t lg = block_log2<B>(b.lg);
      if (vg.block == 0 && threadIdx.x < b.fs.n)
        *b.fs.f[threadIdx.x].nb =
            part_blocks(b.fs.f[threadIdx.x], lg, b.bits_per_key, load_shared_u64(b.count), true);
      part_fill_body<K>(b.fs, b.k, lg, b.bits_per_key, b.count, b.n_rows, b.entries_cap, b.starts, b.entries,
                        vg.block, vg.blocks, true, kBatchTargetBuckets);
      break;
    }
    case kBShared:
      shared_probe_body<B, K>(a, a.shared[task.arg], lds, vg);
      break;
    case kBCopy: {
      for (uint32_t i = threadIdx.x; i < task.n_arg; i += blockDim.x) {
        const CopyPair &c = a.pairs[task.arg + i];
        *c.dst = load_shared_u64(c.src);
      }
      break;
    }
    default:
      break;
  }
}

template <int B, int K>
__global__ void __launch_bounds__(kBatchThreads) k_batch(BatchArgs a) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ uint32_t s_item;
  uint32_t phase = 0xFFFFFFFFu;  // phase of the items finished since the last publish
  uint32_t finished = 0;
  for (;;) {
    __syncthreads();  // the previous item is done with LDS and s_item
    if (threadIdx.x == 0) s_item = atomicAdd(a.head, 1u);
    __syncthreads();
    const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);
    const bool end = item >= a.n_items;
    const uint32_t t = end ? 0 : __builtin_amdgcn_readfirstlane(a.item_task[item]);
    const BTask task = a.tasks[t];
    const uint32_t next = end ? a.n_phases : task.phase;
    if (next != phase) {
      if (finished) publish(a, phase, finished);
      finished = 0;
      phase = next;
      if (end) return;
      if (phase > 0 && threadIdx.x == 0) wait_for_phase(a, phase - 1);
      __syncthreads();
    }
    const uint64_t t_start = a.timeline ? wall_clock64() : 0;
    run_item<B, K>(a, task, VGrid{item - task.first_item, task.n_items}, lds);
    if (a.timeline) {
      __syncthreads();
      if (threadIdx.x == 0) {
        a.timeline[2ull * item] = t_start;
        a.timeline[2ull * item + 1] = wall_clock64();
      }
    }
    finished++;
  }
}

template <int B, int K>
hipError_t launch_batch_kernel(const BatchArgs &a, uint32_t grid, uint64_t lds_bytes, hipStream_t s) {
  hipError_t e = allow_lds(reinterpret_cast<const void *>(k_batch<B, K>), lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_batch<B, K>), dim3(grid), dim3(kBatchThreads), lds_bytes, s, a);
  return hipGetLastError();
}

template <int B, int K>
hipError_t prepare_batch_kernel() {
  return allow_lds(reinterpret_cast<const void *>(k_batch<B, K>),
                   static_cast<uint64_t>(device_info().max_lds_block) - 2048);  // as the launch (static LDS < 2 KB)
}

}  // namespace pt
