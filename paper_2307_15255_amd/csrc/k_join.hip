// k_join.hip - the join phase (Sec. 3.3 of the paper): once the transfer
// phase has reduced the tables, the query's joins run on what is left. The
// join adds one table at a time to tuples of row ids: the added table's
// selected rows go into a hash table keyed on one edge to a table already
// joined, the tuples probe it with that table's key, and every match that
// also satisfies the other edges between the added table and the joined
// ones (a cycle's closing edge, the rest of a composite key) extends a
// tuple.
//
// A hash table is open addressing with linear probing over the 64-bit key
// values, the rows of one key chained through an array. It is sized on the
// device from the number of selected rows, so the small tables a selective
// transfer phase leaves behind stay in L2. Tuples are stored column by
// column; each wave reserves room for its new tuples with one atomic add,
// so the order of the tuples depends on scheduling and their set does not.
#include "pt_common.hpp"

namespace pt {

namespace {

constexpr uint64_t kNoSlot = ~0ull;

// log2 of the slots in use: twice the selected rows rounded up to a power
// of two, within [64, 2^lg_cap]; n receives the selected rows (clamped to
// the table's rows, which the capacity was sized for).
__device__ __forceinline__ uint32_t used_lg(const JoinHash &h, uint64_t &n) {
  n = *h.count;
  if (n > h.n_rows) n = h.n_rows;
  uint32_t lg = 6;
  while (lg < h.lg_cap && (1ull << lg) < 2 * n) lg++;
  return lg;
}

__device__ __forceinline__ uint64_t slot_of(unsigned long long key, uint32_t lg) {
  return static_cast<uint64_t>(key * kHashMul) >> (64 - lg);  // multiply-shift
}

__device__ __forceinline__ uint64_t thread_index() {
  return static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
}

__global__ void __launch_bounds__(kThreads) k_join_iota(uint32_t *ids, uint64_t n, uint64_t *count) {
  for (uint64_t i = thread_index(); i < n; i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    ids[i] = static_cast<uint32_t>(i);
  if (thread_index() == 0) *count = n;
}

__global__ void __launch_bounds__(kThreads) k_join_clear(JoinHash h) {
  uint64_t n;
  const uint64_t used = 1ull << used_lg(h, n);
  for (uint64_t i = thread_index(); i < used; i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    h.keys[i] = kJoinEmptyKey;
    h.heads[i] = kJoinNone;
  }
  if (thread_index() == 0) h.heads[1ull << h.lg_cap] = kJoinNone;
}

// Inserts selected row i (entry i of ids): claims the key's slot with a
// compare-and-swap (or finds it claimed by an equal key), then pushes i on
// the slot's chain. The slots in use are at least twice the rows, so a
// free slot is always reached.
__global__ void __launch_bounds__(kThreads) k_join_insert(JoinHash h) {
  uint64_t n;
  const uint32_t lg = used_lg(h, n);
  const uint64_t mask = (1ull << lg) - 1;
  for (uint64_t i = thread_index(); i < n; i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const unsigned long long key = load_key(h.key, h.key64, h.ids[i]);
    uint64_t s = 1ull << h.lg_cap;  // the slot of kJoinEmptyKey itself
    if (key != kJoinEmptyKey) {
      s = slot_of(key, lg);
      while (true) {
        const unsigned long long prev = atomicCAS(&h.keys[s], kJoinEmptyKey, key);
        if (prev == kJoinEmptyKey || prev == key) break;
        s = (s + 1) & mask;
      }
    }
    h.next[i] = atomicExch(&h.heads[s], static_cast<uint32_t>(i));
  }
}

// Lane j of a wave takes tuple j, finds its key's chain and walks it; in
// every round each lane tests at most one candidate, and the wave stores
// the round's matches together.
__global__ void __launch_bounds__(kThreads) k_join_step(JoinStep st) {
  uint64_t n_sel;
  const uint32_t lg = used_lg(st.h, n_sel);
  const uint64_t mask = (1ull << lg) - 1;
  uint64_t n_in = *st.n_in;
  if (n_in > st.in_cap) n_in = st.in_cap;
  const uint32_t lane = lane_id();
  const uint64_t wave = thread_index() / kWave;
  const uint64_t n_waves = static_cast<uint64_t>(gridDim.x) * (blockDim.x / kWave);
  for (uint64_t base = wave * kWave; base < n_in; base += n_waves * kWave) {
    const uint64_t j = base + lane;
    uint32_t e = kJoinNone;
    if (j < n_in) {
      const unsigned long long key = load_key(st.u_key, st.u64, st.in[st.u_pos][j]);
      uint64_t s = 1ull << st.h.lg_cap;
      if (key != kJoinEmptyKey) {
        s = slot_of(key, lg);
        while (true) {
          const unsigned long long k2 = st.h.keys[s];
          if (k2 == key) break;
          if (k2 == kJoinEmptyKey) {
            s = kNoSlot;
            break;
          }
          s = (s + 1) & mask;
        }
      }
      if (s != kNoSlot) e = st.h.heads[s];
    }
    while (__ballot(e != kJoinNone)) {
      bool emit = false;
      uint32_t r = 0;
      if (e != kJoinNone) {
        r = st.h.ids[e];
        emit = true;
        for (uint32_t c = 0; c < st.n_checks; c++) {
          const JoinCheck &ck = st.checks[c];
          if (load_key(ck.v_col, ck.v64, r) != load_key(ck.p_col, ck.p64, st.in[ck.pos][j])) emit = false;
        }
        e = st.h.next[e];
      }
      const uint64_t m = __ballot(emit);
      if (m == 0) continue;
      const uint32_t n_new = static_cast<uint32_t>(__popcll(m));
      unsigned long long at = 0;
      if (lane == 0) at = atomicAdd(reinterpret_cast<unsigned long long *>(st.n_out), n_new);
      // every lane is active here: lane 0's reservation goes to all
      at = (static_cast<unsigned long long>(__builtin_amdgcn_readlane(static_cast<uint32_t>(at >> 32), 0)) << 32) |
           static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<uint32_t>(at), 0));
      const uint64_t pos =
          at + __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32), __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0));
      if (emit && pos < st.cap) {
        for (uint32_t c = 0; c < st.width; c++) st.out[c][pos] = st.in[c][j];
        st.out[st.width][pos] = r;
      }
      if (lane == 0 && at + n_new > st.cap) raise_status(st.status, PT_STATUS_JOIN_OVERFLOW);
    }
  }
}

__global__ void __launch_bounds__(kThreads)
    k_join_copy(const uint32_t *src, const uint64_t *n, uint64_t cap, uint32_t *dst, uint64_t *n_out,
                uint32_t *status) {
  const uint64_t total = *n;
  const uint64_t m = total < cap ? total : cap;
  for (uint64_t i = thread_index(); i < m; i += static_cast<uint64_t>(gridDim.x) * blockDim.x) dst[i] = src[i];
  if (thread_index() == 0) {
    *n_out = total;
    if (total > cap) raise_status(status, PT_STATUS_JOIN_OVERFLOW);
  }
}

// After the last step: when an intermediate step overflowed, the result
// count becomes the largest count any step reached (a capacity to retry
// with), since later steps saw only the kept tuples.
__global__ void k_join_finish(const uint64_t *step_counts, uint32_t n_steps, uint64_t cap, uint64_t *n_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  uint64_t m = *n_out;
  bool over = false;
  for (uint32_t i = 0; i < n_steps; i++) {
    over = over || step_counts[i] > cap;
    m = step_counts[i] > m ? step_counts[i] : m;
  }
  if (over) *n_out = m;
}

}  // namespace

hipError_t launch_join_finish(const uint64_t *step_counts, uint32_t n_steps, uint64_t cap, uint64_t *n_out,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_join_finish, dim3(1), dim3(64), 0, s, step_counts, n_steps, cap, n_out);
  return hipGetLastError();
}

hipError_t launch_join_ids(const uint64_t *bitmap, uint64_t n_rows, uint32_t *ids, uint64_t *count,
                           uint64_t *partials, hipStream_t s) {
  if (bitmap) return launch_compact(bitmap, n_rows, ids, count, partials, s);
  hipLaunchKernelGGL(k_join_iota, dim3(grid_for((n_rows + 63) / 64, kThreads, 8)), dim3(kThreads), 0, s, ids, n_rows,
                     count);
  return hipGetLastError();
}

hipError_t launch_join_build(const JoinHash &h, hipStream_t s) {
  const uint64_t cap = 1ull << h.lg_cap;
  hipLaunchKernelGGL(k_join_clear, dim3(grid_for(cap / 64, kThreads, 8)), dim3(kThreads), 0, s, h);
  hipLaunchKernelGGL(k_join_insert, dim3(grid_for((h.n_rows + 63) / 64, kThreads, 8)), dim3(kThreads), 0, s, h);
  return hipGetLastError();
}

hipError_t launch_join_step(const JoinStep &st, hipStream_t s) {
  hipLaunchKernelGGL(k_join_step, dim3(grid_for((st.in_cap + 63) / 64, kThreads, 8)), dim3(kThreads), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_join_copy(const uint32_t *src, const uint64_t *n, uint64_t cap, uint32_t *dst, uint64_t *n_out,
                            uint32_t *status, hipStream_t s) {
  hipLaunchKernelGGL(k_join_copy, dim3(grid_for((cap + 63) / 64, kThreads, 8)), dim3(kThreads), 0, s, src, n, cap, dst,
                     n_out, status);
  return hipGetLastError();
}

}  // namespace pt
