// local_impl.hpp - the local filter (Sec. 3.2 of the paper: inherent
// filters applied during the scan; Sec. 3.4: predicates on base tables) as a
// body over a (virtual) grid, shared by its own kernel and the batch kernel.
#pragma once

#include "pt_common.hpp"

namespace pt {

// ---------------------------------------------------------- local filter
//
// Each wave takes seg_words (1..64) consecutive words, builds word j with the
// ballot of step j, keeps it in lane j, and stores the segment with one
// coalesced store. T words are evaluated per step, their loads in flight
// together (8 keep 32 KB in flight per CU with one 1024-thread workgroup
// there, as in the batch kernel, whose registers do not allow 16).

__device__ __forceinline__ bool pred_holds(uint32_t op, int64_t v, int64_t lo, int64_t hi) {
  switch (op) {
    case PT_LT: return v < lo;
    case PT_LE: return v <= lo;
    case PT_GT: return v > lo;
    case PT_GE: return v >= lo;
    case PT_EQ: return v == lo;
    case PT_NE: return v != lo;
    default: return lo <= v && v <= hi;
  }
}

template <int T = 8>
__device__ __forceinline__ void local_body(const PredSet &ps, uint64_t n_rows, uint64_t *__restrict__ bitmap,
                                           unsigned long long *count, uint32_t seg_words, const VGrid &vg) {
  static_assert(T >= 1 && T <= 32, "the keep mask is one 32-bit word");
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
      // bit t of keep: row (w_base + j0 + t) * 64 + lane is still selected
      uint32_t keep = 0;
#pragma unroll
      for (int t = 0; t < T; t++) {
        const uint64_t row = (w_base + j0 + t) * 64 + lane;
        keep |= static_cast<uint32_t>(j0 + t < n_j && row < n_rows) << t;
      }
      if (ps.and_into) {
        uint64_t old[T];
#pragma unroll
        for (int t = 0; t < T; t++) old[t] = bitmap[w_base + min(j0 + t, n_j - 1)];
#pragma unroll
        for (int t = 0; t < T; t++) keep &= ~(static_cast<uint32_t>(((old[t] >> lane) & 1) == 0) << t);
      }
      for (uint32_t i = 0; i < ps.n; i++) {
        const PredRef &p = ps.p[i];
        // the width test stays outside the unrolled loads: inside, each
        // 4-byte load would be waited for before the next one is issued
        int64_t v[T];
        if (p.col64) {
#pragma unroll
          for (int t = 0; t < T; t++) {
            const uint64_t row = (w_base + j0 + t) * 64 + lane;
            v[t] = static_cast<const int64_t *>(p.col)[row < n_rows ? row : n_rows - 1];
          }
        } else {
#pragma unroll
          for (int t = 0; t < T; t++) {
            const uint64_t row = (w_base + j0 + t) * 64 + lane;
            v[t] = static_cast<const int32_t *>(p.col)[row < n_rows ? row : n_rows - 1];
          }
        }
#pragma unroll
        for (int t = 0; t < T; t++) keep &= ~(static_cast<uint32_t>(!pred_holds(p.op, v[t], p.lo, p.hi)) << t);
      }
#pragma unroll
      for (int t = 0; t < T; t++) {
        const uint64_t m = __ballot((keep >> t) & 1);
        if (lane == j0 + t) mine = m;
      }
    }
    if (lane < n_j) bitmap[w_base + lane] = mine;
    cnt += __popcll(mine);
  }
  block_count_add(static_cast<int64_t>(wave_sum(cnt)), &s_cnt, count);
}

}  // namespace pt
