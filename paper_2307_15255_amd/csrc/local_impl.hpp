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
// coalesced store. Eight words are evaluated per step so their loads
// overlap.

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
        if (ps.and_into && j0 + t < n_j) keep[t] = keep[t] && ((uniform64(bitmap[w_base + j0 + t]) >> lane) & 1);
      }
      for (uint32_t i = 0; i < ps.n; i++) {
        const PredRef &p = ps.p[i];
#pragma unroll
        for (int t = 0; t < T; t++) {
          const int64_t v = static_cast<int64_t>(load_key(p.col, p.col64, r[t]));
          keep[t] = keep[t] && pred_holds(p.op, v, p.lo, p.hi);
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

}  // namespace pt
