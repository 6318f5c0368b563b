// k_probe_gen.hip - the Bloom probe for any block size and hash count (both
// read at run time), and the host side of every single-problem probe
// launch: LDS budget, grid and the geometry of the appended survivor keys.
#include "probe_impl.hpp"

namespace pt {

hipError_t launch_probe_generic(const ProbeLaunch &pl, hipStream_t s) { return launch_probe_kernel<0, 0>(pl, s); }

uint64_t probe_queue_bytes() { return static_cast<uint64_t>(kProbeWaves) * 4 * probe_slice_words(); }

// Tables of fewer 1024-row groups than this run four waves per workgroup:
// the same waves then spread over four times as many CUs, whose memory
// pipelines serve their scattered filter reads side by side (a 10 k-row
// probe against a filter in global memory otherwise runs on one CU).
constexpr uint64_t kSmallProbeGroups = 1024;
constexpr uint32_t kSmallProbeThreads = 256;

hipError_t launch_probe(uint32_t block_bits, uint32_t k, const FilterSet &fs, uint64_t n_rows, uint64_t *bitmap,
                        uint64_t *count, bool input_all, AppendSet *app, uint64_t capacity, const ProbeOpts &opt,
                        uint32_t *status, hipStream_t s) {
  const uint64_t n_words = (n_rows + 63) / 64;
  if (n_words == 0 || fs.n == 0) {
    if (app) app->n_cols = 0;
    return hipSuccess;
  }
  const uint32_t lg = log2_of(static_cast<int>(block_bits));
  if (lg == 0) return hipErrorInvalidValue;
  uint64_t want_words = 0;
  for (uint32_t i = 0; i < fs.n; i++) want_words += fs.f[i].cap_words;
  const DeviceInfo &di = device_info();
  const int U = kGroupWords;
  const uint64_t groups = (n_words + U - 1) / U;
  const uint32_t threads = groups < kSmallProbeGroups ? kSmallProbeThreads : kProbeThreads;
  const uint64_t queue_bytes = static_cast<uint64_t>(threads / kWave) * 4 * probe_slice_words();
  // Leave room for the kernel's own static LDS (a few dozen bytes).
  const uint64_t lds_max = static_cast<uint64_t>(di.max_lds_block) - 1024;
  uint64_t filter_bytes = lds_max > queue_bytes ? lds_max - queue_bytes : 0;
  if (opt.lds_budget && filter_bytes > opt.lds_budget) filter_bytes = opt.lds_budget;
  if (filter_bytes > want_words * 4) filter_bytes = want_words * 4;
  filter_bytes &= ~uint64_t(7);  // keep the slices 8-byte aligned
  const uint64_t lds_bytes = filter_bytes + queue_bytes;
  const uint32_t per_cu = lds_bytes * 2 <= lds_max ? 2 : 1;
  ProbeLaunch pl{};
  pl.threads = threads;
  pl.grid = grid_for(groups, threads, threads == kProbeThreads ? per_cu : per_cu * (kProbeThreads / threads));
  pl.lds_filter_words = static_cast<uint32_t>(filter_bytes / 4);
  pl.lds_bytes = lds_bytes;
  pl.fs = fs;
  pl.k = k;
  pl.lg = lg;
  pl.n_rows = n_rows;
  pl.bitmap = bitmap;
  pl.count = reinterpret_cast<unsigned long long *>(count);
  pl.input_all = input_all ? 1u : 0u;
  pl.keep_order = opt.keep_order ? 1u : 0u;
  pl.status = status;
  // Region geometry of the appended keys: one region per wave of the grid,
  // capacity / regions slots each (at most the rows a wave can see).
  if (app && app->n_cols > 0 && app->n_cols <= static_cast<uint32_t>(kMaxAppend) && app->counts) {
    const uint64_t regions = static_cast<uint64_t>(pl.grid) * (threads / kWave);
    const uint64_t most = (groups + regions - 1) / regions * U * 64;
    uint64_t cap = capacity / regions;
    if (cap > most) cap = most;
    if (regions <= kMaxRegions && cap >= 64) {
      pl.app = *app;
      pl.app.n_regions = static_cast<uint32_t>(regions);
      pl.app.region_cap = static_cast<uint32_t>(cap);
      pl.app.group_words = static_cast<uint32_t>(U);
    }
  }
  if (app) *app = pl.app;
  if (block_bits == 512 && k == 3) return launch_probe_512_k3(pl, s);
  return launch_probe_generic(pl, s);
}

}  // namespace pt
