// k_probe_batch.hip - many probes in one launch: every workgroup finds its
// task (one table of one problem) and runs the probe body on the task's
// share of the grid.
#include "probe_impl.hpp"

namespace pt {

namespace {

template <int B, int K>
__global__ void __launch_bounds__(kProbeThreads)
    k_probe_batch(const ProbeTask *__restrict__ tasks, const uint32_t *__restrict__ first, uint32_t n_tasks,
                  uint32_t k, uint32_t lg, uint32_t lds_filter_words, uint32_t *status) {
  VGrid vg;
  const uint32_t t = task_of(first, n_tasks, vg);
  const ProbeTask &task = tasks[t];
  const AppendSet none{};
  probe_body<B, K, false>(task.fs, k, lg, task.n_rows, task.bitmap, reinterpret_cast<unsigned long long *>(task.count),
                          lds_filter_words, task.input_all, 0, status, none, vg);
}

const void *probe_batch_kernel(uint32_t block_bits, uint32_t k) {
  if (block_bits == 512 && k == 3) return reinterpret_cast<const void *>(k_probe_batch<512, 3>);
  return reinterpret_cast<const void *>(k_probe_batch<0, 0>);
}

}  // namespace

hipError_t prepare_probe_batch_kernel(uint32_t block_bits, uint32_t k) {
  const uint64_t lds_max = static_cast<uint64_t>(device_info().max_lds_block) - 1024;
  return allow_lds(probe_batch_kernel(block_bits, k), lds_max);
}

hipError_t launch_probe_batch(uint32_t block_bits, uint32_t k, const ProbeTask *tasks, const uint32_t *first,
                              uint32_t n, uint32_t grid, uint32_t lds_filter_words, uint32_t *status, hipStream_t s) {
  if (n == 0 || grid == 0) return hipSuccess;
  const uint32_t lg = log2_of(static_cast<int>(block_bits));
  if (lg == 0) return hipErrorInvalidValue;
  lds_filter_words &= ~1u;  // keep the slices 8-byte aligned
  const uint64_t lds_bytes = static_cast<uint64_t>(lds_filter_words) * 4 + probe_queue_bytes();
  const void *kern = probe_batch_kernel(block_bits, k);
  hipError_t e = allow_lds(kern, lds_bytes);
  if (e != hipSuccess) return e;
  if (block_bits == 512 && k == 3)
    hipLaunchKernelGGL((k_probe_batch<512, 3>), dim3(grid), dim3(kProbeThreads), lds_bytes, s, tasks, first, n, k, lg,
                       lds_filter_words, status);
  else
    hipLaunchKernelGGL((k_probe_batch<0, 0>), dim3(grid), dim3(kProbeThreads), lds_bytes, s, tasks, first, n, k, lg,
                       lds_filter_words, status);
  return hipGetLastError();
}

}  // namespace pt
