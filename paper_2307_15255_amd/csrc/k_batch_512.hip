// k_batch_512.hip - the persistent batch kernel for 512-bit blocks with
// k = 3 or k = 2 (the settings the autotuner picks from).
#include "batch_impl.hpp"

namespace pt {

hipError_t launch_batch_512_k3(const BatchArgs &a, uint32_t grid, uint64_t lds_bytes, hipStream_t s) {
  return launch_batch_kernel<512, 3>(a, grid, lds_bytes, s);
}

hipError_t launch_batch_512_k2(const BatchArgs &a, uint32_t grid, uint64_t lds_bytes, hipStream_t s) {
  return launch_batch_kernel<512, 2>(a, grid, lds_bytes, s);
}

hipError_t prepare_batch_512() {
  hipError_t e = prepare_batch_kernel<512, 3>();
  if (e != hipSuccess) return e;
  return prepare_batch_kernel<512, 2>();
}

}  // namespace pt
