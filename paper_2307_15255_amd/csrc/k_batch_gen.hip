// k_batch_gen.hip - the persistent batch kernel for any block size and hash
// count (read per task at run time): batches whose problems mix settings.
#include "batch_impl.hpp"

namespace pt {

hipError_t launch_batch_generic(const BatchArgs &a, uint32_t grid, uint64_t lds_bytes, hipStream_t s) {
  return launch_batch_kernel<0, 0>(a, grid, lds_bytes, s);
}

hipError_t prepare_batch_kernels() {
  hipError_t e = prepare_batch_kernel<0, 0>();
  if (e != hipSuccess) return e;
  return prepare_batch_512();
}

}  // namespace pt
