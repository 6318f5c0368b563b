// k_probe_512.hip - the Bloom probe specialised for 512-bit blocks (one
// 64-byte line per key) and k = 3, the default filter of the transfer phase.
#include "probe_impl.hpp"

namespace pt {

hipError_t launch_probe_512_k3(const ProbeLaunch &pl, hipStream_t s) { return launch_probe_kernel<512, 3>(pl, s); }

}  // namespace pt
