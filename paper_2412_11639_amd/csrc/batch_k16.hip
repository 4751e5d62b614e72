// Batched-plan kernels with 16 tiles per prefetch group (every order, plane
// map and waves-per-SIMD variant); see batch_kernels.h.
#include "batch_kernels.h"

namespace spk {

hipError_t launch_batch_k16(const BatchLaunch &b, hipStream_t st) { return launch_kg<16>(b, st); }

}  // namespace spk
