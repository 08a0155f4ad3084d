// Batched passes, FP64 transforms.
#include "batch_kernels.h"

namespace tdse {

hipError_t launch_batch_fp64(bool col, int family, const LineArgs* args, const BatchTile* tiles, int ntiles, size_t lds_bytes,
                             hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  return launch_batch<double2>(col, family, args, tiles, ntiles, lds_bytes, s, e0, e1);
}

}  // namespace tdse
