// Batched passes, complex64 transforms (split precision); the schedule
// table and the launch dispatch of both precisions.
#include "batch_kernels.h"

namespace tdse {

hipError_t launch_batch_fp64(bool col, int family, const LineArgs* args, const BatchTile* tiles, int ntiles, size_t lds_bytes,
                             hipStream_t s, hipEvent_t e0, hipEvent_t e1);

bool batch_schedule_ok(int N, int ept) {
  switch (N * 64 + ept) {
#define X(n, e) case n * 64 + e:
    TDSE_BATCH_SCHEDULES(X)
#undef X
    return true;
    default:
      return false;
  }
}

size_t batch_lds_bytes(int prec, bool col, int N, int ept) {
  const size_t es = prec == P_SPLIT ? sizeof(float2) : sizeof(double2);
  switch (N * 64 + ept) {
#define X(n, e)                                                                                  \
  case n * 64 + e: {                                                                             \
    constexpr int L = BATCH_THREADS / (n / e);                                                   \
    return es * (size_t)(col ? col_lds<double2, n, L>::elems : row_lds<double2, n, L>::elems);   \
  }
    TDSE_BATCH_SCHEDULES(X)
#undef X
    default:
      return 0;
  }
}

int batch_family(int N, int ept) {
  switch (N * 64 + ept) {
#define X(n, e) case n * 64 + e:
    TDSE_BATCH_FAMILY0(X)
    return 0;
    TDSE_BATCH_FAMILY1(X)
    return 1;
    TDSE_BATCH_FAMILY2(X)
    return 2;
#undef X
    default:
      return -1;
  }
}

hipError_t launch_batch_pass(int prec, bool col, int family, const LineArgs* args, const BatchTile* tiles,
                             int ntiles, size_t lds_bytes, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (prec == P_SPLIT) return launch_batch<float2>(col, family, args, tiles, ntiles, lds_bytes, s, e0, e1);
  return launch_batch_fp64(col, family, args, tiles, ntiles, lds_bytes, s, e0, e1);
}

}  // namespace tdse
