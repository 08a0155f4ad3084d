// Batched column and row passes: one launch per schedule family runs a pass
// of every instance of a batch (templates; instantiated per precision in
// batch_fp64.hip and batch_split.hip).
#pragma once
#include <hip/hip_ext.h>

#include "periodic_body.h"

namespace tdse {
//
// Workgroup b takes tile tiles[b]: an instance, its first line and the line
// transform schedule (length N and elements per thread EPT, so TL = N/EPT
// threads per line and LPW = BATCH_THREADS/TL lines per workgroup); the
// instance's launch arguments come from args[instance].  Tiles of different
// instances and lengths share a launch; its LDS size is the largest of its
// schedules.

// (N, EPT) schedules compiled into the batched passes, in three families,
// one kernel each, so that no schedule sets the register budget of another:
// powers of two (and the length-1 column pass of a 1D instance), and
// 3 * 2^a lengths with 6 or with 12 elements per thread.
#define TDSE_BATCH_FAMILY0(X)                                                   \
  X(1, 1) X(64, 4) X(64, 8) X(128, 4) X(128, 8) X(256, 4) X(256, 8) X(512, 4)   \
  X(512, 8) X(1024, 4) X(1024, 8) X(2048, 8)
#define TDSE_BATCH_FAMILY1(X) X(192, 6) X(384, 6) X(768, 6) X(1536, 6)
#define TDSE_BATCH_FAMILY2(X) X(192, 12) X(384, 12) X(768, 12) X(1536, 12)
#define TDSE_BATCH_SCHEDULES(X) TDSE_BATCH_FAMILY0(X) TDSE_BATCH_FAMILY1(X) TDSE_BATCH_FAMILY2(X)

template <typename C, int F>
__global__ __launch_bounds__(BATCH_THREADS) void k_col_batch(const LineArgs* __restrict__ args,
                                                             const BatchTile* __restrict__ tiles) {
  HIP_DYNAMIC_SHARED(double2, tdse_batch_lds)
  C* lds = (C*)tdse_batch_lds;
  const BatchTile tl = tiles[blockIdx.x];
  const LineArgs& a = args[tl.inst];
#define X(n, e)                                                         \
  case n * 64 + e: {                                                    \
    constexpr int T = n / e, L = BATCH_THREADS / T;                     \
    col_body<C, n, L, T>(a, tl.line0, tl.blk, tl.nblk, lds);            \
    break;                                                              \
  }
  if constexpr (F == 0) {
    switch (tl.sched) { TDSE_BATCH_FAMILY0(X) default: break; }
  } else if constexpr (F == 1) {
    switch (tl.sched) { TDSE_BATCH_FAMILY1(X) default: break; }
  } else {
    switch (tl.sched) { TDSE_BATCH_FAMILY2(X) default: break; }
  }
#undef X
}

// PW: the row kernel of instances with no field component along their last
// axis (that axis' factors of E^(j) formed as powers of E^(1)'s)
template <typename C, int F, bool PW = false>
__global__ __launch_bounds__(BATCH_THREADS) void k_row_batch(const LineArgs* __restrict__ args,
                                                             const BatchTile* __restrict__ tiles) {
  HIP_DYNAMIC_SHARED(double2, tdse_batch_lds)
  C* lds = (C*)tdse_batch_lds;
  const BatchTile tl = tiles[blockIdx.x];
  const LineArgs& a = args[tl.inst];
#define X(n, e)                                                         \
  case n * 64 + e: {                                                    \
    constexpr int T = n / e, L = BATCH_THREADS / T;                     \
    row_body<C, n, L, T, PW>(a, tl.line0, lds);                         \
    break;                                                              \
  }
  if constexpr (F == 0) {
    switch (tl.sched) { TDSE_BATCH_FAMILY0(X) default: break; }
  } else if constexpr (F == 1) {
    switch (tl.sched) { TDSE_BATCH_FAMILY1(X) default: break; }
  } else {
    switch (tl.sched) { TDSE_BATCH_FAMILY2(X) default: break; }
  }
#undef X
}

template <typename C, int F, bool PW>
void launch_batch_f(bool col, const LineArgs* args, const BatchTile* tiles, int ntiles, size_t lds_bytes,
                    hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const dim3 grid(ntiles), block(BATCH_THREADS);
  if (e0) {
    if (col) hipExtLaunchKernelGGL((k_col_batch<C, F>), grid, block, lds_bytes, s, e0, e1, 0, args, tiles);
    else hipExtLaunchKernelGGL((k_row_batch<C, F, PW>), grid, block, lds_bytes, s, e0, e1, 0, args, tiles);
  } else {
    if (col) hipLaunchKernelGGL((k_col_batch<C, F>), grid, block, lds_bytes, s, args, tiles);
    else hipLaunchKernelGGL((k_row_batch<C, F, PW>), grid, block, lds_bytes, s, args, tiles);
  }
}

template <typename C>
hipError_t launch_batch(bool col, int family, const LineArgs* args, const BatchTile* tiles, int ntiles,
                        size_t lds_bytes, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (ntiles <= 0) return hipSuccess;
  // families 3..5: the row kernels of families 0..2 for instances whose last
  // axis carries no field (column passes never take them)
  if (col && family >= 3) return hipErrorInvalidValue;
  switch (family) {
    case 0: launch_batch_f<C, 0, false>(col, args, tiles, ntiles, lds_bytes, s, e0, e1); break;
    case 1: launch_batch_f<C, 1, false>(col, args, tiles, ntiles, lds_bytes, s, e0, e1); break;
    case 2: launch_batch_f<C, 2, false>(col, args, tiles, ntiles, lds_bytes, s, e0, e1); break;
    case 3: launch_batch_f<C, 0, true>(col, args, tiles, ntiles, lds_bytes, s, e0, e1); break;
    case 4: launch_batch_f<C, 1, true>(col, args, tiles, ntiles, lds_bytes, s, e0, e1); break;
    case 5: launch_batch_f<C, 2, true>(col, args, tiles, ntiles, lds_bytes, s, e0, e1); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace tdse
