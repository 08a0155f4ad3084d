// Persistent implicit Adams steps of a square 2D periodic FP64 problem,
// gfx950: one co-resident grid marches many steps of eq. (uadamsk) with the
// multistep state held on chip.
//
// The grid has one workgroup per LPW = 2 lines (N/2 workgroups, one per
// compute unit for N = 512).  Workgroup b owns rows 2b, 2b+1 of the mode
// array in the row phase and columns 2b, 2b+1 of the grid in the column
// phase.  Per step m (the same arithmetic as the two-pass path):
//   column phase: inverse FFT along axis 0 of the tile (w = F^-1 B_m on the
//     grid), u = w / (1 + i mu_0 dt V(t_m)), g = V u / (N^2), forward FFT;
//   row phase:    forward FFT along axis 1 (What_m), uhat_m = B_m - i mu_0 dt What_m,
//     B_{m+1} = E^(1)(uhat_m - i dt mu_1 What_m) - i dt sum_{j>=2} mu_j E^(j) What_{m+1-j},
//     What_m into the history ring, inverse FFT along axis 1 (the next tile);
// with a grid barrier after each phase.  The carried state B of a
// workgroup's rows stays in registers and its history ring in LDS for the
// whole launch, so per step only the N^2 tile crosses between workgroups
// (the two transposes of Section 2.2's 2D transform) and the potential is
// read; B and the ring touch memory only at the launch's start and end.
//
// Phase factor of Lemma 1: E^(j)(k1,k2) = T1_j(k1) T2_j(k2) with
// T_a,j(k) = exp(-i k^2 j dt + i k dphi_a,j); the row factor T1 is computed
// per step by 2 (n-1) threads of the workgroup with sincos, the column factor
// is a static table exp(-i k2^2 j dt) in registers times, when the field has
// a component along axis 1, a product of per-step increments
// exp(i k2 (phi_2(t_i) - phi_2(t_{i-1}))) kept as a shift register.
//
// The tile crosses workgroups (and XCDs, whose L2 caches are not coherent
// with each other) through device-scope accesses: every load and store of
// exchanged data is a 16-byte buffer access with device scope (sc1), served
// at the device's point of coherence, so the barrier needs no cache
// writeback or invalidation, only the completion of the workgroup's own
// accesses before its arrival.  Between the phases of a launch the tile is
// kept in a blocked layout: the 2 x 2 block of rows 2r, 2r+1 and columns
// 2c, 2c+1 is 64 contiguous bytes, blocks of a row pair in column order, so
// a row-phase workgroup reads and writes 16 KB contiguously and a
// column-phase workgroup moves whole 64-byte blocks.  The launch's first
// column phase reads the row-major tile of the two-pass path, and a launch
// that stops before T writes its last row phase in row-major order.
//
// The grid barrier counts arrivals per XCD (workgroups are dealt to the
// eight XCDs round-robin, and the count is correct for any placement) and
// the last arrival of each group bumps a grid counter that every workgroup
// polls: a few tens of atomics on each counter instead of one counter taking
// them all.  Its wait is bounded (a flag reports a timeout to the host, and
// a workgroup that timed out stops waiting), so every workgroup always runs
// to the end of the kernel.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "fft_lds.h"
#include "tdse_internal.h"

namespace tdse {

namespace {

__device__ __forceinline__ int smode(int idx, int N) { return idx < (N >> 1) ? idx : idx - N; }

__device__ __forceinline__ double2 mi2(double c, double2 z) { return double2{c * z.y, -c * z.x}; }

// device-scope 16-byte accesses of a buffer (cache policy sc1)
constexpr int SC1 = 16;
__device__ __forceinline__ double2 cload(__amdgpu_buffer_rsrc_t rs, int64_t i) {
  return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)(i * 16), 0, SC1));
}
__device__ __forceinline__ void cstore(__amdgpu_buffer_rsrc_t rs, int64_t i, double2 v) {
  using V4 = decltype(__builtin_amdgcn_raw_buffer_load_b128(rs, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(V4, v), rs, (int)(i * 16), 0, SC1);
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const double2* p, int N) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)p, 0, N * N * 16, 0x00020000);
}
// blocked exchange layout: element (k1, k2) of an N x N tile
__device__ __forceinline__ int64_t blk(int k1, int k2, int N) {
  return ((int64_t)(k1 >> 1) * (N >> 1) + (k2 >> 1)) * 4 + (k1 & 1) * 2 + (k2 & 1);
}

// Grid barrier: every access of this workgroup completes, then one arrival
// on this workgroup's XCD counter (bar[32 (1 + x)]); the last of the group
// arrives on the grid counter bar[0]; wait until all groups are in.
// `target`, `xt` and `late` are thread 0's own (the grid and group arrivals
// expected so far, and whether one of its waits already timed out).
__device__ __forceinline__ void grid_barrier(unsigned* bar, unsigned* flag, int limit, unsigned& target, unsigned& xt,
                                             bool& late) {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned x = blockIdx.x & 7, groups = gridDim.x < 8 ? gridDim.x : 8;
    xt += (gridDim.x - x + groups - 1) / groups;   // workgroups b < gridDim.x with b % 8 == x
    const unsigned old = __hip_atomic_fetch_add(bar + 32 * (1 + x), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old + 1 == xt) __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    target += groups;
    int it = 0;
    while (!late && __hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (++it > limit) {
        late = true;
        __hip_atomic_store(flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

}  // namespace

// PH2: the field has a component along axis 1 (the column factor carries increments)
template <int N, int TL, bool PH2>
__global__ __launch_bounds__(2 * TL) void k_persist2d(Persist2DArgs a) {
  constexpr int LPW = 2, NT = LPW * TL, EPT = N / TL, H = MAXH - 1;
  constexpr int PC = lds_line_len(N) + 1;
  HIP_DYNAMIC_SHARED(double2, p2_lds)
  double2* xch = p2_lds;                          // FFT exchange lines (LPW * PC)
  double2* twl = xch + LPW * PC;                  // twiddles [N]
  double2* t1s = twl + N;                         // row factors T1 [LPW][H]
  double2* ringL = t1s + LPW * H;                 // history of the workgroup's rows [nh][LPW][N]
  const int tid = threadIdx.x, b = blockIdx.x;
  const int nh = a.order - 1;
  const double* __restrict__ tab = a.tab;
  // both phases: line i of the workgroup (lanes alternate between the two
  // lines), element t + TL q of it; row phase: row LPW b + i, column phase:
  // column LPW b + i
  const int i = tid % LPW, t = tid / LPW;
  const int line = LPW * b + i;
  double2* lds_line = xch + i * PC;
  const __amdgpu_buffer_rsrc_t rtile = rsrc(a.tile, N), rx = rsrc(a.xbuf, N);

  for (int q = tid; q < N; q += NT) twl[q] = a.tw[q];
  // state of the workgroup's rows: B in registers, the ring in LDS
  double2 B[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) B[q] = a.B[(int64_t)line * N + t + TL * q];
  for (int s = 0; s < nh; ++s)
#pragma unroll
    for (int q = 0; q < EPT; ++q)
      ringL[(s * LPW + i) * N + t + TL * q] = a.ring[(int64_t)s * N * N + (int64_t)line * N + t + TL * q];
  // static column factors exp(-i k2^2 j dt)
  double2 S2[H][EPT];
#pragma unroll
  for (int j = 1; j <= H; ++j)
#pragma unroll
    for (int q = 0; q < EPT; ++q) S2[j - 1][q] = j <= nh ? a.S2[(j - 1) * N + t + TL * q] : double2{1.0, 0.0};
  double2 dh[PH2 ? H : 1][EPT];
  auto incr2 = [&](double dphi, int q) -> double2 {
    double s, c;
    sincos((double)smode(t + TL * q, N) * dphi, &s, &c);
    return double2{c, s};
  };
  auto dphi2_at = [&](int ii) -> double { return ii >= 1 ? tab[a.oD2 + ii - 1] : 0.0; };
  if constexpr (PH2) {
#pragma unroll
    for (int ii = 1; ii < H; ++ii)
#pragma unroll
      for (int q = 0; q < EPT; ++q) dh[ii][q] = (ii < nh) ? incr2(dphi2_at(a.m0 + 2 - ii), q) : double2{1.0, 0.0};
  }
  __syncthreads();

  unsigned target = 0, xt = 0;
  bool late = false;
  const double scale = a.scale;
  for (int m = a.m0 + 1; m <= a.m1; ++m) {
    const double* st = tab + (int64_t)a.ostep * (m - a.mbase);   // fV[8], dphi1[H]
    // ------------------------------------------------ column phase (column `line`)
    {
      double2 v[EPT];
      double vs[EPT];
      if (m == a.m0 + 1) {   // the row-major tile of the two-pass path
#pragma unroll
        for (int q = 0; q < EPT; ++q) v[q] = cload(rtile, (int64_t)(t + TL * q) * N + line);
      } else {
#pragma unroll
        for (int q = 0; q < EPT; ++q) v[q] = cload(rx, blk(t + TL * q, line, N));
      }
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        double s = 0.0;
        for (int r = 0; r < a.nV; ++r) s += st[r] * a.V[r * a.vstride + (int64_t)(t + TL * q) * N + line];
        vs[q] = s;
      }
      fft_regs<N, TL, true>(v, t, lds_line, twl);
      const bool out = a.write_u && m == a.m1;
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const double qq = a.c0 * vs[q];
        const double iv = 1.0 / (1.0 + qq * qq);
        const double2 u = double2{(v[q].x + qq * v[q].y) * iv, (v[q].y - qq * v[q].x) * iv};
        if (out) a.uout[(int64_t)(t + TL * q) * N + line] = u;
        const double s = vs[q] * scale;
        v[q] = double2{s * u.x, s * u.y};
      }
      if (m == a.nsteps) break;   // the last step ends with u(T)
      fft_regs<N, TL, false>(v, t, lds_line, twl);
#pragma unroll
      for (int q = 0; q < EPT; ++q) cstore(rx, blk(t + TL * q, line, N), v[q]);
    }
    grid_barrier(a.bar, a.flag, a.spin_limit, target, xt, late);
    // ------------------------------------------------ row phase (row `line`)
    {
      double2 v[EPT];
#pragma unroll
      for (int q = 0; q < EPT; ++q) v[q] = cload(rx, blk(line, t + TL * q, N));
      if (tid < LPW * nh) {   // row factors T1_j for the workgroup's two rows
        const int rr = tid / nh, j = tid % nh + 1;
        const double k = (double)smode(LPW * b + rr, N);
        double s, c;
        sincos(-(k * k) * (j * a.dt) + k * st[8 + j - 1], &s, &c);
        t1s[rr * H + j - 1] = double2{c, s};
      }
      fft_regs<N, TL, false>(v, t, lds_line, twl);   // its barriers publish t1s
      const int sw = m % nh;
      if constexpr (PH2) {
#pragma unroll
        for (int q = 0; q < EPT; ++q) dh[0][q] = incr2(dphi2_at(m + 1), q);
      }
      double2 T1[H];
#pragma unroll
      for (int j = 1; j <= H; ++j) T1[j - 1] = j <= nh ? t1s[i * H + j - 1] : double2{1.0, 0.0};
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const int k2 = t + TL * q;
        const double2 W = v[q];
        const double2 uh = cadd(B[q], mi2(a.c0, W));
        double2 D = PH2 ? dh[0][q] : double2{1.0, 0.0};
        double2 E1 = cmul(T1[0], S2[0][q]);
        if constexpr (PH2) E1 = cmul(E1, D);
        double2 acc = cmul(E1, cadd(uh, mi2(a.ch[1], W)));
        double2 hist = double2{0.0, 0.0};
#pragma unroll
        for (int j = 2; j <= H; ++j) {
          if (j <= nh) {
            double2 Ej = cmul(T1[j - 1], S2[j - 1][q]);
            if constexpr (PH2) {
              D = cmul(D, dh[j - 1][q]);
              Ej = cmul(Ej, D);
            }
            const int sr = ((m + 1 - j) % nh + nh) % nh;
            hist = cadd(hist, mi2(a.ch[j], cmul(Ej, ringL[(sr * LPW + i) * N + k2])));
          }
        }
        B[q] = cadd(acc, hist);
        ringL[(sw * LPW + i) * N + k2] = W;
        v[q] = B[q];
      }
      if constexpr (PH2) {
#pragma unroll
        for (int ii = H - 1; ii >= 1; --ii)
#pragma unroll
          for (int q = 0; q < EPT; ++q) dh[ii][q] = dh[ii - 1][q];
      }
      fft_regs<N, TL, true>(v, t, lds_line, twl);
      if (m == a.m1) {   // the launch ends before T: the row-major tile for the two-pass path
#pragma unroll
        for (int q = 0; q < EPT; ++q) a.tile[(int64_t)line * N + t + TL * q] = v[q];
      } else {
#pragma unroll
        for (int q = 0; q < EPT; ++q) cstore(rx, blk(line, t + TL * q, N), v[q]);
      }
    }
    if (m < a.m1) grid_barrier(a.bar, a.flag, a.spin_limit, target, xt, late);
  }
  // the state goes back to memory for the next launch (or the two-pass path)
  if (a.m1 < a.nsteps) {
    __syncthreads();
#pragma unroll
    for (int q = 0; q < EPT; ++q) a.B[(int64_t)line * N + t + TL * q] = B[q];
    for (int s = 0; s < nh; ++s)
#pragma unroll
      for (int q = 0; q < EPT; ++q)
        a.ring[(int64_t)s * N * N + (int64_t)line * N + t + TL * q] = ringL[(s * LPW + i) * N + t + TL * q];
  }
}

__global__ void k_persist2d_reset(unsigned* bar) {
  for (int q = threadIdx.x; q < P2_BAR_WORDS; q += blockDim.x) bar[q] = 0u;
}

#define TDSE_PERSIST2D_SIZES(X) X(32) X(64) X(128) X(256) X(512)

bool persist2d_supported(int N) {
  switch (N) {
#define X(n) case n:
    TDSE_PERSIST2D_SIZES(X)
#undef X
    return true;
    default:
      return false;
  }
}

size_t persist2d_lds_bytes(int N, int order) {
  return sizeof(double2) *
         (2 * (size_t)(lds_line_len(N) + 1) + N + 2 * (MAXH - 1) + (size_t)(order - 1) * 2 * N);
}

template <int N, bool PH2>
hipError_t persist2d_launch(const Persist2DArgs& a, hipStream_t s) {
  constexpr int TL = N / 4;
  Persist2DArgs arg = a;
  void* args[] = {&arg};
  const size_t lds = persist2d_lds_bytes(N, a.order);
  hipLaunchKernelGGL(k_persist2d_reset, dim3(1), dim3(64), 0, s, a.bar);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return hipLaunchCooperativeKernel(k_persist2d<N, TL, PH2>, dim3(N / 2), dim3(2 * TL), args, (unsigned)lds, s);
}

// Workgroups of the co-resident grid that fit the device at once (0 if the
// kernel cannot run), for the launch-time co-residency check.
int persist2d_capacity(int N, int order, bool ph2) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const size_t lds = persist2d_lds_bytes(N, order);
  hipError_t e = hipErrorInvalidValue;
  switch (N) {
#define X(n)                                                                                                 \
  case n:                                                                                                    \
    e = ph2 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persist2d<n, n / 4, true>, n / 2, lds)  \
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_persist2d<n, n / 4, false>, n / 2, lds); \
    break;
    TDSE_PERSIST2D_SIZES(X)
#undef X
    default:
      break;
  }
  return e == hipSuccess ? per * cus : 0;
}

hipError_t launch_persist2d(const Persist2DArgs& a, hipStream_t s) {
  const bool ph2 = a.ph2 != 0;
  switch (a.N) {
#define X(n) \
  case n:    \
    return ph2 ? persist2d_launch<n, true>(a, s) : persist2d_launch<n, false>(a, s);
    TDSE_PERSIST2D_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace tdse
