// LDS-resident complex FFTs along one line, for gfx950 (64-wide wavefronts).
//
// A line of N complex values sits contiguously in LDS.  The transform is a
// self-sorting (Stockham) sequence of radix-R passes: pass p reads butterfly
// inputs j + r*N/R, twiddles them by W_{Ns R}^{r k} with k = j mod Ns, forms
// the R-point DFT in registers and writes it to (j/Ns)*Ns*R + k + r*Ns.
// Every pass is in place: all reads, one barrier, all writes, one barrier.
//
// Forward uses exp(-2 pi i jk/N), inverse exp(+2 pi i jk/N); neither scales.
// Twiddles come from a table tw[m] = exp(-2 pi i m / N), m < N, built on the
// host in extended precision; the inverse conjugates them.
#pragma once
#include <hip/hip_runtime.h>

namespace tdse {

template <typename R_>
struct cplx_t;

template <>
struct cplx_t<double> { using type = double2; };
template <>
struct cplx_t<float> { using type = float2; };

template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename C>
__device__ __forceinline__ C cmulc(C a, C b) {  // a * conj(b)
  return C{a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename C>
__device__ __forceinline__ C cadd(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C>
__device__ __forceinline__ C csub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename C>
__device__ __forceinline__ C rot90(C a) {
  return INV ? C{-a.y, a.x} : C{a.y, -a.x};
}

// ---------------------------------------------------------------- small DFTs

template <bool INV, typename C>
__device__ __forceinline__ void dft2(C* v) {
  C a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <bool INV, typename C>
__device__ __forceinline__ void dft3(C* v) {
  using T = decltype(v[0].x);
  const T c = T(-0.5);
  const T s = INV ? T(0.86602540378443864676) : T(-0.86602540378443864676);
  C a = v[0], b = v[1], d = v[2];
  C t1 = cadd(b, d);
  C t2 = csub(b, d);
  C m1 = C{a.x + c * t1.x, a.y + c * t1.y};
  // s * i * t2
  C m2 = C{-s * t2.y, s * t2.x};
  v[0] = cadd(a, t1);
  v[1] = cadd(m1, m2);
  v[2] = csub(m1, m2);
}

template <bool INV, typename C>
__device__ __forceinline__ void dft4(C* v) {
  C a0 = cadd(v[0], v[2]);
  C a1 = csub(v[0], v[2]);
  C b0 = cadd(v[1], v[3]);
  C b1 = rot90<INV>(csub(v[1], v[3]));
  v[0] = cadd(a0, b0);
  v[2] = csub(a0, b0);
  v[1] = cadd(a1, b1);
  v[3] = csub(a1, b1);
}

template <bool INV, typename C>
__device__ __forceinline__ void dft8(C* v) {
  using T = decltype(v[0].x);
  const T h = T(0.70710678118654752440);
  // stage 1: radix-2 between halves
  C a[8];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    a[r] = cadd(v[r], v[r + 4]);
    a[r + 4] = csub(v[r], v[r + 4]);
  }
  // twiddles W8^r on the odd half: 1, (1 -/+ i)/sqrt2, -/+i, (-1 -/+ i)/sqrt2
  {
    C t = a[5];
    a[5] = INV ? C{h * (t.x - t.y), h * (t.x + t.y)} : C{h * (t.x + t.y), h * (t.y - t.x)};
    a[6] = rot90<INV>(a[6]);
    t = a[7];
    a[7] = INV ? C{-h * (t.x + t.y), h * (t.x - t.y)} : C{h * (t.y - t.x), -h * (t.x + t.y)};
  }
  C e[4] = {a[0], a[1], a[2], a[3]};
  C o[4] = {a[4], a[5], a[6], a[7]};
  dft4<INV>(e);
  dft4<INV>(o);
  // outputs: even frequencies from e, odd from o
  v[0] = e[0]; v[2] = e[1]; v[4] = e[2]; v[6] = e[3];
  v[1] = o[0]; v[3] = o[1]; v[5] = o[2]; v[7] = o[3];
}

template <int R, bool INV, typename C>
__device__ __forceinline__ void dft_small(C* v) {
  if constexpr (R == 2) dft2<INV>(v);
  else if constexpr (R == 3) dft3<INV>(v);
  else if constexpr (R == 4) dft4<INV>(v);
  else if constexpr (R == 8) dft8<INV>(v);
}

// ---------------------------------------------------------------- radix plan

// next radix for a remaining length: 8 while possible, then 4, 2, 3
__host__ __device__ constexpr int next_radix(int rem) {
  return (rem % 8 == 0) ? 8 : (rem % 4 == 0 ? 4 : (rem % 2 == 0 ? 2 : (rem % 3 == 0 ? 3 : 1)));
}

// One Stockham pass over a line in LDS.  Tl threads share the line; thread t
// handles butterflies t, t + Tl, ...  All threads of the block must call it.
template <int N, int R, int Ns, bool INV, int Tl, typename C>
__device__ __forceinline__ void stockham_pass(C* line, int t, const C* __restrict__ tw) {
  constexpr int NB = N / R;
  constexpr int BPT = (NB + Tl - 1) / Tl;
  constexpr int TWS = N / (Ns * R);
  C v[BPT][R];
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = t + b * Tl;
    if (NB % Tl == 0 || j < NB) {
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = line[j + r * NB];
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int j = t + b * Tl;
    if (NB % Tl == 0 || j < NB) {
      const int k = (Ns == 1) ? 0 : (j % Ns);
      if constexpr (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          C w = tw[r * k * TWS];
          if (INV) w.y = -w.y;
          v[b][r] = cmul(v[b][r], w);
        }
      }
      dft_small<R, INV>(v[b]);
      const int base = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) line[base + r * Ns] = v[b][r];
    }
  }
  __syncthreads();
}

template <int N, int Ns, bool INV, int Tl, typename C>
__device__ __forceinline__ void fft_line_rec(C* line, int t, const C* __restrict__ tw) {
  if constexpr (Ns < N) {
    constexpr int R = next_radix(N / Ns);
    static_assert(R > 1, "line length must be 2^a 3^b");
    stockham_pass<N, R, Ns, INV, Tl>(line, t, tw);
    fft_line_rec<N, Ns * R, INV, Tl>(line, t, tw);
  }
}

// Full FFT of one LDS line of length N by Tl cooperating threads.
template <int N, bool INV, int Tl, typename C>
__device__ __forceinline__ void fft_line(C* line, int t, const C* __restrict__ tw) {
  if constexpr (N > 1) fft_line_rec<N, 1, INV, Tl>(line, t, tw);
}

}  // namespace tdse
