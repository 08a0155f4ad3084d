// Register-resident line FFTs with LDS exchanges, for gfx950 (64-wide waves).
//
// A line of N complex values is shared by TL threads; thread t keeps the EPT =
// N/TL elements t + TL*m (m < EPT) in registers.  The transform is a
// self-sorting (Stockham) sequence of radix-R passes, R dividing EPT: pass p
// takes butterfly j = t + b*TL (b < EPT/R) from registers (inputs j + r*N/R,
// i.e. v[b + r*EPT/R]), twiddles by W_{Ns R}^{r k} with k = j mod Ns, forms
// the R-point DFT and writes it to (j/Ns)*Ns*R + k + r*Ns.  Between passes
// the outputs go through LDS and come back in the t + TL*m layout; the last
// pass writes its outputs straight back to registers, again in that layout.
// A line therefore enters and leaves the transform in registers, in the same
// element layout, which is also the layout of the fused pointwise work.
//
// Forward uses exp(-2 pi i jk/N), inverse exp(+2 pi i jk/N); neither scales.
// Twiddles come from a table tw[m] = exp(-2 pi i m / N), m < N, built on the
// host in extended precision (or from two small tables of its entries,
// TwPair); the inverse conjugates them.
#pragma once
#include <hip/hip_runtime.h>

namespace tdse {

template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
  return C{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
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
  C m2 = C{-s * t2.y, s * t2.x};  // s * i * t2
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
  C a[8];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    a[r] = cadd(v[r], v[r + 4]);
    a[r + 4] = csub(v[r], v[r + 4]);
  }
  // W8^r on the difference half: 1, (1 -/+ i)/sqrt2, -/+ i, (-1 -/+ i)/sqrt2
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

// Largest radix in {8, 4, 2} dividing both the remaining length and EPT;
// 3 once the remaining length is odd.
__host__ __device__ constexpr int pick_radix(int rem, int ept) {
  return (rem % 8 == 0 && ept % 8 == 0) ? 8
       : (rem % 4 == 0 && ept % 4 == 0) ? 4
       : (rem % 2 == 0 && ept % 2 == 0) ? 2
       : (rem % 3 == 0 && ept % 3 == 0) ? 3 : 1;
}

__host__ __device__ constexpr bool plan_ok(int N, int ept) {
  int ns = 1;
  while (ns < N) {
    const int r = pick_radix(N / ns, ept);
    if (r == 1) return false;
    ns *= r;
  }
  return ns == N && N % ept == 0;
}

// LDS slot of line element p: one 16-byte pad after every 8 elements, so the
// radix-8 scatter (lane stride 8 elements) and the contiguous gather both
// spread over all banks.  A line needs lds_line_len(N) slots.
__host__ __device__ constexpr int lds_slot(int p) { return p + (p >> 3); }
__host__ __device__ constexpr int lds_line_len(int N) { return N + (N >> 3); }

// Twiddle W_{Ns R}^{e} = tw[e * N / (Ns R)], conjugated for the inverse.
template <bool INV, typename C>
__device__ __forceinline__ C twiddle(const C* tw, int idx) {
  C w = tw[idx];
  if (INV) w.y = -w.y;
  return w;
}

// Two-level twiddle source for long lines: tw[idx] = coarse[idx / F] *
// fine[idx % F] with F = 2^LF, both small tables (N/F + F entries, e.g. in
// LDS) holding entries of the full table; one extra rounding per twiddle.
template <typename C, int LF>
struct TwPair {
  const C* coarse;
  const C* fine;
};
template <bool INV, typename C, int LF>
__device__ __forceinline__ C twiddle(const TwPair<C, LF>& tw, int idx) {
  C w = cmul(tw.coarse[idx >> LF], tw.fine[idx & ((1 << LF) - 1)]);
  if (INV) w.y = -w.y;
  return w;
}

template <int N, int TL, int Ns, bool INV, typename C, typename TW>
__device__ __forceinline__ void fft_regs_rec(C* v, int t, C* line, const TW& tw) {
  constexpr int EPT = N / TL;
  constexpr int R = pick_radix(N / Ns, EPT);
  constexpr int B = EPT / R;   // butterflies per thread
  constexpr int TWS = N / (Ns * R);
  constexpr bool LAST = (Ns * R == N);
  C x[B][R];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = t + b * TL;
    const int k = (Ns == 1) ? 0 : (j % Ns);
#pragma unroll
    for (int r = 0; r < R; ++r) x[b][r] = v[b + r * B];
    if constexpr (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) x[b][r] = cmul(x[b][r], twiddle<INV>(tw, r * k * TWS));
    }
    dft_small<R, INV>(x[b]);
  }
  if constexpr (LAST) {
#pragma unroll
    for (int b = 0; b < B; ++b)
#pragma unroll
      for (int r = 0; r < R; ++r) v[b + r * B] = x[b][r];
  } else {
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = t + b * TL;
      const int k = (Ns == 1) ? 0 : (j % Ns);
      const int base = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) line[lds_slot(base + r * Ns)] = x[b][r];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < EPT; ++m) v[m] = line[lds_slot(t + TL * m)];
    __syncthreads();
    fft_regs_rec<N, TL, Ns * R, INV>(v, t, line, tw);
  }
}

// Two independent lines transformed together, each in its own direction
// (INVA, INVB) and LDS scratch: every exchange round writes both lines, waits
// at one barrier and reads both back, so two lines cost the barriers of one.
template <int N, int TL, int Ns, bool INVA, bool INVB, typename C, typename TW>
__device__ __forceinline__ void fft_regs_dual_rec(C* va, C* vb, int t, C* la, C* lb, const TW& tw) {
  constexpr int EPT = N / TL;
  constexpr int R = pick_radix(N / Ns, EPT);
  constexpr int B = EPT / R;
  constexpr int TWS = N / (Ns * R);
  constexpr bool LAST = (Ns * R == N);
  C xa[B][R], xb[B][R];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = t + b * TL;
    const int k = (Ns == 1) ? 0 : (j % Ns);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      xa[b][r] = va[b + r * B];
      xb[b][r] = vb[b + r * B];
    }
    if constexpr (Ns > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const C w = twiddle<false>(tw, r * k * TWS);
        const C wa = INVA ? C{w.x, -w.y} : w, wb = INVB ? C{w.x, -w.y} : w;
        xa[b][r] = cmul(xa[b][r], wa);
        xb[b][r] = cmul(xb[b][r], wb);
      }
    }
    dft_small<R, INVA>(xa[b]);
    dft_small<R, INVB>(xb[b]);
  }
  if constexpr (LAST) {
#pragma unroll
    for (int b = 0; b < B; ++b)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        va[b + r * B] = xa[b][r];
        vb[b + r * B] = xb[b][r];
      }
  } else {
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int j = t + b * TL;
      const int k = (Ns == 1) ? 0 : (j % Ns);
      const int base = (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        la[lds_slot(base + r * Ns)] = xa[b][r];
        lb[lds_slot(base + r * Ns)] = xb[b][r];
      }
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < EPT; ++m) {
      va[m] = la[lds_slot(t + TL * m)];
      vb[m] = lb[lds_slot(t + TL * m)];
    }
    __syncthreads();
    fft_regs_dual_rec<N, TL, Ns * R, INVA, INVB>(va, vb, t, la, lb, tw);
  }
}

template <int N, int TL, bool INVA, bool INVB, typename C, typename TW>
__device__ __forceinline__ void fft_regs_dual(C* va, C* vb, int t, C* la, C* lb, const TW& tw) {
  static_assert(plan_ok(N, N / TL), "line length must factor into radices dividing N/TL");
  if constexpr (N > 1) fft_regs_dual_rec<N, TL, 1, INVA, INVB>(va, vb, t, la, lb, tw);
}

// FFT of one line held as v[m] = x[t + TL*m]; `line` is lds_line_len(N)
// elements of LDS scratch for this line.  Every thread of the block must call it (barriers).
template <int N, int TL, bool INV, typename C, typename TW>
__device__ __forceinline__ void fft_regs(C* v, int t, C* line, const TW& tw) {
  static_assert(plan_ok(N, N / TL), "line length must factor into radices dividing N/TL");
  if constexpr (N > 1) fft_regs_rec<N, TL, 1, INV>(v, t, line, tw);
}

}  // namespace tdse
