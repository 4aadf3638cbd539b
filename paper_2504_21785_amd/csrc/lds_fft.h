// In-place complex DFT of rows held in LDS (Stockham autosort: radix-8 and
// radix-4 passes for FP32, radix 4 and one radix 2 when log2 n is odd for
// FP64), shared by the batched FFT and the separable Fourier finish.  Rows of
// length n = 2^lg are `rowstride` apart; all threads of the workgroup take part
// and synchronise.
#ifndef FGGC_LDS_FFT_H
#define FGGC_LDS_FFT_H

#include <hip/hip_runtime.h>

namespace fggc {

template <typename T> __device__ __forceinline__ T cmul(T a, T b) {
  return T{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __device__ __forceinline__ T cadd(T a, T b) { return T{a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ T csub(T a, T b) { return T{a.x - b.x, a.y - b.y}; }

constexpr int kMaxBfly = 8;  // radix-4 butterflies per thread per pass (radix 8: half)

// x * (-i) (forward) or x * (+i) (inverse)
template <typename T> __device__ __forceinline__ T rot_quarter(T x, int inverse) {
  return inverse ? T{-x.y, x.x} : T{x.y, -x.x};
}

// In-register 8-point DFT: radix-2 split into the DFT4s of the even and the
// odd samples, then X[k] = E[k] + w^k O[k], X[k + 4] = E[k] - w^k O[k] with
// w = exp(-+ 2 pi i / 8).
template <typename T> __device__ __forceinline__ void dft8(T *x, int inverse) {
  using R = decltype(T{}.x);
  constexpr R h = (R)0.70710678118654752440;  // 1/sqrt(2)
  const T a0 = cadd(x[0], x[4]), a1 = csub(x[0], x[4]);
  const T a2 = cadd(x[2], x[6]), a3 = rot_quarter(csub(x[2], x[6]), inverse);
  const T b0 = cadd(x[1], x[5]), b1 = csub(x[1], x[5]);
  const T b2 = cadd(x[3], x[7]), b3 = rot_quarter(csub(x[3], x[7]), inverse);
  const T e0 = cadd(a0, a2), e2 = csub(a0, a2), e1 = cadd(a1, a3), e3 = csub(a1, a3);
  T o0 = cadd(b0, b2), o2 = csub(b0, b2), o1 = cadd(b1, b3), o3 = csub(b1, b3);
  // w^1 = (1 -+ i)/sqrt(2), w^2 = -+ i, w^3 = (-1 -+ i)/sqrt(2)
  o1 = inverse ? T{(o1.x - o1.y) * h, (o1.x + o1.y) * h} : T{(o1.x + o1.y) * h, (o1.y - o1.x) * h};
  o2 = rot_quarter(o2, inverse);
  o3 = inverse ? T{(-o3.x - o3.y) * h, (o3.x - o3.y) * h} : T{(o3.y - o3.x) * h, (-o3.x - o3.y) * h};
  x[0] = cadd(e0, o0);
  x[4] = csub(e0, o0);
  x[1] = cadd(e1, o1);
  x[5] = csub(e1, o1);
  x[2] = cadd(e2, o2);
  x[6] = csub(e2, o2);
  x[3] = cadd(e3, o3);
  x[7] = csub(e3, o3);
}

// One Stockham pass of radix 2^LGR over all rows (CB butterflies per thread).
template <typename T, int LGR, int CB>
__device__ __forceinline__ void lds_fft_pass(T *sm, int lg, int lgNs, int nrows, int rowstride, int inverse,
                                             const T *__restrict__ tw) {
  constexpr int R = 1 << LGR;
  const int lgstride = lg - LGR;
  const int stride = 1 << lgstride, Ns = 1 << lgNs;
  const int nb = nrows << lgstride;  // butterflies in this pass
  const int tshift = lg - lgNs - LGR;
  T v[CB][R];
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    const int b = threadIdx.x + c * (int)blockDim.x;
    if (b >= nb) break;
    const int l = b >> lgstride, j = b & (stride - 1);
    const int k = j & (Ns - 1);
    const T *sp = sm + l * rowstride;
    const int tstep = k << tshift;
#pragma unroll
    for (int r = 0; r < R; ++r) v[c][r] = sp[j + r * stride];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      T w = tw[r * tstep];
      if (inverse) w.y = -w.y;
      v[c][r] = cmul(v[c][r], w);
    }
    if constexpr (LGR == 3) {
      dft8(v[c], inverse);
    } else if constexpr (LGR == 2) {
      const T s0 = cadd(v[c][0], v[c][2]), d0 = csub(v[c][0], v[c][2]);
      const T s1 = cadd(v[c][1], v[c][3]), d1 = csub(v[c][1], v[c][3]);
      const T jd1 = rot_quarter(d1, inverse);
      v[c][0] = cadd(s0, s1);
      v[c][2] = csub(s0, s1);
      v[c][1] = cadd(d0, jd1);
      v[c][3] = csub(d0, jd1);
    } else {
      const T x0 = v[c][0], x1 = v[c][1];
      v[c][0] = cadd(x0, x1);
      v[c][1] = csub(x0, x1);
    }
    // finish this butterfly before the next one's loads are issued: only the
    // results wait for the barrier, not every butterfly's inputs and twiddles
#pragma unroll
    for (int r = 0; r < R; ++r) asm volatile("" : "+v"(v[c][r].x), "+v"(v[c][r].y));
    asm volatile("" ::: "memory");
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    const int b = threadIdx.x + c * (int)blockDim.x;
    if (b >= nb) break;
    const int l = b >> lgstride, j = b & (stride - 1);
    const int k = j & (Ns - 1);
    const int idxD = ((j >> lgNs) << (lgNs + LGR)) + k;
    T *dp = sm + l * rowstride;
#pragma unroll
    for (int r = 0; r < R; ++r) dp[idxD + r * Ns] = v[c][r];
  }
  __syncthreads();
}

// Radix-8 passes while the remaining factors allow (lg = 3 a + 2 b, b <= 2),
// radix 4 for the rest, radix 2 only for n = 2; without R8 (FP64, whose
// registers the larger butterflies overflow) radix 4 and one radix-2 pass for
// an odd lg.  Rows: nrows * 2^(lg-2) <= blockDim * MB is required, and
// nrows * 2^(lg-1) <= blockDim * MB when a radix-2 pass is taken.
// tw[k] = exp(-2 pi i k / n); inverse = 1 conjugates the twiddles.
template <typename T, int MB = kMaxBfly, bool R8 = (sizeof(T) == 8)>
__device__ __forceinline__ void lds_fft_rows(T *sm, int lg, int nrows, int rowstride, int inverse,
                                             const T *__restrict__ tw) {
  static_assert(MB % 2 == 0, "radix-8 passes take MB / 2 butterflies per thread");
  int n8, n4, n2;
  if (R8 && lg >= 2) {
    n4 = lg % 3 == 0 ? 0 : (lg % 3 == 1 ? 2 : 1);
    n8 = (lg - 2 * n4) / 3;
    n2 = 0;
  } else {
    n8 = 0;
    n4 = lg / 2;
    n2 = lg % 2;
  }
  int lgNs = 0;
  if constexpr (R8)
    for (int i = 0; i < n8; ++i, lgNs += 3) lds_fft_pass<T, 3, MB / 2>(sm, lg, lgNs, nrows, rowstride, inverse, tw);
  for (int i = 0; i < n4; ++i, lgNs += 2) lds_fft_pass<T, 2, MB>(sm, lg, lgNs, nrows, rowstride, inverse, tw);
  if (n2) lds_fft_pass<T, 1, MB>(sm, lg, lgNs, nrows, rowstride, inverse, tw);
}

}  // namespace fggc
#endif
