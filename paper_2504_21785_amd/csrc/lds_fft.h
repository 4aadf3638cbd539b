// In-place complex DFT of rows held in LDS (Stockham autosort, radix 4 and
// one radix 2 when log2 n is odd), shared by the batched FFT and the
// separable Fourier finish.  Rows of length n = 2^lg are `rowstride` apart;
// all threads of the workgroup take part and synchronise.
#ifndef FGGC_LDS_FFT_H
#define FGGC_LDS_FFT_H

#include <hip/hip_runtime.h>

namespace fggc {

template <typename T> __device__ __forceinline__ T cmul(T a, T b) {
  return T{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> __device__ __forceinline__ T cadd(T a, T b) { return T{a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ T csub(T a, T b) { return T{a.x - b.x, a.y - b.y}; }

constexpr int kMaxBfly = 8;  // radix-4 butterflies per thread per pass

// Rows: nrows * 2^(lg-2) <= blockDim * MB is required (radix-4 passes), and
// nrows * 2^(lg-1) <= blockDim * MB when lg is odd (the radix-2 pass).
// tw[k] = exp(-2 pi i k / n); inverse = 1 conjugates the twiddles.
template <typename T, int MB = kMaxBfly>
__device__ __forceinline__ void lds_fft_rows(T *sm, int lg, int nrows, int rowstride, int inverse,
                                             const T *__restrict__ tw) {
  int lgNs = 0;
  int rem = lg;
  while (rem > 0) {
    const int lgR = rem >= 2 ? 2 : 1;
    const int lgstride = lg - lgR;
    const int stride = 1 << lgstride, Ns = 1 << lgNs;
    const int nb = nrows << lgstride;  // butterflies in this pass
    const int tshift = lg - lgNs - lgR;
    T v[MB][4];
#pragma unroll
    for (int c = 0; c < MB; ++c) {
      const int b = threadIdx.x + c * (int)blockDim.x;
      if (b >= nb) break;
      const int l = b >> lgstride, j = b & (stride - 1);
      const int k = j & (Ns - 1);
      const T *sp = sm + l * rowstride;
      const int tstep = k << tshift;
      if (lgR == 2) {
#pragma unroll
        for (int r = 0; r < 4; ++r) v[c][r] = sp[j + r * stride];
#pragma unroll
        for (int r = 1; r < 4; ++r) {
          T w = tw[r * tstep];
          if (inverse) w.y = -w.y;
          v[c][r] = cmul(v[c][r], w);
        }
        const T s0 = cadd(v[c][0], v[c][2]), d0 = csub(v[c][0], v[c][2]);
        const T s1 = cadd(v[c][1], v[c][3]), d1 = csub(v[c][1], v[c][3]);
        // forward: multiply d1 by -i; inverse: by +i
        const T jd1 = inverse ? T{-d1.y, d1.x} : T{d1.y, -d1.x};
        v[c][0] = cadd(s0, s1);
        v[c][2] = csub(s0, s1);
        v[c][1] = cadd(d0, jd1);
        v[c][3] = csub(d0, jd1);
      } else {
        v[c][0] = sp[j];
        v[c][1] = sp[j + stride];
        T w = tw[tstep];
        if (inverse) w.y = -w.y;
        v[c][1] = cmul(v[c][1], w);
        const T x0 = v[c][0], x1 = v[c][1];
        v[c][0] = cadd(x0, x1);
        v[c][1] = csub(x0, x1);
      }
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < MB; ++c) {
      const int b = threadIdx.x + c * (int)blockDim.x;
      if (b >= nb) break;
      const int l = b >> lgstride, j = b & (stride - 1);
      const int k = j & (Ns - 1);
      const int idxD = ((j >> lgNs) << (lgNs + lgR)) + k;
      T *dp = sm + l * rowstride;
      if (lgR == 2) {
#pragma unroll
        for (int r = 0; r < 4; ++r) dp[idxD + r * Ns] = v[c][r];
      } else {
        dp[idxD] = v[c][0];
        dp[idxD + Ns] = v[c][1];
      }
    }
    __syncthreads();
    lgNs += lgR;
    rem -= lgR;
  }
}

}  // namespace fggc
#endif
