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

// In-register forward DFTs of length 2, 4, 8 and 16 (natural order in and
// out): X[k] = sum_n x[n] exp(-2 pi i n k / R).
template <typename T> __device__ __forceinline__ void dft2f(T *x) {
  const T a = x[0], b = x[1];
  x[0] = cadd(a, b);
  x[1] = csub(a, b);
}

template <typename T> __device__ __forceinline__ void dft4f(T *x) {
  const T s0 = cadd(x[0], x[2]), d0 = csub(x[0], x[2]);
  const T s1 = cadd(x[1], x[3]), d1 = rot_quarter(csub(x[1], x[3]), 0);
  x[0] = cadd(s0, s1);
  x[2] = csub(s0, s1);
  x[1] = cadd(d0, d1);
  x[3] = csub(d0, d1);
}

// 16 = 4 x 4: DFT4 over n1 of x[n2 + 4 n1] for each n2, twiddle
// exp(-2 pi i n2 k1 / 16), DFT4 over n2: X[k1 + 4 k2].
template <typename T> __device__ __forceinline__ void dft16f(T *x) {
  using R = decltype(T{}.x);
  constexpr R c1 = (R)0.92387953251128675613;  // cos(pi/8)
  constexpr R s1 = (R)0.38268343236508977173;  // sin(pi/8)
  constexpr R h = (R)0.70710678118654752440;   // cos(pi/4)
  T y[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    T v[4] = {x[n2], x[n2 + 4], x[n2 + 8], x[n2 + 12]};
    dft4f(v);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) y[n2][k1] = v[k1];
  }
  // exp(-2 pi i m / 16) for m = n2 k1 in {1, 2, 3, 4, 6, 9}
  y[1][1] = cmul(y[1][1], T{c1, -s1});
  y[1][2] = cmul(y[1][2], T{h, -h});
  y[1][3] = cmul(y[1][3], T{s1, -c1});
  y[2][1] = cmul(y[2][1], T{h, -h});
  y[2][2] = rot_quarter(y[2][2], 0);
  y[2][3] = cmul(y[2][3], T{-h, -h});
  y[3][1] = cmul(y[3][1], T{s1, -c1});
  y[3][2] = cmul(y[3][2], T{-h, -h});
  y[3][3] = cmul(y[3][3], T{-c1, s1});
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    T v[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
    dft4f(v);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) x[k1 + 4 * k2] = v[k2];
  }
}

// 32 = 2 x 16: the DFT16s of the even and the odd samples, then
// X[k] = E[k] + w^k O[k], X[k + 16] = E[k] - w^k O[k], w = exp(-2 pi i / 32).
template <typename T> __device__ __forceinline__ void dft32f(T *x) {
  using R = decltype(T{}.x);
  // cos(pi k / 16), k = 0 .. 8 (sin(pi k / 16) = cos(pi (8 - k) / 16))
  constexpr R cs[9] = {(R)1.0,
                       (R)0.980785280403230449126182236134,
                       (R)0.923879532511286756128183189397,
                       (R)0.831469612302545237078788377618,
                       (R)0.707106781186547524400844362105,
                       (R)0.555570233019602224742830813949,
                       (R)0.38268343236508977172845998403,
                       (R)0.195090322016128267848284868477,
                       (R)0.0};
  T e[16], o[16];
#pragma unroll
  for (int n = 0; n < 16; ++n) {
    e[n] = x[2 * n];
    o[n] = x[2 * n + 1];
  }
  dft16f(e);
  dft16f(o);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    // w^k = cos(pi k / 16) - i sin(pi k / 16)
    const R c = k <= 8 ? cs[k] : -cs[16 - k], sn = k <= 8 ? cs[8 - k] : cs[k - 8];
    const T t = k == 0 ? o[0] : cmul(o[k], T{c, -sn});
    x[k] = cadd(e[k], t);
    x[k + 16] = csub(e[k], t);
  }
}

template <typename T, int R> __device__ __forceinline__ void dftf(T *x) {
  if constexpr (R == 2) dft2f(x);
  else if constexpr (R == 4) dft4f(x);
  else if constexpr (R == 8) dft8(x, 0);
  else if constexpr (R == 16) dft16f(x);
  else dft32f(x);
}

// Row stride (elements) for lds_fft2_rows on rows of N = 2^lg: the row
// length padded so that rows start a whole number of N2-element blocks
// apart in the LDS banks (N2 = 2^floor(lg/2)).
__host__ __device__ inline int fft2_row_stride(int lg) { return (1 << lg) + (1 << (lg / 2)); }

// Forward DFT of nrows rows of N = N1 N2 points in LDS (N1 = 2^ceil(lg/2),
// N2 = 2^floor(lg/2), 8 <= N <= 512), rows `rs` elements apart, in two
// passes with one unit of work per thread each:
//   A  unit (row, n2): DFT over n1 of x[n2 + N2 n1], times exp(-2 pi i n2 k1 / N),
//      stored at block k1, slot n2 ^ sigma(row, k1) (a swizzle that spreads
//      the next pass's reads over the LDS banks);
//   B  unit (row, k1): DFT over n2 of block k1 gives F[k1 + N1 k2], stored
//      in natural order.
// tw[m] = exp(-2 pi i m / N).  Requires nrows * N2 <= blockDim and
// nrows * N1 <= 2 blockDim; all threads take part and synchronise.  The
// caller passes the thread index (tid) and blockDim (bs): inside a loop it
// can pass them through a compiler fence, so that the passes' addresses are
// formed where they are used instead of being hoisted out of the loop and
// held in registers for its whole length.
template <typename T, int N1, int N2>
__device__ __forceinline__ void lds_fft2_pass(T *sm, int nrows, int rs, const T *__restrict__ tw, int tid,
                                              int bs) {
  constexpr int N = N1 * N2;
  auto sigma = [](int row, int k1) { return ((k1 >> 2) + 4 * row) & (N2 - 1); };
  // pass A
  T x[N1];
  const int ua = tid;
  const bool hasA = ua < nrows * N2;
  const int rowA = ua / N2, n2 = ua % N2;
  if (hasA) {
    const T *src = sm + rowA * rs + n2;
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) x[n1] = src[N2 * n1];
    dftf<T, N1>(x);
#pragma unroll
    for (int k1 = 1; k1 < N1; ++k1) x[k1] = cmul(x[k1], tw[n2 * k1]);
  }
  __syncthreads();
  if (hasA) {
    T *dst = sm + rowA * rs;
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) dst[N2 * k1 + (n2 ^ sigma(rowA, k1))] = x[k1];
  }
  __syncthreads();
  // pass B: up to two units per thread (nrows N1 <= 2 blockDim; one when
  // N1 = N2, as nrows N2 <= blockDim), held until the barrier
  constexpr int UB = N1 > N2 ? 2 : 1;
  T y[UB][N2];
#pragma unroll
  for (int u = 0; u < UB; ++u) {
    const int ub = tid + u * bs;
    if (ub >= nrows * N1) break;
    const int row = ub / N1, k1 = ub % N1;
    const T *src = sm + row * rs + N2 * k1;
    const int sg = sigma(row, k1);
#pragma unroll
    for (int m = 0; m < N2; ++m) y[u][m] = src[m ^ sg];
    dftf<T, N2>(y[u]);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < UB; ++u) {
    const int ub = tid + u * bs;
    if (ub >= nrows * N1) break;
    const int row = ub / N1, k1 = ub % N1;
    T *dst = sm + row * rs + k1;
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) dst[N1 * k2] = y[u][k2];
  }
  __syncthreads();
  (void)N;
}

// MAXLG: the longest rows the caller takes (8: 256 points, 9: 512); the
// 512-point case holds 32 points per thread in its first pass, so kernels
// that never see it are built without it and keep their registers.
template <typename T, int MAXLG = 8>
__device__ __forceinline__ void lds_fft2_rows(T *sm, int lg, int nrows, int rs, const T *__restrict__ tw, int tid,
                                              int bs) {
  if constexpr (MAXLG >= 9) {
    if (lg == 9) {
      lds_fft2_pass<T, 32, 16>(sm, nrows, rs, tw, tid, bs);
      return;
    }
  }
  switch (lg) {
    case 3: lds_fft2_pass<T, 4, 2>(sm, nrows, rs, tw, tid, bs); break;
    case 4: lds_fft2_pass<T, 4, 4>(sm, nrows, rs, tw, tid, bs); break;
    case 5: lds_fft2_pass<T, 8, 4>(sm, nrows, rs, tw, tid, bs); break;
    case 6: lds_fft2_pass<T, 8, 8>(sm, nrows, rs, tw, tid, bs); break;
    case 7: lds_fft2_pass<T, 16, 8>(sm, nrows, rs, tw, tid, bs); break;
    default: lds_fft2_pass<T, 16, 16>(sm, nrows, rs, tw, tid, bs); break;
  }
}

// ---- lengths 2^a 3^b 5^c ------------------------------------------------
// Mixed-radix Stockham passes over rows of any length n = 2^a 3^b 5^c held in
// LDS: radix-4 passes, one radix-2 pass when a is odd, then radix 3 and radix
// 5.  A pass of radix R over the length-n rows, after passes whose radices
// multiply to Ns, takes butterfly j (0 <= j < n / R) of every row: the R
// inputs j + r n / R, each times exp(-+ 2 pi i r (j mod Ns) / (Ns R)), one
// R-point DFT, and the outputs at (j div Ns) Ns R + (j mod Ns) + r Ns.  After
// the last pass the rows hold their DFTs in natural order.

// 3-point DFT: X0 = a + t, X1,2 = a - t / 2 -+ i (sqrt(3) / 2) (b - c) for
// the forward transform (t = b + c); the inverse flips the sign of i.
template <typename T> __device__ __forceinline__ void dft3(T *x, int inverse) {
  using R = decltype(T{}.x);
  constexpr R h = (R)0.86602540378443864676372317075293618;  // sqrt(3) / 2
  const T t = cadd(x[1], x[2]), dd = rot_quarter(csub(x[1], x[2]), inverse);
  const T m = T{x[0].x - (R)0.5 * t.x, x[0].y - (R)0.5 * t.y};
  const T r = T{h * dd.x, h * dd.y};
  x[0] = cadd(x[0], t);
  x[1] = cadd(m, r);
  x[2] = csub(m, r);
}

// 5-point DFT from the symmetric pairs t1 = x1 + x4, t2 = x2 + x3 and
// t3 = x1 - x4, t4 = x2 - x3 (c_j = cos(2 pi j / 5), s_j = sin(2 pi j / 5)):
//   X1, X4 = x0 + c1 t1 + c2 t2 -+ i (s1 t3 + s2 t4)
//   X2, X3 = x0 + c2 t1 + c1 t2 -+ i (s2 t3 - s1 t4)
// (forward signs; the inverse flips the sign of i).
template <typename T> __device__ __forceinline__ void dft5(T *x, int inverse) {
  using R = decltype(T{}.x);
  constexpr R c1 = (R)0.30901699437494742410229341718281906;
  constexpr R c2 = (R)-0.80901699437494742410229341718281906;
  constexpr R s1 = (R)0.95105651629515357211643933337938214;
  constexpr R s2 = (R)0.58778525229247312916870595463907277;
  const T t1 = cadd(x[1], x[4]), t2 = cadd(x[2], x[3]), t3 = csub(x[1], x[4]), t4 = csub(x[2], x[3]);
  const T a1 = T{x[0].x + c1 * t1.x + c2 * t2.x, x[0].y + c1 * t1.y + c2 * t2.y};
  const T a2 = T{x[0].x + c2 * t1.x + c1 * t2.x, x[0].y + c2 * t1.y + c1 * t2.y};
  const T b1 = rot_quarter(T{s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y}, inverse);
  const T b2 = rot_quarter(T{s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y}, inverse);
  x[0] = T{x[0].x + t1.x + t2.x, x[0].y + t1.y + t2.y};
  x[1] = cadd(a1, b1);
  x[4] = csub(a1, b1);
  x[2] = cadd(a2, b2);
  x[3] = csub(a2, b2);
}

template <typename T, int R> __device__ __forceinline__ void dft_any(T *x, int inverse) {
  if constexpr (R == 2) {
    const T a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  } else if constexpr (R == 3) {
    dft3(x, inverse);
  } else if constexpr (R == 4) {
    const T s0 = cadd(x[0], x[2]), d0 = csub(x[0], x[2]);
    const T s1 = cadd(x[1], x[3]), d1 = rot_quarter(csub(x[1], x[3]), inverse);
    x[0] = cadd(s0, s1);
    x[2] = csub(s0, s1);
    x[1] = cadd(d0, d1);
    x[3] = csub(d0, d1);
  } else {
    dft5(x, inverse);
  }
}

// One pass of radix R; CB butterflies per thread at most (the caller's
// element budget: nrows * n <= blockDim * E with CB = ceil(E / R)).
template <typename T, int R, int CB>
__device__ __forceinline__ void lds_mr_pass(T *sm, int n, int Ns, int nrows, int rowstride, int inverse,
                                            const T *__restrict__ tw) {
  const int stride = n / R, nb = nrows * stride, tstep = n / (Ns * R);
  T v[CB][R];
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    const int b = threadIdx.x + c * (int)blockDim.x;
    if (b >= nb) break;
    const int l = b / stride, j = b - l * stride, k = j % Ns;
    const T *sp = sm + l * rowstride;
#pragma unroll
    for (int r = 0; r < R; ++r) v[c][r] = sp[j + r * stride];
#pragma unroll
    for (int r = 1; r < R; ++r) {
      T w = tw[r * k * tstep];
      if (inverse) w.y = -w.y;
      v[c][r] = cmul(v[c][r], w);
    }
    dft_any<T, R>(v[c], inverse);
#pragma unroll
    for (int r = 0; r < R; ++r) asm volatile("" : "+v"(v[c][r].x), "+v"(v[c][r].y));
    asm volatile("" ::: "memory");
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    const int b = threadIdx.x + c * (int)blockDim.x;
    if (b >= nb) break;
    const int l = b / stride, j = b - l * stride, k = j % Ns;
    T *dp = sm + l * rowstride + (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dp[r * Ns] = v[c][r];
  }
  __syncthreads();
}

// DFT of nrows rows of length n = 2^a 3^b 5^c in place (tw[m] =
// exp(-2 pi i m / n); inverse = 1 conjugates).  Requires nrows * n <=
// blockDim * E; all threads take part and synchronise.
template <typename T, int E = 16>
__device__ __forceinline__ void lds_fft_rows_mr(T *sm, int n, int nrows, int rowstride, int inverse,
                                                const T *__restrict__ tw) {
  int rem = n, Ns = 1;
  while (rem % 4 == 0) {
    lds_mr_pass<T, 4, (E + 3) / 4>(sm, n, Ns, nrows, rowstride, inverse, tw);
    Ns *= 4;
    rem /= 4;
  }
  if (rem % 2 == 0) {
    lds_mr_pass<T, 2, (E + 1) / 2>(sm, n, Ns, nrows, rowstride, inverse, tw);
    Ns *= 2;
    rem /= 2;
  }
  while (rem % 3 == 0) {
    lds_mr_pass<T, 3, (E + 2) / 3>(sm, n, Ns, nrows, rowstride, inverse, tw);
    Ns *= 3;
    rem /= 3;
  }
  while (rem % 5 == 0) {
    lds_mr_pass<T, 5, (E + 4) / 5>(sm, n, Ns, nrows, rowstride, inverse, tw);
    Ns *= 5;
    rem /= 5;
  }
}

}  // namespace fggc
#endif
