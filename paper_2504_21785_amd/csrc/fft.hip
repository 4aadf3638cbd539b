// Batched complex FFT in LDS: Stockham autosort passes, one workgroup per
// group of lines along one axis of a row-major array.  Power-of-two lengths
// and strides take radix-8/4/2 passes and shift/mask indexing; other lengths
// n = 2^a 3^b 5^c (and strides that are not powers of two) take the
// mixed-radix passes (radix 4, 2, 3, 5) with general indexing.  A
// d-dimensional transform is d such axis passes.  Twiddles come from a
// table exp(-2 pi i k / n) computed in FP64 on the host (rounded once to the
// working precision) and kept per device for the life of the process.
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>

#include "common.h"
#include "lds_fft.h"

namespace fggc {
namespace {

struct FftAxis {
  int64_t nlines;
  int log2n, log2L;   // line length and lines per workgroup (powers of two)
  int log2inner;      // lines of one axis are 2^log2inner apart (inner stride)
  int inverse;
  int transpose_out;  // lines are contiguous rows: store element i of line l at dst[i * nlines + l]
  int log2big;        // > 0: multiply output i of line (bo, bi) by exp(-+ 2 pi i bi i / 2^log2big)
};

// All index arithmetic on powers of two (shifts and masks, 32-bit inside the
// workgroup, 64-bit only for global offsets).
template <typename T>
__global__ __launch_bounds__(1024) void fft_axis_kernel(const T *src, T *dst, FftAxis a,
                                                        const T *__restrict__ tw,
                                                        const T *__restrict__ twbig) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *sm = reinterpret_cast<T *>(smem_raw);
  const int lg = a.log2n, lgL = a.log2L, lgin = a.log2inner;
  const int n = 1 << lg, L = 1 << lgL;
  const int64_t inner_mask = ((int64_t)1 << lgin) - 1;
  const int64_t line0 = (int64_t)blockIdx.x << lgL;
  const int tot = L << lg;
  T *stw = sm + tot;  // the twiddles, staged in LDS
  for (int i = threadIdx.x; i < n; i += blockDim.x) stw[i] = tw[i];
  // load (coalesced: along the line when lines are contiguous, across lines otherwise)
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    int l, i;
    if (lgin == 0) {
      l = e >> lg;
      i = e & (n - 1);
    } else {
      i = e >> lgL;
      l = e & (L - 1);
    }
    const int64_t line = line0 + l;
    if (line < a.nlines) {
      const int64_t bo = line >> lgin, bi = line & inner_mask;
      sm[(l << lg) + i] = src[((((bo << lg) + i)) << lgin) + bi];
    }
  }
  __syncthreads();
  lds_fft_rows<T>(sm, lg, L, n, a.inverse, stw);
  const int bigmask = (1 << a.log2big) - 1;
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    int l, i;
    if (lgin == 0 && !a.transpose_out) {
      l = e >> lg;
      i = e & (n - 1);
    } else {
      i = e >> lgL;
      l = e & (L - 1);
    }
    const int64_t line = line0 + l;
    if (line < a.nlines) {
      const int64_t bo = line >> lgin, bi = line & inner_mask;
      T v = sm[(l << lg) + i];
      if (a.log2big > 0) {  // four-step twiddle exp(-+ 2 pi i bi i / nbig)
        T w = twbig[((int)bi * i) & bigmask];
        if (a.inverse) w.y = -w.y;
        v = cmul(v, w);
      }
      if (a.transpose_out) dst[(int64_t)i * a.nlines + line] = v;
      else dst[((((bo << lg) + i)) << lgin) + bi] = v;
    }
  }
}

// Lines of any length n = 2^a 3^b 5^c and any inner stride: line `line` is
// (bo, bi) = (line / inner, line % inner), element i at (bo n + i) inner + bi.
struct FftAxisMr {
  int64_t nlines, inner;
  int n, L;  // line length, lines per workgroup
  int inverse;
  int transpose_out;  // store element i of line l at dst[i * nlines + l]
  int64_t nbig;       // > 0: multiply output i of line (bo, bi) by exp(-+ 2 pi i bi i / nbig)
};

constexpr int kMrElems = 16;  // elements per thread of the mixed-radix passes

template <typename T>
__global__ __launch_bounds__(1024) void fft_axis_mr_kernel(const T *src, T *dst, FftAxisMr a,
                                                           const T *__restrict__ tw,
                                                           const T *__restrict__ twbig) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *sm = reinterpret_cast<T *>(smem_raw);
  const int n = a.n, L = a.L, tot = L * n;
  const int64_t line0 = (int64_t)blockIdx.x * L;
  T *stw = sm + tot;
  for (int i = threadIdx.x; i < n; i += blockDim.x) stw[i] = tw[i];
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    // along the line when lines are contiguous, across lines otherwise
    const int l = a.inner == 1 ? e / n : e % L, i = a.inner == 1 ? e % n : e / L;
    const int64_t line = line0 + l;
    if (line < a.nlines) {
      const int64_t bo = line / a.inner, bi = line - bo * a.inner;
      sm[l * n + i] = src[(bo * n + i) * a.inner + bi];
    }
  }
  __syncthreads();
  lds_fft_rows_mr<T, kMrElems>(sm, n, L, n, a.inverse, stw);
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    const bool rowwise = a.inner == 1 && !a.transpose_out;
    const int l = rowwise ? e / n : e % L, i = rowwise ? e % n : e / L;
    const int64_t line = line0 + l;
    if (line < a.nlines) {
      const int64_t bo = line / a.inner, bi = line - bo * a.inner;
      T v = sm[l * n + i];
      if (a.nbig > 0) {  // four-step twiddle exp(-+ 2 pi i bi i / nbig)
        T w = twbig[(bi * i) % a.nbig];
        if (a.inverse) w.y = -w.y;
        v = cmul(v, w);
      }
      if (a.transpose_out) dst[(int64_t)i * a.nlines + line] = v;
      else dst[(bo * n + i) * a.inner + bi] = v;
    }
  }
}

// twiddle tables, per (device, n, precision), created on first use
std::mutex g_tw_mu;
std::map<std::tuple<int, int64_t, int>, void *> g_tw;

const void *twiddles(int64_t n, int precision) {
  int dev = 0;
  FGGC_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_tw_mu);
  auto key = std::make_tuple(dev, n, precision);
  auto it = g_tw.find(key);
  if (it != g_tw.end()) return it->second;
  void *p = nullptr;
  const size_t es = precision == FGGC_FP64 ? 16 : 8;
  FGGC_HIP(hipMalloc(&p, (size_t)n * es));
  std::vector<double> h(2 * (size_t)n);
  for (int64_t k = 0; k < n; ++k) {
    // exp(-2 pi i k/n), evaluated in long double and rounded once
    const long double ang = -2.0L * 3.14159265358979323846264338327950288L * (long double)k / (long double)n;
    h[2 * k] = (double)cosl(ang);
    h[2 * k + 1] = (double)sinl(ang);
  }
  if (precision == FGGC_FP64) {
    FGGC_HIP(hipMemcpy(p, h.data(), (size_t)n * 16, hipMemcpyHostToDevice));
  } else {
    std::vector<float> f(2 * (size_t)n);
    for (size_t i = 0; i < f.size(); ++i) f[i] = (float)h[i];
    FGGC_HIP(hipMemcpy(p, f.data(), (size_t)n * 8, hipMemcpyHostToDevice));
  }
  g_tw[key] = p;
  return p;
}

// The mixed-radix form of launch_axis: L lines per workgroup within the
// element budget (L n <= 1024 kMrElems) and the LDS (rows and twiddles).
template <typename T>
void launch_axis_mr(const T *src, T *dst, int64_t n, int64_t inner, int64_t outer, int inverse,
                    hipStream_t s, int transpose_out, int64_t nbig) {
  const int64_t elem = sizeof(T);
  const int64_t lds_elems = 131072 / elem;
  if (n > 1024 * kMrElems || 2 * n > lds_elems) fail(FGGC_EUNSUPPORTED, "FFT line too long");
  const int64_t nlines = inner * outer;
  int64_t L = inner == 1 && !transpose_out ? std::max<int64_t>(1, 4096 / n) : 64;
  L = std::min(L, lds_elems / n - 1);
  L = std::min(L, (int64_t)1024 * kMrElems / n);
  // keep at least ~256 workgroups when there are enough lines
  L = std::max<int64_t>(1, std::min(L, nlines / 256));
  L = std::min(L, std::max<int64_t>(nlines, 1));
  const int64_t elems = L * n;
  int threads = (int)std::min<int64_t>(1024, std::max<int64_t>(64, (elems + kMrElems - 1) / kMrElems));
  threads = (threads + 63) / 64 * 64;
  FftAxisMr a;
  a.nlines = nlines;
  a.inner = inner;
  a.n = (int)n;
  a.L = (int)L;
  a.inverse = inverse;
  a.transpose_out = transpose_out;
  a.nbig = nbig;
  const T *tw = (const T *)twiddles(n, elem == 8 ? FGGC_FP32 : FGGC_FP64);
  const T *twb = nbig > 0 ? (const T *)twiddles(nbig, elem == 8 ? FGGC_FP32 : FGGC_FP64) : tw;
  const size_t shm = (size_t)(L + 1) * n * elem;  // rows, then twiddles
  const int64_t nblocks = (nlines + L - 1) / L;
  if (nblocks >= ((int64_t)1 << 31)) fail(FGGC_EUNSUPPORTED, "FFT: too many lines");
  fft_axis_mr_kernel<T><<<dim3((unsigned)nblocks), dim3(threads), shm, s>>>(src, dst, a, tw, twb);
  FGGC_HIP(hipGetLastError());
}

template <typename T>
void launch_axis(const T *src, T *dst, int64_t n, int64_t inner, int64_t outer, int inverse,
                 hipStream_t s, int transpose_out = 0, int64_t nbig = 0) {
  if (!is_pow2(n) || !is_pow2(inner) || (nbig > 0 && !is_pow2(nbig))) {
    launch_axis_mr<T>(src, dst, n, inner, outer, inverse, s, transpose_out, nbig);
    return;
  }
  const int64_t elem = sizeof(T);
  const int64_t lds_max = (elem == 8 ? 16384 : 8192);  // elements (128 KB)
  int log2n = 0;
  while (((int64_t)1 << log2n) < n) ++log2n;
  const int64_t nlines = inner * outer;
  int64_t L;
  const int64_t lds_rows = std::max<int64_t>(n, lds_max - n);  // the twiddles take n of it
  if (inner == 1 && !transpose_out) {
    L = std::max<int64_t>(1, std::min<int64_t>(4096 / n, lds_rows / n));
  } else if (inner == 1) {
    L = std::max<int64_t>(1, std::min<int64_t>(64, lds_rows / n));
  } else {
    L = std::max<int64_t>(1, std::min<int64_t>(std::min<int64_t>(64, inner), lds_rows / n));
  }
  // keep at least ~256 workgroups when there are enough lines
  L = std::min(L, std::max<int64_t>(1, nlines / 256));
  L = std::min(L, nlines);
  int lgL = 0;
  while (((int64_t)2 << lgL) <= L) ++lgL;  // lines per workgroup: a power of two
  L = (int64_t)1 << lgL;
  const int R = log2n >= 2 ? 4 : 2;
  int64_t bfly = L * (n / R);
  int threads = (int)std::min<int64_t>(1024, std::max<int64_t>(64, (bfly + 3) / 4));
  threads = (threads + 63) / 64 * 64;
  while ((bfly + threads - 1) / threads > kMaxBfly) {
    // keep per-thread butterflies within the register budget
    if (threads < 1024) threads = std::min(1024, threads * 2);
    else {
      --lgL;
      L = (int64_t)1 << lgL;
      bfly = L * (n / R);
    }
  }
  int lgin = 0;
  while (((int64_t)1 << lgin) < inner) ++lgin;
  if (((int64_t)1 << lgin) != inner) fail(FGGC_EDEVICE, "internal: FFT inner stride must be a power of two");
  int lgbig = 0;
  if (nbig > 0) {
    while (((int64_t)1 << lgbig) < nbig) ++lgbig;
  }
  FftAxis a;
  a.nlines = nlines;
  a.log2n = log2n;
  a.log2L = lgL;
  a.log2inner = lgin;
  a.inverse = inverse;
  a.transpose_out = transpose_out;
  a.log2big = lgbig;
  const T *tw = (const T *)twiddles(n, elem == 8 ? FGGC_FP32 : FGGC_FP64);
  const T *twb = nbig > 0 ? (const T *)twiddles(nbig, elem == 8 ? FGGC_FP32 : FGGC_FP64) : tw;
  const size_t shm = (size_t)(L + 1) * n * elem;  // rows, then twiddles
  const int64_t nblocks = (nlines + L - 1) / L;
  fft_axis_kernel<T><<<dim3((unsigned)nblocks), dim3(threads), shm, s>>>(src, dst, a, tw, twb);
  FGGC_HIP(hipGetLastError());
}

// n = n1 n2 for the four-step form: the divisor n1 <= sqrt(n) nearest sqrt(n)
// with n2 <= 4096 (a power of two splits as 2^floor(lg/2) x 2^ceil(lg/2)).
int64_t four_step_split(int64_t n) {
  for (int64_t n1 = (int64_t)std::sqrt((double)n) + 1; n1 >= 2; --n1)
    if (n1 * n1 <= n && n % n1 == 0 && n / n1 <= 4096) return n1;
  fail(FGGC_EUNSUPPORTED, "FFT length has no four-step split");
}

// d-dimensional transform of one array, src -> dst (src may be dst; src is
// overwritten when the four-step form is used).  One-dimensional sizes above
// 4096 go through the four-step form: column FFTs of the n1 x n2 view with
// the twiddles folded into their store, then row FFTs stored transposed.
template <typename T>
void fft_one(int d, const int64_t *n, int inverse, T *src, T *dst, hipStream_t s) {
  if (d == 1 && n[0] > 4096) {
    const int64_t n1 = four_step_split(n[0]), n2 = n[0] / n1;
    launch_axis<T>(src, src, n1, n2, 1, inverse, s, 0, n[0]);  // columns, twiddled
    launch_axis<T>(src, dst, n2, 1, n1, inverse, s, 1, 0);     // rows, stored transposed
    return;
  }
  const T *in = src;
  for (int k = d - 1; k >= 0; --k) {
    int64_t inner = 1, outer = 1;
    for (int j = k + 1; j < d; ++j) inner *= n[j];
    for (int j = 0; j < k; ++j) outer *= n[j];
    launch_axis<T>(in, dst, n[k], inner, outer, inverse, s);
    in = dst;
  }
}

bool g_attr_set = false;
std::mutex g_attr_mu;

void ensure_attrs() {
  std::lock_guard<std::mutex> lk(g_attr_mu);
  if (g_attr_set) return;
  FGGC_HIP(hipFuncSetAttribute((const void *)fft_axis_kernel<float2>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 131072));
  FGGC_HIP(hipFuncSetAttribute((const void *)fft_axis_kernel<double2>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 131072));
  FGGC_HIP(hipFuncSetAttribute((const void *)fft_axis_mr_kernel<float2>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 131072));
  FGGC_HIP(hipFuncSetAttribute((const void *)fft_axis_mr_kernel<double2>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, 131072));
  g_attr_set = true;
}

}  // namespace

const void *fft_twiddles(int64_t n, int precision) { return twiddles(n, precision); }

size_t fft_workspace_bytes(int d, const int64_t *n, int precision, int64_t batch) {
  if (d == 1 && n[0] > 4096 && batch > 0)
    return (size_t)n[0] * (precision == FGGC_FP64 ? 16 : 8) + 256;
  return 256;
}

void launch_fft(int d, const int64_t *n, int64_t batch, int direction, int precision, void *data,
                Workspace &ws, hipStream_t s, Profiler *prof, const char *stage) {
  ensure_attrs();
  StageScope sc(prof, stage, s);
  const int inverse = direction > 0 ? 1 : 0;
  const size_t es = precision == FGGC_FP64 ? 16 : 8;
  if (d == 1 && n[0] > 4096) {
    // four-step per array, through a scratch copy
    char *tmp = (char *)ws.take((size_t)n[0] * es);
    for (int64_t b = 0; b < batch; ++b) {
      char *x = (char *)data + (size_t)b * n[0] * es;
      FGGC_HIP(hipMemcpyAsync(tmp, x, (size_t)n[0] * es, hipMemcpyDeviceToDevice, s));
      if (precision == FGGC_FP64) fft_one<double2>(1, n, inverse, (double2 *)tmp, (double2 *)x, s);
      else fft_one<float2>(1, n, inverse, (float2 *)tmp, (float2 *)x, s);
    }
    return;
  }
  for (int k = d - 1; k >= 0; --k) {
    int64_t inner = 1, outer = batch;
    for (int j = k + 1; j < d; ++j) inner *= n[j];
    for (int j = 0; j < k; ++j) outer *= n[j];
    if (precision == FGGC_FP64) launch_axis<double2>((double2 *)data, (double2 *)data, n[k], inner, outer, inverse, s);
    else launch_axis<float2>((float2 *)data, (float2 *)data, n[k], inner, outer, inverse, s);
  }
}

void launch_fft_to(int d, const int64_t *n, int direction, int precision, void *src, void *dst,
                   Workspace &, hipStream_t s, Profiler *prof, const char *stage) {
  ensure_attrs();
  StageScope sc(prof, stage, s);
  const int inverse = direction > 0 ? 1 : 0;
  if (precision == FGGC_FP64) fft_one<double2>(d, n, inverse, (double2 *)src, (double2 *)dst, s);
  else fft_one<float2>(d, n, inverse, (float2 *)src, (float2 *)dst, s);
}

}  // namespace fggc
