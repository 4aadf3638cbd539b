// Stable bucket (counting) sort of packet indices by a small integer key, and
// the pre-pass reduction over the packets.
//
// bucket_sort: order[] lists packet indices grouped by ascending key, stable
// (within a key, by index); start[b] is the first position of key b,
// start[nbins] = N.  For nbins <= kMaxLdsBins:
//   hist    each workgroup counts the keys of its contiguous chunk in LDS and
//           writes the counts bin-major into table[bin * G + group];
//   scan    exclusive prefix sum of the table (hipCUB device scan): the offset
//           of every (bin, group) run, and start[] from its first column;
//   place   each workgroup sorts its chunk's (key, local index) words in LDS
//           with a bitonic network and places every element at the offset of
//           its (key, group) run plus its rank among equal keys, so equal keys
//           keep their index order.
// Larger key ranges fall back to a stable hipCUB radix sort of (key, index).
//
// packet_scan: per packet, NaN/Inf and magnitude checks, and per dimension the
// range of floor(P/dp); a two-level reduction (per-workgroup results, then one
// workgroup) -- no global atomics.
#include <hipcub/hipcub.hpp>

#include <climits>

#include "common.h"

namespace fggc {
namespace {

constexpr int64_t kMaxLdsBins = 32768;
constexpr int kSortBlock = 1024;

__global__ __launch_bounds__(kSortBlock) void bucket_hist_kernel(const uint32_t *__restrict__ keys, int64_t N,
                                                                int64_t chunk, int64_t nbins, int G,
                                                                uint32_t *__restrict__ table) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  uint32_t *cnt = reinterpret_cast<uint32_t *>(smem_raw);
  for (int64_t b = threadIdx.x; b < nbins; b += blockDim.x) cnt[b] = 0;
  __syncthreads();
  const int64_t lo = blockIdx.x * chunk, hi = min(N, lo + chunk);
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) atomicAdd(&cnt[keys[i]], 1u);
  __syncthreads();
  for (int64_t b = threadIdx.x; b < nbins; b += blockDim.x) table[b * G + blockIdx.x] = cnt[b];
}

__global__ void bucket_start_kernel(const uint32_t *__restrict__ offs, int64_t nbins, int G, int64_t N,
                                    int64_t *__restrict__ start) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b < nbins) start[b] = offs[b * G];
  if (b == nbins) start[b] = N;
}

// Each workgroup sorts its chunk's (key << lbits | local index) words in LDS
// with a bitonic network; an element's rank among equal keys of the chunk is
// its sorted position minus the first position of its key.  Deterministic,
// and stable by index.
__global__ __launch_bounds__(kSortBlock) void bucket_place_kernel(const uint32_t *__restrict__ keys, int64_t N,
                                                                 int64_t chunk, int lbits, int G,
                                                                 const uint32_t *__restrict__ offs,
                                                                 uint32_t *__restrict__ order) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  uint32_t *a = reinterpret_cast<uint32_t *>(smem_raw);
  const int C = 1 << lbits;  // chunk rounded up to a power of two
  const int64_t lo = blockIdx.x * chunk, hi = min(N, lo + chunk);
  for (int i = threadIdx.x; i < C; i += blockDim.x) {
    const int64_t gi = lo + i;
    a[i] = gi < hi ? ((keys[gi] << lbits) | (uint32_t)i) : 0xffffffffu;
  }
  __syncthreads();
  for (int k = 2; k <= C; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < C; i += blockDim.x) {
        const int ixj = i ^ j;
        if (ixj > i) {
          const uint32_t x = a[i], y = a[ixj];
          const bool up = (i & k) == 0;
          if ((x > y) == up) {
            a[i] = y;
            a[ixj] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  const int n = (int)(hi - lo);
  for (int p = threadIdx.x; p < n; p += blockDim.x) {
    const uint32_t v = a[p];
    const uint32_t key = v >> lbits, li = v & ((1u << lbits) - 1);
    // first sorted position of this key
    int l = 0, r = p;
    const uint32_t kv = key << lbits;
    while (l < r) {
      const int m = (l + r) >> 1;
      if (a[m] < kv) l = m + 1;
      else r = m;
    }
    order[offs[(int64_t)key * G + blockIdx.x] + (p - l)] = (uint32_t)(lo + li);
  }
}

__global__ void iota_kernel(uint32_t *__restrict__ v, int64_t N) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < N) v[i] = (uint32_t)i;
}

// packet pre-pass ---------------------------------------------------------

struct ScanParams {
  int d;
  int64_t N;
  const double *Q, *P, *S, *a;
  double dp[3];
  int want_range;
  int64_t per_block;
};

__device__ __forceinline__ int64_t floor_cell(double v) {
  const double fl = floor(v);
  int64_t i = (int64_t)fl;
  if (v - fl >= 1.0) i += 1;  // the same rounding rule as the int/frac split
  return i;
}

// out[block] = {bad, min0, min1, min2, max0, max1, max2, pad}
__global__ __launch_bounds__(256) void packet_scan_kernel(ScanParams p, long long *__restrict__ out) {
  __shared__ long long red[7][256];
  long long bad = 0, mn[3], mx[3];
  for (int k = 0; k < 3; ++k) {
    mn[k] = LLONG_MAX;
    mx[k] = LLONG_MIN;
  }
  const int64_t lo = blockIdx.x * p.per_block, hi = min(p.N, lo + p.per_block);
  for (int64_t j = lo + threadIdx.x; j < hi; j += blockDim.x) {
    bool ok = isfinite(p.S[j]) && isfinite(p.a[2 * j]) && isfinite(p.a[2 * j + 1]);
    for (int k = 0; k < p.d; ++k) {
      const double q = p.Q[k * p.N + j], pv = p.P[k * p.N + j];
      ok = ok && fabs(q) <= 1.0e9 && fabs(pv) <= 1.0e9;
      if (p.want_range && fabs(pv) <= 1.0e9) {
        const int64_t c = floor_cell(pv / p.dp[k]);
        mn[k] = min(mn[k], (long long)c);
        mx[k] = max(mx[k], (long long)c);
      }
    }
    if (!ok) ++bad;
  }
  red[0][threadIdx.x] = bad;
  for (int k = 0; k < 3; ++k) {
    red[1 + k][threadIdx.x] = mn[k];
    red[4 + k][threadIdx.x] = mx[k];
  }
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      red[0][threadIdx.x] += red[0][threadIdx.x + st];
      for (int k = 0; k < 3; ++k) {
        red[1 + k][threadIdx.x] = min(red[1 + k][threadIdx.x], red[1 + k][threadIdx.x + st]);
        red[4 + k][threadIdx.x] = max(red[4 + k][threadIdx.x], red[4 + k][threadIdx.x + st]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 7) out[blockIdx.x * 8 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void packet_scan_final_kernel(const long long *__restrict__ part, int nb,
                                                                long long *__restrict__ out) {
  __shared__ long long red[7][256];
  long long v[7] = {0, LLONG_MAX, LLONG_MAX, LLONG_MAX, LLONG_MIN, LLONG_MIN, LLONG_MIN};
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    v[0] += part[b * 8];
    for (int k = 0; k < 3; ++k) {
      v[1 + k] = min(v[1 + k], part[b * 8 + 1 + k]);
      v[4 + k] = max(v[4 + k], part[b * 8 + 4 + k]);
    }
  }
  for (int t = 0; t < 7; ++t) red[t][threadIdx.x] = v[t];
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      red[0][threadIdx.x] += red[0][threadIdx.x + st];
      for (int k = 0; k < 3; ++k) {
        red[1 + k][threadIdx.x] = min(red[1 + k][threadIdx.x], red[1 + k][threadIdx.x + st]);
        red[4 + k][threadIdx.x] = max(red[4 + k][threadIdx.x], red[4 + k][threadIdx.x + st]);
      }
    }
    __syncthreads();
  }
  if (threadIdx.x < 7) out[threadIdx.x] = red[threadIdx.x][0];
}

constexpr int kScanBlocks = 1024;

struct SortPlan {
  bool lds;
  int G, lbits;
  int64_t chunk;
  int bits;
  size_t off_table, off_offs, off_tmp, tmp_bytes, off_k2, off_i1, off_i2, total;
};

SortPlan sort_plan(int64_t N, int64_t nbins) {
  SortPlan sp{};
  const int64_t Nn = std::max<int64_t>(N, 1);
  sp.lds = nbins <= kMaxLdsBins && N <= ((int64_t)1 << 22);
  size_t o = 0;
  auto put = [&](size_t b) {
    size_t at = o;
    o = align_up(o + b, 256);
    return at;
  };
  if (sp.lds) {
    // chunks of at most 2^14 elements (LDS bitonic sort); key and local index share 32 bits
    sp.lbits = 12;
    while (((int64_t)1 << sp.lbits) * 1024 < Nn && sp.lbits < 14) ++sp.lbits;
    sp.chunk = (int64_t)1 << sp.lbits;
    sp.G = (int)((Nn + sp.chunk - 1) / sp.chunk);
    int kb = 1;
    while (((int64_t)1 << kb) < nbins) ++kb;
    if (kb + sp.lbits > 31) sp.lds = false;  // padding (all ones) sorts after every entry
  }
  if (sp.lds) {
    const int64_t tn = nbins * sp.G;
    size_t tmp = 0;
    FGGC_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp, (uint32_t *)nullptr, (uint32_t *)nullptr, (int)tn));
    sp.tmp_bytes = tmp;
    sp.off_table = put(tn * 4);
    sp.off_offs = put(tn * 4);
    sp.off_tmp = put(tmp + 256);
  } else {
    sp.bits = 1;
    while (((int64_t)1 << sp.bits) < nbins + 1) ++sp.bits;
    size_t tmp = 0;
    uint32_t *kk = nullptr, *vv = nullptr;
    hipcub::DoubleBuffer<uint32_t> kb(kk, kk), vb(vv, vv);
    FGGC_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, kb, vb, (int)Nn, 0, sp.bits));
    sp.tmp_bytes = tmp;
    sp.off_k2 = put(Nn * 4);
    sp.off_i1 = put(Nn * 4);
    sp.off_i2 = put(Nn * 4);
    sp.off_tmp = put(tmp + 256);
  }
  sp.total = o;
  return sp;
}

__global__ void radix_start_kernel(int64_t N, const uint32_t *__restrict__ skeys, int64_t nbins,
                                   int64_t *__restrict__ start) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b > nbins) return;
  int64_t lo = 0, hi = N;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)skeys[mid] < b) lo = mid + 1;
    else hi = mid;
  }
  start[b] = lo;
}

bool g_sort_attr = false;
std::mutex g_sort_mu;

}  // namespace

size_t bucket_sort_bytes(int64_t N, int64_t nbins) { return sort_plan(N, nbins).total + 256; }

void bucket_sort(uint32_t *keys, int64_t N, int64_t nbins, uint32_t *order, int64_t *start,
                 void *scratch, hipStream_t s) {
  const SortPlan sp = sort_plan(N, nbins);
  char *base = (char *)scratch;
  {
    std::lock_guard<std::mutex> lk(g_sort_mu);
    if (!g_sort_attr) {
      FGGC_HIP(hipFuncSetAttribute((const void *)bucket_hist_kernel,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kMaxLdsBins * 4)));
      FGGC_HIP(hipFuncSetAttribute((const void *)bucket_place_kernel,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, 65536));
      g_sort_attr = true;
    }
  }
  if (sp.lds) {
    uint32_t *table = (uint32_t *)(base + sp.off_table), *offs = (uint32_t *)(base + sp.off_offs);
    const size_t shm = (size_t)nbins * 4;
    if (N > 0) {
      bucket_hist_kernel<<<dim3(sp.G), dim3(kSortBlock), shm, s>>>(keys, N, sp.chunk, nbins, sp.G, table);
      FGGC_HIP(hipGetLastError());
    } else {
      launch_zero(table, (size_t)nbins * sp.G * 4, s);
    }
    size_t tmp = sp.tmp_bytes;
    FGGC_HIP(hipcub::DeviceScan::ExclusiveSum(base + sp.off_tmp, tmp, table, offs, (int)(nbins * sp.G), s));
    bucket_start_kernel<<<dim3((unsigned)((nbins + 1 + 255) / 256)), dim3(256), 0, s>>>(offs, nbins, sp.G, N, start);
    FGGC_HIP(hipGetLastError());
    if (N > 0) {
      const size_t shp = ((size_t)1 << sp.lbits) * 4;
      bucket_place_kernel<<<dim3(sp.G), dim3(kSortBlock), shp, s>>>(keys, N, sp.chunk, sp.lbits, sp.G, offs, order);
      FGGC_HIP(hipGetLastError());
    }
    return;
  }
  // wide key range: stable radix sort of (key, index)
  uint32_t *k2 = (uint32_t *)(base + sp.off_k2), *i1 = (uint32_t *)(base + sp.off_i1),
           *i2 = (uint32_t *)(base + sp.off_i2);
  if (N > 0) {
    iota_kernel<<<dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s>>>(i1, N);
    FGGC_HIP(hipGetLastError());
    hipcub::DoubleBuffer<uint32_t> kb(keys, k2), vb(i1, i2);
    size_t tmp = sp.tmp_bytes;
    FGGC_HIP(hipcub::DeviceRadixSort::SortPairs(base + sp.off_tmp, tmp, kb, vb, (int)N, 0, sp.bits, s));
    FGGC_HIP(hipMemcpyAsync(order, vb.Current(), (size_t)N * 4, hipMemcpyDeviceToDevice, s));
    radix_start_kernel<<<dim3((unsigned)((nbins + 1 + 255) / 256)), dim3(256), 0, s>>>(N, kb.Current(), nbins, start);
  } else {
    radix_start_kernel<<<dim3((unsigned)((nbins + 1 + 255) / 256)), dim3(256), 0, s>>>(0, keys, nbins, start);
  }
  FGGC_HIP(hipGetLastError());
}

__global__ void zero_kernel(uint32_t *__restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// zero-amplitude copies of packet 0 in slots [N, Npad) of SoA arrays sized Npad
__global__ void pad_packets_kernel(int d, int64_t N, int64_t Npad, double *Q, double *P, double *S,
                                   double *a) {
  const int64_t j = N + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= Npad) return;
  for (int k = 0; k < d; ++k) {
    Q[k * Npad + j] = Q[k * Npad];
    P[k * Npad + j] = P[k * Npad];
  }
  S[j] = S[0];
  a[2 * j] = 0.0;
  a[2 * j + 1] = 0.0;
}

void launch_zero(void *p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return;
  if (bytes % 4) fail(FGGC_EDEVICE, "internal: launch_zero needs a multiple of 4 bytes");
  const int64_t n = (int64_t)(bytes / 4);
  const int64_t blocks = std::min<int64_t>(4096, (n + 255) / 256);
  zero_kernel<<<dim3((unsigned)blocks), dim3(256), 0, s>>>((uint32_t *)p, n);
  FGGC_HIP(hipGetLastError());
}

void launch_pad_packets(int d, int64_t N, int64_t Npad, double *Q, double *P, double *S, double *a,
                        hipStream_t s) {
  if (Npad <= N || N < 1) return;
  pad_packets_kernel<<<dim3((unsigned)((Npad - N + 255) / 256)), dim3(256), 0, s>>>(d, N, Npad, Q, P, S, a);
  FGGC_HIP(hipGetLastError());
}

size_t packet_scan_bytes() { return (size_t)kScanBlocks * 8 * 8 + 256; }

void launch_packet_scan(const fggc_packets &pk, const double *dp, long long *part, long long *out,
                        hipStream_t s) {
  ScanParams p{};
  p.d = pk.d;
  p.N = pk.N;
  p.Q = pk.Q;
  p.P = pk.P;
  p.S = pk.S;
  p.a = pk.a;
  p.want_range = dp != nullptr;
  for (int k = 0; k < 3; ++k) p.dp[k] = dp ? dp[k] : 1.0;
  const int nb = (int)std::max<int64_t>(1, std::min<int64_t>(kScanBlocks, (pk.N + 1023) / 1024));
  p.per_block = (pk.N + nb - 1) / nb;
  if (p.per_block < 1) p.per_block = 1;
  packet_scan_kernel<<<dim3(nb), dim3(256), 0, s>>>(p, part);
  FGGC_HIP(hipGetLastError());
  packet_scan_final_kernel<<<dim3(1), dim3(256), 0, s>>>(part, nb, out);
  FGGC_HIP(hipGetLastError());
}

}  // namespace fggc
