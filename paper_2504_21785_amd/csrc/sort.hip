// Counting sort of key slots by a small integer key, and the pre-pass
// reduction over the packets.
//
// bucket_positions: for every slot i with keys[i] in [0, nbins), pos[i] is its
// position in key order (slots with kNoKey get kNoKey); start[b] is the first
// position of key b and start[nbins] the number of keyed slots.  Producers then
// write each slot's record straight to its position (no permutation array and
// no gather).  For nbins <= kMaxLdsBins:
//   rank    each workgroup counts the keys of its contiguous chunk with LDS
//           atomics, keeping each slot's returned count as its rank inside
//           (key, chunk), and writes the counts bin-major into
//           table[bin * G + chunk_column(chunk)];
//   scan    a wave per bin turns its row into offsets inside the bin and a
//           bin total; one workgroup scans the totals into start[];
//   pos     pos[i] = start[key] + offset of (key, chunk) + rank.
// Larger key ranges (up to 2^30) sort in two levels, every step a counting
// pass of our own: the same three steps on the coarse key (key >> fb, at most
// kMaxLdsBins of them) place each slot's index in a permutation array in
// coarse order; then one workgroup per coarse bin counts the fine keys
// (key & (2^fb - 1)) of its contiguous range in LDS, scans them, writes the
// bin's entries of start[] and the final positions.  Nothing is cleared by a
// memset and no count lives across calls, so the whole sort can be captured in
// a graph and replayed.
// The order of slots inside a key follows the LDS atomics (unspecified).
//
// packet_scan: per packet, NaN/Inf and magnitude checks, and per dimension the
// range of floor(P/dp); a two-level reduction (per-workgroup results, then one
// workgroup) -- no global atomics.
#include <climits>

#include "common.h"

namespace fggc {
namespace {

constexpr int64_t kMaxLdsBins = 32768;
constexpr int kSortBlock = 1024;

// (the counted key is keys[i] >> shift: the whole key, or the coarse key of
// the two-level sort)
__global__ __launch_bounds__(kSortBlock) void bucket_rank_kernel(const uint32_t *__restrict__ keys, int64_t N,
                                                                int64_t chunk, int64_t nbins, int G, int shift,
                                                                uint32_t *__restrict__ table,
                                                                uint32_t *__restrict__ rank) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  uint32_t *cnt = reinterpret_cast<uint32_t *>(smem_raw);
  for (int64_t b = threadIdx.x; b < nbins; b += blockDim.x) cnt[b] = 0;
  __syncthreads();
  const int64_t lo = blockIdx.x * chunk, hi = min(N, lo + chunk);
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const uint32_t k = keys[i];
    if (k != kNoKey) rank[i] = atomicAdd(&cnt[k >> shift], 1u);
  }
  __syncthreads();
  const int64_t col = chunk_column(blockIdx.x, G);
  for (int64_t b = threadIdx.x; b < nbins; b += blockDim.x) table[b * G + col] = cnt[b];
}

__global__ void bucket_pos_kernel(const uint32_t *__restrict__ keys, const uint32_t *__restrict__ rank,
                                  int64_t N, int64_t chunk, int G, const uint32_t *__restrict__ offs,
                                  const int64_t *__restrict__ start, uint32_t *__restrict__ pos) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  const uint32_t k = keys[i];
  pos[i] = k == kNoKey ? kNoKey
                       : (uint32_t)start[k] + offs[(int64_t)k * G + chunk_column(i / chunk, G)] + rank[i];
}

// Scan of the count table in two steps.  Row step: one wave per bin turns
// its row of G chunk counts into offsets inside the bin and writes the bin's
// total.
constexpr int kRowMax = 16;  // counts per lane: G <= 64 * kRowMax
__global__ __launch_bounds__(256) void count_rowscan_kernel(const uint32_t *__restrict__ table, int64_t nbins,
                                                            int G, uint32_t *__restrict__ offs,
                                                            uint32_t *__restrict__ rowsum) {
  const int lane = threadIdx.x & 63;
  const int64_t b = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
  if (b >= nbins) return;  // b is the same for the whole wave
  const int per = (G + 63) / 64, c0 = lane * per;
  const uint32_t *row = table + b * G;
  uint32_t v[kRowMax], sum = 0;
#pragma unroll
  for (int i = 0; i < kRowMax; ++i) {
    v[i] = (i < per && c0 + i < G) ? row[c0 + i] : 0u;
    sum += v[i];
  }
  uint32_t incl = sum;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t u = __shfl_up(incl, d, 64);
    if (lane >= d) incl += u;
  }
  uint32_t run = incl - sum;
  uint32_t *orow = offs + b * G;
#pragma unroll
  for (int i = 0; i < kRowMax; ++i) {
    if (i < per && c0 + i < G) orow[c0 + i] = run;
    run += v[i];
  }
  if (lane == 63) rowsum[b] = incl;
}

// Bin step: one workgroup scans the bin totals into start[0 .. nbins].
__global__ __launch_bounds__(1024) void count_binscan_kernel(const uint32_t *__restrict__ rowsum, int64_t nbins,
                                                             int64_t *__restrict__ start) {
  __shared__ int64_t wsum[16];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t per = (nbins + 1023) / 1024, b0 = tid * per;
  int64_t sum = 0;
  for (int64_t i = 0; i < per; ++i)
    if (b0 + i < nbins) sum += rowsum[b0 + i];
  int64_t incl = sum;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t u = __shfl_up(incl, d, 64);
    if (lane >= d) incl += u;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int64_t run = incl - sum;
  for (int j = 0; j < w; ++j) run += wsum[j];
  for (int64_t i = 0; i < per; ++i)
    if (b0 + i < nbins) {
      start[b0 + i] = run;
      run += rowsum[b0 + i];
    }
  if (tid == 1023) start[nbins] = run;
}

// Two-level sort, step 2: the index of every keyed slot goes to its position
// in coarse-key order; unkeyed slots get pos = kNoKey here (the fine step
// writes the positions of the others).
__global__ void coarse_perm_kernel(const uint32_t *__restrict__ keys, const uint32_t *__restrict__ rank,
                                   int64_t N, int64_t chunk, int G, int fb, const uint32_t *__restrict__ offs,
                                   const int64_t *__restrict__ cstart, uint32_t *__restrict__ perm,
                                   uint32_t *__restrict__ pos) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  const uint32_t k = keys[i];
  if (k == kNoKey) {
    pos[i] = kNoKey;
    return;
  }
  const uint32_t c = k >> fb;
  const int64_t at = cstart[c] + offs[(int64_t)c * G + chunk_column(i / chunk, G)] + rank[i];
  perm[at] = (uint32_t)i;
}

// Two-level sort, step 3: one workgroup per coarse bin c.  Its slots occupy
// perm[cstart[c], cstart[c + 1]); the fine keys are counted in LDS (each
// slot's returned count is its rank inside the fine key), scanned in LDS, and
// give start[] of the bin's keys and every slot's final position.
constexpr int kFineThreads = 256;
__global__ __launch_bounds__(kFineThreads) void fine_sort_kernel(const uint32_t *__restrict__ keys,
                                                                 const uint32_t *__restrict__ perm,
                                                                 const int64_t *__restrict__ cstart, int64_t nbins,
                                                                 int64_t ncoarse, int fb,
                                                                 uint32_t *__restrict__ rank2,
                                                                 int64_t *__restrict__ start,
                                                                 uint32_t *__restrict__ pos) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  uint32_t *cnt = reinterpret_cast<uint32_t *>(smem_raw);
  __shared__ uint32_t wsum[kFineThreads / 64];
  const int64_t c = blockIdx.x;
  const int64_t kb = c << fb;
  const int nf = (int)min<int64_t>((int64_t)1 << fb, nbins - kb);  // fine keys of this bin
  const uint32_t fmask = (1u << fb) - 1u;
  const int64_t lo = cstart[c], hi = cstart[c + 1];
  const int tid = threadIdx.x;
  for (int f = tid; f < nf; f += kFineThreads) cnt[f] = 0u;
  __syncthreads();
  for (int64_t j = lo + tid; j < hi; j += kFineThreads) rank2[j] = atomicAdd(&cnt[keys[perm[j]] & fmask], 1u);
  __syncthreads();
  // exclusive scan of cnt[0, nf): contiguous runs per thread, then the waves
  const int per = (nf + kFineThreads - 1) / kFineThreads, f0 = tid * per;
  uint32_t sum = 0;
  for (int q = 0; q < per; ++q)
    if (f0 + q < nf) sum += cnt[f0 + q];
  const int lane = tid & 63, w = tid >> 6;
  uint32_t incl = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = __shfl_up(incl, o, 64);
    if (lane >= o) incl += u;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  uint32_t run = incl - sum;
  for (int x = 0; x < w; ++x) run += wsum[x];
  for (int q = 0; q < per; ++q)
    if (f0 + q < nf) {
      const uint32_t v = cnt[f0 + q];
      cnt[f0 + q] = run;
      start[kb + f0 + q] = lo + run;
      run += v;
    }
  if (c == ncoarse - 1 && tid == 0) start[nbins] = hi;
  __syncthreads();
  for (int64_t j = lo + tid; j < hi; j += kFineThreads) {
    const uint32_t i = perm[j];
    pos[i] = (uint32_t)(lo + cnt[keys[i] & fmask] + rank2[j]);
  }
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

// Reduction of the seven scan values {bad, min0..2, max0..2} over a
// workgroup of 256: shuffles within each wave, then the four wave results.
__device__ __forceinline__ void reduce_scan7(long long v[7], long long *__restrict__ dst) {
  __shared__ long long red[4][7];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    v[0] += __shfl_xor(v[0], o);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      v[1 + k] = min(v[1 + k], __shfl_xor(v[1 + k], o));
      v[4 + k] = max(v[4 + k], __shfl_xor(v[4 + k], o));
    }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0)
    for (int t = 0; t < 7; ++t) red[w][t] = v[t];
  __syncthreads();
  if (threadIdx.x < 7) {
    const int t = threadIdx.x;
    long long r = red[0][t];
    for (int x = 1; x < 4; ++x) r = t == 0 ? r + red[x][t] : (t < 4 ? min(r, red[x][t]) : max(r, red[x][t]));
    dst[t] = r;
  }
}

// out[block] = {bad, min0, min1, min2, max0, max1, max2, pad}
template <int D>
__global__ __launch_bounds__(256) void packet_scan_kernel(ScanParams p, long long *__restrict__ out) {
  long long v[7] = {0, LLONG_MAX, LLONG_MAX, LLONG_MAX, LLONG_MIN, LLONG_MIN, LLONG_MIN};
  const int64_t lo = blockIdx.x * p.per_block, hi = min(p.N, lo + p.per_block);
  // U packets per thread and pass, so that their loads are in flight together
  constexpr int U = 4;
  for (int64_t j0 = lo + threadIdx.x; j0 < hi; j0 += U * (int64_t)blockDim.x) {
    double sv[U], ar[U], ai[U], qv[U][D], pv[U][D];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = j0 + u * (int64_t)blockDim.x;
      if (j >= hi) break;
      const double2 aj = reinterpret_cast<const double2 *>(p.a)[j];
      sv[u] = p.S[j];
      ar[u] = aj.x;
      ai[u] = aj.y;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        qv[u][k] = p.Q[k * p.N + j];
        pv[u][k] = p.P[k * p.N + j];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = j0 + u * (int64_t)blockDim.x;
      if (j >= hi) break;
      bool ok = isfinite(sv[u]) && isfinite(ar[u]) && isfinite(ai[u]);
#pragma unroll
      for (int k = 0; k < D; ++k) {
        ok = ok && fabs(qv[u][k]) <= 1.0e9 && fabs(pv[u][k]) <= 1.0e9;
        if (p.want_range && fabs(pv[u][k]) <= 1.0e9) {
          const long long c = (long long)floor_cell(pv[u][k] / p.dp[k]);
          v[1 + k] = min(v[1 + k], c);
          v[4 + k] = max(v[4 + k], c);
        }
      }
      if (!ok) ++v[0];
    }
  }
  reduce_scan7(v, out + blockIdx.x * 8);
}

__global__ __launch_bounds__(256) void packet_scan_final_kernel(const long long *__restrict__ part, int nb,
                                                                long long *__restrict__ out) {
  long long v[7] = {0, LLONG_MAX, LLONG_MAX, LLONG_MAX, LLONG_MIN, LLONG_MIN, LLONG_MIN};
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    v[0] += part[b * 8];
    for (int k = 0; k < 3; ++k) {
      v[1 + k] = min(v[1 + k], part[b * 8 + 1 + k]);
      v[4 + k] = max(v[4 + k], part[b * 8 + 4 + k]);
    }
  }
  reduce_scan7(v, out);
}

constexpr int kScanBlocks = 1024;

struct SortPlan {
  bool lds;        // one level: nbins <= kMaxLdsBins
  int fb;          // two levels: fine bits (fine keys per coarse bin = 2^fb)
  int64_t ncoarse; // keys counted by the first level (nbins, or the coarse keys)
  int G;
  int64_t chunk;
  size_t off_table, off_offs, off_rank, off_tmp, off_cstart, off_perm, off_rank2, total;
};

SortPlan sort_plan(int64_t N, int64_t nbins, int unit = 1) {
  SortPlan sp{};
  const int64_t Nn = std::max<int64_t>(N, 1);
  sp.lds = nbins <= kMaxLdsBins;
  sp.fb = 0;
  if (!sp.lds) {
    while (((nbins + ((int64_t)1 << sp.fb) - 1) >> sp.fb) > kMaxLdsBins) ++sp.fb;
    if (sp.fb > 15) fail(FGGC_EUNSUPPORTED, "more than 2^30 sort keys");
  }
  sp.ncoarse = (nbins + ((int64_t)1 << sp.fb) - 1) >> sp.fb;
  size_t o = 0;
  auto put = [&](size_t b) {
    size_t at = o;
    o = align_up(o + b, 256);
    return at;
  };
  // chunks of >= 8192 slots, at most 1024 of them (the row scan's limit),
  // and a table of at most ~2^22 entries: every (bin, chunk) count is a
  // separate write, so fewer, larger chunks keep the table cheap
  const int64_t nb1 = std::max<int64_t>(sp.ncoarse, 1);
  int64_t G = std::min<int64_t>(64 * kRowMax, (Nn + 8191) / 8192);
  G = std::max<int64_t>(1, std::min<int64_t>(G, ((int64_t)1 << 22) / nb1));
  if (G >= 8) G &= ~(int64_t)7;  // whole XCD rounds (chunk_column)
  sp.chunk = (Nn + G - 1) / G;
  sp.chunk = (sp.chunk + unit - 1) / unit * unit;  // whole packets per chunk
  sp.G = (int)((Nn + sp.chunk - 1) / sp.chunk);
  const int64_t tn = nb1 * sp.G;
  sp.off_table = put(tn * 4);
  sp.off_offs = put(tn * 4);
  sp.off_rank = put(Nn * 4);
  sp.off_tmp = put(nb1 * 4);  // bin totals
  if (!sp.lds) {
    sp.off_cstart = put((nb1 + 1) * 8);
    sp.off_perm = put(Nn * 4);
    sp.off_rank2 = put(Nn * 4);
  }
  sp.total = o;
  return sp;
}

bool g_sort_attr = false;
std::mutex g_sort_mu;

}  // namespace

size_t bucket_positions_bytes(int64_t N, int64_t nbins) { return sort_plan(N, nbins).total + 256; }

CountPlan count_plan(int64_t N, int64_t nbins, int unit) {
  const SortPlan sp = sort_plan(N, nbins, unit);
  CountPlan c{};
  c.lds = sp.lds;
  c.G = sp.G;
  c.chunk = sp.chunk;
  c.off_table = sp.off_table;
  c.off_offs = sp.off_offs;
  c.off_rank = sp.off_rank;
  c.off_rowsum = sp.off_tmp;
  c.bytes = sp.total + 256;
  return c;
}

void count_positions(const CountPlan &c, const uint32_t *keys, int64_t N, char *scratch, const int64_t *start,
                     uint32_t *pos, hipStream_t s) {
  const uint32_t *rank = (const uint32_t *)(scratch + c.off_rank), *offs = (const uint32_t *)(scratch + c.off_offs);
  bucket_pos_kernel<<<dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s>>>(keys, rank, N, c.chunk, c.G, offs,
                                                                            start, pos);
  FGGC_HIP(hipGetLastError());
}

void count_scan(const CountPlan &c, int64_t nbins, char *scratch, int64_t *start, hipStream_t s) {
  uint32_t *table = (uint32_t *)(scratch + c.off_table), *offs = (uint32_t *)(scratch + c.off_offs),
           *rowsum = (uint32_t *)(scratch + c.off_rowsum);
  count_rowscan_kernel<<<dim3((unsigned)((nbins * 64 + 255) / 256)), dim3(256), 0, s>>>(table, nbins, c.G, offs,
                                                                                      rowsum);
  FGGC_HIP(hipGetLastError());
  count_binscan_kernel<<<dim3(1), dim3(1024), 0, s>>>(rowsum, nbins, start);
  FGGC_HIP(hipGetLastError());
}

// Every path is counting passes of our own with no memset and no state kept
// between calls, so every size can be captured in a graph and replayed.
bool bucket_positions_graph_safe(int64_t, int64_t) { return true; }

void bucket_positions(const uint32_t *keys, int64_t N, int64_t nbins, uint32_t *pos, int64_t *start,
                      void *scratch, hipStream_t s) {
  if (N >= ((int64_t)1 << 31)) fail(FGGC_EUNSUPPORTED, "more than 2^31 sort slots");
  if (nbins >= ((int64_t)1 << 31)) fail(FGGC_EUNSUPPORTED, "more than 2^31 sort keys");
  const SortPlan sp = sort_plan(N, nbins);
  char *base = (char *)scratch;
  {
    std::lock_guard<std::mutex> lk(g_sort_mu);
    if (!g_sort_attr) {
      FGGC_HIP(hipFuncSetAttribute((const void *)bucket_rank_kernel,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kMaxLdsBins * 4)));
      FGGC_HIP(hipFuncSetAttribute((const void *)fine_sort_kernel,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kMaxLdsBins * 4)));
      g_sort_attr = true;
    }
  }
  const unsigned gN = (unsigned)((std::max<int64_t>(N, 1) + 255) / 256);
  // first level: the whole key, or the coarse key
  const int64_t nb1 = sp.ncoarse;
  uint32_t *table = (uint32_t *)(base + sp.off_table), *offs = (uint32_t *)(base + sp.off_offs),
           *rank = (uint32_t *)(base + sp.off_rank);
  if (N > 0) {
    bucket_rank_kernel<<<dim3(sp.G), dim3(kSortBlock), (size_t)nb1 * 4, s>>>(keys, N, sp.chunk, nb1, sp.G,
                                                                             sp.fb, table, rank);
    FGGC_HIP(hipGetLastError());
  } else {
    launch_zero(table, (size_t)nb1 * sp.G * 4, s);
  }
  uint32_t *rowsum = (uint32_t *)(base + sp.off_tmp);
  int64_t *start1 = sp.lds ? start : (int64_t *)(base + sp.off_cstart);
  count_rowscan_kernel<<<dim3((unsigned)((nb1 * 64 + 255) / 256)), dim3(256), 0, s>>>(table, nb1, sp.G, offs,
                                                                                     rowsum);
  FGGC_HIP(hipGetLastError());
  count_binscan_kernel<<<dim3(1), dim3(1024), 0, s>>>(rowsum, nb1, start1);
  FGGC_HIP(hipGetLastError());
  if (sp.lds) {
    if (N > 0) {
      bucket_pos_kernel<<<dim3(gN), dim3(256), 0, s>>>(keys, rank, N, sp.chunk, sp.G, offs, start, pos);
      FGGC_HIP(hipGetLastError());
    }
    return;
  }
  // second level: slot indices in coarse order, then the fine keys per coarse bin
  uint32_t *perm = (uint32_t *)(base + sp.off_perm), *rank2 = (uint32_t *)(base + sp.off_rank2);
  if (N > 0) {
    coarse_perm_kernel<<<dim3(gN), dim3(256), 0, s>>>(keys, rank, N, sp.chunk, sp.G, sp.fb, offs, start1, perm,
                                                      pos);
    FGGC_HIP(hipGetLastError());
  }
  fine_sort_kernel<<<dim3((unsigned)nb1), dim3(kFineThreads), ((size_t)4 << sp.fb), s>>>(
      keys, perm, start1, nbins, nb1, sp.fb, rank2, start, pos);
  FGGC_HIP(hipGetLastError());
}

__global__ void zero_kernel(uint32_t *__restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// Slots [N, Npad) of SoA arrays sized Npad get zero-amplitude copies of
// packets 0, 1, 2, ... (cyclically).  The copies sit where the real packets
// are, so no cell receives more than a few of them; copies of a single
// packet would pile into one cell and serialise the accumulation of its bin.
__global__ void pad_packets_kernel(int d, int64_t N, int64_t Npad, double *Q, double *P, double *S,
                                   double *a) {
  const int64_t j = N + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= Npad) return;
  const int64_t src = (j - N) % N;
  for (int k = 0; k < d; ++k) {
    Q[k * Npad + j] = Q[k * Npad + src];
    P[k * Npad + j] = P[k * Npad + src];
  }
  S[j] = S[src];
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
  if (pk.d == 1) packet_scan_kernel<1><<<dim3(nb), dim3(256), 0, s>>>(p, part);
  else if (pk.d == 2) packet_scan_kernel<2><<<dim3(nb), dim3(256), 0, s>>>(p, part);
  else packet_scan_kernel<3><<<dim3(nb), dim3(256), 0, s>>>(p, part);
  FGGC_HIP(hipGetLastError());
  packet_scan_final_kernel<<<dim3(1), dim3(256), 0, s>>>(part, nb, out);
  FGGC_HIP(hipGetLastError());
}

}  // namespace fggc
