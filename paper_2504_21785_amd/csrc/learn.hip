// Device bookkeeping of multi-step FGGC (Sec. 3.2, Alg. 3).
//
// A run decomposes the current wave function on a fixed (q, p) mesh; mesh
// points whose |A(0)| is at most `prune` times the largest are skipped, and
// of the others only those that no earlier run has evolved are propagated.
// The flow is linear in A, so what a mesh point learns is its final
// (Q, P, S) and the ratio A(T) / A(0), obtained by evolving A(0) = 1; a later
// run reconstructs from those with its own A(0):
//   learn_select   max |A0| (two-level reduction), then one workgroup walks
//                  the mesh in order and compacts the kept points and the new
//                  ones (kept and not learned) with wave ballots, marking the
//                  new ones learned -- index lists in mesh order;
//   learn_start    packets at the new points (Q = q, P = p, S = 0, A = 1);
//   learn_store    their propagated state into the per-point tables;
//   learn_packets  the kept points' learned (Q, P, S) and A0 * ratio: the
//                  reconstruction's packets.
#include <cmath>

#include "common.h"

namespace fggc {
namespace {

constexpr int kMaxBlocks = 1024;

__global__ __launch_bounds__(256) void absmax_kernel(const double2 *__restrict__ A, int64_t n,
                                                     double *__restrict__ part) {
  __shared__ double red[4];
  double m = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    m = fmax(m, hypot(A[i].x, A[i].y));
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

__global__ __launch_bounds__(256) void absmax_final_kernel(const double *__restrict__ part, int nb,
                                                           double *__restrict__ out) {
  __shared__ double red[4];
  double m = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) m = fmax(m, part[b]);
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) *out = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// One workgroup, in mesh order: keep = |A0| > prune * max, new = keep and not
// learned.  counts[0] = kept points, counts[1] = new points.
constexpr int kSelThreads = 1024;
__global__ __launch_bounds__(kSelThreads) void learn_select_kernel(const double2 *__restrict__ A0, int64_t n,
                                                                   const double *__restrict__ amax, double prune,
                                                                   uint8_t *__restrict__ learned,
                                                                   int64_t *__restrict__ keep_idx,
                                                                   int64_t *__restrict__ new_idx,
                                                                   int64_t *__restrict__ counts) {
  __shared__ int wk[kSelThreads / 64], wn[kSelThreads / 64];
  const double thr = prune * *amax;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  int64_t ok = 0, on = 0;
  for (int64_t base = 0; base < n; base += kSelThreads) {
    const int64_t i = base + tid;
    const bool keep = i < n && hypot(A0[i].x, A0[i].y) > thr;
    const bool nw = keep && !learned[i];
    const uint64_t mk = __ballot(keep), mn = __ballot(nw);
    if (lane == 0) {
      wk[w] = __popcll(mk);
      wn[w] = __popcll(mn);
    }
    __syncthreads();
    int64_t pk = ok + __popcll(mk & below), pn = on + __popcll(mn & below);
    int64_t tk = 0, tn = 0;
    for (int x = 0; x < kSelThreads / 64; ++x) {
      if (x < w) {
        pk += wk[x];
        pn += wn[x];
      }
      tk += wk[x];
      tn += wn[x];
    }
    if (keep) keep_idx[pk] = i;
    if (nw) {
      new_idx[pn] = i;
      learned[i] = 1;
    }
    ok += tk;
    on += tn;
    __syncthreads();  // wk and wn are rewritten by the next round
  }
  if (tid == 0) {
    counts[0] = ok;
    counts[1] = on;
  }
}

__global__ void learn_start_kernel(int d, int64_t Nm, int64_t n, const int64_t *__restrict__ idx,
                                   const double *__restrict__ qm, const double *__restrict__ pm,
                                   double *__restrict__ Q, double *__restrict__ P, double *__restrict__ S,
                                   double2 *__restrict__ A) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t i = idx[j];
  for (int k = 0; k < d; ++k) {
    Q[k * n + j] = qm[k * Nm + i];
    P[k * n + j] = pm[k * Nm + i];
  }
  S[j] = 0.0;
  A[j] = make_double2(1.0, 0.0);
}

__global__ void learn_store_kernel(int d, int64_t Nm, int64_t n, const int64_t *__restrict__ idx,
                                   const double *__restrict__ Q, const double *__restrict__ P,
                                   const double *__restrict__ S, const double2 *__restrict__ A,
                                   double *__restrict__ Qf, double *__restrict__ Pf, double *__restrict__ Sf,
                                   double2 *__restrict__ ratio) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t i = idx[j];
  for (int k = 0; k < d; ++k) {
    Qf[k * Nm + i] = Q[k * n + j];
    Pf[k * Nm + i] = P[k * n + j];
  }
  Sf[i] = S[j];
  ratio[i] = A[j];
}

__global__ void learn_packets_kernel(int d, int64_t Nm, int64_t n, const int64_t *__restrict__ idx,
                                     const double *__restrict__ Qf, const double *__restrict__ Pf,
                                     const double *__restrict__ Sf, const double2 *__restrict__ ratio,
                                     const double2 *__restrict__ A0, double *__restrict__ Q,
                                     double *__restrict__ P, double *__restrict__ S, double2 *__restrict__ a) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t i = idx[j];
  for (int k = 0; k < d; ++k) {
    Q[k * n + j] = Qf[k * Nm + i];
    P[k * n + j] = Pf[k * Nm + i];
  }
  S[j] = Sf[i];
  const double2 x = A0[i], r = ratio[i];
  a[j] = make_double2(x.x * r.x - x.y * r.y, x.x * r.y + x.y * r.x);
}

unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + 255) / 256); }

}  // namespace

size_t learn_scratch_bytes() { return (kMaxBlocks + 4) * sizeof(double); }

void launch_learn_select(int64_t Nm, const double *A0, double prune, uint8_t *learned, int64_t *keep_idx,
                         int64_t *new_idx, double *scratch, int64_t *counts, hipStream_t s) {
  const int nb = (int)std::min<int64_t>(kMaxBlocks, (Nm + 255) / 256);
  double *part = scratch, *amax = scratch + kMaxBlocks;
  absmax_kernel<<<dim3((unsigned)std::max(nb, 1)), dim3(256), 0, s>>>((const double2 *)A0, Nm, part);
  FGGC_HIP(hipGetLastError());
  absmax_final_kernel<<<dim3(1), dim3(256), 0, s>>>(part, std::max(nb, 1), amax);
  FGGC_HIP(hipGetLastError());
  learn_select_kernel<<<dim3(1), dim3(kSelThreads), 0, s>>>((const double2 *)A0, Nm, amax, prune, learned,
                                                            keep_idx, new_idx, counts);
  FGGC_HIP(hipGetLastError());
}

void launch_learn_start(int d, int64_t Nm, int64_t n, const int64_t *idx, const double *qm, const double *pm,
                        double *Q, double *P, double *S, double *A, hipStream_t s) {
  if (n == 0) return;
  learn_start_kernel<<<dim3(blocks_for(n)), dim3(256), 0, s>>>(d, Nm, n, idx, qm, pm, Q, P, S, (double2 *)A);
  FGGC_HIP(hipGetLastError());
}

void launch_learn_store(int d, int64_t Nm, int64_t n, const int64_t *idx, const double *Q, const double *P,
                        const double *S, const double *A, double *Qf, double *Pf, double *Sf, double *ratio,
                        hipStream_t s) {
  if (n == 0) return;
  learn_store_kernel<<<dim3(blocks_for(n)), dim3(256), 0, s>>>(d, Nm, n, idx, Q, P, S, (const double2 *)A, Qf,
                                                               Pf, Sf, (double2 *)ratio);
  FGGC_HIP(hipGetLastError());
}

void launch_learn_packets(int d, int64_t Nm, int64_t n, const int64_t *idx, const double *Qf, const double *Pf,
                          const double *Sf, const double *ratio, const double *A0, double *Q, double *P,
                          double *S, double *a, hipStream_t s) {
  if (n == 0) return;
  learn_packets_kernel<<<dim3(blocks_for(n)), dim3(256), 0, s>>>(d, Nm, n, idx, Qf, Pf, Sf,
                                                                 (const double2 *)ratio, (const double2 *)A0, Q,
                                                                 P, S, (double2 *)a);
  FGGC_HIP(hipGetLastError());
}

}  // namespace fggc
