// Frozen Gaussian grid-point correction on gfx950 (Section 2.3, Alg. 2).
//
//   fggc_key      per packet: its own cell (int parts of eq. 3.6) -> bin keys
//                 (p-cell major, q-tile minor), one key slot per q-tile that
//                 its shifted neighbours reach; counting-sort positions of the
//                 slots (sort.hip).
//   fggc_coef     one thread per packet, in packet order, FP64: frac parts
//                 (3.7), right-hand side (3.23), least squares through the
//                 plan's eigenpairs (c^ = V diag(1/lambda) V^H f~), conjugation
//                 to the L2-best coefficients, shift (3.13); the per-dimension
//                 coefficients (the first times scale a exp(i S/eps)) are
//                 written as one record at the sorted position of every slot.
//   fggc_accum    owner-computes form of eq. (2.23)-(2.25): one workgroup per
//                 (window of p-slices, q-tile) of the dense cell array
//                 accumulates, in LDS, the Kronecker products of the packets in
//                 its tile's bins, then writes each of its cells once.
//   fft over q    forward DFT of every p-slice of the cell array (fft.hip).
//   band_mac      owner-computes over the grid spectrum: for each frequency
//                 k' of the M-point grid, the sum over slices l and aliases
//                 k = k' + jM of gamma_l(k) F_l[k mod Nq], where
//                 gamma_l(k) = prod_d sqrt(2 pi eps)/(2 pi) exp(-eps (k_d - p_l,d/eps)^2 / 2)
//                 is the Fourier coefficient of the periodised on-grid packet
//                 G(x; q, p_l) of eq. (2.16) with q = 0, truncated to
//                 |k_d - p_l,d/eps| <= cK / sqrt(eps); accumulated in FP64.
//   inverse fft   of the M^d spectrum gives eq. (2.24) on the grid.
#include <hipcub/hipcub.hpp>

#include <cmath>

#include "common.h"
#include "lds_fft.h"

namespace fggc {
namespace {

__device__ __forceinline__ void int_frac(double v, int64_t &i, double &f) {
  const double fl = floor(v);
  f = v - fl;
  i = (int64_t)fl;
  if (f >= 1.0) {  // a fraction that rounds to 1 moves to the next cell
    f = 0.0;
    i += 1;
  }
}

// unit complex number exp(2 pi i rev), argument reduced in revolutions first
__device__ __forceinline__ void cis_rev(double rev, double &c, double &s) {
  sincospi(2.0 * (rev - rint(rev)), &s, &c);
}

// (c + i s)^n for a small integer n (|z| = 1, so z^-1 = conj z)
__device__ __forceinline__ void cis_pow(double c, double s, int n, double &pc, double &ps) {
  double xr = 1.0, xi = 0.0;
  const int m = n < 0 ? -n : n;
  for (int k = 0; k < m; ++k) {
    const double t = xr * c - xi * s;
    xi = xr * s + xi * c;
    xr = t;
  }
  pc = xr;
  ps = n < 0 ? -xi : xi;
}

// per-dimension least-squares coefficients c_k (after conjugation and shift)
//
// With CC = Cq Cp, the right-hand side (3.23) factors as
//   f~_ab = gq_a gp_b E0 Es^dp_b Et^dq_a D_ab,
//   gq_a = exp(-Cq^2 (dq_a - s)^2 / 4), gp_b = exp(-Cp^2 (dp_b - t)^2 / 4),
//   E0 = exp(i CC s t / 2), Es = exp(i CC s / 2), Et = exp(-i CC t / 2),
//   D_ab = exp(-i CC dq_a dp_b / 2)  (a constant of the plan),
// and the shift of (3.13) as exp(-i CC (s - dq_a) ip) = F0 Fi^dq_a with
//   F0 = exp(-i CC s ip), Fi = exp(i CC ip).
template <int N1>
__device__ __forceinline__ void dim_coeffs(const DimLsq &L, double Q, double P, double dq, double dp,
                                           int64_t &iq, int64_t &ip, double cre[N1], double cim[N1]) {
  double s, t;
  int_frac(Q / dq, iq, s);
  int_frac(P / dp, ip, t);
  const double Cq = L.Cq, Cp = L.Cp, CC = Cq * Cp;
  const int n1 = L.n1;
  constexpr double inv2pi = 1.0 / kTwoPi;
  double e0c, e0s, esc, ess, etc_, ets, f0c, f0s, fic, fis;
  cis_rev(0.5 * CC * s * t * inv2pi, e0c, e0s);
  cis_rev(0.5 * CC * s * inv2pi, esc, ess);
  cis_rev(-0.5 * CC * t * inv2pi, etc_, ets);
  {
    const double w = CC * inv2pi * (double)ip;  // CC ip in revolutions
    cis_rev(w, fic, fis);
    cis_rev(-s * w, f0c, f0s);
  }
  double fre[N1], fim[N1];
#pragma unroll
  for (int j = 0; j < N1; ++j) {
    fre[j] = 0.0;
    fim[j] = 0.0;
    if (j < n1) {
      const double a = (double)L.dq[j] - s, b = (double)L.dp[j] - t;
      const double mag = exp(-0.25 * (Cq * Cq * a * a + Cp * Cp * b * b));
      double pr, pi, qr, qi;
      cis_pow(esc, ess, L.dp[j], pr, pi);
      cis_pow(etc_, ets, L.dq[j], qr, qi);
      // E0 * Es^dp * Et^dq * D
      double xr = e0c * pr - e0s * pi, xi = e0c * pi + e0s * pr;
      double yr = xr * qr - xi * qi, yi = xr * qi + xi * qr;
      const double dr = L.D[2 * j], di = L.D[2 * j + 1];
      xr = yr * dr - yi * di;
      xi = yr * di + yi * dr;
      fre[j] = mag * xr;
      fim[j] = mag * xi;
    }
  }
  // z = diag(inv) V^H f
  double zre[N1], zim[N1];
#pragma unroll
  for (int i = 0; i < N1; ++i) {
    double yr = 0.0, yi = 0.0;
#pragma unroll
    for (int j = 0; j < N1; ++j) {
      if (i < n1 && j < n1) {
        const double vr = L.V[2 * (j * n1 + i)], vi = L.V[2 * (j * n1 + i) + 1];
        // conj(V_ji) * f_j
        yr = fma(vr, fre[j], fma(vi, fim[j], yr));
        yi = fma(vr, fim[j], fma(-vi, fre[j], yi));
      }
    }
    const double w = i < n1 ? L.inv[i] : 0.0;
    zre[i] = yr * w;
    zim[i] = yi * w;
  }
  // c^ = V z ; c~ = conj(c^) ; c = c~ F0 Fi^dq
#pragma unroll
  for (int j = 0; j < N1; ++j) {
    double hr = 0.0, hi = 0.0;
#pragma unroll
    for (int i = 0; i < N1; ++i) {
      if (i < n1 && j < n1) {
        const double vr = L.V[2 * (j * n1 + i)], vi = L.V[2 * (j * n1 + i) + 1];
        hr = fma(vr, zre[i], fma(-vi, zim[i], hr));
        hi = fma(vr, zim[i], fma(vi, zre[i], hi));
      }
    }
    const double tr = hr, ti = -hi;  // conjugate
    double cs = 1.0, sn = 0.0;
    if (j < n1) {
      double pr, pi;
      cis_pow(fic, fis, L.dq[j], pr, pi);
      cs = f0c * pr - f0s * pi;
      sn = f0c * pi + f0s * pr;
    }
    cre[j] = tr * cs - ti * sn;
    cim[j] = tr * sn + ti * cs;
  }
}

// The same with the shift-set sizes fixed (basis j = a NP + b): the Gaussian
// factor splits as gq_a gp_b, and the powers Es^dp_b, Et^dq_a, Fi^dq_a are
// formed once per shift instead of once per basis function.
template <int NQ, int NP>
__device__ __forceinline__ void dim_coeffs_exact(const DimLsq &L, double Q, double P, double dq, double dp,
                                                 int64_t &iq, int64_t &ip, double *cre, double *cim) {
  constexpr int N1 = NQ * NP;
  double s, t;
  int_frac(Q / dq, iq, s);
  int_frac(P / dp, ip, t);
  const double Cq = L.Cq, Cp = L.Cp, CC = Cq * Cp;
  constexpr double inv2pi = 1.0 / kTwoPi;
  double e0c, e0s, esc, ess, etc_, ets, f0c, f0s, fic, fis;
  cis_rev(0.5 * CC * s * t * inv2pi, e0c, e0s);
  cis_rev(0.5 * CC * s * inv2pi, esc, ess);
  cis_rev(-0.5 * CC * t * inv2pi, etc_, ets);
  {
    const double w = CC * inv2pi * (double)ip;  // CC ip in revolutions
    cis_rev(w, fic, fis);
    cis_rev(-s * w, f0c, f0s);
  }
  double gq[NQ], qr[NQ], qi[NQ], hr[NQ], hi[NQ];
#pragma unroll
  for (int a = 0; a < NQ; ++a) {
    const int dqa = L.dq[a * NP];
    const double x = (double)dqa - s;
    gq[a] = exp(-0.25 * Cq * Cq * x * x);
    cis_pow(etc_, ets, dqa, qr[a], qi[a]);
    cis_pow(fic, fis, dqa, hr[a], hi[a]);
  }
  double gp[NP], pr[NP], pi[NP];
#pragma unroll
  for (int b = 0; b < NP; ++b) {
    const int dpb = L.dp[b];
    const double x = (double)dpb - t;
    gp[b] = exp(-0.25 * Cp * Cp * x * x);
    cis_pow(esc, ess, dpb, pr[b], pi[b]);
  }
  double fre[N1], fim[N1];
#pragma unroll
  for (int a = 0; a < NQ; ++a)
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      const int j = a * NP + b;
      // E0 * Es^dp * Et^dq * D, times gq gp
      double xr = e0c * pr[b] - e0s * pi[b], xi = e0c * pi[b] + e0s * pr[b];
      const double yr = xr * qr[a] - xi * qi[a], yi = xr * qi[a] + xi * qr[a];
      const double dr = L.D[2 * j], di = L.D[2 * j + 1];
      const double mag = gq[a] * gp[b];
      fre[j] = mag * (yr * dr - yi * di);
      fim[j] = mag * (yr * di + yi * dr);
    }
  double zre[N1], zim[N1];
#pragma unroll
  for (int i = 0; i < N1; ++i) {
    double yr = 0.0, yi = 0.0;
#pragma unroll
    for (int j = 0; j < N1; ++j) {
      const double vr = L.V[2 * (j * N1 + i)], vi = L.V[2 * (j * N1 + i) + 1];
      yr = fma(vr, fre[j], fma(vi, fim[j], yr));
      yi = fma(vr, fim[j], fma(-vi, fre[j], yi));
    }
    zre[i] = yr * L.inv[i];
    zim[i] = yi * L.inv[i];
  }
#pragma unroll
  for (int j = 0; j < N1; ++j) {
    double gr = 0.0, gi = 0.0;
#pragma unroll
    for (int i = 0; i < N1; ++i) {
      const double vr = L.V[2 * (j * N1 + i)], vi = L.V[2 * (j * N1 + i) + 1];
      gr = fma(vr, zre[i], fma(-vi, zim[i], gr));
      gi = fma(vr, zim[i], fma(vi, zre[i], gi));
    }
    const double tr = gr, ti = -gi;  // conjugate
    const int a = j / NP;
    const double cs = f0c * hr[a] - f0s * hi[a], sn = f0c * hi[a] + f0s * hr[a];
    cre[j] = tr * cs - ti * sn;
    cim[j] = tr * sn + ti * cs;
  }
}

// Sort keys of a packet: its own p-cell (relative to the box of packet
// p-cells) major, a q-tile minor -- one key slot for every q-tile its
// neighbours [q + mindq, q + maxdq] reach (at most two per dimension, as a
// tile is at least as wide as the shift set), so that a workgroup owning a
// tile finds every packet that touches it in that tile's own bins.
struct KeyParams {
  int64_t N;
  const double *Q, *P;
  int64_t Nq[3], pmin[3], npc[3], tile[3], ntq[3];
  double dq[3], dp[3];
  int mindq, maxdq;
  int ns;  // key slots per packet: 2^d with halo slots, 1 for the own tile only
};

// The key slots of packet j (kNoKey for unused halo slots).  The rank kernel,
// the key kernel and the coefficient kernel all call this, so their keys agree
// bit for bit.
template <int D>
__device__ __forceinline__ void packet_keys(const KeyParams &p, int64_t j, uint32_t *key) {
  int64_t pcf = 0, nqt = 1, ta[3], tb[3];
  for (int k = 0; k < D; ++k) {
    int64_t iq, ip;
    double s, t;
    int_frac(p.Q[k * p.N + j] / p.dq[k], iq, s);
    int_frac(p.P[k * p.N + j] / p.dp[k], ip, t);
    const int64_t msk = p.Nq[k] - 1;
    const int64_t qi = (iq + p.Nq[k] / 2) & msk;
    // the cell box comes from the same floor(P/dp), so this clamp never binds;
    // it keeps every key inside [0, nbins) whatever the caller's box
    int64_t pc = ip - p.pmin[k];
    pc = pc < 0 ? 0 : (pc >= p.npc[k] ? p.npc[k] - 1 : pc);
    pcf = pcf * p.npc[k] + pc;
    if (p.ns == 1) {
      ta[k] = tb[k] = qi / p.tile[k];
    } else {
      ta[k] = ((qi + p.mindq) & msk) / p.tile[k];
      tb[k] = ((qi + p.maxdq) & msk) / p.tile[k];
    }
    nqt *= p.ntq[k];
  }
  if (p.ns == 1) {
    int64_t tf = 0;
    for (int k = 0; k < D; ++k) tf = tf * p.ntq[k] + ta[k];
    key[0] = (uint32_t)(pcf * nqt + tf);
    return;
  }
  constexpr int NS = 1 << D;
#pragma unroll
  for (int m = 0; m < NS; ++m) {
    bool ok = true;
    int64_t tf = 0;
    for (int k = 0; k < D; ++k) {
      const int bit = (m >> k) & 1;
      if (bit && tb[k] == ta[k]) ok = false;
      tf = tf * p.ntq[k] + (bit ? tb[k] : ta[k]);
    }
    key[m] = ok ? (uint32_t)(pcf * nqt + tf) : kNoKey;
  }
}

template <int D>
__global__ void fggc_key_kernel(KeyParams p, uint32_t *__restrict__ key) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= p.N) return;
  uint32_t k[1 << D];
  packet_keys<D>(p, j, k);
  for (int m = 0; m < p.ns; ++m) key[j * p.ns + m] = k[m];
}

// Counting pass of the LDS counting sort with the keys computed in place:
// workgroup g counts the key slots of its chunk of packets in LDS, keeping
// each slot's returned count as its rank inside (key, chunk), writes the
// counts bin-major into table[bin * G + g] and the keys for the position pass.
template <int D>
__global__ __launch_bounds__(1024) void fggc_rank_kernel(KeyParams p, int64_t chunk, int64_t nbins, int G,
                                                         uint32_t *__restrict__ table,
                                                         uint32_t *__restrict__ rank,
                                                         uint32_t *__restrict__ keys) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  uint32_t *cnt = reinterpret_cast<uint32_t *>(smem_raw);
  for (int64_t b = threadIdx.x; b < nbins; b += blockDim.x) cnt[b] = 0;
  __syncthreads();
  const int64_t j0 = blockIdx.x * chunk / p.ns, j1 = min(p.N, (blockIdx.x + 1) * chunk / p.ns);
  for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
    uint32_t k[1 << D];
    packet_keys<D>(p, j, k);
    for (int m = 0; m < p.ns; ++m) {
      keys[j * p.ns + m] = k[m];
      if (k[m] != kNoKey) rank[j * p.ns + m] = atomicAdd(&cnt[k[m]], 1u);
    }
  }
  __syncthreads();
  for (int64_t b = threadIdx.x; b < nbins; b += blockDim.x) table[b * G + blockIdx.x] = cnt[b];
}

// Record of one packet (one per key slot, in bin order): its q index and p-cell (relative) per
// dimension, then the per-dimension least-squares coefficients c_d[a*np+b]
// (after conjugation and shift), the first dimension's multiplied by
// scale * a exp(i S / eps).
template <int D> struct RecIdx { int32_t q[D], pc[D]; };
template <int D> __host__ __device__ constexpr int rec_idx_bytes() { return 16 * ((8 * D + 15) / 16); }
template <int D, int N1, typename T> __host__ __device__ constexpr int rec_bytes() {
  return rec_idx_bytes<D>() + D * N1 * (int)sizeof(T);
}

struct CoefParams {
  int ns;  // key slots per packet
  int64_t N;
  const double *Q, *P, *S, *a;
  double eps, scale;
  const DimLsq *lsq;  // [d], device copy of the plan
  int64_t Nq[3], pmin[3];
  double dq[3], dp[3];
};

// One thread per packet, in packet order (coalesced reads); the record is
// written to the sorted position of each of the packet's key slots.
template <int D, int N1, int NQ, int NP, typename T>
__global__ __launch_bounds__(256) void fggc_coef_kernel(CoefParams p, const uint32_t *__restrict__ pos,
                                                        char *__restrict__ recs) {
  using R = decltype(T{}.x);
  // one dimension: the plan is staged in LDS and read as broadcasts instead of
  // held in scalar registers (which the eigenvector matrix overflows); with
  // more dimensions the scalar path measured faster
  __shared__ DimLsq sl[1];
  if constexpr (D == 1) {
    const uint4 *src = reinterpret_cast<const uint4 *>(p.lsq);
    uint4 *dst = reinterpret_cast<uint4 *>(sl);
    for (int e = threadIdx.x; e < (int)(sizeof(DimLsq) / 16); e += blockDim.x) dst[e] = src[e];
    __syncthreads();
  }
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= p.N) return;
  double cre[D][N1], cim[D][N1];
  int64_t iq[D], ip[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const double qv = p.Q[k * p.N + j], pv = p.P[k * p.N + j];
    if constexpr (NQ > 0) {
      if constexpr (D == 1)
        dim_coeffs_exact<NQ, NP>(sl[0], qv, pv, p.dq[k], p.dp[k], iq[k], ip[k], cre[k], cim[k]);
      else
        dim_coeffs_exact<NQ, NP>(p.lsq[k], qv, pv, p.dq[k], p.dp[k], iq[k], ip[k], cre[k], cim[k]);
    } else {
      if constexpr (D == 1)
        dim_coeffs<N1>(sl[0], qv, pv, p.dq[k], p.dp[k], iq[k], ip[k], cre[k], cim[k]);
      else
        dim_coeffs<N1>(p.lsq[k], qv, pv, p.dq[k], p.dp[k], iq[k], ip[k], cre[k], cim[k]);
    }
  }
  double sn, cs;
  {
    const double rev = p.S[j] / (kTwoPi * p.eps);
    sincospi(2.0 * (rev - rint(rev)), &sn, &cs);
  }
  const double ar = p.scale * p.a[2 * j], ai = p.scale * p.a[2 * j + 1];
  const double alr = ar * cs - ai * sn, ali = ar * sn + ai * cs;
  RecIdx<D> ri;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    ri.q[k] = (int32_t)((iq[k] + p.Nq[k] / 2) & (p.Nq[k] - 1));
    ri.pc[k] = (int32_t)(ip[k] - p.pmin[k]);
  }
  T cv[D][N1];
#pragma unroll
  for (int k = 0; k < D; ++k)
#pragma unroll
    for (int m = 0; m < N1; ++m) {
      double xr = cre[k][m], xi = cim[k][m];
      if (k == 0) {
        const double nr = alr * xr - ali * xi;
        xi = alr * xi + ali * xr;
        xr = nr;
      }
      cv[k][m] = T{(R)xr, (R)xi};
    }
  constexpr int NS = 1 << D;
#pragma unroll
  for (int m = 0; m < NS; ++m) {
    if (m >= p.ns) break;
    const uint32_t at = pos[j * p.ns + m];
    if (at == kNoKey) continue;
    char *r = recs + (int64_t)at * rec_bytes<D, N1, T>();
    *reinterpret_cast<RecIdx<D> *>(r) = ri;
    T *c = reinterpret_cast<T *>(r + rec_idx_bytes<D>());
#pragma unroll
    for (int k = 0; k < D; ++k)
#pragma unroll
      for (int n = 0; n < N1; ++n) c[k * N1 + n] = cv[k][n];
  }
}

// Owner-computes accumulation of eq. (2.25): one workgroup per (window of
// S slices per dimension, q-tile) of the cell array holds those cells in LDS,
// adds the contributions of the packets in the bins of its own tile (halo
// packets are binned into every tile they touch) for the p-cells that reach
// its slices, and writes each of its cells exactly once (no zeroing pass, no
// global atomics).
struct AccParams {
  const char *recs;
  const int64_t *start;
  int64_t sn[3], npc[3], Nq[3], tile[3], ntq[3], S[3], nsw[3];
  int nq, np;
  int dq[8], dp[8];
  int mindp, maxdp;
};

template <int D, int N1, typename T>
__global__ __launch_bounds__(256) void fggc_accum_generic_kernel(AccParams p, T *__restrict__ cells) {
  using R = decltype(T{}.x);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R *lre = reinterpret_cast<R *>(smem_raw);
  int64_t tq_cells = 1, sw_cells = 1, nqt_all = 1, ncell_q = 1;
  for (int k = 0; k < D; ++k) {
    tq_cells *= p.tile[k];
    sw_cells *= p.S[k];
    nqt_all *= p.ntq[k];
    ncell_q *= p.Nq[k];
  }
  const int64_t tcells = tq_cells * sw_cells;
  R *lim = lre + tcells;
  for (int64_t e = threadIdx.x; e < tcells; e += blockDim.x) {
    lre[e] = 0;
    lim[e] = 0;
  }
  // this workgroup's q-tile (minor) and slice window (major)
  int64_t blk = blockIdx.x, tq[3] = {0, 0, 0}, w[3] = {0, 0, 0};
  for (int k = D - 1; k >= 0; --k) {
    tq[k] = blk % p.ntq[k];
    blk /= p.ntq[k];
  }
  for (int k = D - 1; k >= 0; --k) {
    w[k] = blk % p.nsw[k];
    blk /= p.nsw[k];
  }
  // slices [s0, s1) per dimension; packet p-cells reaching them: slice =
  // pc + dp - mindp, so pc in [s0 - (maxdp - mindp), s1 - 1]
  int64_t s0[3], s1[3], pc0[3], pcn[3];
  bool any = true;
  for (int k = 0; k < 3; ++k) {
    s0[k] = 0;
    s1[k] = 1;
    pc0[k] = 0;
    pcn[k] = 1;
  }
  for (int k = 0; k < D; ++k) {
    s0[k] = w[k] * p.S[k];
    s1[k] = min(s0[k] + p.S[k], p.sn[k]);
    int64_t a = s0[k] - (p.maxdp - p.mindp), b = s1[k] - 1;
    if (a < 0) a = 0;
    if (b > p.npc[k] - 1) b = p.npc[k] - 1;
    pc0[k] = a;
    pcn[k] = b - a + 1;
    any = any && pcn[k] > 0;
  }
  int64_t tflat = 0;
  for (int k = 0; k < D; ++k) tflat = tflat * p.ntq[k] + tq[k];
  __syncthreads();
  if (any) {
    int64_t npcs = 1;
    for (int k = 0; k < D; ++k) npcs *= pcn[k];
    constexpr int RB = rec_bytes<D, N1, T>();
    for (int64_t pcv = 0; pcv < npcs; ++pcv) {
      int64_t rem = pcv, pcf = 0, pcs[3] = {0, 0, 0};
      for (int k = D - 1; k >= 0; --k) {
        pcs[k] = pc0[k] + rem % pcn[k];
        rem /= pcn[k];
      }
      for (int k = 0; k < D; ++k) pcf = pcf * p.npc[k] + pcs[k];
      // local slice of basis index b in each dimension, or -1 outside the window
      int ls[3][8];
      for (int k = 0; k < D; ++k)
        for (int b = 0; b < 8; ++b) {
          ls[k][b] = -1;
          if (b < p.np) {
            const int64_t sl = pcs[k] + p.dp[b] - p.mindp;
            if (sl >= s0[k] && sl < s1[k]) ls[k][b] = (int)(sl - s0[k]);
          }
        }
      const int64_t bin = pcf * nqt_all + tflat;
      const int64_t r0 = p.start[bin], r1 = p.start[bin + 1];
      for (int64_t r = r0 + threadIdx.x; r < r1; r += blockDim.x) {
        const char *rec = p.recs + r * (int64_t)RB;
        const RecIdx<D> ri = *reinterpret_cast<const RecIdx<D> *>(rec);
        const T *c = reinterpret_cast<const T *>(rec + rec_idx_bytes<D>());
        // local q offsets of this packet's neighbours inside the tile, or -1
        int lq[3][8];
        for (int k = 0; k < D; ++k)
          for (int a = 0; a < 8; ++a) {
            lq[k][a] = -1;
            if (a < p.nq) {
              const int64_t qv = (ri.q[k] + p.dq[a] - tq[k] * p.tile[k]) & (p.Nq[k] - 1);
              if (qv < p.tile[k]) lq[k][a] = (int)qv;
            }
          }
        if (D == 1) {
          for (int b0 = 0; b0 < p.np; ++b0) {
            if (ls[0][b0] < 0) continue;
            const int64_t sb = ls[0][b0] * p.tile[0];
            for (int a0 = 0; a0 < p.nq; ++a0) {
              if (lq[0][a0] < 0) continue;
              const T v = c[a0 * p.np + b0];
              atomicAdd(&lre[sb + lq[0][a0]], v.x);
              atomicAdd(&lim[sb + lq[0][a0]], v.y);
            }
          }
        } else if (D == 2) {
          for (int b0 = 0; b0 < p.np; ++b0) {
            if (ls[0][b0] < 0) continue;
            for (int b1 = 0; b1 < p.np; ++b1) {
              if (ls[1][b1] < 0) continue;
              const int64_t sb = (ls[0][b0] * p.S[1] + ls[1][b1]) * tq_cells;
              for (int a0 = 0; a0 < p.nq; ++a0) {
                if (lq[0][a0] < 0) continue;
                const T u = c[a0 * p.np + b0];
                for (int a1 = 0; a1 < p.nq; ++a1) {
                  if (lq[1][a1] < 0) continue;
                  const T v = c[N1 + a1 * p.np + b1];
                  const int64_t li = sb + lq[0][a0] * p.tile[1] + lq[1][a1];
                  atomicAdd(&lre[li], u.x * v.x - u.y * v.y);
                  atomicAdd(&lim[li], u.x * v.y + u.y * v.x);
                }
              }
            }
          }
        } else {
          for (int b0 = 0; b0 < p.np; ++b0) {
            if (ls[0][b0] < 0) continue;
            for (int b1 = 0; b1 < p.np; ++b1) {
              if (ls[1][b1] < 0) continue;
              for (int b2 = 0; b2 < p.np; ++b2) {
                if (ls[2][b2] < 0) continue;
                const int64_t sb = ((ls[0][b0] * p.S[1] + ls[1][b1]) * p.S[2] + ls[2][b2]) * tq_cells;
                for (int a0 = 0; a0 < p.nq; ++a0) {
                  if (lq[0][a0] < 0) continue;
                  const T u = c[a0 * p.np + b0];
                  for (int a1 = 0; a1 < p.nq; ++a1) {
                    if (lq[1][a1] < 0) continue;
                    const T v1 = c[N1 + a1 * p.np + b1];
                    const R ur = u.x * v1.x - u.y * v1.y, ui = u.x * v1.y + u.y * v1.x;
                    for (int a2 = 0; a2 < p.nq; ++a2) {
                      if (lq[2][a2] < 0) continue;
                      const T v2 = c[2 * N1 + a2 * p.np + b2];
                      const int64_t li = sb + (lq[0][a0] * p.tile[1] + lq[1][a1]) * p.tile[2] + lq[2][a2];
                      atomicAdd(&lre[li], ur * v2.x - ui * v2.y);
                      atomicAdd(&lim[li], ur * v2.y + ui * v2.x);
                    }
                  }
                }
              }
            }
          }
        }
      }
    }
  }
  __syncthreads();
  // write the window: every cell of the array is owned by exactly one workgroup
  for (int64_t e = threadIdx.x; e < tcells; e += blockDim.x) {
    int64_t rem = e, lqv[3] = {0, 0, 0}, lsv[3] = {0, 0, 0};
    for (int k = D - 1; k >= 0; --k) {
      lqv[k] = rem % p.tile[k];
      rem /= p.tile[k];
    }
    for (int k = D - 1; k >= 0; --k) {
      lsv[k] = rem % p.S[k];
      rem /= p.S[k];
    }
    bool in = true;
    int64_t slf = 0, q = 0;
    for (int k = 0; k < D; ++k) {
      const int64_t sl = s0[k] + lsv[k];
      in = in && sl < s1[k];
      slf = slf * p.sn[k] + sl;
      q = q * p.Nq[k] + tq[k] * p.tile[k] + lqv[k];
    }
    if (in) cells[slf * ncell_q + q] = T{lre[e], lim[e]};
  }
}

// The same accumulation with the shift-set sizes fixed at compile time (the
// tensor strategies Q2P2, Q4P2, Q2P4, Q4P4): every loop over shifts is
// unrolled, each record is loaded once with 16-byte loads into registers, and
// the records of all the workgroup's bins form one index space, so that every
// lane has work and the loads of two records are in flight together.
constexpr int kMaxBinsPerPass = 64;

template <int D, int NQ, int NP, typename T>
__device__ __forceinline__ void add_record(const uint4 *__restrict__ src, const AccParams &p,
                                           const int *s0, const int *sw, const int *tq0,
                                           int tile1, int tile2, int tq_cells,
                                           decltype(T{}.x) *lre, decltype(T{}.x) *lim) {
  using R = decltype(T{}.x);
  constexpr int N1 = NQ * NP;
  constexpr int RB = rec_bytes<D, N1, T>();
  constexpr int NV = RB / 16;
  uint4 raw[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) raw[v] = src[v];
  const RecIdx<D> ri = *reinterpret_cast<const RecIdx<D> *>(raw);
  const T *c = reinterpret_cast<const T *>(reinterpret_cast<const char *>(raw) + rec_idx_bytes<D>());
  int lq[D][NQ], ls[D][NP];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    const int msk = (int)p.Nq[k] - 1, tl = (int)p.tile[k];
#pragma unroll
    for (int a = 0; a < NQ; ++a) {
      const int qv = (ri.q[k] + p.dq[a] - tq0[k]) & msk;
      lq[k][a] = qv < tl ? qv : -1;
    }
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      const int sl = ri.pc[k] + p.dp[b] - p.mindp - s0[k];
      ls[k][b] = (sl >= 0 && sl < sw[k]) ? sl : -1;
    }
  }
  if constexpr (D == 1) {
#pragma unroll
    for (int b = 0; b < NP; ++b)
#pragma unroll
      for (int a = 0; a < NQ; ++a)
        if (ls[0][b] >= 0 && lq[0][a] >= 0) {
          const int li = ls[0][b] * (int)p.tile[0] + lq[0][a];
          const T v = c[a * NP + b];
          atomicAdd(&lre[li], v.x);
          atomicAdd(&lim[li], v.y);
        }
  } else if constexpr (D == 2) {
#pragma unroll
    for (int b0 = 0; b0 < NP; ++b0)
#pragma unroll
      for (int b1 = 0; b1 < NP; ++b1) {
        if (ls[0][b0] < 0 || ls[1][b1] < 0) continue;
        const int sb = (ls[0][b0] * (int)p.S[1] + ls[1][b1]) * tq_cells;
#pragma unroll
        for (int a0 = 0; a0 < NQ; ++a0) {
          const T u = c[a0 * NP + b0];
#pragma unroll
          for (int a1 = 0; a1 < NQ; ++a1)
            if (lq[0][a0] >= 0 && lq[1][a1] >= 0) {
              const T v = c[N1 + a1 * NP + b1];
              const int li = sb + lq[0][a0] * tile1 + lq[1][a1];
              atomicAdd(&lre[li], u.x * v.x - u.y * v.y);
              atomicAdd(&lim[li], u.x * v.y + u.y * v.x);
            }
        }
      }
  } else {
#pragma unroll
    for (int b0 = 0; b0 < NP; ++b0)
#pragma unroll
      for (int b1 = 0; b1 < NP; ++b1)
#pragma unroll
        for (int b2 = 0; b2 < NP; ++b2) {
          if (ls[0][b0] < 0 || ls[1][b1] < 0 || ls[2][b2] < 0) continue;
          const int sb = ((ls[0][b0] * (int)p.S[1] + ls[1][b1]) * (int)p.S[2] + ls[2][b2]) * tq_cells;
#pragma unroll
          for (int a0 = 0; a0 < NQ; ++a0) {
            const T u = c[a0 * NP + b0];
#pragma unroll
            for (int a1 = 0; a1 < NQ; ++a1) {
              const T v1 = c[N1 + a1 * NP + b1];
              const R ur = u.x * v1.x - u.y * v1.y, ui = u.x * v1.y + u.y * v1.x;
#pragma unroll
              for (int a2 = 0; a2 < NQ; ++a2)
                if (lq[0][a0] >= 0 && lq[1][a1] >= 0 && lq[2][a2] >= 0) {
                  const T v2 = c[2 * N1 + a2 * NP + b2];
                  const int li = sb + (lq[0][a0] * tile1 + lq[1][a1]) * tile2 + lq[2][a2];
                  atomicAdd(&lre[li], ur * v2.x - ui * v2.y);
                  atomicAdd(&lim[li], ur * v2.y + ui * v2.x);
                }
            }
          }
        }
  }
}

template <int D, int NQ, int NP, typename T>
__global__ __launch_bounds__(256) void fggc_accum_kernel(AccParams p, T *__restrict__ cells) {
  using R = decltype(T{}.x);
  constexpr int RB = rec_bytes<D, NQ * NP, T>();
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int64_t s_r0[kMaxBinsPerPass], s_pre[kMaxBinsPerPass + 1];
  R *lre = reinterpret_cast<R *>(smem_raw);
  int tq_cells = 1, sw_cells = 1;
  int64_t nqt_all = 1, ncell_q = 1;
  for (int k = 0; k < D; ++k) {
    tq_cells *= (int)p.tile[k];
    sw_cells *= (int)p.S[k];
    nqt_all *= p.ntq[k];
    ncell_q *= p.Nq[k];
  }
  const int tcells = tq_cells * sw_cells;
  R *lim = lre + tcells;
  for (int e = threadIdx.x; e < tcells; e += blockDim.x) {
    lre[e] = 0;
    lim[e] = 0;
  }
  int64_t blk = blockIdx.x;
  int tq[3] = {0, 0, 0}, s0[3] = {0, 0, 0}, sw[3] = {1, 1, 1}, tq0[3] = {0, 0, 0};
  int64_t w[3] = {0, 0, 0}, pc0[3] = {0, 0, 0}, pcn[3] = {1, 1, 1};
  for (int k = D - 1; k >= 0; --k) {
    tq[k] = (int)(blk % p.ntq[k]);
    blk /= p.ntq[k];
  }
  for (int k = D - 1; k >= 0; --k) {
    w[k] = blk % p.nsw[k];
    blk /= p.nsw[k];
  }
  bool any = true;
  for (int k = 0; k < D; ++k) {
    s0[k] = (int)(w[k] * p.S[k]);
    sw[k] = (int)min(p.S[k], p.sn[k] - s0[k]);
    tq0[k] = tq[k] * (int)p.tile[k];
    int64_t a = s0[k] - (p.maxdp - p.mindp), b = s0[k] + sw[k] - 1;
    if (a < 0) a = 0;
    if (b > p.npc[k] - 1) b = p.npc[k] - 1;
    pc0[k] = a;
    pcn[k] = b - a + 1;
    any = any && pcn[k] > 0;
  }
  int64_t tflat = 0;
  for (int k = 0; k < D; ++k) tflat = tflat * p.ntq[k] + tq[k];
  const int tile1 = D > 1 ? (int)p.tile[1] : 1, tile2 = D > 2 ? (int)p.tile[2] : 1;
  int64_t npcs = 1;
  for (int k = 0; k < D; ++k) npcs *= pcn[k];
  if (!any) npcs = 0;
  __syncthreads();
  for (int64_t bb = 0; bb < npcs; bb += kMaxBinsPerPass) {
    const int nb = (int)min<int64_t>(kMaxBinsPerPass, npcs - bb);
    if ((int)threadIdx.x < nb) {
      int64_t rem = bb + threadIdx.x, pcf = 0, pcs[3] = {0, 0, 0};
      for (int k = D - 1; k >= 0; --k) {
        pcs[k] = pc0[k] + rem % pcn[k];
        rem /= pcn[k];
      }
      for (int k = 0; k < D; ++k) pcf = pcf * p.npc[k] + pcs[k];
      const int64_t bin = pcf * nqt_all + tflat;
      s_r0[threadIdx.x] = p.start[bin];
      s_pre[threadIdx.x + 1] = p.start[bin + 1] - p.start[bin];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      s_pre[0] = 0;
      for (int i = 1; i <= nb; ++i) s_pre[i] += s_pre[i - 1];
    }
    __syncthreads();
    const int64_t total = s_pre[nb];
    // consecutive records of a bin often come from one packet-mesh point and
    // hit the same cells: spread the lanes of a wave over the bin with a
    // stride coprime to the record count, so that their LDS atomics rarely
    // collide on one address
    int64_t stride = 1;
    if (total > 64) {
      const int64_t cand[6] = {97, 89, 83, 79, 73, 71};
      for (int c = 0; c < 6; ++c) {
        int64_t x = total, y = cand[c];
        while (y) {
          const int64_t t = x % y;
          x = y;
          y = t;
        }
        if (x == 1) {
          stride = cand[c];
          break;
        }
      }
    }
    auto rec_of = [&](int64_t i0) {
      const int64_t i = (i0 * stride) % total;
      int lo = 0, hi = nb - 1;  // last bin with s_pre[bin] <= i
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_pre[mid] <= i) lo = mid;
        else hi = mid - 1;
      }
      return reinterpret_cast<const uint4 *>(p.recs + (s_r0[lo] + (i - s_pre[lo])) * (int64_t)RB);
    };
    for (int64_t i = threadIdx.x; i < total; i += 2 * (int64_t)blockDim.x) {
      const int64_t i2 = i + blockDim.x;
      const uint4 *ra = rec_of(i);
      const uint4 *rb = i2 < total ? rec_of(i2) : ra;
      add_record<D, NQ, NP, T>(ra, p, s0, sw, tq0, tile1, tile2, tq_cells, lre, lim);
      if (i2 < total) add_record<D, NQ, NP, T>(rb, p, s0, sw, tq0, tile1, tile2, tq_cells, lre, lim);
    }
    __syncthreads();
  }
  // write the window: every cell of the array is owned by exactly one workgroup
  for (int e = threadIdx.x; e < tcells; e += blockDim.x) {
    int rem = e, lqv[3] = {0, 0, 0}, lsv[3] = {0, 0, 0};
    for (int k = D - 1; k >= 0; --k) {
      lqv[k] = rem % (int)p.tile[k];
      rem /= (int)p.tile[k];
    }
    for (int k = D - 1; k >= 0; --k) {
      lsv[k] = rem % (int)p.S[k];
      rem /= (int)p.S[k];
    }
    bool in = true;
    int64_t slf = 0, q = 0;
    for (int k = 0; k < D; ++k) {
      in = in && lsv[k] < sw[k];
      slf = slf * p.sn[k] + s0[k] + lsv[k];
      q = q * p.Nq[k] + tq0[k] + lqv[k];
    }
    if (in) cells[slf * ncell_q + q] = T{lre[e], lim[e]};
  }
}

// Accumulation without atomics (d = 1, 2): one wave per (slice, q-tile); the
// tile lives in LDS as interleaved complex values and is updated with plain
// read-modify-writes.  Two lanes can hit the same cell in one instruction only
// when their records share (p-cell, q-cell); before adding, lanes claim an LDS
// hash slot of that key and only the lane that holds its slot adds in this
// pass, the others in later passes -- so each pass writes distinct cells.
constexpr int kHashSlots = 256;

template <int D, int NQ, int NP, typename T>
__global__ __launch_bounds__(64) void fggc_accum_wave_kernel(AccParams p, T *__restrict__ cells) {
  using R = decltype(T{}.x);
  constexpr int N1 = NQ * NP;
  constexpr int RB = rec_bytes<D, N1, T>();
  constexpr int NV = RB / 16;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ int64_t s_r0[kMaxBinsPerPass], s_pre[kMaxBinsPerPass + 1];
  __shared__ int s_claim[kHashSlots];
  T *tile = reinterpret_cast<T *>(smem_raw);
  const int lane = threadIdx.x;
  int tq_cells = 1;
  int64_t nqt_all = 1, ncell_q = 1;
  for (int k = 0; k < D; ++k) {
    tq_cells *= (int)p.tile[k];
    nqt_all *= p.ntq[k];
    ncell_q *= p.Nq[k];
  }
  for (int e = lane; e < tq_cells; e += 64) tile[e] = T{0, 0};
  int64_t blk = blockIdx.x;
  int tq0[3] = {0, 0, 0}, tq[3] = {0, 0, 0};
  int64_t sl[3] = {0, 0, 0}, pc0[3] = {0, 0, 0}, pcn[3] = {1, 1, 1};
  for (int k = D - 1; k >= 0; --k) {
    tq[k] = (int)(blk % p.ntq[k]);
    blk /= p.ntq[k];
  }
  for (int k = D - 1; k >= 0; --k) {
    sl[k] = blk % p.sn[k];
    blk /= p.sn[k];
  }
  bool any = true;
  for (int k = 0; k < D; ++k) {
    tq0[k] = tq[k] * (int)p.tile[k];
    int64_t a = sl[k] - (p.maxdp - p.mindp), b = sl[k];
    if (a < 0) a = 0;
    if (b > p.npc[k] - 1) b = p.npc[k] - 1;
    pc0[k] = a;
    pcn[k] = b - a + 1;
    any = any && pcn[k] > 0;
  }
  int64_t tflat = 0;
  for (int k = 0; k < D; ++k) tflat = tflat * p.ntq[k] + tq[k];
  int64_t npcs = 1;
  for (int k = 0; k < D; ++k) npcs *= pcn[k];
  if (!any) npcs = 0;
  const int tile1 = D > 1 ? (int)p.tile[1] : 1;
  __syncthreads();
  for (int64_t bb = 0; bb < npcs; bb += kMaxBinsPerPass) {
    const int nb = (int)min<int64_t>(kMaxBinsPerPass, npcs - bb);
    for (int t = lane; t < nb; t += 64) {
      int64_t rem = bb + t, pcf = 0, pcs[3] = {0, 0, 0};
      for (int k = D - 1; k >= 0; --k) {
        pcs[k] = pc0[k] + rem % pcn[k];
        rem /= pcn[k];
      }
      for (int k = 0; k < D; ++k) pcf = pcf * p.npc[k] + pcs[k];
      const int64_t bin = pcf * nqt_all + tflat;
      s_r0[t] = p.start[bin];
      s_pre[t + 1] = p.start[bin + 1] - p.start[bin];
    }
    __syncthreads();
    if (lane == 0) {
      s_pre[0] = 0;
      for (int i = 1; i <= nb; ++i) s_pre[i] += s_pre[i - 1];
    }
    __syncthreads();
    const int64_t total = s_pre[nb];
    for (int64_t base = 0; base < total; base += 64) {
      const int64_t i = base + lane;
      const bool valid = i < total;
      uint4 raw[NV];
      if (valid) {
        int lo = 0, hi = nb - 1;  // last bin with s_pre[bin] <= i
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_pre[mid] <= i) lo = mid;
          else hi = mid - 1;
        }
        const uint4 *src = reinterpret_cast<const uint4 *>(p.recs + (s_r0[lo] + (i - s_pre[lo])) * (int64_t)RB);
#pragma unroll
        for (int v = 0; v < NV; ++v) raw[v] = src[v];
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) raw[v] = make_uint4(0, 0, 0, 0);
      }
      const RecIdx<D> ri = *reinterpret_cast<const RecIdx<D> *>(raw);
      const T *c = reinterpret_cast<const T *>(reinterpret_cast<const char *>(raw) + rec_idx_bytes<D>());
      int lq[D][NQ];
      bool okb[D][NP];
      uint32_t h = 0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const int msk = (int)p.Nq[k] - 1, tl = (int)p.tile[k];
#pragma unroll
        for (int a = 0; a < NQ; ++a) {
          const int qv = (ri.q[k] + p.dq[a] - tq0[k]) & msk;
          lq[k][a] = qv < tl ? qv : -1;
        }
#pragma unroll
        for (int b = 0; b < NP; ++b) okb[k][b] = (int64_t)ri.pc[k] + p.dp[b] - p.mindp == sl[k];
        h = h * 0x9E3779B1u + (uint32_t)ri.q[k] * 0x85EBCA77u + (uint32_t)ri.pc[k] * 0xC2B2AE3Du;
      }
      h = (h ^ (h >> 15)) & (kHashSlots - 1);
      // passes: the loop condition is wave-uniform; the barriers (a single
      // wave here) order the claims and the cell updates between lanes
      volatile int *claim = s_claim;
      bool todo = valid;
      while (__ballot(todo)) {
        if (todo) claim[h] = lane;
        __syncthreads();
        const bool win = todo && claim[h] == lane;
        if (win) {
          todo = false;
          if constexpr (D == 1) {
#pragma unroll
            for (int b = 0; b < NP; ++b) {
              if (!okb[0][b]) continue;
#pragma unroll
              for (int a = 0; a < NQ; ++a) {
                if (lq[0][a] < 0) continue;
                const T v = c[a * NP + b];
                T o = tile[lq[0][a]];
                o.x += v.x;
                o.y += v.y;
                tile[lq[0][a]] = o;
              }
            }
          } else {
#pragma unroll
            for (int b0 = 0; b0 < NP; ++b0)
#pragma unroll
              for (int b1 = 0; b1 < NP; ++b1) {
                if (!okb[0][b0] || !okb[1][b1]) continue;
#pragma unroll
                for (int a0 = 0; a0 < NQ; ++a0) {
                  if (lq[0][a0] < 0) continue;
                  const T u = c[a0 * NP + b0];
#pragma unroll
                  for (int a1 = 0; a1 < NQ; ++a1) {
                    if (lq[1][a1] < 0) continue;
                    const T v = c[N1 + a1 * NP + b1];
                    const int li = lq[0][a0] * tile1 + lq[1][a1];
                    T o = tile[li];
                    o.x += u.x * v.x - u.y * v.y;
                    o.y += u.x * v.y + u.y * v.x;
                    tile[li] = o;
                  }
                }
              }
          }
        }
        __syncthreads();
      }
    }
    __syncthreads();
  }
  int64_t slf = 0;
  for (int k = 0; k < D; ++k) slf = slf * p.sn[k] + sl[k];
  T *dst = cells + slf * ncell_q;
  for (int e = lane; e < tq_cells; e += 64) {
    int rem = e, q = 0, lqv[3] = {0, 0, 0};
    for (int k = D - 1; k >= 0; --k) {
      lqv[k] = rem % (int)p.tile[k];
      rem /= (int)p.tile[k];
    }
    int64_t qf = 0;
    for (int k = 0; k < D; ++k) qf = qf * p.Nq[k] + tq0[k] + lqv[k];
    (void)q;
    dst[qf] = tile[e];
  }
}

// One dimension, without atomics.  Packets of one (p-cell, q-cell) add to
// the same cells with the same shifts, so their coefficient vectors can be
// summed first:
//   aggregate  one workgroup per bin (p-cell, q-tile); thread (q-cell, m)
//              owns A[p-cell][q-cell][m] and adds c[m] of every record of the
//              bin that sits in its q-cell (records are read by all threads:
//              broadcast loads); deterministic;
//   stencil    cells[s][q] = sum over b, a of A[s + mindp - dp_b][q - dq_a][a np + b]
//              (eq. 2.25 with the shifts applied on the aggregated vectors).
struct Agg1Params {
  const char *recs;
  const int64_t *start;
  int64_t Nq, tile, ntq, npc;
};

// Eight waves split the bin's records; within a wave, lane l owns
// coefficient m = l % N1 of the q-cells l / N1 + (64 / N1) j (j < N1 / 2) of
// the 32-cell tile; the partial tiles are summed through LDS at the end.
constexpr int kAggWaves = 8;

template <int N1, typename T>
__global__ __launch_bounds__(64 * kAggWaves) void fggc_agg1_kernel(Agg1Params p, T *__restrict__ A) {
  using R = decltype(T{}.x);
  constexpr int RB = rec_bytes<1, N1, T>();
  constexpr int K = N1 / 2, STEP = 64 / N1, U = 16;
  __shared__ T part[kAggWaves][32 * N1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int m = lane % N1, q0 = lane / N1;
  const int64_t bin = blockIdx.x;
  const int64_t pc = bin / p.ntq, t = bin - pc * p.ntq;
  const int tbase = (int)(t * p.tile);
  const int64_t r0 = p.start[bin], r1 = p.start[bin + 1], n = r1 - r0;
  const int64_t ra = r0 + (n * w) / kAggWaves, rb = r0 + (n * (w + 1)) / kAggWaves;
  R ar[K], ai[K];
#pragma unroll
  for (int j = 0; j < K; ++j) ar[j] = ai[j] = 0;
  int64_t r = ra;
  for (; r + U <= rb; r += U) {
    int qq[U];
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const char *rec = p.recs + (r + u) * (int64_t)RB;
      qq[u] = *reinterpret_cast<const int32_t *>(rec) - tbase - q0;
      v[u] = reinterpret_cast<const T *>(rec + rec_idx_bytes<1>())[m];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int j = 0; j < K; ++j)
        if (qq[u] == STEP * j) {
          ar[j] += v[u].x;
          ai[j] += v[u].y;
        }
  }
  for (; r < rb; ++r) {
    const char *rec = p.recs + r * (int64_t)RB;
    const int qq = *reinterpret_cast<const int32_t *>(rec) - tbase - q0;
    const T v = reinterpret_cast<const T *>(rec + rec_idx_bytes<1>())[m];
#pragma unroll
    for (int j = 0; j < K; ++j)
      if (qq == STEP * j) {
        ar[j] += v.x;
        ai[j] += v.y;
      }
  }
#pragma unroll
  for (int j = 0; j < K; ++j) part[w][(q0 + STEP * j) * N1 + m] = T{ar[j], ai[j]};
  __syncthreads();
  for (int e = threadIdx.x; e < 32 * N1; e += blockDim.x) {
    const int ql = e / N1;
    T sum = part[0][e];
#pragma unroll
    for (int x = 1; x < kAggWaves; ++x) {
      sum.x += part[x][e].x;
      sum.y += part[x][e].y;
    }
    if (ql < p.tile) A[(pc * p.Nq + tbase + ql) * N1 + (e % N1)] = sum;
  }
}

struct Stencil1Params {
  int64_t Nq, sn, npc;
  int n1, nq, np, mindp;
  int dq[8], dp[8];
};

template <typename T>
__global__ void fggc_stencil1_kernel(Stencil1Params p, const T *__restrict__ A, int n1s,
                                     T *__restrict__ cells) {
  using R = decltype(T{}.x);
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= p.sn * p.Nq) return;
  const int64_t sl = e / p.Nq, q = e - sl * p.Nq;
  R ar = 0, ai = 0;
  for (int b = 0; b < p.np; ++b) {
    const int64_t pc = sl + p.mindp - p.dp[b];
    if (pc < 0 || pc >= p.npc) continue;
    for (int a = 0; a < p.nq; ++a) {
      const int64_t qs = (q - p.dq[a]) & (p.Nq - 1);
      const T v = A[(pc * p.Nq + qs) * n1s + a * p.np + b];
      ar += v.x;
      ai += v.y;
    }
  }
  cells[e] = T{ar, ai};
}

// Band tables per dimension: for slice index l (p = (slo + l) dp) the first
// frequency kstart of its band and gamma values for kstart .. kstart + nb - 1.
struct BandParams {
  int d;
  double eps, cK;
  int64_t slo[3], sn[3];
  double dp[3];
  int64_t nb[3];    // table width per dimension
  int64_t toff[3];  // offset of each dimension's gamma table (entries)
  int64_t koff[3];  // offset of each dimension's kstart table (entries)
};

// First frequency of slice l's band, and gamma at frequency k = k0 + i
// (0 outside the truncated band); used by the table kernel and inline.
__device__ __forceinline__ int64_t band_start(double p, double eps, double cK) {
  return (int64_t)ceil(p / eps - cK / sqrt(eps));
}
__device__ __forceinline__ double band_gamma(double p, int64_t k, double eps, double cK) {
  const double cst = sqrt(kTwoPi * eps) / kTwoPi;
  const double dk = eps * (double)k - p;  // eps (k - p/eps)
  const double ex = -dk * dk / (2.0 * eps);
  return (ex >= -0.5 * cK * cK * (1.0 + 1e-12)) ? cst * exp(ex) : 0.0;
}

template <typename R>
__global__ void band_table_kernel(BandParams b, R *__restrict__ gam, int64_t *__restrict__ kst) {
  const int k = blockIdx.y;
  if (k >= b.d) return;
  const int64_t total = b.sn[k] * b.nb[k];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = e / b.nb[k], i = e - l * b.nb[k];
    const double p = (double)(b.slo[k] + l) * b.dp[k];
    const int64_t k0 = band_start(p, b.eps, b.cK);
    gam[b.toff[k] + e] = (R)band_gamma(p, k0 + i, b.eps, b.cK);
    if (i == 0) kst[b.koff[k] + l] = k0;
  }
}

struct MacParams {
  double dp[3];
  int64_t M[3], Nq[3], sn[3], nb[3], toff[3], koff[3];
  int64_t kmin[3], kmax[3];  // union of the bands per dimension
  double lo_c[3], inv_dp[3], eps, cK;  // l range helpers
  int64_t slo[3];
};

template <int D, typename T, typename R>
__global__ __launch_bounds__(256) void band_mac_kernel(MacParams m, const T *__restrict__ F,
                                                       const R *__restrict__ gam,
                                                       const int64_t *__restrict__ kst,
                                                       T *__restrict__ U) {
  int64_t npts = 1;
  for (int k = 0; k < D; ++k) npts *= m.M[k];
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= npts) return;
  int64_t kp[3] = {0, 0, 0};
  {
    int64_t rem = e;
    for (int k = D - 1; k >= 0; --k) {
      kp[k] = rem % m.M[k];
      rem /= m.M[k];
    }
  }
  int64_t nqt = 1;
  for (int k = 0; k < D; ++k) nqt *= m.Nq[k];
  const double se = sqrt(m.eps);
  // per dimension: the aliases k = k' + jM that can lie in some band, and for
  // each the slice range whose band holds it
  double accr = 0.0, acci = 0.0;
  int64_t j0[3], j1[3];
  for (int k = 0; k < D; ++k) {
    // smallest j with k' + jM >= kmin, largest with k' + jM <= kmax
    int64_t a = m.kmin[k] - kp[k], b = m.kmax[k] - kp[k];
    j0[k] = a >= 0 ? (a + m.M[k] - 1) / m.M[k] : -((-a) / m.M[k]);
    j1[k] = b >= 0 ? b / m.M[k] : -((-b + m.M[k] - 1) / m.M[k]);
  }
  auto lrange = [&](int k, int64_t kk, int64_t &la, int64_t &lb) {
    // slices whose band [kst, kst + nb) holds kk; start from the real-valued estimate
    const double pk = m.eps * (double)kk;
    int64_t a = (int64_t)floor((pk - m.cK * se) * m.inv_dp[k]) - m.slo[k] - 1;
    int64_t b = (int64_t)ceil((pk + m.cK * se) * m.inv_dp[k]) - m.slo[k] + 1;
    if (a < 0) a = 0;
    if (b > m.sn[k] - 1) b = m.sn[k] - 1;
    la = a;
    lb = b;
  };
  const int64_t ts0 = m.koff[0], ts1 = m.koff[1], ts2 = m.koff[2];
  for (int64_t ja = j0[0]; ja <= j1[0]; ++ja) {
    const int64_t k0 = kp[0] + ja * m.M[0];
    int64_t la0, lb0;
    lrange(0, k0, la0, lb0);
    const int64_t q0 = ((k0 % m.Nq[0]) + m.Nq[0]) % m.Nq[0];
    for (int64_t l0 = la0; l0 <= lb0; ++l0) {
      const int64_t i0 = k0 - kst[ts0 + l0];
      if (i0 < 0 || i0 >= m.nb[0]) continue;
      const double g0 = (double)gam[m.toff[0] + l0 * m.nb[0] + i0];
      if (g0 == 0.0) continue;
      if (D == 1) {
        const T f = F[l0 * nqt + q0];
        accr = fma(g0, (double)f.x, accr);
        acci = fma(g0, (double)f.y, acci);
        continue;
      }
      for (int64_t jb = j0[1]; jb <= j1[1]; ++jb) {
        const int64_t k1 = kp[1] + jb * m.M[1];
        int64_t la1, lb1;
        lrange(1, k1, la1, lb1);
        const int64_t q1 = ((k1 % m.Nq[1]) + m.Nq[1]) % m.Nq[1];
        for (int64_t l1 = la1; l1 <= lb1; ++l1) {
          const int64_t i1 = k1 - kst[ts1 + l1];
          if (i1 < 0 || i1 >= m.nb[1]) continue;
          const double g01 = g0 * (double)gam[m.toff[1] + l1 * m.nb[1] + i1];
          if (g01 == 0.0) continue;
          if (D == 2) {
            const T f = F[(l0 * m.sn[1] + l1) * nqt + q0 * m.Nq[1] + q1];
            accr = fma(g01, (double)f.x, accr);
            acci = fma(g01, (double)f.y, acci);
            continue;
          }
          for (int64_t jc = j0[2]; jc <= j1[2]; ++jc) {
            const int64_t k2 = kp[2] + jc * m.M[2];
            int64_t la2, lb2;
            lrange(2, k2, la2, lb2);
            const int64_t q2 = ((k2 % m.Nq[2]) + m.Nq[2]) % m.Nq[2];
            for (int64_t l2 = la2; l2 <= lb2; ++l2) {
              const int64_t i2 = k2 - kst[ts2 + l2];
              if (i2 < 0 || i2 >= m.nb[2]) continue;
              const double g = g01 * (double)gam[m.toff[2] + l2 * m.nb[2] + i2];
              const T f = F[((l0 * m.sn[1] + l1) * m.sn[2] + l2) * nqt +
                            (q0 * m.Nq[1] + q1) * m.Nq[2] + q2];
              accr = fma(g, (double)f.x, accr);
              acci = fma(g, (double)f.y, acci);
            }
          }
        }
      }
    }
  }
  U[e] = T{(R)accr, (R)acci};
}

// One dimension: eight lanes per frequency split the slice loop, then a
// shuffle reduction (FP64) -- eight times the waves of the plain kernel.
template <typename T, typename R>
__global__ __launch_bounds__(256) void band_mac1_kernel(MacParams m, const T *__restrict__ F,
                                                         const R *__restrict__ gam,
                                                         const int64_t *__restrict__ kst,
                                                         T *__restrict__ U) {
  const int64_t id = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t e = id >> 3;
  const int g = (int)(id & 7);
  const bool live = e < m.M[0];
  double accr = 0.0, acci = 0.0;
  if (live) {
    const double se = sqrt(m.eps);
    const int64_t a = m.kmin[0] - e, b = m.kmax[0] - e, M = m.M[0];
    const int64_t j0 = a >= 0 ? (a + M - 1) / M : -((-a) / M);
    const int64_t j1 = b >= 0 ? b / M : -((-b + M - 1) / M);
    for (int64_t ja = j0; ja <= j1; ++ja) {
      const int64_t k0 = e + ja * M;
      const double pk = m.eps * (double)k0;
      int64_t la = (int64_t)floor((pk - m.cK * se) * m.inv_dp[0]) - m.slo[0] - 1;
      int64_t lb = (int64_t)ceil((pk + m.cK * se) * m.inv_dp[0]) - m.slo[0] + 1;
      if (la < 0) la = 0;
      if (lb > m.sn[0] - 1) lb = m.sn[0] - 1;
      const int64_t q0 = ((k0 % m.Nq[0]) + m.Nq[0]) % m.Nq[0];
      for (int64_t l0 = la + g; l0 <= lb; l0 += 8) {
        // gamma evaluated in place, exactly as the band table would hold it
        const double p = (double)(m.slo[0] + l0) * m.dp[0];
        const int64_t i0 = k0 - band_start(p, m.eps, m.cK);
        if (i0 < 0 || i0 >= m.nb[0]) continue;
        const double g0 = (double)(R)band_gamma(p, k0, m.eps, m.cK);
        const T f = F[l0 * m.Nq[0] + q0];
        accr = fma(g0, (double)f.x, accr);
        acci = fma(g0, (double)f.y, acci);
      }
    }
  }
#pragma unroll
  for (int o = 1; o < 8; o <<= 1) {
    accr += __shfl_xor(accr, o);
    acci += __shfl_xor(acci, o);
  }
  if (live && g == 0) U[e] = T{(R)accr, (R)acci};
}

// Separable Fourier finish (d >= 2).  The band weight gamma_l(k) and the DFT
// both factor over dimensions, so the sum over slices l and cells i of
// eq. (2.24) in Fourier space is a product of one-dimensional operators
//   K_k(k'; l, i) = sum_j gamma_{l,k}(k' + j M_k) exp(-2 pi i (k' + j M_k) i / Nq_k)
// applied one dimension at a time, last dimension first.  A pass reads the
// array as [O][L][A][N][B] (L slices and N q-cells of dimension k), FFTs each
// (slice, b) row over q in LDS, folds the slices into the M grid frequencies
// with the band weights (FP64 accumulation) and writes [O][A][M][B].
struct ContractParams {
  int64_t O, L, A, B, M;
  int lgN, W, Lc, R;  // W: b values per workgroup; Lc: slices per LDS chunk; R: outputs per thread
  int MS;             // workgroups sharing one line group, each with M / MS of the frequencies
  int64_t nb, toff, koff, slo, kmin, kmax;
  double eps, cK, inv_dp;
};


template <typename T, typename R>
__global__ __launch_bounds__(256) void fft_contract_kernel(ContractParams p, const T *__restrict__ X,
                                                           T *__restrict__ Y, const R *__restrict__ gam,
                                                           const int64_t *__restrict__ kst,
                                                           const T *__restrict__ tw) {
  using RR = decltype(T{}.x);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *sm = reinterpret_cast<T *>(smem_raw);
  const int N = 1 << p.lgN, W = p.W, M = (int)p.M;
  const int64_t nbc = p.B / W;
  int64_t g = blockIdx.x;
  const int mg = (int)(g % p.MS);
  g /= p.MS;
  const int64_t bc = g % nbc;
  g /= nbc;
  const int64_t a = g % p.A, o = g / p.A;
  const int64_t b0 = bc * W;
  const int Mg = M / p.MS, k0g = mg * Mg;  // this workgroup's frequencies [k0g, k0g + Mg)
  const int nout = Mg * W;
  const int nb = (int)p.nb;
  // LDS: rows of the chunk, one accumulator per output ([w][k]), band rows
  T *acc = sm + (size_t)p.Lc * N * W;
  R *bg = reinterpret_cast<R *>(acc + nout);
  int *bk = reinterpret_cast<int *>(bg + (size_t)p.Lc * nb);
  for (int e = threadIdx.x; e < nout; e += blockDim.x) acc[e] = T{0, 0};
  const double se = sqrt(p.eps);
  const int kmin = (int)p.kmin, kmax = (int)p.kmax, slo = (int)p.slo;
  for (int lc0 = 0; lc0 < (int)p.L; lc0 += p.Lc) {
    const int lcn = min(p.Lc, (int)p.L - lc0);
    const int tot = lcn * N * W;
    for (int e = threadIdx.x; e < tot; e += blockDim.x) {
      const int w = e % W, rest = e / W;
      const int n = rest & (N - 1), l = rest >> p.lgN;
      sm[(l * W + w) * N + n] = X[(((o * p.L + lc0 + l) * p.A + a) * N + n) * p.B + b0 + w];
    }
    for (int e = threadIdx.x; e < lcn * nb; e += blockDim.x) bg[e] = gam[p.toff + (int64_t)lc0 * nb + e];
    for (int e = threadIdx.x; e < lcn; e += blockDim.x) bk[e] = (int)kst[p.koff + lc0 + e];
    __syncthreads();
    lds_fft_rows<T>(sm, p.lgN, lcn * W, N, 0, tw);
    for (int e = threadIdx.x; e < nout; e += blockDim.x) {
      const int kp = k0g + e % Mg, w = e / Mg;
      // aliases kk = kp + j M inside [kmin, kmax]
      const int lo = kmin - kp, hi = kmax - kp;
      const int j0 = lo >= 0 ? (lo + M - 1) / M : -((-lo) / M);
      const int j1 = hi >= 0 ? hi / M : -((-hi + M - 1) / M);
      double xr = 0.0, xi = 0.0;
      for (int j = j0; j <= j1; ++j) {
        const int kk = kp + j * M;
        const double pk = p.eps * (double)kk;
        int la = (int)floor((pk - p.cK * se) * p.inv_dp) - slo - 1;
        int lb = (int)ceil((pk + p.cK * se) * p.inv_dp) - slo + 1;
        la = max(la, lc0);
        lb = min(lb, lc0 + lcn - 1);
        const int q = kk & (N - 1);
        for (int l = la; l <= lb; ++l) {
          const int ll = l - lc0;
          const int i0 = kk - bk[ll];
          if (i0 < 0 || i0 >= nb) continue;
          const double gv = (double)bg[ll * nb + i0];
          const T v = sm[(ll * W + w) * N + q];
          xr = fma(gv, (double)v.x, xr);
          xi = fma(gv, (double)v.y, xi);
        }
      }
      T c = acc[e];
      c.x += (RR)xr;
      c.y += (RR)xi;
      acc[e] = c;
    }
    __syncthreads();
  }
  // write coalesced along b
  for (int e = threadIdx.x; e < nout; e += blockDim.x) {
    const int kl = e / W, w = e % W;
    Y[((o * p.A + a) * p.M + k0g + kl) * p.B + b0 + w] = acc[w * Mg + kl];
  }
}

struct FggcLayout {
  int d, N1, rec_b, ns;
  bool agg1;  // one dimension: aggregate + stencil instead of tile accumulation
  int64_t ncells, nslices, npts, nbins, nslots, tiles, ntq[3], tile[3], npc[3], pmin[3], S[3], nsw[3];
  int64_t nb[3], toff[3], koff[3], ntab, nkst;
  int mindp, maxdp, mindq, maxdq;
  size_t off_lsq, off_keys, off_pos, off_sort, off_start, off_recs, off_agg, off_cells, off_gam, off_kst,
      off_spec, off_x1, off_x2, total;
};

int n1_bucket(int n1) { return n1 <= 4 ? 4 : (n1 <= 8 ? 8 : 16); }

FggcLayout fggc_layout(const FggcArgs &a) {
  FggcLayout L{};
  const int d = a.g.d;
  L.d = d;
  const bool f64 = a.precision == FGGC_FP64;
  const size_t es = f64 ? 16 : 8;
  const DimLsq &l0 = a.lsq[0];
  L.N1 = n1_bucket(l0.n1);
  L.rec_b = 16 * ((8 * d + 15) / 16) + d * L.N1 * (int)es;
  L.mindp = L.maxdp = l0.dp[0];
  L.mindq = L.maxdq = l0.dq[0];
  for (int m = 1; m < l0.n1; ++m) {
    L.mindp = std::min(L.mindp, l0.dp[m]);
    L.maxdp = std::max(L.maxdp, l0.dp[m]);
    L.mindq = std::min(L.mindq, l0.dq[m]);
    L.maxdq = std::max(L.maxdq, l0.dq[m]);
  }
  // q-tile and slice window of one accumulation workgroup: the LDS holds
  // S^d * tile^d cells; a tile is at least as wide as the q-shift set
  static const int64_t deft[4] = {0, 32, 32, 16}, defs[4] = {0, 1, 1, 1};
  int64_t tmin = 1;
  while (tmin < L.maxdq - L.mindq + 1) tmin *= 2;
  L.nslices = 1;
  int64_t nqt = 1;
  L.npts = 1;
  L.ntab = 0;
  L.nkst = 0;
  L.nbins = 1;
  L.tiles = 1;
  for (int k = 0; k < 3; ++k) {
    if (k < d) {
      L.nslices *= a.sn[k];
      nqt *= a.Nq[k];
      L.npts *= a.g.n[k];
      // one dimension aggregates by own q-cell (no halo): tiles of exactly 32
      // cells, the width of the aggregation workgroup
      L.tile[k] = d == 1 ? std::min<int64_t>(a.Nq[k], 32)
                         : std::min<int64_t>(a.Nq[k], std::max<int64_t>(deft[d], tmin));
      L.ntq[k] = a.Nq[k] / L.tile[k];
      L.pmin[k] = a.slo[k] - L.mindp;
      L.npc[k] = a.sn[k] - (L.maxdp - L.mindp);
      L.S[k] = std::min<int64_t>(defs[d], a.sn[k]);
      L.nsw[k] = (a.sn[k] + L.S[k] - 1) / L.S[k];
      L.nbins *= L.npc[k] * L.ntq[k];
      L.tiles *= L.nsw[k] * L.ntq[k];
      L.nb[k] = (int64_t)std::floor(2.0 * a.cK / std::sqrt(a.eps)) + 2;
      L.toff[k] = L.ntab;
      L.koff[k] = L.nkst;
      L.ntab += a.sn[k] * L.nb[k];
      L.nkst += a.sn[k];
    } else {
      L.tile[k] = L.ntq[k] = L.npc[k] = L.S[k] = L.nsw[k] = 1;
      L.pmin[k] = 0;
      L.nb[k] = 1;
      L.toff[k] = 0;
      L.koff[k] = 0;
    }
  }
  if (L.nbins >= ((int64_t)1 << 32)) fail(FGGC_EUNSUPPORTED, "too many packet bins");
  L.ncells = L.nslices * nqt;
  if (L.tiles >= ((int64_t)1 << 31)) fail(FGGC_EUNSUPPORTED, "too many accumulation workgroups");
  const int64_t N = std::max<int64_t>(a.pk->N, 1);
  L.agg1 = d == 1;
  L.ns = L.agg1 ? 1 : (1 << d);  // key slots per packet: own tile, or 2^d with halo tiles
  L.nslots = a.pk->N * L.ns;
  const int64_t NS = std::max<int64_t>(L.nslots, 1);
  size_t o = 0;
  auto put = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.off_lsq = put(3 * sizeof(DimLsq));
  L.off_keys = put(NS * 4);
  L.off_pos = put(NS * 4);
  L.off_sort = put(std::max(bucket_positions_bytes(L.nslots, L.nbins), count_plan(L.nslots, L.nbins, L.ns).bytes));
  L.off_start = put((size_t)(L.nbins + 1) * 8);
  L.off_recs = put((size_t)NS * L.rec_b);  // at most one record per slot
  L.off_agg = put(L.agg1 ? (size_t)L.npc[0] * a.Nq[0] * L.N1 * es : 0);
  (void)N;
  L.off_cells = put((size_t)L.ncells * es);
  L.off_gam = put((size_t)L.ntab * (es / 2));
  L.off_kst = put((size_t)L.nkst * 8 + 64);
  L.off_spec = put((size_t)L.npts * es);  // grid spectrum (the inverse FFT writes u from it)
  // separable finish (d >= 2): outputs of the passes over the last and the
  // middle dimension, [l_<k][i_<k][grid frequencies of dims >= k]
  L.off_x1 = L.off_x2 = 0;
  if (d >= 2) {
    auto pass_out = [&](int k) {
      size_t v = 1;
      for (int j = 0; j < k; ++j) v *= (size_t)a.sn[j] * (size_t)a.Nq[j];
      for (int j = k; j < d; ++j) v *= (size_t)a.g.n[j];
      return v;
    };
    L.off_x1 = put(pass_out(d - 1) * es);
    if (d == 3) L.off_x2 = put(pass_out(1) * es);
  }
  L.total = o;
  return L;
}

template <int D, int N1, typename T>
void launch_coef_accum(const FggcArgs &a, const FggcLayout &L, const CoefParams &cp,
                       const uint32_t *pos, char *recs, const int64_t *start, void *agg, T *cells,
                       hipStream_t s) {
  const DimLsq &c0 = a.lsq[0];
  int cnp = 0;
  for (int m = 0; m < c0.n1; ++m)
    if (c0.dq[m] == c0.dq[0]) ++cnp;
  const int cnq = c0.n1 / cnp;
  if (cp.N > 0) {
    StageScope sc(a.prof, "fggc_coef", s);
    const dim3 g((unsigned)((cp.N + 255) / 256)), b(256);
    if (N1 == 4 && cnq == 2 && cnp == 2) fggc_coef_kernel<D, N1, 2, 2, T><<<g, b, 0, s>>>(cp, pos, recs);
    else if (N1 == 8 && cnq == 4 && cnp == 2) fggc_coef_kernel<D, N1, 4, 2, T><<<g, b, 0, s>>>(cp, pos, recs);
    else if (N1 == 8 && cnq == 2 && cnp == 4) fggc_coef_kernel<D, N1, 2, 4, T><<<g, b, 0, s>>>(cp, pos, recs);
    else if (N1 == 16 && cnq == 4 && cnp == 4) fggc_coef_kernel<D, N1, 4, 4, T><<<g, b, 0, s>>>(cp, pos, recs);
    else fggc_coef_kernel<D, N1, 0, 0, T><<<g, b, 0, s>>>(cp, pos, recs);
    FGGC_HIP(hipGetLastError());
  }
  AccParams ap{};
  ap.recs = recs;
  ap.start = start;
  const DimLsq &l0 = a.lsq[0];
  for (int k = 0; k < 3; ++k) {
    ap.sn[k] = a.sn[k];
    ap.npc[k] = L.npc[k];
    ap.Nq[k] = a.Nq[k];
    ap.tile[k] = L.tile[k];
    ap.ntq[k] = L.ntq[k];
    ap.S[k] = L.S[k];
    ap.nsw[k] = L.nsw[k];
  }
  // one-dimensional shift sets (basis index a * np + b)
  int nq = 0, np = 0;
  for (int m = 0; m < l0.n1; ++m) {
    if (l0.dq[m] == l0.dq[0]) ++np;
  }
  nq = l0.n1 / np;
  ap.nq = nq;
  ap.np = np;
  for (int i = 0; i < 8; ++i) {
    ap.dq[i] = i < nq ? l0.dq[i * np] : 0;
    ap.dp[i] = i < np ? l0.dp[i] : 0;
  }
  ap.mindp = L.mindp;
  ap.maxdp = L.maxdp;
  if (L.agg1) {
    StageScope sc(a.prof, "fggc_accum", s);
    T *A = reinterpret_cast<T *>(agg);
    Agg1Params gp{};
    gp.recs = recs;
    gp.start = start;
    gp.Nq = a.Nq[0];
    gp.tile = L.tile[0];
    gp.ntq = L.ntq[0];
    gp.npc = L.npc[0];
    const dim3 gg((unsigned)L.nbins), gb(64 * kAggWaves);
    fggc_agg1_kernel<N1, T><<<gg, gb, 0, s>>>(gp, A);
    FGGC_HIP(hipGetLastError());
    Stencil1Params sp{};
    sp.Nq = a.Nq[0];
    sp.sn = a.sn[0];
    sp.npc = L.npc[0];
    sp.n1 = l0.n1;
    sp.nq = nq;
    sp.np = np;
    sp.mindp = L.mindp;
    for (int i = 0; i < 8; ++i) {
      sp.dq[i] = ap.dq[i];
      sp.dp[i] = ap.dp[i];
    }
    const int64_t ncl = a.sn[0] * a.Nq[0];
    fggc_stencil1_kernel<T><<<dim3((unsigned)((ncl + 255) / 256)), dim3(256), 0, s>>>(sp, A, N1, cells);
    FGGC_HIP(hipGetLastError());
    return;
  }
  int64_t tc = 1;
  for (int k = 0; k < D; ++k) tc *= L.tile[k] * L.S[k];
  const size_t shm = 2 * (size_t)tc * sizeof(decltype(T{}.x));
  if (shm > 65536) fail(FGGC_EUNSUPPORTED, "accumulation tile exceeds 64 KB of LDS");
  StageScope sc(a.prof, "fggc_accum", s);
  const dim3 grid((unsigned)L.tiles), blk(256);
  const bool wave = D <= 2 && L.S[0] == 1 && (D < 2 || L.S[1] == 1);
  if (wave) {
    const size_t wshm = (size_t)(tc)*sizeof(T);
    const dim3 wblk(64);
    if (N1 == 4 && nq == 2 && np == 2) {
      fggc_accum_wave_kernel<D, 2, 2, T><<<grid, wblk, wshm, s>>>(ap, cells);
      FGGC_HIP(hipGetLastError());
      return;
    }
    if (N1 == 8 && nq == 4 && np == 2) {
      fggc_accum_wave_kernel<D, 4, 2, T><<<grid, wblk, wshm, s>>>(ap, cells);
      FGGC_HIP(hipGetLastError());
      return;
    }
    if (N1 == 8 && nq == 2 && np == 4) {
      fggc_accum_wave_kernel<D, 2, 4, T><<<grid, wblk, wshm, s>>>(ap, cells);
      FGGC_HIP(hipGetLastError());
      return;
    }
    if (N1 == 16 && nq == 4 && np == 4) {
      fggc_accum_wave_kernel<D, 4, 4, T><<<grid, wblk, wshm, s>>>(ap, cells);
      FGGC_HIP(hipGetLastError());
      return;
    }
  }
  if (N1 == 4 && nq == 2 && np == 2)
    fggc_accum_kernel<D, 2, 2, T><<<grid, blk, shm, s>>>(ap, cells);
  else if (N1 == 8 && nq == 4 && np == 2)
    fggc_accum_kernel<D, 4, 2, T><<<grid, blk, shm, s>>>(ap, cells);
  else if (N1 == 8 && nq == 2 && np == 4)
    fggc_accum_kernel<D, 2, 4, T><<<grid, blk, shm, s>>>(ap, cells);
  else if (N1 == 16 && nq == 4 && np == 4 && D < 3)
    fggc_accum_kernel<D, 4, 4, T><<<grid, blk, shm, s>>>(ap, cells);
  else
    fggc_accum_generic_kernel<D, N1, T><<<grid, blk, shm, s>>>(ap, cells);
  FGGC_HIP(hipGetLastError());
}

bool g_rank_attr = false;
std::mutex g_rank_mu;

// bin the packets' key slots, compute their coefficients into bin order, and fill
// the cell array of eq. (2.25) (every cell written once)
void cells_stage(const FggcArgs &a, const FggcLayout &L, char *base, void *cells, hipStream_t s) {
  const int d = a.g.d;
  const bool f64 = a.precision == FGGC_FP64;
  const DimLsq *dlsq = a.lsq_dev;
  if (!dlsq) {
    DimLsq *tmp = (DimLsq *)(base + L.off_lsq);
    FGGC_HIP(hipMemcpyAsync(tmp, a.lsq, d * sizeof(DimLsq), hipMemcpyHostToDevice, s));
    dlsq = tmp;
  }
  const int64_t N = a.pk->N;
  uint32_t *keys = (uint32_t *)(base + L.off_keys), *pos = (uint32_t *)(base + L.off_pos);
  int64_t *start = (int64_t *)(base + L.off_start);
  char *recs = base + L.off_recs;
  KeyParams kp{};
  kp.N = N;
  kp.Q = a.pk->Q;
  kp.P = a.pk->P;
  for (int k = 0; k < 3; ++k) {
    kp.Nq[k] = a.Nq[k];
    kp.pmin[k] = L.pmin[k];
    kp.npc[k] = L.npc[k];
    kp.tile[k] = L.tile[k];
    kp.ntq[k] = L.ntq[k];
    kp.dq[k] = kTwoPi / (double)a.Nq[k];
    kp.dp[k] = a.dp[k];
  }
  kp.mindq = L.mindq;
  kp.maxdq = L.maxdq;
  kp.ns = L.ns;
  const CountPlan cpn = count_plan(L.nslots, L.nbins, L.ns);
  uint32_t *rank = (uint32_t *)(base + L.off_sort + cpn.off_rank);
  {
    std::lock_guard<std::mutex> lk(g_rank_mu);
    if (!g_rank_attr) {
      FGGC_HIP(hipFuncSetAttribute((const void *)fggc_rank_kernel<1>, hipFuncAttributeMaxDynamicSharedMemorySize, 131072));
      FGGC_HIP(hipFuncSetAttribute((const void *)fggc_rank_kernel<2>, hipFuncAttributeMaxDynamicSharedMemorySize, 131072));
      FGGC_HIP(hipFuncSetAttribute((const void *)fggc_rank_kernel<3>, hipFuncAttributeMaxDynamicSharedMemorySize, 131072));
      g_rank_attr = true;
    }
  }
  {
    StageScope sc(a.prof, "fggc_sort", s);
    if (cpn.lds) {
      // keys computed in place: ranks here, positions in the coefficient kernel
      char *sc_base = base + L.off_sort;
      uint32_t *table = (uint32_t *)(sc_base + cpn.off_table);
      if (N > 0) {
        const dim3 g((unsigned)cpn.G), b(1024);
        const size_t shm = (size_t)L.nbins * 4;
        if (d == 1) fggc_rank_kernel<1><<<g, b, shm, s>>>(kp, cpn.chunk, L.nbins, cpn.G, table, rank, keys);
        else if (d == 2) fggc_rank_kernel<2><<<g, b, shm, s>>>(kp, cpn.chunk, L.nbins, cpn.G, table, rank, keys);
        else fggc_rank_kernel<3><<<g, b, shm, s>>>(kp, cpn.chunk, L.nbins, cpn.G, table, rank, keys);
        FGGC_HIP(hipGetLastError());
      } else {
        launch_zero(table, (size_t)L.nbins * cpn.G * 4, s);
      }
      count_scan(cpn, L.nbins, sc_base, start, s);
      if (N > 0) count_positions(cpn, keys, L.nslots, sc_base, pos, s);
    } else if (N > 0) {
      const dim3 g((unsigned)((N + 255) / 256)), b(256);
      if (d == 1) fggc_key_kernel<1><<<g, b, 0, s>>>(kp, keys);
      else if (d == 2) fggc_key_kernel<2><<<g, b, 0, s>>>(kp, keys);
      else fggc_key_kernel<3><<<g, b, 0, s>>>(kp, keys);
      FGGC_HIP(hipGetLastError());
      bucket_positions(keys, L.nslots, L.nbins, pos, start, base + L.off_sort, s);
    } else {
      bucket_positions(keys, L.nslots, L.nbins, pos, start, base + L.off_sort, s);
    }
  }
  CoefParams cp{};
  cp.ns = L.ns;
  cp.N = N;
  cp.Q = a.pk->Q;
  cp.P = a.pk->P;
  cp.S = a.pk->S;
  cp.a = a.pk->a;
  cp.eps = a.eps;
  cp.scale = a.scale;
  cp.lsq = dlsq;
  for (int k = 0; k < 3; ++k) {
    cp.Nq[k] = a.Nq[k];
    cp.pmin[k] = L.pmin[k];
    cp.dq[k] = kTwoPi / (double)a.Nq[k];
    cp.dp[k] = a.dp[k];
  }
#define FGGC_CA(DD, NN)                                                                           \
  if (f64) launch_coef_accum<DD, NN, double2>(a, L, cp, pos, recs, start, base + L.off_agg, (double2 *)cells, s); \
  else launch_coef_accum<DD, NN, float2>(a, L, cp, pos, recs, start, base + L.off_agg, (float2 *)cells, s);
  if (d == 1) {
    if (L.N1 == 4) { FGGC_CA(1, 4) } else if (L.N1 == 8) { FGGC_CA(1, 8) } else { FGGC_CA(1, 16) }
  } else if (d == 2) {
    if (L.N1 == 4) { FGGC_CA(2, 4) } else if (L.N1 == 8) { FGGC_CA(2, 8) } else { FGGC_CA(2, 16) }
  } else {
    if (L.N1 == 4) { FGGC_CA(3, 4) } else if (L.N1 == 8) { FGGC_CA(3, 8) }
    else fail(FGGC_EUNSUPPORTED, "3D strategies need nq * np <= 8");
  }
#undef FGGC_CA
}

bool g_contract_attr = false;
std::mutex g_contract_mu;

// One separable pass over dimension k (see fft_contract_kernel).
template <typename T, typename R>
void launch_contract(const FggcArgs &a, const FggcLayout &L, int k, const T *in, T *out, const R *gam,
                     const int64_t *kst, const MacParams &m, hipStream_t s) {
  {
    std::lock_guard<std::mutex> lk(g_contract_mu);
    if (!g_contract_attr) {
      FGGC_HIP(hipFuncSetAttribute((const void *)fft_contract_kernel<float2, float>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, 131072));
      FGGC_HIP(hipFuncSetAttribute((const void *)fft_contract_kernel<double2, double>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, 131072));
      g_contract_attr = true;
    }
  }
  const int d = a.g.d;
  ContractParams p{};
  p.O = 1;
  p.A = 1;
  p.B = 1;
  for (int j = 0; j < k; ++j) {
    p.O *= a.sn[j];
    p.A *= a.Nq[j];
  }
  for (int j = k + 1; j < d; ++j) p.B *= a.g.n[j];
  p.L = a.sn[k];
  p.M = a.g.n[k];
  int lgN = 0;
  while (((int64_t)1 << lgN) < a.Nq[k]) ++lgN;
  p.lgN = lgN;
  const int64_t N = a.Nq[k];
  const size_t es = sizeof(T);
  // b values per workgroup: coalesced runs along b, at most 4096 outputs per workgroup
  int64_t W = 1;
  while (W * 2 <= std::min<int64_t>(16, p.B) && W * 2 * p.M <= 4096) W *= 2;
  // LDS chunk: rows * N elements within the butterfly budget of lds_fft_rows
  // for 256 threads, counting the radix-2 pass of an odd log2 N
  // (rows * N / 2 <= 256 * kMaxBfly)
  const int64_t elems = 256 * kMaxBfly * 2;
  while (W > 1 && N * W > elems) W /= 2;
  if (N * W > elems) fail(FGGC_EUNSUPPORTED, "q-mesh too long for the separable finish");
  p.W = (int)W;
  p.Lc = (int)std::max<int64_t>(1, std::min<int64_t>(p.L, elems / (N * W)));
  // split the frequencies of a line group over several workgroups when there
  // are few line groups (each recomputes the group's FFTs)
  const int64_t groups = p.O * p.A * (p.B / W);
  int MS = 1;
  while (groups * MS < 1024 && MS * 2 <= 16 && (p.M / (MS * 2)) * W >= 256) MS *= 2;
  p.MS = MS;
  p.R = 0;
  p.nb = L.nb[k];
  p.toff = L.toff[k];
  p.koff = L.koff[k];
  p.slo = a.slo[k];
  p.kmin = m.kmin[k];
  p.kmax = m.kmax[k];
  p.eps = a.eps;
  p.cK = a.cK;
  p.inv_dp = 1.0 / a.dp[k];
  const size_t rows_b = ((size_t)p.Lc * N * W + (size_t)(p.M / MS) * W) * es;
  const size_t band_b = (size_t)p.Lc * p.nb * sizeof(R) + (size_t)p.Lc * 4;
  const size_t shm = rows_b + band_b + 16;
  if (shm > 131072) fail(FGGC_EUNSUPPORTED, "separable finish needs more than 128 KB of LDS");
  const int64_t blocks = groups * MS;
  if (blocks >= ((int64_t)1 << 31)) fail(FGGC_EUNSUPPORTED, "too many workgroups for the separable finish");
  const T *tw = (const T *)fft_twiddles(N, a.precision);
  fft_contract_kernel<T, R><<<dim3((unsigned)blocks), dim3(256), shm, s>>>(p, in, out, gam, kst, tw);
  FGGC_HIP(hipGetLastError());
}

template <typename T, typename R>
void finish_stage(const FggcArgs &a, const FggcLayout &L, char *base, T *cells, R *gam, int64_t *kst,
                  void *spec, Workspace &ws, hipStream_t s) {
  const int d = a.g.d;
  const int prec = a.precision;
  // F5: forward DFT over q of every p-slice (one dimension; higher dimensions
  // fold the DFT into the separable passes below)
  if (d == 1) launch_fft(d, a.Nq, L.nslices, -1, prec, cells, ws, s, a.prof, "fggc_fft_q");
  // band tables
  BandParams bp{};
  bp.d = d;
  bp.eps = a.eps;
  bp.cK = a.cK;
  for (int k = 0; k < 3; ++k) {
    bp.slo[k] = a.slo[k];
    bp.sn[k] = a.sn[k];
    bp.dp[k] = a.dp[k];
    bp.nb[k] = L.nb[k];
    bp.toff[k] = L.toff[k];
    bp.koff[k] = L.koff[k];
  }
  if (d >= 2) {  // one dimension evaluates gamma in place
    StageScope sc(a.prof, "fggc_band_table", s);
    band_table_kernel<R><<<dim3(64, (unsigned)d), dim3(256), 0, s>>>(bp, gam, kst);
    FGGC_HIP(hipGetLastError());
  }
  // F6: band multiply-accumulate into the grid spectrum (written into u)
  MacParams m{};
  const double se = std::sqrt(a.eps);
  for (int k = 0; k < 3; ++k) {
    m.M[k] = k < d ? a.g.n[k] : 1;
    m.Nq[k] = k < d ? a.Nq[k] : 1;
    m.sn[k] = a.sn[k];
    m.nb[k] = L.nb[k];
    m.toff[k] = L.toff[k];
    m.koff[k] = L.koff[k];
    m.slo[k] = a.slo[k];
    m.dp[k] = a.dp[k];
    m.inv_dp[k] = 1.0 / a.dp[k];
    if (k < d) {
      m.kmin[k] = (int64_t)std::floor((double)a.slo[k] * a.dp[k] / a.eps - a.cK / se) - 1;
      m.kmax[k] = (int64_t)std::ceil((double)(a.slo[k] + a.sn[k] - 1) * a.dp[k] / a.eps + a.cK / se) + 1;
    }
  }
  m.eps = a.eps;
  m.cK = a.cK;
  T *U = (T *)spec;
  const unsigned nblk = (unsigned)((L.npts + 255) / 256);
  if (d >= 2) {
    // F5 + F6 as d separable passes, last dimension first, into the spectrum
    StageScope sc(a.prof, "fggc_contract", s);
    T *x1 = (T *)(base + L.off_x1), *x2 = (T *)(base + L.off_x2);
    const T *in = cells;
    for (int k = d - 1; k >= 0; --k) {
      T *out = k == 0 ? U : (k == d - 1 ? x1 : x2);
      launch_contract<T, R>(a, L, k, in, out, gam, kst, m, s);
      in = out;
    }
  } else {
  StageScope sc(a.prof, "fggc_band_mac", s);
  if (d == 1)
    band_mac1_kernel<T, R><<<(unsigned)((8 * L.npts + 255) / 256), 256, 0, s>>>(m, cells, gam, kst, U);
  else if (d == 2) band_mac_kernel<2, T, R><<<nblk, 256, 0, s>>>(m, cells, gam, kst, U);
  else band_mac_kernel<3, T, R><<<nblk, 256, 0, s>>>(m, cells, gam, kst, U);
  FGGC_HIP(hipGetLastError());
  }
  // F7: inverse DFT of the grid spectrum into u
  launch_fft_to(d, a.g.n, +1, prec, U, a.u, ws, s, a.prof, "fggc_ifft");
}

}  // namespace

size_t fggc_workspace_bytes(const FggcArgs &a) { return fggc_layout(a).total + 1024; }

bool fggc_graph_safe(const FggcArgs &a) {
  const FggcLayout L = fggc_layout(a);
  return bucket_positions_graph_safe(L.nslots, L.nbins);
}

size_t fggc_cells_workspace_bytes(const FggcArgs &a) {
  FggcLayout L = fggc_layout(a);
  return L.off_cells + 1024;
}

void launch_fggc_cells(const FggcArgs &a, void *cells, Workspace &ws, hipStream_t s) {
  FggcLayout L = fggc_layout(a);
  char *base = (char *)ws.take(L.off_cells);
  cells_stage(a, L, base, cells, s);
}

void launch_fggc(const FggcArgs &a, Workspace &ws, hipStream_t s) {
  FggcLayout L = fggc_layout(a);
  char *base = (char *)ws.take(L.total);
  void *cells = base + L.off_cells;
  cells_stage(a, L, base, cells, s);
  if (a.precision == FGGC_FP64)
    finish_stage<double2, double>(a, L, base, (double2 *)cells, (double *)(base + L.off_gam),
                                  (int64_t *)(base + L.off_kst), base + L.off_spec, ws, s);
  else
    finish_stage<float2, float>(a, L, base, (float2 *)cells, (float *)(base + L.off_gam),
                                (int64_t *)(base + L.off_kst), base + L.off_spec, ws, s);
}

}  // namespace fggc
