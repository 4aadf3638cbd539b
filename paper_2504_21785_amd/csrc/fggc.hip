// Frozen Gaussian grid-point correction on gfx950 (Section 2.3, Alg. 2).
//
//   fggc_key      per packet: its own cell (int parts of eq. 3.6) -> bin key
//                 (p-cell major, q-tile minor); radix sort of the packets by bin.
//   fggc_coef     one thread per packet, in bin order, FP64: frac parts (3.7),
//                 right-hand side (3.23), least squares through the plan's
//                 eigenpairs (c^ = V diag(1/lambda) V^H f~), conjugation to the
//                 L2-best coefficients, shift (3.13); the per-dimension
//                 coefficients (the first times scale a exp(i S/eps)) are
//                 written as one record per packet.
//   fggc_accum    owner-computes form of eq. (2.23)-(2.25): one workgroup per
//                 (p-slice, q-tile) of the dense cell array accumulates, in LDS,
//                 the Kronecker products of every packet of the bins that reach
//                 it, then writes each of its cells once.
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

// Sort key of a packet: its own p-cell (relative to the box of packet p-cells)
// major, its q-tile minor.  Packets of one key form one bin.
struct KeyParams {
  int64_t N;
  const double *Q, *P;
  int64_t Nq[3], pmin[3], npc[3], tile[3], ntq[3];
  double dq[3], dp[3];
};

template <int D>
__global__ void fggc_key_kernel(KeyParams p, uint32_t *__restrict__ key) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= p.N) return;
  int64_t kp = 0, kq = 0;
  for (int k = 0; k < D; ++k) {
    int64_t iq, ip;
    double s, t;
    int_frac(p.Q[k * p.N + j] / p.dq[k], iq, s);
    int_frac(p.P[k * p.N + j] / p.dp[k], ip, t);
    const int64_t qi = (iq + p.Nq[k] / 2) & (p.Nq[k] - 1);
    // the cell box comes from the same floor(P/dp), so this clamp never binds;
    // it keeps every key inside [0, nbins) whatever the caller's box
    int64_t pc = ip - p.pmin[k];
    pc = pc < 0 ? 0 : (pc >= p.npc[k] ? p.npc[k] - 1 : pc);
    kp = kp * p.npc[k] + pc;
    kq = kq * p.ntq[k] + qi / p.tile[k];
  }
  int64_t nqt = 1;
  for (int k = 0; k < D; ++k) nqt *= p.ntq[k];
  key[j] = (uint32_t)(kp * nqt + kq);
}

// Record of one packet in bin order: its q index and p-cell (relative) per
// dimension, then the per-dimension least-squares coefficients c_d[a*np+b]
// (after conjugation and shift), the first dimension's multiplied by
// scale * a exp(i S / eps).
template <int D> struct RecIdx { int32_t q[D], pc[D]; };
template <int D> __host__ __device__ constexpr int rec_idx_bytes() { return 16 * ((8 * D + 15) / 16); }
template <int D, int N1, typename T> __host__ __device__ constexpr int rec_bytes() {
  return rec_idx_bytes<D>() + D * N1 * (int)sizeof(T);
}

struct CoefParams {
  int64_t N;
  const double *Q, *P, *S, *a;
  double eps, scale;
  const DimLsq *lsq;  // [d], device copy of the plan
  int64_t Nq[3], pmin[3];
  double dq[3], dp[3];
};

template <int D, int N1, typename T>
__global__ __launch_bounds__(256) void fggc_coef_kernel(CoefParams p, const uint32_t *__restrict__ order,
                                                        char *__restrict__ recs) {
  using R = decltype(T{}.x);
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= p.N) return;
  const int64_t j = order[i];
  double cre[D][N1], cim[D][N1];
  int64_t iq[D], ip[D];
#pragma unroll
  for (int k = 0; k < D; ++k)
    dim_coeffs<N1>(p.lsq[k], p.Q[k * p.N + j], p.P[k * p.N + j], p.dq[k], p.dp[k], iq[k], ip[k],
                   cre[k], cim[k]);
  double sn, cs;
  {
    const double rev = p.S[j] / (kTwoPi * p.eps);
    sincospi(2.0 * (rev - rint(rev)), &sn, &cs);
  }
  const double ar = p.scale * p.a[2 * j], ai = p.scale * p.a[2 * j + 1];
  const double alr = ar * cs - ai * sn, ali = ar * sn + ai * cs;
  char *r = recs + i * (int64_t)rec_bytes<D, N1, T>();
  RecIdx<D> ri;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    ri.q[k] = (int32_t)((iq[k] + p.Nq[k] / 2) & (p.Nq[k] - 1));
    ri.pc[k] = (int32_t)(ip[k] - p.pmin[k]);
  }
  *reinterpret_cast<RecIdx<D> *>(r) = ri;
  T *c = reinterpret_cast<T *>(r + rec_idx_bytes<D>());
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
      c[k * N1 + m] = T{(R)xr, (R)xi};
    }
}

// Owner-computes accumulation of eq. (2.25): one workgroup per (p-slice,
// q-tile) of the cell array holds its cells in LDS, adds the contributions of
// every packet of the bins that can reach it, and writes each of its cells
// exactly once (no zeroing pass, no global atomics).
struct AccParams {
  const char *recs;
  const int64_t *start;
  int64_t sn[3], npc[3], Nq[3], tile[3], ntq[3];
  int nq, np;
  int dq[8], dp[8];
  int mindp, maxdp, mindq, maxdq;
  int bofs[32];  // dp value - mindp -> index b, or -1
};

template <int D, int N1, typename T>
__global__ __launch_bounds__(256) void fggc_accum_kernel(AccParams p, T *__restrict__ cells) {
  using R = decltype(T{}.x);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R *lre = reinterpret_cast<R *>(smem_raw);
  int64_t tcells = 1, nqt_all = 1, ncell_q = 1;
  for (int k = 0; k < D; ++k) {
    tcells *= p.tile[k];
    nqt_all *= p.ntq[k];
    ncell_q *= p.Nq[k];
  }
  R *lim = lre + tcells;
  for (int64_t e = threadIdx.x; e < tcells; e += blockDim.x) {
    lre[e] = 0;
    lim[e] = 0;
  }
  // which slice and q-tile this workgroup owns
  int64_t blk = blockIdx.x, tq[3] = {0, 0, 0}, sl[3] = {0, 0, 0};
  for (int k = D - 1; k >= 0; --k) {
    tq[k] = blk % p.ntq[k];
    blk /= p.ntq[k];
  }
  for (int k = D - 1; k >= 0; --k) {
    sl[k] = blk % p.sn[k];
    blk /= p.sn[k];
  }
  // packet p-cells that reach slice sl: pc in [sl + mindp - maxdp, sl], clipped
  int64_t pc0[3], pcn[3];
  // packet q bins that reach the tile: q in [t T - maxdq, t T + T - 1 - mindq] mod Nq
  int64_t ia[3][2], ic[3][2], ilen[3][2];
  int nint[3];
  for (int k = 0; k < 3; ++k) {
    pc0[k] = 0;
    pcn[k] = 1;
    nint[k] = 1;
    ia[k][0] = ic[k][0] = 0;
    ilen[k][0] = 1;
    ilen[k][1] = 0;
  }
  for (int k = 0; k < D; ++k) {
    int64_t a = sl[k] + p.mindp - p.maxdp, b = sl[k];
    if (a < 0) a = 0;
    if (b > p.npc[k] - 1) b = p.npc[k] - 1;
    pc0[k] = a;
    pcn[k] = b - a + 1;  // may be <= 0: nothing reaches this slice
    const int64_t nk = p.Nq[k], bw = p.tile[k], nb = p.ntq[k];
    const int64_t lo = tq[k] * bw - p.maxdq, hi = tq[k] * bw + bw - 1 - p.mindq;
    if (hi - lo + 1 >= nk) {
      ia[k][0] = 0;
      ic[k][0] = nb - 1;
    } else {
      const int64_t lm = ((lo % nk) + nk) % nk, hm = ((hi % nk) + nk) % nk;
      if (lm <= hm) {
        ia[k][0] = lm / bw;
        ic[k][0] = hm / bw;
      } else if (hm / bw + 1 >= lm / bw) {
        ia[k][0] = 0;
        ic[k][0] = nb - 1;
      } else {
        nint[k] = 2;
        ia[k][0] = lm / bw;
        ic[k][0] = nb - 1;
        ia[k][1] = 0;
        ic[k][1] = hm / bw;
      }
    }
    ilen[k][0] = ic[k][0] - ia[k][0] + 1;
    ilen[k][1] = nint[k] == 2 ? ic[k][1] - ia[k][1] + 1 : 0;
  }
  bool any = true;
  for (int k = 0; k < D; ++k) any = any && pcn[k] > 0;
  __syncthreads();
  if (any) {
    // enumerate packet p-cells x q-bin rows (all q dims but the last), runs in the last q dim
    int64_t npcs = 1, nqrows = 1, qcnt[3];
    for (int k = 0; k < D; ++k) {
      npcs *= pcn[k];
      qcnt[k] = ilen[k][0] + ilen[k][1];
    }
    for (int k = 0; k < D - 1; ++k) nqrows *= qcnt[k];
    const int kl = D - 1;
    constexpr int RB = rec_bytes<D, N1, T>();
    for (int64_t pcv = 0; pcv < npcs; ++pcv) {
      int64_t rem = pcv, pcf = 0, pcs[3];
      for (int k = D - 1; k >= 0; --k) {
        pcs[k] = pc0[k] + rem % pcn[k];
        rem /= pcn[k];
      }
      for (int k = 0; k < D; ++k) pcf = pcf * p.npc[k] + pcs[k];
      // the basis index b per dimension that lands this p-cell on the slice
      // (slice = pc + dp - mindp, so dp - mindp = slice - pc)
      int bsel[3];
      for (int k = 0; k < D; ++k) bsel[k] = p.bofs[(int)(sl[k] - pcs[k])];
      for (int64_t row = 0; row < nqrows; ++row) {
        int64_t rr = row, qb = 0, qidx[3] = {0, 0, 0};
        for (int k = D - 2; k >= 0; --k) {
          const int64_t r0 = rr % qcnt[k];
          rr /= qcnt[k];
          qidx[k] = r0 < ilen[k][0] ? ia[k][0] + r0 : ia[k][1] + (r0 - ilen[k][0]);
        }
        for (int k = 0; k < D - 1; ++k) qb = qb * p.ntq[k] + qidx[k];
        for (int run = 0; run < nint[kl]; ++run) {
          const int64_t b0 = (pcf * nqt_all) + qb * p.ntq[kl] + ia[kl][run];
          const int64_t b1 = (pcf * nqt_all) + qb * p.ntq[kl] + ic[kl][run] + 1;
          const int64_t s0 = p.start[b0], s1 = p.start[b1];
          for (int64_t r = s0 + threadIdx.x; r < s1; r += blockDim.x) {
            const char *rec = p.recs + r * (int64_t)RB;
            const RecIdx<D> ri = *reinterpret_cast<const RecIdx<D> *>(rec);
            const T *c = reinterpret_cast<const T *>(rec + rec_idx_bytes<D>());
            // local q offsets of this packet's neighbours inside the tile
            int lq[3][8];
            for (int k = 0; k < D; ++k)
              for (int a = 0; a < 8; ++a) {
                lq[k][a] = -1;
                if (a < p.nq) {
                  const int64_t qv = (ri.q[k] + p.dq[a] - tq[k] * p.tile[k] + 2 * p.Nq[k]) & (p.Nq[k] - 1);
                  if (qv < p.tile[k]) lq[k][a] = (int)qv;
                }
              }
            if (D == 1) {
              for (int a0 = 0; a0 < p.nq; ++a0) {
                if (lq[0][a0] < 0) continue;
                const T v = c[a0 * p.np + bsel[0]];
                atomicAdd(&lre[lq[0][a0]], v.x);
                atomicAdd(&lim[lq[0][a0]], v.y);
              }
            } else if (D == 2) {
              for (int a0 = 0; a0 < p.nq; ++a0) {
                if (lq[0][a0] < 0) continue;
                const T u = c[a0 * p.np + bsel[0]];
                for (int a1 = 0; a1 < p.nq; ++a1) {
                  if (lq[1][a1] < 0) continue;
                  const T w = c[N1 + a1 * p.np + bsel[1]];
                  const int64_t li = lq[0][a0] * p.tile[1] + lq[1][a1];
                  atomicAdd(&lre[li], u.x * w.x - u.y * w.y);
                  atomicAdd(&lim[li], u.x * w.y + u.y * w.x);
                }
              }
            } else {
              for (int a0 = 0; a0 < p.nq; ++a0) {
                if (lq[0][a0] < 0) continue;
                const T u = c[a0 * p.np + bsel[0]];
                for (int a1 = 0; a1 < p.nq; ++a1) {
                  if (lq[1][a1] < 0) continue;
                  const T w1 = c[N1 + a1 * p.np + bsel[1]];
                  const R ur = u.x * w1.x - u.y * w1.y, ui = u.x * w1.y + u.y * w1.x;
                  for (int a2 = 0; a2 < p.nq; ++a2) {
                    if (lq[2][a2] < 0) continue;
                    const T w2 = c[2 * N1 + a2 * p.np + bsel[2]];
                    const int64_t li = (lq[0][a0] * p.tile[1] + lq[1][a1]) * p.tile[2] + lq[2][a2];
                    atomicAdd(&lre[li], ur * w2.x - ui * w2.y);
                    atomicAdd(&lim[li], ur * w2.y + ui * w2.x);
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
  // write the tile: every cell of the array is owned by exactly one workgroup
  int64_t slf = 0;
  for (int k = 0; k < D; ++k) slf = slf * p.sn[k] + sl[k];
  T *dst = cells + slf * ncell_q;
  for (int64_t e = threadIdx.x; e < tcells; e += blockDim.x) {
    int64_t rem = e, q = 0, lo[3];
    for (int k = D - 1; k >= 0; --k) {
      lo[k] = rem % p.tile[k];
      rem /= p.tile[k];
    }
    for (int k = 0; k < D; ++k) q = q * p.Nq[k] + tq[k] * p.tile[k] + lo[k];
    dst[q] = T{lre[e], lim[e]};
  }
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

template <typename R>
__global__ void band_table_kernel(BandParams b, R *__restrict__ gam, int64_t *__restrict__ kst) {
  const int k = blockIdx.y;
  if (k >= b.d) return;
  const int64_t total = b.sn[k] * b.nb[k];
  const double se = sqrt(b.eps);
  const double cst = sqrt(kTwoPi * b.eps) / kTwoPi;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = e / b.nb[k], i = e - l * b.nb[k];
    const double p = (double)(b.slo[k] + l) * b.dp[k];
    const int64_t k0 = (int64_t)ceil(p / b.eps - b.cK / se);
    const double dk = b.eps * (double)(k0 + i) - p;  // eps (k - p/eps)
    const double ex = -dk * dk / (2.0 * b.eps);
    const double v = (ex >= -0.5 * b.cK * b.cK * (1.0 + 1e-12)) ? cst * exp(ex) : 0.0;
    gam[b.toff[k] + e] = (R)v;
    if (i == 0) kst[b.koff[k] + l] = k0;
  }
}

struct MacParams {
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

struct FggcLayout {
  int d, N1, rec_b;
  int64_t ncells, nslices, npts, nbins, tiles, ntq[3], tile[3], npc[3], pmin[3];
  int64_t nb[3], toff[3], koff[3], ntab, nkst;
  int mindp, maxdp, mindq, maxdq;
  size_t off_lsq, off_keys, off_order, off_sort, off_start, off_recs, off_cells, off_gam, off_kst,
      off_spec, total;
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
  static const int64_t deft[4] = {0, 32, 32, 16};
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
      L.tile[k] = std::min<int64_t>(a.Nq[k], deft[d]);
      L.ntq[k] = a.Nq[k] / L.tile[k];
      L.pmin[k] = a.slo[k] - L.mindp;
      L.npc[k] = a.sn[k] - (L.maxdp - L.mindp);
      L.nbins *= L.npc[k] * L.ntq[k];
      L.tiles *= a.sn[k] * L.ntq[k];
      L.nb[k] = (int64_t)std::floor(2.0 * a.cK / std::sqrt(a.eps)) + 2;
      L.toff[k] = L.ntab;
      L.koff[k] = L.nkst;
      L.ntab += a.sn[k] * L.nb[k];
      L.nkst += a.sn[k];
    } else {
      L.tile[k] = L.ntq[k] = L.npc[k] = 1;
      L.pmin[k] = 0;
      L.nb[k] = 1;
      L.toff[k] = 0;
      L.koff[k] = 0;
    }
  }
  if (L.nbins >= ((int64_t)1 << 32)) fail(FGGC_EUNSUPPORTED, "too many packet bins");
  L.ncells = L.nslices * nqt;
  const int64_t N = std::max<int64_t>(a.pk->N, 1);
  size_t o = 0;
  auto put = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.off_lsq = put(3 * sizeof(DimLsq));
  L.off_keys = put(N * 4);
  L.off_order = put(N * 4);
  L.off_sort = put(bucket_sort_bytes(a.pk->N, L.nbins));
  L.off_start = put((size_t)(L.nbins + 1) * 8);
  L.off_recs = put((size_t)N * L.rec_b);
  L.off_cells = put((size_t)L.ncells * es);
  L.off_gam = put((size_t)L.ntab * (es / 2));
  L.off_kst = put((size_t)L.nkst * 8 + 64);
  L.off_spec = put((size_t)L.npts * es);  // grid spectrum (the inverse FFT writes u from it)
  L.total = o;
  return L;
}

template <int D, int N1, typename T>
void launch_coef_accum(const FggcArgs &a, const FggcLayout &L, const CoefParams &cp,
                       const uint32_t *order, char *recs, const int64_t *start, T *cells,
                       hipStream_t s) {
  {
    StageScope sc(a.prof, "fggc_coef", s);
    fggc_coef_kernel<D, N1, T><<<dim3((unsigned)((cp.N + 255) / 256)), dim3(256), 0, s>>>(cp, order, recs);
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
  ap.mindq = L.mindq;
  ap.maxdq = L.maxdq;
  for (int i = 0; i < 32; ++i) ap.bofs[i] = -1;
  for (int b = 0; b < np; ++b) ap.bofs[ap.dp[b] - L.mindp] = b;
  int64_t tc = 1;
  for (int k = 0; k < D; ++k) tc *= L.tile[k];
  const size_t shm = 2 * (size_t)tc * sizeof(decltype(T{}.x));
  StageScope sc(a.prof, "fggc_accum", s);
  fggc_accum_kernel<D, N1, T><<<dim3((unsigned)L.tiles), dim3(256), shm, s>>>(ap, cells);
  FGGC_HIP(hipGetLastError());
}

// sort packets into bins, compute their coefficients in bin order, and fill
// the cell array of eq. (2.25) (every cell written once)
void cells_stage(const FggcArgs &a, const FggcLayout &L, char *base, void *cells, hipStream_t s) {
  const int d = a.g.d;
  const bool f64 = a.precision == FGGC_FP64;
  DimLsq *dlsq = (DimLsq *)(base + L.off_lsq);
  FGGC_HIP(hipMemcpyAsync(dlsq, a.lsq, d * sizeof(DimLsq), hipMemcpyHostToDevice, s));
  const int64_t N = a.pk->N;
  uint32_t *keys = (uint32_t *)(base + L.off_keys), *order = (uint32_t *)(base + L.off_order);
  int64_t *start = (int64_t *)(base + L.off_start);
  char *recs = base + L.off_recs;
  {
    StageScope sc(a.prof, "fggc_sort", s);
    if (N > 0) {
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
      const dim3 g((unsigned)((N + 255) / 256)), b(256);
      if (d == 1) fggc_key_kernel<1><<<g, b, 0, s>>>(kp, keys);
      else if (d == 2) fggc_key_kernel<2><<<g, b, 0, s>>>(kp, keys);
      else fggc_key_kernel<3><<<g, b, 0, s>>>(kp, keys);
      FGGC_HIP(hipGetLastError());
    }
    bucket_sort(keys, N, L.nbins, order, start, base + L.off_sort, s);
  }
  CoefParams cp{};
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
  if (f64) launch_coef_accum<DD, NN, double2>(a, L, cp, order, recs, start, (double2 *)cells, s); \
  else launch_coef_accum<DD, NN, float2>(a, L, cp, order, recs, start, (float2 *)cells, s);
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

template <typename T, typename R>
void finish_stage(const FggcArgs &a, const FggcLayout &L, T *cells, R *gam, int64_t *kst,
                  void *spec, Workspace &ws, hipStream_t s) {
  const int d = a.g.d;
  const int prec = a.precision;
  // F5: forward DFT over q of every p-slice
  launch_fft(d, a.Nq, L.nslices, -1, prec, cells, ws, s, a.prof, "fggc_fft_q");
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
  {
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
  {
  StageScope sc(a.prof, "fggc_band_mac", s);
  if (d == 1) band_mac_kernel<1, T, R><<<nblk, 256, 0, s>>>(m, cells, gam, kst, U);
  else if (d == 2) band_mac_kernel<2, T, R><<<nblk, 256, 0, s>>>(m, cells, gam, kst, U);
  else band_mac_kernel<3, T, R><<<nblk, 256, 0, s>>>(m, cells, gam, kst, U);
  FGGC_HIP(hipGetLastError());
  }
  // F7: inverse DFT of the grid spectrum into u
  launch_fft_to(d, a.g.n, +1, prec, U, a.u, ws, s, a.prof, "fggc_ifft");
}

}  // namespace

size_t fggc_workspace_bytes(const FggcArgs &a) { return fggc_layout(a).total + 1024; }

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
    finish_stage<double2, double>(a, L, (double2 *)cells, (double *)(base + L.off_gam),
                                  (int64_t *)(base + L.off_kst), base + L.off_spec, ws, s);
  else
    finish_stage<float2, float>(a, L, (float2 *)cells, (float *)(base + L.off_gam),
                                (int64_t *)(base + L.off_kst), base + L.off_spec, ws, s);
}

}  // namespace fggc
