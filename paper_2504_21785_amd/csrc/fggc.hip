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

#include <cmath>
#include <type_traits>

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

// x mod n in [0, n) (floor convention) for q-mesh indices of any mesh size;
// the common case, x already in range, costs one comparison
__device__ __forceinline__ int wrapq(int x, int n) {
  if ((unsigned)x < (unsigned)n) return x;
  x %= n;
  return x < 0 ? x + n : x;
}
__device__ __forceinline__ int64_t wrapq(int64_t x, int64_t n) {
  if ((uint64_t)x < (uint64_t)n) return x;
  x %= n;
  return x < 0 ? x + n : x;
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

// The same with the shift-set sizes fixed (basis j = a NP + b), up to a factor
// that every basis function of the packet shares.  With CC = Cq Cp, the
// smallest shifts dq0, dp0, x0 = dq0 - s, y0 = dp0 - t and the offsets
// Eq_a = dq_a - dq0, Ep_b = dp_b - dp0 (whole numbers >= 0), the Gaussian
// factor of (3.23) splits about (x0, y0) and the right-hand side becomes
//   f~_ab = W uq^Eq_a up^Ep_b DK_ab,
//   uq = exp(-Cq^2 x0 / 2) exp(-i CC t / 2),  up = exp(-Cp^2 y0 / 2) exp(i CC s / 2),
//   DK_ab = D_ab exp(-(Cq^2 Eq_a^2 + Cp^2 Ep_b^2) / 4)   (a plan constant),
//   W = exp(-(Cq^2 x0^2 + Cp^2 y0^2) / 4) exp(i CC (s t + s dp0 - t dq0) / 2),
// and the shift of (3.13) is exp(-i CC (s - dq0) ip) Fi^Eq_a with Fi = exp(i CC ip).
// The solve is linear and c~ = conj(c^), so W leaves it as conj(W); that and
// exp(-i CC (s - dq0) ip) are gathered, over all dimensions, into the one
// per-packet factor that common_factor() returns (log-magnitude and phase in
// revolutions).  What is left is computed here:
//   z = diag(inv) V^H g,  g_ab = uq^Eq_a up^Ep_b DK_ab;  c_ab = conj(V z)_ab Fi^Eq_a  (x alpha).
__device__ __forceinline__ void common_factor(const DimLsq &L, double s, double t, int64_t ip, double &lg,
                                              double &rev) {
  const double Cq = L.Cq, Cp = L.Cp, CC = Cq * Cp;
  const double x0 = (double)L.dq0 - s, y0 = (double)L.dp0 - t;
  lg -= 0.25 * (Cq * Cq * x0 * x0 + Cp * Cp * y0 * y0);
  rev -= CC * (0.5 * (s * t + s * (double)L.dp0 - t * (double)L.dq0) - x0 * (double)ip) * (1.0 / kTwoPi);
}

// A compiler fence between rows of a matrix product: loads are neither
// merged nor moved across it, and the running sums passed in are complete
// before it, so each row's loads and arithmetic stay together.
template <int N>
__device__ __forceinline__ void row_fence(double (&xr)[N], double (&xi)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) asm volatile("" : "+v"(xr[i]), "+v"(xi[i]));
  asm volatile("" ::: "memory");
}
__device__ __forceinline__ void row_fence(double &xr, double &xi) {
  asm volatile("" : "+v"(xr), "+v"(xi)::"memory");
}

// exp(i th) for |th| <= 0.5 from the Taylor series of cos and sin (through
// th^14 and th^15; the first omitted terms are below 3e-18 and 2e-19)
__device__ __forceinline__ void cis_small(double th, double &c, double &s) {
  const double x = th * th;
  double pc = 1.0 / 87178291200.0;           // 1/14!
  pc = fma(pc, -x, 1.0 / 479001600.0);       // 1/12!
  pc = fma(pc, -x, 1.0 / 3628800.0);         // 1/10!
  pc = fma(pc, -x, 1.0 / 40320.0);           // 1/8!
  pc = fma(pc, -x, 1.0 / 720.0);             // 1/6!
  pc = fma(pc, -x, 1.0 / 24.0);              // 1/4!
  pc = fma(pc, -x, 0.5);                     // 1/2!
  c = fma(pc, -x, 1.0);
  double ps = 1.0 / 1307674368000.0;         // 1/15!
  ps = fma(ps, -x, 1.0 / 6227020800.0);      // 1/13!
  ps = fma(ps, -x, 1.0 / 39916800.0);        // 1/11!
  ps = fma(ps, -x, 1.0 / 362880.0);          // 1/9!
  ps = fma(ps, -x, 1.0 / 5040.0);            // 1/7!
  ps = fma(ps, -x, 1.0 / 120.0);             // 1/5!
  ps = fma(ps, -x, 1.0 / 6.0);               // 1/3!
  s = th * fma(ps, -x, 1.0);
}

// z^n for a small whole n >= 0 (uniform across the wave)
__device__ __forceinline__ void cpow(double zr, double zi, int n, double &pr, double &pi) {
  double xr = 1.0, xi = 0.0;
  for (int k = 0; k < n; ++k) {
    const double t = xr * zr - xi * zi;
    xi = xr * zi + xi * zr;
    xr = t;
  }
  pr = xr;
  pi = xi;
}

template <int NQ, int NP, typename T>
__device__ __forceinline__ void dim_coeffs_exact(const DimLsq &L, double s, double t, int64_t ip, bool first,
                                                 double alr, double ali, T *cv) {
  using R = decltype(T{}.x);
  constexpr int N1 = NQ * NP;
  const double Cq = L.Cq, Cp = L.Cp, CC = Cq * Cp;
  constexpr double inv2pi = 1.0 / kTwoPi;
  double uqr, uqi, upr, upi, fir, fii;
  {
    // the angles CC t / 2 and CC s / 2 stay below CC / 2 (s, t in [0, 1))
    const bool small = CC <= 1.0;
    double c, sn;
    if (small) cis_small(-0.5 * CC * t, c, sn);
    else cis_rev(-0.5 * CC * t * inv2pi, c, sn);
    const double m = exp(-0.5 * Cq * Cq * ((double)L.dq0 - s));
    uqr = m * c;
    uqi = m * sn;
    if (small) cis_small(0.5 * CC * s, c, sn);
    else cis_rev(0.5 * CC * s * inv2pi, c, sn);
    const double mp = exp(-0.5 * Cp * Cp * ((double)L.dp0 - t));
    upr = mp * c;
    upi = mp * sn;
    cis_rev(CC * inv2pi * (double)ip, fir, fii);
  }
  double ppr[NP], ppi[NP];
#pragma unroll
  for (int b = 0; b < NP; ++b) cpow(upr, upi, L.dp[b] - L.dp0, ppr[b], ppi[b]);
  // z = diag(inv) V^H (DK .* h) = W^T h, accumulated one basis function at a
  // time (h_j is never stored); uq^Eq_a is kept as a running power over a
  double zr[N1], zi[N1];
#pragma unroll
  for (int i = 0; i < N1; ++i) zr[i] = zi[i] = 0.0;
  double pqr = 1.0, pqi = 0.0;
  int ea = 0;
#pragma unroll
  for (int a = 0; a < NQ; ++a) {
    {
      double xr, xi;
      const int e = L.dq[a * NP] - L.dq0;
      cpow(uqr, uqi, e - ea, xr, xi);
      const double nr = pqr * xr - pqi * xi;
      pqi = pqr * xi + pqi * xr;
      pqr = nr;
      ea = e;
    }
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      const int j = a * NP + b;
      const double hr = pqr * ppr[b] - pqi * ppi[b], hi = pqr * ppi[b] + pqi * ppr[b];
      // one row of W at a time: the compiler would otherwise load all of it
      // at once, at a cost in occupancy
      row_fence(zr, zi);
#pragma unroll
      for (int i = 0; i < N1; ++i) {
        const double wr = L.W[2 * (j * N1 + i)], wi = L.W[2 * (j * N1 + i) + 1];
        // W_ji h_j
        zr[i] = fma(wr, hr, fma(-wi, hi, zr[i]));
        zi[i] = fma(wr, hi, fma(wi, hr, zi[i]));
      }
    }
  }
  // c = conj(V z) Fi^Eq_a, Fi^Eq_a again as a running power over a
  pqr = 1.0;
  pqi = 0.0;
  ea = 0;
#pragma unroll
  for (int a = 0; a < NQ; ++a) {
    {
      double xr, xi;
      const int e = L.dq[a * NP] - L.dq0;
      cpow(fir, fii, e - ea, xr, xi);
      const double nr = pqr * xr - pqi * xi;
      pqi = pqr * xi + pqi * xr;
      pqr = nr;
      ea = e;
    }
#pragma unroll
    for (int b = 0; b < NP; ++b) {
      const int j = a * NP + b;
      double gr = 0.0, gi = 0.0;
#pragma unroll
      for (int i = 0; i < N1; ++i) {
        const double vr = L.V[2 * (j * N1 + i)], vi = L.V[2 * (j * N1 + i) + 1];
        gr = fma(vr, zr[i], fma(-vi, zi[i], gr));
        gi = fma(vr, zi[i], fma(vi, zr[i], gi));
        if (N1 > 4 && i == N1 / 2 - 1) row_fence(gr, gi);  // half a row of V in flight
      }
      row_fence(gr, gi);
      // conj(g) Fi^Eq_a
      double xr = gr * pqr + gi * pqi, xi = gr * pqi - gi * pqr;
      if (first) {
        const double nr = alr * xr - ali * xi;
        xi = alr * xi + ali * xr;
        xr = nr;
      }
      cv[j] = T{(R)xr, (R)xi};
    }
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
  // bin order: 0 = (p-cell, q-tile); 1 = (p-cells of the leading dimensions,
  // q-tile, p-cell of the last dimension), so that the bins of a run of
  // last-dimension p-cells are adjacent (the fused three-dimensional finish)
  int pc_last;
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
    const int64_t qi = wrapq(iq + p.Nq[k] / 2, p.Nq[k]);
    // the cell box comes from the same floor(P/dp), so this clamp never binds;
    // it keeps every key inside [0, nbins) whatever the caller's box
    int64_t pc = ip - p.pmin[k];
    pc = pc < 0 ? 0 : (pc >= p.npc[k] ? p.npc[k] - 1 : pc);
    pcf = pcf * p.npc[k] + pc;
    if (p.ns == 1) {
      ta[k] = tb[k] = qi / p.tile[k];
    } else {
      ta[k] = wrapq(qi + p.mindq, p.Nq[k]) / p.tile[k];
      tb[k] = wrapq(qi + p.maxdq, p.Nq[k]) / p.tile[k];
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
  const int64_t pch = p.pc_last ? pcf / p.npc[D - 1] : pcf, pcl = p.pc_last ? pcf % p.npc[D - 1] : 0,
                nl = p.pc_last ? p.npc[D - 1] : 1;
#pragma unroll
  for (int m = 0; m < NS; ++m) {
    bool ok = true;
    int64_t tf = 0;
    for (int k = 0; k < D; ++k) {
      const int bit = (m >> k) & 1;
      if (bit && tb[k] == ta[k]) ok = false;
      tf = tf * p.ntq[k] + (bit ? tb[k] : ta[k]);
    }
    key[m] = ok ? (uint32_t)((pch * nqt + tf) * nl + pcl) : kNoKey;
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
// counts bin-major into table[bin * G + chunk_column(g)] and the keys for the
// position pass.
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
  // U packets per thread and pass: their loads and key arithmetic are
  // independent, so they overlap instead of forming one latency chain
  constexpr int U = 4;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += U * (int64_t)blockDim.x) {
    uint32_t k[U][1 << D];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t ju = j + u * (int64_t)blockDim.x;
      if (ju < j1) packet_keys<D>(p, ju, k[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t ju = j + u * (int64_t)blockDim.x;
      if (ju >= j1) break;
      for (int m = 0; m < p.ns; ++m) {
        keys[ju * p.ns + m] = k[u][m];
        if (k[u][m] != kNoKey) rank[ju * p.ns + m] = atomicAdd(&cnt[k[u][m]], 1u);
      }
    }
  }
  __syncthreads();
  const int64_t col = chunk_column(blockIdx.x, G);
  for (int64_t b = threadIdx.x; b < nbins; b += blockDim.x) table[b * G + col] = cnt[b];
}

// Record of one packet (one per key slot, in bin order): its q index and p-cell (relative) per
// dimension, then the per-dimension least-squares coefficients c_d[a*np+b]
// (after conjugation and shift), the first dimension's multiplied by
// scale * a exp(i S / eps).
// In three dimensions the indices are 16-bit (q < 8192, and the layout
// refuses p-cell boxes wider than 65535), so that the index part of a record
// is one 16-byte word as in one and two dimensions.
template <int D> struct RecIdx { int32_t q[D], pc[D]; };
template <> struct RecIdx<3> { uint16_t q[3], pc[3]; };
template <int D> __host__ __device__ constexpr int rec_idx_bytes() {
  return 16 * (((int)sizeof(RecIdx<D>) + 15) / 16);
}
template <int D, int N1, typename T> __host__ __device__ constexpr int rec_bytes() {
  return rec_idx_bytes<D>() + D * N1 * (int)sizeof(T);
}

struct CoefParams {
  int ns;  // key slots per packet
  int64_t N;
  const double *Q, *P, *S, *a;
  double inv_2pi_eps, scale;  // 1 / (2 pi eps): S in revolutions
  const DimLsq *lsq;  // [d], device copy of the plan
  int64_t Nq[3], pmin[3];
  double dq[3], dp[3];
};

// One thread per packet, in packet order (coalesced reads); the record is
// written to the sorted position of each of the packet's key slots.
template <int D, int N1, int NQ, int NP, typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(D == 1 && N1 <= 8 && NQ > 0 ? 4 : 1))) void fggc_coef_kernel(CoefParams p, const uint32_t *__restrict__ pos,
                                                        char *__restrict__ recs) {
  using R = decltype(T{}.x);
  // the plan is staged in LDS and read as broadcasts, a row of V at a time,
  // rather than through scalar registers (which V overflows)
  __shared__ DimLsq sl[D];
  {
    // per dimension: the fields before V, and the n1 x n1 corners of V and W
    // in use (both are stored with row stride n1)
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const uint4 *src = reinterpret_cast<const uint4 *>(p.lsq + k);
      uint4 *dst = reinterpret_cast<uint4 *>(sl + k);
      const int n1 = p.lsq[k].n1;
      const int nv = (int)(offsetof(DimLsq, V) / 16) + n1 * n1, w0 = (int)(offsetof(DimLsq, W) / 16);
      for (int e = threadIdx.x; e < nv + n1 * n1; e += blockDim.x) {
        const int at = e < nv ? e : w0 + (e - nv);
        dst[at] = src[at];
      }
    }
    __syncthreads();
  }
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= p.N) return;
  constexpr int NS = 1 << D;
  constexpr int RB = rec_bytes<D, N1, T>();
  // the record of every key slot of the packet (kNoKey: none)
  uint32_t at[NS];
#pragma unroll
  for (int m = 0; m < NS; ++m) at[m] = m < p.ns ? pos[j * p.ns + m] : kNoKey;
  // three dimensions: records (112 bytes in FP32 with two shifts, so not
  // aligned to cache lines) of up to 128 coefficient bytes are assembled in
  // registers and written as whole 16-byte words, once per key slot (on the
  // 2^24-packet 256^3 workload 3.3 -> 2.5 ms); otherwise dimension by dimension, which
  // keeps the registers of the one- and two-dimensional kernels
  constexpr bool kStage = D == 3 && D * N1 * (int)sizeof(T) <= 128;
  T allc[kStage ? D * N1 : 1];
  auto put_coeffs = [&](int k, const T *cv) {
    if constexpr (kStage) {
#pragma unroll
      for (int n = 0; n < N1; ++n) allc[k * N1 + n] = cv[n];
    } else {
#pragma unroll
      for (int m = 0; m < NS; ++m) {
        if (at[m] == kNoKey) continue;
        T *c = reinterpret_cast<T *>(recs + (int64_t)at[m] * RB + rec_idx_bytes<D>()) + k * N1;
#pragma unroll
        for (int n = 0; n < N1; ++n) c[n] = cv[n];
      }
    }
  };
  int64_t iq[D], ip[D];
  if constexpr (NQ > 0) {
    // every dimension's cell first: the per-packet factor spans them
    double s[D], t[D];
    double lg = 0.0, rev = p.S[j] * p.inv_2pi_eps;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      int_frac(p.Q[k * p.N + j] / p.dq[k], iq[k], s[k]);
      int_frac(p.P[k * p.N + j] / p.dp[k], ip[k], t[k]);
      common_factor(sl[k], s[k], t[k], ip[k], lg, rev);
    }
    double cs, sn;
    cis_rev(rev, cs, sn);
    const double m = p.scale * exp(lg);
    const double ar = m * p.a[2 * j], ai = m * p.a[2 * j + 1];
    const double alr = ar * cs - ai * sn, ali = ar * sn + ai * cs;
    // each dimension's coefficients go out as soon as they are known, so
    // that only one dimension's are held at a time
#pragma unroll
    for (int k = 0; k < D; ++k) {
      T cv[N1];
      dim_coeffs_exact<NQ, NP, T>(sl[k], s[k], t[k], ip[k], k == 0, alr, ali, cv);
      put_coeffs(k, cv);
    }
  } else {
    double cre[D][N1], cim[D][N1];
#pragma unroll
    for (int k = 0; k < D; ++k) {
      const double qv = p.Q[k * p.N + j], pv = p.P[k * p.N + j];
      dim_coeffs<N1>(sl[k], qv, pv, p.dq[k], p.dp[k], iq[k], ip[k], cre[k], cim[k]);
    }
    double sn, cs;
    cis_rev(p.S[j] * p.inv_2pi_eps, cs, sn);
    const double ar = p.scale * p.a[2 * j], ai = p.scale * p.a[2 * j + 1];
    const double alr = ar * cs - ai * sn, ali = ar * sn + ai * cs;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      T cv[N1];
#pragma unroll
      for (int n = 0; n < N1; ++n) {
        double xr = cre[k][n], xi = cim[k][n];
        if (k == 0) {
          const double nr = alr * xr - ali * xi;
          xi = alr * xi + ali * xr;
          xr = nr;
        }
        cv[n] = T{(R)xr, (R)xi};
      }
      put_coeffs(k, cv);
    }
  }
  RecIdx<D> ri;
#pragma unroll
  for (int k = 0; k < D; ++k) {
    // (narrowed to the record's index type: 16-bit in three dimensions)
    ri.q[k] = static_cast<std::remove_reference_t<decltype(ri.q[k])>>(wrapq(iq[k] + p.Nq[k] / 2, p.Nq[k]));
    ri.pc[k] = static_cast<std::remove_reference_t<decltype(ri.pc[k])>>(ip[k] - p.pmin[k]);
  }
  if constexpr (kStage) {
    constexpr int NW = RB / 16;
    uint4 w[NW];
#pragma unroll
    for (int v = 0; v < NW; ++v) w[v] = make_uint4(0, 0, 0, 0);
    __builtin_memcpy(&w[0], &ri, sizeof(ri));
    __builtin_memcpy(reinterpret_cast<char *>(w) + rec_idx_bytes<D>(), allc, sizeof(allc));
#pragma unroll
    for (int m = 0; m < NS; ++m) {
      if (at[m] == kNoKey) continue;
      uint4 *dst = reinterpret_cast<uint4 *>(recs + (int64_t)at[m] * RB);
#pragma unroll
      for (int v = 0; v < NW; ++v) dst[v] = w[v];
    }
  } else {
#pragma unroll
    for (int m = 0; m < NS; ++m)
      if (at[m] != kNoKey) *reinterpret_cast<RecIdx<D> *>(recs + (int64_t)at[m] * RB) = ri;
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
  // two dimensions: per (slice, q-tile) emptiness; an empty tile is not
  // written (null: every tile is written)
  uint8_t *empty;
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
              const int64_t qv = wrapq(ri.q[k] + p.dq[a] - tq[k] * p.tile[k], p.Nq[k]);
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
    const int nqk = (int)p.Nq[k], tl = (int)p.tile[k];
#pragma unroll
    for (int a = 0; a < NQ; ++a) {
      const int qv = wrapq(ri.q[k] + p.dq[a] - tq0[k], nqk);
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

// Accumulation without atomics (d = 2, 3): one wave per (slice, q-tile); the
// tile lives in LDS as interleaved complex values and is updated with plain
// read-modify-writes.  Each lane first picks, per dimension, the one p-shift
// that lands its record on the slice and the coefficients at it, so that
// every lane runs the same n_q^d contributions.  Two lanes can hit the same
// cell in one instruction only when their records share the q-cell; before
// adding, lanes claim an LDS hash slot of it and only the lane that holds its
// slot adds in this pass, the others in later passes -- so each pass writes
// distinct cells.
constexpr int kHashSlots = 512;

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
  const int tile1 = D > 1 ? (int)p.tile[1] : 1, tile2 = D > 2 ? (int)p.tile[2] : 1;
  __syncthreads();
  bool any_rec = false;
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
    any_rec = any_rec || total > 0;
    // record i of this pass (zeros past the end)
    auto load = [&](int64_t i, uint4 (&r)[NV]) {
      if (i < total) {
        int lo = 0, hi = nb - 1;  // last bin with s_pre[bin] <= i
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (s_pre[mid] <= i) lo = mid;
          else hi = mid - 1;
        }
        const uint4 *src = reinterpret_cast<const uint4 *>(p.recs + (s_r0[lo] + (i - s_pre[lo])) * (int64_t)RB);
#pragma unroll
        for (int v = 0; v < NV; ++v) r[v] = src[v];
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) r[v] = make_uint4(0, 0, 0, 0);
      }
    };
    // small records: the next chunk's loads are issued before this chunk is
    // accumulated, so that their latency overlaps the LDS work
    constexpr bool kAhead = NV <= 10;
    uint4 nxt[kAhead ? NV : 1];
    if constexpr (kAhead) load(lane, nxt);
    for (int64_t base = 0; base < total; base += 64) {
      const int64_t i = base + lane;
      const bool valid = i < total;
      uint4 raw[NV];
      if constexpr (kAhead) {
#pragma unroll
        for (int v = 0; v < NV; ++v) raw[v] = nxt[v];
        if (base + 64 < total) load(i + 64, nxt);
      } else {
        load(i, raw);
      }
      const RecIdx<D> ri = *reinterpret_cast<const RecIdx<D> *>(raw);
      const T *c = reinterpret_cast<const T *>(reinterpret_cast<const char *>(raw) + rec_idx_bytes<D>());
      int lq[D][NQ];
      // the p-shift of each dimension that lands on this slice (at most one:
      // the window is one slice), and the coefficients at it
      int bsel[D];
      uint32_t h = 0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const int nqk = (int)p.Nq[k], tl = (int)p.tile[k];
#pragma unroll
        for (int a = 0; a < NQ; ++a) {
          const int qv = wrapq(ri.q[k] + p.dq[a] - tq0[k], nqk);
          lq[k][a] = qv < tl ? qv : -1;
        }
        bsel[k] = -1;
#pragma unroll
        for (int b = 0; b < NP; ++b)
          if ((int64_t)ri.pc[k] + p.dp[b] - p.mindp == sl[k]) bsel[k] = b;
        h = h * 0x9E3779B1u + (uint32_t)ri.q[k] * 0x85EBCA77u;
      }
      h = (h ^ (h >> 15)) & (kHashSlots - 1);
      bool reach = true;
      T cu[D][NQ];
#pragma unroll
      for (int k = 0; k < D; ++k) {
        reach = reach && bsel[k] >= 0;
#pragma unroll
        for (int a = 0; a < NQ; ++a) {
          cu[k][a] = T{0, 0};
#pragma unroll
          for (int b = 0; b < NP; ++b)
            if (b == bsel[k]) cu[k][a] = c[k * N1 + a * NP + b];
        }
      }
      // passes: the loop condition is wave-uniform; the barriers (a single
      // wave here) order the claims and the cell updates between lanes.  One
      // instruction fixes the q-shifts, so two lanes write the same cell in it
      // only if their records share the q-cell: the claims are keyed by q-cell.
      // an LDS-qualified pointer: a generic volatile one is accessed with
      // flat instructions that wait on the vector memory counter
      volatile __attribute__((address_space(3))) int *claim = (volatile __attribute__((address_space(3))) int *)s_claim;
      bool todo = valid && reach;
      while (__ballot(todo)) {
        if (todo) claim[h] = lane;
        __syncthreads();
        const bool win = todo && claim[h] == lane;
        if (win) {
          todo = false;
          if constexpr (D == 1) {
#pragma unroll
            for (int a = 0; a < NQ; ++a) {
              if (lq[0][a] < 0) continue;
              const T v = cu[0][a];
              T o = tile[lq[0][a]];
              o.x += v.x;
              o.y += v.y;
              tile[lq[0][a]] = o;
            }
          } else if constexpr (D == 2) {
#pragma unroll
            for (int a0 = 0; a0 < NQ; ++a0) {
              if (lq[0][a0] < 0) continue;
              const T u = cu[0][a0];
#pragma unroll
              for (int a1 = 0; a1 < NQ; ++a1) {
                if (lq[1][a1] < 0) continue;
                const T v = cu[1][a1];
                const int li = lq[0][a0] * tile1 + lq[1][a1];
                T o = tile[li];
                o.x += u.x * v.x - u.y * v.y;
                o.y += u.x * v.y + u.y * v.x;
                tile[li] = o;
              }
            }
          } else {
#pragma unroll
            for (int a0 = 0; a0 < NQ; ++a0) {
              if (lq[0][a0] < 0) continue;
              const T u = cu[0][a0];
#pragma unroll
              for (int a1 = 0; a1 < NQ; ++a1) {
                if (lq[1][a1] < 0) continue;
                const T v = cu[1][a1];
                const T uv = T{u.x * v.x - u.y * v.y, u.x * v.y + u.y * v.x};
#pragma unroll
                for (int a2 = 0; a2 < NQ; ++a2) {
                  if (lq[2][a2] < 0) continue;
                  const T w = cu[2][a2];
                  const int li = (lq[0][a0] * tile1 + lq[1][a1]) * tile2 + lq[2][a2];
                  T o = tile[li];
                  o.x += uv.x * w.x - uv.y * w.y;
                  o.y += uv.x * w.y + uv.y * w.x;
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
  if (p.empty) {  // an empty tile is only marked (the finish reads it as zeros)
    if (lane == 0) p.empty[slf * nqt_all + tflat] = any_rec ? 0 : 1;
    if (!any_rec) return;
  }
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

// One dimension, without float atomics.  Packets of one (p-cell, q-cell) add
// to the same cells with the same shifts, so their coefficient vectors can be
// summed first:
//   aggregate  one workgroup per bin (p-cell, q-tile).
//              The bin's records pass through LDS in chunks; an LDS counting
//              sort (integer atomics) groups each chunk by q-cell, and thread
//              (q-cell, m) adds coefficient m of its q-cell's records into a
//              register, so A[p-cell][q-cell][m] is written once;
//   stencil    cells[s][q] = sum over b, a of A[s + mindp - dp_b][q - dq_a][a np + b]
//              (eq. 2.25 with the shifts applied on the aggregated vectors).
// The order of the terms inside a q-cell follows the sort (unspecified), so
// the sums may differ from call to call at the rounding level.
struct Agg1Params {
  const char *recs;
  const int64_t *start;
  int64_t Nq, tile, ntq, npc;
  int splits;  // workgroups per bin, each with its share of the records and its own copy of A
};

constexpr int kAggThreads = 256;
// q-cells per one-dimensional bin (the sort's q-tile): fewer, larger bins make
// the counting sort cheaper, more bins give the aggregate more workgroups
constexpr int kAgg1Tile = 32;

// records per LDS chunk: up to 256, at most ~40 KB
template <int RB> __host__ __device__ constexpr int agg1_chunk() {
  return RB * 256 <= 40960 ? 256 : (RB * 128 <= 40960 ? 128 : 64);
}

template <int N1, typename T, int TILE>
__global__ __launch_bounds__(kAggThreads) void fggc_agg1_kernel(Agg1Params p, T *__restrict__ A) {
  using R = decltype(T{}.x);
  constexpr int RB = rec_bytes<1, N1, T>();
  static_assert(RB % 16 == 0 && rec_idx_bytes<1>() == 16, "records are whole 16-byte words");
  constexpr int W = RB / 16, CH = agg1_chunk<RB>();
  constexpr int PAIRS = TILE * N1, PER = (PAIRS + kAggThreads - 1) / kAggThreads;
  static_assert(CH <= kAggThreads, "one record per thread and chunk");
  static_assert(TILE <= 128 && kAggThreads >= TILE, "at most two waves scan the histogram");
  __shared__ uint4 rs[CH * W];
  __shared__ int hist[TILE], incl[TILE];
  __shared__ uint16_t perm[CH];
  const int tid = threadIdx.x;
  const int64_t bin = blockIdx.x / p.splits;
  const int sp = (int)(blockIdx.x - bin * p.splits);
  const int64_t pc = bin / p.ntq, t = bin - pc * p.ntq;
  const int tbase = (int)(t * p.tile);
  const int64_t b0 = p.start[bin], nrec = p.start[bin + 1] - b0;
  const int64_t r0 = b0 + nrec * sp / p.splits, r1 = b0 + nrec * (sp + 1) / p.splits;
  const uint4 *src = reinterpret_cast<const uint4 *>(p.recs);
  A += (int64_t)sp * p.npc * p.Nq * N1;
  R accr[PER], acci[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) accr[i] = acci[i] = 0;
  if (tid < TILE) hist[tid] = 0;
  for (int64_t c0 = r0; c0 < r1; c0 += CH) {
    const int cnt = (int)min<int64_t>(CH, r1 - c0);
    for (int w = tid; w < cnt * W; w += kAggThreads) rs[w] = src[c0 * W + w];
    __syncthreads();
    int ql = 0, rk = 0;
    if (tid < cnt) {
      // the record's q-cell lies in this bin's tile by construction of the
      // keys; the clamp only keeps the LDS indexes in range
      ql = reinterpret_cast<const int32_t *>(&rs[tid * W])[0] - tbase;
      ql = ql < 0 ? 0 : (ql >= TILE ? TILE - 1 : ql);
      rk = atomicAdd(&hist[ql], 1);
    }
    __syncthreads();
    if (tid < TILE) {  // inclusive scan within each wave
      int v = hist[tid];
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int u = __shfl_up(v, d, 64);
        if ((tid & 63) >= d) v += u;
      }
      incl[tid] = v;
    }
    __syncthreads();
    // first position of q-cell q in the chunk's grouped order
    auto first = [&](int q) {
      if constexpr (TILE > 64) return incl[q] - hist[q] + (q >= 64 ? incl[63] : 0);
      else return incl[q] - hist[q];
    };
    if (tid < cnt) perm[first(ql) + rk] = (uint16_t)tid;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * kAggThreads;
      if (e < PAIRS) {
        const int q = e / N1, m = e - (e / N1) * N1;
        const int b = first(q), n = hist[q];
        for (int k = 0; k < n; ++k) {
          const T v = reinterpret_cast<const T *>(&rs[perm[b + k] * W + 1])[m];
          accr[i] += v.x;
          acci[i] += v.y;
        }
      }
    }
    __syncthreads();
    if (tid < TILE) hist[tid] = 0;
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = tid + i * kAggThreads;
    if (e < PAIRS) {
      const int q = e / N1, m = e - (e / N1) * N1;
      if (q < p.tile) A[(pc * p.Nq + tbase + q) * N1 + m] = T{accr[i], acci[i]};
    }
  }
}

struct Stencil1Params {
  int64_t Nq, sn, npc;
  int n1, nq, np, mindp;
  int dq[8], dp[8];
  int splits;  // copies of A to add
};

template <typename T>
__device__ __forceinline__ T stencil1_cell(const Stencil1Params &p, const T *__restrict__ A, int n1s,
                                           int64_t sl, int64_t q) {
  using R = decltype(T{}.x);
  R ar = 0, ai = 0;
  for (int b = 0; b < p.np; ++b) {
    const int64_t pc = sl + p.mindp - p.dp[b];
    if (pc < 0 || pc >= p.npc) continue;
    for (int a = 0; a < p.nq; ++a) {
      const int64_t qs = wrapq(q - p.dq[a], p.Nq);
      for (int c = 0; c < p.splits; ++c) {
        const T v = A[((c * p.npc + pc) * p.Nq + qs) * n1s + a * p.np + b];
        ar += v.x;
        ai += v.y;
      }
    }
  }
  return T{ar, ai};
}

template <typename T>
__global__ void fggc_stencil1_kernel(Stencil1Params p, const T *__restrict__ A, int n1s,
                                     T *__restrict__ cells) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= p.sn * p.Nq) return;
  const int64_t sl = e / p.Nq;
  cells[e] = stencil1_cell(p, A, n1s, sl, e - sl * p.Nq);
}

// The stencil and the forward DFT over q of one slice per workgroup (eq. 2.25,
// then the first step of the Fourier finish): the slice's cells are built in
// LDS, transformed there and written once as their spectrum.
template <typename T>
__global__ __launch_bounds__(256) void fggc_stencil_fft1_kernel(Stencil1Params p, const T *__restrict__ A,
                                                                int n1s, int lgN, const T *__restrict__ tw,
                                                                T *__restrict__ spec) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T *row = reinterpret_cast<T *>(smem_raw);
  const int64_t sl = blockIdx.x;
  const int N = (int)p.Nq;  // 2^lgN, or any 2^a 3^b 5^c when lgN < 0
  T *stw = row + N;  // the twiddles, staged in LDS
  for (int q = threadIdx.x; q < N; q += blockDim.x) {
    row[q] = stencil1_cell(p, A, n1s, sl, q);
    stw[q] = tw[q];
  }
  __syncthreads();
  if (lgN >= 0) lds_fft_rows<T>(row, lgN, 1, N, 0, stw);
  else lds_fft_rows_mr<T, 16>(row, N, 1, N, 0, stw);
  T *dst = spec + sl * N;
  for (int q = threadIdx.x; q < N; q += blockDim.x) dst[q] = row[q];
}

// First frequency of slice l's band, and gamma at frequency k (0 outside the
// truncated band).
__device__ __forceinline__ int64_t band_start(double p, double eps, double cK) {
  return (int64_t)ceil(p / eps - cK / sqrt(eps));
}
__device__ __forceinline__ double band_gamma(double p, int64_t k, double eps, double cK) {
  const double cst = sqrt(kTwoPi * eps) / kTwoPi;
  const double dk = eps * (double)k - p;  // eps (k - p/eps)
  const double ex = -dk * dk / (2.0 * eps);
  return (ex >= -0.5 * cK * cK * (1.0 + 1e-12)) ? cst * exp(ex) : 0.0;
}

struct MacParams {
  double dp[3];
  int64_t M[3], Nq[3], sn[3], nb[3];
  int64_t kmin[3], kmax[3];  // union of the bands per dimension
  double lo_c[3], inv_dp[3], eps, cK;  // l range helpers
  int64_t slo[3];
};

// One dimension: eight lanes per frequency split the slice loop, then a
// shuffle reduction (FP64) -- eight times the waves of the plain kernel.
template <typename T, typename R>
__global__ __launch_bounds__(256) void band_mac1_kernel(MacParams m, const T *__restrict__ F,
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
        // gamma evaluated in place, rounded to the record precision
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
  int N, lgN, lgWA, lgW;  // q-line length (and its log2 when a power of two); lines of consecutive a and of
                         // consecutive b per workgroup
  int Lc;              // slices per LDS chunk
  int MS;              // workgroups sharing one line group, each with a share of the frequencies
  int64_t kmin, kmax;  // union of the slices' bands (grid frequencies before aliasing)
  int64_t slo;
  double eps, dp, cK;
  // two dimensions, pass over the cells: per (slice, q-tile) emptiness; an
  // empty tile was not written and reads as zeros (null: read everything)
  const uint8_t *empty;
  int64_t ntq0, ntq1;
  int lgt0, lgt1;  // log2 of the q-tile sizes
};

constexpr int kContractThreads = 512;
constexpr int kContractBfly = 4;  // butterflies per thread and FFT pass
constexpr int kContractOut = 4;   // outputs per thread (2048 per workgroup)
constexpr int kContractFlags = 4096;  // (row, q-tile) emptiness flags of one chunk (<= 4096 / tile)

// One pass of the separable finish over dimension k of the cell array (or of
// the previous pass's output), viewed as X[O][L][A][N][B]:
//   Y[o][a][k'][b] = sum_l sum_{kk = k' (mod M)} gamma_l(kk) F_{o,l,a,b}[kk mod N],
// F the length-N DFT over n of X[o][l][a][.][b] and gamma_l the band of slice
// l in this dimension (eq. 2.24 factors over dimensions; kk runs over the
// truncated band |kk - p_l/eps| <= cK/sqrt(eps)).  A workgroup loads chunks of
// Lc slices of its 2^lgWA x 2^lgW lines into LDS, transforms them there and
// adds each slice's band into per-thread FP64 sums of its outputs; gamma is
// evaluated in place.  Frequencies no band reaches are written as zeros.
// MR: q-lines of any length 2^a 3^b 5^c (mixed-radix passes, general
// indexing); otherwise powers of two (shifts and masks).
template <typename T, typename R, bool MR>
__global__ __launch_bounds__(kContractThreads) void fft_contract_kernel(ContractParams p, const T *__restrict__ X,
                                                           T *__restrict__ Y, const T *__restrict__ tw) {
  using RR = decltype(T{}.x);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  __shared__ uint8_t s_empty[kContractFlags];
  T *sm = reinterpret_cast<T *>(smem_raw);
  const int lgN = p.lgN, N = MR ? p.N : 1 << lgN, WA = 1 << p.lgWA, W = 1 << p.lgW, P = WA * W;
  const int M = (int)p.M;
  const int64_t nbc = p.B >> p.lgW, nac = p.A >> p.lgWA;
  T *stw = sm + (size_t)p.Lc * P * N;  // the twiddles, staged in LDS
  for (int i = threadIdx.x; i < N; i += blockDim.x) stw[i] = tw[i];
  int64_t g = blockIdx.x;
  const int mg = (int)(g % p.MS);
  g /= p.MS;
  const int64_t bc = g % nbc;
  g /= nbc;
  const int64_t ac = g % nac, o = g / nac;
  const int64_t b0 = bc << p.lgW, a0 = ac << p.lgWA;
  // frequencies in band order t = (k' - kmin) mod M: the first nact reach a
  // band; this workgroup takes t in [t0, t0 + Mg)
  const int nact = (int)min<int64_t>(M, p.kmax - p.kmin + 1);
  const int Mg = (M + p.MS - 1) / p.MS, t0 = mg * Mg;
  const int Mgt = max(0, min(Mg, M - t0));     // this workgroup's share (the last may be short)
  const int na = max(0, min(Mgt, nact - t0));  // active frequencies of this workgroup
  const int nown = na * P;
  const int kmod = (int)(((p.kmin % M) + M) % M);
  double accr[kContractOut], acci[kContractOut];
#pragma unroll
  for (int c = 0; c < kContractOut; ++c) accr[c] = acci[c] = 0.0;
  const double cst = sqrt(kTwoPi * p.eps) / kTwoPi, cut = -0.5 * p.cK * p.cK * (1.0 + 1e-12);
  const double inv2e = 1.0 / (2.0 * p.eps);
  for (int lc0 = 0; lc0 < (int)p.L; lc0 += p.Lc) {
    const int lcn = min(p.Lc, (int)p.L - lc0);
    // rows [l][wa][w] of N, loaded with b fastest, then n, then a
    const int tot = lcn * P * N;
    if (p.empty) {
      // the chunk's (row, q1-tile) emptiness into LDS (rows [l][wa]; one b),
      // and a chunk of empty tiles adds nothing: skip it
      const int nf = lcn * WA * (int)p.ntq1;
      int any = 0;
      for (int f = threadIdx.x; f < nf; f += blockDim.x) {
        const int t1 = f % (int)p.ntq1, r = f / (int)p.ntq1;
        const int wa = r & (WA - 1), l = r >> p.lgWA;
        const int64_t slf = o * p.L + lc0 + l;  // cells of [slice][q0 = a][q1 = n]
        const uint8_t e = p.empty[(slf * p.ntq0 + ((a0 + wa) >> p.lgt0)) * p.ntq1 + t1];
        s_empty[f] = e;
        any |= e == 0;
      }
      if (!__syncthreads_or(any)) continue;
    }
    for (int e = threadIdx.x; e < tot; e += blockDim.x) {
      const int en = e >> p.lgW;
      const int w = e & (W - 1), n = MR ? en % N : en & (N - 1), rest = MR ? en / N : en >> lgN;
      const int wa = rest & (WA - 1), l = rest >> p.lgWA;
      const int row = (((l << p.lgWA) + wa) << p.lgW) + w;
      const bool full = !p.empty || !s_empty[((l << p.lgWA) + wa) * (int)p.ntq1 + (n >> p.lgt1)];
      sm[row * N + n] = full ? X[(((o * p.L + lc0 + l) * p.A + a0 + wa) * N + n) * p.B + b0 + w] : T{0, 0};
    }
    __syncthreads();
    if constexpr (MR) lds_fft_rows_mr<T, 2 * kContractBfly>(sm, N, lcn * P, N, 0, stw);
    else lds_fft_rows<T, kContractBfly>(sm, lgN, lcn * P, N, 0, stw);
#pragma unroll
    for (int c = 0; c < kContractOut; ++c) {
      const int e = threadIdx.x + c * (int)blockDim.x;
      if (e >= nown) break;
      // e = (wa, t, w) with w fastest (coalesced along b), then t
      const int w = e & (W - 1), rest = e >> p.lgW;
      const int t = rest % na, wa = rest / na;
      const T *rows = sm + ((wa << p.lgW) + w) * N;  // slice l at rows + l * P * N
      double xr = 0.0, xi = 0.0;
      for (int64_t kk = p.kmin + t0 + t; kk <= p.kmax; kk += M) {
        const T *fq = rows + (MR ? (int)wrapq(kk, (int64_t)N) : (int)(kk & (N - 1)));
        const double dk0 = p.eps * (double)kk - (double)(p.slo + lc0) * p.dp;
        for (int l = 0; l < lcn; ++l) {
          const double dk = dk0 - (double)l * p.dp;  // eps (kk - p_l / eps)
          const double ex = -dk * dk * inv2e;
          if (ex < cut) continue;
          double gv;
          if constexpr (sizeof(R) == 4) gv = (double)(float)(cst * (double)__expf((float)ex));
          else gv = cst * exp(ex);
          const T v = fq[l * P * N];
          xr = fma(gv, (double)v.x, xr);
          xi = fma(gv, (double)v.y, xi);
        }
      }
      accr[c] += xr;
      acci[c] += xi;
    }
    __syncthreads();
  }
#pragma unroll
  for (int c = 0; c < kContractOut; ++c) {
    const int e = threadIdx.x + c * (int)blockDim.x;
    if (e >= nown) break;
    const int w = e & (W - 1), rest = e >> p.lgW;
    const int t = rest % na, wa = rest / na;
    const int kp = (kmod + t0 + t) % M;
    Y[((o * p.A + a0 + wa) * p.M + kp) * p.B + b0 + w] = T{(RR)accr[c], (RR)acci[c]};
  }
  // frequencies of this workgroup's share that no band reaches
  const int nz = (Mgt - na) * P;
  for (int e = threadIdx.x; e < nz; e += blockDim.x) {
    const int w = e & (W - 1), rest = e >> p.lgW;
    const int t = na + rest % (Mgt - na), wa = rest / (Mgt - na);
    const int kp = (kmod + t0 + t) % M;
    Y[((o * p.A + a0 + wa) * p.M + kp) * p.B + b0 + w] = T{0, 0};
  }
}

// Three dimensions: the accumulation of eq. (2.25) fused with the separable
// pass over the last dimension, so that the dense cell array never exists.
// One workgroup owns the q-lines (q0, q1) of one q-tile of dimensions 0 and 1
// at one slice pair (l0, l1), over every q2 and every slice l2.  For Lc slices
// l2 at a time it
//   - adds the Kronecker contributions of the packets that reach its lines
//     into those lines in LDS (one slice per wave, plain read-modify-writes;
//     the order of the terms in a cell follows the sort, so sums may differ
//     at the rounding level),
//   - transforms the lines over q2 in LDS,
//   - folds the slices into the grid frequencies m2 with the band weights
//     gamma_l2 (tabulated once per call, staged per chunk; sums per thread in
//     the working precision: an output gathers one term per slice and alias),
// and finally writes what the pass over the last dimension writes,
// Y[l0][l1][q0][q1][m2] (zeros at frequencies no band reaches).  Packets are
// binned by (p-cell 0, p-cell 1, q-tile, p-cell 2), so the records that reach
// a chunk are one contiguous run per (p-cell 0, p-cell 1).
// arr[i] for a run-time i, by selects (the array stays in registers)
template <int K, typename V> __device__ __forceinline__ V pick(const V (&arr)[K], int i) {
  V v = arr[0];
#pragma unroll
  for (int k = 1; k < K; ++k)
    if (i == k) v = arr[k];
  return v;
}

constexpr int kFusedThreads = 512;
constexpr int kFusedOut = 8;   // outputs per thread
constexpr int kFusedRuns = 16; // (p-cell 0, p-cell 1) pairs that reach a slice pair: (p-shift span + 1)^2
constexpr size_t kFusedMaxLds = 144 * 1024;  // dynamic LDS (the kernel's static LDS comes on top)
constexpr int kFusedClaimBits = 8;
constexpr int kFusedClaim = 1 << kFusedClaimBits;  // claim slots per wave

struct Fused3Params {
  const char *recs;
  const int64_t *start;
  int64_t sn[3], npc[3], Nq[3];
  int64_t ntq0, ntq1;  // q-tiles of dimensions 0 and 1 (a tile is T0 x T1 x Nq2)
  int T0, T1, lgN, Lc, TPL;
  int dq[8], dp[8];
  int mindp, maxdp;
  int64_t M, kmin, kmax, slo;  // last dimension: grid points, band union, first slice
  double eps, dp2, cK;
  const double *gtab;  // [sn2][kmax - kmin + 1] band weights (band_table_kernel)
};

// Band weights of one dimension, once per call (the fused finish and the
// dense passes): gtab[l][t] = gamma_l(kmin + t) =
// sqrt(2 pi eps) / (2 pi) exp(-eps (k - p_l / eps)^2 / 2), p_l = (slo + l) dp,
// zero outside the truncated band |k - p_l / eps| <= cK / sqrt(eps).
__global__ void band_table_kernel(int64_t L, int64_t kmin, int64_t kmax, int64_t slo, double eps, double dp,
                                  double cK, double *__restrict__ gtab) {
  const int ng = (int)(kmax - kmin + 1);
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= L * ng) return;
  const int64_t l = e / ng, t = e - l * ng;
  const double cst = sqrt(kTwoPi * eps) / kTwoPi, cut = -0.5 * cK * cK * (1.0 + 1e-12);
  const double dk = eps * (double)(kmin + t) - (double)(slo + l) * dp;  // eps (k - p_l / eps)
  const double ex = -dk * dk / (2.0 * eps);
  gtab[e] = ex < cut ? 0.0 : cst * exp(ex);
}

template <int D, int NQ, int NP, typename T, int MAXLG = 8, int NF = 1>
__global__ __launch_bounds__(kFusedThreads) void fggc_fused_kernel(Fused3Params p, T *__restrict__ Y,
                                                                    const T *__restrict__ tw) {
  using RR = decltype(T{}.x);
  constexpr int N1 = NQ * NP;
  constexpr int RB = rec_bytes<D, N1, T>();
  // the lines' leading dimensions: 0 and 1 in three dimensions, 0 alone in
  // two (the parameters then give dimension 1 one slice, one q-cell and a
  // tile of one line); the last dimension is the lines' own
  constexpr int NQ1 = D == 3 ? NQ : 1;
  constexpr int CPL = kFusedOut / NF;  // lines per thread in the fold
  constexpr int NV = RB / 16;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lgN = p.lgN, N = 1 << lgN, T0 = p.T0, T1 = p.T1, P = T0 * T1;
  const int M = (int)p.M;
  const int ng = (int)(p.kmax - p.kmin + 1);
  const int nact = min(M, ng);
  const int bs = (int)blockDim.x, tid0 = (int)threadIdx.x;
  // the lines (at most 512 points) are transformed in two register passes
  // (lds_fft2_rows) on padded rows
  const int rs = fft2_row_stride(lgN);               // row stride of the lines
  T *cl = reinterpret_cast<T *>(smem_raw);            // [Lc][P][rs] the chunk's lines
  T *stw = cl + (size_t)p.Lc * P * rs;                // [N] twiddles
  const int nw = (int)blockDim.x >> 6;
  // [waves][kFusedRuns] runs of records: first record and length (record
  // indices are below 2^32, the key-slot count)
  uint32_t *s_r0 = reinterpret_cast<uint32_t *>(stw + N);
  int *s_n = reinterpret_cast<int *>(s_r0 + nw * kFusedRuns);
  RR *gam = reinterpret_cast<RR *>(s_n + nw * kFusedRuns);  // [Lc][ng] band weights, working precision
  int *s_claim = reinterpret_cast<int *>(gam + p.Lc * ng);  // [waves][kFusedClaim]
  for (int i = tid0; i < N; i += bs) stw[i] = tw[i];
  // workgroup -> (q-tile, l0, l1); workgroups run on the eight XCDs in turn,
  // and each XCD takes a contiguous range of the work, so that the slice pairs
  // of one tile (which read the same bins) share that XCD's L2
  // (32-bit index arithmetic: the grid, the slices and the bins are below
  // 2^31, 2^16 and 2^32)
  const uint32_t nblk = gridDim.x, bid = blockIdx.x;
  const uint32_t per = nblk >> 3, rem = nblk & 7, xcd = bid & 7, i8 = bid >> 3;
  const uint32_t g = (xcd < rem ? xcd * (per + 1) : rem * (per + 1) + (xcd - rem) * per) + i8;
  const uint32_t sn0 = (uint32_t)p.sn[0], sn1 = (uint32_t)p.sn[1], ntq1 = (uint32_t)p.ntq1;
  const int l1 = (int)(g % sn1), l0 = (int)((g / sn1) % sn0);
  const uint32_t tq = g / (sn1 * sn0);
  const int q00 = (int)(tq / ntq1) * T0, q10 = (int)(tq % ntq1) * T1;
  const int span = p.maxdp - p.mindp;
  const int a0lo = max(0, l0 - span), a0hi = min((int)p.npc[0] - 1, l0);
  const int a1lo = max(0, l1 - span), a1hi = min((int)p.npc[1] - 1, l1);
  const uint32_t nqt = (uint32_t)(p.ntq0 * p.ntq1), npc1 = (uint32_t)p.npc[1], npc2 = (uint32_t)p.npc[2];
  const int msk0 = (int)p.Nq[0] - 1, msk1 = (int)p.Nq[1] - 1, msk2 = N - 1;
  const int kmod = (int)(((p.kmin % M) + M) % M);
  const int kmin = (int)p.kmin, kmax = (int)p.kmax;  // the band union (|k| < 2^31)
  // fold and output mapping: TPL threads per line group (a power of two >=
  // the active frequencies), G = blockDim / TPL groups
  const int TPL = p.TPL, G = bs / TPL;
  // the fold's sums, in the working precision (an output adds at most its
  // band's aliases of the slices along the last dimension)
  RR accr[kFusedOut], acci[kFusedOut];
#pragma unroll
  for (int c = 0; c < kFusedOut; ++c) accr[c] = acci[c] = 0;
  // Accumulation, one slice per wave: wave w adds the contributions to slice
  // l2 = c0 + w, read from the records whose p-cell 2 reaches it -- per
  // (p-cell 0, p-cell 1) that reaches (l0, l1), one contiguous run of bins
  // over p-cell 2.  Waves write disjoint rows, so the cells are updated with
  // plain LDS read-modify-writes.  Inside a wave, two lanes write the same
  // cell in one instruction only if their records share the q-cell (the
  // instruction fixes the q-shifts; the slice is the wave's); such lanes are
  // taken in turn, by claiming a slot of a hash of the q-cell in a per-wave
  // table (the last writer of a slot goes first).  A wave issues its LDS operations in order, so
  // updates of one cell by different instructions are ordered too.
  const int n1r = (int)(a1hi - a1lo + 1), nruns = (int)(a0hi - a0lo + 1) * n1r;
  const int sn2 = (int)p.sn[2];
  // The bounds of run `lane` of the slice wave `wv` takes in the chunk at c:
  // loaded one chunk ahead into registers, so that their latency overlaps
  // the previous chunk's work.
  auto run_bounds = [&](int c, int wv, int lane, int64_t &r0, int64_t &r1) {
    r0 = r1 = 0;
    if (lane < nruns && wv < min(p.Lc, sn2 - c)) {
      const int l2 = c + wv;
      const int a2lo = max(0, l2 - span), a2hi = min((int)npc2 - 1, l2);
      const uint32_t a0 = (uint32_t)(a0lo + lane / n1r), a1 = (uint32_t)(a1lo + lane % n1r);
      const uint32_t kb = ((a0 * npc1 + a1) * nqt + tq) * npc2;
      if (a2lo <= a2hi) {
        r0 = p.start[(size_t)kb + a2lo];
        r1 = p.start[(size_t)kb + a2hi + 1];
      }
    }
  };
  int64_t nr0, nr1;
  run_bounds(0, tid0 >> 6, tid0 & 63, nr0, nr1);
  bool dirty = true;  // the lines may hold data (a chunk without records leaves them zero)
  for (int c0 = 0; c0 < sn2; c0 += p.Lc) {
    const int lcn = min(p.Lc, sn2 - c0);
    // the thread index through a compiler fence: addresses are formed in each
    // chunk where they are used, not hoisted out of the loop into registers
    int tid = tid0;
    asm volatile("" : "+v"(tid));
    const int wv = tid >> 6, lane = tid & 63;
    if (lane < nruns && wv < lcn) {
      s_r0[wv * kFusedRuns + lane] = (uint32_t)nr0;
      s_n[wv * kFusedRuns + lane] = (int)(nr1 - nr0);
    }
    if (c0 + p.Lc < sn2) run_bounds(c0 + p.Lc, wv, lane, nr0, nr1);
    if (dirty)
      for (int e = tid; e < lcn * P * rs; e += bs) cl[e] = T{0, 0};
    __syncthreads();
    // the chunk's records over all its slices (read before the barrier that
    // ends the accumulation, so that the next chunk may rewrite the runs)
    int ctotal = 0;
    for (int w = 0; w < lcn; ++w)
      for (int x = 0; x < nruns; ++x) ctotal += s_n[w * kFusedRuns + x];
    // this chunk's band weights into LDS (the fold reads them, after the
    // barrier that ends the accumulation)
    if (ctotal > 0)
      for (int e = tid; e < lcn * ng; e += bs) gam[e] = (RR)p.gtab[(int64_t)c0 * ng + e];
    if (wv < lcn) {
      const int l2 = c0 + wv;
      int total = 0;
      const uint32_t *wr0 = s_r0 + wv * kFusedRuns;
      const int *wn = s_n + wv * kFusedRuns;
      for (int x = 0; x < nruns; ++x) total += wn[x];
      // (through an LDS-qualified pointer: the table lives in dynamic LDS,
      // and a generic volatile pointer would be accessed with flat
      // instructions)
      volatile __attribute__((address_space(3))) int *claim =
          (volatile __attribute__((address_space(3))) int *)(s_claim + wv * kFusedClaim);
      for (int base = 0; base < total; base += 64) {
        const int i = base + lane;
        bool todo = i < total;
        const char *rec = nullptr;
        if (todo) {
          int run = 0, off = i;
          while (off >= wn[run]) off -= wn[run++];
          rec = p.recs + ((size_t)wr0[run] + (size_t)off) * RB;
        }
        // records of up to 256 bytes are loaded whole (one round trip);
        // larger ones (FP64 with four shifts) index first, then only the
        // coefficients the slice takes, so as not to hold the whole record
        constexpr bool kWhole = NV <= 16;
        uint4 raw[kWhole ? NV : 2];
#pragma unroll
        for (int v = 0; v < (kWhole ? NV : 2); ++v)
          raw[v] = todo ? reinterpret_cast<const uint4 *>(rec)[v] : make_uint4(0, 0, 0, 0);
        const RecIdx<D> ri = *reinterpret_cast<const RecIdx<D> *>(raw);
        constexpr int KL = D - 1;  // the last dimension's index in the record
        int b0 = -1, b1 = D == 3 ? -1 : 0, b2 = -1;
#pragma unroll
        for (int b = 0; b < NP; ++b) {
          if (ri.pc[0] + p.dp[b] - p.mindp == l0) b0 = b;
          if constexpr (D == 3)
            if (ri.pc[1] + p.dp[b] - p.mindp == l1) b1 = b;
          if (ri.pc[KL] + p.dp[b] - p.mindp == l2) b2 = b;
        }
        todo = todo && b0 >= 0 && b1 >= 0 && b2 >= 0;
        int la0[NQ], la1[NQ1], q2[NQ];
#pragma unroll
        for (int a = 0; a < NQ; ++a) {
          const int v0 = ((ri.q[0] + p.dq[a]) & msk0) - q00;
          la0[a] = v0 >= 0 && v0 < T0 ? v0 : -1;
          if constexpr (D == 3) {
            const int v1 = ((ri.q[1] + p.dq[a]) & msk1) - q10;
            la1[a] = v1 >= 0 && v1 < T1 ? v1 : -1;
          }
          q2[a] = (ri.q[KL] + p.dq[a]) & msk2;
        }
        if constexpr (D == 2) la1[0] = 0;
        // the coefficients this slice takes: the leading dimensions at (b0,
        // b1), the last at b2 (two dimensions: dimension 1 is the last, and
        // u1 = 1 stands for the missing middle one)
        T u0[NQ], u1[NQ1], u2[NQ];
        if constexpr (D == 2) u1[0] = T{1, 0};
        if constexpr (kWhole) {
          const T *c = reinterpret_cast<const T *>(reinterpret_cast<const char *>(raw) + rec_idx_bytes<D>());
#pragma unroll
          for (int a = 0; a < NQ; ++a) {
            u0[a] = u2[a] = T{0, 0};
            if constexpr (D == 3) u1[a] = T{0, 0};
#pragma unroll
            for (int b = 0; b < NP; ++b) {
              if (b == b0) u0[a] = c[a * NP + b];
              if constexpr (D == 3)
                if (b == b1) u1[a] = c[N1 + a * NP + b];
              if (b == b2) u2[a] = c[KL * N1 + a * NP + b];
            }
          }
        } else {
          const T *c = reinterpret_cast<const T *>(rec + rec_idx_bytes<D>());
#pragma unroll
          for (int a = 0; a < NQ; ++a) {
            u0[a] = todo ? c[a * NP + b0] : T{0, 0};
            if constexpr (D == 3) u1[a] = todo ? c[N1 + a * NP + b1] : T{0, 0};
            u2[a] = todo ? c[KL * N1 + a * NP + b2] : T{0, 0};
          }
        }
        uint32_t h = (uint32_t)ri.q[0] * 0x9E3779B1u + (uint32_t)ri.q[KL] * 0xC2B2AE3Du;
        if constexpr (D == 3) h += (uint32_t)ri.q[1] * 0x85EBCA77u;
        h >>= 32 - kFusedClaimBits;
        T *rows = cl + (size_t)wv * P * rs;
        while (__ballot(todo)) {
          if (todo) claim[h] = lane;
          const bool win = todo && claim[h] == lane;
          if (win) {
            todo = false;
            // two q-shifts: every contribution unrolled; four: the first
            // dimension's shift in a loop (the 64-fold unrolling would not fit
            // the registers), its values picked without indexing registers
#pragma unroll(NQ == 2 || D == 2 ? NQ : 1)
            for (int a0i = 0; a0i < NQ; ++a0i) {
              const int la0v = pick<NQ>(la0, a0i);
              if (la0v < 0) continue;
              const T u0v = pick<NQ>(u0, a0i);
#pragma unroll
              for (int a1i = 0; a1i < NQ1; ++a1i) {
                if (la1[a1i] < 0) continue;
                const T uw = D == 3 ? cmul(u0v, u1[a1i]) : u0v;
                T *line = rows + (la0v * T1 + la1[a1i]) * rs;
#pragma unroll
                for (int a2i = 0; a2i < NQ; ++a2i) {
                  const T z = cmul(uw, u2[a2i]);
                  T o = line[q2[a2i]];
                  o.x += z.x;
                  o.y += z.y;
                  line[q2[a2i]] = o;
                  asm volatile("" ::: "memory");
                }
              }
            }
          }
        }
      }
    }
    __syncthreads();
    // a chunk whose slices took no record left its lines zero: nothing to
    // transform or fold, nor to clear for the next chunk (sparse packet sets
    // skip most chunks)
    dirty = ctotal > 0;
    if (!dirty) continue;
    lds_fft2_rows<T, MAXLG>(cl, lgN, lcn * P, rs, stw, tid, bs);
    // thread (g, t): frequency t of lines g, g + G, g + 2 G, ... -- one band
    // weight per (slice, alias) serves all of them
    // sum f * CPL + c of a thread: frequency t + f TPL of line lg0 + c G
    const int t = tid & (TPL - 1), lg0 = tid / TPL;
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const int tf = t + f * TPL;
      if (tf >= nact) break;
      for (int kk = kmin + tf; kk <= kmax; kk += M) {
        const T *fq = cl + lg0 * rs + (kk & msk2);
        const RR *gb = gam + (kk - kmin);
        for (int l = 0; l < lcn; ++l) {
          const RR gv = gb[l * ng];
          if (gv == (RR)0) continue;  // outside this slice's band (coherent: t runs along k)
#pragma unroll
          for (int c = 0; c < CPL; ++c) {
            if (lg0 + c * G >= P) break;
            const T v = fq[((size_t)l * P + c * G) * rs];
            accr[f * CPL + c] = fma(gv, v.x, accr[f * CPL + c]);
            acci[f * CPL + c] = fma(gv, v.y, acci[f * CPL + c]);
          }
        }
      }
    }
    __syncthreads();
  }
  const int64_t base = (l0 * p.sn[1] + l1) * p.Nq[0];
  const int t = tid0 & (TPL - 1), lg0 = tid0 / TPL;
  // every frequency of this thread's lines: the band's sums in the first NF
  // blocks of TPL frequencies, zeros elsewhere
  for (int tt = t, f = 0; tt < M; tt += TPL, ++f) {
    const int kp = (kmod + tt) % M;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const int line = lg0 + c * G;
      if (line >= P) break;
      const int64_t q0 = q00 + line / T1, q1 = q10 + line % T1;
      T v = T{0, 0};
#pragma unroll
      for (int f2 = 0; f2 < NF; ++f2)
        if (f == f2 && tt < nact) v = T{(RR)accr[f2 * CPL + c], (RR)acci[f2 * CPL + c]};
      Y[((base + q0) * p.Nq[1] + q1) * p.M + kp] = v;
    }
  }
}

// A separable pass over a dense input (the passes after the first in three
// dimensions, the last pass in two), the same contraction as
// fft_contract_kernel: Y[o][a][k'][b] = sum_l sum_{kk = k' (mod M)}
// gamma_l(kk) F_{o,l,a,b}[kk mod N].  A workgroup owns W consecutive b (one
// 128-byte run of the input per (slice, n)) at one (o, a); for Lc slices at a
// time it loads the W lines into LDS (as rows, padded for the register FFT),
// transforms them with lds_fft2_rows and folds them through the band weights
// gamma (a table per call) into sums in the working precision, thread (group g, frequency t)
// holding frequency t of lines g, g + G, ...  The sums go out through LDS, so
// that the writes run along b as well.
struct Contract2Params {
  int64_t O, L, A, B, M;
  int lgN, W, lgW, Lc, TPL;
  int64_t kmin, kmax;    // union of the slices' bands
  const double *gtab;    // [L][kmax - kmin + 1] band weights
};

template <typename T>
__global__ __launch_bounds__(kFusedThreads) void fft_contract2_kernel(Contract2Params p, const T *__restrict__ X,
                                                                      T *__restrict__ Y, const T *__restrict__ tw) {
  using RR = decltype(T{}.x);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lgN = p.lgN, N = 1 << lgN, W = p.W, M = (int)p.M;
  const int ng = (int)(p.kmax - p.kmin + 1), nact = min(M, ng);
  const int bs = (int)blockDim.x, tid0 = (int)threadIdx.x;
  const int rs = fft2_row_stride(lgN);
  T *cl = reinterpret_cast<T *>(smem_raw);            // [Lc][W][rs]
  T *stw = cl + (size_t)p.Lc * W * rs;                // [N]
  RR *gam = reinterpret_cast<RR *>(stw + N);          // [Lc][ng], working precision
  for (int i = tid0; i < N; i += bs) stw[i] = tw[i];
  // (32-bit index arithmetic within the grid, 64-bit addresses; W and N
  // are powers of two)
  const int lgW = p.lgW;
  const uint32_t nbc = (uint32_t)(p.B >> lgW), A = (uint32_t)p.A, g = blockIdx.x;
  const uint32_t oa = g / nbc, bc = g - oa * nbc;  // oa = o * A + a
  const uint32_t o = oa / A, a = oa - o * A;
  const size_t B = (size_t)p.B, b0 = (size_t)bc << lgW;
  const size_t sL = (size_t)A * ((size_t)N * B);  // input stride of a slice
  const int TPL = p.TPL, G = bs / TPL;
  const int kmod = (int)(((p.kmin % M) + M) % M);
  const int kmin = (int)p.kmin, kmax = (int)p.kmax;
  RR accr[kFusedOut], acci[kFusedOut];  // sums in the working precision
#pragma unroll
  for (int c = 0; c < kFusedOut; ++c) accr[c] = acci[c] = 0;
  for (int l0 = 0; l0 < (int)p.L; l0 += p.Lc) {
    const int lcn = min(p.Lc, (int)p.L - l0);
    int tid = tid0;
    asm volatile("" : "+v"(tid));
    for (int e = tid; e < lcn * ng; e += bs) gam[e] = (RR)p.gtab[(int64_t)l0 * ng + e];
    // rows (l, w) of N, loaded with w fastest (runs of W along b), eight
    // loads in flight per thread before their LDS stores
    const int tot = lcn * N * W;
    const T *Xc = X + ((((size_t)o * p.L + l0) * A + a) << lgN) * B + b0;
    for (int e0 = tid; e0 < tot; e0 += 8 * bs) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * bs;
        if (e < tot) {
          const int w = e & (W - 1), n = (e >> lgW) & (N - 1), l = e >> (lgW + lgN);
          v[u] = Xc[(size_t)l * sL + (size_t)n * B + w];
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + u * bs;
        if (e < tot) {
          const int w = e & (W - 1), n = (e >> lgW) & (N - 1), l = e >> (lgW + lgN);
          cl[(l * W + w) * rs + n] = v[u];
        }
      }
    }
    __syncthreads();
    lds_fft2_rows<T>(cl, lgN, lcn * W, rs, stw, tid, bs);
    const int t = tid & (TPL - 1), lg0 = tid / TPL;
    if (t < nact) {
      for (int kk = kmin + t; kk <= kmax; kk += M) {
        const T *fq = cl + lg0 * rs + (kk & (N - 1));
        const RR *gb = gam + (kk - kmin);
        for (int l = 0; l < lcn; ++l) {
          const RR gv = gb[l * ng];
          if (gv == (RR)0) continue;  // outside this slice's band
#pragma unroll
          for (int c = 0; c < kFusedOut; ++c) {
            if (lg0 + c * G >= W) break;
            const T v = fq[((size_t)l * W + c * G) * rs];
            accr[c] = fma(gv, v.x, accr[c]);
            acci[c] = fma(gv, v.y, acci[c]);
          }
        }
      }
    }
    __syncthreads();
  }
  // the sums into LDS as [k'][w], then out along b
  const int t = tid0 & (TPL - 1), lg0 = tid0 / TPL;
  T *ob = cl;  // [M][W]
  for (int tt = t; tt < M; tt += TPL) {
    const int kp = (kmod + tt) % M;
#pragma unroll
    for (int c = 0; c < kFusedOut; ++c) {
      const int w = lg0 + c * G;
      if (w >= W) break;
      ob[kp * W + w] = tt < nact ? T{(RR)accr[c], (RR)acci[c]} : T{0, 0};
    }
  }
  __syncthreads();
  T *Yo = Y + (size_t)oa * p.M * B + b0;
  for (int e = tid0; e < M * W; e += bs) {
    const int w = e & (W - 1), kp = e >> lgW;
    Yo[(size_t)kp * B + w] = ob[e];
  }
}

// One dimension: the aggregate's stencil writes each slice's q-spectrum
// directly (fggc_stencil_fft1_kernel, one slice per workgroup in LDS).
bool fft1_fused(const FggcArgs &a) { return a.g.d == 1 && a.Nq[0] <= 4096; }

struct FggcLayout {
  int d, N1, rec_b, ns;
  bool agg1;  // one dimension: aggregate + stencil instead of tile accumulation
  // three dimensions: accumulation fused with the pass over the last
  // dimension (no dense cell array); lines T0 x T1 per workgroup, Lc slices
  // of the last dimension per LDS chunk, the kernel's LDS bytes
  bool fused;
  int fT0, fT1, fLc, fnq, fnp, fTPL, fNF, fThreads;
  size_t fshm;
  int agg_splits;  // one dimension: workgroups (and copies of the aggregate) per bin
  int64_t ncells, nslices, npts, nbins, nslots, tiles, ntq[3], tile[3], npc[3], pmin[3], S[3], nsw[3];
  int64_t nb[3];
  int mindp, maxdp, mindq, maxdq;
  size_t off_gam[3];  // band weights gamma_l(k) per dimension [sn_k][ng_k] (FP64; 0: not used)
  size_t off_lsq, off_keys, off_pos, off_sort, off_start, off_recs, off_agg, off_cells, off_occ,
      off_spec, off_x1, off_x2, total;
};

int n1_bucket(int n1) { return n1 <= 4 ? 4 : (n1 <= 8 ? 8 : 16); }

// Grid frequencies of dimension k that some slice's truncated band reaches
// (before aliasing): |k - p_l / eps| <= cK / sqrt(eps), padded by one.
void band_range(const FggcArgs &a, int k, int64_t &kmin, int64_t &kmax) {
  const double se = std::sqrt(a.eps);
  kmin = (int64_t)std::floor((double)a.slo[k] * a.dp[k] / a.eps - a.cK / se) - 1;
  kmax = (int64_t)std::ceil((double)(a.slo[k] + a.sn[k] - 1) * a.dp[k] / a.eps + a.cK / se) + 1;
}

// The fused finish (accumulation and the pass over the last dimension in one
// kernel), when the strategy and sizes allow it: two or three dimensions, a
// tensor shift set of 2 x 2, 4 x 2 or 2 x 4, power-of-two q-meshes of at
// least 4 points along the leading dimensions and 8 to 256 along the last
// (512 in two dimensions in FP32),
// a workgroup's outputs and its LDS chunk within their budgets.
bool plan_fused(const FggcArgs &a, FggcLayout &L, int nq, int np) {
  const int d = a.g.d;
  if (d != 2 && d != 3) return false;
  if (!((nq == 2 && np == 2) || (nq == 4 && np == 2) || (nq == 2 && np == 4))) return false;
  if (L.N1 != nq * np) return false;
  const int kl = d - 1;
  const int64_t N = a.Nq[kl];
  if (N < 8 || N > 512 || !is_pow2(N) || a.Nq[0] < 4 || !is_pow2(a.Nq[0])) return false;
  // 512-point lines: two dimensions in FP32 only (their first FFT pass holds
  // 32 points per thread)
  if (N == 512 && (d != 2 || a.precision == FGGC_FP64)) return false;
  if (d == 3 && (a.Nq[1] < 4 || !is_pow2(a.Nq[1]))) return false;
  const int qspan = L.maxdq - L.mindq + 1, pspan = L.maxdp - L.mindp + 1;
  if ((d == 3 ? pspan * pspan : pspan) > kFusedRuns) return false;  // the runs of bins a chunk reads
  // two dimensions: fused only when the packets' contributions are fewer than
  // the cells (a sparse box, where the dense array would be mostly zeros);
  // dense sets are faster through the cell array and its tiled accumulation
  if (d == 2) {
    const double contrib = (double)a.pk->N * (double)(nq * np) * (double)(nq * np);
    const double cells = (double)a.sn[0] * (double)a.sn[1] * (double)a.Nq[0] * (double)a.Nq[1];
    if (contrib >= cells) return false;
  }
  int64_t kmin, kmax;
  band_range(a, kl, kmin, kmax);
  const int64_t ng = kmax - kmin + 1, nact = std::min<int64_t>(a.g.n[kl], ng);
  // fold: TPL threads per group of lines (a power of two), one frequency
  // each in every one of NF <= 2 blocks of TPL frequencies
  int64_t TPL0 = 1;
  while (TPL0 < nact) TPL0 *= 2;
  if (TPL0 > 2 * kFusedThreads) return false;
  // lines per workgroup and threads.  Three dimensions: 4 x 2 lines on 256
  // threads (several workgroups per CU), else 4 x 4 on 512, else 2 x 2 on 256
  // or 512.  Two dimensions: 8 lines on 256 or 512 threads, else 4.  A tile
  // spans the q-shifts, and a thread holds at most kFusedOut outputs.
  static const int t3[4][3] = {{4, 2, 256}, {4, 4, 512}, {2, 2, 256}, {2, 2, 512}};
  static const int t2[4][3] = {{8, 1, 256}, {8, 1, 512}, {4, 1, 256}, {4, 1, 512}};
  int T0 = 0, T1 = 0, threads = 0;
  int64_t TPL = 0, NF = 0, CPL = 0;
  for (auto &t : (d == 3 ? t3 : t2)) {
    if (t[0] < qspan || (d == 3 && t[1] < qspan) || t[0] > a.Nq[0] || (d == 3 && t[1] > a.Nq[1])) continue;
    const int64_t tpl = std::min<int64_t>(TPL0, t[2]), nf = (nact + tpl - 1) / tpl, g = t[2] / tpl;
    const int64_t cpl = ((int64_t)t[0] * t[1] + g - 1) / g;
    if (nf > (d == 3 ? 1 : 2) || nf * cpl > kFusedOut) continue;
    T0 = t[0];
    T1 = t[1];
    threads = t[2];
    TPL = tpl;
    NF = nf;
    CPL = cpl;
    break;
  }
  if (!T0) return false;
  const bool f64 = a.precision == FGGC_FP64;
  const size_t es = f64 ? 16 : 8;
  int lg = 0;
  while (((int64_t)1 << lg) < N) ++lg;
  const int64_t P = (int64_t)T0 * T1;
  // lines of N <= 512 points: the two-pass register FFT (lds_fft2_rows), one
  // unit per thread in its first pass and up to two in its second, on rows
  // padded to fft2_row_stride
  const int64_t rs = fft2_row_stride(lg);
  const int64_t N1 = (int64_t)1 << ((lg + 1) / 2), N2 = (int64_t)1 << (lg / 2);
  const int64_t maxrows = std::min<int64_t>(threads / N2, 2 * threads / N1);
  if (P > maxrows) return false;
  // at most one slice per wave (the accumulation gives each wave a slice)
  int Lc = (int)std::min<int64_t>(std::min<int64_t>(a.sn[kl], threads / 64), std::max<int64_t>(1, maxrows / P));
  // lines, twiddles, runs, the chunk's band weights (in the working
  // precision) and the claim tables
  const size_t waves = threads / 64;
  auto shm_of = [&](int lc) {
    return (size_t)lc * P * rs * es + (size_t)N * es + waves * kFusedRuns * 16 + (size_t)lc * ng * (es / 2) +
           waves * kFusedClaim * 4;
  };
  // LDS for five 256-thread (two 512-thread) workgroups per CU, the most the
  // registers allow: more resident workgroups beat fuller lanes in the
  // transforms (measured: chunks of 2, 3 and 4 slices, 22.7, 23.8 and 24.9 ms
  // on the 3D workload)
  const size_t budget = threads == 256 ? 32 * 1024 : 80 * 1024;
  while (Lc > 1 && shm_of(Lc) > budget) --Lc;
  if ((int64_t)Lc * P > maxrows || shm_of(Lc) > kFusedMaxLds) return false;
  const int64_t blocks = a.sn[0] * (d == 3 ? a.sn[1] * (a.Nq[1] / T1) : 1) * (a.Nq[0] / T0);
  if (blocks >= ((int64_t)1 << 31)) return false;
  L.fT0 = T0;
  L.fT1 = T1;
  L.fTPL = (int)TPL;
  L.fNF = (int)NF;
  L.fThreads = threads;
  L.fLc = Lc;
  L.fnq = nq;
  L.fnp = np;
  L.fshm = shm_of(Lc);
  return true;
}

// The dense register-FFT pass (fft_contract2_kernel) over dimension k, when
// it applies: a pass that reads a dense input (not the fused finish's, not
// two dimensions' first pass over the cells with its empty-tile map), a
// q-mesh of 8 to 256 points, and its lines, outputs and LDS within budget.
struct Contract2Plan {
  bool ok = false;
  int W = 0, Lc = 0, TPL = 0;
  size_t shm = 0;
};

Contract2Plan contract2_plan(const FggcArgs &a, int k, bool fused) {
  Contract2Plan c;
  const int d = a.g.d;
  if (d < 2 || k >= d || (d == 2 && k == 1) || (fused && k == d - 1)) return c;
  const int64_t N = a.Nq[k];
  if (N < 8 || N > 256 || (N & (N - 1))) return c;
  int lg = 0;
  while (((int64_t)1 << lg) < N) ++lg;
  int64_t B = 1;
  for (int j = k + 1; j < d; ++j) B *= a.g.n[j];
  int W = 16;
  while (W > 1 && B % W) W /= 2;
  int64_t kmin, kmax;
  band_range(a, k, kmin, kmax);
  const int64_t ng = kmax - kmin + 1, M = a.g.n[k], nact = std::min<int64_t>(M, ng);
  int64_t TPL = 1;
  while (TPL < nact) TPL *= 2;
  const int threads = kFusedThreads;
  if (TPL > threads) return c;
  const int64_t G = threads / TPL;
  if ((W + G - 1) / G > kFusedOut) return c;
  const size_t es = a.precision == FGGC_FP64 ? 16 : 8;
  const int64_t rs = fft2_row_stride(lg), N1 = (int64_t)1 << ((lg + 1) / 2), N2 = (int64_t)1 << (lg / 2);
  const int64_t maxrows = std::min<int64_t>(threads / N2, 2 * threads / N1);
  int Lc = (int)std::min<int64_t>(a.sn[k], std::max<int64_t>(1, maxrows / W));
  auto shm_of = [&](int lc) {
    // the lines double as the output staging [M][W]
    const size_t lines = std::max<size_t>((size_t)lc * W * rs, (size_t)M * W);
    return lines * es + (size_t)N * es + (size_t)lc * ng * (es / 2);
  };
  while (Lc > 1 && shm_of(Lc) > 80 * 1024) --Lc;
  if ((int64_t)Lc * W > maxrows || shm_of(Lc) > kFusedMaxLds) return c;
  c.ok = true;
  c.W = W;
  c.Lc = Lc;
  c.TPL = (int)TPL;
  c.shm = shm_of(Lc);
  return c;
}

bool contract2_ok(const FggcArgs &a, const FggcLayout &L, int k) { return contract2_plan(a, k, L.fused).ok; }

FggcLayout fggc_layout(const FggcArgs &a, bool allow_fused = true) {
  FggcLayout L{};
  const int d = a.g.d;
  L.d = d;
  const bool f64 = a.precision == FGGC_FP64;
  const size_t es = f64 ? 16 : 8;
  const DimLsq &l0 = a.lsq[0];
  L.N1 = n1_bucket(l0.n1);
  L.rec_b = (d == 1 ? rec_idx_bytes<1>() : (d == 2 ? rec_idx_bytes<2>() : rec_idx_bytes<3>())) + d * L.N1 * (int)es;
  L.mindp = L.maxdp = l0.dp[0];
  L.mindq = L.maxdq = l0.dq[0];
  for (int m = 1; m < l0.n1; ++m) {
    L.mindp = std::min(L.mindp, l0.dp[m]);
    L.maxdp = std::max(L.maxdp, l0.dp[m]);
    L.mindq = std::min(L.mindq, l0.dq[m]);
    L.maxdq = std::max(L.maxdq, l0.dq[m]);
  }
  {
    int np = 0;
    for (int m = 0; m < l0.n1; ++m)
      if (l0.dq[m] == l0.dq[0]) ++np;
    L.fused = allow_fused && plan_fused(a, L, l0.n1 / np, np);
  }
  // q-tile and slice window of one accumulation workgroup: the LDS holds
  // S^d * tile^d cells; a tile is at least as wide as the q-shift set
  static const int64_t deft[4] = {0, 32, 32, 16}, defs[4] = {0, 1, 1, 1};
  int64_t tmin = 1;
  while (tmin < L.maxdq - L.mindq + 1) tmin *= 2;
  L.nslices = 1;
  int64_t nqt = 1;
  L.npts = 1;
  L.nbins = 1;
  L.tiles = 1;
  for (int k = 0; k < 3; ++k) {
    if (k < d) {
      L.nslices *= a.sn[k];
      nqt *= a.Nq[k];
      L.npts *= a.g.n[k];
      // one dimension aggregates by own q-cell (no halo): tiles of at most 32
      // cells, the width of the aggregation workgroup (the largest divisor
      // of Nq up to 32); two and three dimensions take power-of-two tiles
      // that divide Nq and span the q-shifts
      if (d == 1) {
        L.tile[k] = std::min<int64_t>(a.Nq[k], kAgg1Tile);
        while (a.Nq[k] % L.tile[k]) --L.tile[k];
      } else {
        L.tile[k] = std::min<int64_t>(a.Nq[k], std::max<int64_t>(deft[d], tmin));
        while (L.tile[k] > 1 && a.Nq[k] % L.tile[k]) L.tile[k] /= 2;
        if (L.tile[k] < tmin)
          fail(FGGC_EUNSUPPORTED, "q-mesh of " + std::to_string(a.Nq[k]) +
                                      " cells: its power-of-two factor is below the q-shift span");
      }
      if (L.fused) L.tile[k] = k == d - 1 ? a.Nq[k] : (k == 0 ? L.fT0 : L.fT1);
      L.ntq[k] = a.Nq[k] / L.tile[k];
      L.pmin[k] = a.slo[k] - L.mindp;
      L.npc[k] = a.sn[k] - (L.maxdp - L.mindp);
      L.S[k] = std::min<int64_t>(defs[d], a.sn[k]);
      L.nsw[k] = (a.sn[k] + L.S[k] - 1) / L.S[k];
      L.nbins *= L.npc[k] * L.ntq[k];
      L.tiles *= L.nsw[k] * L.ntq[k];
      L.nb[k] = (int64_t)std::floor(2.0 * a.cK / std::sqrt(a.eps)) + 2;
    } else {
      L.tile[k] = L.ntq[k] = L.npc[k] = L.S[k] = L.nsw[k] = 1;
      L.pmin[k] = 0;
      L.nb[k] = 1;
    }
  }
  if (L.nbins >= ((int64_t)1 << 32)) fail(FGGC_EUNSUPPORTED, "too many packet bins");
  if (d == 3)
    for (int k = 0; k < 3; ++k)
      if (L.npc[k] > 65535) fail(FGGC_EUNSUPPORTED, "3D p-cell box wider than 65535 cells");
  L.ncells = L.nslices * nqt;
  if (L.tiles >= ((int64_t)1 << 31)) fail(FGGC_EUNSUPPORTED, "too many accumulation workgroups");
  const int64_t N = std::max<int64_t>(a.pk->N, 1);
  L.agg1 = d == 1;
  // key slots per packet: own tile, or 2^d with halo tiles (the fused finish
  // has one tile along the last dimension: halo slots in dims 0 and 1 only)
  L.ns = L.agg1 ? 1 : (L.fused ? 1 << (d - 1) : (1 << d));
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
  // few, crowded bins (a coarse mesh) get several workgroups each, ~2048
  // records apiece, each adding into its own copy of the aggregate
  L.agg_splits = 1;
  if (L.agg1) {
    const int64_t per_bin = a.pk->N / std::max<int64_t>(L.nbins, 1);
    L.agg_splits = (int)std::min<int64_t>(32, std::max<int64_t>(1, (per_bin + 2047) / 2048));
  }
  L.off_agg = put(L.agg1 ? (size_t)L.agg_splits * L.npc[0] * a.Nq[0] * L.N1 * es : 0);
  (void)N;
  L.off_cells = put(L.fused ? 0 : (size_t)L.ncells * es);
  // after the cells: the cells-only entry point (whose cells are the
  // caller's) writes every tile and takes no occupancy map
  L.off_occ = put(d == 2 ? (size_t)L.nslices * L.ntq[0] * L.ntq[1] : 0);  // empty-tile map
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
  // band tables: the fused finish's last dimension, and every dimension a
  // dense register-FFT pass contracts
  for (int k = 0; k < 3; ++k) {
    L.off_gam[k] = 0;
    const bool fusedk = L.fused && k == d - 1, densek = d >= 2 && contract2_ok(a, L, k);
    if (k < d && (fusedk || densek)) {
      int64_t kmin, kmax;
      band_range(a, k, kmin, kmax);
      L.off_gam[k] = put((size_t)a.sn[k] * (size_t)(kmax - kmin + 1) * 8);
    }
  }
  L.total = o;
  return L;
}

bool g_wave3_attr = false;
std::mutex g_wave3_mu;

bool g_sfft_attr = false;
std::mutex g_sfft_mu;
template <int D, int N1, typename T>
void launch_coef_accum(const FggcArgs &a, const FggcLayout &L, const CoefParams &cp,
                       const uint32_t *pos, char *recs, const int64_t *start, void *agg, T *cells,
                       uint8_t *occ, bool spectra, hipStream_t s) {
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
  if (L.fused) return;  // the fused finish accumulates the records itself
  AccParams ap{};
  ap.recs = recs;
  ap.start = start;
  ap.empty = nullptr;
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
    gp.splits = L.agg_splits;
    const dim3 gg((unsigned)(L.nbins * L.agg_splits)), gb(kAggThreads);
    fggc_agg1_kernel<N1, T, kAgg1Tile><<<gg, gb, 0, s>>>(gp, A);
    FGGC_HIP(hipGetLastError());
    Stencil1Params sp{};
    sp.Nq = a.Nq[0];
    sp.sn = a.sn[0];
    sp.npc = L.npc[0];
    sp.n1 = l0.n1;
    sp.nq = nq;
    sp.np = np;
    sp.mindp = L.mindp;
    sp.splits = L.agg_splits;
    for (int i = 0; i < 8; ++i) {
      sp.dq[i] = ap.dq[i];
      sp.dp[i] = ap.dp[i];
    }
    const int64_t ncl = a.sn[0] * a.Nq[0];
    if (spectra && fft1_fused(a)) {
      // cells straight into their q-spectra (the finish skips its q-DFT)
      int lgN = 0;
      while (((int64_t)1 << lgN) < a.Nq[0]) ++lgN;
      if (((int64_t)1 << lgN) != a.Nq[0]) lgN = -1;  // mixed-radix passes
      // 256 threads: N <= 4096 keeps the FFT within 8 butterflies per thread
      const T *tw = (const T *)fft_twiddles(a.Nq[0], a.precision);
      {
        std::lock_guard<std::mutex> lk(g_sfft_mu);
        if (!g_sfft_attr) {
          FGGC_HIP(hipFuncSetAttribute((const void *)fggc_stencil_fft1_kernel<float2>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 131072));
          FGGC_HIP(hipFuncSetAttribute((const void *)fggc_stencil_fft1_kernel<double2>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 131072));
          g_sfft_attr = true;
        }
      }
      fggc_stencil_fft1_kernel<T><<<dim3((unsigned)a.sn[0]), dim3(256), 2 * a.Nq[0] * sizeof(T), s>>>(
          sp, A, N1, lgN, tw, cells);
    } else {
      fggc_stencil1_kernel<T><<<dim3((unsigned)((ncl + 255) / 256)), dim3(256), 0, s>>>(sp, A, N1, cells);
    }
    FGGC_HIP(hipGetLastError());
    return;
  }
  int64_t tc = 1;
  for (int k = 0; k < D; ++k) tc *= L.tile[k] * L.S[k];
  const size_t shm = 2 * (size_t)tc * sizeof(decltype(T{}.x));
  if (shm > 65536) fail(FGGC_EUNSUPPORTED, "accumulation tile exceeds 64 KB of LDS");
  StageScope sc(a.prof, "fggc_accum", s);
  const dim3 grid((unsigned)L.tiles), blk(256);
  const bool wave = L.S[0] == 1 && (D < 2 || L.S[1] == 1) && (D < 3 || L.S[2] == 1) && N1 == nq * np &&
                    ((nq == 2 && np == 2) || (nq == 4 && np == 2) || (nq == 2 && np == 4) || (nq == 4 && np == 4)) &&
                    tc * sizeof(T) <= 65536 && (D < 3 || N1 == 4);  // 3D: Q2P2 (larger sets unroll too far)
  if (wave && D == 3) {
    std::lock_guard<std::mutex> lk(g_wave3_mu);
    if (!g_wave3_attr) {
      const void *ks[] = {(const void *)fggc_accum_wave_kernel<3, 2, 2, float2>,
                          (const void *)fggc_accum_wave_kernel<3, 2, 2, double2>};
      for (const void *kf : ks)
        FGGC_HIP(hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, 65536));
      g_wave3_attr = true;
    }
  }
  if (D == 2 && occ) {
    if (wave) ap.empty = occ;  // the one-wave kernel marks every (slice, tile)
    else launch_zero(occ, (size_t)L.nslices * L.ntq[0] * L.ntq[1], s);  // no tile is skipped
  }
  if (wave) {
    const size_t wshm = (size_t)(tc)*sizeof(T);
    const dim3 wblk(64);
    if (N1 == 4 && nq == 2 && np == 2) {
      fggc_accum_wave_kernel<D, 2, 2, T><<<grid, wblk, wshm, s>>>(ap, cells);
      FGGC_HIP(hipGetLastError());
      return;
    }
    if (D < 3 && N1 == 8 && nq == 4 && np == 2) {
      fggc_accum_wave_kernel<(D < 3 ? D : 2), 4, 2, T><<<grid, wblk, wshm, s>>>(ap, cells);
      FGGC_HIP(hipGetLastError());
      return;
    }
    if (D < 3 && N1 == 8 && nq == 2 && np == 4) {
      fggc_accum_wave_kernel<(D < 3 ? D : 2), 2, 4, T><<<grid, wblk, wshm, s>>>(ap, cells);
      FGGC_HIP(hipGetLastError());
      return;
    }
    if (D < 3 && N1 == 16 && nq == 4 && np == 4) {
      fggc_accum_wave_kernel<(D < 3 ? D : 2), 4, 4, T><<<grid, wblk, wshm, s>>>(ap, cells);
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
void cells_stage(const FggcArgs &a, const FggcLayout &L, char *base, void *cells, uint8_t *occ,
                 bool spectra, hipStream_t s) {
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
  kp.pc_last = L.fused ? 1 : 0;
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
      if (N > 0) count_positions(cpn, keys, L.nslots, sc_base, start, pos, s);
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
  cp.inv_2pi_eps = 1.0 / (kTwoPi * a.eps);
  cp.scale = a.scale;
  cp.lsq = dlsq;
  for (int k = 0; k < 3; ++k) {
    cp.Nq[k] = a.Nq[k];
    cp.pmin[k] = L.pmin[k];
    cp.dq[k] = kTwoPi / (double)a.Nq[k];
    cp.dp[k] = a.dp[k];
  }
#define FGGC_CA(DD, NN)                                                                           \
  if (f64) launch_coef_accum<DD, NN, double2>(a, L, cp, pos, recs, start, base + L.off_agg, (double2 *)cells, occ, spectra, s); \
  else launch_coef_accum<DD, NN, float2>(a, L, cp, pos, recs, start, base + L.off_agg, (float2 *)cells, occ, spectra, s);
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
void launch_contract(const FggcArgs &a, const FggcLayout &L, int k, const T *in, T *out, const uint8_t *occ,
                     const MacParams &m, hipStream_t s) {
  {
    std::lock_guard<std::mutex> lk(g_contract_mu);
    if (!g_contract_attr) {
      const void *ks[] = {(const void *)fft_contract_kernel<float2, float, false>,
                          (const void *)fft_contract_kernel<double2, double, false>,
                          (const void *)fft_contract_kernel<float2, float, true>,
                          (const void *)fft_contract_kernel<double2, double, true>};
      for (const void *kf : ks)
        FGGC_HIP(hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, 131072));
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
  const int64_t N = a.Nq[k];
  const bool mr = !is_pow2(N);  // a q-mesh with factors 3 or 5: mixed-radix passes
  int lgN = 0;
  while (((int64_t)1 << lgN) < N) ++lgN;
  p.N = (int)N;
  p.lgN = mr ? 0 : lgN;
  // lines per workgroup: runs of up to 4 consecutive b (contiguous in memory),
  // or, when b is a single line, up to 16 consecutive a (whole rows of N);
  // a chunk holds at most 4096 elements (the butterfly budget of
  // lds_fft_rows for kContractThreads threads, counting the radix-2 pass of
  // an odd log2 N)
  constexpr int64_t kElems = kContractThreads * kContractBfly * 2;
  if (N > kElems) fail(FGGC_EUNSUPPORTED, "q-mesh too long for the separable finish");
  // (powers of two that divide B and A, so that the groups tile them)
  int lgW = 0, lgWA = 0;
  while ((2 << lgW) <= std::min<int64_t>(4, p.B) && (N << (lgW + 1)) <= kElems && p.B % (2 << lgW) == 0) ++lgW;
  if (p.B == 1)
    while ((2 << lgWA) <= std::min<int64_t>(16, p.A) && (N << (lgWA + 1)) <= 1024 &&
           (p.M << (lgWA + 1)) <= kContractThreads * kContractOut && p.A % (2 << lgWA) == 0)
      ++lgWA;
  p.lgW = lgW;
  p.lgWA = lgWA;
  const int64_t P = (int64_t)1 << (lgW + lgWA);
  if (p.B % (1 << lgW) || p.A % (1 << lgWA)) fail(FGGC_EUNSUPPORTED, "separable finish: uneven line packing");
  p.Lc = (int)std::max<int64_t>(1, std::min<int64_t>(p.L, kElems / (N * P)));
  // frequencies split over MS workgroups: at most 2048 outputs
  // each, and more splits (each redoing the group's DFTs) when there are
  // few line groups
  const int64_t groups = p.O * (p.A / (1 << lgWA)) * (p.B / (1 << lgW));
  // (shares of ceil(M / MS) frequencies; the last share may be short)
  int MS = 1;
  while (((p.M + MS - 1) / MS) * P > kContractThreads * kContractOut) MS *= 2;
  while (groups * MS < 1024 && MS * 2 <= 16 && (p.M / (MS * 2)) * P >= kContractThreads) MS *= 2;
  p.MS = MS;
  p.kmin = m.kmin[k];
  p.kmax = m.kmax[k];
  p.slo = a.slo[k];
  p.eps = a.eps;
  p.dp = a.dp[k];
  p.cK = a.cK;
  p.empty = (d == 2 && k == 1) ? occ : nullptr;
  // a chunk holds at most 4096 / N rows of N / tile q1-tiles (the accumulate
  // has already skipped the empty tiles, so the map must be honoured)
  if (p.empty && (int64_t)p.Lc * (1 << lgWA) * L.ntq[1] > kContractFlags)
    fail(FGGC_EUNSUPPORTED, "separable finish: too many tile flags per chunk");
  p.ntq0 = L.ntq[0];
  p.ntq1 = L.ntq[1];
  p.lgt0 = p.lgt1 = 0;
  while (((int64_t)1 << p.lgt0) < L.tile[0]) ++p.lgt0;
  while (((int64_t)1 << p.lgt1) < L.tile[1]) ++p.lgt1;
  const size_t shm = (size_t)(p.Lc * P + 1) * N * sizeof(T) + 16;  // rows, then twiddles
  const int64_t blocks = groups * MS;
  if (blocks >= ((int64_t)1 << 31)) fail(FGGC_EUNSUPPORTED, "too many workgroups for the separable finish");
  const T *tw = (const T *)fft_twiddles(N, a.precision);
  if (mr) fft_contract_kernel<T, R, true><<<dim3((unsigned)blocks), dim3(kContractThreads), shm, s>>>(p, in, out, tw);
  else fft_contract_kernel<T, R, false><<<dim3((unsigned)blocks), dim3(kContractThreads), shm, s>>>(p, in, out, tw);
  FGGC_HIP(hipGetLastError());
}

void launch_band_table(const FggcArgs &a, int k, const MacParams &m, double *gtab, hipStream_t s) {
  const int64_t nt = a.sn[k] * (m.kmax[k] - m.kmin[k] + 1);
  band_table_kernel<<<dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s>>>(a.sn[k], m.kmin[k], m.kmax[k], a.slo[k],
                                                                            a.eps, a.dp[k], a.cK, gtab);
  FGGC_HIP(hipGetLastError());
}

bool g_c2_attr = false;
std::mutex g_c2_mu;

// One dense separable pass over dimension k on the register FFT (see
// fft_contract2_kernel); the caller has checked contract2_plan(...).ok.
template <typename T>
void launch_contract2(const FggcArgs &a, const FggcLayout &L, int k, char *base, const T *in, T *out,
                      const MacParams &m, hipStream_t s) {
  {
    std::lock_guard<std::mutex> lk(g_c2_mu);
    if (!g_c2_attr) {
      FGGC_HIP(hipFuncSetAttribute((const void *)fft_contract2_kernel<float2>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFusedMaxLds));
      FGGC_HIP(hipFuncSetAttribute((const void *)fft_contract2_kernel<double2>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFusedMaxLds));
      g_c2_attr = true;
    }
  }
  const Contract2Plan c = contract2_plan(a, k, L.fused);
  if (!c.ok) fail(FGGC_EDEVICE, "internal: dense pass not planned");
  const int d = a.g.d;
  Contract2Params p{};
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
  p.lgN = 0;
  while (((int64_t)1 << p.lgN) < a.Nq[k]) ++p.lgN;
  p.W = c.W;
  p.lgW = 0;
  while ((1 << p.lgW) < c.W) ++p.lgW;
  p.Lc = c.Lc;
  p.TPL = c.TPL;
  p.kmin = m.kmin[k];
  p.kmax = m.kmax[k];
  double *gtab = (double *)(base + L.off_gam[k]);
  p.gtab = gtab;
  launch_band_table(a, k, m, gtab, s);
  const int64_t blocks = p.O * p.A * (p.B / p.W);
  if (blocks >= ((int64_t)1 << 31)) fail(FGGC_EUNSUPPORTED, "too many workgroups for the separable finish");
  const T *tw = (const T *)fft_twiddles(a.Nq[k], a.precision);
  fft_contract2_kernel<T><<<dim3((unsigned)blocks), dim3(kFusedThreads), c.shm, s>>>(p, in, out, tw);
  FGGC_HIP(hipGetLastError());
}

bool g_fused_attr = false;
std::mutex g_fused_mu;

template <typename T>
void launch_fused(const FggcArgs &a, const FggcLayout &L, char *base, const MacParams &m, T *out,
                  hipStream_t s) {
  {
    std::lock_guard<std::mutex> lk(g_fused_mu);
    if (!g_fused_attr) {
      const void *ks[] = {(const void *)fggc_fused_kernel<3, 2, 2, float2>,
                          (const void *)fggc_fused_kernel<3, 4, 2, float2>,
                          (const void *)fggc_fused_kernel<3, 2, 4, float2>,
                          (const void *)fggc_fused_kernel<3, 2, 2, double2>,
                          (const void *)fggc_fused_kernel<3, 4, 2, double2>,
                          (const void *)fggc_fused_kernel<3, 2, 4, double2>,
                          (const void *)fggc_fused_kernel<2, 2, 2, float2>,
                          (const void *)fggc_fused_kernel<2, 4, 2, float2>,
                          (const void *)fggc_fused_kernel<2, 2, 4, float2>,
                          (const void *)fggc_fused_kernel<2, 2, 2, double2>,
                          (const void *)fggc_fused_kernel<2, 4, 2, double2>,
                          (const void *)fggc_fused_kernel<2, 2, 4, double2>,
                          (const void *)fggc_fused_kernel<2, 2, 2, float2, 8, 2>,
                          (const void *)fggc_fused_kernel<2, 4, 2, float2, 8, 2>,
                          (const void *)fggc_fused_kernel<2, 2, 4, float2, 8, 2>,
                          (const void *)fggc_fused_kernel<2, 2, 2, double2, 8, 2>,
                          (const void *)fggc_fused_kernel<2, 4, 2, double2, 8, 2>,
                          (const void *)fggc_fused_kernel<2, 2, 4, double2, 8, 2>,
                          (const void *)fggc_fused_kernel<2, 2, 2, float2, 9>,
                          (const void *)fggc_fused_kernel<2, 4, 2, float2, 9>,
                          (const void *)fggc_fused_kernel<2, 2, 4, float2, 9>,
                          (const void *)fggc_fused_kernel<2, 2, 2, float2, 9, 2>,
                          (const void *)fggc_fused_kernel<2, 4, 2, float2, 9, 2>,
                          (const void *)fggc_fused_kernel<2, 2, 4, float2, 9, 2>};
      for (const void *kf : ks)
        FGGC_HIP(hipFuncSetAttribute(kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kFusedMaxLds));
      g_fused_attr = true;
    }
  }
  const int d = a.g.d, kl = d - 1;
  const DimLsq &l0 = a.lsq[0];
  Fused3Params p{};
  p.recs = base + L.off_recs;
  p.start = (const int64_t *)(base + L.off_start);
  // [leading dimension 0, leading dimension 1, last dimension]; two
  // dimensions give the middle entry one slice, one p-cell and one q-cell
  for (int k = 0; k < 3; ++k) {
    const int src = k == 2 ? kl : k;
    const bool dummy = d == 2 && k == 1;
    p.sn[k] = dummy ? 1 : a.sn[src];
    p.npc[k] = dummy ? 1 : L.npc[src];
    p.Nq[k] = dummy ? 1 : a.Nq[src];
  }
  p.ntq0 = L.ntq[0];
  p.ntq1 = d == 3 ? L.ntq[1] : 1;
  p.T0 = L.fT0;
  p.T1 = L.fT1;
  p.Lc = L.fLc;
  p.TPL = L.fTPL;
  p.lgN = 0;
  while (((int64_t)1 << p.lgN) < a.Nq[kl]) ++p.lgN;
  for (int i = 0; i < 8; ++i) {
    p.dq[i] = i < L.fnq ? l0.dq[i * L.fnp] : 0;
    p.dp[i] = i < L.fnp ? l0.dp[i] : 0;
  }
  p.mindp = L.mindp;
  p.maxdp = L.maxdp;
  p.M = a.g.n[kl];
  p.kmin = m.kmin[kl];
  p.kmax = m.kmax[kl];
  p.slo = a.slo[kl];
  p.eps = a.eps;
  p.dp2 = a.dp[kl];
  p.cK = a.cK;
  p.gtab = (const double *)(base + L.off_gam[kl]);
  launch_band_table(a, kl, m, (double *)(base + L.off_gam[kl]), s);
  const int64_t blocks = p.sn[0] * p.sn[1] * p.ntq0 * p.ntq1;
  const T *tw = (const T *)fft_twiddles(a.Nq[kl], a.precision);
  const dim3 g((unsigned)blocks), b((unsigned)L.fThreads);
  // <dimensions, q-shifts, p-shifts, type, longest line (log2), frequency blocks>
  auto go = [&](auto kern) { kern<<<g, b, L.fshm, s>>>(p, out, tw); };
  const int sh = L.fnq == 2 && L.fnp == 2 ? 0 : (L.fnq == 4 ? 1 : 2);
  if (d == 3) {
    if (sh == 0) go(fggc_fused_kernel<3, 2, 2, T>);
    else if (sh == 1) go(fggc_fused_kernel<3, 4, 2, T>);
    else go(fggc_fused_kernel<3, 2, 4, T>);
  } else if (p.lgN <= 8 && L.fNF == 1) {
    if (sh == 0) go(fggc_fused_kernel<2, 2, 2, T>);
    else if (sh == 1) go(fggc_fused_kernel<2, 4, 2, T>);
    else go(fggc_fused_kernel<2, 2, 4, T>);
  } else if (p.lgN <= 8) {
    if (sh == 0) go(fggc_fused_kernel<2, 2, 2, T, 8, 2>);
    else if (sh == 1) go(fggc_fused_kernel<2, 4, 2, T, 8, 2>);
    else go(fggc_fused_kernel<2, 2, 4, T, 8, 2>);
  } else {
    // 512-point lines (FP32 only, see plan_fused)
    if constexpr (sizeof(T) == 8) {
      if (L.fNF == 1) {
        if (sh == 0) go(fggc_fused_kernel<2, 2, 2, T, 9>);
        else if (sh == 1) go(fggc_fused_kernel<2, 4, 2, T, 9>);
        else go(fggc_fused_kernel<2, 2, 4, T, 9>);
      } else {
        if (sh == 0) go(fggc_fused_kernel<2, 2, 2, T, 9, 2>);
        else if (sh == 1) go(fggc_fused_kernel<2, 4, 2, T, 9, 2>);
        else go(fggc_fused_kernel<2, 2, 4, T, 9, 2>);
      }
    } else {
      fail(FGGC_EDEVICE, "internal: 512-point fused lines planned in FP64");
    }
  }
  FGGC_HIP(hipGetLastError());
}

template <typename T, typename R>
void finish_stage(const FggcArgs &a, const FggcLayout &L, char *base, T *cells, const uint8_t *occ,
                  void *spec, Workspace &ws, hipStream_t s) {
  const int d = a.g.d;
  const int prec = a.precision;
  // F5: forward DFT over q of every p-slice (one dimension; higher dimensions
  // fold the DFT into the separable passes below)
  if (d == 1 && !fft1_fused(a)) launch_fft(d, a.Nq, L.nslices, -1, prec, cells, ws, s, a.prof, "fggc_fft_q");
  // F6: band multiply-accumulate into the grid spectrum (gamma evaluated in place)
  MacParams m{};
  for (int k = 0; k < 3; ++k) {
    m.M[k] = k < d ? a.g.n[k] : 1;
    m.Nq[k] = k < d ? a.Nq[k] : 1;
    m.sn[k] = a.sn[k];
    m.nb[k] = L.nb[k];
    m.slo[k] = a.slo[k];
    m.dp[k] = a.dp[k];
    m.inv_dp[k] = 1.0 / a.dp[k];
    if (k < d) band_range(a, k, m.kmin[k], m.kmax[k]);
  }
  m.eps = a.eps;
  m.cK = a.cK;
  T *U = (T *)spec;
  if (d >= 2) {
    // F5 + F6 as d separable passes, last dimension first, into the spectrum
    // (three dimensions: the first pass fused with the accumulation)
    T *x1 = (T *)(base + L.off_x1), *x2 = (T *)(base + L.off_x2);
    if (L.fused) {
      StageScope sc(a.prof, "fggc_fused", s);
      launch_fused<T>(a, L, base, m, x1, s);
    }
    StageScope sc(a.prof, "fggc_contract", s);
    const T *in = L.fused ? x1 : cells;
    for (int k = L.fused ? d - 2 : d - 1; k >= 0; --k) {
      T *out = k == 0 ? U : (k == d - 1 ? x1 : x2);
      if (contract2_ok(a, L, k)) launch_contract2<T>(a, L, k, base, in, out, m, s);
      else launch_contract<T, R>(a, L, k, in, out, k == d - 1 ? occ : nullptr, m, s);
      in = out;
    }
  } else {
    StageScope sc(a.prof, "fggc_band_mac", s);
    band_mac1_kernel<T, R><<<(unsigned)((8 * L.npts + 255) / 256), 256, 0, s>>>(m, cells, U);
    FGGC_HIP(hipGetLastError());
  }
  // F7: inverse DFT of the grid spectrum into u
  launch_fft_to(d, a.g.n, +1, prec, U, a.u, ws, s, a.prof, "fggc_ifft");
}

// Per-packet coefficients for inspection: the coefficient kernel's records
// in packet order (identity positions), then the Kronecker product over
// dimensions of each record's per-dimension coefficients, c_K for every basis
// K (row-major over dimensions, each index over the one-dimensional shift
// set in plan order), and the packet's cell (q index, p-cell) per dimension.
__global__ void iota_kernel(uint32_t *__restrict__ pos, int64_t N) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j < N) pos[j] = (uint32_t)j;
}

template <int D, int N1>
__global__ void coef_extract_kernel(int64_t N, int n1, const char *__restrict__ recs, double2 *__restrict__ c_out,
                                    int32_t *__restrict__ cell_out) {
  constexpr int RB = rec_bytes<D, N1, double2>();
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= N) return;
  const char *r = recs + j * (int64_t)RB;
  const RecIdx<D> ri = *reinterpret_cast<const RecIdx<D> *>(r);
  const double2 *c = reinterpret_cast<const double2 *>(r + rec_idx_bytes<D>());
  for (int k = 0; k < D; ++k) {
    cell_out[j * 2 * D + k] = ri.q[k];
    cell_out[j * 2 * D + D + k] = ri.pc[k];
  }
  int nk = 1;
  for (int k = 0; k < D; ++k) nk *= n1;
  for (int K = 0; K < nk; ++K) {
    double2 v = make_double2(1.0, 0.0);
    int rem = K;
    for (int k = D - 1; k >= 0; --k) {
      const double2 ck = c[k * N1 + rem % n1];
      rem /= n1;
      v = make_double2(v.x * ck.x - v.y * ck.y, v.x * ck.y + v.y * ck.x);
    }
    c_out[j * nk + K] = v;
  }
}

}  // namespace

void launch_fggc_coefficients(const FggcArgs &a, double *c_out, int32_t *cell_out, Workspace &ws, hipStream_t s) {
  const int d = a.g.d;
  const int64_t N = a.pk->N;
  if (N == 0) return;
  const DimLsq &l0 = a.lsq[0];
  const int N1 = n1_bucket(l0.n1);
  const int rb = 16 * ((8 * d + 15) / 16) + d * N1 * 16;
  char *base = (char *)ws.take(3 * sizeof(DimLsq) + 256 + (size_t)N * 4 + 256 + (size_t)N * rb);
  DimLsq *dl = (DimLsq *)base;
  uint32_t *pos = (uint32_t *)(base + align_up(3 * sizeof(DimLsq), 256));
  char *recs = (char *)pos + align_up((size_t)N * 4, 256);
  const DimLsq *dlsq = a.lsq_dev;
  if (!dlsq) {
    FGGC_HIP(hipMemcpyAsync(dl, a.lsq, d * sizeof(DimLsq), hipMemcpyHostToDevice, s));
    dlsq = dl;
  }
  const dim3 g((unsigned)((N + 255) / 256)), b(256);
  iota_kernel<<<g, b, 0, s>>>(pos, N);
  FGGC_HIP(hipGetLastError());
  CoefParams cp{};
  cp.ns = 1;
  cp.N = N;
  cp.Q = a.pk->Q;
  cp.P = a.pk->P;
  cp.S = a.pk->S;
  cp.a = a.pk->a;
  cp.inv_2pi_eps = 1.0 / (kTwoPi * a.eps);
  cp.scale = a.scale;
  cp.lsq = dlsq;
  for (int k = 0; k < 3; ++k) {
    cp.Nq[k] = a.Nq[k];
    cp.pmin[k] = 0;
    cp.dq[k] = kTwoPi / (double)a.Nq[k];
    cp.dp[k] = a.dp[k];
  }
  int cnp = 0;
  for (int m = 0; m < l0.n1; ++m)
    if (l0.dq[m] == l0.dq[0]) ++cnp;
  const int cnq = l0.n1 / cnp;
#define FGGC_COEF_ONE(DD, NN)                                                                                 \
  {                                                                                                            \
    if (NN == 4 && cnq == 2 && cnp == 2) fggc_coef_kernel<DD, NN, 2, 2, double2><<<g, b, 0, s>>>(cp, pos, recs); \
    else if (NN == 8 && cnq == 4 && cnp == 2) fggc_coef_kernel<DD, NN, 4, 2, double2><<<g, b, 0, s>>>(cp, pos, recs); \
    else if (NN == 8 && cnq == 2 && cnp == 4) fggc_coef_kernel<DD, NN, 2, 4, double2><<<g, b, 0, s>>>(cp, pos, recs); \
    else if (NN == 16 && cnq == 4 && cnp == 4) fggc_coef_kernel<DD, NN, 4, 4, double2><<<g, b, 0, s>>>(cp, pos, recs); \
    else fggc_coef_kernel<DD, NN, 0, 0, double2><<<g, b, 0, s>>>(cp, pos, recs);                                  \
    FGGC_HIP(hipGetLastError());                                                                               \
    coef_extract_kernel<DD, NN><<<g, b, 0, s>>>(N, l0.n1, recs, (double2 *)c_out, cell_out);                   \
    FGGC_HIP(hipGetLastError());                                                                               \
  }
  if (d == 1) {
    if (N1 == 4) FGGC_COEF_ONE(1, 4) else if (N1 == 8) FGGC_COEF_ONE(1, 8) else FGGC_COEF_ONE(1, 16)
  } else if (d == 2) {
    if (N1 == 4) FGGC_COEF_ONE(2, 4) else if (N1 == 8) FGGC_COEF_ONE(2, 8) else FGGC_COEF_ONE(2, 16)
  } else {
    if (N1 == 4) FGGC_COEF_ONE(3, 4) else if (N1 == 8) FGGC_COEF_ONE(3, 8)
    else fail(FGGC_EUNSUPPORTED, "3D strategies need nq * np <= 8");
  }
#undef FGGC_COEF_ONE
}

size_t fggc_coefficients_workspace_bytes(const FggcArgs &a) {
  const int d = a.g.d;
  const int N1 = n1_bucket(a.lsq[0].n1);
  const int rb = 16 * ((8 * d + 15) / 16) + d * N1 * 16;
  return 3 * sizeof(DimLsq) + 256 + (size_t)a.pk->N * 4 + 256 + (size_t)a.pk->N * rb + 1024;
}

namespace {
}  // namespace

size_t fggc_workspace_bytes(const FggcArgs &a) { return fggc_layout(a).total + 1024; }

bool fggc_graph_safe(const FggcArgs &a) {
  const FggcLayout L = fggc_layout(a);
  return bucket_positions_graph_safe(L.nslots, L.nbins);
}

size_t fggc_cells_workspace_bytes(const FggcArgs &a) {
  FggcLayout L = fggc_layout(a, false);
  return L.off_cells + 1024;
}

void launch_fggc_cells(const FggcArgs &a, void *cells, Workspace &ws, hipStream_t s) {
  FggcLayout L = fggc_layout(a, false);
  char *base = (char *)ws.take(L.off_cells);
  cells_stage(a, L, base, cells, nullptr, false, s);
}

void launch_fggc(const FggcArgs &a, Workspace &ws, hipStream_t s) {
  FggcLayout L = fggc_layout(a);
  char *base = (char *)ws.take(L.total);
  void *cells = base + L.off_cells;
  uint8_t *occ = a.g.d == 2 ? (uint8_t *)(base + L.off_occ) : nullptr;
  cells_stage(a, L, base, cells, occ, true, s);
  if (a.precision == FGGC_FP64)
    finish_stage<double2, double>(a, L, base, (double2 *)cells, occ, base + L.off_spec, ws, s);
  else
    finish_stage<float2, float>(a, L, base, (float2 *)cells, occ, base + L.off_spec, ws, s);
}

}  // namespace fggc
