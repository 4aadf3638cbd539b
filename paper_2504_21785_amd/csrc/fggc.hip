// Frozen Gaussian grid-point correction on gfx950 (Section 2.3, Alg. 2).
//
//   coef_scatter  one thread per packet, FP64: int/frac split (3.6)-(3.7) per
//                 dimension, right-hand side (3.23), least squares through the
//                 plan's eigenpairs (c^ = V diag(1/lambda) V^H f~), conjugation
//                 to the L2-best coefficients, shift (3.13), Kronecker product
//                 over dimensions, times scale a exp(i S/eps); the contributions
//                 are added into the dense cell array of eq. (2.25) with
//                 hardware float atomics (FP32 or FP64 cells).
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

__global__ void range_init_kernel(long long *r) {
  if (threadIdx.x < 3) {
    r[threadIdx.x] = 0x7fffffffffffffffLL;
    r[3 + threadIdx.x] = -0x7fffffffffffffffLL - 1;
  }
}

__global__ void pcell_range_kernel(int d, int64_t N, const double *__restrict__ P, double dp0,
                                   double dp1, double dp2, long long *r) {
  __shared__ long long smin[3][256], smax[3][256];
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const double dp[3] = {dp0, dp1, dp2};
  for (int k = 0; k < 3; ++k) {
    long long mn = 0x7fffffffffffffffLL, mx = -0x7fffffffffffffffLL - 1;
    if (k < d && j < N) {
      int64_t ip;
      double t;
      const double w = P[k * N + j] / dp[k];
      if (isfinite(w) && fabs(w) < 9.0e15) {
        int_frac(w, ip, t);
        mn = mx = ip;
      } else {  // poisons the range so that the host rejects the request
        mn = -0x7fffffffffffffffLL - 1;
        mx = 0x7fffffffffffffffLL;
      }
    }
    smin[k][threadIdx.x] = mn;
    smax[k][threadIdx.x] = mx;
  }
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st)
      for (int k = 0; k < 3; ++k) {
        smin[k][threadIdx.x] = min(smin[k][threadIdx.x], smin[k][threadIdx.x + st]);
        smax[k][threadIdx.x] = max(smax[k][threadIdx.x], smax[k][threadIdx.x + st]);
      }
    __syncthreads();
  }
  if (threadIdx.x < d) {
    atomicMin(&r[threadIdx.x], smin[threadIdx.x][0]);
    atomicMax(&r[3 + threadIdx.x], smax[threadIdx.x][0]);
  }
}

template <typename T>
__global__ void fill_zero_kernel(T *__restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = T{0, 0};
}

struct CoefParams {
  int64_t N;
  const double *Q, *P, *S, *a;
  double eps, scale;
  const DimLsq *lsq;  // [d], device copy of the plan
  int64_t Nq[3], slo[3], sn[3];
  double dq[3], dp[3];
};

// per-dimension least-squares coefficients c_k (after conjugation and shift)
template <int N1>
__device__ __forceinline__ void dim_coeffs(const DimLsq &L, double Q, double P, double dq, double dp,
                                           int64_t &iq, int64_t &ip, double cre[N1], double cim[N1]) {
  double s, t;
  int_frac(Q / dq, iq, s);
  int_frac(P / dp, ip, t);
  const double Cq = L.Cq, Cp = L.Cp, CC = Cq * Cp;
  const int n1 = L.n1;
  double fre[N1], fim[N1];
#pragma unroll
  for (int j = 0; j < N1; ++j) {
    fre[j] = 0.0;
    fim[j] = 0.0;
    if (j < n1) {
      // eq. (3.23)
      const double a = (double)L.dq[j] - s, b = (double)L.dp[j] - t;
      const double mag = exp(-0.25 * (Cq * Cq * a * a + Cp * Cp * b * b));
      double sn, cs;
      sincos(0.5 * CC * (s - (double)L.dq[j]) * ((double)L.dp[j] + t), &sn, &cs);
      fre[j] = mag * cs;
      fim[j] = mag * sn;
    }
  }
  // z = diag(inv) V^H f
  double zre[N1], zim[N1];
#pragma unroll
  for (int i = 0; i < N1; ++i) {
    double yr = 0.0, yi = 0.0;
#pragma unroll
    for (int j = 0; j < N1; ++j) {
      const double vr = L.V[2 * (j * n1 + i)], vi = L.V[2 * (j * n1 + i) + 1];
      if (i < n1 && j < n1) {
        // conj(V_ji) * f_j
        yr = fma(vr, fre[j], fma(vi, fim[j], yr));
        yi = fma(vr, fim[j], fma(-vi, fre[j], yi));
      }
    }
    const double w = i < n1 ? L.inv[i] : 0.0;
    zre[i] = yr * w;
    zim[i] = yi * w;
  }
  // c^ = V z ; c~ = conj(c^) ; c = c~ exp(-i Cq Cp (s - dq_j) ip)
#pragma unroll
  for (int j = 0; j < N1; ++j) {
    double hr = 0.0, hi = 0.0;
#pragma unroll
    for (int i = 0; i < N1; ++i) {
      const double vr = L.V[2 * (j * n1 + i)], vi = L.V[2 * (j * n1 + i) + 1];
      if (i < n1 && j < n1) {
        hr = fma(vr, zre[i], fma(-vi, zim[i], hr));
        hi = fma(vr, zim[i], fma(vi, zre[i], hi));
      }
    }
    const double tr = hr, ti = -hi;  // conjugate
    double sn = 0.0, cs = 1.0;
    if (j < n1) {
      // phase -Cq Cp (s - dq_j) ip in revolutions, reduced before sin/cos
      const double rev = -CC * (s - (double)L.dq[j]) * (double)ip * (1.0 / kTwoPi);
      sincospi(2.0 * (rev - rint(rev)), &sn, &cs);
    }
    cre[j] = tr * cs - ti * sn;
    cim[j] = tr * sn + ti * cs;
  }
}

template <int D, int N1, bool F64>
__global__ __launch_bounds__(256) void coef_scatter_kernel(CoefParams p, void *__restrict__ cells_v) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= p.N) return;
  double cre[D][N1], cim[D][N1];
  int64_t iq[D], ip[D];
#pragma unroll
  for (int k = 0; k < D; ++k)
    dim_coeffs<N1>(p.lsq[k], p.Q[k * p.N + j], p.P[k * p.N + j], p.dq[k], p.dp[k], iq[k], ip[k],
                   cre[k], cim[k]);
  // alpha = scale a exp(i S / eps), phase reduced in revolutions
  double sn, cs;
  {
    const double rev = p.S[j] / (kTwoPi * p.eps);
    sincospi(2.0 * (rev - rint(rev)), &sn, &cs);
  }
  const double ar = p.scale * p.a[2 * j], ai = p.scale * p.a[2 * j + 1];
  const double alr = ar * cs - ai * sn, ali = ar * sn + ai * cs;
  const int n1 = p.lsq[0].n1;
  // strides of the cell array and this packet's base indices per dimension
  int64_t nqt = 1, sstr[3] = {0, 0, 0}, qstr[3] = {0, 0, 0}, sbase[3] = {0, 0, 0}, qbase[3] = {0, 0, 0},
          qmask[3] = {0, 0, 0};
  {
    int64_t ss = 1, qs = 1;
    for (int k = D - 1; k >= 0; --k) {
      sstr[k] = ss;
      qstr[k] = qs;
      ss *= p.sn[k];
      qs *= p.Nq[k];
      sbase[k] = ip[k] - p.slo[k];
      qbase[k] = iq[k] + p.Nq[k] / 2;
      qmask[k] = p.Nq[k] - 1;  // Nq is a power of two
    }
    nqt = qs;
  }
  auto emit = [&](double vr, double vi, int64_t sl, int64_t qi) {
    const int64_t cell = sl * nqt + qi;
    if (F64) {
      double *c = (double *)cells_v + 2 * cell;
      atomicAdd(c, vr);
      atomicAdd(c + 1, vi);
    } else {
      float *c = (float *)cells_v + 2 * cell;
      atomicAdd(c, (float)vr);
      atomicAdd(c + 1, (float)vi);
    }
  };
  const DimLsq &L0 = p.lsq[0];
#pragma unroll
  for (int a0 = 0; a0 < N1; ++a0) {
    if (a0 >= n1) break;
    const double v0r = alr * cre[0][a0] - ali * cim[0][a0];
    const double v0i = alr * cim[0][a0] + ali * cre[0][a0];
    const int64_t s0 = (sbase[0] + L0.dp[a0]) * sstr[0];
    const int64_t q0 = ((qbase[0] + L0.dq[a0]) & qmask[0]) * qstr[0];
    if (D == 1) {
      emit(v0r, v0i, s0, q0);
      continue;
    }
    const DimLsq &L1 = p.lsq[D > 1 ? 1 : 0];
#pragma unroll
    for (int a1 = 0; a1 < N1; ++a1) {
      if (a1 >= n1) break;
      const double v1r = v0r * cre[D > 1 ? 1 : 0][a1] - v0i * cim[D > 1 ? 1 : 0][a1];
      const double v1i = v0r * cim[D > 1 ? 1 : 0][a1] + v0i * cre[D > 1 ? 1 : 0][a1];
      const int64_t s1 = s0 + (sbase[1] + L1.dp[a1]) * sstr[1];
      const int64_t q1 = q0 + ((qbase[1] + L1.dq[a1]) & qmask[1]) * qstr[1];
      if (D == 2) {
        emit(v1r, v1i, s1, q1);
        continue;
      }
      const DimLsq &L2 = p.lsq[D > 2 ? 2 : 0];
#pragma unroll
      for (int a2 = 0; a2 < N1; ++a2) {
        if (a2 >= n1) break;
        const double v2r = v1r * cre[D > 2 ? 2 : 0][a2] - v1i * cim[D > 2 ? 2 : 0][a2];
        const double v2i = v1r * cim[D > 2 ? 2 : 0][a2] + v1i * cre[D > 2 ? 2 : 0][a2];
        emit(v2r, v2i, s1 + (sbase[2] + L2.dp[a2]) * sstr[2],
             q1 + ((qbase[2] + L2.dq[a2]) & qmask[2]) * qstr[2]);
      }
    }
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
  int64_t ncells, nslices, npts;
  int64_t nb[3], toff[3], koff[3], ntab, nkst;
  size_t off_lsq, off_cells, off_gam, off_kst, total;
};

FggcLayout fggc_layout(const FggcArgs &a) {
  FggcLayout L{};
  const int d = a.g.d;
  const size_t es = a.precision == FGGC_FP64 ? 16 : 8;
  L.nslices = 1;
  int64_t nqt = 1;
  L.npts = 1;
  L.ntab = 0;
  L.nkst = 0;
  for (int k = 0; k < 3; ++k) {
    if (k < d) {
      L.nslices *= a.sn[k];
      nqt *= a.Nq[k];
      L.npts *= a.g.n[k];
      L.nb[k] = (int64_t)std::floor(2.0 * a.cK / std::sqrt(a.eps)) + 2;
      L.toff[k] = L.ntab;
      L.koff[k] = L.nkst;
      L.ntab += a.sn[k] * L.nb[k];
      L.nkst += a.sn[k];
    } else {
      L.nb[k] = 1;
      L.toff[k] = 0;
      L.koff[k] = 0;
    }
  }
  L.ncells = L.nslices * nqt;
  size_t o = 0;
  auto put = [&](size_t bytes) {
    size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  L.off_lsq = put(3 * sizeof(DimLsq));
  L.off_cells = put((size_t)L.ncells * es);
  L.off_gam = put((size_t)L.ntab * (es / 2));
  L.off_kst = put((size_t)L.nkst * 8 + 64);
  L.total = o;
  return L;
}

template <int D, bool F64>
void launch_coef(const CoefParams &cp, void *cells, int n1, hipStream_t s) {
  const dim3 grid((unsigned)((cp.N + 255) / 256)), blk(256);
  if (n1 <= 4) {
    coef_scatter_kernel<D, 4, F64><<<grid, blk, 0, s>>>(cp, cells);
  } else if (n1 <= 8) {
    coef_scatter_kernel<D, 8, F64><<<grid, blk, 0, s>>>(cp, cells);
  } else {
    if constexpr (D < 3) coef_scatter_kernel<D, 16, F64><<<grid, blk, 0, s>>>(cp, cells);
    else fail(FGGC_EUNSUPPORTED, "3D strategies need nq * np <= 8");
  }
  FGGC_HIP(hipGetLastError());
}

// zero the cells and add every packet's contributions
void cells_stage(const FggcArgs &a, const FggcLayout &L, void *cells, DimLsq *dlsq, hipStream_t s) {
  const int d = a.g.d;
  const bool f64 = a.precision == FGGC_FP64;
  FGGC_HIP(hipMemcpyAsync(dlsq, a.lsq, d * sizeof(DimLsq), hipMemcpyHostToDevice, s));
  {
    StageScope sc(a.prof, "fggc_zero", s);
    const int64_t n = L.ncells;
    const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
    if (f64) fill_zero_kernel<double2><<<nb, 256, 0, s>>>((double2 *)cells, n);
    else fill_zero_kernel<float2><<<nb, 256, 0, s>>>((float2 *)cells, n);
    FGGC_HIP(hipGetLastError());
  }
  if (a.pk->N == 0) return;
  CoefParams cp{};
  cp.N = a.pk->N;
  cp.Q = a.pk->Q;
  cp.P = a.pk->P;
  cp.S = a.pk->S;
  cp.a = a.pk->a;
  cp.eps = a.eps;
  cp.scale = a.scale;
  cp.lsq = dlsq;
  for (int k = 0; k < 3; ++k) {
    cp.Nq[k] = a.Nq[k];
    cp.slo[k] = a.slo[k];
    cp.sn[k] = a.sn[k];
    cp.dq[k] = kTwoPi / (double)a.Nq[k];
    cp.dp[k] = a.dp[k];
  }
  const int n1 = a.lsq[0].n1;
  StageScope sc(a.prof, "fggc_coef_scatter", s);
  if (d == 1) { if (f64) launch_coef<1, true>(cp, cells, n1, s); else launch_coef<1, false>(cp, cells, n1, s); }
  else if (d == 2) { if (f64) launch_coef<2, true>(cp, cells, n1, s); else launch_coef<2, false>(cp, cells, n1, s); }
  else { if (f64) launch_coef<3, true>(cp, cells, n1, s); else launch_coef<3, false>(cp, cells, n1, s); }
}

template <typename T, typename R>
void finish_stage(const FggcArgs &a, const FggcLayout &L, T *cells, R *gam, int64_t *kst,
                  Workspace &ws, hipStream_t s) {
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
  T *U = (T *)a.u;
  const unsigned nblk = (unsigned)((L.npts + 255) / 256);
  {
  StageScope sc(a.prof, "fggc_band_mac", s);
  if (d == 1) band_mac_kernel<1, T, R><<<nblk, 256, 0, s>>>(m, cells, gam, kst, U);
  else if (d == 2) band_mac_kernel<2, T, R><<<nblk, 256, 0, s>>>(m, cells, gam, kst, U);
  else band_mac_kernel<3, T, R><<<nblk, 256, 0, s>>>(m, cells, gam, kst, U);
  FGGC_HIP(hipGetLastError());
  }
  // F7: inverse DFT of the grid spectrum
  launch_fft(d, a.g.n, 1, +1, prec, U, ws, s, a.prof, "fggc_ifft");
}

}  // namespace

void launch_pcell_range(const fggc_packets &pk, const double *dp, long long *dev, hipStream_t s) {
  range_init_kernel<<<1, 64, 0, s>>>(dev);
  FGGC_HIP(hipGetLastError());
  if (pk.N == 0) return;
  pcell_range_kernel<<<dim3((unsigned)((pk.N + 255) / 256)), dim3(256), 0, s>>>(
      pk.d, pk.N, pk.P, dp[0], pk.d > 1 ? dp[1] : 1.0, pk.d > 2 ? dp[2] : 1.0, dev);
  FGGC_HIP(hipGetLastError());
}

size_t fggc_workspace_bytes(const FggcArgs &a) { return fggc_layout(a).total + 1024; }

size_t fggc_cells_workspace_bytes(const FggcArgs &a) {
  FggcLayout L = fggc_layout(a);
  return L.off_cells + 1024;
}

void launch_fggc_cells(const FggcArgs &a, void *cells, Workspace &ws, hipStream_t s) {
  FggcLayout L = fggc_layout(a);
  DimLsq *dlsq = (DimLsq *)ws.take(3 * sizeof(DimLsq));
  cells_stage(a, L, cells, dlsq, s);
}

void launch_fggc(const FggcArgs &a, Workspace &ws, hipStream_t s) {
  FggcLayout L = fggc_layout(a);
  char *base = (char *)ws.take(L.total);
  DimLsq *dlsq = (DimLsq *)(base + L.off_lsq);
  void *cells = base + L.off_cells;
  cells_stage(a, L, cells, dlsq, s);
  if (a.precision == FGGC_FP64)
    finish_stage<double2, double>(a, L, (double2 *)cells, (double *)(base + L.off_gam),
                                  (int64_t *)(base + L.off_kst), ws, s);
  else
    finish_stage<float2, float>(a, L, (float2 *)cells, (float *)(base + L.off_gam),
                                (int64_t *)(base + L.off_kst), ws, s);
}

}  // namespace fggc
