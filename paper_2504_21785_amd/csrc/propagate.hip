// The steps either side of the reconstruction, on gfx950:
//   - the initial decomposition (2.7): A(0, q, p) = 2^{d/2} u0^(q, p) by
//     windowed quadrature on the grid, one wave per packet;
//   - the packet flow of eq. (2.3)-(2.6): one thread per packet, FP64,
//     classical fourth-order Runge-Kutta.
//
// State of a packet: Q and P (d each), S, A (complex) and the Jacobians
// JQ = dz Q and JP = dz P (d x d complex, dz = d_q - i d_p) whose combination
// Z = JQ + i JP enters (2.6).  Differentiating (2.3)-(2.4) along dz gives
//   dJQ/dt = JP,   dJP/dt = -Hess V(Q) JQ,
// and (2.6) reads dA/dt = (A/2) tr(Z^{-1} dZ/dt) with dZ/dt = JP - i Hess V(Q) JQ.
// The potential family is
//   V(x) = c0 + sum_k w_k x_k^2 / 2 + c1 sum_k cos(kappa x_k) + c2 exp(c3 |x|^2),
// with its gradient and Hessian in closed form.
//
// The state lives in registers as NV doubles; a step keeps the state, the
// running RK4 sum, the stage point and one stage derivative.
#include <rocblas/rocblas.h>

#include "common.h"

namespace fggc {
namespace {

template <int D> struct FlowLayout {
  static constexpr int kQ = 0, kP = D, kS = 2 * D, kA = 2 * D + 1, kJQ = 2 * D + 3, kJP = kJQ + 2 * D * D;
  static constexpr int NV = kJP + 2 * D * D;
};

struct PropParams {
  int64_t N;
  double *Q, *P, *S, *a;  // [d][N], [d][N], [N], [N] complex
  double *jac;            // [N][2][d][d] complex or null
  fggc_potential V;
  double dt;
  int64_t nsteps;
};

// d/dt of the state y, written to k
template <int D>
__device__ __forceinline__ void flow_rhs(const double *y, const fggc_potential &V, double *k) {
  using L = FlowLayout<D>;
  const double *q = y + L::kQ, *p = y + L::kP;
  double r2 = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) r2 = fma(q[i], q[i], r2);
  const double E = V.c2 != 0.0 ? V.c2 * exp(V.c3 * r2) : 0.0;
  double val = V.c0 + E, g[D], hd[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    double sn = 0.0, cs = 0.0;
    if (V.c1 != 0.0) sincos(V.kappa * q[i], &sn, &cs);
    val += 0.5 * V.w[i] * q[i] * q[i] + V.c1 * cs;
    g[i] = V.w[i] * q[i] - V.c1 * V.kappa * sn + 2.0 * V.c3 * q[i] * E;
    hd[i] = V.w[i] - V.c1 * V.kappa * V.kappa * cs + 2.0 * V.c3 * E;
  }
  double H[D][D];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int m = 0; m < D; ++m) H[i][m] = (i == m ? hd[i] : 0.0) + 4.0 * V.c3 * V.c3 * q[i] * q[m] * E;

  double ps = 0.0;
#pragma unroll
  for (int i = 0; i < D; ++i) {
    k[L::kQ + i] = p[i];
    k[L::kP + i] = -g[i];
    ps = fma(p[i], p[i], ps);
  }
  k[L::kS] = 0.5 * ps - val;
  // dJQ = JP; dJP = -H JQ (complex entries as (re, im) pairs, row-major)
  const double *jq = y + L::kJQ, *jp = y + L::kJP;
#pragma unroll
  for (int e = 0; e < 2 * D * D; ++e) k[L::kJQ + e] = jp[e];
#pragma unroll
  for (int i = 0; i < D; ++i)
#pragma unroll
    for (int m = 0; m < D; ++m) {
      double re = 0.0, im = 0.0;
#pragma unroll
      for (int l = 0; l < D; ++l) {
        re = fma(-H[i][l], jq[2 * (l * D + m)], re);
        im = fma(-H[i][l], jq[2 * (l * D + m) + 1], im);
      }
      k[L::kJP + 2 * (i * D + m)] = re;
      k[L::kJP + 2 * (i * D + m) + 1] = im;
    }
  // Z = JQ + i JP and dZ = dJQ + i dJP
  double zr[D * D], zi[D * D], wr[D * D], wi[D * D];
#pragma unroll
  for (int e = 0; e < D * D; ++e) {
    zr[e] = jq[2 * e] - jp[2 * e + 1];
    zi[e] = jq[2 * e + 1] + jp[2 * e];
    wr[e] = k[L::kJQ + 2 * e] - k[L::kJP + 2 * e + 1];
    wi[e] = k[L::kJQ + 2 * e + 1] + k[L::kJP + 2 * e];
  }
  // tr(Z^{-1} dZ) = tr(adj(Z) dZ) / det Z
  double cr[D * D], ci[D * D], detr, deti;  // cofactor matrix C (adj = C^T)
  if constexpr (D == 1) {
    cr[0] = 1.0;
    ci[0] = 0.0;
    detr = zr[0];
    deti = zi[0];
  } else if constexpr (D == 2) {
    cr[0] = zr[3]; ci[0] = zi[3];
    cr[1] = -zr[2]; ci[1] = -zi[2];
    cr[2] = -zr[1]; ci[2] = -zi[1];
    cr[3] = zr[0]; ci[3] = zi[0];
    detr = zr[0] * zr[3] - zi[0] * zi[3] - (zr[1] * zr[2] - zi[1] * zi[2]);
    deti = zr[0] * zi[3] + zi[0] * zr[3] - (zr[1] * zi[2] + zi[1] * zr[2]);
  } else {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        const int i1 = (i + 1) % 3, i2 = (i + 2) % 3, m1 = (m + 1) % 3, m2 = (m + 2) % 3;
        // C_im = z[i1][m1] z[i2][m2] - z[i1][m2] z[i2][m1]
        const double ar = zr[i1 * 3 + m1], ai = zi[i1 * 3 + m1], br = zr[i2 * 3 + m2], bi = zi[i2 * 3 + m2];
        const double cr2 = zr[i1 * 3 + m2], ci2 = zi[i1 * 3 + m2], dr = zr[i2 * 3 + m1], di = zi[i2 * 3 + m1];
        cr[i * 3 + m] = ar * br - ai * bi - (cr2 * dr - ci2 * di);
        ci[i * 3 + m] = ar * bi + ai * br - (cr2 * di + ci2 * dr);
      }
    detr = deti = 0.0;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      detr += zr[m] * cr[m] - zi[m] * ci[m];
      deti += zr[m] * ci[m] + zi[m] * cr[m];
    }
  }
  // tr(adj(Z) dZ) = sum_{i,m} C_mi dZ_mi
  double tr = 0.0, ti = 0.0;
#pragma unroll
  for (int e = 0; e < D * D; ++e) {
    tr += cr[e] * wr[e] - ci[e] * wi[e];
    ti += cr[e] * wi[e] + ci[e] * wr[e];
  }
  const double dd = detr * detr + deti * deti;
  const double qr = (tr * detr + ti * deti) / dd, qi = (ti * detr - tr * deti) / dd;
  const double ar = y[L::kA], ai = y[L::kA + 1];
  k[L::kA] = 0.5 * (ar * qr - ai * qi);
  k[L::kA + 1] = 0.5 * (ar * qi + ai * qr);
}

template <int D>
__global__ __launch_bounds__(D < 3 ? 256 : 64) void propagate_kernel(PropParams p) {
  using L = FlowLayout<D>;
  constexpr int NV = L::NV;
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= p.N) return;
  double y[NV];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    y[L::kQ + i] = p.Q[i * p.N + j];
    y[L::kP + i] = p.P[i * p.N + j];
  }
  y[L::kS] = p.S[j];
  y[L::kA] = p.a[2 * j];
  y[L::kA + 1] = p.a[2 * j + 1];
  if (p.jac) {
    const double *src = p.jac + (size_t)j * 4 * D * D;
#pragma unroll
    for (int e = 0; e < 4 * D * D; ++e) y[L::kJQ + e] = src[e];
  } else {
#pragma unroll
    for (int i = 0; i < D; ++i)
#pragma unroll
      for (int m = 0; m < D; ++m) {
        y[L::kJQ + 2 * (i * D + m)] = i == m ? 1.0 : 0.0;
        y[L::kJQ + 2 * (i * D + m) + 1] = 0.0;
        y[L::kJP + 2 * (i * D + m)] = 0.0;
        y[L::kJP + 2 * (i * D + m) + 1] = i == m ? -1.0 : 0.0;
      }
  }
  const fggc_potential V = p.V;
  const double h = p.dt, h2 = 0.5 * p.dt, h3 = p.dt / 3.0, h6 = p.dt / 6.0;
  for (int64_t n = 0; n < p.nsteps; ++n) {
    double acc[NV], st[NV], k[NV];
    flow_rhs<D>(y, V, k);
#pragma unroll
    for (int e = 0; e < NV; ++e) {
      acc[e] = fma(h6, k[e], y[e]);
      st[e] = fma(h2, k[e], y[e]);
    }
    flow_rhs<D>(st, V, k);
#pragma unroll
    for (int e = 0; e < NV; ++e) {
      acc[e] = fma(h3, k[e], acc[e]);
      st[e] = fma(h2, k[e], y[e]);
    }
    flow_rhs<D>(st, V, k);
#pragma unroll
    for (int e = 0; e < NV; ++e) {
      acc[e] = fma(h3, k[e], acc[e]);
      st[e] = fma(h, k[e], y[e]);
    }
    flow_rhs<D>(st, V, k);
#pragma unroll
    for (int e = 0; e < NV; ++e) y[e] = fma(h6, k[e], acc[e]);
  }
#pragma unroll
  for (int i = 0; i < D; ++i) {
    p.Q[i * p.N + j] = y[L::kQ + i];
    p.P[i * p.N + j] = y[L::kP + i];
  }
  p.S[j] = y[L::kS];
  p.a[2 * j] = y[L::kA];
  p.a[2 * j + 1] = y[L::kA + 1];
  if (p.jac) {
    double *dst = p.jac + (size_t)j * 4 * D * D;
#pragma unroll
    for (int e = 0; e < 4 * D * D; ++e) dst[e] = y[L::kJQ + e];
  }
}

struct DecParams {
  int d;
  int64_t N;
  int64_t n[3];
  double dx[3];
  int64_t W[3];   // window half-width in grid steps
  double R2, inv2eps, inveps, wscale;  // wscale = 2^{d/2} prod dx
  const double *u0;  // grid, complex, row-major
  const double *q, *p;
  double *A;
};

// u0^(q, p) = sum over grid points m with |y| <= R of
//   u0(x_m) exp(-i p.y / eps - |y|^2 / (2 eps)) prod dx,  y = minimum image of x_m - q,
// the lanes of a wave striding over the box of grid points around q.
__global__ __launch_bounds__(256) void decompose_kernel(DecParams p) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= p.N) return;  // uniform per wave
  double qk[3] = {0, 0, 0}, pk[3] = {0, 0, 0};
  int64_t start[3] = {0, 0, 0}, side[3] = {1, 1, 1}, total = 1;
  for (int k = 0; k < p.d; ++k) {
    qk[k] = p.q[k * p.N + j];
    pk[k] = p.p[k * p.N + j];
    const double t = (qk[k] + kPi) - kTwoPi * floor((qk[k] + kPi) / kTwoPi);
    int64_t c = (int64_t)rint(t / p.dx[k]);
    if (c >= p.n[k]) c -= p.n[k];
    if (2 * p.W[k] + 1 >= p.n[k]) {
      start[k] = 0;
      side[k] = p.n[k];
    } else {
      start[k] = c - p.W[k];
      if (start[k] < 0) start[k] += p.n[k];
      side[k] = 2 * p.W[k] + 1;
    }
    total *= side[k];
  }
  double ar = 0.0, ai = 0.0;
  for (int64_t e = lane; e < total; e += 64) {
    int64_t rem = e, flat = 0;
    double r2 = 0.0, th = 0.0;
    int64_t mk[3] = {0, 0, 0};
    for (int k = p.d - 1; k >= 0; --k) {
      int64_t m = start[k] + rem % side[k];
      rem /= side[k];
      if (m >= p.n[k]) m -= p.n[k];
      mk[k] = m;
    }
    for (int k = 0; k < p.d; ++k) {
      double y = (-kPi + (double)mk[k] * p.dx[k]) - qk[k];
      y -= kTwoPi * floor((y + kPi) / kTwoPi);
      r2 = fma(y, y, r2);
      th = fma(-pk[k], y, th);
      flat = flat * p.n[k] + mk[k];
    }
    if (r2 <= p.R2) {
      const double g = exp(-r2 * p.inv2eps);
      double sn, cs;
      sincos(th * p.inveps, &sn, &cs);
      const double ur = p.u0[2 * flat], ui = p.u0[2 * flat + 1];
      ar = fma(g, ur * cs - ui * sn, ar);
      ai = fma(g, ur * sn + ui * cs, ai);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    ar += __shfl_xor(ar, off);
    ai += __shfl_xor(ai, off);
  }
  if (lane == 0) {
    p.A[2 * j] = p.wscale * ar;
    p.A[2 * j + 1] = p.wscale * ai;
  }
}

}  // namespace

void launch_decompose(int d, const int64_t *n, const double *u0, double eps, double R, int64_t N,
                      const double *q, const double *pm, double *A, hipStream_t s) {
  if (N == 0) return;
  DecParams p{};
  p.d = d;
  p.N = N;
  p.wscale = std::pow(2.0, 0.5 * d);
  for (int k = 0; k < 3; ++k) {
    p.n[k] = k < d ? n[k] : 1;
    p.dx[k] = k < d ? kTwoPi / (double)n[k] : 1.0;
    p.W[k] = k < d ? (int64_t)std::floor(R / p.dx[k]) + 1 : 0;
    if (k < d) p.wscale *= p.dx[k];
  }
  p.R2 = R * R;
  p.inv2eps = 1.0 / (2.0 * eps);
  p.inveps = 1.0 / eps;
  p.u0 = u0;
  p.q = q;
  p.p = pm;
  p.A = A;
  decompose_kernel<<<dim3((unsigned)((N + 3) / 4)), dim3(256), 0, s>>>(p);
  FGGC_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Decomposition on a product mesh whose q-points are grid points: with the
// window |y_k| <= R per dimension the kernel of (2.7) factors, and for q on
// grid point c the offsets y = (m - c) dx are the same for every q.  Per
// dimension, E_k[j][o] = sqrt(2) dx_k exp(-(o dx_k)^2 / (2 eps) - i p_j o dx_k / eps),
// o = -W..W, so that for each q
//   A(q, .) = E_0 W_q E_1^T,   W_q = the (2W_0+1) x (2W_1+1) window of u0 about q,
// two complex matrix products (FP64) per q, done as strided-batched ZGEMMs
// (rocBLAS) over a periodically padded copy of u0.
namespace {

// E for one dimension; col_major_pj: element (j, o) at j + o * pn, else at o + j * L
__global__ void phase_matrix_kernel(double2 *E, int pn, int L, int W, double dx, double eps, double p0, double dp,
                                    double wscale, int col_major_pj) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= pn * L) return;
  const int j = t % pn, o = t / pn;
  const double y = (double)(o - W) * dx, pj = p0 + (double)j * dp;
  double sn, cs;
  sincos(-pj * y / eps, &sn, &cs);
  const double g = wscale * exp(-y * y / (2.0 * eps));
  E[col_major_pj ? (size_t)j + (size_t)o * pn : (size_t)o + (size_t)j * L] = make_double2(g * cs, g * sn);
}

// U_pad[a][b] = u0[(a - W0) mod n0][(b - W1) mod n1]
__global__ void pad_periodic_kernel(const double2 *u0, double2 *up, int64_t n0, int64_t n1, int64_t W0, int64_t W1) {
  const int64_t cols = n1 + 2 * W1, total = (n0 + 2 * W0) * cols;
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int64_t a = t / cols, b = t % cols;
  int64_t r = (a - W0) % n0, c = (b - W1) % n1;
  if (r < 0) r += n0;
  if (c < 0) c += n1;
  up[t] = u0[r * n1 + c];
}

}  // namespace

void launch_propagate(int d, int64_t N, double *Q, double *P, double *S, double *a, double *jac,
                      const fggc_potential &V, double dt, int64_t nsteps, hipStream_t s) {
  if (N == 0) return;
  PropParams p{};
  p.N = N;
  p.Q = Q;
  p.P = P;
  p.S = S;
  p.a = a;
  p.jac = jac;
  p.V = V;
  p.dt = dt;
  p.nsteps = nsteps;
  const int blk = d < 3 ? 256 : 64;
  const dim3 g((unsigned)((N + blk - 1) / blk)), b(blk);
  if (d == 1) propagate_kernel<1><<<g, b, 0, s>>>(p);
  else if (d == 2) propagate_kernel<2><<<g, b, 0, s>>>(p);
  else propagate_kernel<3><<<g, b, 0, s>>>(p);
  FGGC_HIP(hipGetLastError());
}

}  // namespace fggc

namespace fggc {

size_t decompose_mesh_bytes(int d, const int64_t *n, double R, const int64_t *q_n, const int64_t *p_n) {
  int64_t W[2] = {0, 0}, L[2] = {1, 1};
  for (int k = 0; k < d; ++k) {
    W[k] = (int64_t)std::floor(R / (kTwoPi / (double)n[k]));
    L[k] = 2 * W[k] + 1;
  }
  const int64_t pad = (n[0] + 2 * W[0]) * (d == 2 ? n[1] + 2 * W[1] : 1);
  const int64_t pn1 = d == 2 ? p_n[1] : 1, qn1 = d == 2 ? q_n[1] : 1;
  return (size_t)pad * 16 + (size_t)p_n[0] * L[0] * 16 + (size_t)pn1 * L[1] * 16 +
         (d == 2 ? (size_t)qn1 * pn1 * L[0] * 16 : 0) + 4 * 256;
}

void decompose_mesh(void **blas, int d, const int64_t *n, const double *u0, double eps, double R, const int64_t *Nq,
                    const int64_t *q_lo, const int64_t *q_n, const double *dp, const int64_t *p_lo,
                    const int64_t *p_n, double *A, Workspace &ws, hipStream_t s) {
  if (!*blas) {
    rocblas_handle h = nullptr;
    if (rocblas_create_handle(&h) != rocblas_status_success) fail(FGGC_EDEVICE, "rocblas_create_handle failed");
    *blas = (void *)h;
  }
  rocblas_handle h = (rocblas_handle)*blas;
  if (rocblas_set_stream(h, s) != rocblas_status_success) fail(FGGC_EDEVICE, "rocblas_set_stream failed");
  int64_t W[2] = {0, 0}, L[2] = {1, 1}, st[2] = {1, 1};
  double dx[2] = {1, 1};
  for (int k = 0; k < d; ++k) {
    dx[k] = kTwoPi / (double)n[k];
    W[k] = (int64_t)std::floor(R / dx[k]);
    L[k] = 2 * W[k] + 1;
    st[k] = n[k] / Nq[k];
  }
  const int64_t n1 = d == 2 ? n[1] : 1;
  const int64_t pad_rows = n[0] + 2 * W[0], pad_cols = d == 2 ? n1 + 2 * W[1] : 1;
  // workspace: padded u0, E per dimension, and one q-row of intermediate products
  const int64_t pn0 = p_n[0], pn1 = d == 2 ? p_n[1] : 1, qn1 = d == 2 ? q_n[1] : 1;
  const size_t b_up = (size_t)pad_rows * pad_cols * 16, b_e0 = (size_t)pn0 * L[0] * 16,
               b_e1 = (size_t)pn1 * L[1] * 16, b_t = d == 2 ? (size_t)qn1 * pn1 * L[0] * 16 : 0;
  // the caller reserved decompose_mesh_bytes() in ws
  double2 *up = (double2 *)ws.take(b_up), *E0 = (double2 *)ws.take(b_e0), *E1 = (double2 *)ws.take(b_e1);
  double2 *T = d == 2 ? (double2 *)ws.take(b_t) : nullptr;
  const int64_t tot = pad_rows * pad_cols;
  if (d == 1) {
    pad_periodic_kernel<<<dim3((unsigned)((tot + 255) / 256)), 256, 0, s>>>((const double2 *)u0, up, n[0], 1, W[0], 0);
  } else {
    pad_periodic_kernel<<<dim3((unsigned)((tot + 255) / 256)), 256, 0, s>>>((const double2 *)u0, up, n[0], n1, W[0],
                                                                              W[1]);
  }
  FGGC_HIP(hipGetLastError());
  const double w2 = std::sqrt(2.0);
  // dimension 0: 1D uses (j, o) column-major (pn x L); 2D uses E0^T column-major (L0 x pn0)
  phase_matrix_kernel<<<dim3((unsigned)((pn0 * L[0] + 255) / 256)), 256, 0, s>>>(
      E0, (int)pn0, (int)L[0], (int)W[0], dx[0], eps, (double)p_lo[0] * dp[0], dp[0], w2 * dx[0], d == 1);
  FGGC_HIP(hipGetLastError());
  if (d == 2) {
    phase_matrix_kernel<<<dim3((unsigned)((pn1 * L[1] + 255) / 256)), 256, 0, s>>>(
        E1, (int)pn1, (int)L[1], (int)W[1], dx[1], eps, (double)p_lo[1] * dp[1], dp[1], w2 * dx[1], 1);
    FGGC_HIP(hipGetLastError());
  }
  const rocblas_double_complex one = {1.0, 0.0}, zero = {0.0, 0.0};
  auto check = [](rocblas_status r) {
    if (r != rocblas_status_success) fail(FGGC_EDEVICE, std::string("rocBLAS ZGEMM failed: ") + rocblas_status_to_string(r));
  };
  double2 *out = (double2 *)A;
  if (d == 1) {
    // A(q_i, .) = E (pn x L) . u_pad[c_i .. c_i + L), c_i = (q_lo + i) st: one batch over q
    const double2 *b0 = up + q_lo[0] * st[0];
    check(rocblas_zgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_none, (rocblas_int)pn0, 1,
                                        (rocblas_int)L[0], &one, (const rocblas_double_complex *)E0, (rocblas_int)pn0,
                                        0, (const rocblas_double_complex *)b0, (rocblas_int)L[0], st[0], &zero,
                                        (rocblas_double_complex *)out, (rocblas_int)pn0, pn0, (rocblas_int)q_n[0]));
    return;
  }
  // 2D, one q-row i0 at a time (column-major views of row-major arrays):
  //   T_i1^T (pn1 x L0) = E1 (pn1 x L1) . W_q^T (L1 x L0),  W_q^T at up + c0 * pad_cols + c1, ld pad_cols
  //   A_q^T  (pn1 x pn0) = T_i1^T . E0^T (L0 x pn0)
  for (int64_t i0 = 0; i0 < q_n[0]; ++i0) {
    const int64_t c0 = (q_lo[0] + i0) * st[0];
    const double2 *bq = up + c0 * pad_cols + q_lo[1] * st[1];
    check(rocblas_zgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_none, (rocblas_int)pn1,
                                        (rocblas_int)L[0], (rocblas_int)L[1], &one,
                                        (const rocblas_double_complex *)E1, (rocblas_int)pn1, 0,
                                        (const rocblas_double_complex *)bq, (rocblas_int)pad_cols, st[1], &zero,
                                        (rocblas_double_complex *)T, (rocblas_int)pn1, pn1 * L[0], (rocblas_int)qn1));
    check(rocblas_zgemm_strided_batched(h, rocblas_operation_none, rocblas_operation_none, (rocblas_int)pn1,
                                        (rocblas_int)pn0, (rocblas_int)L[0], &one, (const rocblas_double_complex *)T,
                                        (rocblas_int)pn1, pn1 * L[0], (const rocblas_double_complex *)E0,
                                        (rocblas_int)L[0], 0, &zero,
                                        (rocblas_double_complex *)(out + i0 * qn1 * pn0 * pn1), (rocblas_int)pn1,
                                        pn0 * pn1, (rocblas_int)qn1));
  }
}

void destroy_blas(void *blas) {
  if (blas) (void)rocblas_destroy_handle((rocblas_handle)blas);
}

}  // namespace fggc
