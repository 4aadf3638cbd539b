/*
 * oracle.c -- plain, slow, FP64 CPU oracle for Gaussian wave-packet
 * reconstruction.  TEST INFRASTRUCTURE ONLY: the product library never links,
 * loads or calls this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark do.  It shares no code, header or table with
 * the HIP path.
 *
 * What it computes, after Chai & Deng, "Frozen Gaussian Grid-point
 * Correction for Semi-classical Schroedinger Equation":
 *
 *   oracle_direct_sum        the discrete reconstruction sum, eq. (2.10) and
 *                            eq. (2.19), on the periodic grid [-pi,pi)^d,
 *                            minimum image, Euclidean window |y| <= R.
 *   oracle_direct_sum_boxwin the same sum with a box window: every component
 *                            of the minimum image satisfies |y_k| <= R.
 *   oracle_direct_bruteforce the same sum with no window, over all periodic
 *                            images n in [-nimg,nimg]^d (for tiny inputs).
 *   oracle_inner             packet inner product, eq. (2.17).
 *   oracle_gram / oracle_rhs shifted normal equations of Theorem 2 written
 *                            without eps, eq. (3.22) and eq. (3.23).
 *   oracle_lsa               per-packet least squares, eq. (2.11)-(2.14),
 *                            (2.22), in the shifted form of Theorem 2
 *                            (3.9)-(3.13); returns the coefficients and the
 *                            relative error E_LSA of eq. (3.4).
 *   oracle_mlsa              M_LSA, eq. (3.24)-(3.25), as the maximum of
 *                            E_LSA over a sample grid of the unit cell.
 *   oracle_fggc_cells        the on-grid combination A~(q,p) of eq. (2.25):
 *                            Alg. 2 step 3 (int/frac split eq. (3.6)-(3.7),
 *                            precomputed Gram, coefficient shift eq. (3.13))
 *                            and the scatter of eq. (2.23)-(2.25).
 *   oracle_eval_cells        eq. (2.24) evaluated plainly over the cells
 *                            (no FFT), minimum image, window |y| <= Ro.
 *   oracle_fggc_points       the two above at a list of grid points, keeping
 *                            only the cells within Ro of those points (for
 *                            grids whose dense cell array does not fit).
 *
 * Readings of the paper taken here (each is pinned by a test):
 *   - Conjugation.  With <g,h> = int g conj(h) (eq. 2.14), A_jk = <psi_j,psi_k>
 *     and f_j = <psi_j,phi> (eq. 2.13), the printed system A c = f is the
 *     complex conjugate of the normal equations of min ||phi - sum c psi||.
 *     The L2-best coefficients are therefore conj(A^+ f).  The shift of
 *     eq. (3.13) then carries a minus sign:
 *         c_k = c~_k * exp(-i Cq Cp (s - dq_k) ip)
 *     where s = frac(Q)/dq, ip = floor(P/dp), Cq = dq/sqrt(eps),
 *     Cp = dp/sqrt(eps).
 *   - Tensor strategies.  For a shift set that is a tensor product over
 *     dimensions, the Gram matrix and right-hand side of eq. (3.22)-(3.23)
 *     factor over dimensions, so the d-dimensional coefficients are the
 *     Kronecker product of one-dimensional ones.  oracle_fggc_cells uses this
 *     factorisation; oracle_lsa solves the full d-dimensional system, which is
 *     how the factorisation is checked.
 *   - Pseudo-inverse (remark after Alg. 1).  rcond > 0 drops eigenvalues
 *     below rcond * lambda_max of the Gram matrix; rcond == 0 is the exact
 *     least-squares solution (Cholesky).  Linear algebra on the Gram matrix is
 *     done in long double so that the oracle's own error stays far below the
 *     FP64 conditioning floor of the method.
 *   - Cells.  q-mesh q_i = -pi + i*dq (dq = 2 pi / Nq, Nq even) is the floor
 *     anchoring of eq. (2.20) at 0, stored at index (iq + dq_k + Nq/2) mod Nq;
 *     p-mesh p_l = l*dp is not wrapped.  A fractional part that rounds to 1
 *     is moved to the next cell.
 *
 * All complex arrays are interleaved (re, im) doubles.  Grid points are
 * x_m = -pi + m * 2 pi / M per dimension, flattened row-major (last
 * dimension fastest).  Every function returns 0 on success and a negative
 * value on invalid arguments.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef long double _Complex cld;

#define TWO_PI (2.0 * M_PI)
#define MAXN 64 /* largest basis handled by oracle_lsa (d-dimensional) */
#define MAXN1 16 /* largest per-dimension basis handled by oracle_fggc_cells */

/* ------------------------------------------------------------------------ */
/* small helpers                                                            */
/* ------------------------------------------------------------------------ */

/* y wrapped into [-pi, pi): the minimum-image displacement on the torus. */
static double wrap_pi(double y) { return y - TWO_PI * floor((y + M_PI) / TWO_PI); }

static int64_t imod(int64_t a, int64_t m) {
  int64_t r = a % m;
  return r < 0 ? r + m : r;
}

static void unflatten(int d, const int64_t *M, int64_t flat, int64_t *m) {
  for (int k = d - 1; k >= 0; --k) {
    m[k] = flat % M[k];
    flat /= M[k];
  }
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the oracle's parallel loops (n >= 1); returns the previous count. */
int oracle_set_threads(int n) {
  const int prev = omp_get_max_threads();
  if (n >= 1) omp_set_num_threads(n);
  return prev;
}

/* ------------------------------------------------------------------------ */
/* direct sum, eq. (2.10) / (2.19)                                          */
/* ------------------------------------------------------------------------ */

/* One packet term a * exp(i (S + P.y)/eps - |y|^2/(2 eps)) for displacement y. */
static double complex packet_term(int d, const double *y, double Pj[3], double Sj, double complex aj,
                                  double eps) {
  double r2 = 0.0, py = 0.0;
  for (int k = 0; k < d; ++k) {
    r2 += y[k] * y[k];
    py += Pj[k] * y[k];
  }
  double ph = (Sj + py) / eps;
  return aj * exp(-r2 / (2.0 * eps)) * (cos(ph) + I * sin(ph));
}

/*
 * u_m = scale * sum_j a_j exp(i (S_j + P_j.y)/eps - |y|^2/(2 eps)) [ |y|^2 <= R^2 ],
 * y = minimum image of x_m - Q_j.  Q, P are [d][N]; S is [N]; a is [N]
 * complex.  pts lists npts flat grid indices (NULL: every grid point, in
 * order); u receives npts complex values.  Requires 0 < R < pi.
 *
 * Packets are grouped in a uniform bin grid whose bins are at least R wide,
 * so that a point only visits the 3^d bins around its own; every candidate is
 * still tested against the window exactly.
 */
static int direct_sum_window(int d, int64_t N, const double *Q, const double *P, const double *S,
                             const double *a, double eps, const int64_t *M, double R, double scale,
                             int64_t npts, const int64_t *pts, double *u, int box) {
  if (d < 1 || d > 3 || N < 0 || !(eps > 0) || !(R > 0) || !(R < M_PI)) return -1;
  int64_t total = 1;
  for (int k = 0; k < d; ++k) {
    if (M[k] < 1) return -1;
    total *= M[k];
  }
  if (!pts) npts = total;
  int64_t B = (int64_t)floor(TWO_PI / R);
  if (B < 1) B = 1;
  const double bw = TWO_PI / (double)B;
  int64_t nb = 1;
  for (int k = 0; k < d; ++k) nb *= B;
  int64_t *start = (int64_t *)calloc((size_t)nb + 1, sizeof(int64_t));
  int64_t *order = (int64_t *)malloc((size_t)(N > 0 ? N : 1) * sizeof(int64_t));
  int64_t *binof = (int64_t *)malloc((size_t)(N > 0 ? N : 1) * sizeof(int64_t));
  if (!start || !order || !binof) {
    free(start); free(order); free(binof);
    return -2;
  }
  for (int64_t j = 0; j < N; ++j) {
    int64_t b = 0;
    for (int k = 0; k < d; ++k) {
      int64_t c = (int64_t)floor((wrap_pi(Q[k * N + j]) + M_PI) / bw);
      if (c < 0) c = 0;
      if (c >= B) c = B - 1;
      b = b * B + c;
    }
    binof[j] = b;
    start[b + 1]++;
  }
  for (int64_t b = 0; b < nb; ++b) start[b + 1] += start[b];
  {
    int64_t *fill = (int64_t *)malloc((size_t)nb * sizeof(int64_t));
    memcpy(fill, start, (size_t)nb * sizeof(int64_t));
    for (int64_t j = 0; j < N; ++j) order[fill[binof[j]]++] = j;
    free(fill);
  }
  /* neighbour offsets per dimension: {-1,0,1} when B >= 3, else every bin once */
  int noff = B >= 3 ? 3 : (int)B;
  int64_t offs[3];
  if (B >= 3) { offs[0] = -1; offs[1] = 0; offs[2] = 1; }
  else for (int i = 0; i < noff; ++i) offs[i] = i;

#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t ip = 0; ip < npts; ++ip) {
    int64_t flat = pts ? pts[ip] : ip, m[3] = {0, 0, 0}, cb[3] = {0, 0, 0};
    double x[3] = {0, 0, 0};
    unflatten(d, M, flat, m);
    for (int k = 0; k < d; ++k) {
      x[k] = -M_PI + (double)m[k] * (TWO_PI / (double)M[k]);
      cb[k] = (int64_t)floor((x[k] + M_PI) / bw);
      if (cb[k] >= B) cb[k] = B - 1;
    }
    double complex acc = 0.0;
    int nvis = 1;
    for (int k = 0; k < d; ++k) nvis *= noff;
    for (int v = 0; v < nvis; ++v) {
      int64_t b = 0;
      int vv = v;
      for (int k = 0; k < d; ++k) {
        int o = vv % noff;
        vv /= noff;
        int64_t c = B >= 3 ? imod(cb[k] + offs[o], B) : offs[o];
        b = b * B + c;
      }
      for (int64_t t = start[b]; t < start[b + 1]; ++t) {
        int64_t j = order[t];
        double y[3], r2 = 0.0, ymax = 0.0, Pj[3] = {0, 0, 0};
        for (int k = 0; k < d; ++k) {
          y[k] = wrap_pi(x[k] - Q[k * N + j]);
          r2 += y[k] * y[k];
          ymax = fmax(ymax, fabs(y[k]));
          Pj[k] = P[k * N + j];
        }
        if (box ? ymax > R : r2 > R * R) continue;
        acc += packet_term(d, y, Pj, S[j], a[2 * j] + I * a[2 * j + 1], eps);
      }
    }
    acc *= scale;
    u[2 * ip] = creal(acc);
    u[2 * ip + 1] = cimag(acc);
  }
  free(start); free(order); free(binof);
  return 0;
}

int oracle_direct_sum(int d, int64_t N, const double *Q, const double *P, const double *S,
                      const double *a, double eps, const int64_t *M, double R, double scale,
                      int64_t npts, const int64_t *pts, double *u) {
  return direct_sum_window(d, N, Q, P, S, a, eps, M, R, scale, npts, pts, u, 0);
}

/*
 * The sum of oracle_direct_sum with the window max_k |y_k| <= R (a box of
 * half-width R about the packet centre) instead of the ball |y| <= R.  The
 * box contains the ball, so this sum drops less of each packet's tail.
 */
int oracle_direct_sum_boxwin(int d, int64_t N, const double *Q, const double *P, const double *S,
                             const double *a, double eps, const int64_t *M, double R, double scale,
                             int64_t npts, const int64_t *pts, double *u) {
  return direct_sum_window(d, N, Q, P, S, a, eps, M, R, scale, npts, pts, u, 1);
}

/*
 * Untruncated sum over every packet and every periodic image
 * y = wrap(x_m - Q_j) + 2 pi n, n in [-nimg, nimg]^d, at every grid point.
 * Cost N * prod(M) * (2 nimg + 1)^d: for tiny inputs only.
 */
int oracle_direct_bruteforce(int d, int64_t N, const double *Q, const double *P, const double *S,
                             const double *a, double eps, const int64_t *M, int nimg,
                             double scale, double *u) {
  if (d < 1 || d > 3 || N < 0 || !(eps > 0) || nimg < 0) return -1;
  int64_t total = 1;
  for (int k = 0; k < d; ++k) {
    if (M[k] < 1) return -1;
    total *= M[k];
  }
  int side = 2 * nimg + 1, nimgs = 1;
  for (int k = 0; k < d; ++k) nimgs *= side;
#pragma omp parallel for schedule(static)
  for (int64_t flat = 0; flat < total; ++flat) {
    int64_t m[3] = {0, 0, 0};
    double x[3] = {0, 0, 0};
    unflatten(d, M, flat, m);
    for (int k = 0; k < d; ++k) x[k] = -M_PI + (double)m[k] * (TWO_PI / (double)M[k]);
    double complex acc = 0.0;
    for (int64_t j = 0; j < N; ++j) {
      double Pj[3] = {0, 0, 0}, y0[3] = {0, 0, 0};
      for (int k = 0; k < d; ++k) {
        Pj[k] = P[k * N + j];
        y0[k] = wrap_pi(x[k] - Q[k * N + j]);
      }
      for (int v = 0; v < nimgs; ++v) {
        double y[3];
        int vv = v;
        for (int k = 0; k < d; ++k) {
          y[k] = y0[k] + TWO_PI * (double)(vv % side - nimg);
          vv /= side;
        }
        acc += packet_term(d, y, Pj, S[j], a[2 * j] + I * a[2 * j + 1], eps);
      }
    }
    acc *= scale;
    u[2 * flat] = creal(acc);
    u[2 * flat + 1] = cimag(acc);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* packet inner products, eq. (2.17), (3.22), (3.23)                        */
/* ------------------------------------------------------------------------ */

/*
 * <G(.;Qa,Pa), G(.;Qb,Pb)> = int G_a conj(G_b) dx
 *   = (pi eps)^{d/2} exp(-|Qb-Qa|^2/(4 eps) - |Pb-Pa|^2/(4 eps)
 *                        + i (Qb-Qa).(Pb+Pa)/(2 eps)),   eq. (2.17).
 * Q*, P* are [d]; out is one complex value.
 */
int oracle_inner(int d, const double *Qa, const double *Pa, const double *Qb, const double *Pb,
                 double eps, double *out) {
  if (d < 1 || d > 3 || !(eps > 0)) return -1;
  double dq2 = 0, dp2 = 0, ph = 0;
  for (int k = 0; k < d; ++k) {
    dq2 += (Qb[k] - Qa[k]) * (Qb[k] - Qa[k]);
    dp2 += (Pb[k] - Pa[k]) * (Pb[k] - Pa[k]);
    ph += (Qb[k] - Qa[k]) * (Pb[k] + Pa[k]);
  }
  double complex v = pow(M_PI * eps, 0.5 * d) *
                     cexp(-dq2 / (4 * eps) - dp2 / (4 * eps) + I * ph / (2 * eps));
  out[0] = creal(v);
  out[1] = cimag(v);
  return 0;
}

/* eq. (3.22) entry for shifts (dqj,dpj), (dqk,dpk) in d dimensions, long double. */
static cld gram_entry(int d, const int *dqj, const int *dpj, const int *dqk, const int *dpk,
                      const double *Cq, const double *Cp) {
  long double re = 0, im = 0;
  for (int l = 0; l < d; ++l) {
    long double cq = Cq[l], cp = Cp[l];
    long double a = dqj[l] - dqk[l], b = dpj[l] - dpk[l];
    re += -cq * cq * a * a / 4 - cp * cp * b * b / 4;
    im += cq * cp * (long double)(dqk[l] - dqj[l]) * (long double)(dpj[l] + dpk[l]) / 2;
  }
  return cexpl(re + I * im);
}

/* eq. (3.23) entry for shift (dqj,dpj) and fractional position (s,t). */
static cld rhs_entry(int d, const int *dqj, const int *dpj, const double *s, const double *t,
                     const double *Cq, const double *Cp) {
  long double re = 0, im = 0;
  for (int l = 0; l < d; ++l) {
    long double cq = Cq[l], cp = Cp[l];
    long double a = (long double)dqj[l] - s[l], b = (long double)dpj[l] - t[l];
    re += -cq * cq * a * a / 4 - cp * cp * b * b / 4;
    im += cq * cp * ((long double)s[l] - dqj[l]) * ((long double)dpj[l] + t[l]) / 2;
  }
  return cexpl(re + I * im);
}

/* Gram matrix of eq. (3.22) for n shifts (dq, dp are [n][d]); out is [n][n] complex. */
int oracle_gram(int d, int n, const int *dq, const int *dp, const double *Cq, const double *Cp,
                double *out) {
  if (d < 1 || d > 3 || n < 1) return -1;
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k) {
      cld v = gram_entry(d, dq + j * d, dp + j * d, dq + k * d, dp + k * d, Cq, Cp);
      out[2 * (j * n + k)] = (double)creall(v);
      out[2 * (j * n + k) + 1] = (double)cimagl(v);
    }
  return 0;
}

/* Right-hand side of eq. (3.23); out is [n] complex. */
int oracle_rhs(int d, int n, const int *dq, const int *dp, const double *Cq, const double *Cp,
               const double *s, const double *t, double *out) {
  if (d < 1 || d > 3 || n < 1) return -1;
  for (int j = 0; j < n; ++j) {
    cld v = rhs_entry(d, dq + j * d, dp + j * d, s, t, Cq, Cp);
    out[2 * j] = (double)creall(v);
    out[2 * j + 1] = (double)cimagl(v);
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* linear algebra on the (small) Gram matrix, long double                  */
/* ------------------------------------------------------------------------ */

/* A = L L^H for Hermitian positive definite A (n x n); L lower.  0 on success. */
static int cholesky(int n, const cld *A, cld *L) {
  memset(L, 0, sizeof(cld) * n * n);
  for (int j = 0; j < n; ++j) {
    long double dsum = creall(A[j * n + j]);
    for (int k = 0; k < j; ++k) dsum -= creall(L[j * n + k] * conjl(L[j * n + k]));
    if (!(dsum > 0)) return -1;
    long double djj = sqrtl(dsum);
    L[j * n + j] = djj;
    for (int i = j + 1; i < n; ++i) {
      cld v = A[i * n + j];
      for (int k = 0; k < j; ++k) v -= L[i * n + k] * conjl(L[j * n + k]);
      L[i * n + j] = v / djj;
    }
  }
  return 0;
}

static void cholesky_solve(int n, const cld *L, const cld *f, cld *x) {
  cld y[MAXN];
  for (int i = 0; i < n; ++i) {
    cld v = f[i];
    for (int k = 0; k < i; ++k) v -= L[i * n + k] * y[k];
    y[i] = v / L[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    cld v = y[i];
    for (int k = i + 1; k < n; ++k) v -= conjl(L[k * n + i]) * x[k];
    x[i] = v / conjl(L[i * n + i]);
  }
}

/*
 * Cyclic Jacobi eigen-decomposition of a real symmetric m x m matrix (long
 * double).  On return w holds eigenvalues and V (row-major) the eigenvectors
 * as columns.
 */
static void jacobi_sym(int m, long double *A, long double *w, long double *V) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) V[i * m + j] = (i == j);
  for (int sweep = 0; sweep < 100; ++sweep) {
    long double off = 0, tot = 0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        tot += A[i * m + j] * A[i * m + j];
        if (i != j) off += A[i * m + j] * A[i * m + j];
      }
    if (off <= 1e-38L * tot) break;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) {
        long double apq = A[p * m + q];
        if (apq == 0) continue;
        long double theta = (A[q * m + q] - A[p * m + p]) / (2 * apq);
        long double t = (theta >= 0 ? 1 : -1) / (fabsl(theta) + sqrtl(theta * theta + 1));
        long double c = 1 / sqrtl(t * t + 1), s = t * c;
        for (int k = 0; k < m; ++k) { /* A <- A J */
          long double akp = A[k * m + p], akq = A[k * m + q];
          A[k * m + p] = c * akp - s * akq;
          A[k * m + q] = s * akp + c * akq;
        }
        for (int k = 0; k < m; ++k) { /* A <- J^T A */
          long double apk = A[p * m + k], aqk = A[q * m + k];
          A[p * m + k] = c * apk - s * aqk;
          A[q * m + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < m; ++k) {
          long double vkp = V[k * m + p], vkq = V[k * m + q];
          V[k * m + p] = c * vkp - s * vkq;
          V[k * m + q] = s * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < m; ++i) w[i] = A[i * m + i];
}

/*
 * Solver for the printed system  A~ c' = f~  (n x n Hermitian A~).
 * rcond == 0: Cholesky (exact least squares).  rcond > 0: pseudo-inverse
 * through the real 2n x 2n embedding [[Re A, -Im A], [Im A, Re A]], whose
 * eigenvalues are those of A~ (each twice), dropping those below
 * rcond * lambda_max.
 */
typedef struct {
  int n, mode;
  cld L[MAXN * MAXN];
  long double *Pinv; /* 2n x 2n real pseudo-inverse of the embedding */
} solver_t;

static int solver_init(solver_t *sv, int n, const cld *A, double rcond) {
  sv->n = n;
  sv->Pinv = NULL;
  if (rcond <= 0) {
    sv->mode = 0;
    return cholesky(n, A, sv->L);
  }
  sv->mode = 1;
  int m = 2 * n;
  long double *E = (long double *)malloc(sizeof(long double) * m * m);
  long double *V = (long double *)malloc(sizeof(long double) * m * m);
  long double *w = (long double *)malloc(sizeof(long double) * m);
  sv->Pinv = (long double *)calloc((size_t)m * m, sizeof(long double));
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      long double re = creall(A[i * n + j]), im = cimagl(A[i * n + j]);
      E[i * m + j] = re;
      E[i * m + (j + n)] = -im;
      E[(i + n) * m + j] = im;
      E[(i + n) * m + (j + n)] = re;
    }
  jacobi_sym(m, E, w, V);
  long double wmax = 0;
  for (int i = 0; i < m; ++i) wmax = fmaxl(wmax, w[i]);
  for (int k = 0; k < m; ++k) {
    if (!(w[k] > (long double)rcond * wmax)) continue;
    long double inv = 1 / w[k];
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) sv->Pinv[i * m + j] += V[i * m + k] * inv * V[j * m + k];
  }
  free(E); free(V); free(w);
  return 0;
}

static void solver_apply(const solver_t *sv, const cld *f, cld *x) {
  int n = sv->n;
  if (sv->mode == 0) {
    cholesky_solve(n, sv->L, f, x);
    return;
  }
  int m = 2 * n;
  for (int i = 0; i < n; ++i) {
    long double re = 0, im = 0;
    for (int j = 0; j < n; ++j) {
      re += sv->Pinv[i * m + j] * creall(f[j]) + sv->Pinv[i * m + j + n] * cimagl(f[j]);
      im += sv->Pinv[(i + n) * m + j] * creall(f[j]) + sv->Pinv[(i + n) * m + j + n] * cimagl(f[j]);
    }
    x[i] = re + I * im;
  }
}

static void solver_free(solver_t *sv) { free(sv->Pinv); }

/*
 * Least-squares approximation of G(.; Cq s, Cp t) by G(.; Cq dq_k, Cp dp_k),
 * k = 0..n-1, in the eps-free variables of Theorem 3 (eq. 3.19-3.23).
 * dq, dp are [n][d] integer shifts; s, t are [d] in [0,1].
 * c_out[n] (complex) receives the L2-best coefficients c~ = conj(A~^+ f~);
 * *E_out receives E_LSA of eq. (3.4):
 *   E^2 = 1 - 2 Re(sum_k c_k f~_k) + sum_{k,j} c_k conj(c_j) A~_kj.
 */
int oracle_lsa(int d, int n, const int *dq, const int *dp, const double *Cq, const double *Cp,
               double rcond, const double *s, const double *t, double *c_out, double *E_out) {
  if (d < 1 || d > 3 || n < 1 || n > MAXN) return -1;
  cld *A = (cld *)malloc(sizeof(cld) * n * n);
  cld f[MAXN], ch[MAXN], c[MAXN];
  for (int j = 0; j < n; ++j)
    for (int k = 0; k < n; ++k) A[j * n + k] = gram_entry(d, dq + j * d, dp + j * d, dq + k * d, dp + k * d, Cq, Cp);
  for (int j = 0; j < n; ++j) f[j] = rhs_entry(d, dq + j * d, dp + j * d, s, t, Cq, Cp);
  solver_t *sv = (solver_t *)malloc(sizeof(solver_t));
  if (solver_init(sv, n, A, rcond) != 0) {
    solver_free(sv); free(sv); free(A);
    return -3;
  }
  solver_apply(sv, f, ch);
  for (int k = 0; k < n; ++k) c[k] = conjl(ch[k]);
  long double e2 = 1;
  cld cf = 0, quad = 0;
  for (int k = 0; k < n; ++k) cf += c[k] * f[k];
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j) quad += c[k] * conjl(c[j]) * A[k * n + j];
  e2 += -2 * creall(cf) + creall(quad);
  if (c_out)
    for (int k = 0; k < n; ++k) {
      c_out[2 * k] = (double)creall(c[k]);
      c_out[2 * k + 1] = (double)cimagl(c[k]);
    }
  if (E_out) *E_out = (double)sqrtl(fmaxl(e2, 0));
  solver_free(sv);
  free(sv);
  free(A);
  return 0;
}

/*
 * M_LSA of eq. (3.25) for a one-dimensional strategy: the maximum of E_LSA
 * over the (ns x nt) grid s_i = i/(ns-1), t_j = j/(nt-1) of the unit cell
 * (eq. 3.15).  Returns the maximum and where it is attained.
 */
int oracle_mlsa(int n, const int *dq, const int *dp, double Cq, double Cp, double rcond, int ns,
                int nt, double *sup, double *s_at, double *t_at) {
  if (n < 1 || n > MAXN1 || ns < 2 || nt < 2) return -1;
  double best = -1, bs = 0, bt = 0;
  int bad = 0;
#pragma omp parallel for schedule(dynamic, 4) collapse(2)
  for (int i = 0; i < ns; ++i)
    for (int j = 0; j < nt; ++j) {
      double s = (double)i / (ns - 1), t = (double)j / (nt - 1), E = 0;
      if (oracle_lsa(1, n, dq, dp, &Cq, &Cp, rcond, &s, &t, NULL, &E) != 0) {
#pragma omp atomic write
        bad = 1;
        continue;
      }
#pragma omp critical
      {
        if (E > best) { best = E; bs = s; bt = t; }
      }
    }
  if (bad) return -3;
  *sup = best;
  if (s_at) *s_at = bs;
  if (t_at) *t_at = bt;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* FGGC: on-grid combination (2.23)-(2.25) and its evaluation (2.24)        */
/* ------------------------------------------------------------------------ */

/* integer and fractional part of v per eq. (3.6)-(3.7); a fraction that rounds to 1 moves up a cell */
static void int_frac(double v, int64_t *ip, double *fr) {
  double fl = floor(v);
  double f = v - fl;
  int64_t i = (int64_t)fl;
  if (f >= 1.0) {
    f = 0.0;
    i += 1;
  }
  *ip = i;
  *fr = f;
}

/* floor(P/dp) range per dimension over all packets. */
int oracle_pcell_bounds(int d, int64_t N, const double *P, const double *dpm, int64_t *lo,
                        int64_t *hi) {
  if (d < 1 || d > 3 || N < 1) return -1;
  for (int k = 0; k < d; ++k) {
    int64_t mn = INT64_MAX, mx = INT64_MIN;
    for (int64_t j = 0; j < N; ++j) {
      int64_t ip;
      double t;
      int_frac(P[k * N + j] / dpm[k], &ip, &t);
      if (ip < mn) mn = ip;
      if (ip > mx) mx = ip;
    }
    lo[k] = mn;
    hi[k] = mx;
  }
  return 0;
}

/*
 * Where a cell (slice sl, q index qi) is stored.  Dense: every cell, at
 * sl * nstore + qi (nstore = all q indices).  Sparse: only the q indices
 * listed in qmap (qmap[qi] >= 0, a compact q slot), q-major at
 * qmap[qi] * nstore + sl (nstore = slices); a contribution to any other q is
 * not stored.  The arithmetic of each stored cell is the same in both.
 */
typedef struct {
  const int64_t *qmap; /* NULL: dense */
  int64_t nstore;
} cellstore_t;

static int64_t cell_slot(const cellstore_t *cs, int64_t sl, int64_t qi) {
  if (!cs->qmap) return sl * cs->nstore + qi;
  const int64_t k = cs->qmap[qi];
  return k < 0 ? -1 : k * cs->nstore + sl;
}

/*
 * The scatter of eq. (2.23)-(2.25) over every packet:
 *   cell(ip + dp_K, iq + dq_K) += scale * a_j exp(i S_j/eps) c_j^(K).
 * In the sparse form a packet none of whose neighbours is stored adds nothing,
 * so its coefficients are not formed.
 */
static int fggc_scatter(int d, int64_t N, const double *Q, const double *P, const double *S,
                        const double *a, double eps, const int64_t *Nq, const double *dpm, int nq,
                        const int *dq_off, int np, const int *dp_off, double rcond, double scale,
                        const int64_t *slo, const int64_t *sn, const cellstore_t *cs, double *cells) {
  if (d < 1 || d > 3 || N < 0 || !(eps > 0) || nq < 1 || np < 1 || nq * np > MAXN1) return -1;
  int n1 = nq * np;
  double Cq[3], Cp[3];
  for (int k = 0; k < d; ++k) {
    if (Nq[k] < 2 || Nq[k] % 2 || !(dpm[k] > 0) || sn[k] < 1) return -1;
    Cq[k] = (TWO_PI / (double)Nq[k]) / sqrt(eps);
    Cp[k] = dpm[k] / sqrt(eps);
  }
  /* per-dimension shift lists and precomputed solver (Alg. 2, step 0) */
  int sq[MAXN1], sp[MAXN1];
  for (int ia = 0; ia < nq; ++ia)
    for (int ib = 0; ib < np; ++ib) {
      sq[ia * np + ib] = dq_off[ia];
      sp[ia * np + ib] = dp_off[ib];
    }
  solver_t *sv = (solver_t *)calloc(3, sizeof(solver_t));
  for (int k = 0; k < d; ++k) {
    cld A[MAXN1 * MAXN1];
    for (int j = 0; j < n1; ++j)
      for (int i = 0; i < n1; ++i) A[j * n1 + i] = gram_entry(1, &sq[j], &sp[j], &sq[i], &sp[i], &Cq[k], &Cp[k]);
    if (solver_init(&sv[k], n1, A, rcond) != 0) {
      for (int q = 0; q <= k; ++q) solver_free(&sv[q]);
      free(sv);
      return -3;
    }
  }
  int64_t nK = 1, nqK = 1;
  for (int k = 0; k < d; ++k) {
    nK *= n1;
    nqK *= nq;
  }
  int err = 0;

#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t j = 0; j < N; ++j) {
    cld c1[3][MAXN1];
    int64_t iq[3], ip[3];
    double s[3], t[3];
    for (int k = 0; k < d; ++k) {
      int_frac(Q[k * N + j] / (TWO_PI / (double)Nq[k]), &iq[k], &s[k]);
      int_frac(P[k * N + j] / dpm[k], &ip[k], &t[k]);
    }
    if (cs->qmap) {
      /* is any of the packet's q neighbours stored? */
      int any = 0;
      for (int64_t K = 0; K < nqK && !any; ++K) {
        int64_t rem = K, qi = 0;
        int kk[3];
        for (int k = d - 1; k >= 0; --k) {
          kk[k] = (int)(rem % nq);
          rem /= nq;
        }
        for (int k = 0; k < d; ++k) qi = qi * Nq[k] + imod(iq[k] + dq_off[kk[k]] + Nq[k] / 2, Nq[k]);
        any = cs->qmap[qi] >= 0;
      }
      if (!any) continue;
    }
    for (int k = 0; k < d; ++k) {
      cld f[MAXN1], ch[MAXN1];
      for (int i = 0; i < n1; ++i) f[i] = rhs_entry(1, &sq[i], &sp[i], &s[k], &t[k], &Cq[k], &Cp[k]);
      solver_apply(&sv[k], f, ch);
      for (int i = 0; i < n1; ++i) {
        /* c~ = conj(A~^+ f~), then the shift of eq. (3.13) */
        long double ph = -(long double)Cq[k] * Cp[k] * ((long double)s[k] - sq[i]) * (long double)ip[k];
        c1[k][i] = conjl(ch[i]) * cexpl(I * ph);
      }
    }
    double ph0 = S[j] / eps;
    double complex alpha = scale * (a[2 * j] + I * a[2 * j + 1]) * (cos(ph0) + I * sin(ph0));
    for (int64_t K = 0; K < nK; ++K) {
      int64_t rem = K, sl = 0, qi = 0;
      cld coef = 1;
      int ok = 1;
      int kk[3];
      for (int k = d - 1; k >= 0; --k) {
        kk[k] = (int)(rem % n1);
        rem /= n1;
      }
      for (int k = 0; k < d; ++k) {
        int b = kk[k];
        coef *= c1[k][b];
        int64_t l = ip[k] + sp[b] - slo[k];
        if (l < 0 || l >= sn[k]) ok = 0;
        sl = sl * sn[k] + l;
        qi = qi * Nq[k] + imod(iq[k] + sq[b] + Nq[k] / 2, Nq[k]);
      }
      if (!ok) {
#pragma omp atomic write
        err = 1;
        continue;
      }
      const int64_t at = cell_slot(cs, sl, qi);
      if (at < 0) continue;
      double complex v = alpha * (double complex)coef;
      double *cell = cells + 2 * at;
#pragma omp atomic
      cell[0] += creal(v);
#pragma omp atomic
      cell[1] += cimag(v);
    }
  }
  for (int k = 0; k < d; ++k) solver_free(&sv[k]);
  free(sv);
  return err ? -4 : 0;
}

/*
 * Dense cell array A~(q_i, p_l) of eq. (2.25) (times `scale`):
 *   cells[l][i] += scale * a_j exp(i S_j/eps) c_j^(k)
 * for every packet j and neighbour k (eq. 2.23).  The strategy is the tensor
 * product over dimensions of the one-dimensional shift set
 * {(dq_off[a], dp_off[b])}, a < nq, b < np (basis index a*np + b), with
 * dq = 2 pi / Nq[k] and dp = dpm[k] per dimension.
 * slo[d] / sn[d] give the box of p-cells stored: slice l (row-major over the
 * box) holds p-cells slo + l; q index i (row-major, last dim fastest) holds
 * q = -pi + i dq.  cells is [prod sn][prod Nq] complex and is ADDED to.
 */
int oracle_fggc_cells(int d, int64_t N, const double *Q, const double *P, const double *S,
                      const double *a, double eps, const int64_t *Nq, const double *dpm, int nq,
                      const int *dq_off, int np, const int *dp_off, double rcond, double scale,
                      const int64_t *slo, const int64_t *sn, double *cells) {
  if (d < 1 || d > 3) return -1;
  cellstore_t cs = {NULL, 1};
  for (int k = 0; k < d; ++k) cs.nstore *= Nq[k];
  return fggc_scatter(d, N, Q, P, S, a, eps, Nq, dpm, nq, dq_off, np, dp_off, rcond, scale, slo, sn, &cs,
                      cells);
}

/*
 * The q indices a grid point x sees: per dimension the indices within reach
 * of x +- Ro (each visited once), minimum image y = wrap(x - q_i), and only
 * those with |y| <= Ro.  Calls back with (flat q index, y) in row-major order.
 */
typedef void (*ball_fn)(void *ctx, int64_t qi, const double *y);

static void visit_ball(int d, const double *x, const int64_t *Nq, double Ro, ball_fn fn, void *ctx) {
  int64_t i0[3] = {0, 0, 0}, ni[3] = {1, 1, 1};
  for (int k = 0; k < d; ++k) {
    double dqk = TWO_PI / (double)Nq[k];
    int64_t lo = (int64_t)floor((x[k] - Ro + M_PI) / dqk) - 1;
    int64_t hi = (int64_t)ceil((x[k] + Ro + M_PI) / dqk) + 1;
    if (hi - lo + 1 >= Nq[k]) {
      i0[k] = 0;
      ni[k] = Nq[k];
    } else {
      i0[k] = lo;
      ni[k] = hi - lo + 1;
    }
  }
  int64_t nbox = 1;
  for (int k = 0; k < d; ++k) nbox *= ni[k];
  for (int64_t bq = 0; bq < nbox; ++bq) {
    int64_t rem = bq, qi = 0;
    double y[3] = {0, 0, 0}, r2 = 0;
    int64_t idx[3];
    for (int k = d - 1; k >= 0; --k) {
      idx[k] = imod(i0[k] + rem % ni[k], Nq[k]);
      rem /= ni[k];
    }
    for (int k = 0; k < d; ++k) {
      double qv = -M_PI + (double)idx[k] * (TWO_PI / (double)Nq[k]);
      y[k] = wrap_pi(x[k] - qv);
      r2 += y[k] * y[k];
      qi = qi * Nq[k] + idx[k];
    }
    if (r2 > Ro * Ro) continue;
    fn(ctx, qi, y);
  }
}

static void grid_point(int d, const int64_t *M, int64_t flat, double *x) {
  int64_t m[3] = {0, 0, 0};
  unflatten(d, M, flat, m);
  for (int k = 0; k < d; ++k) x[k] = -M_PI + (double)m[k] * (TWO_PI / (double)M[k]);
}

/* sum over the cells at one q index of A~(q, p_l) G(x; q, p_l), eq. (2.24) */
typedef struct {
  int d;
  const double *cells;
  const cellstore_t *cs;
  const int64_t *slo, *sn;
  const double *dpm;
  double eps;
  int64_t nsl;
  double complex acc;
  int missing;
} evalctx_t;

static void eval_at_q(void *vp, int64_t qi, const double *y) {
  evalctx_t *e = (evalctx_t *)vp;
  const int d = e->d;
  if (cell_slot(e->cs, 0, qi) < 0) {
    e->missing = 1;
    return;
  }
  double r2 = 0;
  for (int k = 0; k < d; ++k) r2 += y[k] * y[k];
  double g = exp(-r2 / (2 * e->eps));
  for (int64_t l = 0; l < e->nsl; ++l) {
    const double *cell = e->cells + 2 * cell_slot(e->cs, l, qi);
    if (cell[0] == 0.0 && cell[1] == 0.0) continue;
    int64_t lr = l, li[3];
    for (int k = d - 1; k >= 0; --k) {
      li[k] = lr % e->sn[k];
      lr /= e->sn[k];
    }
    double py = 0;
    for (int k = 0; k < d; ++k) py += (double)(e->slo[k] + li[k]) * e->dpm[k] * y[k];
    double ph = py / e->eps;
    e->acc += (cell[0] + I * cell[1]) * g * (cos(ph) + I * sin(ph));
  }
}

/* the q indices (and their y) a point sees, collected in visiting order */
typedef struct {
  int d;
  int64_t n, cap;
  int64_t *qi;
  double *y;
} balllist_t;

static void collect_q(void *vp, int64_t qi, const double *y) {
  balllist_t *b = (balllist_t *)vp;
  if (b->n == b->cap) {
    b->cap = b->cap ? 2 * b->cap : 4096;
    b->qi = (int64_t *)realloc(b->qi, sizeof(int64_t) * b->cap);
    b->y = (double *)realloc(b->y, sizeof(double) * 3 * b->cap);
  }
  b->qi[b->n] = qi;
  for (int k = 0; k < 3; ++k) b->y[3 * b->n + k] = k < b->d ? y[k] : 0.0;
  b->n += 1;
}

static int eval_cells_store(int d, const double *cells, const cellstore_t *cs, const int64_t *slo,
                            const int64_t *sn, const int64_t *Nq, const double *dpm, double eps,
                            const int64_t *M, double Ro, int64_t npts, const int64_t *pts, double *u) {
  if (d < 1 || d > 3 || !(eps > 0) || !(Ro > 0) || !(Ro < M_PI)) return -1;
  int64_t total = 1, nsl = 1;
  for (int k = 0; k < d; ++k) {
    if (M[k] < 1 || Nq[k] < 2 || Nq[k] % 2 || sn[k] < 1) return -1;
    total *= M[k];
    nsl *= sn[k];
  }
  if (!pts) npts = total;
  int missing = 0;
  if (npts >= 4 * oracle_num_threads()) {
    /* many points: one point per iteration */
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t ipt = 0; ipt < npts; ++ipt) {
      double x[3] = {0, 0, 0};
      grid_point(d, M, pts ? pts[ipt] : ipt, x);
      evalctx_t e = {d, cells, cs, slo, sn, dpm, eps, nsl, 0.0, 0};
      visit_ball(d, x, Nq, Ro, eval_at_q, &e);
      if (e.missing) {
#pragma omp atomic write
        missing = 1;
      }
      u[2 * ipt] = creal(e.acc);
      u[2 * ipt + 1] = cimag(e.acc);
    }
    return missing ? -5 : 0;
  }
  /* few points: the q indices of one point are shared out instead (the same
     terms, summed in another order) */
  balllist_t b = {d, 0, 0, NULL, NULL};
  for (int64_t ipt = 0; ipt < npts; ++ipt) {
    double x[3] = {0, 0, 0};
    grid_point(d, M, pts ? pts[ipt] : ipt, x);
    b.n = 0;
    visit_ball(d, x, Nq, Ro, collect_q, &b);
    double re = 0.0, im = 0.0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : re, im)
    for (int64_t i = 0; i < b.n; ++i) {
      evalctx_t e = {d, cells, cs, slo, sn, dpm, eps, nsl, 0.0, 0};
      eval_at_q(&e, b.qi[i], b.y + 3 * i);
      if (e.missing) {
#pragma omp atomic write
        missing = 1;
      }
      re += creal(e.acc);
      im += cimag(e.acc);
    }
    u[2 * ipt] = re;
    u[2 * ipt + 1] = im;
  }
  free(b.qi);
  free(b.y);
  return missing ? -5 : 0;
}

/*
 * u_m = sum over cells of A~(q_i, p_l) G(x_m; q_i, p_l), eq. (2.24), evaluated
 * directly: minimum image y = wrap(x_m - q_i), cells with |y| <= Ro only.
 * Layout of cells as in oracle_fggc_cells; pts / npts / u as in
 * oracle_direct_sum.  Requires 0 < Ro < pi.
 */
int oracle_eval_cells(int d, const double *cells, const int64_t *slo, const int64_t *sn,
                      const int64_t *Nq, const double *dpm, double eps, const int64_t *M, double Ro,
                      int64_t npts, const int64_t *pts, double *u) {
  if (d < 1 || d > 3) return -1;
  cellstore_t cs = {NULL, 1};
  for (int k = 0; k < d; ++k) cs.nstore *= Nq[k];
  return eval_cells_store(d, cells, &cs, slo, sn, Nq, dpm, eps, M, Ro, npts, pts, u);
}

/* marks q indices (qmap[qi] = 0) */
static void mark_q(void *vp, int64_t qi, const double *y) {
  (void)y;
  ((int64_t *)vp)[qi] = 0;
}

typedef struct {
  const int64_t *qmap;
  int64_t fresh;
} countctx_t;

static void count_new_q(void *vp, int64_t qi, const double *y) {
  (void)y;
  countctx_t *c = (countctx_t *)vp;
  if (c->qmap[qi] < 0) c->fresh += 1;
}

/*
 * FGGC at the grid points pts[0..npts) without the dense cell array: the same
 * scatter (eq. 2.23-2.25) and the same plain evaluation of eq. (2.24) as
 * oracle_fggc_cells followed by oracle_eval_cells, but only the cells whose q
 * lies within Ro of the points are kept.  Points are taken in batches whose
 * kept cells fit in max_bytes (at least one point per batch); every batch
 * scatters all packets into its own cells.  slo / sn as in oracle_fggc_cells
 * (they must contain every p-cell the packets touch).  u receives npts complex.
 */
int oracle_fggc_points(int d, int64_t N, const double *Q, const double *P, const double *S,
                       const double *a, double eps, const int64_t *Nq, const double *dpm, int nq,
                       const int *dq_off, int np, const int *dp_off, double rcond, double scale,
                       const int64_t *slo, const int64_t *sn, const int64_t *M, double Ro, int64_t npts,
                       const int64_t *pts, double max_bytes, double *u) {
  if (d < 1 || d > 3 || npts < 0 || !pts || !(Ro > 0) || !(Ro < M_PI) || !(max_bytes > 0)) return -1;
  int64_t nqt = 1, nsl = 1;
  for (int k = 0; k < d; ++k) {
    if (Nq[k] < 2 || Nq[k] % 2 || sn[k] < 1 || M[k] < 1) return -1;
    nqt *= Nq[k];
    nsl *= sn[k];
  }
  int64_t *qmap = (int64_t *)malloc(sizeof(int64_t) * nqt);
  if (!qmap) return -2;
  int rc = 0;
  for (int64_t i0 = 0; i0 < npts && rc == 0;) {
    for (int64_t q = 0; q < nqt; ++q) qmap[q] = -1;
    /* grow the batch while its cells fit */
    int64_t nq_used = 0, i1 = i0;
    while (i1 < npts) {
      double x[3] = {0, 0, 0};
      grid_point(d, M, pts[i1], x);
      countctx_t c = {qmap, 0};
      visit_ball(d, x, Nq, Ro, count_new_q, &c);
      if (i1 > i0 && (double)(nq_used + c.fresh) * (double)nsl * 16.0 > max_bytes) break;
      visit_ball(d, x, Nq, Ro, mark_q, qmap);
      nq_used += c.fresh;
      ++i1;
    }
    int64_t ns = 0;
    for (int64_t q = 0; q < nqt; ++q)
      if (qmap[q] >= 0) qmap[q] = ns++;
    double *cells = (double *)calloc((size_t)(ns * nsl) * 2 + 2, sizeof(double));
    if (!cells) {
      rc = -2;
      break;
    }
    cellstore_t cs = {qmap, nsl};
    rc = fggc_scatter(d, N, Q, P, S, a, eps, Nq, dpm, nq, dq_off, np, dp_off, rcond, scale, slo, sn, &cs,
                      cells);
    if (rc == 0)
      rc = eval_cells_store(d, cells, &cs, slo, sn, Nq, dpm, eps, M, Ro, i1 - i0, pts + i0, u + 2 * i0);
    free(cells);
    i0 = i1;
  }
  free(qmap);
  return rc;
}
