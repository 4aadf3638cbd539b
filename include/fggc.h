/*
 * fggc.h -- C ABI of libfggc, the MI355X (gfx950) library that reconstructs
 * a wave function on a uniform periodic grid from frozen Gaussian
 * wave-packets.
 *
 * Method: Chai & Deng, "Frozen Gaussian Grid-point Correction for
 * Semi-classical Schroedinger Equation" (arXiv 2504.21785).
 *
 *   u(x) = scale * sum_j a_j exp( i (S_j + P_j.(x - Q_j)) / eps - |x - Q_j|^2 / (2 eps) )
 *
 * is the discrete reconstruction sum of eq. (2.10) / (2.19) with the
 * prefactor (dq dp)^d / (2 pi eps)^{3d/2} of that equation folded into the
 * caller's `scale`.  Two forms compute it:
 *   fggc_direct_sum   every packet at every grid point within a window radius;
 *   fggc_reconstruct  frozen Gaussian grid-point correction (Section 2.3 and
 *                     Alg. 2): each packet is replaced by its least-squares fit
 *                     on on-grid packets (eq. 2.20-2.22, 3.9-3.13, 3.22-3.23),
 *                     the coefficients are summed per phase-space cell
 *                     (eq. 2.25) and eq. (2.24) is evaluated with FFTs.
 * fggc_direct_sum_separable evaluates the direct sum under a box window as a
 * product of matrices on the matrix cores (2D).  The steps around the
 * reconstruction are here too: fggc_decompose (initial packets, eq. 2.7) and
 * fggc_propagate (the packet flow, eq. 2.3-2.6).
 *
 * Conventions shared by every call
 *   - Domain [-pi, pi)^d, periodic; grid x_m = -pi + m * 2 pi / n per
 *     dimension; d in {1, 2, 3}.  Distances use the minimum image.
 *   - Packets are structure-of-arrays FP64: Q[d][N], P[d][N], S[N], and
 *     a[N] complex128 (interleaved re, im).
 *   - Output u is row-major over the grid (last dimension fastest),
 *     interleaved complex: complex64 for FGGC_FP32, complex128 for FGGC_FP64.
 *   - Pointers may be device memory (hipMalloc, or a torch CUDA tensor's
 *     data_ptr) or ordinary host memory; host buffers are staged through the
 *     context's device workspace and the call then completes before it
 *     returns.  The caller owns every buffer; the library keeps no pointer
 *     after a call returns.
 *   - `stream` is a hipStream_t (NULL = the default stream).  With device
 *     buffers the call is stream-ordered: it enqueues work and returns;
 *     buffers must stay valid until the stream has passed the call.
 *   - Every call returns an fggc_status; no C++ exception crosses the ABI.
 *     fggc_last_error() describes the last failure on the calling thread.
 *   - A context is used by one thread at a time (calls on one context are
 *     serialised by an internal lock).
 */
#ifndef FGGC_H
#define FGGC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FGGC_OK = 0,
  FGGC_EINVAL = -1,       /* invalid argument (NaN/Inf input, eps <= 0, bad d, bad size, ...) */
  FGGC_ENOMEM = -2,       /* device allocation failed */
  FGGC_EBUDGET = -3,      /* the request can never fit in the context's HBM budget */
  FGGC_EUNSUPPORTED = -4, /* valid but not supported (e.g. an FFT size with a prime factor above 5) */
  FGGC_EDEVICE = -5,      /* a HIP runtime call failed */
  FGGC_ECANCELLED = -6,   /* a served request was cancelled */
  FGGC_ETIMEOUT = -7      /* fggc_server_wait timed out; the request is still pending */
} fggc_status;

typedef enum { FGGC_FP32 = 0, FGGC_FP64 = 1 } fggc_precision;

typedef struct fggc_ctx fggc_ctx;

/* Periodic grid [-pi,pi)^d with n[k] points in dimension k (n[k] >= 1). */
typedef struct {
  int32_t d;
  int64_t n[3];
} fggc_grid;

/* N packets in d dimensions; see the conventions above.  N = 0 is allowed. */
typedef struct {
  int32_t d;
  int64_t N;
  const double *Q; /* [d][N] centres */
  const double *P; /* [d][N] momenta */
  const double *S; /* [N] actions */
  const double *a; /* [N] complex128 amplitudes (re, im) */
} fggc_packets;

/*
 * Mesh and neighbour strategy of eq. (3.5) and Definition 1 (eq. 2.20).
 *   q-mesh: Nq[k] points over [-pi, pi) (dq = 2 pi / Nq[k]; Nq[k] even and of
 *           the form 2^a 3^b 5^c, 4 <= Nq[k] <= 8192; in two and three
 *           dimensions the power of two in Nq[k] must reach the span of the
 *           q-shifts rounded up to a power of two, e.g. 4 for Q4 sets);
 *           cell anchoring floor(Q / dq) as in (2.20).
 *   p-mesh: step dp[k] > 0, cells floor(P / dp), not wrapped.
 *   Shift set: the tensor product over dimensions of the one-dimensional set
 *           {(dq_off[i], dp_off[j])}, i < nq, j < np (nq * np <= 16), as in the
 *           strategies Q2P2, Q4P2, Q2P4, Q4P4 of Section 3.1.
 *   cutoff: relative eigenvalue cutoff of the pseudo-inverse (remark after
 *           Alg. 1): eigenvalues of the eps-free Gram matrix (3.22) below
 *           cutoff * lambda_max are dropped.  0 = exact least squares.
 */
typedef struct {
  int64_t Nq[3];
  double dp[3];
  int32_t nq, np;
  int32_t dq_off[8];
  int32_t dp_off[8];
  double cutoff;
} fggc_strategy;

/* ------------------------------------------------------------------------ */
/* context                                                                   */
/* ------------------------------------------------------------------------ */

/* Create a context on HIP device `device`.  hbm_budget_bytes caps the
 * workspace the context may hold (0 = 90% of the device's free memory).
 * Errors: FGGC_EINVAL (bad device, out == NULL), FGGC_EDEVICE. */
int fggc_create(fggc_ctx **out, int device, size_t hbm_budget_bytes);

/* Release the context and its workspace (waits for its own stream). */
void fggc_destroy(fggc_ctx *ctx);

/* Message for the last failing call on this thread ("" if none).  The string
 * stays valid until the next call on this thread. */
const char *fggc_last_error(void);

/* Library version string. */
const char *fggc_version(void);

/* ------------------------------------------------------------------------ */
/* reconstruction                                                            */
/* ------------------------------------------------------------------------ */

/*
 * Windowed direct sum, eq. (2.10): every packet is evaluated at every grid
 * point with |x - Q_j| <= window_radius (Euclidean, minimum image,
 * inclusive); 0 < window_radius < pi.
 * FGGC_FP64: all arithmetic in FP64.  FGGC_FP32: the phase argument
 * (S + P.(x-Q))/eps is formed and reduced modulo 2 pi in FP64, the Gaussian,
 * sine, cosine and products in FP32, the grid sums accumulated in FP64 over
 * FP32 partial sums of at most 32 terms.
 * u_out: prod(grid->n) complex values (see conventions).
 * Errors: FGGC_EINVAL (d mismatch, eps <= 0, radius out of range, grid size
 * < 1, NaN or Inf in S or a, |Q| or |P| above 1e9 or not finite -- checked
 * on the device before any output is written; the call synchronises the
 * stream once for this check), FGGC_ENOMEM, FGGC_EBUDGET, FGGC_EDEVICE.
 */
int fggc_direct_sum(fggc_ctx *ctx, const fggc_packets *pk, double eps, const fggc_grid *grid,
                    double window_radius, double scale, int precision, void *u_out, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * windowed direct sum as fggc_direct_sum, with the same kernels and results,
 * that allocates nothing.  Its scratch (pre-pass results, sort keys and
 * positions, packet records, partial grids) lives in one library-owned device
 * array of FGGC_NOALLOC_SCRATCH_BYTES per GPU, set up by fggc_create and held
 * until the process ends; the call makes no hipMalloc, hipFree or other
 * allocating call.
 * Packets and u_out must be device memory of ctx's device (host pointers:
 * FGGC_EINVAL).  A request whose scratch exceeds the limit fails with
 * FGGC_EBUDGET before anything is launched (about 120 bytes per packet plus
 * the partial grids: ~2e6 packets on a 16384-point 1D grid).  Every call on
 * one GPU shares that GPU's array, so calls that overlap in time on one GPU
 * (other host threads, other streams) race: the caller orders them.  The call
 * synchronises `stream` once (the packet check), like fggc_direct_sum.
 * Errors: as fggc_direct_sum, plus FGGC_EBUDGET for the scratch limit.
 */
#define FGGC_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
int fggc_direct_sum_noalloc(fggc_ctx *ctx, const fggc_packets *pk, double eps, const fggc_grid *grid,
                            double window_radius, double scale, int precision, void *u_out, void *stream);

/*
 * The direct sum of fggc_direct_sum at the grid points of a box only:
 * points m with box_lo[k] <= m_k < box_lo[k] + box_n[k] (0 <= box_lo,
 * box_lo + box_n <= grid->n); u_out holds prod(box_n) values, row-major over
 * the box.  Same arguments, precision and errors otherwise.
 */
int fggc_direct_sum_box(fggc_ctx *ctx, const fggc_packets *pk, double eps, const fggc_grid *grid,
                        const int64_t *box_lo, const int64_t *box_n, double window_radius,
                        double scale, int precision, void *u_out, void *stream);

/*
 * The direct sum of eq. (2.10) with a box window, evaluated as a matrix
 * product (d = 2, FP32 only):
 *   u_m = scale * sum_j a_j exp(i (S_j + P_j.y)/eps - |y|^2/(2 eps)) * [|y_0| <= h] [|y_1| <= h],
 *   y = minimum image of x_m - Q_j, h = window_half_width.
 * Under this window every term is a product of a factor of m_0 and a factor
 * of m_1, so a tile of u is a sum over packets of outer products: the call
 * evaluates it on the matrix cores.  The box contains the ball of radius h,
 * so the result differs from fggc_direct_sum's at the same h only by terms
 * smaller than exp(-h^2/(2 eps)) relative (about 1.5e-8 at h = 6 sqrt(eps)).
 * Arguments, layout, ownership and staging as in fggc_direct_sum; u_out holds
 * the whole grid as complex64.  Errors: FGGC_EINVAL as fggc_direct_sum;
 * FGGC_EUNSUPPORTED when d != 2, precision != FGGC_FP32 or an axis exceeds
 * 2^20 points.
 */
int fggc_direct_sum_separable(fggc_ctx *ctx, const fggc_packets *pk, double eps, const fggc_grid *grid,
                              double window_half_width, double scale, int precision, void *u_out,
                              void *stream);

/*
 * Initial decomposition, eq. (2.6)-(2.7): for each of N phase-space points
 * (q_j, p_j),
 *   A_j = 2^{d/2} sum_m u0(x_m) exp(-i p_j.y / eps - |y|^2 / (2 eps)) prod_k (2 pi / n_k),
 * y = minimum image of x_m - q_j, over the grid points with |y| <= window_radius
 * (the quadrature of u0^ on the grid; the Gaussian bounds the dropped tail
 * by exp(-R^2 / (2 eps))).  u0: the grid's values, complex128, row-major;
 * q, p: [d][N] FP64; A_out: [N] complex128, the amplitudes A(0, q, p) that
 * start the flow (fggc_propagate) and, with the weight
 * (dq dp)^d / (2 pi eps)^{3d/2}, reproduce u0 through eq. (2.9).
 * Buffers may be device or host memory.  FP64.  Errors: FGGC_EINVAL for a
 * bad grid, eps <= 0, window_radius outside (0, pi), N < 0 or a NULL array.
 */
int fggc_decompose(fggc_ctx *ctx, const fggc_grid *grid, const double *u0, double eps, double window_radius,
                   int64_t N, const double *q, const double *p, double *A_out, void *stream);

/*
 * The initial decomposition (2.7) on a product mesh whose q-points are grid
 * points, with a box window (every |y_k| <= window_half_width):
 *   q_k = -pi + (q_lo[k] + i) 2 pi / Nq[k], i < q_n[k];  p_k = (p_lo[k] + j) dp[k], j < p_n[k].
 * Because q sits on a grid point, the offsets y = x_m - q are the same for
 * every q, the kernel factors over dimensions, and for each q the values
 * over all p are E_0 W_q E_1^T: products of the window W_q of u0 with two
 * fixed phase matrices, evaluated as batched FP64 complex GEMMs on the matrix
 * cores.  The box contains the ball of fggc_decompose's window, so the two
 * differ only by terms below exp(-R^2/(2 eps)) relative.
 * u0: grid values, complex128, row-major.  A_out: [prod q_n][prod p_n]
 * complex128, q-index major and p-index minor, each row-major over the
 * dimensions (the order of packets listed q-major for fggc_decompose).
 * d = 1 or 2.  Buffers may be device or host memory.  Errors: FGGC_EINVAL
 * when a grid size is not a multiple of Nq, a q range leaves [0, Nq), a p
 * range is empty, dp <= 0, eps <= 0, the window is wider than the grid or
 * outside (0, pi); FGGC_EUNSUPPORTED for d = 3; FGGC_EDEVICE when the GEMM
 * library fails.
 */
int fggc_decompose_mesh(fggc_ctx *ctx, const fggc_grid *grid, const double *u0, double eps,
                        double window_half_width, const int64_t *Nq, const int64_t *q_lo, const int64_t *q_n,
                        const double *dp, const int64_t *p_lo, const int64_t *p_n, double *A_out, void *stream);

/*
 * The seeded synthetic workloads (configurations 0-3):
 *   0: 1D, eps = 1/64, N = 256 x 256 (q, p), grid 1024;
 *   1: 1D, eps = 1/1024, N = 1024 x 1024, grid 16384;
 *   2: 2D, eps = 1/256, N = 64^2 q x 32^2 p, grid 1024^2;
 *   3: 3D, eps = 1/128, N = 32^3 q x 8^3 p, grid 256^3.
 * Packets start on a (q, p) mesh (q uniform over [-pi, pi)^d; p random in
 * 1D, an endpoint-inclusive mesh in 2D/3D), are carried by free flow
 * (eq. 2.3-2.4 with V = 0) to t = 0.5, and carry a uniform random action and
 * a Gaussian-in-q amplitude with a uniform random phase; random numbers are
 * SplitMix64 counter streams (the package's Python generator draws the same
 * values).  The window radius of the direct sum is 6 sqrt(eps).
 * fggc_config_info returns the sizes (any output pointer may be NULL).
 * fggc_gen_config fills caller-allocated host arrays out->Q, out->P
 * ([d][N]), out->S ([N]) and out->a ([N] complex128), written through the
 * pointers of `out`; out->d and out->N must equal the configuration's.
 * seed = 0 selects the default seed of the configuration.  Host only, no
 * GPU call.  Errors: FGGC_EINVAL for an unknown config_id or a mismatching out.
 */
int fggc_config_info(int config_id, int32_t *d, int64_t *N, double *eps, fggc_grid *grid, double *window_radius);
int fggc_gen_config(int config_id, uint64_t seed, fggc_packets *out);

/*
 * Potential of the packet flow:
 *   V(x) = c0 + sum_k w[k] x_k^2 / 2 + c1 sum_k cos(kappa x_k) + c2 exp(c3 |x|^2).
 * The paper's examples (Sec. 4) are members: 1 - cos(pi x) (c0 = 1, c1 = -1,
 * kappa = pi), |x|^2 / 2 (w = 1) and 1 - exp(-|x|^2) (c0 = 1, c2 = -1, c3 = -1).
 */
typedef struct {
  double c0;
  double w[3];
  double c1, kappa;
  double c2, c3;
} fggc_potential;

/*
 * Propagate N packets along the Hamiltonian flow of eq. (2.3)-(2.6) for
 * nsteps steps of the classical fourth-order Runge-Kutta scheme with step dt
 * (the paper's time integrator, Sec. 4), in FP64, one thread per packet.
 *   Q, P: [d][N] in/out; S: [N] in/out; a: [N] complex128 in/out (the
 *   amplitude A of (2.6)).  Q is not wrapped into [-pi, pi): the flow is on
 *   R^d, and the reconstruction calls take Q modulo 2 pi.
 *   jac: NULL, or [N][2][d][d] complex128 in/out holding dz Q then dz P
 *   (dz = d_q - i d_p, row-major), the Jacobians whose combination
 *   Z = dz Q + i dz P enters (2.6).  With NULL every packet starts from
 *   dz Q = I, dz P = -i I, i.e. from its initial point (q, p) of (2.3)-(2.4),
 *   and the Jacobians are not returned; pass jac to continue a flow across
 *   several calls.
 * Buffers may be device or host memory (host buffers are staged and the call
 * completes before it returns).  Errors: FGGC_EINVAL for d outside 1..3,
 * N < 0, nsteps < 0, a NULL array with N > 0, a non-finite dt or potential
 * coefficient.
 */
int fggc_propagate(fggc_ctx *ctx, int32_t d, int64_t N, double *Q, double *P, double *S, double *a,
                   double *jac, const fggc_potential *V, double dt, int64_t nsteps, void *stream);

/*
 * The least-squares coefficients of the FGGC correction, per packet, as the
 * reconstruction's coefficient kernel computes them (Sec. 2.2-2.3: the
 * int/frac split (3.6)-(3.7), right-hand side (3.23), the solve against the
 * Gram matrix (3.22) through its eigenpairs, conjugation, shift (3.13),
 * Kronecker product over dimensions), in FP64:
 *   c_out[j][K] = scale * a_j exp(i S_j / eps) c_K(Q_j, P_j), K = (k_0, .., k_{d-1})
 *   row-major, each k over the strategy's nq * np one-dimensional basis in
 *   the order q-shift major, p-shift minor ([N][(nq np)^d] complex128);
 *   cell_out[j][0][k] = the packet's q-cell index (floor(Q/dq) + Nq/2) mod Nq
 *   and cell_out[j][1][k] = its p-cell floor(P/dp), per dimension ([N][2][d]).
 * With a = 1 and S = 0 these are the c^(k) of the paper's least-squares
 * approximation of G(x; Q, P) by its neighbouring on-grid packets (the
 * coefficient maps of Sec. 2.2 and the E_LSA of Sec. 3.1 follow from them).
 * Packets and outputs are device memory; the call synchronises `stream`
 * once (the packet check).  Errors: FGGC_EINVAL as fggc_reconstruct;
 * FGGC_EUNSUPPORTED for 3D shift sets above 8.
 */
int fggc_coefficients(fggc_ctx *ctx, const fggc_packets *pk, double eps, const fggc_strategy *st, double scale,
                      double *c_out, int32_t *cell_out, void *stream);

/*
 * Multi-step FGGC (Sec. 3.2, Alg. 3): the bookkeeping of the learned map on
 * the device.  A fixed mesh of Nm phase-space points (q, p) is decomposed at
 * the start of every run (fggc_decompose / fggc_decompose_mesh give A0);
 * points with |A0| <= prune * max |A0| are skipped in that run, and of the
 * others only those no earlier run has evolved are propagated.  The flow is
 * linear in A, so a point learns its final (Q, P, S) and the ratio
 * A(T) / A(0) (evolved from A(0) = 1); later runs reconstruct from those with
 * their own A0.  All buffers are device memory on ctx's device, stream-ordered
 * on `stream`; complex arrays are interleaved complex128.
 *
 * fggc_learn_select: keep_idx[0 .. *n_keep) = the points with
 * |A0| > prune * max |A0|, and new_idx[0 .. *n_new) = those of them whose
 * learned[i] is 0, both in mesh order; learned[i] is set to 1 for the new
 * ones.  keep_idx and new_idx hold Nm entries each; the call synchronises
 * `stream` once to return the two counts.  Errors: FGGC_EINVAL (Nm < 0, NULL
 * arrays, prune not in [0, 1)).
 */
int fggc_learn_select(fggc_ctx *ctx, int64_t Nm, const double *A0, double prune, uint8_t *learned,
                      int64_t *keep_idx, int64_t *new_idx, int64_t *n_keep, int64_t *n_new, void *stream);

/*
 * fggc_learn_start: the n packets at mesh points idx[0 .. n) to be evolved:
 * Q[k][j] = qm[k][idx[j]], P[k][j] = pm[k][idx[j]], S[j] = 0, A[j] = 1
 * (qm, pm: [d][Nm]; Q, P: [d][n]; S: [n]; A: [n] complex).
 * fggc_learn_store: the evolved packets back into the per-point tables
 * Qf, Pf ([d][Nm]), Sf ([Nm]) and ratio ([Nm] complex) at idx.
 * fggc_learn_packets: the reconstruction's packets of the kept points idx:
 * (Q, P, S) = the learned (Qf, Pf, Sf) and a[j] = A0[idx[j]] * ratio[idx[j]].
 * Errors: FGGC_EINVAL (d outside 1..3, n < 0, n > Nm, NULL arrays with n > 0).
 */
int fggc_learn_start(fggc_ctx *ctx, int32_t d, int64_t Nm, int64_t n, const int64_t *idx, const double *qm,
                     const double *pm, double *Q, double *P, double *S, double *A, void *stream);
int fggc_learn_store(fggc_ctx *ctx, int32_t d, int64_t Nm, int64_t n, const int64_t *idx, const double *Q,
                     const double *P, const double *S, const double *A, double *Qf, double *Pf, double *Sf,
                     double *ratio, void *stream);
int fggc_learn_packets(fggc_ctx *ctx, int32_t d, int64_t Nm, int64_t n, const int64_t *idx, const double *Qf,
                       const double *Pf, const double *Sf, const double *ratio, const double *A0, double *Q,
                       double *P, double *S, double *a, void *stream);

/*
 * FGGC reconstruction (Alg. 2 steps 3-4 with eq. 2.23-2.25):
 *   per packet and dimension, int/frac split (3.6)-(3.7), right-hand side
 *   (3.23), least squares against the precomputed Gram matrix (3.22) through
 *   its eigenpairs, conjugation of the printed system's solution to the
 *   L2-best coefficients, coefficient shift (3.13) with the sign that goes
 *   with it, Kronecker product over dimensions; scatter-add of
 *   scale * a_j exp(i S_j / eps) c_j^(k) into the dense cell array over the
 *   occupied p-cell box (2.25); then eq. (2.24) by a forward FFT over q per
 *   p-slice, a Gaussian band multiply-accumulate into the grid spectrum
 *   (the Fourier transform of (2.16) with the on-grid centre and momentum),
 *   and one inverse FFT of size prod(grid->n).
 * grid->n[k] must be of the form 2^a 3^b 5^c (2 .. 16384 for 1D FP32, 8192
 * for FP64, 4096 for d >= 2).  Nq as in fggc_strategy.
 * FGGC_FP64: FP64 throughout.  FGGC_FP32: least squares, phase reductions
 * and band weights in FP64; cells, FFTs and products in FP32; the band folds
 * sum one term per slice and alias, in FP64 in one dimension and in the
 * general separable pass, in FP32 in the register-FFT passes and the fused
 * three-dimensional finish.
 * Errors: as fggc_direct_sum, plus FGGC_EUNSUPPORTED for sizes outside the
 * ranges above and FGGC_EBUDGET when the cell array cannot fit.
 */
int fggc_reconstruct(fggc_ctx *ctx, const fggc_packets *pk, double eps, const fggc_grid *grid,
                     const fggc_strategy *st, double scale, int precision, void *u_out,
                     void *stream);

/*
 * Fill *out with a named strategy at the mesh of eq. (3.5) recommended after
 * the Section 3.1 tables: dq ~ sqrt(eps)/2 with Nq the power of two nearest
 * 2 pi / (sqrt(eps)/2), dp = pi sqrt(eps)/8.  name: "Q2P2"
 * (dq {0,1} x dp {0,1}), "Q4P2" (dq {-1,0,1,2} x dp {0,1}), "Q2P4"
 * (dq {0,1} x dp {-1,0,1,2}) or "Q4P4".  cutoff = 0.  Host only.
 * Errors: FGGC_EINVAL.
 */
int fggc_default_strategy(int d, double eps, const char *name, fggc_strategy *out);

/* ------------------------------------------------------------------------ */
/* stages of the FGGC path (exposed for inspection and testing)              */
/* ------------------------------------------------------------------------ */

/*
 * The occupied p-cell box of a packet set under strategy `st`: slice_lo[k]
 * and slice_n[k] such that every p-cell floor(P/dp) + dp_off lies in
 * [slice_lo, slice_lo + slice_n).  Synchronises the stream.
 */
int fggc_cell_box(fggc_ctx *ctx, const fggc_packets *pk, const fggc_strategy *st,
                  int64_t *slice_lo, int64_t *slice_n, void *stream);

/*
 * The dense cell array A~(q_i, p_l) of eq. (2.25), times scale, over the box
 * returned by fggc_cell_box: layout [slice][q] with slice row-major over the
 * box and q row-major over Nq (q_i = -pi + i dq); complex64 (FGGC_FP32) or
 * complex128 (FGGC_FP64).  cells_bytes must be at least the array's size.
 * Errors: FGGC_EINVAL when the box does not match the packets.
 */
int fggc_cells(fggc_ctx *ctx, const fggc_packets *pk, double eps, const fggc_strategy *st,
               double scale, int precision, const int64_t *slice_lo, const int64_t *slice_n,
               void *cells_out, size_t cells_bytes, void *stream);

/*
 * In-place batched d-dimensional complex DFT on device memory:
 *   forward (direction = -1): X[k] = sum_n x[n] exp(-2 pi i k.n / n)
 *   inverse (direction = +1): X[k] = sum_n x[n] exp(+2 pi i k.n / n), unnormalised.
 * data: batch consecutive arrays of prod(n[0..d-1]) complex values
 * (complex64 for FGGC_FP32, complex128 for FGGC_FP64), row-major.
 * Sizes: 2^a 3^b 5^c, 2 .. 16384 (FP32) or 8192 (FP64) per dimension; in two
 * and three dimensions at most 4096 unless a power of two.  Lengths with
 * factors 3 or 5 take mixed-radix passes (radix 4, 2, 3 and 5); one
 * dimension above 4096 points takes the four-step form n = n1 n2.
 * Errors: FGGC_EUNSUPPORTED for other sizes.
 */
int fggc_fft(fggc_ctx *ctx, int d, const int64_t *n, int64_t batch, int direction, int precision,
             void *data, void *stream);

/*
 * Eigen-decomposition used by the plan: Gram matrix (3.22) of the
 * one-dimensional shift set for C_q = dq/sqrt(eps), C_p = dp/sqrt(eps),
 * n1 = nq * np (basis index i * np + j).  evals[n1] ascending; evecs
 * [n1][n1] complex128, column k the unit eigenvector of evals[k].  Host only.
 */
int fggc_plan_gram(int nq, const int32_t *dq_off, int np, const int32_t *dp_off, double Cq,
                   double Cp, double *evals, double *evecs);

/*
 * Per-stage timing for benchmarks.  With enable = 1 every later call on the
 * context records HIP events around each of its stages (on the stream the
 * stage runs on); enable = 0 stops recording.  Either resets the totals.
 * Stages: "prepass", "ds_prep", "ds_sort", "ds_kernel",
 * "ds_reduce", "fggc_sort", "fggc_coef", "fggc_accum", "fggc_fft_q",
 * "fggc_band_table", "fggc_band_mac", "fggc_ifft", "fft".
 */
int fggc_profile(fggc_ctx *ctx, int enable);

/* Total milliseconds and number of launches recorded for one stage since the
 * last fggc_profile call (waits for the recorded events). */
int fggc_stage_time(fggc_ctx *ctx, const char *stage, double *total_ms, int64_t *count);

/* ------------------------------------------------------------------------ */
/* serving                                                                   */
/* ------------------------------------------------------------------------ */

typedef struct fggc_server fggc_server;
typedef int64_t fggc_ticket;

/*
 * A persistent scheduler on the context's device (the serving mode of the
 * reconstruction step; the paper states the single reconstruction, eq. 2.10
 * and eq. 2.19, and this wraps it for a stream of independent requests).
 * `n_streams` (1..8) executor slots each own a worker thread, a non-blocking
 * stream and a workspace.  Queued requests are admitted in arrival order as
 * soon as a slot is idle and the request's memory estimate fits the
 * context's HBM budget (idle slots release memory when that makes it fit);
 * admitted requests overlap on the device.  A slot runs a request's kernel
 * pipeline eagerly the first time its shape is seen, captures it into a
 * hipGraph the second time and replays that graph afterwards (up to 128
 * graphs per slot, least recently used dropped).  Shapes repeat because the
 * packet count is padded to a quarter-octave bucket (m 2^e, m in 4..8, at
 * least 64) with zero-amplitude copies of packets 0, 1, 2, ..., which add
 * exactly nothing, and the p-cell box is widened to even cell indices.  The budget
 * covers the slots' workspaces; synchronous calls on the same context
 * during serving allocate outside it.
 * Errors: FGGC_EINVAL (NULL out or ctx, n_streams out of range),
 * FGGC_EDEVICE.
 */
int fggc_server_create(fggc_ctx *ctx, int n_streams, fggc_server **out);

/*
 * Enqueue a reconstruction and return its ticket.  st == NULL selects the
 * direct sum with window radius 6 sqrt(eps); otherwise FGGC with *st.
 * Packet arrays must be all host or all device memory.  Host packets are
 * copied (and checked) before submit returns, so the caller may free them;
 * device packets are checked by a small kernel at submit and read in place,
 * so they must stay valid and unchanged until the ticket is waited for.
 * u_out (host or device, prod(grid->n) complex values, complex64 for FP32,
 * complex128 for FP64, row-major) is written before the ticket completes.
 * The request's memory estimate is fixed here; a request whose estimate
 * exceeds the budget fails at once with FGGC_EBUDGET and blocks nobody.
 * N == 0 completes at once with u = 0.
 * Errors: FGGC_EINVAL (bad arguments or packets, as for the synchronous
 * calls; N > 2^30), FGGC_EUNSUPPORTED (grid sizes FGGC does not handle),
 * FGGC_EBUDGET, FGGC_ECANCELLED (server shutting down), FGGC_EDEVICE.
 */
int fggc_server_submit(fggc_server *srv, const fggc_packets *pk, double eps, const fggc_grid *grid,
                       const fggc_strategy *st, double scale, int precision, void *u_out,
                       fggc_ticket *ticket);

/* Wait for a ticket; returns its final status (and forgets the ticket), or
 * FGGC_ETIMEOUT if timeout_s (< 0: forever) elapsed first (the ticket stays
 * valid).  FGGC_EINVAL for an unknown or already-waited ticket. */
int fggc_server_wait(fggc_server *srv, fggc_ticket ticket, double timeout_s);

/* Latency percentiles (submit to completion, seconds) and throughput
 * (packets per second of wall time since the first submit) of the
 * completed requests. */
int fggc_server_stats(fggc_server *srv, double *p50_s, double *p99_s, double *packets_per_s,
                      int64_t *completed);

/* How the completed requests ran: eagerly (first sighting of a shape, or
 * a shape that could not be captured), by capturing a new graph, or by
 * replaying a cached one. */
int fggc_server_counters(fggc_server *srv, int64_t *eager, int64_t *captured, int64_t *replayed);

/* Clear the latency, throughput and graph counters (e.g. after a warm-up). */
int fggc_server_reset_stats(fggc_server *srv);

/* Stop the scheduler after the queued requests have finished; free it. */
void fggc_server_destroy(fggc_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* FGGC_H */
