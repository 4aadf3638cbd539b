// Host-side plan of the FGGC correction: strategies, the eps-free Gram
// matrix of eq. (3.22) per dimension and its eigen-decomposition (Alg. 2,
// step 0: the pseudo-inverse is precomputed once per mesh and neighbour
// strategy, here as eigenpairs so that it is applied as V diag(1/lambda) V^H
// and never formed as an explicit matrix).
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <memory>
#include <string>

#include "common.h"

namespace fggc {

namespace {
using cld = std::complex<long double>;

// Cyclic complex Jacobi for a Hermitian n x n matrix in long double.  Each
// rotation first turns the (p,q) entry real with a diagonal phase, then
// applies a real plane rotation that zeroes it.
void jacobi_hermitian(int n, std::vector<cld> &A, std::vector<cld> &V) {
  V.assign((size_t)n * n, cld(0));
  for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1;
  for (int sweep = 0; sweep < 60; ++sweep) {
    long double off = 0, tot = 0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        long double m = std::norm(A[(size_t)i * n + j]);
        tot += m;
        if (i != j) off += m;
      }
    if (off <= 1e-36L * tot) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        cld h = A[(size_t)p * n + q];
        long double r = std::abs(h);
        if (r == 0) continue;
        cld e = h / r;  // e^{i phi}
        long double a = A[(size_t)p * n + p].real(), b = A[(size_t)q * n + q].real();
        long double zeta = (b - a) / (2 * r);
        long double t = (zeta >= 0 ? 1 : -1) / (std::fabs(zeta) + std::sqrt(1 + zeta * zeta));
        long double c = 1 / std::sqrt(1 + t * t), s = t * c;
        // G = diag(1, conj(e)) * [[c, s], [-s, c]]  on columns (p, q)
        cld g00 = c, g01 = s, g10 = -s * std::conj(e), g11 = c * std::conj(e);
        for (int k = 0; k < n; ++k) {  // A <- A G
          cld akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
          A[(size_t)k * n + p] = akp * g00 + akq * g10;
          A[(size_t)k * n + q] = akp * g01 + akq * g11;
        }
        for (int k = 0; k < n; ++k) {  // A <- G^H A
          cld apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
          A[(size_t)p * n + k] = std::conj(g00) * apk + std::conj(g10) * aqk;
          A[(size_t)q * n + k] = std::conj(g01) * apk + std::conj(g11) * aqk;
        }
        for (int k = 0; k < n; ++k) {  // V <- V G
          cld vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
          V[(size_t)k * n + p] = vkp * g00 + vkq * g10;
          V[(size_t)k * n + q] = vkp * g01 + vkq * g11;
        }
      }
  }
}

// eq. (3.22) for one dimension: exp(-Cq^2 (dq_j-dq_k)^2/4 - Cp^2 (dp_j-dp_k)^2/4
//                                   + i Cq Cp (dq_k-dq_j)(dp_j+dp_k)/2)
cld gram_1d(int dqj, int dpj, int dqk, int dpk, long double Cq, long double Cp) {
  long double a = dqj - dqk, b = dpj - dpk;
  long double re = -Cq * Cq * a * a / 4 - Cp * Cp * b * b / 4;
  long double im = Cq * Cp * (long double)(dqk - dqj) * (long double)(dpj + dpk) / 2;
  return std::exp(re) * cld(std::cos(im), std::sin(im));
}

void eig_sorted(int n, std::vector<cld> &A, long double *evals, std::vector<cld> &V) {
  jacobi_hermitian(n, A, V);
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j)
      if (A[(size_t)order[j] * n + order[j]].real() < A[(size_t)order[i] * n + order[i]].real())
        std::swap(order[i], order[j]);
  std::vector<cld> Vs((size_t)n * n);
  for (int k = 0; k < n; ++k) {
    evals[k] = A[(size_t)order[k] * n + order[k]].real();
    for (int i = 0; i < n; ++i) Vs[(size_t)i * n + k] = V[(size_t)i * n + order[k]];
  }
  V.swap(Vs);
}
}  // namespace

void hermitian_eig(int n, const double *A, double *evals, double *evecs) {
  std::vector<cld> M((size_t)n * n), V;
  for (int i = 0; i < n * n; ++i) M[i] = cld(A[2 * i], A[2 * i + 1]);
  std::vector<long double> w(n);
  eig_sorted(n, M, w.data(), V);
  for (int k = 0; k < n; ++k) evals[k] = (double)w[k];
  for (int i = 0; i < n * n; ++i) {
    evecs[2 * i] = (double)V[i].real();
    evecs[2 * i + 1] = (double)V[i].imag();
  }
}

void build_dim_lsq(const fggc_strategy &st, int dim, double eps, DimLsq *out) {
  const int n1 = st.nq * st.np;
  out->n1 = n1;
  for (int a = 0; a < st.nq; ++a)
    for (int b = 0; b < st.np; ++b) {
      out->dq[a * st.np + b] = st.dq_off[a];
      out->dp[a * st.np + b] = st.dp_off[b];
    }
  const long double se = std::sqrt((long double)eps);
  const long double Cq = ((long double)2 * 3.14159265358979323846264338327950288L / st.Nq[dim]) / se;
  const long double Cp = (long double)st.dp[dim] / se;
  out->Cq = (double)Cq;
  out->Cp = (double)Cp;
  std::vector<cld> A((size_t)n1 * n1), V;
  for (int j = 0; j < n1; ++j)
    for (int k = 0; k < n1; ++k)
      A[(size_t)j * n1 + k] = gram_1d(out->dq[j], out->dp[j], out->dq[k], out->dp[k], Cq, Cp);
  long double w[kMaxN1];
  eig_sorted(n1, A, w, V);
  long double wmax = 0;
  for (int k = 0; k < n1; ++k) wmax = std::max(wmax, w[k]);
  // exact least squares drops only eigenvalues that are zero to working precision
  long double cut = st.cutoff > 0 ? (long double)st.cutoff * wmax : 1e-18L * wmax;
  for (int k = 0; k < n1; ++k) out->inv[k] = w[k] > cut ? (double)(1 / w[k]) : 0.0;
  for (int i = 0; i < n1; ++i)
    for (int k = 0; k < n1; ++k) {
      out->V[2 * (i * n1 + k)] = (double)V[(size_t)i * n1 + k].real();
      out->V[2 * (i * n1 + k) + 1] = (double)V[(size_t)i * n1 + k].imag();
    }
  out->dq0 = *std::min_element(st.dq_off, st.dq_off + st.nq);
  out->dp0 = *std::min_element(st.dp_off, st.dp_off + st.np);
  for (int k = 0; k < n1; ++k) {
    const long double ph = -Cq * Cp * (long double)out->dq[k] * (long double)out->dp[k] / 2;
    out->D[2 * k] = (double)std::cos(ph);
    out->D[2 * k + 1] = (double)std::sin(ph);
    const long double eq = out->dq[k] - out->dq0, ep = out->dp[k] - out->dp0;
    const long double g = std::exp(-(Cq * Cq * eq * eq + Cp * Cp * ep * ep) / 4);
    out->DK[2 * k] = (double)(g * std::cos(ph));
    out->DK[2 * k + 1] = (double)(g * std::sin(ph));
    const cld dk = g * cld(std::cos(ph), std::sin(ph));
    for (int i = 0; i < n1; ++i) {
      const long double iv = w[i] > cut ? 1 / w[i] : 0.0L;
      const cld x = iv * std::conj(V[(size_t)k * n1 + i]) * dk;
      out->W[2 * (k * n1 + i)] = (double)x.real();
      out->W[2 * (k * n1 + i) + 1] = (double)x.imag();
    }
  }
}

namespace {
struct PlanEntry {
  int device, d;
  double eps;
  fggc_strategy st;
  Plan plan;
};
std::mutex g_plan_mu;
std::vector<std::unique_ptr<PlanEntry>> g_plans;
constexpr size_t kMaxPlans = 1024;

bool same_strategy(const fggc_strategy &a, const fggc_strategy &b, int d) {
  if (a.nq != b.nq || a.np != b.np || a.cutoff != b.cutoff) return false;
  for (int k = 0; k < d; ++k)
    if (a.Nq[k] != b.Nq[k] || a.dp[k] != b.dp[k]) return false;
  for (int i = 0; i < a.nq; ++i)
    if (a.dq_off[i] != b.dq_off[i]) return false;
  for (int i = 0; i < a.np; ++i)
    if (a.dp_off[i] != b.dp_off[i]) return false;
  return true;
}
}  // namespace

Plan plan_for(const fggc_strategy &st, int d, double eps) {
  int dev = 0;
  FGGC_HIP(hipGetDevice(&dev));
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (auto &e : g_plans)
      if (e->device == dev && e->d == d && e->eps == eps && same_strategy(e->st, st, d)) return e->plan;
  }
  Plan pl{};
  for (int k = 0; k < d; ++k) build_dim_lsq(st, k, eps, &pl.host[k]);
  std::lock_guard<std::mutex> lk(g_plan_mu);
  if (g_plans.size() >= kMaxPlans) return pl;  // callers copy the host plan themselves
  DimLsq *dv = nullptr;
  FGGC_HIP(hipMalloc((void **)&dv, 3 * sizeof(DimLsq)));
  FGGC_HIP(hipMemcpy(dv, pl.host, 3 * sizeof(DimLsq), hipMemcpyHostToDevice));
  pl.dev = dv;  // kept for the life of the process (graphs may refer to it)
  auto e = std::make_unique<PlanEntry>();
  e->device = dev;
  e->d = d;
  e->eps = eps;
  e->st = st;
  e->plan = pl;
  g_plans.push_back(std::move(e));
  return pl;
}

}  // namespace fggc

extern "C" int fggc_plan_gram(int nq, const int32_t *dq_off, int np, const int32_t *dp_off,
                              double Cq, double Cp, double *evals, double *evecs) {
  try {
    if (nq < 1 || np < 1 || nq * np > fggc::kMaxN1 || !dq_off || !dp_off || !evals || !evecs ||
        !(Cq > 0) || !(Cp > 0)) {
      fggc::set_last_error("fggc_plan_gram: invalid argument");
      return FGGC_EINVAL;
    }
    const int n1 = nq * np;
    int sq[fggc::kMaxN1], sp[fggc::kMaxN1];
    for (int a = 0; a < nq; ++a)
      for (int b = 0; b < np; ++b) {
        sq[a * np + b] = dq_off[a];
        sp[a * np + b] = dp_off[b];
      }
    std::vector<double> Ar(2 * (size_t)n1 * n1);
    for (int j = 0; j < n1; ++j)
      for (int k = 0; k < n1; ++k) {
        auto v = fggc::gram_1d(sq[j], sp[j], sq[k], sp[k], Cq, Cp);
        Ar[2 * (j * n1 + k)] = (double)v.real();
        Ar[2 * (j * n1 + k) + 1] = (double)v.imag();
      }
    fggc::hermitian_eig(n1, Ar.data(), evals, evecs);
    return FGGC_OK;
  } catch (const fggc::Error &e) {
    fggc::set_last_error(e.msg);
    return e.code;
  } catch (...) {
    fggc::set_last_error("fggc_plan_gram: internal error");
    return FGGC_EDEVICE;
  }
}

extern "C" int fggc_default_strategy(int d, double eps, const char *name, fggc_strategy *out) {
  if (d < 1 || d > 3 || !(eps > 0) || !std::isfinite(eps) || !name || !out) {
    fggc::set_last_error("fggc_default_strategy: invalid argument");
    return FGGC_EINVAL;
  }
  std::string nm(name);
  static const int32_t q2[2] = {0, 1}, q4[4] = {-1, 0, 1, 2};
  int nq, np;
  const int32_t *sq, *sp;
  if (nm == "Q2P2") { nq = 2; sq = q2; np = 2; sp = q2; }
  else if (nm == "Q4P2") { nq = 4; sq = q4; np = 2; sp = q2; }
  else if (nm == "Q2P4") { nq = 2; sq = q2; np = 4; sp = q4; }
  else if (nm == "Q4P4") { nq = 4; sq = q4; np = 4; sp = q4; }
  else {
    fggc::set_last_error("fggc_default_strategy: unknown strategy name " + nm);
    return FGGC_EINVAL;
  }
  std::memset(out, 0, sizeof(*out));
  // dq ~ sqrt(eps)/2 with Nq the power of two nearest (in ratio) 2 pi / (sqrt(eps)/2)
  double target = 4.0 * fggc::kPi / std::sqrt(eps);
  int e2 = (int)std::lround(std::log2(target));
  if (e2 < 2) e2 = 2;
  if (e2 > 13) e2 = 13;
  for (int k = 0; k < 3; ++k) {
    out->Nq[k] = k < d ? (int64_t)1 << e2 : 1;
    out->dp[k] = k < d ? fggc::kPi * std::sqrt(eps) / 8.0 : 1.0;
  }
  out->nq = nq;
  out->np = np;
  for (int i = 0; i < nq; ++i) out->dq_off[i] = sq[i];
  for (int i = 0; i < np; ++i) out->dp_off[i] = sp[i];
  out->cutoff = 0.0;
  return FGGC_OK;
}
