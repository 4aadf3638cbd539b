// Internal declarations shared by the libfggc sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <exception>
#include <list>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fggc.h"

namespace fggc {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;

// Internal failure, converted to an fggc_status at the ABI boundary.
struct Error {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const std::string &msg);
void set_last_error(const std::string &msg);

#define FGGC_HIP(x)                                                                      \
  do {                                                                                   \
    hipError_t e_ = (x);                                                                 \
    if (e_ != hipSuccess)                                                                \
      ::fggc::fail(FGGC_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_));        \
  } while (0)

// Bump allocator over one growable device buffer.  Growing synchronises the
// device (old contents are not kept); a call reserves everything it needs up
// front, then carves.
class Workspace {
 public:
  Workspace() = default;
  // a view of memory owned elsewhere (never grown or freed)
  Workspace(void *base, size_t cap) : base_((char *)base), cap_(cap), owned_(false) {}
  Workspace(const Workspace &) = delete;
  Workspace &operator=(const Workspace &) = delete;
  ~Workspace();
  void reserve(size_t bytes, size_t budget);  // ensure capacity (may reallocate)
  void reset() { used_ = 0; }
  void release();                             // free the memory (capacity 0)
  size_t mark() const { return used_; }       // current take position
  void rewind(size_t m) { used_ = m; }        // drop takes made after mark()
  // stream whose completion is awaited before a reallocation (default: the device)
  void set_stream(hipStream_t s) { stream_ = s; has_stream_ = true; }
  void *take(size_t bytes);                   // 256-byte aligned slice
  size_t capacity() const { return cap_; }
  const void *base() const { return base_; }

 private:
  char *base_ = nullptr;
  size_t cap_ = 0, used_ = 0;
  hipStream_t stream_ = nullptr;
  bool has_stream_ = false;
  bool owned_ = true;
};

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Optional per-stage timing: HIP events recorded around each stage on the
// stream it is launched on, read back when queried.
class Profiler {
 public:
  ~Profiler();
  void start(const char *stage, hipStream_t s);  // record a start event
  void stop(const char *stage, hipStream_t s);   // record the matching end event
  // accumulated milliseconds and launch count of one stage (synchronises its events)
  void query(const std::string &stage, double *ms, int64_t *count);
  void reset();
  std::vector<std::string> stages();

 private:
  struct Pending {
    std::string stage;
    hipEvent_t a, b;
  };
  struct Acc {
    double ms = 0;
    int64_t count = 0;
  };
  void drain();
  std::mutex mu_;
  std::vector<Pending> pending_;
  std::vector<std::pair<std::string, Acc>> acc_;
  std::vector<std::pair<std::string, hipEvent_t>> open_;
};

// RAII stage scope: no-op when prof is null.
struct StageScope {
  Profiler *p;
  const char *name;
  hipStream_t s;
  StageScope(Profiler *p_, const char *n, hipStream_t s_) : p(p_), name(n), s(s_) {
    if (p) p->start(name, s);
  }
  ~StageScope() {
    if (p) p->stop(name, s);
  }
};

// --------------------------------------------------------------------------
// plan (host): per-dimension least-squares data of the FGGC correction
// --------------------------------------------------------------------------

constexpr int kMaxN1 = 16;  // largest one-dimensional basis (nq * np)

// Eigenpairs of the eps-free Gram matrix (3.22) of one dimension, with the
// reciprocal eigenvalues already cut: A~^+ = V diag(inv) V^H.
// Column of counting chunk g in the bin-major count table [bin][column]:
// workgroups are dealt to the eight XCDs in turn, so mapping the chunks of one
// XCD to adjacent columns keeps each cache line of the table written from one
// L2.  Any bijection is correct: it only orders the chunks inside a bin.
__host__ __device__ inline int64_t chunk_column(int64_t g, int G) {
  return (G & 7) ? g : (g & 7) * (G >> 3) + (g >> 3);
}

struct alignas(16) DimLsq {
  int n1;
  int dq0, dp0;  // smallest q and p shifts
  int dq[kMaxN1], dp[kMaxN1];
  double Cq, Cp;
  double inv[kMaxN1];    // 1/lambda or 0 when cut
  double D[2 * kMaxN1];  // exp(-i Cq Cp dq_k dp_k / 2), the constant phase of (3.23)
  // D_k exp(-(Cq^2 (dq_k - dq0)^2 + Cp^2 (dp_k - dp0)^2) / 4): the constant
  // part of the right-hand side once the Gaussian factor is split about the
  // smallest shifts
  double DK[2 * kMaxN1];
  double V[2 * kMaxN1 * kMaxN1];  // [row][col] complex, columns are eigenvectors
  // W[j][i] = inv_i conj(V[j][i]) DK_j: the first product of the solve with
  // the right-hand side's constant factor and 1/lambda folded in, so that
  // z = diag(inv) V^H (DK .* h) is one product W^T h per packet.  The second
  // product V z stays separate (the pseudo-inverse is never formed).
  double W[2 * kMaxN1 * kMaxN1];
};
static_assert(offsetof(DimLsq, V) % 16 == 0 && offsetof(DimLsq, W) % 16 == 0,
              "the plan is staged in 16-byte units");

// Hermitian eigen-decomposition of a complex n x n matrix (cyclic Jacobi on
// the real symmetric 2n x 2n embedding, FP64).  evals ascending, evecs
// [n][n] complex columns.
void hermitian_eig(int n, const double *A, double *evals, double *evecs);
void build_dim_lsq(const fggc_strategy &st, int dim, double eps, DimLsq *out);

// The plan of a (strategy, d, eps) on the current device: host copy and a
// device copy uploaded once and kept for the life of the process (dev is null
// when the cache is full; the caller then copies `host` itself).
struct Plan {
  DimLsq host[3];
  const DimLsq *dev = nullptr;
};
Plan plan_for(const fggc_strategy &st, int d, double eps);

// --------------------------------------------------------------------------
// device-side parameter blocks (passed by value to kernels)
// --------------------------------------------------------------------------

static_assert(sizeof(DimLsq) % 16 == 0, "DimLsq is copied in 16-byte units");

// Packet record for the direct sum, one per packet, sorted by spatial bin.
struct alignas(16) DsRec {
  int32_t mq[3];    // nearest grid index per dimension
  float la2;        // log2 |scale a| (FP32 path)
  double delta[3];  // Q - x_mq (minimum image), |delta| <= dx/2
  double phi0;      // phase at x_mq in revolutions, frac((S - P.delta)/(2 pi eps) + arg(scale a)/(2 pi))
  double omega[3];  // phase step per grid point in revolutions, frac(P_d / (eps n_d))
  double lnamp;     // log |scale a|
  float deltaf[3];  // delta rounded to FP32 (FP32 path)
  int32_t pad;
};
static_assert(sizeof(DsRec) == 96, "DsRec layout");

struct GridGeom {
  int d;
  int64_t n[3];
  double dx[3];
};

struct Box {
  int64_t lo[3], n[3];
};

// --------------------------------------------------------------------------
// launchers (defined in the .hip files)
// --------------------------------------------------------------------------

// Pre-pass over the packets: out[0] = number of packets with NaN/Inf or
// |Q|, |P| > 1e9; out[1..3] / out[4..6] = min / max of floor(P/dp) per
// dimension (when dp != nullptr).  `part` holds packet_scan_bytes().
size_t packet_scan_bytes();
void launch_packet_scan(const fggc_packets &pk, const double *dp, long long *part, long long *out,
                        hipStream_t s);

// Zero `bytes` (a multiple of 4) of device memory with a kernel (capturable
// in a graph, unlike a memset node).
void launch_zero(void *p, size_t bytes, hipStream_t s);
// Fill slots [N, Npad) of SoA packet arrays sized Npad with zero-amplitude
// copies of packets 0, 1, 2, ... (they add exactly nothing to any sum).
void launch_pad_packets(int d, int64_t N, int64_t Npad, double *Q, double *P, double *S, double *a,
                        hipStream_t s);

// Counting sort positions: for slot i with keys[i] in [0, nbins), pos[i] is
// its position in key order; slots with keys[i] == kNoKey get kNoKey.
// start[b] = first position of key b, start[nbins] = number of keyed slots.
// The order of slots inside one key is unspecified.  `scratch` holds
// bucket_positions_bytes(N, nbins).
constexpr uint32_t kNoKey = 0xffffffffu;
size_t bucket_positions_bytes(int64_t N, int64_t nbins);
// True when the sort's launches may be captured into a graph and replayed.
bool bucket_positions_graph_safe(int64_t N, int64_t nbins);

// The LDS counting sort in pieces, for callers that compute their keys in
// their own counting kernel: slots are counted in G chunks of `chunk` slots (a
// multiple of `unit`); the caller's kernel writes table[bin * G + chunk_column(chunk)], each
// slot's rank inside (bin, chunk) and its key; count_scan turns the table into
// offsets inside each bin and start[]; count_positions gives each slot its position.
// Only for lds == true (nbins <= 2^15).
struct CountPlan {
  bool lds;
  int G;
  int64_t chunk;
  size_t off_table, off_offs, off_rank, off_rowsum, bytes;  // in the scratch area
};
CountPlan count_plan(int64_t N, int64_t nbins, int unit);
void count_scan(const CountPlan &c, int64_t nbins, char *scratch, int64_t *start, hipStream_t s);
// pos[i] = start[keys[i]] + offs[keys[i] * G + chunk_column(i / chunk)] + rank[i]
// (kNoKey for kNoKey slots)
void count_positions(const CountPlan &c, const uint32_t *keys, int64_t N, char *scratch, const int64_t *start,
                     uint32_t *pos, hipStream_t s);
void bucket_positions(const uint32_t *keys, int64_t N, int64_t nbins, uint32_t *pos, int64_t *start,
                      void *scratch, hipStream_t s);

// Direct sum.  Returns after enqueuing; `ws` supplies scratch.
// Initial decomposition (2.7) by windowed quadrature; device pointers, stream-ordered.
void launch_decompose(int d, const int64_t *n, const double *u0, double eps, double R, int64_t N,
                      const double *q, const double *p, double *A, hipStream_t s);
// Decomposition (2.7) on a product mesh with q on grid points, by batched ZGEMMs
// (rocBLAS handle created in *blas on first use); device pointers; ws must hold
// decompose_mesh_bytes().
size_t decompose_mesh_bytes(int d, const int64_t *n, double R, const int64_t *q_n, const int64_t *p_n);
void decompose_mesh(void **blas, int d, const int64_t *n, const double *u0, double eps, double R, const int64_t *Nq,
                    const int64_t *q_lo, const int64_t *q_n, const double *dp, const int64_t *p_lo,
                    const int64_t *p_n, double *A, Workspace &ws, hipStream_t s);
void destroy_blas(void *blas);
// Packet flow (RK4 for eq. 2.3-2.6); device pointers, stream-ordered.
void launch_propagate(int d, int64_t N, double *Q, double *P, double *S, double *a, double *jac,
                      const fggc_potential &V, double dt, int64_t nsteps, hipStream_t s);

// multi-step FGGC bookkeeping (learn.hip); scratch: learn_scratch_bytes()
size_t learn_scratch_bytes();
void launch_learn_select(int64_t Nm, const double *A0, double prune, uint8_t *learned, int64_t *keep_idx,
                         int64_t *new_idx, double *scratch, int64_t *counts, hipStream_t s);
void launch_learn_start(int d, int64_t Nm, int64_t n, const int64_t *idx, const double *qm, const double *pm,
                        double *Q, double *P, double *S, double *A, hipStream_t s);
void launch_learn_store(int d, int64_t Nm, int64_t n, const int64_t *idx, const double *Q, const double *P,
                        const double *S, const double *A, double *Qf, double *Pf, double *Sf, double *ratio,
                        hipStream_t s);
void launch_learn_packets(int d, int64_t Nm, int64_t n, const int64_t *idx, const double *Qf, const double *Pf,
                          const double *Sf, const double *ratio, const double *A0, double *Q, double *P,
                          double *S, double *a, hipStream_t s);

struct DirectArgs {
  const fggc_packets *pk;
  double eps, R, scale;
  GridGeom g;
  Box box;  // output points (row-major over the box)
  int precision;
  int box_window = 0;  // 1: window |y_k| <= R per dimension, separable evaluation (d = 2, FP32)
  void *u;  // device output
  Profiler *prof = nullptr;
};
size_t direct_workspace_bytes(const DirectArgs &a);
// True when launch_direct's launches may be captured into a graph and replayed.
bool direct_graph_safe(const DirectArgs &a);
void launch_direct(const DirectArgs &a, Workspace &ws, hipStream_t s);

// FGGC.
struct FggcArgs {
  const fggc_packets *pk;
  double eps, scale;
  GridGeom g;
  int precision;
  const DimLsq *lsq;  // [d], host
  const DimLsq *lsq_dev = nullptr;  // [d], device copy when the plan is cached
  int64_t Nq[3];
  double dp[3];
  int64_t slo[3], sn[3];  // p-cell box
  double cK;              // band half-width in units of 1/sqrt(eps)
  void *u;                // device output
  Profiler *prof = nullptr;
};
size_t fggc_workspace_bytes(const FggcArgs &a);
// True when launch_fggc's launches may be captured into a graph and replayed.
bool fggc_graph_safe(const FggcArgs &a);
void launch_fggc(const FggcArgs &a, Workspace &ws, hipStream_t s);
// Only the cell array (eq. 2.25) into `cells` (device).
void launch_fggc_cells(const FggcArgs &a, void *cells, Workspace &ws, hipStream_t s);
// The coefficient kernel's per-packet coefficients (FP64): c_out [N][n1^d]
// complex, cell_out [N][2][d] (q index, p-cell); a.slo, a.sn are not used.
void launch_fggc_coefficients(const FggcArgs &a, double *c_out, int32_t *cell_out, Workspace &ws, hipStream_t s);
size_t fggc_coefficients_workspace_bytes(const FggcArgs &a);
size_t fggc_cells_workspace_bytes(const FggcArgs &a);


// Device table exp(-2 pi i k / n), k < n, in the working precision (cached).
const void *fft_twiddles(int64_t n, int precision);

// Batched in-place d-dimensional FFT (powers of two).
size_t fft_workspace_bytes(int d, const int64_t *n, int precision, int64_t batch);
void launch_fft(int d, const int64_t *n, int64_t batch, int direction, int precision, void *data,
                Workspace &ws, hipStream_t s, Profiler *prof = nullptr, const char *stage = "fft");
// One d-dimensional FFT from src to dst (src may be overwritten).
void launch_fft_to(int d, const int64_t *n, int direction, int precision, void *src, void *dst,
                   Workspace &ws, hipStream_t s, Profiler *prof = nullptr, const char *stage = "fft");

// --------------------------------------------------------------------------
// argument checks shared by the entry points (api.cpp)
// --------------------------------------------------------------------------

bool is_pow2(int64_t v);
bool is_fft_size(int64_t v);  // v >= 2 and v = 2^a 3^b 5^c
// true when `p` can be dereferenced by kernels on the current device as is
bool device_accessible(const void *p);
// true when any packet array is not device-accessible
bool packets_on_host(const fggc_packets &pk);
void check_packets(const fggc_packets *pk, int d);
GridGeom check_grid(const fggc_grid *g);
void check_eps(double eps);
void check_strategy(const fggc_strategy *st, int d);
void fill_fggc_args(FggcArgs &fa, const fggc_packets *pk, double eps, const GridGeom &g,
                    const fggc_strategy &st, double scale, int precision, const DimLsq *lsq,
                    const int64_t *slo, const int64_t *sn);
int64_t prod3(const int64_t *v, int d);

// Run f, turning exceptions into a status code and a thread-local message.
template <class F> int guarded(const char *what, F &&f) {
  try {
    f();
    return FGGC_OK;
  } catch (const Error &e) {
    set_last_error(std::string(what) + ": " + e.msg);
    return e.code;
  } catch (const std::exception &e) {
    set_last_error(std::string(what) + ": " + e.what());
    return FGGC_EDEVICE;
  } catch (...) {
    set_last_error(std::string(what) + ": unknown internal error");
    return FGGC_EDEVICE;
  }
}

}  // namespace fggc

// The context behind the opaque ABI handle.
struct fggc_ctx {
  int device = 0;
  size_t budget = 0;
  hipStream_t stream = nullptr;
  fggc::Workspace ws;
  long long *dev_scan = nullptr;  // device scratch of the packet pre-pass (+ its 8 results)
  long long *host_scan = nullptr; // pinned copy of the 8 results
  bool profiling = false;
  fggc::Profiler prof;
  std::mutex mu;
  // the stream that last used the workspace and an event recorded after that
  // use (a call on another stream waits for it)
  hipStream_t last_stream = nullptr;
  bool has_last = false;
  hipEvent_t ws_event = nullptr;
  // executable graphs of repeated device-resident reconstructions, most recent first
  hipStream_t cap_stream = nullptr;
  std::list<std::pair<std::vector<int64_t>, hipGraphExec_t>> graphs;
  std::map<std::vector<int64_t>, int> seen;
  const void *graphs_ws = nullptr;
  void *blas = nullptr;  // rocBLAS handle of the mesh decomposition, created on first use
};
