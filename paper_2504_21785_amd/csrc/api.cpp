// C ABI of libfggc: argument checks, context and workspace, host/device
// staging, and the error model (every entry point returns an fggc_status and
// records a thread-local message; no exception crosses the ABI).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <string>

#include "common.h"

// Scratch of fggc_direct_sum_noalloc: one array per GPU (each device holds its
// own copy, at its own address), reached only through the address that
// hipGetSymbolAddress returns for the device (noalloc_scratch below).
static __device__ __align__(256) unsigned char scratch[FGGC_NOALLOC_SCRATCH_BYTES];

namespace fggc {

namespace {
thread_local std::string g_last_error;

std::mutex g_noalloc_mu;
std::vector<void *> g_noalloc_ptr;  // device address of `scratch`, per device

// Once per device, with that device current: look up the array's device address.
void noalloc_setup(int device) {
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if ((int)g_noalloc_ptr.size() <= device) g_noalloc_ptr.resize((size_t)device + 1, nullptr);
  if (g_noalloc_ptr[(size_t)device]) return;
  void *ptr = nullptr;
  FGGC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) fail(FGGC_EDEVICE, "no device address for the no-allocation scratch");
  g_noalloc_ptr[(size_t)device] = ptr;
}

char *noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (device < 0 || (size_t)device >= g_noalloc_ptr.size() || !g_noalloc_ptr[(size_t)device])
    fail(FGGC_EDEVICE, "no-allocation scratch not set up on this device");
  return (char *)g_noalloc_ptr[(size_t)device];
}
}  // namespace

void set_last_error(const std::string &msg) { g_last_error = msg; }

void fail(int code, const std::string &msg) { throw Error{code, msg}; }

Workspace::~Workspace() {
  if (base_ && owned_) (void)hipFree(base_);
}

void Workspace::reserve(size_t bytes, size_t budget) {
  used_ = 0;
  if (bytes <= cap_) return;
  if (!owned_) fail(FGGC_EBUDGET, "request needs " + std::to_string(bytes) + " bytes of scratch, " +
                                      std::to_string(cap_) + " are available");
  if (bytes > budget)
    fail(FGGC_EBUDGET, "request needs " + std::to_string(bytes) + " bytes of workspace, budget is " +
                           std::to_string(budget));
  if (base_) {
    if (has_stream_) FGGC_HIP(hipStreamSynchronize(stream_));
    else FGGC_HIP(hipDeviceSynchronize());
    FGGC_HIP(hipFree(base_));
    base_ = nullptr;
    cap_ = 0;
  }
  size_t want = std::min(budget, std::max(bytes, bytes + bytes / 4));
  if (hipMalloc((void **)&base_, want) != hipSuccess) {
    (void)hipGetLastError();
    want = bytes;
    if (hipMalloc((void **)&base_, want) != hipSuccess) {
      (void)hipGetLastError();
      base_ = nullptr;
      fail(FGGC_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    }
  }
  cap_ = want;
}

void Workspace::release() {
  used_ = 0;
  if (!base_ || !owned_) return;
  if (has_stream_) FGGC_HIP(hipStreamSynchronize(stream_));
  else FGGC_HIP(hipDeviceSynchronize());
  FGGC_HIP(hipFree(base_));
  base_ = nullptr;
  cap_ = 0;
}

void *Workspace::take(size_t bytes) {
  size_t at = used_;
  used_ = align_up(used_ + bytes, 256);
  if (used_ > cap_) fail(FGGC_EDEVICE, "internal: workspace overrun");
  return base_ + at;
}

Profiler::~Profiler() {
  for (auto &q : pending_) {
    (void)hipEventDestroy(q.a);
    (void)hipEventDestroy(q.b);
  }
  for (auto &o : open_) (void)hipEventDestroy(o.second);
}

void Profiler::start(const char *stage, hipStream_t s) {
  std::lock_guard<std::mutex> lk(mu_);
  hipEvent_t e;
  FGGC_HIP(hipEventCreate(&e));
  FGGC_HIP(hipEventRecord(e, s));
  open_.push_back({stage, e});
}

void Profiler::stop(const char *stage, hipStream_t s) {
  std::lock_guard<std::mutex> lk(mu_);
  for (size_t i = open_.size(); i-- > 0;) {
    if (open_[i].first == stage) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess || hipEventRecord(e, s) != hipSuccess) {
        (void)hipGetLastError();
        return;
      }
      pending_.push_back({open_[i].first, open_[i].second, e});
      open_.erase(open_.begin() + (long)i);
      return;
    }
  }
}

void Profiler::drain() {
  for (auto &q : pending_) {
    float ms = 0.f;
    if (hipEventSynchronize(q.b) == hipSuccess && hipEventElapsedTime(&ms, q.a, q.b) == hipSuccess) {
      bool found = false;
      for (auto &a : acc_)
        if (a.first == q.stage) {
          a.second.ms += ms;
          a.second.count += 1;
          found = true;
        }
      if (!found) acc_.push_back({q.stage, Acc{ms, 1}});
    } else {
      (void)hipGetLastError();
    }
    (void)hipEventDestroy(q.a);
    (void)hipEventDestroy(q.b);
  }
  pending_.clear();
}

void Profiler::query(const std::string &stage, double *ms, int64_t *count) {
  std::lock_guard<std::mutex> lk(mu_);
  drain();
  *ms = 0;
  *count = 0;
  for (auto &a : acc_)
    if (a.first == stage) {
      *ms = a.second.ms;
      *count = a.second.count;
    }
}

void Profiler::reset() {
  std::lock_guard<std::mutex> lk(mu_);
  drain();
  acc_.clear();
}

std::vector<std::string> Profiler::stages() {
  std::lock_guard<std::mutex> lk(mu_);
  drain();
  std::vector<std::string> v;
  for (auto &a : acc_) v.push_back(a.first);
  return v;
}

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

bool is_fft_size(int64_t v) {
  if (v < 2) return false;
  for (int f : {2, 3, 5})
    while (v % f == 0) v /= f;
  return v == 1;
}

// true when `p` can be dereferenced by kernels on the current device as is
bool device_accessible(const void *p) {
  hipPointerAttribute_t at;
  hipError_t e = hipPointerGetAttributes(&at, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged ||
         at.type == hipMemoryTypeUnified;
}

void check_packets(const fggc_packets *pk, int d) {
  if (!pk) fail(FGGC_EINVAL, "packets is NULL");
  if (pk->d != d) fail(FGGC_EINVAL, "packets->d does not match grid->d");
  if (pk->N < 0 || pk->N > 0x7fffffffLL) fail(FGGC_EINVAL, "packet count out of range [0, 2^31)");
  if (pk->N > 0 && (!pk->Q || !pk->P || !pk->S || !pk->a)) fail(FGGC_EINVAL, "packet array is NULL");
}

GridGeom check_grid(const fggc_grid *g) {
  if (!g) fail(FGGC_EINVAL, "grid is NULL");
  if (g->d < 1 || g->d > 3) fail(FGGC_EINVAL, "grid->d must be 1, 2 or 3");
  GridGeom gg{};
  gg.d = g->d;
  int64_t total = 1;
  for (int k = 0; k < 3; ++k) {
    if (k < g->d) {
      if (g->n[k] < 1 || g->n[k] > (1 << 24)) fail(FGGC_EINVAL, "grid size out of range [1, 2^24]");
      gg.n[k] = g->n[k];
      gg.dx[k] = kTwoPi / (double)g->n[k];
      total *= g->n[k];
    } else {
      gg.n[k] = 1;
      gg.dx[k] = 1.0;
    }
  }
  if (total > (int64_t)1 << 31) fail(FGGC_EINVAL, "grid has more than 2^31 points");
  return gg;
}

void check_eps(double eps) {
  if (!(eps > 0) || !std::isfinite(eps)) fail(FGGC_EINVAL, "eps must be finite and > 0");
}

// Inputs as device pointers: staged through the workspace when on the host.
struct Staged {
  fggc_packets pk;
  bool host_out = false;
  void *u_dev = nullptr;
};

size_t staging_bytes(const fggc_packets &pk, bool any_host, size_t out_bytes, bool host_out) {
  size_t b = 0;
  if (any_host) b += align_up(pk.N * (size_t)(2 * pk.d + 3) * 8, 256) + 256;
  if (host_out) b += align_up(out_bytes, 256) + 256;
  return b;
}

struct Guard {
  fggc_ctx *ctx;
  explicit Guard(fggc_ctx *c) : ctx(c) {
    ctx->mu.lock();
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) {
      ctx->mu.unlock();
      fail(FGGC_EDEVICE, std::string("hipSetDevice: ") + hipGetErrorString(e));
    }
  }
  ~Guard() { ctx->mu.unlock(); }
};


// Copy host-resident packet arrays into `dst` (device); returns device views.
fggc_packets stage_packets(const fggc_packets &pk, char *dst, hipStream_t s) {
  fggc_packets out = pk;
  const size_t dN = (size_t)pk.d * pk.N * 8, N8 = (size_t)pk.N * 8;
  double *Q = (double *)dst, *P = Q + (size_t)pk.d * pk.N, *S = P + (size_t)pk.d * pk.N,
         *a = S + pk.N;
  FGGC_HIP(hipMemcpyAsync(Q, pk.Q, dN, hipMemcpyHostToDevice, s));
  FGGC_HIP(hipMemcpyAsync(P, pk.P, dN, hipMemcpyHostToDevice, s));
  FGGC_HIP(hipMemcpyAsync(S, pk.S, N8, hipMemcpyHostToDevice, s));
  FGGC_HIP(hipMemcpyAsync(a, pk.a, 2 * N8, hipMemcpyHostToDevice, s));
  out.Q = Q;
  out.P = P;
  out.S = S;
  out.a = a;
  return out;
}

bool packets_on_host(const fggc_packets &pk) {
  if (pk.N == 0) return false;
  return !(device_accessible(pk.Q) && device_accessible(pk.P) && device_accessible(pk.S) &&
           device_accessible(pk.a));
}

// Packet pre-pass (validity and, with dp, the p-cell range); one synchronisation.
void prepass(fggc_ctx *ctx, const fggc_packets &pk, const double *dp, hipStream_t s) {
  if (pk.N == 0) return;
  long long *out = ctx->dev_scan + packet_scan_bytes() / 8;
  {
    StageScope sc(ctx->profiling ? &ctx->prof : nullptr, "prepass", s);
    launch_packet_scan(pk, dp, ctx->dev_scan, out, s);
  }
  FGGC_HIP(hipMemcpyAsync(ctx->host_scan, out, 8 * sizeof(long long), hipMemcpyDeviceToHost, s));
  FGGC_HIP(hipStreamSynchronize(s));
  if (ctx->host_scan[0] != 0)
    fail(FGGC_EINVAL, std::to_string(ctx->host_scan[0]) +
                          " packet(s) with NaN/Inf in Q, P, S or a, or |Q| or |P| above 1e9");
}

void check_strategy(const fggc_strategy *st, int d) {
  if (!st) fail(FGGC_EINVAL, "strategy is NULL");
  if (st->nq < 1 || st->np < 1 || st->nq > 8 || st->np > 8 || st->nq * st->np > kMaxN1)
    fail(FGGC_EINVAL, "strategy needs 1 <= nq, np <= 8 and nq * np <= 16");
  for (int i = 0; i < st->nq; ++i)
    for (int j = i + 1; j < st->nq; ++j)
      if (st->dq_off[i] == st->dq_off[j]) fail(FGGC_EINVAL, "repeated q shift in strategy");
  for (int i = 0; i < st->np; ++i)
    for (int j = i + 1; j < st->np; ++j)
      if (st->dp_off[i] == st->dp_off[j]) fail(FGGC_EINVAL, "repeated p shift in strategy");
  for (int i = 0; i < st->nq; ++i)
    if (std::abs(st->dq_off[i]) > 64) fail(FGGC_EINVAL, "q shift out of range [-64, 64]");
  for (int i = 0; i < st->np; ++i)
    if (std::abs(st->dp_off[i]) > 64) fail(FGGC_EINVAL, "p shift out of range [-64, 64]");
  if (!(st->cutoff >= 0) || !(st->cutoff < 1)) fail(FGGC_EINVAL, "cutoff must be in [0, 1)");
  {
    int a = st->dq_off[0], b = st->dq_off[0], c = st->dp_off[0], e = st->dp_off[0];
    for (int i = 1; i < st->nq; ++i) { a = std::min(a, st->dq_off[i]); b = std::max(b, st->dq_off[i]); }
    for (int i = 1; i < st->np; ++i) { c = std::min(c, st->dp_off[i]); e = std::max(e, st->dp_off[i]); }
    if (b - a > 31 || e - c > 31) fail(FGGC_EINVAL, "shift sets must span at most 31 cells");
  }
  for (int k = 0; k < d; ++k) {
    if (st->Nq[k] < 4 || st->Nq[k] > 8192 || st->Nq[k] % 2 || !is_fft_size(st->Nq[k]))
      fail(FGGC_EUNSUPPORTED, "Nq must be an even 2^a 3^b 5^c in [4, 8192]");
    if (!(st->dp[k] > 0) || !std::isfinite(st->dp[k])) fail(FGGC_EINVAL, "dp must be finite and > 0");
  }
}

// p-cell box of the packets (from the pre-pass, which must have run with dp).
void cell_box(fggc_ctx *ctx, const fggc_packets &pk, const fggc_strategy &st, int64_t *slo,
              int64_t *sn) {
  if (pk.N == 0) fail(FGGC_EINVAL, "no packets");
  int mn = st.dp_off[0], mx = st.dp_off[0];
  for (int i = 1; i < st.np; ++i) {
    mn = std::min(mn, st.dp_off[i]);
    mx = std::max(mx, st.dp_off[i]);
  }
  for (int k = 0; k < pk.d; ++k) {
    const long long lo = ctx->host_scan[1 + k], hi = ctx->host_scan[4 + k];
    if (hi < lo || lo < -((long long)1 << 40) || hi > ((long long)1 << 40))
      fail(FGGC_EINVAL, "momenta out of range for the p-mesh");
    slo[k] = lo + mn;
    sn[k] = hi + mx - slo[k] + 1;
  }
  for (int k = pk.d; k < 3; ++k) {
    slo[k] = 0;
    sn[k] = 1;
  }
}

void fill_fggc_args(FggcArgs &fa, const fggc_packets *pk, double eps, const GridGeom &g,
                    const fggc_strategy &st, double scale, int precision, const DimLsq *lsq,
                    const int64_t *slo, const int64_t *sn) {
  fa.pk = pk;
  fa.eps = eps;
  fa.scale = scale;
  fa.g = g;
  fa.precision = precision;
  fa.lsq = lsq;
  for (int k = 0; k < 3; ++k) {
    fa.Nq[k] = k < g.d ? st.Nq[k] : 1;
    fa.dp[k] = k < g.d ? st.dp[k] : 1.0;
    fa.slo[k] = slo[k];
    fa.sn[k] = sn[k];
  }
  fa.cK = precision == FGGC_FP64 ? 8.0 : 6.0;
}

int64_t prod3(const int64_t *v, int d) {
  int64_t p = 1;
  for (int k = 0; k < d; ++k) p *= v[k];
  return p;
}

namespace {

// The workspace is shared by the calls on a context: a call on a different
// stream than the previous one makes its stream wait (on the device) for the
// event recorded after the previous call's work.
struct WsUse {
  fggc_ctx *ctx;
  hipStream_t s;
  WsUse(fggc_ctx *c, hipStream_t st) : ctx(c), s(st) {
    if (ctx->has_last && ctx->last_stream != s) FGGC_HIP(hipStreamWaitEvent(s, ctx->ws_event, 0));
  }
  ~WsUse() {
    if (hipEventRecord(ctx->ws_event, s) == hipSuccess) {
      ctx->last_stream = s;
      ctx->has_last = true;
    } else {
      (void)hipGetLastError();
    }
  }
};

void clear_graphs(fggc_ctx *ctx) {
  for (auto &g : ctx->graphs) (void)hipGraphExecDestroy(g.second);
  ctx->graphs.clear();
}

int64_t dbits(double x) {
  int64_t b;
  std::memcpy(&b, &x, 8);
  return b;
}

constexpr size_t kCtxGraphs = 8;

// Run `launch(stream)` on s, through a cached executable graph when the same
// key (shape, buffers and workspace) has been seen before: the first sighting
// runs eagerly, the second is captured on the context's capture stream, later
// ones replay the graph.  A capture that fails falls back to eager runs for
// that key.
template <class F> void run_cached(fggc_ctx *ctx, std::vector<int64_t> key, hipStream_t s, F &&launch) {
  if (ctx->graphs_ws != ctx->ws.base()) {
    clear_graphs(ctx);
    ctx->seen.clear();
    ctx->graphs_ws = ctx->ws.base();
  }
  key.push_back((int64_t)(uintptr_t)ctx->ws.base());
  key.push_back((int64_t)ctx->ws.capacity());
  for (auto it = ctx->graphs.begin(); it != ctx->graphs.end(); ++it)
    if (it->first == key) {
      ctx->graphs.splice(ctx->graphs.begin(), ctx->graphs, it);
      FGGC_HIP(hipGraphLaunch(ctx->graphs.front().second, s));
      return;
    }
  if (ctx->seen.size() > 4096) ctx->seen.clear();
  int &n = ctx->seen[key];
  const size_t mark = ctx->ws.mark();
  if (++n >= 2) {
    hipStream_t cs = ctx->cap_stream;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      try {
        launch(cs);
      } catch (...) {
        ok = false;
      }
      if (hipStreamEndCapture(cs, &graph) != hipSuccess) ok = false;
      if (ok && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) ok = false;
      if (graph) (void)hipGraphDestroy(graph);
    }
    if (ok) {
      if (ctx->graphs.size() >= kCtxGraphs) {
        (void)hipGraphExecDestroy(ctx->graphs.back().second);
        ctx->graphs.pop_back();
      }
      ctx->graphs.emplace_front(key, exec);
      FGGC_HIP(hipGraphLaunch(exec, s));
      return;
    }
    (void)hipGetLastError();
    if (exec) (void)hipGraphExecDestroy(exec);
    n = -(1 << 30);
    ctx->ws.rewind(mark);
  }
  launch(s);
}

}  // namespace

}  // namespace fggc

using namespace fggc;

extern "C" {

const char *fggc_last_error(void) { return g_last_error.c_str(); }

const char *fggc_version(void) { return "fggc 0.1 (gfx950)"; }

int fggc_create(fggc_ctx **out, int device, size_t hbm_budget_bytes) {
  return guarded("fggc_create", [&] {
    if (!out) fail(FGGC_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    FGGC_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) fail(FGGC_EINVAL, "no such device");
    FGGC_HIP(hipSetDevice(device));
    noalloc_setup(device);
    fggc_ctx *c = new fggc_ctx();
    c->device = device;
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      (void)hipGetLastError();
      fr = tot = 0;
    }
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.9 * (double)fr);
    try {
      FGGC_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      FGGC_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
      FGGC_HIP(hipEventCreateWithFlags(&c->ws_event, hipEventDisableTiming));
      FGGC_HIP(hipMalloc((void **)&c->dev_scan, packet_scan_bytes() + 256));
      FGGC_HIP(hipHostMalloc((void **)&c->host_scan, 256, hipHostMallocDefault));
    } catch (...) {
      fggc_destroy(c);
      throw;
    }
    *out = c;
  });
}

void fggc_destroy(fggc_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  if (ctx->ws_event) {
    (void)hipEventSynchronize(ctx->ws_event);
    (void)hipEventDestroy(ctx->ws_event);
  }
  clear_graphs(ctx);
  fggc::destroy_blas(ctx->blas);
  if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
  if (ctx->dev_scan) (void)hipFree(ctx->dev_scan);
  if (ctx->host_scan) (void)hipHostFree(ctx->host_scan);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

namespace {
int direct_impl(const char *what, fggc_ctx *ctx, const fggc_packets *pk, double eps,
                const fggc_grid *grid, const int64_t *box_lo, const int64_t *box_n,
                double window_radius, double scale, int precision, void *u_out, void *stream,
                int box_window = 0) {
  return guarded(what, [&] {
    if (!ctx) fail(FGGC_EINVAL, "ctx is NULL");
    GridGeom g = check_grid(grid);
    check_packets(pk, g.d);
    check_eps(eps);
    if (!(window_radius > 0) || !(window_radius < kPi))
      fail(FGGC_EINVAL, "window_radius must be in (0, pi)");
    if (!std::isfinite(scale)) fail(FGGC_EINVAL, "scale must be finite");
    if (precision != FGGC_FP32 && precision != FGGC_FP64) fail(FGGC_EINVAL, "bad precision");
    if (!u_out) fail(FGGC_EINVAL, "u_out is NULL");
    if (box_window) {
      if (g.d != 2) fail(FGGC_EUNSUPPORTED, "the separable direct sum is two-dimensional (d = 2)");
      if (precision != FGGC_FP32) fail(FGGC_EUNSUPPORTED, "the separable direct sum computes in FP32");
      if (g.n[0] > (1 << 20) || g.n[1] > (1 << 20)) fail(FGGC_EUNSUPPORTED, "grid axes above 2^20 points");
    }
    Box box{};
    int64_t npts = 1;
    for (int k = 0; k < 3; ++k) {
      box.lo[k] = 0;
      box.n[k] = g.n[k];
      if (k < g.d && box_lo && box_n) {
        if (box_lo[k] < 0 || box_n[k] < 1 || box_lo[k] + box_n[k] > g.n[k])
          fail(FGGC_EINVAL, "box outside the grid");
        box.lo[k] = box_lo[k];
        box.n[k] = box_n[k];
      }
      if (k < g.d) npts *= box.n[k];
    }
    Guard lock(ctx);
    hipStream_t s = (hipStream_t)stream;
    WsUse wsu(ctx, s);
    const size_t out_bytes = (size_t)npts * (precision == FGGC_FP64 ? 16 : 8);
    const bool host_in = packets_on_host(*pk);
    const bool host_out = !device_accessible(u_out);
    DirectArgs da{};
    fggc_packets dpk = *pk;
    da.pk = &dpk;
    da.eps = eps;
    da.R = window_radius;
    da.scale = scale;
    da.g = g;
    da.box = box;
    da.precision = precision;
    da.box_window = box_window;
    da.prof = ctx->profiling ? &ctx->prof : nullptr;
    const size_t need = staging_bytes(*pk, host_in, out_bytes, host_out) + direct_workspace_bytes(da);
    ctx->ws.reserve(need, ctx->budget);
    if (host_in) dpk = stage_packets(*pk, (char *)ctx->ws.take((size_t)pk->N * (2 * pk->d + 3) * 8), s);
    da.u = host_out ? ctx->ws.take(out_bytes) : u_out;
    prepass(ctx, dpk, nullptr, s);
    launch_direct(da, ctx->ws, s);
    if (host_out) {
      FGGC_HIP(hipMemcpyAsync(u_out, da.u, out_bytes, hipMemcpyDeviceToHost, s));
      FGGC_HIP(hipStreamSynchronize(s));
    } else if (host_in) {
      FGGC_HIP(hipStreamSynchronize(s));
    }
  });
}
}  // namespace

int fggc_direct_sum(fggc_ctx *ctx, const fggc_packets *pk, double eps, const fggc_grid *grid,
                    double window_radius, double scale, int precision, void *u_out, void *stream) {
  return direct_impl("fggc_direct_sum", ctx, pk, eps, grid, nullptr, nullptr, window_radius, scale,
                     precision, u_out, stream);
}

int fggc_direct_sum_box(fggc_ctx *ctx, const fggc_packets *pk, double eps, const fggc_grid *grid,
                        const int64_t *box_lo, const int64_t *box_n, double window_radius,
                        double scale, int precision, void *u_out, void *stream) {
  if (!box_lo || !box_n) {
    set_last_error("fggc_direct_sum_box: box is NULL");
    return FGGC_EINVAL;
  }
  return direct_impl("fggc_direct_sum_box", ctx, pk, eps, grid, box_lo, box_n, window_radius, scale,
                     precision, u_out, stream);
}

int fggc_direct_sum_noalloc(fggc_ctx *ctx, const fggc_packets *pk, double eps, const fggc_grid *grid,
                            double window_radius, double scale, int precision, void *u_out, void *stream) {
  return guarded("fggc_direct_sum_noalloc", [&] {
    if (!ctx) fail(FGGC_EINVAL, "ctx is NULL");
    GridGeom g = check_grid(grid);
    check_packets(pk, g.d);
    check_eps(eps);
    if (!(window_radius > 0) || !(window_radius < kPi))
      fail(FGGC_EINVAL, "window_radius must be in (0, pi)");
    if (!std::isfinite(scale)) fail(FGGC_EINVAL, "scale must be finite");
    if (precision != FGGC_FP32 && precision != FGGC_FP64) fail(FGGC_EINVAL, "bad precision");
    if (!u_out) fail(FGGC_EINVAL, "u_out is NULL");
    Guard lock(ctx);
    if (packets_on_host(*pk) || !device_accessible(u_out))
      fail(FGGC_EINVAL, "packets and u_out must be device memory (staging host buffers would allocate)");
    hipStream_t s = (hipStream_t)stream;
    char *scr = noalloc_scratch(ctx->device);
    DirectArgs da{};
    fggc_packets dpk = *pk;
    da.pk = &dpk;
    da.eps = eps;
    da.R = window_radius;
    da.scale = scale;
    da.g = g;
    for (int k = 0; k < 3; ++k) {
      da.box.lo[k] = 0;
      da.box.n[k] = g.n[k];
    }
    da.precision = precision;
    da.u = u_out;
    da.prof = nullptr;
    // [pre-pass partials and results][the direct sum's workspace]
    const size_t scan_b = align_up(packet_scan_bytes() + 8 * sizeof(long long), 256);
    const size_t need = scan_b + direct_workspace_bytes(da);
    if (need > FGGC_NOALLOC_SCRATCH_BYTES)
      fail(FGGC_EBUDGET, "request needs " + std::to_string(need) + " bytes of scratch, the limit is " +
                             std::to_string((size_t)FGGC_NOALLOC_SCRATCH_BYTES));
    if (pk->N > 0) {
      long long *part = (long long *)scr, *res = part + packet_scan_bytes() / 8;
      launch_packet_scan(dpk, nullptr, part, res, s);
      long long host[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      FGGC_HIP(hipMemcpyAsync(host, res, sizeof(host), hipMemcpyDeviceToHost, s));
      FGGC_HIP(hipStreamSynchronize(s));
      if (host[0] != 0)
        fail(FGGC_EINVAL, std::to_string(host[0]) +
                              " packet(s) with NaN/Inf in Q, P, S or a, or |Q| or |P| above 1e9");
    }
    Workspace view(scr + scan_b, FGGC_NOALLOC_SCRATCH_BYTES - scan_b);
    launch_direct(da, view, s);
  });
}

int fggc_direct_sum_separable(fggc_ctx *ctx, const fggc_packets *pk, double eps, const fggc_grid *grid,
                              double window_half_width, double scale, int precision, void *u_out,
                              void *stream) {
  return direct_impl("fggc_direct_sum_separable", ctx, pk, eps, grid, nullptr, nullptr, window_half_width,
                     scale, precision, u_out, stream, 1);
}

int fggc_decompose(fggc_ctx *ctx, const fggc_grid *grid, const double *u0, double eps, double window_radius,
                   int64_t N, const double *q, const double *p, double *A_out, void *stream) {
  return guarded("fggc_decompose", [&] {
    if (!ctx) fail(FGGC_EINVAL, "ctx is NULL");
    GridGeom g = check_grid(grid);
    check_eps(eps);
    if (!(window_radius > 0) || !(window_radius < kPi)) fail(FGGC_EINVAL, "window_radius must be in (0, pi)");
    if (N < 0 || N > 0x7fffffffLL) fail(FGGC_EINVAL, "packet count out of range [0, 2^31)");
    if (!u0) fail(FGGC_EINVAL, "u0 is NULL");
    if (N > 0 && (!q || !p || !A_out)) fail(FGGC_EINVAL, "packet array is NULL");
    if (N == 0) return;
    Guard lock(ctx);
    hipStream_t s = (hipStream_t)stream;
    WsUse wsu(ctx, s);
    int64_t npts = 1;
    for (int k = 0; k < g.d; ++k) npts *= g.n[k];
    const size_t ub = (size_t)npts * 16, qb = (size_t)g.d * N * 8, ab = (size_t)N * 16;
    const bool host = !(device_accessible(u0) && device_accessible(q) && device_accessible(p) &&
                        device_accessible(A_out));
    if (!host) {
      launch_decompose(g.d, g.n, u0, eps, window_radius, N, q, p, A_out, s);
      return;
    }
    ctx->ws.reserve(ub + 2 * qb + ab + 4 * 256, ctx->budget);
    double *du = (double *)ctx->ws.take(ub), *dq = (double *)ctx->ws.take(qb), *dp = (double *)ctx->ws.take(qb);
    double *da = (double *)ctx->ws.take(ab);
    FGGC_HIP(hipMemcpyAsync(du, u0, ub, hipMemcpyDefault, s));
    FGGC_HIP(hipMemcpyAsync(dq, q, qb, hipMemcpyDefault, s));
    FGGC_HIP(hipMemcpyAsync(dp, p, qb, hipMemcpyDefault, s));
    launch_decompose(g.d, g.n, du, eps, window_radius, N, dq, dp, da, s);
    FGGC_HIP(hipMemcpyAsync(A_out, da, ab, hipMemcpyDefault, s));
    FGGC_HIP(hipStreamSynchronize(s));
  });
}

int fggc_decompose_mesh(fggc_ctx *ctx, const fggc_grid *grid, const double *u0, double eps,
                        double window_half_width, const int64_t *Nq, const int64_t *q_lo, const int64_t *q_n,
                        const double *dp, const int64_t *p_lo, const int64_t *p_n, double *A_out, void *stream) {
  return guarded("fggc_decompose_mesh", [&] {
    if (!ctx || !u0 || !Nq || !q_lo || !q_n || !dp || !p_lo || !p_n || !A_out) fail(FGGC_EINVAL, "NULL argument");
    GridGeom g = check_grid(grid);
    if (g.d > 2) fail(FGGC_EUNSUPPORTED, "the mesh decomposition is one- or two-dimensional");
    check_eps(eps);
    const double R = window_half_width;
    if (!(R > 0) || !(R < kPi)) fail(FGGC_EINVAL, "window_half_width must be in (0, pi)");
    int64_t nq = 1, np = 1;
    for (int k = 0; k < g.d; ++k) {
      if (Nq[k] < 1 || g.n[k] % Nq[k] != 0) fail(FGGC_EINVAL, "grid size must be a multiple of Nq (q on grid points)");
      if (q_n[k] < 1 || q_lo[k] < 0 || q_lo[k] + q_n[k] > Nq[k]) fail(FGGC_EINVAL, "q range outside [0, Nq)");
      if (p_n[k] < 1 || !(dp[k] > 0) || !std::isfinite(dp[k])) fail(FGGC_EINVAL, "bad p range or dp");
      if (2 * (int64_t)std::floor(R / (kTwoPi / (double)g.n[k])) + 1 > g.n[k])
        fail(FGGC_EINVAL, "window wider than the grid");
      nq *= q_n[k];
      np *= p_n[k];
    }
    if (nq * np > 0x7fffffffLL) fail(FGGC_EINVAL, "mesh larger than 2^31 points");
    Guard lock(ctx);
    hipStream_t s = (hipStream_t)stream;
    WsUse wsu(ctx, s);
    int64_t npts = 1;
    for (int k = 0; k < g.d; ++k) npts *= g.n[k];
    const size_t ub = (size_t)npts * 16, ab = (size_t)nq * np * 16;
    const bool host = !(device_accessible(u0) && device_accessible(A_out));
    const size_t need = decompose_mesh_bytes(g.d, g.n, R, q_n, p_n) + (host ? ub + ab + 2 * 256 : 0);
    ctx->ws.reserve(need, ctx->budget);
    const double *du = u0;
    double *da = A_out;
    if (host) {
      du = (const double *)ctx->ws.take(ub);
      da = (double *)ctx->ws.take(ab);
      FGGC_HIP(hipMemcpyAsync((void *)du, u0, ub, hipMemcpyDefault, s));
    }
    decompose_mesh(&ctx->blas, g.d, g.n, du, eps, R, Nq, q_lo, q_n, dp, p_lo, p_n, da, ctx->ws, s);
    if (host) {
      FGGC_HIP(hipMemcpyAsync(A_out, da, ab, hipMemcpyDefault, s));
      FGGC_HIP(hipStreamSynchronize(s));
    }
  });
}

int fggc_propagate(fggc_ctx *ctx, int32_t d, int64_t N, double *Q, double *P, double *S, double *a,
                   double *jac, const fggc_potential *V, double dt, int64_t nsteps, void *stream) {
  return guarded("fggc_propagate", [&] {
    if (!ctx || !V) fail(FGGC_EINVAL, "NULL argument");
    if (d < 1 || d > 3) fail(FGGC_EINVAL, "d must be 1, 2 or 3");
    if (N < 0 || N > 0x7fffffffLL) fail(FGGC_EINVAL, "packet count out of range [0, 2^31)");
    if (nsteps < 0) fail(FGGC_EINVAL, "nsteps must be >= 0");
    if (N > 0 && (!Q || !P || !S || !a)) fail(FGGC_EINVAL, "packet array is NULL");
    if (!std::isfinite(dt)) fail(FGGC_EINVAL, "dt must be finite");
    const double coef[] = {V->c0, V->w[0], V->w[1], V->w[2], V->c1, V->kappa, V->c2, V->c3};
    for (double c : coef)
      if (!std::isfinite(c)) fail(FGGC_EINVAL, "potential coefficients must be finite");
    if (N == 0 || nsteps == 0) return;
    Guard lock(ctx);
    hipStream_t s = (hipStream_t)stream;
    WsUse wsu(ctx, s);
    const size_t dN = (size_t)d * N * 8, N8 = (size_t)N * 8, jb = jac ? (size_t)N * 4 * d * d * 8 : 0;
    const bool host = !(device_accessible(Q) && device_accessible(P) && device_accessible(S) &&
                        device_accessible(a) && (!jac || device_accessible(jac)));
    if (!host) {
      launch_propagate(d, N, Q, P, S, a, jac, *V, dt, nsteps, s);
      return;
    }
    ctx->ws.reserve(2 * dN + 3 * N8 + jb + 5 * 256, ctx->budget);
    double *dQ = (double *)ctx->ws.take(dN), *dP = (double *)ctx->ws.take(dN);
    double *dS = (double *)ctx->ws.take(N8), *da = (double *)ctx->ws.take(2 * N8);
    double *dj = jac ? (double *)ctx->ws.take(jb) : nullptr;
    struct Arr { double *host, *dev; size_t bytes; } arrs[] = {
        {Q, dQ, dN}, {P, dP, dN}, {S, dS, N8}, {a, da, 2 * N8}, {jac, dj, jb}};
    for (const Arr &x : arrs)
      if (x.bytes) FGGC_HIP(hipMemcpyAsync(x.dev, x.host, x.bytes, hipMemcpyDefault, s));
    launch_propagate(d, N, dQ, dP, dS, da, dj, *V, dt, nsteps, s);
    for (const Arr &x : arrs)
      if (x.bytes) FGGC_HIP(hipMemcpyAsync(x.host, x.dev, x.bytes, hipMemcpyDefault, s));
    FGGC_HIP(hipStreamSynchronize(s));
  });
}

namespace {
// every pointer device memory of the current device (host buffers are refused)
void need_device(std::initializer_list<const void *> ps) {
  for (const void *p : ps)
    if (!device_accessible(p)) fail(FGGC_EINVAL, "buffers must be device memory");
}

void check_learn(int d, int64_t Nm, int64_t n) {
  if (d < 1 || d > 3) fail(FGGC_EINVAL, "d must be 1, 2 or 3");
  if (Nm < 0 || Nm > 0x7fffffffLL) fail(FGGC_EINVAL, "mesh size out of range [0, 2^31)");
  if (n < 0 || n > Nm) fail(FGGC_EINVAL, "n must be in [0, Nm]");
}
}  // namespace

int fggc_learn_select(fggc_ctx *ctx, int64_t Nm, const double *A0, double prune, uint8_t *learned,
                      int64_t *keep_idx, int64_t *new_idx, int64_t *n_keep, int64_t *n_new, void *stream) {
  return guarded("fggc_learn_select", [&] {
    if (!ctx || !n_keep || !n_new) fail(FGGC_EINVAL, "NULL argument");
    check_learn(1, Nm, 0);
    if (!(prune >= 0) || !(prune < 1)) fail(FGGC_EINVAL, "prune must be in [0, 1)");
    *n_keep = *n_new = 0;
    if (Nm == 0) return;
    if (!A0 || !learned || !keep_idx || !new_idx) fail(FGGC_EINVAL, "NULL array");
    Guard lock(ctx);
    need_device({A0, learned, keep_idx, new_idx});
    hipStream_t s = (hipStream_t)stream;
    // the pre-pass scratch: the max reduction's partials, then the two counts
    double *scr = (double *)ctx->dev_scan;
    int64_t *counts = (int64_t *)(scr + learn_scratch_bytes() / 8);
    static_assert(sizeof(long long) == sizeof(int64_t), "count size");
    if (learn_scratch_bytes() + 16 > packet_scan_bytes() + 256) fail(FGGC_EDEVICE, "internal: scratch too small");
    launch_learn_select(Nm, A0, prune, learned, keep_idx, new_idx, scr, counts, s);
    FGGC_HIP(hipMemcpyAsync(ctx->host_scan, counts, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, s));
    FGGC_HIP(hipStreamSynchronize(s));
    *n_keep = ctx->host_scan[0];
    *n_new = ctx->host_scan[1];
  });
}

int fggc_learn_start(fggc_ctx *ctx, int32_t d, int64_t Nm, int64_t n, const int64_t *idx, const double *qm,
                     const double *pm, double *Q, double *P, double *S, double *A, void *stream) {
  return guarded("fggc_learn_start", [&] {
    if (!ctx) fail(FGGC_EINVAL, "ctx is NULL");
    check_learn(d, Nm, n);
    if (n == 0) return;
    if (!idx || !qm || !pm || !Q || !P || !S || !A) fail(FGGC_EINVAL, "NULL array");
    Guard lock(ctx);
    need_device({idx, qm, pm, Q, P, S, A});
    launch_learn_start(d, Nm, n, idx, qm, pm, Q, P, S, A, (hipStream_t)stream);
  });
}

int fggc_learn_store(fggc_ctx *ctx, int32_t d, int64_t Nm, int64_t n, const int64_t *idx, const double *Q,
                     const double *P, const double *S, const double *A, double *Qf, double *Pf, double *Sf,
                     double *ratio, void *stream) {
  return guarded("fggc_learn_store", [&] {
    if (!ctx) fail(FGGC_EINVAL, "ctx is NULL");
    check_learn(d, Nm, n);
    if (n == 0) return;
    if (!idx || !Q || !P || !S || !A || !Qf || !Pf || !Sf || !ratio) fail(FGGC_EINVAL, "NULL array");
    Guard lock(ctx);
    need_device({idx, Q, P, S, A, Qf, Pf, Sf, ratio});
    launch_learn_store(d, Nm, n, idx, Q, P, S, A, Qf, Pf, Sf, ratio, (hipStream_t)stream);
  });
}

int fggc_learn_packets(fggc_ctx *ctx, int32_t d, int64_t Nm, int64_t n, const int64_t *idx, const double *Qf,
                       const double *Pf, const double *Sf, const double *ratio, const double *A0, double *Q,
                       double *P, double *S, double *a, void *stream) {
  return guarded("fggc_learn_packets", [&] {
    if (!ctx) fail(FGGC_EINVAL, "ctx is NULL");
    check_learn(d, Nm, n);
    if (n == 0) return;
    if (!idx || !Qf || !Pf || !Sf || !ratio || !A0 || !Q || !P || !S || !a) fail(FGGC_EINVAL, "NULL array");
    Guard lock(ctx);
    need_device({idx, Qf, Pf, Sf, ratio, A0, Q, P, S, a});
    launch_learn_packets(d, Nm, n, idx, Qf, Pf, Sf, ratio, A0, Q, P, S, a, (hipStream_t)stream);
  });
}

int fggc_cell_box(fggc_ctx *ctx, const fggc_packets *pk, const fggc_strategy *st,
                  int64_t *slice_lo, int64_t *slice_n, void *stream) {
  return guarded("fggc_cell_box", [&] {
    if (!ctx || !pk || !slice_lo || !slice_n) fail(FGGC_EINVAL, "NULL argument");
    if (pk->d < 1 || pk->d > 3) fail(FGGC_EINVAL, "packets->d must be 1, 2 or 3");
    check_packets(pk, pk->d);
    check_strategy(st, pk->d);
    Guard lock(ctx);
    hipStream_t s = (hipStream_t)stream;
    WsUse wsu(ctx, s);
    const bool host_in = packets_on_host(*pk);
    fggc_packets dpk = *pk;
    ctx->ws.reserve(staging_bytes(*pk, host_in, 0, false) + 256, ctx->budget);
    if (host_in) dpk = stage_packets(*pk, (char *)ctx->ws.take((size_t)pk->N * (2 * pk->d + 3) * 8), s);
    prepass(ctx, dpk, st->dp, s);
    int64_t lo[3], n[3];
    cell_box(ctx, dpk, *st, lo, n);
    for (int k = 0; k < pk->d; ++k) {
      slice_lo[k] = lo[k];
      slice_n[k] = n[k];
    }
  });
}

int fggc_coefficients(fggc_ctx *ctx, const fggc_packets *pk, double eps, const fggc_strategy *st, double scale,
                      double *c_out, int32_t *cell_out, void *stream) {
  return guarded("fggc_coefficients", [&] {
    if (!ctx || !pk || !st || !c_out || !cell_out) fail(FGGC_EINVAL, "NULL argument");
    if (pk->d < 1 || pk->d > 3) fail(FGGC_EINVAL, "packets->d must be 1, 2 or 3");
    const int d = pk->d;
    check_packets(pk, d);
    check_eps(eps);
    check_strategy(st, d);
    if (!std::isfinite(scale)) fail(FGGC_EINVAL, "scale must be finite");
    if (d == 3 && st->nq * st->np > 8) fail(FGGC_EUNSUPPORTED, "3D strategies need nq * np <= 8");
    if (pk->N == 0) return;
    Guard lock(ctx);
    hipStream_t s = (hipStream_t)stream;
    WsUse wsu(ctx, s);
    if (packets_on_host(*pk) || !device_accessible(c_out) || !device_accessible(cell_out))
      fail(FGGC_EINVAL, "packets and outputs must be device memory");
    const Plan plan = plan_for(*st, d, eps);
    GridGeom g{};
    g.d = d;
    for (int k = 0; k < 3; ++k) {
      g.n[k] = 1;
      g.dx[k] = 1.0;
    }
    const int64_t zero[3] = {0, 0, 0}, one[3] = {1, 1, 1};
    fggc_packets dpk = *pk;
    FggcArgs fa{};
    fill_fggc_args(fa, &dpk, eps, g, *st, scale, FGGC_FP64, plan.host, zero, one);
    fa.lsq_dev = plan.dev;
    prepass(ctx, dpk, st->dp, s);
    ctx->ws.reserve(fggc_coefficients_workspace_bytes(fa), ctx->budget);
    launch_fggc_coefficients(fa, c_out, cell_out, ctx->ws, s);
  });
}

int fggc_cells(fggc_ctx *ctx, const fggc_packets *pk, double eps, const fggc_strategy *st,
               double scale, int precision, const int64_t *slice_lo, const int64_t *slice_n,
               void *cells_out, size_t cells_bytes, void *stream) {
  return guarded("fggc_cells", [&] {
    if (!ctx || !pk || !slice_lo || !slice_n || !cells_out) fail(FGGC_EINVAL, "NULL argument");
    if (pk->d < 1 || pk->d > 3) fail(FGGC_EINVAL, "packets->d must be 1, 2 or 3");
    const int d = pk->d;
    check_packets(pk, d);
    check_eps(eps);
    check_strategy(st, d);
    if (!std::isfinite(scale)) fail(FGGC_EINVAL, "scale must be finite");
    if (precision != FGGC_FP32 && precision != FGGC_FP64) fail(FGGC_EINVAL, "bad precision");
    Guard lock(ctx);
    hipStream_t s = (hipStream_t)stream;
    WsUse wsu(ctx, s);
    int64_t slo[3] = {0, 0, 0}, sn[3] = {1, 1, 1};
    for (int k = 0; k < d; ++k) {
      slo[k] = slice_lo[k];
      sn[k] = slice_n[k];
      if (sn[k] < 1) fail(FGGC_EINVAL, "slice_n must be >= 1");
    }
    const size_t bytes = (size_t)(prod3(sn, d) * prod3(st->Nq, d)) * (precision == FGGC_FP64 ? 16 : 8);
    if (cells_bytes < bytes) fail(FGGC_EINVAL, "cells_out too small");
    const bool host_in = packets_on_host(*pk);
    const bool host_out = !device_accessible(cells_out);
    fggc_packets dpk = *pk;
    const Plan plan = plan_for(*st, d, eps);
    const DimLsq *lsq = plan.host;
    GridGeom g{};
    g.d = d;
    for (int k = 0; k < 3; ++k) {
      g.n[k] = 1;
      g.dx[k] = 1.0;
    }
    FggcArgs fa{};
    fill_fggc_args(fa, &dpk, eps, g, *st, scale, precision, lsq, slo, sn);
    fa.lsq_dev = plan.dev;
    ctx->ws.reserve(staging_bytes(*pk, host_in, bytes, host_out) + fggc_cells_workspace_bytes(fa),
                    ctx->budget);
    if (host_in) dpk = stage_packets(*pk, (char *)ctx->ws.take((size_t)pk->N * (2 * d + 3) * 8), s);
    void *cells = host_out ? ctx->ws.take(bytes) : cells_out;
    prepass(ctx, dpk, st->dp, s);
    // the box must hold every p-cell the packets touch
    if (dpk.N > 0) {
      int64_t lo[3], n[3];
      cell_box(ctx, dpk, *st, lo, n);
      for (int k = 0; k < d; ++k)
        if (lo[k] < slo[k] || lo[k] + n[k] > slo[k] + sn[k])
          fail(FGGC_EINVAL, "slice box does not contain the packets' p-cells");
    }
    launch_fggc_cells(fa, cells, ctx->ws, s);
    if (host_out) {
      FGGC_HIP(hipMemcpyAsync(cells_out, cells, bytes, hipMemcpyDeviceToHost, s));
      FGGC_HIP(hipStreamSynchronize(s));
    } else if (host_in) {
      FGGC_HIP(hipStreamSynchronize(s));
    }
  });
}

int fggc_reconstruct(fggc_ctx *ctx, const fggc_packets *pk, double eps, const fggc_grid *grid,
                     const fggc_strategy *st, double scale, int precision, void *u_out,
                     void *stream) {
  return guarded("fggc_reconstruct", [&] {
    if (!ctx) fail(FGGC_EINVAL, "ctx is NULL");
    GridGeom g = check_grid(grid);
    const int d = g.d;
    check_packets(pk, d);
    check_eps(eps);
    check_strategy(st, d);
    if (!std::isfinite(scale)) fail(FGGC_EINVAL, "scale must be finite");
    if (precision != FGGC_FP32 && precision != FGGC_FP64) fail(FGGC_EINVAL, "bad precision");
    if (!u_out) fail(FGGC_EINVAL, "u_out is NULL");
    const int64_t maxM = d == 1 ? (precision == FGGC_FP64 ? 8192 : 16384) : 4096;
    for (int k = 0; k < d; ++k)
      if (!is_fft_size(g.n[k]) || g.n[k] > maxM)
        fail(FGGC_EUNSUPPORTED, "FGGC needs grid sizes 2^a 3^b 5^c in [2, " + std::to_string(maxM) + "]");
    Guard lock(ctx);
    hipStream_t s = (hipStream_t)stream;
    WsUse wsu(ctx, s);
    const int64_t npts = prod3(g.n, d);
    const size_t out_bytes = (size_t)npts * (precision == FGGC_FP64 ? 16 : 8);
    const bool host_in = packets_on_host(*pk);
    const bool host_out = !device_accessible(u_out);
    fggc_packets dpk = *pk;
    // stage, validate and find the p-cell box (one synchronisation)
    ctx->ws.reserve(staging_bytes(*pk, host_in, out_bytes, host_out) + 256, ctx->budget);
    if (host_in) dpk = stage_packets(*pk, (char *)ctx->ws.take((size_t)pk->N * (2 * d + 3) * 8), s);
    if (dpk.N == 0) {
      void *u = host_out ? ctx->ws.take(out_bytes) : u_out;
      launch_zero(u, out_bytes, s);
      if (host_out) FGGC_HIP(hipMemcpyAsync(u_out, u, out_bytes, hipMemcpyDeviceToHost, s));
      FGGC_HIP(hipStreamSynchronize(s));
      return;
    }
    prepass(ctx, dpk, st->dp, s);
    int64_t slo[3], sn[3];
    cell_box(ctx, dpk, *st, slo, sn);
    const Plan plan = plan_for(*st, d, eps);
    FggcArgs fa{};
    fill_fggc_args(fa, &dpk, eps, g, *st, scale, precision, plan.host, slo, sn);
    fa.lsq_dev = plan.dev;
    // the staged packets must survive the re-reservation: reserve everything once more
    const size_t stage_b = staging_bytes(*pk, host_in, out_bytes, host_out);
    const size_t need = stage_b + fggc_workspace_bytes(fa);
    if (need > ctx->ws.capacity()) {
      if (need > ctx->budget)
        fail(FGGC_EBUDGET, "FGGC needs " + std::to_string(need) + " bytes, budget is " +
                               std::to_string(ctx->budget));
      ctx->ws.reserve(need, ctx->budget);
      if (host_in) dpk = stage_packets(*pk, (char *)ctx->ws.take((size_t)pk->N * (2 * d + 3) * 8), s);
    } else {
      ctx->ws.reset();
      if (host_in) (void)ctx->ws.take((size_t)pk->N * (2 * d + 3) * 8);
    }
    fa.pk = &dpk;
    fa.u = host_out ? ctx->ws.take(out_bytes) : u_out;
    fa.prof = ctx->profiling ? &ctx->prof : nullptr;
    if (!host_in && !host_out && !ctx->profiling && plan.dev && fggc_graph_safe(fa)) {
      std::vector<int64_t> key = {1, d, precision, dpk.N, dbits(eps), dbits(scale),
                                  (int64_t)(uintptr_t)dpk.Q, (int64_t)(uintptr_t)dpk.P,
                                  (int64_t)(uintptr_t)dpk.S, (int64_t)(uintptr_t)dpk.a,
                                  (int64_t)(uintptr_t)u_out, (int64_t)(uintptr_t)plan.dev};
      for (int k = 0; k < 3; ++k) {
        key.push_back(g.n[k]);
        key.push_back(slo[k]);
        key.push_back(sn[k]);
        key.push_back(st->Nq[k]);
        key.push_back(dbits(st->dp[k]));
      }
      run_cached(ctx, std::move(key), s, [&](hipStream_t ls) { launch_fggc(fa, ctx->ws, ls); });
    } else {
      launch_fggc(fa, ctx->ws, s);
    }
    if (host_out) {
      FGGC_HIP(hipMemcpyAsync(u_out, fa.u, out_bytes, hipMemcpyDeviceToHost, s));
      FGGC_HIP(hipStreamSynchronize(s));
    } else if (host_in) {
      FGGC_HIP(hipStreamSynchronize(s));
    }
  });
}

int fggc_profile(fggc_ctx *ctx, int enable) {
  return guarded("fggc_profile", [&] {
    if (!ctx) fail(FGGC_EINVAL, "ctx is NULL");
    Guard lock(ctx);
    ctx->profiling = enable != 0;
    if (enable < 0 || enable > 1) fail(FGGC_EINVAL, "enable must be 0 or 1");
    ctx->prof.reset();
  });
}

int fggc_stage_time(fggc_ctx *ctx, const char *stage, double *total_ms, int64_t *count) {
  return guarded("fggc_stage_time", [&] {
    if (!ctx || !stage || !total_ms || !count) fail(FGGC_EINVAL, "NULL argument");
    Guard lock(ctx);
    ctx->prof.query(stage, total_ms, count);
  });
}

int fggc_fft(fggc_ctx *ctx, int d, const int64_t *n, int64_t batch, int direction, int precision,
             void *data, void *stream) {
  return guarded("fggc_fft", [&] {
    if (!ctx || !n || !data) fail(FGGC_EINVAL, "NULL argument");
    if (d < 1 || d > 3) fail(FGGC_EINVAL, "d must be 1, 2 or 3");
    if (batch < 0) fail(FGGC_EINVAL, "batch must be >= 0");
    if (direction != -1 && direction != 1) fail(FGGC_EINVAL, "direction must be -1 or +1");
    if (precision != FGGC_FP32 && precision != FGGC_FP64) fail(FGGC_EINVAL, "bad precision");
    const int64_t maxn = precision == FGGC_FP64 ? 8192 : 16384;
    for (int k = 0; k < d; ++k)
      if (!is_fft_size(n[k]) || n[k] > maxn || (d > 1 && !is_pow2(n[k]) && n[k] > 4096))
        fail(FGGC_EUNSUPPORTED, "FFT sizes must be 2^a 3^b 5^c in [2, " + std::to_string(maxn) +
                                    "] (at most 4096 unless a power of two, in two and three dimensions)");
    Guard lock(ctx);
    hipStream_t s = (hipStream_t)stream;
    WsUse wsu(ctx, s);
    if (!device_accessible(data)) fail(FGGC_EINVAL, "fggc_fft needs device memory");
    if (batch == 0) return;
    ctx->ws.reserve(fft_workspace_bytes(d, n, precision, batch), ctx->budget);
    launch_fft(d, n, batch, direction, precision, data, ctx->ws, s,
               ctx->profiling ? &ctx->prof : nullptr, "fft");
  });
}

}  // extern "C"
