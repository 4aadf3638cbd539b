// Continuous-batching reconstruction service behind fggc_server_*.
//
// Requests are validated and sized at submit (host packets are copied into
// server-owned memory; device packets are referenced in place and scanned on
// the device), queued in arrival order, and handed to executor slots as soon
// as a slot is idle and the request's memory fits the budget (admission.h).
// Each slot is a persistent worker thread with its own non-blocking stream
// and workspace, so admitted requests overlap on the device.  A slot runs a
// request's kernel pipeline eagerly the first time its shape is seen, captures
// it into a hipGraph the second time, and replays the graph after that; the
// packet count is padded to a quarter-octave bucket with zero-amplitude
// packets and the p-cell box is aligned, so shapes repeat across requests.
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <memory>
#include <set>
#include <thread>
#include <unordered_map>

#include "admission.h"
#include "common.h"

namespace fggc {
namespace {

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
  fggc_ticket id = 0;
  bool use_fggc = false;
  fggc_strategy st{};
  GridGeom g{};
  int d = 1;
  double eps = 0, scale = 1, R = 0;
  int precision = FGGC_FP32;
  int64_t N = 0, Npad = 0;
  bool host_in = false;
  std::vector<double> hbuf;  // host copy: Q[d][N], P[d][N], S[N], a[2N]
  fggc_packets dev{};        // caller's device arrays (host_in == false)
  void *u_out = nullptr;
  bool host_out = true;
  size_t out_bytes = 0;
  int64_t slo[3] = {0, 0, 0}, sn[3] = {1, 1, 1};
  size_t need = 0;
  double t_submit = 0, t_done = 0;
  int status = FGGC_OK;
  bool done = false;
  std::string err;
  std::vector<int64_t> key;  // shape key (filled at submit)
};

// Everything a captured pipeline depends on besides the slot's buffers.
struct ShapeKey {
  std::vector<int64_t> v;
  bool operator<(const ShapeKey &o) const { return v < o.v; }
};

int64_t bits(double x) {
  int64_t b;
  std::memcpy(&b, &x, 8);
  return b;
}

ShapeKey shape_key(const Request &r) {
  ShapeKey k;
  k.v = {r.use_fggc, r.d, r.precision, r.Npad, bits(r.eps), bits(r.scale), bits(r.R)};
  for (int i = 0; i < 3; ++i) k.v.push_back(r.g.n[i]);
  if (r.use_fggc) {
    for (int i = 0; i < 3; ++i) {
      k.v.push_back(r.st.Nq[i]);
      k.v.push_back(bits(r.st.dp[i]));
      k.v.push_back(r.slo[i]);
      k.v.push_back(r.sn[i]);
    }
    k.v.push_back(r.st.nq);
    k.v.push_back(r.st.np);
    for (int i = 0; i < 8; ++i) {
      k.v.push_back(r.st.dq_off[i]);
      k.v.push_back(r.st.dp_off[i]);
    }
    k.v.push_back(bits(r.st.cutoff));
  }
  return k;
}

size_t packet_bytes(int d, int64_t N) { return (size_t)N * (2 * d + 3) * 8; }

}  // namespace
}  // namespace fggc

using namespace fggc;

struct fggc_server;

namespace fggc {
namespace {

// cached executable graphs per slot: a slot may serve every shape of a stream
// (the scheduler reuses the smallest slot that fits), and an LRU smaller than
// the set of shapes in rotation misses on every request
constexpr int kMaxGraphs = 128;

struct Slot {
  int idx = 0;
  hipStream_t stream = nullptr;
  Workspace ws;
  size_t cap = 0;     // bytes held (as seen by the scheduler)
  size_t limit = 0;   // bytes the current request may grow the slot to
  bool busy = false;
  bool release = false;
  DimLsq *lsq = nullptr;  // pinned host copy of the current plan (graph memcpy source)
  std::shared_ptr<Request> cur;
  std::list<std::pair<ShapeKey, hipGraphExec_t>> graphs;  // most recent first (worker only)
  std::set<ShapeKey> cached;  // keys of `graphs`, read by the scheduler (under the server lock)
  std::thread th;
};

}  // namespace
}  // namespace fggc

struct fggc_server {
  fggc_ctx *ctx = nullptr;
  int device = 0;
  size_t budget = 0;
  std::mutex mu;
  std::condition_variable cv;  // work for slots, completions for waiters
  std::deque<std::shared_ptr<Request>> queue;
  std::unordered_map<fggc_ticket, std::shared_ptr<Request>> reqs;
  std::vector<std::unique_ptr<Slot>> slots;
  bool stopping = false;
  fggc_ticket next_id = 1;
  // submit-time scan of device-resident packets
  std::mutex intake_mu;
  hipStream_t intake = nullptr;
  long long *dev_scan = nullptr, *host_scan = nullptr;
  // statistics
  std::vector<double> lat;
  int64_t packets_done = 0, completed = 0;
  double t_first = -1, t_last = 0;
  int64_t n_eager = 0, n_capture = 0, n_replay = 0;
  std::map<ShapeKey, int> seen;  // sightings of each shape, over all slots

  void dispatch();  // under mu
  void worker(Slot *sl);
  void run(Slot *sl, Request &r);
  void finish(Request &r, int status, const std::string &msg);  // under mu
};

void fggc_server::finish(Request &r, int status, const std::string &msg) {
  r.status = status;
  r.err = msg;
  r.done = true;
  r.t_done = now_s();
  if (status == FGGC_OK) {
    lat.push_back(r.t_done - r.t_submit);
    packets_done += r.N;
    completed += 1;
    t_last = std::max(t_last, r.t_done);
  }
}

void fggc_server::dispatch() {
  while (!queue.empty()) {
    auto r = queue.front();
    // an idle slot that already holds this shape's graph takes it
    ShapeKey key;
    key.v = r->key;
    Slot *hit = nullptr;
    for (auto &s : slots)
      if (!s->busy && !s->cur && s->cap >= r->need && s->cached.count(key)) {
        hit = s.get();
        break;
      }
    if (hit) {
      hit->cur = r;
      hit->busy = true;
      hit->limit = hit->cap;
      queue.pop_front();
      cv.notify_all();
      continue;
    }
    std::vector<SlotState> st;
    for (auto &s : slots) st.push_back({s->cap, s->busy || s->cur != nullptr});
    Admission a = plan_admission(st, r->need, budget);
    if (a.slot < 0) return;
    for (int j : a.release) {
      Slot *s = slots[j].get();
      s->release = true;  // its worker frees the memory before anything else
      s->cap = 0;
      s->busy = true;
      cv.notify_all();
    }
    Slot *s = slots[a.slot].get();
    s->cur = r;
    s->busy = true;
    s->limit = a.limit;
    s->cap = std::max(s->cap, r->need);
    queue.pop_front();
    cv.notify_all();
  }
}

namespace {
// drop a slot's graphs (caller does not hold the server lock)
void clear_graphs(std::mutex &mu, Slot *sl) {
  for (auto &g : sl->graphs) (void)hipGraphExecDestroy(g.second);
  sl->graphs.clear();
  std::lock_guard<std::mutex> lk(mu);
  sl->cached.clear();
}
}  // namespace

// Capture the pipeline that `enqueue` launches on the slot's stream into an
// executable graph at the front of the slot's cache.  Runs on the second
// sighting of a shape, so twiddle tables and kernel attributes already exist.
// A shape that cannot be captured is run eagerly from then on.
template <class F>
bool capture(std::mutex &mu, std::map<ShapeKey, int> &seen, Slot *sl, const ShapeKey &key, F &&enqueue) {
  hipStream_t s = sl->stream;
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    std::lock_guard<std::mutex> lk(mu);
    seen[key] = -(1 << 30);
    return false;
  }
  bool ok = true;
  try {
    enqueue();
  } catch (...) {
    ok = false;
  }
  if (hipStreamEndCapture(s, &graph) != hipSuccess) ok = false;
  hipGraphExec_t exec = nullptr;
  if (ok && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) ok = false;
  if (graph) (void)hipGraphDestroy(graph);
  std::lock_guard<std::mutex> lk(mu);
  if (!ok) {
    (void)hipGetLastError();
    if (exec) (void)hipGraphExecDestroy(exec);
    seen[key] = -(1 << 30);
    return false;
  }
  if ((int)sl->graphs.size() >= kMaxGraphs) {
    (void)hipGraphExecDestroy(sl->graphs.back().second);
    sl->cached.erase(sl->graphs.back().first);
    sl->graphs.pop_back();
  }
  sl->graphs.emplace_front(key, exec);
  sl->cached.insert(key);
  return true;
}

void fggc_server::run(Slot *sl, Request &r) {
  hipStream_t s = sl->stream;
  if (r.need > sl->ws.capacity()) {
    clear_graphs(mu, sl);
    FGGC_HIP(hipStreamSynchronize(s));
    sl->ws.reserve(r.need, std::max(r.need, sl->limit));
  } else {
    sl->ws.reset();
  }
  // slot buffers: padded packets, output, then the pipeline's own scratch
  const int d = r.d;
  double *pk = (double *)sl->ws.take(packet_bytes(d, r.Npad));
  double *Q = pk, *P = Q + (size_t)d * r.Npad, *S = P + (size_t)d * r.Npad, *A = S + r.Npad;
  void *u = sl->ws.take(r.out_bytes);
  const size_t dN = (size_t)d * r.N * 8, N8 = (size_t)r.N * 8;
  if (r.host_in) {
    const double *h = r.hbuf.data();
    for (int k = 0; k < d; ++k) {
      FGGC_HIP(hipMemcpyAsync(Q + (size_t)k * r.Npad, h + (size_t)k * r.N, N8, hipMemcpyHostToDevice, s));
      FGGC_HIP(hipMemcpyAsync(P + (size_t)k * r.Npad, h + dN / 8 + (size_t)k * r.N, N8,
                              hipMemcpyHostToDevice, s));
    }
    FGGC_HIP(hipMemcpyAsync(S, h + 2 * dN / 8, N8, hipMemcpyHostToDevice, s));
    FGGC_HIP(hipMemcpyAsync(A, h + 2 * dN / 8 + r.N, 2 * N8, hipMemcpyHostToDevice, s));
  } else {
    for (int k = 0; k < d; ++k) {
      FGGC_HIP(hipMemcpyAsync(Q + (size_t)k * r.Npad, r.dev.Q + (size_t)k * r.N, N8,
                              hipMemcpyDeviceToDevice, s));
      FGGC_HIP(hipMemcpyAsync(P + (size_t)k * r.Npad, r.dev.P + (size_t)k * r.N, N8,
                              hipMemcpyDeviceToDevice, s));
    }
    FGGC_HIP(hipMemcpyAsync(S, r.dev.S, N8, hipMemcpyDeviceToDevice, s));
    FGGC_HIP(hipMemcpyAsync(A, r.dev.a, 2 * N8, hipMemcpyDeviceToDevice, s));
  }
  launch_pad_packets(d, r.N, r.Npad, Q, P, S, A, s);
  fggc_packets dpk{};
  dpk.d = d;
  dpk.N = r.Npad;
  dpk.Q = Q;
  dpk.P = P;
  dpk.S = S;
  dpk.a = A;

  FggcArgs fa{};
  DirectArgs da{};
  if (r.use_fggc) {
    const Plan plan = plan_for(r.st, d, r.eps);
    // the host plan lives in the slot's pinned copy: a captured graph's
    // memcpy node reads it there when the device plan is not cached
    std::memcpy(sl->lsq, plan.host, sizeof(plan.host));
    fill_fggc_args(fa, &dpk, r.eps, r.g, r.st, r.scale, r.precision, sl->lsq, r.slo, r.sn);
    fa.lsq_dev = plan.dev;
    fa.u = u;
  } else {
    da.pk = &dpk;
    da.eps = r.eps;
    da.R = r.R;
    da.scale = r.scale;
    da.g = r.g;
    for (int k = 0; k < 3; ++k) {
      da.box.lo[k] = 0;
      da.box.n[k] = r.g.n[k];
    }
    da.precision = r.precision;
    da.u = u;
  }
  const size_t mark = sl->ws.mark();
  auto enqueue = [&] {
    sl->ws.rewind(mark);
    if (r.use_fggc) launch_fggc(fa, sl->ws, s);
    else launch_direct(da, sl->ws, s);
  };
  ShapeKey key;
  key.v = r.key;
  auto sighting = [&](const ShapeKey &k) {
    std::lock_guard<std::mutex> lk(mu);
    return ++seen[k];
  };
  auto it = sl->graphs.begin();
  for (; it != sl->graphs.end(); ++it)
    if (!(it->first < key) && !(key < it->first)) break;
  const bool graph_ok = r.use_fggc ? fggc_graph_safe(fa) : direct_graph_safe(da);
  if (!graph_ok) {
    enqueue();
    std::lock_guard<std::mutex> lk(mu);
    n_eager += 1;
  } else if (it != sl->graphs.end()) {
    sl->graphs.splice(sl->graphs.begin(), sl->graphs, it);
    FGGC_HIP(hipGraphLaunch(sl->graphs.front().second, s));
    std::lock_guard<std::mutex> lk(mu);
    n_replay += 1;
  } else if (sighting(key) >= 2 && capture(mu, seen, sl, key, enqueue)) {
    FGGC_HIP(hipGraphLaunch(sl->graphs.front().second, s));
    std::lock_guard<std::mutex> lk(mu);
    n_capture += 1;
  } else {
    enqueue();
    std::lock_guard<std::mutex> lk(mu);
    n_eager += 1;
  }
  FGGC_HIP(hipMemcpyAsync(r.u_out, u, r.out_bytes,
                          r.host_out ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice, s));
  FGGC_HIP(hipStreamSynchronize(s));
}

void fggc_server::worker(Slot *sl) {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv.wait(lk, [&] { return stopping || sl->cur != nullptr || sl->release; });
    if (sl->release) {
      lk.unlock();
      clear_graphs(mu, sl);
      (void)hipStreamSynchronize(sl->stream);
      sl->ws.release();
      lk.lock();
      sl->release = false;
      if (!sl->cur) sl->busy = false;
      dispatch();
      cv.notify_all();
      continue;
    }
    if (!sl->cur) {
      if (stopping) return;
      continue;
    }
    auto r = sl->cur;
    lk.unlock();
    int status = FGGC_OK;
    std::string msg;
    try {
      run(sl, *r);
    } catch (const Error &e) {
      status = e.code;
      msg = e.msg;
    } catch (const std::exception &e) {
      status = FGGC_EDEVICE;
      msg = e.what();
    } catch (...) {
      status = FGGC_EDEVICE;
      msg = "unknown internal error";
    }
    if (status != FGGC_OK) {
      // leave the slot clean: drop whatever the stream still holds
      (void)hipStreamSynchronize(sl->stream);
      (void)hipGetLastError();
    }
    lk.lock();
    sl->cap = sl->ws.capacity();
    r->hbuf.clear();
    r->hbuf.shrink_to_fit();
    finish(*r, status, msg);
    sl->cur.reset();
    sl->busy = false;
    dispatch();
    cv.notify_all();
  }
}

namespace fggc {
namespace {

// Host packets: copy into the request and scan them in one pass
// (NaN/Inf, |Q|,|P| <= 1e9, and the min/max momentum per dimension).
void intake_host(Request &r, const fggc_packets &pk, double pmin[3], double pmax[3]) {
  const int d = r.d;
  const int64_t N = r.N;
  r.hbuf.resize((size_t)N * (2 * d + 3));
  double *h = r.hbuf.data();
  bool bad = false;
  for (int k = 0; k < d; ++k) {
    const double *q = pk.Q + (size_t)k * N, *p = pk.P + (size_t)k * N;
    double *hq = h + (size_t)k * N, *hp = h + (size_t)(d + k) * N;
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t j = 0; j < N; ++j) {
      const double x = q[j], y = p[j];
      hq[j] = x;
      hp[j] = y;
      bad |= !(std::fabs(x) <= 1e9) || !(std::fabs(y) <= 1e9);
      lo = y < lo ? y : lo;
      hi = y > hi ? y : hi;
    }
    pmin[k] = lo;
    pmax[k] = hi;
  }
  std::memcpy(h + (size_t)2 * d * N, pk.S, (size_t)N * 8);
  std::memcpy(h + (size_t)(2 * d + 1) * N, pk.a, (size_t)N * 16);
  const double *sa = h + (size_t)2 * d * N;
  for (int64_t j = 0; j < 3 * N; ++j) bad |= !std::isfinite(sa[j]);
  if (bad) fail(FGGC_EINVAL, "packets with NaN/Inf in Q, P, S or a, or |Q| or |P| above 1e9");
}

int64_t cell_of(double v, double dp) {
  // the same split as the device: floor of the IEEE quotient, a fraction
  // that rounds to 1 moving to the next cell
  const double x = v / dp, fl = std::floor(x);
  int64_t i = (int64_t)fl;
  if (x - fl >= 1.0) i += 1;
  return i;
}

}  // namespace
}  // namespace fggc

extern "C" {

int fggc_server_create(fggc_ctx *ctx, int n_streams, fggc_server **out) {
  return guarded("fggc_server_create", [&] {
    if (!out) fail(FGGC_EINVAL, "out is NULL");
    *out = nullptr;
    if (!ctx) fail(FGGC_EINVAL, "ctx is NULL");
    if (n_streams < 1 || n_streams > 8) fail(FGGC_EINVAL, "n_streams must be in [1, 8]");
    FGGC_HIP(hipSetDevice(ctx->device));
    auto srv = std::make_unique<fggc_server>();
    srv->ctx = ctx;
    srv->device = ctx->device;
    srv->budget = ctx->budget;
    FGGC_HIP(hipStreamCreateWithFlags(&srv->intake, hipStreamNonBlocking));
    FGGC_HIP(hipMalloc((void **)&srv->dev_scan, packet_scan_bytes() + 256));
    FGGC_HIP(hipHostMalloc((void **)&srv->host_scan, 256, hipHostMallocDefault));
    for (int i = 0; i < n_streams; ++i) {
      auto sl = std::make_unique<Slot>();
      sl->idx = i;
      FGGC_HIP(hipStreamCreateWithFlags(&sl->stream, hipStreamNonBlocking));
      sl->ws.set_stream(sl->stream);
      FGGC_HIP(hipHostMalloc((void **)&sl->lsq, 3 * sizeof(DimLsq), hipHostMallocDefault));
      srv->slots.push_back(std::move(sl));
    }
    fggc_server *raw = srv.get();
    for (auto &sl : srv->slots) {
      Slot *p = sl.get();
      p->th = std::thread([raw, p] { raw->worker(p); });
    }
    *out = srv.release();
  });
}

int fggc_server_submit(fggc_server *srv, const fggc_packets *pk, double eps, const fggc_grid *grid,
                       const fggc_strategy *st, double scale, int precision, void *u_out,
                       fggc_ticket *ticket) {
  return guarded("fggc_server_submit", [&] {
    if (!srv || !ticket) fail(FGGC_EINVAL, "NULL argument");
    *ticket = 0;
    GridGeom g = check_grid(grid);
    const int d = g.d;
    check_packets(pk, d);
    check_eps(eps);
    if (!std::isfinite(scale)) fail(FGGC_EINVAL, "scale must be finite");
    if (precision != FGGC_FP32 && precision != FGGC_FP64) fail(FGGC_EINVAL, "bad precision");
    if (!u_out) fail(FGGC_EINVAL, "u_out is NULL");
    if (pk->N > ((int64_t)1 << 30)) fail(FGGC_EINVAL, "served requests hold at most 2^30 packets");
    FGGC_HIP(hipSetDevice(srv->device));
    auto r = std::make_shared<Request>();
    r->d = d;
    r->g = g;
    r->eps = eps;
    r->scale = scale;
    r->precision = precision;
    r->N = pk->N;
    r->Npad = pk->N > 0 ? padded_count(pk->N) : 0;
    r->u_out = u_out;
    r->host_out = !device_accessible(u_out);
    r->out_bytes = (size_t)prod3(g.n, d) * (precision == FGGC_FP64 ? 16 : 8);
    r->use_fggc = st != nullptr;
    if (st) {
      check_strategy(st, d);
      r->st = *st;
      const int64_t maxM = d == 1 ? (precision == FGGC_FP64 ? 8192 : 16384) : 4096;
      for (int k = 0; k < d; ++k)
        if (!is_fft_size(g.n[k]) || g.n[k] > maxM)
          fail(FGGC_EUNSUPPORTED, "FGGC needs grid sizes 2^a 3^b 5^c in [2, " + std::to_string(maxM) + "]");
    } else {
      r->R = 6.0 * std::sqrt(eps);
      if (!(r->R < kPi)) fail(FGGC_EINVAL, "eps too large for the direct-sum window 6 sqrt(eps) < pi");
    }
    // validate, copy or scan, and find the momentum range
    double pmin[3] = {0, 0, 0}, pmax[3] = {0, 0, 0};
    if (r->N > 0) {
      const int ndev = (int)device_accessible(pk->Q) + (int)device_accessible(pk->P) +
                       (int)device_accessible(pk->S) + (int)device_accessible(pk->a);
      if (ndev != 0 && ndev != 4) fail(FGGC_EINVAL, "packet arrays must be all host or all device");
      r->host_in = ndev == 0;
      if (r->host_in) {
        intake_host(*r, *pk, pmin, pmax);
      } else {
        std::lock_guard<std::mutex> lk(srv->intake_mu);
        long long *o = srv->dev_scan + packet_scan_bytes() / 8;
        launch_packet_scan(*pk, st ? st->dp : nullptr, srv->dev_scan, o, srv->intake);
        FGGC_HIP(hipMemcpyAsync(srv->host_scan, o, 8 * sizeof(long long), hipMemcpyDeviceToHost,
                                srv->intake));
        FGGC_HIP(hipStreamSynchronize(srv->intake));
        if (srv->host_scan[0] != 0)
          fail(FGGC_EINVAL, "packets with NaN/Inf in Q, P, S or a, or |Q| or |P| above 1e9");
        r->dev = *pk;
        if (st)
          for (int k = 0; k < d; ++k) {
            r->slo[k] = srv->host_scan[1 + k];
            r->sn[k] = srv->host_scan[4 + k];  // max cell for now
          }
      }
    }
    size_t need = packet_bytes(d, r->Npad) + align_up(r->out_bytes, 256) + 512;
    if (st && r->N > 0) {
      int mn = st->dp_off[0], mx = st->dp_off[0];
      for (int i = 1; i < st->np; ++i) {
        mn = std::min(mn, st->dp_off[i]);
        mx = std::max(mx, st->dp_off[i]);
      }
      for (int k = 0; k < d; ++k) {
        int64_t lo, hi;
        if (r->host_in) {
          lo = cell_of(pmin[k], st->dp[k]);
          hi = cell_of(pmax[k], st->dp[k]);
        } else {
          lo = r->slo[k];
          hi = r->sn[k];
        }
        r->slo[k] = lo + mn;
        r->sn[k] = hi + mx - r->slo[k] + 1;
        align_box(r->slo[k], r->sn[k], 2);
      }
      fggc_packets shape{};
      shape.d = d;
      shape.N = r->Npad;
      FggcArgs fa{};
      const Plan plan = plan_for(*st, d, eps);  // the layout reads the shift sets from the plan
      fill_fggc_args(fa, &shape, eps, g, *st, scale, precision, plan.host, r->slo, r->sn);
      need += fggc_workspace_bytes(fa);
    } else if (r->N > 0) {
      fggc_packets shape{};
      shape.d = d;
      shape.N = r->Npad;
      DirectArgs da{};
      da.pk = &shape;
      da.eps = eps;
      da.R = r->R;
      da.scale = scale;
      da.g = g;
      for (int k = 0; k < 3; ++k) {
        da.box.lo[k] = 0;
        da.box.n[k] = g.n[k];
      }
      da.precision = precision;
      need += direct_workspace_bytes(da);
    }
    r->need = need;
    r->key = shape_key(*r).v;
    if (need > srv->budget)
      fail(FGGC_EBUDGET, "request needs " + std::to_string(need) + " bytes, budget is " +
                             std::to_string(srv->budget));
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stopping) fail(FGGC_ECANCELLED, "server is shutting down");
    r->id = srv->next_id++;
    r->t_submit = now_s();
    if (srv->t_first < 0) srv->t_first = r->t_submit;
    srv->reqs[r->id] = r;
    *ticket = r->id;
    if (r->N == 0) {
      // nothing to sum: u = 0, written here
      if (r->host_out) std::memset(u_out, 0, r->out_bytes);
      else FGGC_HIP(hipMemset(u_out, 0, r->out_bytes));
      srv->finish(*r, FGGC_OK, "");
      srv->cv.notify_all();
      return;
    }
    srv->queue.push_back(r);
    srv->dispatch();
  });
}

int fggc_server_wait(fggc_server *srv, fggc_ticket ticket, double timeout_s) {
  if (!srv) {
    set_last_error("fggc_server_wait: server is NULL");
    return FGGC_EINVAL;
  }
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) {
    set_last_error("fggc_server_wait: unknown ticket");
    return FGGC_EINVAL;
  }
  auto r = it->second;
  auto pred = [&] { return r->done; };
  if (timeout_s < 0) {
    srv->cv.wait(lk, pred);
  } else if (!srv->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), pred)) {
    set_last_error("fggc_server_wait: timed out");
    return FGGC_ETIMEOUT;
  }
  srv->reqs.erase(ticket);
  if (r->status != FGGC_OK) set_last_error("fggc_server_wait: " + r->err);
  return r->status;
}

int fggc_server_stats(fggc_server *srv, double *p50_s, double *p99_s, double *packets_per_s,
                      int64_t *completed) {
  return guarded("fggc_server_stats", [&] {
    if (!srv || !p50_s || !p99_s || !packets_per_s || !completed) fail(FGGC_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    std::vector<double> v = srv->lat;
    std::sort(v.begin(), v.end());
    // nearest-rank percentiles
    auto pct = [&](double q) {
      if (v.empty()) return 0.0;
      size_t k = (size_t)std::ceil(q * (double)v.size());
      k = std::min(std::max<size_t>(k, 1), v.size());
      return v[k - 1];
    };
    *p50_s = pct(0.50);
    *p99_s = pct(0.99);
    const double span = srv->t_last - srv->t_first;
    *packets_per_s = (srv->completed > 0 && span > 0) ? (double)srv->packets_done / span : 0.0;
    *completed = srv->completed;
  });
}

int fggc_server_counters(fggc_server *srv, int64_t *eager, int64_t *captured, int64_t *replayed) {
  return guarded("fggc_server_counters", [&] {
    if (!srv || !eager || !captured || !replayed) fail(FGGC_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(srv->mu);
    *eager = srv->n_eager;
    *captured = srv->n_capture;
    *replayed = srv->n_replay;
  });
}

int fggc_server_reset_stats(fggc_server *srv) {
  return guarded("fggc_server_reset_stats", [&] {
    if (!srv) fail(FGGC_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->lat.clear();
    srv->packets_done = srv->completed = 0;
    srv->t_first = -1;
    srv->t_last = 0;
    srv->n_eager = srv->n_capture = srv->n_replay = 0;
  });
}

void fggc_server_destroy(fggc_server *srv) {
  if (!srv) return;
  {
    std::unique_lock<std::mutex> lk(srv->mu);
    // queued requests still run; then the workers leave
    srv->cv.wait(lk, [&] {
      if (!srv->queue.empty()) return false;
      for (auto &s : srv->slots)
        if (s->cur || s->release) return false;
      return true;
    });
    srv->stopping = true;
    srv->cv.notify_all();
  }
  for (auto &s : srv->slots)
    if (s->th.joinable()) s->th.join();
  (void)hipSetDevice(srv->device);
  for (auto &s : srv->slots) {
    clear_graphs(srv->mu, s.get());
    if (s->stream) {
      (void)hipStreamSynchronize(s->stream);
      (void)hipStreamDestroy(s->stream);
    }
    if (s->lsq) (void)hipHostFree(s->lsq);
  }
  srv->slots.clear();
  if (srv->intake) (void)hipStreamDestroy(srv->intake);
  if (srv->dev_scan) (void)hipFree(srv->dev_scan);
  if (srv->host_scan) (void)hipHostFree(srv->host_scan);
  delete srv;
}

}  // extern "C"
