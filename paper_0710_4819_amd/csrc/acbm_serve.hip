// acbm_serve.hip -- a request loop for frame-pair motion estimation.
//
// Each video stream keeps its reference frame and its previous motion field
// on the device, so a request only uploads the new frame.  A worker thread
// admits queued requests as soon as (a) the stream has no request on the GPU
// (pair t needs pair t-1's field), (b) one of `max_inflight` slots is free and
// (c) the request's device footprint (results + workspace) fits in what is
// left of the pool.  Admitted requests run concurrently on their slots' HIP
// streams (continuous batching: new work joins while other work runs); the
// worker polls their completion events and stamps the latency.  Every
// request runs the same kernels as the *_frame calls, so its result does not
// depend on what else is in flight.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "acbm_internal.h"

using namespace acbm;

namespace {

using Clock = std::chrono::steady_clock;

__global__ void k_field_of(const acbm_block_result* __restrict__ res, int nb,
                           acbm_mv* __restrict__ field) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nb) field[i] = res[i].mv;
}

// First-fit allocator over one device allocation.
class Pool {
 public:
  int init(size_t bytes) {
    hipError_t e = hipMalloc(&base_, bytes);
    if (e != hipSuccess) return hip_fail(e, "allocating the serve pool");
    size_ = bytes;
    free_[0] = bytes;
    return ACBM_OK;
  }
  ~Pool() {
    if (base_) (void)hipFree(base_);
  }
  size_t size() const { return size_; }
  char* alloc(size_t n) {
    n = align256(n);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        const size_t off = it->first, left = it->second - n;
        free_.erase(it);
        if (left) free_[off + n] = left;
        used_[off] = n;
        return base_ + off;
      }
    }
    return nullptr;
  }
  void release(char* p) {
    if (!p) return;
    size_t off = (size_t)(p - base_);
    auto u = used_.find(off);
    if (u == used_.end()) return;
    size_t n = u->second;
    used_.erase(u);
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && off + n == nx->first) {
      n += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == off) {
        pv->second += n;
        return;
      }
    }
    free_[off] = n;
  }

 private:
  char* base_ = nullptr;
  size_t size_ = 0;
  std::map<size_t, size_t> free_, used_;
};

struct Request {
  uint64_t ticket = 0;
  uint32_t stream = 0;
  std::vector<uint8_t> frame;  // host copy, height*pitch bytes
  acbm_geom g{};
  acbm_params prm{};
  uint32_t algo = 0;
  Clock::time_point t_submit, t_start, t_done;
  bool done = false;
  int status = ACBM_OK;
  std::vector<acbm_block_result> results;
};

struct StreamState {
  bool open = false;
  acbm_geom g{};
  KGeom k{};
  char* frame[2] = {nullptr, nullptr};  // [ref, spare]
  acbm_mv* field = nullptr;
  bool has_field = false;
  bool busy = false;
};

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  std::shared_ptr<Request> req;
  char* res_dev = nullptr;
  char* ws_dev = nullptr;
  size_t ws_bytes = 0;
  uint8_t* pin_in = nullptr;
  size_t pin_in_bytes = 0;
  acbm_block_result* pin_out = nullptr;  // results, then the workspace header
  size_t pin_out_bytes = 0;
};

}  // namespace

struct acbm_server {
  acbm_serve_cfg cfg{};
  int device = 0;
  Pool pool;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<uint64_t, std::shared_ptr<Request>> tickets;
  std::vector<StreamState> streams;
  std::vector<Slot> slots;
  std::thread worker;
  bool stop = false;
  uint64_t next_ticket = 1;
  uint64_t completed = 0, rejected = 0;
  std::vector<double> lat_us;
  std::vector<std::pair<double, double>> busy;  // [start, done] in us since epoch
  Clock::time_point epoch = Clock::now();
  bool any = false;
  Clock::time_point first_submit, last_done;
  int fatal = ACBM_OK;

  ~acbm_server();
  void run();
  bool try_start(const std::shared_ptr<Request>& r, Slot& s);
  void finish(Slot& s);
};

static size_t frame_bytes(const acbm_geom& g) { return (size_t)g.pitch * g.height; }

static size_t ws_for(const KGeom& k, uint32_t algo) {
  return algo == ACBM_ALGO_FSBM ? fsbm_ws_bytes(k, 1) : predictive_ws_bytes(k, 1);
}

acbm_server::~acbm_server() {
  for (Slot& s : slots) {
    if (s.st) (void)hipStreamSynchronize(s.st);
    if (s.ev) (void)hipEventDestroy(s.ev);
    if (s.st) (void)hipStreamDestroy(s.st);
    if (s.pin_in) (void)hipHostFree(s.pin_in);
    if (s.pin_out) (void)hipHostFree(s.pin_out);
  }
}

constexpr uint32_t kRefOnly = 0xFFFFFFFFu;  // algo of a stream's first frame

static int grow_pinned(void** p, size_t* have, size_t need) {
  if (*have >= need) return ACBM_OK;
  if (*p) (void)hipHostFree(*p);
  *p = nullptr;
  *have = 0;
  hipError_t e = hipHostMalloc(p, need, hipHostMallocDefault);
  if (e != hipSuccess) return hip_fail(e, "allocating pinned staging memory");
  *have = need;
  return ACBM_OK;
}

// Called with the lock held.  Returns false when the request does not fit
// the pool yet (it stays queued).
bool acbm_server::try_start(const std::shared_ptr<Request>& r, Slot& s) {
  StreamState& ss = streams[r->stream];
  const size_t fb = frame_bytes(r->g);
  if (!ss.open) {
    KGeom k;
    check_geom(&r->g, &k);
    char* f0 = pool.alloc(fb);
    char* f1 = pool.alloc(fb);
    char* fld = pool.alloc((size_t)k.nb * sizeof(acbm_mv));
    if (!f0 || !f1 || !fld) {
      pool.release(f0);
      pool.release(f1);
      pool.release(fld);
      return false;
    }
    ss.open = true;
    ss.g = r->g;
    ss.k = k;
    ss.frame[0] = f0;
    ss.frame[1] = f1;
    ss.field = reinterpret_cast<acbm_mv*>(fld);
    ss.has_field = false;
  }
  const KGeom& k = ss.k;
  const bool ref_only = r->algo == kRefOnly;
  const size_t rb = ref_only ? 0 : (size_t)k.nb * sizeof(acbm_block_result);
  const size_t wsb = ref_only ? 0 : ws_for(k, r->algo);
  char* res = nullptr;
  char* ws = nullptr;
  if (!ref_only) {
    res = pool.alloc(rb);
    ws = pool.alloc(wsb);
    if (!res || !ws) {
      pool.release(res);
      pool.release(ws);
      return false;
    }
  }
  int rc = grow_pinned((void**)&s.pin_in, &s.pin_in_bytes, fb);
  if (!rc) rc = grow_pinned((void**)&s.pin_out, &s.pin_out_bytes, rb + sizeof(WsHeader));
  s.req = r;
  s.res_dev = res;
  s.ws_dev = ws;
  s.ws_bytes = wsb;
  ss.busy = true;
  r->t_start = Clock::now();
  hipError_t e = hipSuccess;
  if (!rc) {
    std::memcpy(s.pin_in, r->frame.data(), fb);
    e = hipMemcpyAsync(ss.frame[1], s.pin_in, fb, hipMemcpyHostToDevice, s.st);
    if (e != hipSuccess) rc = hip_fail(e, "uploading a frame");
  }
  if (!rc && !ref_only) {
    const uint8_t* frames[2] = {reinterpret_cast<const uint8_t*>(ss.frame[0]),
                                reinterpret_cast<const uint8_t*>(ss.frame[1])};
    auto* out = reinterpret_cast<acbm_block_result*>(res);
    if (r->algo == ACBM_ALGO_FSBM)
      rc = launch_fsbm(k, r->prm, frames, 1, ws, wsb, out, s.st);
    else
      rc = launch_predictive(k, r->prm, (int)r->algo, frames, 1,
                             ss.has_field ? ss.field : nullptr, ws, wsb, out, s.st);
    if (!rc) {
      {
        ProfScope ps("field", s.st);
        hipLaunchKernelGGL(k_field_of, dim3((k.nb + 255) / 256), dim3(256), 0, s.st, out, k.nb,
                           ss.field);
      }
      e = hipGetLastError();
      if (e == hipSuccess) e = hipMemcpyAsync(s.pin_out, out, rb, hipMemcpyDeviceToHost, s.st);
      // the predictive kernel reports failed waits in the workspace header
      if (e == hipSuccess)
        e = hipMemcpyAsync(reinterpret_cast<char*>(s.pin_out) + rb, ws, sizeof(WsHeader),
                           hipMemcpyDeviceToHost, s.st);
      if (e != hipSuccess) rc = hip_fail(e, "launching a served request");
    }
  }
  if (!rc) {
    e = hipEventRecord(s.ev, s.st);
    if (e != hipSuccess) rc = hip_fail(e, "recording completion");
  }
  r->status = rc;
  return true;
}

// Called with the lock held once the slot's event has fired (or its launch
// failed).
void acbm_server::finish(Slot& s) {
  std::shared_ptr<Request> r = s.req;
  StreamState& ss = streams[r->stream];
  const KGeom& k = ss.k;
  r->t_done = Clock::now();
  if (r->status == ACBM_OK && r->algo != kRefOnly) {
    const size_t rb = (size_t)k.nb * sizeof(acbm_block_result);
    WsHeader h;
    std::memcpy(&h, reinterpret_cast<char*>(s.pin_out) + rb, sizeof(h));
    if (r->algo != ACBM_ALGO_FSBM && h.status) r->status = ACBM_E_TIMEOUT;
    r->results.assign(s.pin_out, s.pin_out + k.nb);
    ss.has_field = true;
    lat_us.push_back(std::chrono::duration<double, std::micro>(r->t_done - r->t_submit).count());
    busy.emplace_back(std::chrono::duration<double, std::micro>(r->t_start - epoch).count(),
                      std::chrono::duration<double, std::micro>(r->t_done - epoch).count());
    ++completed;
    last_done = r->t_done;
  }
  if (r->status == ACBM_OK) std::swap(ss.frame[0], ss.frame[1]);  // new frame is the next reference
  ss.busy = false;
  pool.release(s.res_dev);
  pool.release(s.ws_dev);
  s.res_dev = s.ws_dev = nullptr;
  s.req.reset();
  r->done = true;
  cv_done.notify_all();
}

void acbm_server::run() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    bool inflight = false;
    for (Slot& s : slots) {
      if (!s.req) continue;
      hipError_t q = s.req->status == ACBM_OK ? hipEventQuery(s.ev) : hipSuccess;
      if (q == hipSuccess) finish(s);
      else if (q == hipErrorNotReady) inflight = true;
      else {
        s.req->status = hip_fail(q, "a served request failed on the device");
        finish(s);
      }
    }
    for (auto it = queue.begin(); it != queue.end();) {
      const auto& r = *it;
      if (streams[r->stream].busy) {
        ++it;
        continue;
      }
      Slot* free_slot = nullptr;
      for (Slot& s : slots)
        if (!s.req) {
          free_slot = &s;
          break;
        }
      if (!free_slot) break;
      if (try_start(r, *free_slot)) {
        inflight = true;
        it = queue.erase(it);
      } else {
        ++it;  // does not fit now; later requests of other streams may
      }
    }
    if (stop && queue.empty() && !inflight) return;
    if (!inflight) {
      cv_work.wait(lk);
    } else {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
      lk.lock();
    }
  }
}

extern "C" {

int acbm_serve(const acbm_serve_cfg* cfg, acbm_server** out) {
  if (!cfg || !out) return fail(ACBM_E_INVAL, "cfg or out is NULL");
  if (!cfg->pool_bytes || !cfg->max_streams || !cfg->max_inflight || !cfg->queue_depth)
    return fail(ACBM_E_INVAL, "zero in the serve configuration");
  int rc = check_device();
  if (rc) return rc;
  auto srv = std::make_unique<acbm_server>();
  srv->cfg = *cfg;
  if (hipGetDevice(&srv->device) != hipSuccess) return fail(ACBM_E_DEVICE, "hipGetDevice");
  if ((rc = srv->pool.init(cfg->pool_bytes))) return rc;
  srv->streams.resize(cfg->max_streams);
  srv->slots.resize(cfg->max_inflight);
  for (Slot& s : srv->slots) {
    hipError_t e = hipStreamCreateWithFlags(&s.st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.ev, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "creating serve streams");
  }
  acbm_server* raw = srv.get();
  srv->worker = std::thread([raw] { raw->run(); });
  *out = srv.release();
  return ACBM_OK;
}

int acbm_serve_submit(acbm_server* s, uint32_t stream_id, const uint8_t* host_frame,
                      const acbm_geom* g, const acbm_params* prm, uint32_t algo,
                      uint64_t* ticket) {
  if (!s || !host_frame || !g || !prm || !ticket) return fail(ACBM_E_INVAL, "NULL argument");
  KGeom k;
  int rc = check_geom(g, &k);
  if (rc) return rc;
  if ((rc = check_params(prm, k))) return rc;
  if (algo > ACBM_ALGO_ACBM) return fail(ACBM_E_INVAL, "unknown algorithm");
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->fatal) return s->fatal;
  if (stream_id >= s->streams.size()) return fail(ACBM_E_INVAL, "stream id out of range");
  if (s->queue.size() >= s->cfg.queue_depth) {
    ++s->rejected;
    return fail(ACBM_E_BUSY, "serve queue full");
  }
  // the largest footprint a request of this stream can need at once
  const size_t need = 2 * align256(frame_bytes(*g)) + align256((size_t)k.nb * sizeof(acbm_mv)) +
                      align256((size_t)k.nb * sizeof(acbm_block_result)) + align256(ws_for(k, algo));
  if (need > s->pool.size()) {
    ++s->rejected;
    return fail(ACBM_E_NOMEM, "request larger than the serve pool");
  }
  // a stream keeps one geometry; its first frame only becomes the reference
  StreamState& ss = s->streams[stream_id];
  const acbm_geom* first = ss.open ? &ss.g : nullptr;
  for (const auto& q : s->queue)
    if (!first && q->stream == stream_id) first = &q->g;
  if (first && std::memcmp(first, g, sizeof(*g)) != 0)
    return fail(ACBM_E_SHAPE, "geometry differs from the stream's first frame");
  const bool known = first != nullptr;
  auto r = std::make_shared<Request>();
  r->ticket = s->next_ticket++;
  r->stream = stream_id;
  r->frame.assign(host_frame, host_frame + frame_bytes(*g));
  r->g = *g;
  r->prm = *prm;
  r->algo = known ? algo : kRefOnly;
  r->t_submit = Clock::now();
  if (!s->any) {
    s->any = true;
    s->first_submit = r->t_submit;
  }
  s->tickets[r->ticket] = r;
  s->queue.push_back(r);
  *ticket = r->ticket;
  s->cv_work.notify_one();
  return ACBM_OK;
}

int acbm_serve_wait(acbm_server* s, uint64_t ticket, acbm_block_result* host_out,
                    int64_t timeout_us) {
  if (!s) return fail(ACBM_E_INVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return fail(ACBM_E_INVAL, "unknown ticket");
  std::shared_ptr<Request> r = it->second;
  auto ready = [&] { return r->done; };
  if (timeout_us < 0) s->cv_done.wait(lk, ready);
  else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready))
    return fail(ACBM_E_TIMEOUT, "request not finished yet");
  s->tickets.erase(ticket);
  if (r->status) return fail(r->status, "served request failed");
  if (host_out && !r->results.empty())
    std::memcpy(host_out, r->results.data(), r->results.size() * sizeof(acbm_block_result));
  return ACBM_OK;
}

int acbm_serve_stats_get(acbm_server* s, acbm_serve_stats* st) {
  if (!s || !st) return fail(ACBM_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(st, 0, sizeof(*st));
  st->completed = s->completed;
  st->rejected = s->rejected;
  if (!s->lat_us.empty()) {
    std::vector<double> v = s->lat_us;
    std::sort(v.begin(), v.end());
    auto pct = [&](double q) { return v[std::min(v.size() - 1, (size_t)(q * (v.size() - 1) + 0.5))]; };
    st->p50_us = pct(0.50);
    st->p99_us = pct(0.99);
    double sum = 0;
    for (double x : v) sum += x;
    st->mean_us = sum / v.size();
    const double span =
        std::chrono::duration<double, std::micro>(s->last_done - s->first_submit).count();
    st->throughput_rps = span > 0 ? s->completed / (span * 1e-6) : 0;
    // union of busy intervals over the span
    std::vector<std::pair<double, double>> b = s->busy;
    std::sort(b.begin(), b.end());
    double covered = 0, cs = -1, ce = -1;
    for (auto& iv : b) {
      if (iv.first > ce) {
        if (ce > cs) covered += ce - cs;
        cs = iv.first;
        ce = iv.second;
      } else {
        ce = std::max(ce, iv.second);
      }
    }
    if (ce > cs) covered += ce - cs;
    st->gpu_busy_frac = span > 0 ? std::min(1.0, covered / span) : 0;
  }
  return ACBM_OK;
}

int acbm_serve_close(acbm_server* s) {
  if (!s) return fail(ACBM_E_INVAL, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  delete s;
  return ACBM_OK;
}

}  // extern "C"
