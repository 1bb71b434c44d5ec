// acbm_serve.hip -- continuous batching of frame-pair motion estimation
// requests.
//
// Each video stream keeps its reference frame and its motion field on the
// device, so a request only uploads its new frame.  A worker thread turns the
// queue into passes: whenever one of `lanes` HIP streams is free, it gathers
// every queued request that can run now into one pass -- in submit order, at
// most one request per stream (pair t needs pair t-1's field and frame),
// while the requests on the GPU stay within `max_inflight` and the pass's
// results and workspace fit in the largest free block of the device pool
// (admission by HBM footprint).  A pass is one acbm_batch-style enqueue on
// its lane: the frame uploads, one full-search launch per search class and
// one resolve launch over every FSBM request, one row-walker launch per
// block size for the PBM/ACBM requests, one kernel that stores every
// request's field, and one download of all results.  Requests that arrive
// while passes run join the next pass, and passes on different lanes overlap
// on the device.  A request's kernels compute exactly what the *_frame calls
// compute for that pair, so its result does not depend on what it was
// batched with.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <thread>
#include <vector>

#include "acbm_internal.h"

using namespace acbm;

namespace {

using Clock = std::chrono::steady_clock;

// dst[i] = src[i].mv for the blocks of up to kFieldsPerLaunch requests
// (blockIdx.y picks the request).
struct FieldCopy {
  const acbm_block_result* src;
  acbm_mv* dst;
  uint32_t nb, pad;
};
constexpr int kFieldsPerLaunch = 64;
struct FieldTable {
  FieldCopy e[kFieldsPerLaunch];
};

__global__ void k_fields_of(const FieldTable t) {
  const FieldCopy c = t.e[blockIdx.y];
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < c.nb; i += gridDim.x * blockDim.x)
    c.dst[i] = c.src[i].mv;
}

// First-fit allocator over one block of memory the owner allocated.
class Arena {
 public:
  void init(char* base, size_t bytes) {
    base_ = base;
    size_ = bytes;
    free_.clear();
    used_.clear();
    if (bytes) free_[0] = bytes;
  }
  char* base() const { return base_; }
  size_t size() const { return size_; }
  size_t used() const { return used_bytes_; }
  size_t largest_free() const {
    size_t m = 0;
    for (const auto& f : free_) m = std::max(m, f.second);
    return m;
  }
  char* alloc(size_t n) {
    n = align256(std::max<size_t>(n, 1));
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        const size_t off = it->first, left = it->second - n;
        free_.erase(it);
        if (left) free_[off + n] = left;
        used_[off] = n;
        used_bytes_ += n;
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
    used_bytes_ -= n;
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
  size_t size_ = 0, used_bytes_ = 0;
  std::map<size_t, size_t> free_, used_;
};

constexpr uint32_t kRefOnly = 0xFFFFFFFFu;  // algo of a stream's first frame

struct Request {
  uint64_t ticket = 0;
  uint32_t stream = 0;
  char* pinned = nullptr;      // the frame, staged in the pinned arena, or
  std::vector<uint8_t> heap;   // in host memory when the arena was full
  acbm_geom g{};
  acbm_params prm{};
  uint32_t algo = 0;
  Clock::time_point t_submit, t_done;
  bool queued = false, done = false;
  int status = ACBM_OK;
  std::vector<acbm_block_result> results;
  const uint8_t* frame() const {
    return pinned ? reinterpret_cast<const uint8_t*>(pinned) : heap.data();
  }
};

struct StreamState {
  bool declared = false;  // its first frame was submitted (fixes the geometry)
  acbm_geom g{};
  KGeom k{};
  bool open = false;      // device memory below is allocated
  char* frame[2] = {nullptr, nullptr};  // [reference, next]
  acbm_mv* field = nullptr;
  bool has_field = false;
  bool busy = false;      // a request of this stream is in a pass
};

// One gathered launch on a lane.
struct Pass {
  std::vector<std::shared_ptr<Request>> reqs;
  std::vector<size_t> res_off;      // per request: offset of its results, or SIZE_MAX
  std::vector<const uint8_t*> fptr; // two frame pointers per compute request
  char* dev = nullptr;              // [results][batch workspace] in the device pool
  size_t res_bytes = 0, ws_bytes = 0;
  char* pin_out = nullptr;          // results, then the walker status words
  size_t nstatus = 0;
  int status = ACBM_OK;             // enqueue failure
};

struct Lane {
  hipStream_t st = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // timing events around the pass
  std::unique_ptr<Pass> pass;
};

}  // namespace

struct acbm_server {
  acbm_serve_cfg cfg{};
  int device = 0;
  char* pool_base = nullptr;
  char* pin_base = nullptr;
  Arena pool, pin;
  size_t pin_frame_cap = 0;  // frames may take this much of the pinned arena
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<uint64_t, std::shared_ptr<Request>> tickets;
  std::vector<StreamState> streams;
  std::vector<Lane> lanes;
  hipEvent_t ev_ref = nullptr;  // time origin of the device intervals
  std::thread worker;
  bool stop = false;
  uint64_t next_ticket = 1;
  uint64_t completed = 0, rejected = 0, passes = 0, batched = 0;
  size_t on_gpu = 0;  // requests in passes
  std::vector<double> lat_us;
  std::vector<std::pair<double, double>> dev_busy;  // pass [start, end], ms since ev_ref
  bool any = false;
  Clock::time_point first_submit, last_done;
  int fatal = ACBM_OK;

  ~acbm_server();
  void run();
  bool gather(Pass& P);
  int enqueue(Lane& L, Pass& P);
  void finish(Lane& L);
  void release_pass(Pass& P);
};

static size_t frame_bytes(const acbm_geom& g) { return (size_t)g.pitch * g.height; }

acbm_server::~acbm_server() {
  for (Lane& L : lanes) {
    if (L.st) (void)hipStreamSynchronize(L.st);
    if (L.ev0) (void)hipEventDestroy(L.ev0);
    if (L.ev1) (void)hipEventDestroy(L.ev1);
    if (L.st) (void)hipStreamDestroy(L.st);
  }
  if (ev_ref) (void)hipEventDestroy(ev_ref);
  if (pin_base) (void)hipHostFree(pin_base);
  if (pool_base) (void)hipFree(pool_base);
}

static size_t round_results(const KGeom& k) {
  return align256((size_t)k.nb * sizeof(acbm_block_result));
}

// Moves every queued request that can run now into P, in submit order.
// Called with the lock held.
bool acbm_server::gather(Pass& P) {
  std::set<uint32_t> blocked;  // streams whose next request cannot join this pass
  std::vector<acbm_job> jobs;
  size_t res_bytes = 0, ws_bytes = 0;
  for (auto it = queue.begin(); it != queue.end();) {
    if (on_gpu + P.reqs.size() >= cfg.max_inflight) break;
    const std::shared_ptr<Request>& r = *it;
    StreamState& ss = streams[r->stream];
    if (!r->queued || ss.busy || blocked.count(r->stream)) {  // queued: its frame is copied
      blocked.insert(r->stream);
      ++it;
      continue;
    }
    blocked.insert(r->stream);  // one request per stream per pass
    if (!ss.open) {
      char* f0 = pool.alloc(frame_bytes(ss.g));
      char* f1 = pool.alloc(frame_bytes(ss.g));
      char* fld = pool.alloc((size_t)ss.k.nb * sizeof(acbm_mv));
      if (!f0 || !f1 || !fld) {
        pool.release(f0);
        pool.release(f1);
        pool.release(fld);
        ++it;
        continue;  // no room for this stream's frames yet
      }
      ss.open = true;
      ss.frame[0] = f0;
      ss.frame[1] = f1;
      ss.field = reinterpret_cast<acbm_mv*>(fld);
      ss.has_field = false;
    }
    size_t rb = res_bytes, wb = ws_bytes;
    if (r->algo != kRefOnly) {
      acbm_job j{};
      j.geom = r->g;
      j.params = r->prm;
      j.algo = r->algo;
      j.nframes = 2;
      jobs.push_back(j);
      rb += round_results(ss.k);
      if (acbm_batch_workspace_size(jobs.data(), jobs.size(), &wb) != ACBM_OK) {
        jobs.pop_back();
        r->status = fail(ACBM_E_INVAL, "request rejected by the batch planner");
        r->done = true;
        it = queue.erase(it);
        cv_done.notify_all();
        continue;
      }
      wb = align256(wb);
      if (rb + wb > pool.largest_free() || rb + 64 * (jobs.size() + 1) > pin.largest_free()) {
        jobs.pop_back();
        ++it;
        continue;  // does not fit now; requests of other streams may
      }
    }
    res_bytes = rb;
    ws_bytes = wb;
    ss.busy = true;
    P.reqs.push_back(r);
    it = queue.erase(it);
  }
  if (P.reqs.empty()) return false;
  P.res_bytes = res_bytes;
  P.ws_bytes = ws_bytes;
  if (res_bytes + ws_bytes) {
    P.dev = pool.alloc(res_bytes + ws_bytes);
    P.pin_out = pin.alloc(res_bytes + 64 * (jobs.size() + 1));
    if (!P.dev || !P.pin_out) {  // cannot happen after the checks above; give the requests back
      pool.release(P.dev);
      pin.release(P.pin_out);
      P.dev = P.pin_out = nullptr;
      for (auto rit = P.reqs.rbegin(); rit != P.reqs.rend(); ++rit) {
        streams[(*rit)->stream].busy = false;
        queue.push_front(*rit);
      }
      P.reqs.clear();
      return false;
    }
  }
  size_t off = 0;
  for (const auto& r : P.reqs) {
    if (r->algo == kRefOnly) {
      P.res_off.push_back(SIZE_MAX);
    } else {
      P.res_off.push_back(off);
      off += round_results(streams[r->stream].k);
    }
  }
  return true;
}

// Enqueues a gathered pass on its lane (called without the lock: the
// requests' streams are marked busy, so nothing else touches their state).
int acbm_server::enqueue(Lane& L, Pass& P) {
  hipError_t e = hipEventRecord(L.ev0, L.st);
  if (e != hipSuccess) return hip_fail(e, "recording a pass start");
  for (const auto& r : P.reqs) {
    StreamState& ss = streams[r->stream];
    e = hipMemcpyAsync(ss.frame[1], r->frame(), frame_bytes(ss.g), hipMemcpyHostToDevice, L.st);
    if (e != hipSuccess) return hip_fail(e, "uploading a frame");
  }
  std::vector<acbm_job> jobs;
  std::vector<const acbm_mv*> prev;
  std::vector<FieldCopy> fields;
  P.fptr.resize(2 * P.reqs.size());
  for (size_t i = 0; i < P.reqs.size(); ++i) {
    const auto& r = P.reqs[i];
    if (r->algo == kRefOnly) continue;
    StreamState& ss = streams[r->stream];
    P.fptr[2 * i] = reinterpret_cast<const uint8_t*>(ss.frame[0]);
    P.fptr[2 * i + 1] = reinterpret_cast<const uint8_t*>(ss.frame[1]);
    acbm_job j{};
    j.geom = r->g;
    j.params = r->prm;
    j.algo = r->algo;
    j.nframes = 2;
    j.frames = &P.fptr[2 * i];
    j.out = reinterpret_cast<acbm_block_result*>(P.dev + P.res_off[i]);
    jobs.push_back(j);
    prev.push_back(r->algo != ACBM_ALGO_FSBM && ss.has_field ? ss.field : nullptr);
    fields.push_back(FieldCopy{j.out, ss.field, (uint32_t)ss.k.nb, 0});
  }
  if (jobs.empty()) {
    e = hipEventRecord(L.ev1, L.st);
    return e == hipSuccess ? ACBM_OK : hip_fail(e, "recording a pass end");
  }
  std::vector<const uint32_t*> status_words;
  int rc = batch_enqueue(jobs.data(), jobs.size(), prev.data(), P.dev + P.res_bytes, P.ws_bytes,
                         L.st, false, &status_words);
  if (rc) return rc;
  for (size_t f0 = 0; f0 < fields.size(); f0 += kFieldsPerLaunch) {
    FieldTable t{};
    const size_t n = std::min<size_t>(kFieldsPerLaunch, fields.size() - f0);
    uint32_t nbmax = 0;
    for (size_t k = 0; k < n; ++k) {
      t.e[k] = fields[f0 + k];
      nbmax = std::max(nbmax, t.e[k].nb);
    }
    ProfScope ps("field", L.st);
    hipLaunchKernelGGL(k_fields_of, dim3(std::min<uint32_t>((nbmax + 255) / 256, 64), (unsigned)n),
                       dim3(256), 0, L.st, t);
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "storing the served fields");
  }
  e = hipMemcpyAsync(P.pin_out, P.dev, P.res_bytes, hipMemcpyDeviceToHost, L.st);
  if (e != hipSuccess) return hip_fail(e, "downloading served results");
  P.nstatus = std::min<size_t>(status_words.size(), 16 * (jobs.size() + 1));
  for (size_t k = 0; k < P.nstatus; ++k) {
    e = hipMemcpyAsync(P.pin_out + P.res_bytes + 4 * k, status_words[k], 4, hipMemcpyDeviceToHost,
                       L.st);
    if (e != hipSuccess) return hip_fail(e, "downloading a walker status");
  }
  e = hipEventRecord(L.ev1, L.st);
  return e == hipSuccess ? ACBM_OK : hip_fail(e, "recording a pass end");
}

// Returns a pass's memory (lock held; its work has finished or been waited for).
void acbm_server::release_pass(Pass& P) {
  pool.release(P.dev);
  pin.release(P.pin_out);
  for (const auto& r : P.reqs) {
    pin.release(r->pinned);
    r->pinned = nullptr;
    r->heap.clear();
    r->heap.shrink_to_fit();
  }
  P.dev = P.pin_out = nullptr;
}

// Completes the pass of a lane whose end event has fired, or whose enqueue
// failed (lock held).
void acbm_server::finish(Lane& L) {
  Pass& P = *L.pass;
  const Clock::time_point now = Clock::now();
  bool timed_out = false;
  if (P.status == ACBM_OK) {
    for (size_t k = 0; k < P.nstatus; ++k) {
      uint32_t v = 0;
      std::memcpy(&v, P.pin_out + P.res_bytes + 4 * k, 4);
      if (v) timed_out = true;
    }
    float t0 = 0, t1 = 0;
    if (hipEventElapsedTime(&t0, ev_ref, L.ev0) == hipSuccess &&
        hipEventElapsedTime(&t1, ev_ref, L.ev1) == hipSuccess)
      dev_busy.emplace_back(t0, t1);
    if (P.res_bytes) ++passes;  // passes that computed something (not uploads alone)
  }
  for (size_t i = 0; i < P.reqs.size(); ++i) {
    const auto& r = P.reqs[i];
    StreamState& ss = streams[r->stream];
    r->t_done = now;
    if (P.status != ACBM_OK) {
      r->status = P.status;
      ss.has_field = false;
    } else {
      std::swap(ss.frame[0], ss.frame[1]);  // the uploaded frame is the next reference
      if (r->algo != kRefOnly) {
        const acbm_block_result* res =
            reinterpret_cast<const acbm_block_result*>(P.pin_out + P.res_off[i]);
        r->results.assign(res, res + ss.k.nb);
        if (timed_out && r->algo != ACBM_ALGO_FSBM) {
          r->status = ACBM_E_TIMEOUT;  // incomplete: not a predictor for the next pair
          ss.has_field = false;
        } else {
          ss.has_field = true;
          lat_us.push_back(std::chrono::duration<double, std::micro>(now - r->t_submit).count());
          ++completed;
          ++batched;
          last_done = now;
        }
      }
    }
    ss.busy = false;
    r->done = true;
  }
  on_gpu -= P.reqs.size();
  release_pass(P);
  L.pass.reset();
  cv_done.notify_all();
}

void acbm_server::run() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    bool inflight = false;
    for (Lane& L : lanes) {
      if (!L.pass) continue;
      const hipError_t q = hipEventQuery(L.ev1);
      if (q == hipSuccess) {
        finish(L);
      } else if (q == hipErrorNotReady) {
        inflight = true;
      } else {
        fatal = L.pass->status = hip_fail(q, "a served pass failed on the device");
        finish(L);
      }
    }
    for (Lane& L : lanes) {
      if (L.pass || queue.empty() || fatal) continue;
      auto P = std::make_unique<Pass>();
      if (!gather(*P)) break;
      on_gpu += P->reqs.size();
      Pass* raw = P.get();
      L.pass = std::move(P);
      lk.unlock();
      const int rc = enqueue(L, *raw);
      if (rc) (void)hipStreamSynchronize(L.st);  // whatever was enqueued has finished
      lk.lock();
      if (rc) {
        raw->status = rc;
        fatal = rc;
        finish(L);
      } else {
        inflight = true;
      }
    }
    if (fatal) {  // fail what is still queued
      for (const auto& r : queue) {
        r->status = fatal;
        r->done = true;
      }
      queue.clear();
      cv_done.notify_all();
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
  if (cfg->lanes > 16) return fail(ACBM_E_INVAL, "at most 16 lanes");
  int rc = check_device();
  if (rc) return rc;
  auto srv = std::make_unique<acbm_server>();
  srv->cfg = *cfg;
  if (!srv->cfg.lanes) srv->cfg.lanes = 4;
  if (!srv->cfg.pinned_bytes) srv->cfg.pinned_bytes = (size_t)512 << 20;
  if (hipGetDevice(&srv->device) != hipSuccess) return fail(ACBM_E_DEVICE, "hipGetDevice");
  hipError_t e = hipMalloc(&srv->pool_base, cfg->pool_bytes);
  if (e != hipSuccess) return hip_fail(e, "allocating the serve pool");
  srv->pool.init(srv->pool_base, cfg->pool_bytes);
  e = hipHostMalloc(&srv->pin_base, srv->cfg.pinned_bytes, hipHostMallocDefault);
  if (e != hipSuccess) return hip_fail(e, "allocating the pinned staging arena");
  srv->pin.init(srv->pin_base, srv->cfg.pinned_bytes);
  srv->pin_frame_cap = srv->cfg.pinned_bytes / 4 * 3;  // the rest is kept for results
  srv->streams.resize(cfg->max_streams);
  srv->lanes.resize(srv->cfg.lanes);
  for (Lane& L : srv->lanes) {
    e = hipStreamCreateWithFlags(&L.st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&L.ev0);
    if (e == hipSuccess) e = hipEventCreate(&L.ev1);
    if (e != hipSuccess) return hip_fail(e, "creating serve lanes");
  }
  e = hipEventCreate(&srv->ev_ref);
  if (e == hipSuccess) e = hipEventRecord(srv->ev_ref, srv->lanes[0].st);
  if (e == hipSuccess) e = hipEventSynchronize(srv->ev_ref);
  if (e != hipSuccess) return hip_fail(e, "recording the serve time origin");
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
  const size_t fb = frame_bytes(*g);
  auto r = std::make_shared<Request>();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->fatal) return fail(s->fatal, "the server stopped after a device error");
    if (stream_id >= s->streams.size()) return fail(ACBM_E_INVAL, "stream id out of range");
    if (s->queue.size() >= s->cfg.queue_depth) {
      ++s->rejected;
      return fail(ACBM_E_BUSY, "serve queue full");
    }
    // the largest footprint a request of this stream can need at once: its
    // frames and field, plus its results and workspace alone in a pass
    acbm_job j{};
    j.geom = *g;
    j.params = *prm;
    j.algo = algo;
    j.nframes = 2;
    size_t wb = 0;
    if ((rc = acbm_batch_workspace_size(&j, 1, &wb))) return rc;
    const size_t need = 2 * align256(fb) + align256((size_t)k.nb * sizeof(acbm_mv)) +
                        round_results(k) + align256(wb);
    if (need > s->pool.size() || round_results(k) + 128 > s->pin.size() - s->pin_frame_cap) {
      ++s->rejected;
      return fail(ACBM_E_NOMEM, "request larger than the serve pool");
    }
    // a stream keeps one geometry; its first frame only becomes the reference
    StreamState& ss = s->streams[stream_id];
    if (ss.declared && std::memcmp(&ss.g, g, sizeof(*g)) != 0)
      return fail(ACBM_E_SHAPE, "geometry differs from the stream's first frame");
    r->algo = ss.declared ? algo : kRefOnly;
    if (!ss.declared) {
      ss.declared = true;
      ss.g = *g;
      ss.k = k;
    }
    r->ticket = s->next_ticket++;
    r->stream = stream_id;
    r->g = *g;
    r->prm = *prm;
    r->t_submit = Clock::now();
    if (s->pin.used() + align256(fb) <= s->pin_frame_cap) r->pinned = s->pin.alloc(fb);
    if (!s->any) {
      s->any = true;
      s->first_submit = r->t_submit;
    }
    s->tickets[r->ticket] = r;
    // queued now (submit order), runnable once the copy below is done
    s->queue.push_back(r);
  }
  if (r->pinned)
    std::memcpy(r->pinned, host_frame, fb);
  else
    r->heap.assign(host_frame, host_frame + fb);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    r->queued = true;
  }
  s->cv_work.notify_one();
  *ticket = r->ticket;
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

int acbm_serve_stats(acbm_server* s, acbm_serve_report* st) {
  if (!s || !st) return fail(ACBM_E_INVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(st, 0, sizeof(*st));
  st->completed = s->completed;
  st->rejected = s->rejected;
  st->passes = s->passes;
  st->mean_batch = s->passes ? (double)s->batched / (double)s->passes : 0;
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
  }
  if (!s->dev_busy.empty()) {
    // union of the passes' device intervals over the span they cover
    std::vector<std::pair<double, double>> b = s->dev_busy;
    std::sort(b.begin(), b.end());
    double covered = 0, cs = b[0].first, ce = b[0].second, lo = b[0].first, hi = b[0].second;
    for (const auto& iv : b) {
      hi = std::max(hi, iv.second);
      if (iv.first > ce) {
        covered += ce - cs;
        cs = iv.first;
        ce = iv.second;
      } else {
        ce = std::max(ce, iv.second);
      }
    }
    covered += ce - cs;
    st->device_busy_frac = hi > lo ? std::min(1.0, covered / (hi - lo)) : 0;
    st->device_busy_ms = covered;
  }
  return ACBM_OK;
}

int acbm_serve_stats_get(acbm_server* s, acbm_serve_report* st) {
  return acbm_serve_stats(s, st);
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
