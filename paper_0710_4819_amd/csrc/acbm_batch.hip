// acbm_batch.hip -- many sequences of uneven geometry in one call.
//
// FSBM jobs (Section 2.3) are grouped by block size and window-search plan
// (at most 64 jobs a group); each group runs as one full-search launch with
// a workgroup per (job, pair, block) item (per 2x2 tile of 8x8 blocks with a
// tiled plan), then a single resolve launch
// takes every pair of every FSBM job at once.  PBM/ACBM jobs (Sections 2.2,
// 3.2) are grouped by block size and precision (at most 256 jobs a group);
// each group runs as one row-walker launch whose walkers take the rows of
// all its jobs in level order, so the jobs' dependency chains run side by
// side.  The job tables those launches read are written into the caller's
// workspace by small kernels whose arguments carry the bytes, so the whole
// call is stream-ordered and needs no host staging memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <map>
#include <tuple>
#include <vector>

#include "acbm_internal.h"

#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>

using namespace acbm;

namespace {

// A PBM/ACBM job joins a walker group unless its pairs exceed what a row
// word can name; such a job runs on its own, in launches of up to
// kMaxPairsPerLaunch pairs.
bool grouped(const acbm_job& j) { return j.nframes - 1 <= kPredMaxPairs; }

int job_ws(const acbm_job& j, size_t* bytes) {
  KGeom k;
  int rc = check_geom(&j.geom, &k);
  if (rc) return rc;
  if (j.nframes < 2) return fail(ACBM_E_INVAL, "a job needs at least two frames");
  const uint32_t npairs = j.nframes - 1;
  switch (j.algo) {
    case ACBM_ALGO_FSBM: *bytes = align256(fsbm_ws_bytes(k, npairs)); return ACBM_OK;
    case ACBM_ALGO_PBM:
    case ACBM_ALGO_ACBM:
      // grouped: the vector words of every pair; alone: the single-job workspace
      *bytes = grouped(j) ? align256((size_t)npairs * k.nb * sizeof(uint32_t))
                          : align256(predictive_ws_bytes(k, npairs));
      return ACBM_OK;
    default: return fail(ACBM_E_INVAL, "unknown algorithm");
  }
}

// PBM/ACBM jobs of one block size and precision that run as one launch.
struct PGroup {
  int bw = 0, bh = 0;
  bool hp = false;
  std::vector<size_t> job_index;  // into the caller's job array
  uint32_t total_rows = 0;
  size_t nptr = 0;                // frame pointers of its jobs
  size_t off_args = 0, off_ptrs = 0;   // within the table region
  size_t off_hdr = 0, off_order = 0;   // within the scratch region
};

// Everything one acbm_batch call enqueues, planned on the host.
struct Class {
  int N = 0, M = 0;
  SearchPlan pl{};
  std::vector<BatchJob> jobs;
  std::vector<size_t> job_index;  // into the caller's job array
  uint32_t items = 0;
  size_t lds_search = 0;
  size_t lds_resolve = 0;  // the resolve of this class's pairs
  uint32_t pair0 = 0, pairs = 0;
  int steps = 0;           // longest anti-diagonal walk of its resolves, bx + 2(by - 1)
  int max_by = 0;          // most block rows of its frames
};

struct Plan {
  std::vector<size_t> slice;      // workspace offset of each job
  std::vector<Class> classes;
  std::vector<size_t> predictive; // PBM/ACBM jobs that run alone
  std::vector<PGroup> pgroups;    // PBM/ACBM jobs that run in groups
  size_t jobs_bytes = 0;          // job slices
  size_t table_off = 0, table_bytes = 0;
  size_t scratch_off = 0, scratch_bytes = 0;  // group headers and row orders
  size_t off_jobs = 0, off_ptrs = 0;  // within the table region
  size_t njob_fsbm = 0, nptr = 0;
  uint32_t pairs = 0;             // FSBM pairs (resolve workgroups)
  size_t lds_resolve = 0;
  int max_by = 0;
};

// Groups the jobs and lays out the workspace: job slices first, then the
// table region [BatchJob per FSBM job][frame pointers][per walker group: its
// job table, its frame pointers], then the scratch region [per walker group:
// header, row order].
int make_plan(const acbm_job* jobs, size_t njobs, Plan* pl) {
  std::map<std::tuple<int, int, int, int, int>, size_t> cls;
  std::map<std::tuple<int, int, int>, size_t> pcls;
  size_t off = 0;
  pl->slice.resize(njobs);
  for (size_t i = 0; i < njobs; ++i) {
    const acbm_job& j = jobs[i];
    size_t b = 0;
    int rc = job_ws(j, &b);
    if (rc) return rc;
    pl->slice[i] = off;
    off += b;
    if (j.algo != ACBM_ALGO_FSBM) {
      if (!grouped(j)) {
        pl->predictive.push_back(i);
        continue;
      }
      KGeom k;
      check_geom(&j.geom, &k);
      const auto key = std::make_tuple(k.bw, k.bh, j.params.subpel ? 1 : 0);
      auto it = pcls.find(key);
      if (it != pcls.end() && pl->pgroups[it->second].job_index.size() == (size_t)kPredMaxJobs) {
        pcls.erase(it);  // a full group: later jobs of this kind open a new one
        it = pcls.end();
      }
      if (it == pcls.end()) {
        it = pcls.emplace(key, pl->pgroups.size()).first;
        pl->pgroups.emplace_back();
        pl->pgroups.back().bw = k.bw;
        pl->pgroups.back().bh = k.bh;
        pl->pgroups.back().hp = j.params.subpel != 0;
      }
      PGroup& pg = pl->pgroups[it->second];
      const uint64_t rows = (uint64_t)(j.nframes - 1) * k.by;
      if (pg.total_rows + rows > 0xFFFFFFFFull)
        return fail(ACBM_E_RANGE, "too many block rows in one batch group");
      pg.total_rows += (uint32_t)rows;
      pg.nptr += j.nframes;
      pg.job_index.push_back(i);
      continue;
    }
    KGeom k;
    check_geom(&j.geom, &k);
    const SearchPlan sp = plan_fsbm_search(k);
    if (!sp.R) return fail(ACBM_E_UNSUPPORTED, "search window does not fit in LDS");
    const auto key = std::make_tuple(k.bw, k.bh, sp.R, sp.threads, sp.tile);
    auto it = cls.find(key);
    if (it != cls.end() && pl->classes[it->second].jobs.size() == 64) {
      cls.erase(it);  // a full group: later jobs of this kind open a new one
      it = cls.end();
    }
    if (it == cls.end()) {
      it = cls.emplace(key, pl->classes.size()).first;
      pl->classes.emplace_back();
      pl->classes.back().N = k.bw;
      pl->classes.back().M = k.bh;
      pl->classes.back().pl = sp;
    }
    Class& c = pl->classes[it->second];
    const uint32_t npairs = j.nframes - 1;
    const uint32_t per_pair = sp.tile == 2 ? (uint32_t)k.nb / 4 : (uint32_t)k.nb;  // items
    if ((uint64_t)c.items + (uint64_t)npairs * per_pair > 0xFFFFFFFFull)
      return fail(ACBM_E_RANGE, "too many blocks in one batch group");
    BatchJob bj{};
    bj.g = k;
    bj.s = sp.tile == 2 ? window_shape_host(16, 16, k.p, sp.R)
                        : window_shape_host(k.bw, k.bh, k.p, sp.R);
    bj.slack = fsbm_slack(k.p, j.params);
    bj.lam = j.params.lambda;
    bj.subpel = j.params.subpel;
    bj.npairs = npairs;
    bj.item0 = c.items;
    c.items += npairs * per_pair;
    c.lds_search = std::max<size_t>(c.lds_search, (size_t)sp.lds_bytes);
    if (fsbm_mv_in_lds(k)) c.lds_resolve = std::max<size_t>(c.lds_resolve, (size_t)k.nb * 4);
    c.steps = std::max(c.steps, k.bx + 2 * (k.by - 1));
    c.max_by = std::max(c.max_by, k.by);
    c.jobs.push_back(bj);
    c.job_index.push_back(i);
    pl->njob_fsbm += 1;
    pl->nptr += j.nframes;
  }
  // Classes whose resolves walk the most anti-diagonal steps search first,
  // so that with a side stream their resolves overlap the later searches.
  std::stable_sort(pl->classes.begin(), pl->classes.end(),
                   [](const Class& a, const Class& b) { return a.steps > b.steps; });
  // resolve workgroups are numbered across all FSBM jobs, in table order
  for (Class& c : pl->classes) {
    c.pair0 = pl->pairs;
    for (BatchJob& bj : c.jobs) {
      bj.pair0 = pl->pairs;
      pl->pairs += bj.npairs;
    }
    c.pairs = pl->pairs - c.pair0;
    pl->lds_resolve = std::max(pl->lds_resolve, c.lds_resolve);
    pl->max_by = std::max(pl->max_by, c.max_by);
  }
  pl->jobs_bytes = off;
  pl->table_off = off;
  pl->off_jobs = 0;
  pl->off_ptrs = pl->off_jobs + align256(pl->njob_fsbm * sizeof(BatchJob));
  size_t t = pl->classes.empty() ? 0 : pl->off_ptrs + align256(pl->nptr * sizeof(void*));
  size_t sc = 0;
  for (PGroup& pg : pl->pgroups) {
    pg.off_args = t;
    t += align256(pg.job_index.size() * sizeof(PredArgs));
    pg.off_ptrs = t;
    t += align256(pg.nptr * sizeof(void*));
    pg.off_hdr = sc;
    sc += align256(sizeof(WsHeader));
    pg.off_order = sc;
    sc += align256((size_t)pg.total_rows * sizeof(uint32_t));
  }
  pl->table_bytes = t;
  pl->scratch_off = pl->table_off + t;
  pl->scratch_bytes = sc;
  return ACBM_OK;
}

// Up to 448 eight-byte words per launch travel as kernel arguments (under
// the 4 KiB argument limit) and are stored by one thread each.
constexpr int kTableWords = 448;
struct TableChunk {
  uint64_t w[kTableWords];
};
__global__ void k_put_table(uint64_t* __restrict__ dst, const TableChunk c, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = c.w[i];
}

// Fills the device pointers of the plan, plans the walker groups and
// enqueues the table writes.
int write_tables(const acbm_job* jobs, const acbm_mv* const* prev0, Plan* pl,
                 std::vector<PredGroupPlan>* gplans, char* ws, hipStream_t st) {
  if (!pl->table_bytes) return ACBM_OK;
  char* table = ws + pl->table_off;
  std::vector<uint64_t> host(pl->table_bytes / 8, 0);
  char* hb = reinterpret_cast<char*>(host.data());
  size_t jo = 0, po = 0;
  for (Class& c : pl->classes) {
    for (size_t n = 0; n < c.jobs.size(); ++n) {
      const acbm_job& j = jobs[c.job_index[n]];
      BatchJob& bj = c.jobs[n];
      char* sl = ws + pl->slice[c.job_index[n]];
      bj.recs = reinterpret_cast<BlockRec*>(sl + fsbm_recs_offset());
      bj.ovf = reinterpret_cast<uint16_t*>(sl + fsbm_ovf_offset(bj.g, bj.npairs));
      bj.mv_ws = fsbm_mv_in_lds(bj.g) ? nullptr
                                      : reinterpret_cast<uint32_t*>(sl + fsbm_mv_offset(bj.g, bj.npairs));
      bj.out = j.out;
      bj.frames = reinterpret_cast<const uint8_t* const*>(table + pl->off_ptrs + po * sizeof(void*));
      std::memcpy(hb + pl->off_ptrs + po * sizeof(void*), j.frames, j.nframes * sizeof(void*));
      po += j.nframes;
    }
    std::memcpy(hb + pl->off_jobs + jo * sizeof(BatchJob), c.jobs.data(),
                c.jobs.size() * sizeof(BatchJob));
    jo += c.jobs.size();
  }
  gplans->resize(pl->pgroups.size());
  for (size_t gi = 0; gi < pl->pgroups.size(); ++gi) {
    const PGroup& pg = pl->pgroups[gi];
    std::vector<KGeom> geoms(pg.job_index.size());
    for (size_t n = 0; n < pg.job_index.size(); ++n) check_geom(&jobs[pg.job_index[n]].geom, &geoms[n]);
    PredGroupPlan& gp = (*gplans)[gi];
    int rc = plan_predictive_group(geoms.data(), (int)geoms.size(), pg.hp, pg.total_rows, &gp);
    if (rc) return rc;
    WsHeader* hdr = reinterpret_cast<WsHeader*>(ws + pl->scratch_off + pg.off_hdr);
    size_t pp = 0;
    for (size_t n = 0; n < pg.job_index.size(); ++n) {
      const acbm_job& j = jobs[pg.job_index[n]];
      PredArgs a = predictive_args(geoms[n], j.params, (int)j.algo, gp.R, j.nframes - 1);
      a.hdr = hdr;
      a.words = reinterpret_cast<uint32_t*>(ws + pl->slice[pg.job_index[n]]);
      a.frames = reinterpret_cast<const uint8_t* const*>(table + pg.off_ptrs + pp * sizeof(void*));
      a.out = j.out;
      if (prev0 && prev0[pg.job_index[n]]) {  // the job's first pair has a temporal field
        a.prev0 = reinterpret_cast<const uint8_t*>(prev0[pg.job_index[n]]);
        a.prev0_stride = sizeof(acbm_mv);
      }
      std::memcpy(hb + pg.off_ptrs + pp * sizeof(void*), j.frames, j.nframes * sizeof(void*));
      pp += j.nframes;
      std::memcpy(hb + pg.off_args + n * sizeof(PredArgs), &a, sizeof(PredArgs));
    }
  }
  uint64_t* dst = reinterpret_cast<uint64_t*>(table);
  const size_t nw = host.size();
  for (size_t k = 0; k < nw; k += kTableWords) {
    const int n = (int)std::min<size_t>(kTableWords, nw - k);
    TableChunk chunk;
    std::memcpy(chunk.w, host.data() + k, (size_t)n * 8);
    hipLaunchKernelGGL(k_put_table, dim3((n + 63) / 64), dim3(64), 0, st, dst + k, chunk, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "writing the batch job table");
  }
  return ACBM_OK;
}

int validate_jobs(const acbm_job* jobs, size_t njobs, void* ws, size_t ws_bytes) {
  if (!jobs && njobs) return fail(ACBM_E_INVAL, "jobs is NULL");
  size_t need = 0;
  int rc = acbm_batch_workspace_size(jobs, njobs, &need);
  if (rc) return rc;
  if (ws_bytes < need || (!ws && need)) return fail(ACBM_E_NOMEM, "workspace too small");
  for (size_t i = 0; i < njobs; ++i) {
    const acbm_job& j = jobs[i];
    KGeom k;
    if ((rc = check_geom(&j.geom, &k)) || (rc = check_params(&j.params, k))) return rc;
    if (!j.frames || !j.out) return fail(ACBM_E_INVAL, "job frames or out is NULL");
    for (uint32_t f = 0; f < j.nframes; ++f)
      if ((rc = check_frame_ptr(j.frames[f], "frame"))) return rc;
  }
  return check_device();
}

}  // namespace

extern "C" {

int acbm_batch_workspace_size(const acbm_job* jobs, size_t njobs, size_t* bytes) {
  if (!jobs || !bytes) return fail(ACBM_E_INVAL, "jobs or bytes is NULL");
  Plan pl;
  int rc = make_plan(jobs, njobs, &pl);
  if (rc) return rc;
  *bytes = pl.jobs_bytes + pl.table_bytes + pl.scratch_bytes;
  return ACBM_OK;
}

}  // extern "C"

namespace {

// Side streams for a batch's walker launches, one set per device, created on
// first use and kept until the process ends.  The walker launches depend on
// nothing but the job tables, and each is bound by its dependency chain
// rather than by the device's issue rate, so running them side by side (and
// beside the FSBM searches) fills what one of them leaves idle: the
// 64-sequence mix's two walker groups take 12.7 ms side by side against
// 14.3 ms one after the other.  The lock keeps two host threads from
// interleaving their fork and join events.
constexpr int kSideStreams = 4;
struct SidePool {
  hipStream_t s[kSideStreams] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kSideStreams] = {};
  hipEvent_t searched = nullptr;  // a search class done: its resolve may start
};
std::mutex g_side_mu;
std::map<int, SidePool> g_side;

// Side streams a batch may use: ACBM_BATCH_STREAMS (0 to 4) overrides the
// default of four; 0 keeps every launch on the caller's stream.
int side_streams() {
  const char* e = std::getenv("ACBM_BATCH_STREAMS");
  if (!e) return kSideStreams;
  return std::max(0, std::min(kSideStreams, std::atoi(e)));
}

// Whether the resolves of a batch with several search classes get sized
// workgroups (launch_resolve_batch): ACBM_BATCH_RESOLVE_SIZED=0 keeps
// 1024-thread groups, which may sweep.  Read at every call.
bool resolve_sized() {
  const char* e = std::getenv("ACBM_BATCH_RESOLVE_SIZED");
  return !(e && e[0] == '0');
}

// The side streams of device `dev`, the current device; g_side_mu is held.
int side_pool(int dev, SidePool** out) {
  auto it = g_side.find(dev);
  if (it == g_side.end()) {
    SidePool p;
    hipError_t e = hipEventCreateWithFlags(&p.fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p.searched, hipEventDisableTiming);
    for (int i = 0; i < kSideStreams && e == hipSuccess; ++i) {
      e = hipStreamCreateWithFlags(&p.s[i], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&p.join[i], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
      for (int i = 0; i < kSideStreams; ++i) {
        if (p.s[i]) (void)hipStreamDestroy(p.s[i]);
        if (p.join[i]) (void)hipEventDestroy(p.join[i]);
      }
      if (p.fork) (void)hipEventDestroy(p.fork);
      if (p.searched) (void)hipEventDestroy(p.searched);
      return hip_fail(e, "creating the batch's side streams");
    }
    it = g_side.emplace(dev, p).first;
  }
  *out = &it->second;
  return ACBM_OK;
}

int enqueue_fsbm(const acbm_job* jobs, const Plan& pl, char* base, const BatchJob* all,
                 hipStream_t st, const hipStream_t* rs, int nrs, hipEvent_t searched);

}  // namespace

// Creates the current device's side streams now rather than at the first
// batch that forks (where a global-mode stream capture would refuse it).
int acbm::batch_side_streams_init() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_side_mu);
  SidePool* sp = nullptr;
  return side_pool(dev, &sp);
}

namespace {

// Enqueues every job of a validated batch, ordered on `st`: the job tables
// first; then one row-walker launch per PBM/ACBM group and one for each
// PBM/ACBM job that runs alone, on side streams forked off `st`; then one
// persistent search and one resolve launch per FSBM group on `st`, which
// finally waits for the side streams.  Kernels and stream-ordering events
// only, so the sequence can be recorded into a graph as it is (the side
// streams become parallel branches).
int enqueue_batch(const acbm_job* jobs, size_t njobs, const acbm_mv* const* prev0, void* ws,
                  hipStream_t st, bool allow_side, std::vector<const uint32_t*>* status_words) {
  Plan pl;
  int rc = make_plan(jobs, njobs, &pl);
  if (rc) return rc;
  char* base = static_cast<char*>(ws);
  std::vector<PredGroupPlan> gplans;
  if ((rc = write_tables(jobs, prev0, &pl, &gplans, base, st))) return rc;
  if (status_words) {
    status_words->clear();
    for (const PGroup& pg : pl.pgroups)
      status_words->push_back(reinterpret_cast<const uint32_t*>(
          base + pl.scratch_off + pg.off_hdr + offsetof(WsHeader, status)));
    for (size_t i : pl.predictive)
      status_words->push_back(
          reinterpret_cast<const uint32_t*>(base + pl.slice[i] + offsetof(WsHeader, status)));
  }
  const BatchJob* all = reinterpret_cast<const BatchJob*>(base + pl.table_off + pl.off_jobs);

  // Walker launches: the groups, then the jobs that run alone, round robin
  // over the side streams and, when the batch has no FSBM job, `st` as well.
  // (Two side streams can share a hardware queue and then run one after the
  // other; `st` and a side stream were measured to run side by side.)  With
  // several FSBM search classes, one more side stream takes their resolves,
  // each starting when its class's search is done, beside the later searches.
  const size_t nunits = pl.pgroups.size() + pl.predictive.size();
  const bool has_fsbm = !pl.classes.empty();
  const size_t off_st = has_fsbm ? nunits : nunits - std::min<size_t>(nunits, 1);
  const bool resolve_side = pl.classes.size() > 1;
  // resolve streams wanted: one for the first run of classes (the longest
  // chain), and one for each later class, at most three (see enqueue_fsbm)
  int runs_later = 0;
  for (size_t i = 1; i < pl.classes.size(); ++i)
    if (pl.classes[i].steps < pl.classes[0].steps) ++runs_later;
  const int want_r = resolve_side ? 1 + std::min(runs_later, 3) : 0;
  std::unique_lock<std::mutex> lk(g_side_mu, std::defer_lock);
  SidePool* sp = nullptr;
  int nside = 0;
  const int want_w =
      allow_side ? std::min<int>(side_streams(), (int)std::min<size_t>(kSideStreams, off_st)) : 0;
  int want = allow_side ? std::min<int>(side_streams(), want_w + want_r) : 0;
  if (want > 0) {
    int cur = -1;
    hipDevice_t sdev = -1;
    if (hipGetDevice(&cur) == hipSuccess && hipStreamGetDevice(st, &sdev) == hipSuccess &&
        sdev == cur) {
      lk.lock();
      if ((rc = side_pool(cur, &sp))) return rc;
      // A side stream forked into a capture stays in it until that capture
      // ends, which another thread may not have done yet.  Fork only onto
      // side streams that are idle or already in the capture `st` is in;
      // otherwise keep every launch on `st`.
      hipStreamCaptureStatus ost = hipStreamCaptureStatusNone;
      unsigned long long oid = 0;
      hipError_t e = hipStreamGetCaptureInfo(st, &ost, &oid);
      if (e != hipSuccess) return hip_fail(e, "querying the stream's capture state");
      bool usable = true;
      for (int i = 0; i < want && usable; ++i) {
        hipStreamCaptureStatus sst = hipStreamCaptureStatusNone;
        unsigned long long sid = 0;
        e = hipStreamGetCaptureInfo(sp->s[i], &sst, &sid);
        if (e != hipSuccess) return hip_fail(e, "querying a side stream's capture state");
        if (sst != hipStreamCaptureStatusNone &&
            !(sst == hipStreamCaptureStatusActive && ost == hipStreamCaptureStatusActive &&
              sid == oid))
          usable = false;
      }
      if (!usable) {
        lk.unlock();
        sp = nullptr;
        want = 0;
      }
    }
  }
  if (want > 0 && sp) {
    hipError_t e = hipEventRecord(sp->fork, st);
    if (e != hipSuccess) return hip_fail(e, "forking the batch's side streams");
    for (; nside < want; ++nside)
      if ((e = hipStreamWaitEvent(sp->s[nside], sp->fork, 0)) != hipSuccess) {
        rc = hip_fail(e, "forking the batch's side streams");
        break;
      }
  }
  const int nside_w = std::min(nside, want_w);  // side streams of walker launches
  // the resolve stream: a side stream of its own when one is left, else the
  // last walker stream
  hipStream_t rs[kSideStreams] = {};
  int nrs = 0;
  if (resolve_side && nside > 0) {
    for (int i = nside_w; i < nside; ++i) rs[nrs++] = sp->s[i];
    if (!nrs) rs[nrs++] = sp->s[nside - 1];  // shared with the last walker stream
  }
  const int lanes = nside_w + (has_fsbm && nside_w ? 0 : 1);  // lane nside_w is `st`
  for (size_t u = 0; u < nunits && !rc; ++u) {
    const int lane = (int)(u % lanes);
    hipStream_t su = lane < nside_w ? sp->s[lane] : st;
    if (u < pl.pgroups.size()) {
      const PGroup& pg = pl.pgroups[u];
      rc = launch_predictive_group(
          pg.bw, pg.bh, pg.hp, gplans[u],
          reinterpret_cast<const PredArgs*>(base + pl.table_off + pg.off_args),
          (int)pg.job_index.size(),
          reinterpret_cast<uint32_t*>(base + pl.scratch_off + pg.off_order),
          reinterpret_cast<WsHeader*>(base + pl.scratch_off + pg.off_hdr), pg.total_rows, su);
    } else {
      const size_t i = pl.predictive[u - pl.pgroups.size()];
      const acbm_job& j = jobs[i];
      KGeom k;
      check_geom(&j.geom, &k);
      size_t b = 0;
      job_ws(j, &b);
      rc = launch_predictive(k, j.params, (int)j.algo, j.frames, j.nframes - 1,
                             prev0 ? prev0[i] : nullptr, base + pl.slice[i], b, j.out, su);
    }
  }
  if (!rc) rc = enqueue_fsbm(jobs, pl, base, all, st, rs, nrs, nrs ? sp->searched : nullptr);
  // join every forked stream, after an error too, so that a capture of `st`
  // still ends with every branch joined
  for (int i = 0; i < nside; ++i) {
    hipError_t e = hipEventRecord(sp->join[i], sp->s[i]);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, sp->join[i], 0);
    if (e != hipSuccess && !rc) rc = hip_fail(e, "joining the batch's side streams");
  }
  return rc;
}

// The FSBM jobs of a batch on `st`: a search launch per group, the half-pel
// preparation of half-pel jobs, and one resolve over every FSBM pair; or,
// with a resolve stream `rs` (forked from `st` and joined back by the
// caller), resolve launches on `rs` that start as soon as their groups are
// searched.
int enqueue_fsbm(const acbm_job* jobs, const Plan& pl, char* base, const BatchJob* all,
                 hipStream_t st, const hipStream_t* rss, int nrs, hipEvent_t searched) {
  hipStream_t rs = nrs ? rss[0] : nullptr;  // the first run's resolve stream
  int next_rs = 0;                          // later classes rotate over the rest
  int rc = ACBM_OK;
  size_t jo = 0;
  size_t pend = 0, pend_jo = 0;  // first class (and its job) not yet resolved
  for (const Class& c : pl.classes) {
    const acbm_job& j0 = jobs[c.job_index[0]];
    if (c.jobs.size() == 1 && j0.nframes - 1 <= (uint32_t)kMaxPairsPerLaunch) {
      // a group of one job: the plain per-block search reads its frame
      // pointers from kernel arguments, without the job-table lookup
      const BatchJob& bj = c.jobs[0];
      char* sl = base + pl.slice[c.job_index[0]];
      rc = launch_search_plan(bj.g, c.pl, j0.frames, (int)bj.npairs,
                              reinterpret_cast<BlockRec*>(sl + fsbm_recs_offset()),
                              reinterpret_cast<uint16_t*>(sl + fsbm_ovf_offset(bj.g, bj.npairs)),
                              bj.slack, st);
    } else {
      rc = launch_search_batch(c.N, c.M, c.pl, c.lds_search, all + jo, (int)c.jobs.size(),
                               c.items, st);
    }
    if (rc) return rc;
    // half-pel jobs: the SADs around single possible winners, before the
    // resolve (kernel arguments carry up to 64 pairs' frame pointers)
    for (size_t q = 0; q < c.jobs.size(); ++q) {
      const BatchJob& bj = c.jobs[q];
      if (!bj.subpel) continue;
      const acbm_job& jj = jobs[c.job_index[q]];
      char* sl = base + pl.slice[c.job_index[q]];
      BlockRec* recs = reinterpret_cast<BlockRec*>(sl + fsbm_recs_offset());
      uint16_t* ovf = reinterpret_cast<uint16_t*>(sl + fsbm_ovf_offset(bj.g, bj.npairs));
      const size_t ovf_per_pair = (size_t)bj.g.nb * fsbm_ovf_entries(bj.g.p);
      for (uint32_t p0 = 0; p0 < bj.npairs; p0 += kMaxPairsPerLaunch) {
        const int n = (int)std::min<uint32_t>(kMaxPairsPerLaunch, bj.npairs - p0);
        FramePtrs fr{};
        for (int k = 0; k <= n; ++k) fr.f[k] = jj.frames[p0 + k];
        if ((rc = launch_half_prep(bj.g, fr, n, recs + (size_t)p0 * bj.g.nb,
                                   ovf + p0 * ovf_per_pair, st)))
          return rc;
      }
    }
    jo += c.jobs.size();
    // With a resolve stream, the classes whose resolves walk the same longest
    // chain resolve in one launch once the last of them is searched (one
    // launch, so their pairs resolve side by side rather than one class
    // after the other on the stream); the classes sort by that chain, so
    // the long resolves overlap the searches of the classes after them.
    // Classes after the first run resolve one launch each, as soon as each is
    // searched, on the other resolve streams in turn (side by side, so that
    // their chains do not add up): the last one's resolve alone is left after
    // the searches.
    const size_t ci = (size_t)(&c - pl.classes.data());
    const bool first_run = c.steps == pl.classes[0].steps;
    if (rs && (!first_run || ci + 1 == pl.classes.size() || pl.classes[ci + 1].steps < c.steps)) {
      hipStream_t to = rs;
      if (!first_run && nrs > 1) to = rss[1 + next_rs++ % (nrs - 1)];
      hipError_t e = hipEventRecord(searched, st);
      if (e == hipSuccess) e = hipStreamWaitEvent(to, searched, 0);
      if (e != hipSuccess) return hip_fail(e, "ordering a batch resolve after its search");
      const Class& c0 = pl.classes[pend];
      size_t lds = 0;
      int max_by = 0;
      for (size_t k = pend; k <= ci; ++k) {
        lds = std::max(lds, pl.classes[k].lds_resolve);
        max_by = std::max(max_by, pl.classes[k].max_by);
      }
      // with several classes every resolve is sized: all but the last run
      // beside later searches, and the last one, on the mixed batch, steps
      // faster than it sweeps
      if ((rc = launch_resolve_batch(all + pend_jo, (int)(jo - pend_jo), c0.pair0,
                                     c.pair0 + c.pairs - c0.pair0, lds, max_by,
                                     pl.classes.size() > 1 && resolve_sized(), to)))
        return rc;
      pend = ci + 1;
      pend_jo = jo;
    }
  }
  if (!nrs && pl.njob_fsbm &&
      (rc = launch_resolve_batch(all, (int)pl.njob_fsbm, 0, pl.pairs, pl.lds_resolve, pl.max_by,
                                 false, st)))
    return rc;
  return ACBM_OK;
}

}  // namespace

// A validated batch whose PBM/ACBM jobs may start from a temporal field
// (prev0[i], acbm_mv per block, or null for zeros), enqueued on `st` alone
// or with side streams; status_words receives the device addresses of the
// walker launches' status words.
int acbm::batch_enqueue(const acbm_job* jobs, size_t njobs, const acbm_mv* const* prev0,
                        void* ws, size_t ws_bytes, hipStream_t st, bool side_streams,
                        std::vector<const uint32_t*>* status_words) {
  int rc = validate_jobs(jobs, njobs, ws, ws_bytes);
  if (rc) return rc;
  return enqueue_batch(jobs, njobs, prev0, ws, st, side_streams, status_words);
}

struct acbm_batch_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~acbm_batch_graph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

extern "C" {

int acbm_batch(const acbm_job* jobs, size_t njobs, void* ws, size_t ws_bytes, void* stream) {
  int rc = validate_jobs(jobs, njobs, ws, ws_bytes);
  if (rc) return rc;
  return enqueue_batch(jobs, njobs, nullptr, ws, static_cast<hipStream_t>(stream), true, nullptr);
}

int acbm_batch_graph_create(const acbm_job* jobs, size_t njobs, void* ws, size_t ws_bytes,
                            acbm_batch_graph** out) {
  if (!out) return fail(ACBM_E_INVAL, "out is NULL");
  *out = nullptr;
  int rc = validate_jobs(jobs, njobs, ws, ws_bytes);
  if (rc) return rc;
  hipStream_t st = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "creating the capture stream");
  e = hipStreamBeginCapture(st, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) {
    (void)hipStreamDestroy(st);
    return hip_fail(e, "beginning the batch capture");
  }
  rc = enqueue_batch(jobs, njobs, nullptr, ws, st, true, nullptr);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(st, &graph);
  (void)hipStreamDestroy(st);
  if (!rc && e != hipSuccess) rc = hip_fail(e, "ending the batch capture");
  if (rc) {
    if (graph) (void)hipGraphDestroy(graph);
    return rc;
  }
  auto gr = std::make_unique<acbm_batch_graph>();
  gr->graph = graph;
  e = hipGraphInstantiate(&gr->exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return hip_fail(e, "instantiating the batch graph");
  *out = gr.release();
  return ACBM_OK;
}

int acbm_batch_status(const acbm_job* jobs, size_t njobs, const void* ws, size_t ws_bytes,
                      void* stream, int* status) {
  if (!jobs || !ws || !status) return fail(ACBM_E_INVAL, "jobs, workspace or status is NULL");
  Plan pl;
  int rc = make_plan(jobs, njobs, &pl);
  if (rc) return rc;
  if (ws_bytes < pl.jobs_bytes + pl.table_bytes + pl.scratch_bytes)
    return fail(ACBM_E_NOMEM, "workspace too small");
  // headers: one per walker group, and at the start of each solo job's slice
  const char* base = static_cast<const char*>(ws);
  std::vector<const char*> at;
  for (const PGroup& pg : pl.pgroups) at.push_back(base + pl.scratch_off + pg.off_hdr);
  for (size_t i : pl.predictive) at.push_back(base + pl.slice[i]);
  std::vector<uint32_t> st(at.size(), 0);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipSuccess;
  for (size_t k = 0; k < at.size() && e == hipSuccess; ++k)
    e = hipMemcpyAsync(&st[k], at[k] + offsetof(WsHeader, status), sizeof(uint32_t),
                       hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "reading the batch headers");
  *status = ACBM_OK;
  for (uint32_t v : st)
    if (v) *status = ACBM_E_TIMEOUT;
  return ACBM_OK;
}

int acbm_batch_graph_launch(acbm_batch_graph* gr, void* stream) {
  if (!gr || !gr->exec) return fail(ACBM_E_INVAL, "graph is NULL");
  hipError_t e = hipGraphLaunch(gr->exec, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? ACBM_OK : hip_fail(e, "launching the batch graph");
}

int acbm_batch_graph_destroy(acbm_batch_graph* gr) {
  if (!gr) return fail(ACBM_E_INVAL, "graph is NULL");
  delete gr;
  return ACBM_OK;
}

}  // extern "C"
