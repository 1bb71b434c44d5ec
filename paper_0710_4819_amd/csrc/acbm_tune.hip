// acbm_tune.hip -- measured choice of the window-search plan.
//
// The cost model of the search planner ranks the row blockings R well but
// not exactly (LDS bank conflicts, occupancy and the epilogue vary with R and
// p); acbm_autotune times every candidate on the device instead and records
// the fastest.  The search result never depends on R (every plan computes
// the same exact SADs), so tuning only moves time.  With ACBM_TUNE_CACHE
// naming a file, each measured plan is appended to it and later processes
// take it from there instead of timing again.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "acbm_internal.h"

using namespace acbm;

namespace {

// Deterministic pseudo-random bytes (an integer hash of the index), so that
// the timed search sees textured data rather than a constant frame.
__global__ void k_fill_hash(uint8_t* __restrict__ p, size_t n, uint32_t seed) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x) {
    uint32_t x = (uint32_t)i * 0x9E3779B1u ^ seed;
    x ^= x >> 15;
    x *= 0x85EBCA77u;
    x ^= x >> 13;
    p[i] = (uint8_t)(x >> 24);
  }
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  ~Events() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

}  // namespace

extern "C" int acbm_autotune(const acbm_geom* g, uint32_t* best_rows, float* best_ms,
                             void* stream) {
  KGeom k;
  int rc = check_geom(g, &k);
  if (rc) return rc;
  if ((rc = check_device())) return rc;
  // 8x8 blocks on an even grid of blocks search in 2x2 tiles: tune those
  const int tile = tiles_apply(k) ? 2 : 1;
  SearchPlan cached{0, 0, 0};
  float cached_ms = 0;
  if (cached_plan(k.bw, k.bh, k.p, tile, &cached, &cached_ms)) {
    // measured by an earlier process on this architecture: reuse it
    if (best_rows) *best_rows = (uint32_t)cached.R;
    if (best_ms) *best_ms = cached_ms;
    return ACBM_OK;
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t fb = align256((size_t)k.pitch * k.height);
  const size_t wsb = fsbm_ws_bytes(k, 1);
  DevBuf buf;
  hipError_t e = hipMalloc(&buf.p, 2 * fb + wsb);
  if (e != hipSuccess) return hip_fail(e, "allocating autotune scratch");
  uint8_t* frames = static_cast<uint8_t*>(buf.p);
  char* ws = static_cast<char*>(buf.p) + 2 * fb;
  hipLaunchKernelGGL(k_fill_hash, dim3(1024), dim3(256), 0, st, frames, 2 * fb, 0x5EEDu);
  if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "filling autotune frames");
  const uint8_t* fp[2] = {frames, frames + fb};
  BlockRec* recs = reinterpret_cast<BlockRec*>(ws + fsbm_recs_offset());
  uint16_t* ovf = reinterpret_cast<uint16_t*>(ws + fsbm_ovf_offset(k, 1));
  const uint32_t slack = 8u * (uint32_t)(rate_max(k.p) - 2);
  Events ev;
  if ((e = hipEventCreate(&ev.a)) != hipSuccess || (e = hipEventCreate(&ev.b)) != hipSuccess)
    return hip_fail(e, "creating autotune events");
  SearchPlan best{0, 0, 0};
  float best_t = 0;
  for (int R : {1, 2, 3, 4, 5, 6, 8, 11, 16}) {
    const SearchPlan pl = plan_search_model(k.bw, k.bh, k.p, R, tile);
    if (!pl.R) continue;
    if ((rc = launch_search_plan(k, pl, fp, 1, recs, ovf, slack, st))) return rc;  // warm-up
    // one timed launch sizes the run: enough launches for about 3 ms, so that a
    // 20-microsecond search is not decided by the noise of three launches
    float one = 0;
    if ((e = hipEventRecord(ev.a, st)) != hipSuccess) return hip_fail(e, "timing");
    if ((rc = launch_search_plan(k, pl, fp, 1, recs, ovf, slack, st))) return rc;
    if ((e = hipEventRecord(ev.b, st)) != hipSuccess) return hip_fail(e, "timing");
    if ((e = hipEventSynchronize(ev.b)) != hipSuccess) return hip_fail(e, "timing");
    if ((e = hipEventElapsedTime(&one, ev.a, ev.b)) != hipSuccess) return hip_fail(e, "timing");
    const int reps = std::max(5, std::min(200, (int)(3.0f / std::max(one, 1e-3f))));
    if ((e = hipEventRecord(ev.a, st)) != hipSuccess) return hip_fail(e, "timing");
    for (int i = 0; i < reps; ++i)
      if ((rc = launch_search_plan(k, pl, fp, 1, recs, ovf, slack, st))) return rc;
    if ((e = hipEventRecord(ev.b, st)) != hipSuccess) return hip_fail(e, "timing");
    if ((e = hipEventSynchronize(ev.b)) != hipSuccess) return hip_fail(e, "timing");
    float ms = 0;
    if ((e = hipEventElapsedTime(&ms, ev.a, ev.b)) != hipSuccess) return hip_fail(e, "timing");
    ms /= (float)reps;
    if (!best.R || ms < best_t) {
      best = pl;
      best_t = ms;
    }
  }
  if (!best.R) return fail(ACBM_E_UNSUPPORTED, "search window does not fit in LDS");
  save_tuned_plan(k.bw, k.bh, k.p, best, best_t);
  if (best_rows) *best_rows = (uint32_t)best.R;
  if (best_ms) *best_ms = best_t;
  return ACBM_OK;
}
