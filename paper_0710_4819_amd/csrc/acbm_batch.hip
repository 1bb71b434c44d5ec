// acbm_batch.hip -- many sequences of uneven geometry in one call.
#include <hip/hip_runtime.h>

#include <vector>

#include "acbm_internal.h"

using namespace acbm;

namespace {

int job_ws(const acbm_job& j, size_t* bytes) {
  KGeom k;
  int rc = check_geom(&j.geom, &k);
  if (rc) return rc;
  if (j.nframes < 2) return fail(ACBM_E_INVAL, "a job needs at least two frames");
  const uint32_t npairs = j.nframes - 1;
  switch (j.algo) {
    case ACBM_ALGO_FSBM: *bytes = align256(fsbm_ws_bytes(k, npairs)); return ACBM_OK;
    case ACBM_ALGO_PBM:
    case ACBM_ALGO_ACBM: *bytes = align256(predictive_ws_bytes(k, npairs)); return ACBM_OK;
    default: return fail(ACBM_E_INVAL, "unknown algorithm");
  }
}

}  // namespace

extern "C" {

int acbm_batch_workspace_size(const acbm_job* jobs, size_t njobs, size_t* bytes) {
  if (!jobs || !bytes) return fail(ACBM_E_INVAL, "jobs or bytes is NULL");
  size_t total = 0;
  for (size_t i = 0; i < njobs; ++i) {
    size_t b = 0;
    int rc = job_ws(jobs[i], &b);
    if (rc) return rc;
    total += b;
  }
  *bytes = total;
  return ACBM_OK;
}

int acbm_batch(const acbm_job* jobs, size_t njobs, void* ws, size_t ws_bytes, void* stream) {
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
  if ((rc = check_device())) return rc;
  char* base = static_cast<char*>(ws);
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (size_t i = 0; i < njobs; ++i) {
    const acbm_job& j = jobs[i];
    KGeom k;
    check_geom(&j.geom, &k);
    size_t b = 0;
    job_ws(j, &b);
    const uint32_t npairs = j.nframes - 1;
    if (j.algo == ACBM_ALGO_FSBM)
      rc = launch_fsbm(k, j.params, j.frames, npairs, base, b, j.out, st);
    else
      rc = launch_predictive(k, j.params, (int)j.algo, j.frames, npairs, nullptr, base, b, j.out, st);
    if (rc) return rc;
    base += b;
  }
  return ACBM_OK;
}

}  // extern "C"
