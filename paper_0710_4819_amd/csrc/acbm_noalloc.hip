// acbm_noalloc.hip -- ACBM for one frame pair with no allocation at all.
//
// acbm_acbm_frame takes its scratch (dependency-wait header, row order,
// published vector words, frame-pointer and job tables) from a workspace the
// caller allocates.  Callers that cannot allocate (code under stream
// capture, tight serving loops, hosts that forbid hipMalloc) use
// acbm_acbm_frame_noalloc instead: the same kernels with the scratch taken
// from a fixed device array of this library, one per GPU, kept until the
// process ends.  Every call on a GPU uses that GPU's array, so calls that
// overlap on one GPU race; the kernels initialise everything they read from
// it (the set-up kernel resets the header and the words, the job kernel
// writes the tables), so nothing needs clearing between calls.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "acbm_internal.h"

using namespace acbm;

// Scratch of the allocation-free entry point: 2 MiB covers frames of up to
// about 520,000 blocks (every 16x16 frame the library takes, and 8x8 frames
// up to 4096x8192).
static constexpr size_t kNoallocScratchBytes = (size_t)2 << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch`, per GPU

__global__ void k_copy_status(const WsHeader* __restrict__ hdr, uint32_t* __restrict__ out) {
  if (threadIdx.x == 0) out[0] = hdr->status;
}

// The device address of the current GPU's scratch array, looked up once per
// device (the array's name is only a host-side stand-in).
int scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(ACBM_E_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "looking up the scratch array");
    if (!p) return fail(ACBM_E_DEVICE, "the scratch array has no device address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return ACBM_OK;
}

}  // namespace

int acbm::noalloc_scratch_init() {
  void* p = nullptr;
  return scratch_ptr(&p);
}

extern "C" int acbm_acbm_frame_noalloc(const acbm_geom* g, const acbm_params* prm,
                                       const uint8_t* cur, const uint8_t* ref,
                                       const acbm_mv* prev_field, acbm_block_result* out,
                                       uint32_t* status, void* stream) {
  KGeom k;
  int rc = check_geom(g, &k);
  if (rc) return rc;
  if ((rc = check_params(prm, k))) return rc;
  if ((rc = check_frame_ptr(cur, "cur")) || (rc = check_frame_ptr(ref, "ref"))) return rc;
  if (!out) return fail(ACBM_E_INVAL, "out is NULL");
  const size_t need = predictive_ws_bytes(k, 1);
  if (need > kNoallocScratchBytes)
    return fail(ACBM_E_NOMEM, "frame needs " + std::to_string(need) +
                                  " bytes of scratch; the allocation-free entry point has " +
                                  std::to_string(kNoallocScratchBytes));
  if ((rc = check_device())) return rc;
  void* ws = nullptr;
  if ((rc = scratch_ptr(&ws))) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const uint8_t* frames[2] = {ref, cur};
  if ((rc = launch_predictive(k, *prm, ACBM_ALGO_ACBM, frames, 1, prev_field, ws,
                              kNoallocScratchBytes, out, st)))
    return rc;
  if (status) {
    hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, st,
                       static_cast<const WsHeader*>(ws), status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "copying the run status");
  }
  return ACBM_OK;
}
