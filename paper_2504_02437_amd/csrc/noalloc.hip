// gs_insert_distance_noalloc: the distance-tested insertion of Eq. 7 with
// its per-candidate scratch in a file-scope device array instead of a
// caller buffer, for callers that cannot allocate device memory.
//
// The array lives in this library's code object: every GPU the library runs
// on holds its own copy (kNoAllocCandidates x 8 bytes) until the process
// ends.  Host code never passes the array's name to a kernel (on the host
// it is only a stand-in symbol); the device address of each GPU's copy is
// looked up once per device with hipGetSymbolAddress, with that device
// current, and that address is what the kernels receive.  Every call on a
// GPU shares its copy: calls that overlap on one GPU race.  The insertion
// kernels clear the candidates' slots (a fill kernel, no memset) before
// using them, so nothing carries over from a previous call.

#include <mutex>

#include "gs_internal.h"

namespace gs {
namespace {

constexpr int kNoAllocCandidates = 65536;   // 9 x n_pts for n_pts <= 7281
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned long long scratch[kNoAllocCandidates];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of `scratch` (current device).
int scratch_address(void** out) {
  int dev = -1;
  if (int rc = check_hip(hipGetDevice(&dev), "hipGetDevice")) return rc;
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d beyond the %d this entry point tracks", dev,
              kMaxDevices);
    return GS_E_INVALID;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (int rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)),
                           "hipGetSymbolAddress"))
      return rc;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GS_OK;
}

}  // namespace
}  // namespace gs

using namespace gs;

extern "C" GS_API int gs_insert_distance_noalloc(
    gs_params* params, gs_params* adam_m, gs_params* adam_v,
    const gs_camera* cam, int32_t width, int32_t height, const float* kf_rgb,
    const float* pts_uvd, int32_t n_pts, float tau, int32_t centre_only,
    const float* mlp_out, int32_t* n_inserted_dev, int32_t* status_dev,
    void* stream) {
  const long long cand = (long long)n_pts * (centre_only ? 1 : 9);
  if (n_pts < 0 || cand > kNoAllocCandidates) {
    set_error("insert_distance_noalloc: %lld candidates exceed the %d the "
              "static scratch holds", cand, kNoAllocCandidates);
    return GS_E_CAPACITY;
  }
  void* ptr = nullptr;
  if (int rc = scratch_address(&ptr)) return rc;
  return gs_insert_distance(params, adam_m, adam_v, cam, width, height, kf_rgb,
                            pts_uvd, n_pts, tau, centre_only, mlp_out,
                            (uint64_t*)ptr, n_inserted_dev, status_dev,
                            stream);
}
