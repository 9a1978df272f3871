// pulsar_fwd_noalloc: the forward pass for callers that cannot allocate
// device memory (code under HIP graph capture, serving loops). It runs the
// same kernels as pulsar_fwd with a file-scope device array as the workspace.
//
// In host code the array's name is a host-side stand-in, not a device
// address: the address each device holds it at is taken once per device with
// hipGetSymbolAddress (with that device current) and only that pointer is
// passed to kernels.
#include <mutex>

#include "pulsar_internal.h"

namespace pulsar {
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // PULSAR_NOALLOC_SCRATCH_BYTES
static_assert(kScratchBytes == PULSAR_NOALLOC_SCRATCH_BYTES, "header and library agree");
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// The current device's address of `scratch` (resolved on its first use there).
int scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip(e);
  if (dev < 0 || dev >= kMaxDevices) return PULSAR_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return fail_hip(e);
    if (!p) return PULSAR_ERR_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PULSAR_OK;
}

}  // namespace
}  // namespace pulsar

extern "C" int pulsar_fwd_noalloc(const float* pos, const float* radius, const float* opacity,
                                  const float* payload, int32_t n, int32_t C,
                                  const float* background, const pulsar_camera_t* cam,
                                  const pulsar_params_t* params, float* image, float* aux,
                                  void* stream) {
  if (!cam) return PULSAR_ERR_INVALID_ARGUMENT;
  const size_t need = pulsar_workspace_size(n, cam->width, cam->height, C, params);
  // an invalid request plans nothing: pulsar_fwd names the error, on the host
  if (need == 0)
    return pulsar_fwd(pos, radius, opacity, payload, n, C, background, cam, params, image, aux,
                      nullptr, 0, stream);
  if (need > pulsar::kScratchBytes) return PULSAR_ERR_SCRATCH;
  void* ws = nullptr;
  const int rc = pulsar::scratch_address(&ws);
  if (rc != PULSAR_OK) return rc;
  return pulsar_fwd(pos, radius, opacity, payload, n, C, background, cam, params, image, aux, ws,
                    pulsar::kScratchBytes, stream);
}
