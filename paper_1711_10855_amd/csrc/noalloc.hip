// Device scratch of the allocation-free batched entry point
// (fdas_convolve_batch_noalloc): the batch descriptor table and the work
// counter live in one file-scope device array instead of memory the plan
// allocates. Each GPU holds its own copy of the array at its own address;
// the host never uses the array's name as a device address, only the
// address hipGetSymbolAddress returns for the current device.
#include <hip/hip_runtime.h>

#include <mutex>

#include "noalloc.hpp"
#include "plan.hpp"

namespace fdas {

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};
}  // namespace

int noalloc_scratch(int device, void **out) {
  if (device < 0 || device >= kMaxDevices)
    return set_error(FDAS_ERR_UNSUPPORTED, "device %d beyond the %d the scratch table holds",
                     device, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[device]) {
    // the caller has made `device` current
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_error(e, "hipGetSymbolAddress(scratch)");
    if (!p) return set_error(FDAS_ERR_DEVICE, "hipGetSymbolAddress(scratch) returned null");
    g_scratch[device] = p;
  }
  *out = g_scratch[device];
  return FDAS_OK;
}

__global__ void desc_upload_kernel(DescChunk c, SeriesDesc *dst) {
  const int i = threadIdx.x;
  if (i < c.n) dst[c.first + i] = c.d[i];
}

hipError_t launch_desc_upload(const DescChunk &c, SeriesDesc *dst, hipStream_t s) {
  hipLaunchKernelGGL(desc_upload_kernel, dim3(1), dim3(kDescChunk), 0, s, c, dst);
  return hipGetLastError();
}

}  // namespace fdas
