// Workspace of the allocation-free fixed-resolution render: a static device
// array (one copy per GPU, held until the process ends) instead of context
// memory, so a call needs no device allocation.  Host code reaches the array
// only through the address hipGetSymbolAddress returns for each device.
#include <mutex>

#include "air_common.h"

namespace air {

namespace {

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEVICES] = {};

struct ViewArg {
  DevView v[AIR_NOALLOC_MAX_VIEWS];
  int n;
};

// counters cleared with plain stores (a memset node would not replay
// correctly under graph capture) and the view table written from the
// kernel argument
__global__ __launch_bounds__(256) void k_noalloc_setup(ViewArg va, DevView* views, unsigned long long* ctr) {
  for (int k = threadIdx.x; k < CTR_COUNT; k += blockDim.x) ctr[k] = 0;
  if ((int)threadIdx.x < va.n) views[threadIdx.x] = va.v[threadIdx.x];
}

}  // namespace

hipError_t noalloc_init(int device, void** out) {
  *out = nullptr;
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[device]) {
    // the caller has made `device` current: the address is that device's copy
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_ptr[device] = p;
  }
  *out = g_ptr[device];
  return hipSuccess;
}

hipError_t launch_noalloc_setup(const DevView* views, int n, void* scratch_ptr, hipStream_t s) {
  if (n < 0 || n > AIR_NOALLOC_MAX_VIEWS) return hipErrorInvalidValue;
  ViewArg va;
  for (int k = 0; k < n; ++k) va.v[k] = views[k];
  va.n = n;
  unsigned char* base = static_cast<unsigned char*>(scratch_ptr);
  hipLaunchKernelGGL(k_noalloc_setup, dim3(1), dim3(256), 0, s, va,
                     reinterpret_cast<DevView*>(base + NOALLOC_VIEWS_OFF),
                     reinterpret_cast<unsigned long long*>(base + NOALLOC_CTR_OFF));
  return hipGetLastError();
}

}  // namespace air
