// Allocation-free variant of kfac_rand_eig for callers that cannot allocate device memory
// (code under hipGraph capture, tight serving loops, harnesses that forbid hipMalloc).
//
// Its scratch is one file-scope device array of fixed size: every GPU the library runs on
// holds its own copy of it from module load until the process ends.  The array's host-side
// name is not a device address, so its address is looked up with hipGetSymbolAddress once
// per device (with that device current) and only that pointer is handed to the kernels.
// Calls that overlap on one GPU share the array and race; calls on one stream are ordered.
// The path is the one kfac_rand_eig runs, whose kernels write every scratch word before
// reading it, so the contents a previous call left behind do not matter.
#include <hip/hip_runtime.h>
#include <mutex>
#include "kfac.h"

namespace {

constexpr size_t kScratchBytes = KFAC_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_lock;
void* g_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (nullptr on failure).
void* scratch_on_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_lock);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" {

kfac_status kfac_rand_eig_noalloc(const float* F, int64_t d, int64_t ldf, const uint16_t* F_bf16, int64_t ldfb,
                                  int64_t r, int64_t p, int q, uint64_t seed, uint64_t stream_id,
                                  uint32_t inversion_index, kfac_variant v, kfac_precision prec, float* U,
                                  int64_t ldu, float* D, int32_t* dev_status, kfac_stream_t stream) {
  if (d < 1 || r < 1 || r > d || p < 0 || q < 0) return KFAC_EINVAL;
  const size_t need = kfac_rand_eig_workspace(d, r, p, q, v, prec);
  if (need == 0) return KFAC_EINVAL;
  if (need > kScratchBytes) return KFAC_ESCRATCH;
  void* ws = scratch_on_current_device();
  if (!ws) return KFAC_EHIP;
  return kfac_rand_eig(F, d, ldf, F_bf16, ldfb, r, p, q, seed, stream_id, inversion_index, v, prec, U, ldu, D, ws,
                       kScratchBytes, dev_status, stream);
}

}  // extern "C"
