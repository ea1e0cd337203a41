// Z^* y without a caller workspace: the adjoint's scratch (its per-tile
// partial inner products, or the stacked operand of the decompress-then-GEMM
// path) lives in a file-scope device array of fixed size, one per GPU, held
// until the process ends.  For callers that cannot allocate device memory.
#include <mutex>

#include "tv_internal.h"

// Device array; in host code this name is a stand-in for the symbol, never a
// device address: only the pointer hipGetSymbolAddress returns is used.
static __device__ __align__(256) unsigned char scratch[TV_STATIC_SCRATCH_BYTES];

namespace {

constexpr size_t kScratchBytes = (size_t)TV_STATIC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

std::mutex g_lock;
void* g_ptr[kMaxDevices] = {};

// The calling thread's current device's copy of the array (looked up once
// per device, with that device current).
tv_status scratch_ptr(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return tv::hip_error(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return tv::set_error(TV_ERR_NOT_SUPPORTED, "device index");
  std::lock_guard<std::mutex> g(g_lock);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return tv::hip_error(e, "hipGetSymbolAddress(scratch)");
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return TV_OK;
}

}  // namespace

extern "C" tv_status tv_rmatvec_noalloc(tv_plan p, const void* y, int64_t ldy, int32_t nrhs,
                                        void* x, int64_t ldx, void* stream) {
  tv::clear_error();
  if (!p) return tv::set_error(TV_ERR_INVALID_ARG, "plan is NULL");
  size_t need = 0;
  tv_status st = tv_workspace_bytes(p, 1, nrhs, &need);
  if (st != TV_OK) return st;
  if (need > kScratchBytes) {
    char buf[160];
    snprintf(buf, sizeof buf,
             "the adjoint needs %zu bytes of scratch; the static scratch holds %zu "
             "(use tv_rmatvec with a workspace)", need, kScratchBytes);
    return tv::set_error(TV_ERR_WORKSPACE, buf);
  }
  void* ws = nullptr;
  if ((st = scratch_ptr(&ws)) != TV_OK) return st;
  // every scratch entry the kernels read is written earlier in the same call
  return tv_rmatvec(p, y, ldy, nrhs, x, ldx, ws, kScratchBytes, stream);
}
