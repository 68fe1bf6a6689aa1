// fossils_solve_noalloc: FOSSILS with every device buffer carved from one file-scope device array
// (`scratch`), for callers that cannot allocate device memory (code under stream capture, tight
// serving loops, harnesses that forbid allocation).
//
// Each GPU the library runs on holds its own copy of `scratch` (FS_NOALLOC_SCRATCH_BYTES) from the
// moment the library's code is loaded on it until the process ends.  In host code the array's name
// is only a host-side handle: its device address comes from hipGetSymbolAddress, taken once per
// device (with that device current) on the entry point's first call there, and only that pointer is
// handed to kernels and copies.  Every call on one GPU uses the same array, so calls that overlap
// in time on one GPU (two threads, or two streams in flight) race; each call starts its kernels
// from buffers it initializes itself (barrier counters, sums and flags are cleared by fill kernels
// at every use), so nothing carries over from the previous call's contents.
#include <mutex>

#include "../../include/fossils.h"
#include "common.hpp"
#include "context.hpp"

static __device__ __align__(256) unsigned char scratch[FS_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device `dev` (looked up once per device)
fs_status scratch_ptr(int dev, unsigned char** out) {
  if (dev < 0 || dev >= kMaxDevices) return FS_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      fs_set_last_hip_error(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)", __FILE__,
                            __LINE__);
      return FS_ERR_DEVICE;
    }
    g_scratch_ptr[dev] = (unsigned char*)p;
  }
  *out = g_scratch_ptr[dev];
  return FS_OK;
}

}  // namespace

extern "C" {

fs_status fossils_solve_noalloc(fs_context ctx, int64_t m, int32_t n, const double* A, int64_t lda, const double* b,
                                double* x, const fs_options* opts, fs_info* info) {
  if (!ctx) return FS_ERR_INVALID_ARG;
  FS_TRY(fs_validate_problem(m, n, A, lda, b, x));
  fs_options o;
  if (opts) o = *opts;
  else FS_TRY(fs_options_default(m, n, &o));
  o.overlap_svd = 0;   // the second stream and its event would be created on first use
  o.graph_sweeps = 0;  // instantiating a graph allocates
  FS_TRY(fs_validate_options(m, n, o));
  if (fs_carve_workspace(ctx->ws, nullptr, m, n, o, ctx->num_cu) > FS_NOALLOC_SCRATCH_BYTES) return FS_ERR_TOO_LARGE;
  FS_HIP(hipSetDevice(ctx->device));
  unsigned char* base = nullptr;
  FS_TRY(scratch_ptr(ctx->device, &base));
  return fs_fossils_solve_fixed(ctx, base, FS_NOALLOC_SCRATCH_BYTES, m, n, A, lda, b, x, o, info);
}
}  // extern "C"
