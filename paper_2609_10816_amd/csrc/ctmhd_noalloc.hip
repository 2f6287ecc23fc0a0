// ctmhd_noalloc.hip -- ctmhd_step without a caller workspace, for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).
//
// The workspace of the step is a fixed file-scope device array, `scratch`,
// of kScratchBytes.  Each GPU that runs this entry point holds its own copy
// of it (loaded with this translation unit's code object on that device)
// until the process ends.  Host code never passes `scratch` itself to a
// kernel or a copy: in host code the name denotes a host-side shadow, not a
// device address.  The device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and kept in g_scratch_ptr.
//
// The step itself is ctmhd_step on that memory: the same kernels, the same
// result bit for bit.  Every call on one GPU shares the array and it keeps
// the last call's contents; ctmhd_step clears what must start at zero (its
// dt slots, stop flag and flag counters) with a kernel at the start of every
// call.  Calls that overlap on one GPU (different host threads or streams
// without ordering between them) race on the array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ctmhd.h"

// one error message per host thread, shared with the other entry points
extern thread_local char g_err[256];

namespace {

constexpr size_t kScratchBytes = size_t(256) << 20;  // 256 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

int fail_na(int code, const char* msg) {
  snprintf(g_err, sizeof(g_err), "%s", msg);
  return code;
}

// Device address of this device's `scratch`, looked up on the first call on
// the device (with it current) and kept for later calls.
int scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail_na(CTMHD_EHIP, "ctmhd_step_noalloc: no current HIP device");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      snprintf(g_err, sizeof(g_err), "ctmhd_step_noalloc: hipGetSymbolAddress failed (%s)",
               hipGetErrorString(e));
      return CTMHD_EHIP;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return CTMHD_OK;
}

}  // namespace

extern "C" {

size_t ctmhd_noalloc_scratch_bytes(void) { return kScratchBytes; }

int ctmhd_step_noalloc(const ctmhd_params* p, const ctmhd_box* box, double* const cons[5],
                       double* const bface[3], int nsteps, const double* dt_fixed,
                       double* dt_out, int64_t* diag, void* stream) {
  g_err[0] = 0;
  const size_t need = ctmhd_workspace_bytes(p, box, 1);
  if (need == 0) return CTMHD_EARG;  // bad params or box; g_err says which
  if (need > kScratchBytes) {
    snprintf(g_err, sizeof(g_err),
             "ctmhd_step_noalloc: this box needs %zu bytes of scratch, more than the %zu bytes "
             "(256 MiB) the entry point holds per GPU; use ctmhd_step with a workspace",
             need, kScratchBytes);
    return CTMHD_EARG;
  }
  if (nsteps == 0) return ctmhd_step(p, box, cons, bface, 0, dt_fixed, dt_out, diag, nullptr, 0,
                                     stream);
  void* ptr = nullptr;
  int rc = scratch_address(&ptr);
  if (rc) return rc;
  return ctmhd_step(p, box, cons, bface, nsteps, dt_fixed, dt_out, diag, ptr, kScratchBytes,
                    stream);
}

}  // extern "C"
