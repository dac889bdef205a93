// The adjoint evaluation for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc): xg_eval_adjoint with its workspace taken from a
// fixed device array of this library instead of a caller's buffer.
//
// The array is a file-scope device variable, so every GPU the library runs
// on holds its own copy (XG_NOALLOC_SCRATCH_BYTES) from its set-up until
// the process ends.  On the host the array's name is only a stand-in for
// the symbol: its device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and only that address is
// ever passed to kernels.  Every call on one GPU shares that GPU's array,
// so calls that overlap on one GPU (two streams, two threads) race.  The
// adjoint kernels write every workspace element before they read it, so
// the array needs no clearing between calls.
#include <cstdint>
#include <cstdio>
#include <mutex>
#include <string>

#include <hip/hip_runtime.h>

#include "xg_internal.h"
#include "xg_program.h"

static __device__ __align__(256) unsigned char scratch[XG_NOALLOC_SCRATCH_BYTES];

namespace xg {

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// Device address of `scratch` on the current device, looked up on the
// first call for that device.  The first lookup may load this library's
// device code onto the GPU (which allocates the array); later calls only
// read the table.
bool noalloc_scratch(void** ptr, std::string& err) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) { err = "hipGetDevice failed"; return false; }
  if (dev < 0 || dev >= kMaxDevices) { err = "device index beyond the library's table"; return false; }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return false;
    }
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return true;
}

}  // namespace xg

using namespace xg;

extern "C" xg_status xg_eval_adjoint_noalloc(xg_program* p, int64_t n, const void* const* d_in,
                                             const int64_t* ld_in, const void* const* d_out_bar,
                                             const int64_t* ld_out_bar, void* const* d_out,
                                             const int64_t* ld_out, void* const* d_in_bar,
                                             const int64_t* ld_in_bar, void* stream) {
  void* ws = nullptr;
  std::string err;
  if (!noalloc_scratch(&ws, err)) { set_error(err); return XG_EDEVICE; }
  return eval_adjoint_loaded(p, n, d_in, ld_in, d_out_bar, ld_out_bar, d_out, ld_out, d_in_bar,
                             ld_in_bar, ws, (size_t)XG_NOALLOC_SCRATCH_BYTES, stream);
}
