// Static device scratch of the allocation-free mutation entry point
// (rjsmc_mutate_noalloc).
//
// The per-particle scratch of a mutation sweep (proposal mask, move type, gradient
// validity, adaptive-birth log correction, evaluation order and its counting-sort
// counters) lives in one file-scope device array instead of the context's workspace, so
// the call needs no device allocation at any time.  Each GPU the library runs on holds
// its own copy of the array until the process ends.  In host code the array's name is
// not a device address: its address on a device is obtained once per device, with that
// device current, by hipGetSymbolAddress (at context creation) and only that address is
// handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rjsmc_internal.h"

namespace {
// [lq: 8 B][mask][type][gvalid][perm: 4 B each] per particle, then the sort counters;
// every block starts on a 256-byte boundary.
constexpr size_t kCap = RJSMC_NOALLOC_MAX_PARTICLES;
constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
constexpr size_t kOffLq = 0;
constexpr size_t kOffMask = align256(kOffLq + sizeof(double) * kCap);
constexpr size_t kOffType = align256(kOffMask + sizeof(int32_t) * kCap);
constexpr size_t kOffGvalid = align256(kOffType + sizeof(int32_t) * kCap);
constexpr size_t kOffPerm = align256(kOffGvalid + sizeof(int32_t) * kCap);
constexpr size_t kOffCnt = align256(kOffPerm + sizeof(int32_t) * kCap);
constexpr size_t kScratchBytes = align256(kOffCnt + sizeof(int) * 2 * rjsmc::kMaxLayers);
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace rjsmc {

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void *g_addr[kMaxDevices] = {};
hipError_t g_status[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mutex);
  if (g_addr[device]) return hipSuccess;
  int current = -1;
  hipError_t e = hipGetDevice(&current);
  if (e != hipSuccess) return e;
  if (current != device) return hipErrorInvalidDevice;   // the caller makes `device` current
  void *ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) (void)hipGetLastError();   // leave no error behind for later launches
  if (e == hipSuccess && !ptr) e = hipErrorInvalidSymbol;
  g_status[device] = e;
  if (e != hipSuccess) return e;
  g_addr[device] = ptr;
  return hipSuccess;
}

hipError_t static_scratch_status(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mutex);
  return g_addr[device] ? hipSuccess : (g_status[device] != hipSuccess ? g_status[device] : hipErrorNotInitialized);
}

bool static_scratch(int device, MutateWorkspace *ws) {
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mutex);
    if (device >= 0 && device < kMaxDevices) base = g_addr[device];
  }
  if (!base) return false;
  unsigned char *b = static_cast<unsigned char *>(base);
  ws->lq = reinterpret_cast<double *>(b + kOffLq);
  ws->mask = reinterpret_cast<int32_t *>(b + kOffMask);
  ws->type = reinterpret_cast<int32_t *>(b + kOffType);
  ws->gvalid = reinterpret_cast<int32_t *>(b + kOffGvalid);
  ws->perm = reinterpret_cast<int32_t *>(b + kOffPerm);
  ws->cnt = reinterpret_cast<int *>(b + kOffCnt);
  ws->n = (int64_t)kCap;
  return true;
}

}  // namespace rjsmc
