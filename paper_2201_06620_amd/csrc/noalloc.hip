// Block tensordot without any allocation: rn_block_tensordot_noalloc runs
// the same plan and kernels as rn_block_tensordot, with the workspace taken
// from a fixed device array compiled into the library instead of a caller
// buffer.  Every GPU the library runs on holds its own copy of the array
// (RN_NOALLOC_SCRATCH_BYTES) until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "rn_internal.hpp"

namespace rn {

static __device__ __align__(256) unsigned char scratch[RN_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {nullptr};  // device address of `scratch`, per device
}  // namespace

// Called by rn_create with `device` current: looks up this device's address
// of the array once (the host-side name of a __device__ variable is not a
// device address, so kernels and copies are only ever given this pointer).
rn_status noalloc_init(int device) {
  if (device < 0 || device >= kMaxDevices) return fail(RN_ERR_INVALID, "device index too large");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return RN_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(RN_ERR_HIP, std::string("hipGetSymbolAddress (no-alloc scratch): ") +
                                hipGetErrorString(e));
  g_ptr[device] = p;
  return RN_OK;
}

static void* noalloc_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ptr[device];
}

}  // namespace rn

using namespace rn;

extern "C" rn_status rn_block_tensordot_noalloc(rn_handle h, const rn_tensor* A,
                                                const rn_tensor* B, int32_t k,
                                                const int32_t* axesA, const int32_t* axesB,
                                                rn_tensor* C, rn_mode mode, void* stream) {
  if (!h) return fail(RN_ERR_INVALID, "null handle");
  TdPlan P;
  rn_status st;
  if ((st = plan_tensordot(A, B, k, axesA, axesB, mode, &P, true, &h->split, true)) != RN_OK)
    return st;
  if ((st = check_c(P, C)) != RN_OK) return st;
  if (!A->data || !B->data) return fail(RN_ERR_INVALID, "null operand data");
  if (C->data == A->data || C->data == B->data) return fail(RN_ERR_INVALID, "C aliases an operand");
  if (P.ws_bytes > RN_NOALLOC_SCRATCH_BYTES)
    return fail(RN_ERR_WORKSPACE, "needs " + std::to_string(P.ws_bytes) +
                                      " bytes of workspace; the no-alloc scratch holds " +
                                      std::to_string((long long)RN_NOALLOC_SCRATCH_BYTES));
  hipError_t e = hipSetDevice(h->device);
  if (e != hipSuccess) return fail(RN_ERR_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e));
  void* ws = noalloc_ptr(h->device);
  if (!ws) return fail(RN_ERR_HIP, "no-alloc scratch not set up on this device");
  // No kernel timing here: the timing events come from a pool that grows.
  return enqueue_tensordot(P, A, B, C, ws, static_cast<hipStream_t>(stream), nullptr,
                           tuned_tile(h, P.mode, P.mbits, P.nbits, P.kbits));
}
