// Allocation-free deterministic sum (GrM_reduce_dense_noalloc, declared in
// include/nbgrb.h) for callers that cannot allocate device memory: code
// under stream capture, tight serving loops, hosts that forbid it.
//
// It runs the same two-level reduction kernel as GrB_Vector_reduce_FP64
// (per-workgroup FP64 partials, the last workgroup adds them in workgroup
// order), but its scratch -- the partials and the last-workgroup ticket --
// lives in the file-scope device array `scratch` below instead of buffers
// from the library's allocator.  Every GPU holds its own copy of the array
// at its own address; the host learns that address once per device with
// hipGetSymbolAddress (noalloc_setup, called from GrB_init) and only ever
// passes that address to kernels: the array's name in host code is a
// host-side stand-in, not a device address.
//
// All calls on one device share its array: two calls that overlap on that
// device (different streams, or different host threads) race on the
// partials and the ticket.  The kernel's last workgroup resets the ticket,
// so consecutive calls in stream order need no clearing.
#include <hip/hip_runtime.h>

#include "abi_util.h"

// REDUCE_GRID FP64 partials, then the ticket in a 256-byte slot of its own.
constexpr int SCRATCH_PARTIALS = nbgrb::REDUCE_GRID;
constexpr int SCRATCH_DOUBLES = SCRATCH_PARTIALS + 256 / (int)sizeof(double);

static __device__ __align__(256) double scratch[SCRATCH_DOUBLES];

namespace nbgrb {

namespace {

constexpr int MAX_DEVICES = 64;
double* g_scratch_dev[MAX_DEVICES] = {};  // device address of `scratch`, per device

}  // namespace

// Looks up this device's copy of `scratch` (the device must be current) and
// zeroes its ticket with a kernel.  Idempotent per device.
void noalloc_setup(int device, hipStream_t s) {
  if (device < 0 || device >= MAX_DEVICES) fail(GrB_PANIC, "device index beyond the scratch table");
  if (g_scratch_dev[device]) return;
  double* d = nullptr;
  hip_check(hipGetSymbolAddress((void**)&d, HIP_SYMBOL(scratch)), "scratch symbol address");
  if (!d) fail(GrB_PANIC, "scratch symbol has no device address");
  hip_check(launch_zero(d + SCRATCH_PARTIALS, 256, s), "zero scratch ticket");
  hip_check(hipStreamSynchronize(s), "sync");
  g_scratch_dev[device] = d;
}

}  // namespace nbgrb

using namespace nbgrb;

extern "C" {

GrB_Info GrM_reduce_dense_noalloc(double* sum_dev, const void* x_dev, GrB_Type type, GrB_Index n) {
  API_BEGIN
  require_init();
  need(sum_dev, "sum_dev");
  need(type, "type");
  const int t = type->code;
  if (t != T_FP32 && t != T_FP64) fail(GrB_DOMAIN_MISMATCH, "the sum takes FP32 or FP64 values");
  if (n > (GrB_Index)GRM_NOALLOC_MAX_N) fail(GrB_INVALID_VALUE, "n beyond GRM_NOALLOC_MAX_N");
  if (n > 0) need(x_dev, "x_dev");
  Ctx& c = ctx();
  double* d = (c.device >= 0 && c.device < MAX_DEVICES) ? g_scratch_dev[c.device] : nullptr;
  if (!d) fail(GrB_PANIC, "scratch of this device was not set up by GrB_init");
  // the reduction launches at most REDUCE_GRID workgroups, one partial each
  static_assert(REDUCE_GRID <= SCRATCH_PARTIALS, "scratch holds one partial per workgroup");
  RedScratch scr{d, (unsigned*)(d + SCRATCH_PARTIALS)};
  ReduceOut out{sum_dev, nullptr};
  hip_check(launch_reduce((int64_t)n, Operand{x_dev, t, 0.0}, 0, Operand{nullptr, T_FP64, 0.0}, 0, out, scr,
                          nullptr, c.stream),
            "reduce");
  launch_mark(false);
  API_END
}

}  // extern "C"
