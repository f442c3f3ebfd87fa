// y = A x through a file-scope device buffer instead of the context's own
// staging vectors, for callers that must not allocate device memory during
// the call.
//
// The product is cpr_spmv's: x (natural order) is permuted into the
// colour-split order, multiplied by the block 7-point Jacobian with the
// border of the rate-controlled wells, and permuted back into y.  The two
// colour-split staging vectors live in `scratch`, a static array of
// NOALLOC_SCRATCH_DOUBLES doubles that every GPU the library runs on holds
// until the process ends.  Its device address is looked up once per device
// (hipGetSymbolAddress, with that device current) and kept; host code never
// passes the array's name itself.  Calls on one GPU share the array: calls
// that overlap on one GPU (two streams, two threads) race.  Nothing in the
// array needs to start at zero: every staging entry is written before it is
// read.
#include <mutex>

#include "internal.h"

namespace {

constexpr size_t NOALLOC_SCRATCH_DOUBLES = size_t(1) << 23;   // 64 MiB
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

std::mutex g_mu;
double* g_ptr[MAX_DEVICES] = {};

// Device address of `scratch` on the device of `stream` (the current device
// for the null stream), looked up once per device with that device current.
hipError_t scratch_ptr(hipStream_t stream, double** out) {
  int dev = 0, cur = 0;
  hipError_t e = stream ? hipStreamGetDevice(stream, &dev) : hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    if ((e = hipGetDevice(&cur)) != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" long long cpr_spmv_noalloc_max_unknowns(void) { return (long long)(NOALLOC_SCRATCH_DOUBLES / 2); }

extern "C" int cpr_spmv_noalloc(cpr_ctx_t* ctx, const double* x, double* y) {
  if (!ctx) return CPR_EINVAL;
  if (!x || !y) return set_err(ctx, CPR_EINVAL, "null argument");
  const long len = vec_len(ctx);
  if ((size_t)len > NOALLOC_SCRATCH_DOUBLES / 2)
    return set_err(ctx, CPR_EINVAL,
                   "cpr_spmv_noalloc: " + std::to_string(len) + " unknowns exceed its static buffer of " +
                       std::to_string(NOALLOC_SCRATCH_DOUBLES / 2) + " per staging vector");
  double* base = nullptr;
  hipError_t e = scratch_ptr(ctx->stream, &base);
  if (e != hipSuccess) return set_hip_err(ctx, e, "hipGetSymbolAddress(scratch)");
  double* xin = base;
  double* yout = base + NOALLOC_SCRATCH_DOUBLES / 2;
  CPR_TRY(vec_nat_to_cs(ctx, x, xin));
  system_spmv(ctx, xin, yout, nullptr);
  CPR_TRY(vec_cs_to_nat(ctx, yout, y));
  return launch_check(ctx, "cpr_spmv_noalloc");
}
