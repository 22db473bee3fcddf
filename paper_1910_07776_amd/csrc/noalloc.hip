// The entry point that allocates nothing: sugg_load_features with its FP64
// column-statistics partials (Section 2, Tier 1: counters normalised by the
// cycle count, then standardised per column) in a static device array of the
// library instead of a plan workspace that the first call allocates.
//
// The array exists once per GPU (each device holds its own copy from the
// moment the library's code is loaded on it until the process ends); its
// address on a device is looked up with hipGetSymbolAddress at context
// creation, with that device current, and only that address is ever given to
// kernels (in host code the array's name does not denote device memory).
#include <hip/hip_runtime.h>

#include <mutex>

#include "ctx.hpp"
#include "plan.hpp"

constexpr int64_t kScratchDoubles = int64_t(1) << 19;   // 4 MiB: 2 x 256 events x 1024 chunks
static_assert(kScratchDoubles * 8 == SUGG_NOALLOC_SCRATCH_BYTES, "scratch size and its public limit differ");

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};   // scratch's device address per device (null: not looked up)

double* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_ptr[device];
}

}  // namespace

int noalloc_scratch_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return SUGG_E_ARG;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_ptr[device]) return SUGG_OK;
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != device) return SUGG_E_HIP;
  void* p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return SUGG_E_HIP;
  }
  g_ptr[device] = static_cast<double*>(p);
  return SUGG_OK;
}

extern "C" {

int32_t sugg_load_features_noalloc(sugg_ctx* ctx, const sugg_plan* plan, const void* counters, const void* cycles,
                                   int32_t mode, void* z_out, hipStream_t stream) {
  if (!ctx) return SUGG_E_ARG;
  if (!plan || plan->ctx != ctx) return ctx->fail(SUGG_E_ARG, "plan missing or from another context");
  double* ptr = scratch_ptr(ctx->device);
  if (!ptr) return ctx->fail(SUGG_E_HIP, "static scratch of device %d not set up", ctx->device);
  if ((int64_t)2 * plan->E * plan->stat_chunks > kScratchDoubles)
    return ctx->fail(SUGG_E_BUDGET, "statistics partials of %lld bytes exceed the %d-byte static scratch",
                     (long long)(16 * (int64_t)plan->E * plan->stat_chunks), SUGG_NOALLOC_SCRATCH_BYTES);
  return load_features_core(ctx, plan, counters, cycles, mode, z_out, stream, ptr);
}

}  // extern "C"
