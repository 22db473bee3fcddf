// Internal: the library context shared by the C entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "ibk.hpp"
#include "m5p.hpp"
#include "kernels.hpp"
#include "sugg.h"

namespace sugg_detail {

template <typename P>
void dfree(P*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

}  // namespace sugg_detail

using sugg_detail::dfree;

struct sugg_ctx {
  int device = 0;
  sugg_params params{};
  std::string err;
  int32_t* d_status = nullptr;
  // model
  int E = 0, D = 0;
  bool has_stats = false, has_model = false;
  double *mu64 = nullptr, *sig64 = nullptr, *isg64 = nullptr, *W64 = nullptr;
  float *mu32 = nullptr, *isg32 = nullptr, *W32 = nullptr;
  std::vector<int64_t> counts;
  // instance-based model (separate from the linear one)
  IbkModel* ibk = nullptr;
  // model-tree (M5P) model (separate from the linear one)
  M5pModel* m5p = nullptr;
  int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    return code;
  }
  int hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return SUGG_OK;
    return fail(SUGG_E_HIP, "%s: %s", what, hipGetErrorString(e));
  }
  void free_model() {
    dfree(mu64); dfree(sig64); dfree(isg64); dfree(W64);
    dfree(mu32); dfree(isg32); dfree(W32);
    E = D = 0;
    has_stats = has_model = false;
    counts.clear();
  }
  // (re)allocate model buffers for shape (e, d); keeps them when unchanged
  int ensure_model(int e, int d) {
    if (e == E && d == D && mu64) return SUGG_OK;
    free_model();
    hipError_t r = hipSuccess;
    if (r == hipSuccess) r = hipMalloc((void**)&mu64, sizeof(double) * e);
    if (r == hipSuccess) r = hipMalloc((void**)&sig64, sizeof(double) * e);
    if (r == hipSuccess) r = hipMalloc((void**)&isg64, sizeof(double) * e);
    if (r == hipSuccess) r = hipMalloc((void**)&mu32, sizeof(float) * e);
    if (r == hipSuccess) r = hipMalloc((void**)&isg32, sizeof(float) * e);
    if (r == hipSuccess && d > 0) r = hipMalloc((void**)&W64, sizeof(double) * (size_t)d * (e + 1));
    if (r == hipSuccess && d > 0) r = hipMalloc((void**)&W32, sizeof(float) * (size_t)d * sugg::w32_ld(e));
    if (r != hipSuccess) {
      free_model();
      return hip(r, "model allocation");
    }
    E = e;
    D = d;
    counts.assign(d, 0);
    return SUGG_OK;
  }
};


inline bool device_ok(sugg_ctx* ctx) {
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return false;
  if (cur != ctx->device) return hipSetDevice(ctx->device) == hipSuccess;
  return true;
}
