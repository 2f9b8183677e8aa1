// The context behind the C ABI's opaque bddc_ctx, and the error handling
// shared by the translation units that implement the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <new>
#include <string>

#include "../../include/bddc.h"
#include "adapt.h"
#include "host.h"
#include "solver.h"

struct bddc_ctx {
  bddc_options opt{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  bddc::Problem P;
  std::unique_ptr<bddc::Solver> S;
  bddc::AdaptState adapt;
  int state = 0;  // 0 created, 1 set up, 2 factored
  std::string err;
};

namespace bddc {

inline bddc_status fail(bddc_ctx *c, int code, const std::string &m) {
  if (c) c->err = m;
  return (bddc_status)code;
}

// runs f, turning exceptions into status codes and the context's message;
// the per-launch timing hook, the GEMM autotuning switch and the unbatched
// (per-substructure) launch switch hold for the duration of the call
template <class F>
bddc_status guarded(bddc_ctx *c, F f) {
  struct Hook {
    explicit Hook(bddc_ctx *c) {
      launch_timing() = (c && c->S && c->S->timer.mode == 2) ? &c->S->timer : nullptr;
      autotune_enabled() = c && c->opt.autotune != 0;
      per_entry_launches() = c && c->opt.per_substructure_launches != 0;
      fused_workspace() = (c && c->S && c->opt.chol_launch != 1) ? &c->S->alloc : nullptr;
      fused_max_tasks() = (c && c->opt.chol_launch == 2) ? INT64_MAX : kFusedAutoTasks;
    }
    ~Hook() {
      launch_timing() = nullptr;
      autotune_enabled() = false;
      per_entry_launches() = false;
      fused_workspace() = nullptr;
      fused_max_tasks() = kFusedAutoTasks;
    }
  } hook(c);
  try {
    f();
    if (c) c->err.clear();
    return BDDC_OK;
  } catch (const BddcError &e) {
    return fail(c, e.code, e.what());
  } catch (const std::bad_alloc &) {
    return fail(c, BDDC_ERR_OOM, "host allocation failed");
  } catch (const std::exception &e) {
    return fail(c, BDDC_ERR_DEVICE, e.what());
  }
}

inline void check_hip(hipError_t e, const char *what) {
  if (e != hipSuccess) throw DeviceError(std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace bddc
