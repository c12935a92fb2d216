// Library context and shared host helpers of the C ABI implementation.
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <string>
#include <utility>

#include "../../include/uot.h"
#include "uot_device.h"

struct uot_ctx {
  hipStream_t user = nullptr;   // caller's stream
  hipStream_t work = nullptr;   // library stream (capture-capable)
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  uot::Ctrl* pinned = nullptr;  // host mirror of the control block
  int device = 0;
  void* scratch = nullptr;                 // device address of the library's scratch array on `device`
  hipError_t scratch_err = hipSuccess;     // why it is missing, if it is
  std::map<std::string, std::pair<int, int>> batch_tuned;   // batch signature -> (R, blocks per CU)
  std::map<std::string, int> dense_tuned;                    // matrix-core product shape -> block target
  // an asynchronous solve whose result uot_sync_result has not collected:
  // its chunk graph (kept until the stream has run it) and the events
  // around its iterations
  bool pending = false;
  hipGraph_t pending_graph = nullptr;
  hipGraphExec_t pending_exec = nullptr;
  hipEvent_t ev_t0 = nullptr, ev_t1 = nullptr;
};

namespace uot {

extern thread_local std::string g_err;
int fail(int code, const std::string& msg);

#define HIP_TRY(expr)                                                                                  \
  do {                                                                                                 \
    hipError_t e_ = (expr);                                                                            \
    if (e_ != hipSuccess) return ::uot::fail(UOT_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// stream handshake: the library stream waits for the caller's stream at the
// start of a call, and the caller's stream waits for the library's at the end
inline int begin(uot_ctx* ctx) {
  if (ctx->pending)
    return fail(UOT_E_INVALID, "an asynchronous solve is pending on this context: call uot_sync_result first");
  HIP_TRY(hipEventRecord(ctx->ev_in, ctx->user));
  HIP_TRY(hipStreamWaitEvent(ctx->work, ctx->ev_in, 0));
  return UOT_OK;
}

inline int finish(uot_ctx* ctx) {
  HIP_TRY(hipEventRecord(ctx->ev_out, ctx->work));
  HIP_TRY(hipStreamWaitEvent(ctx->user, ctx->ev_out, 0));
  return UOT_OK;
}

}  // namespace uot
