// Library-internal host structures shared by the C ABI translation units
// (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "hgs.h"
#include "hgs_internal.h"

namespace hgs {

// Records `msg` as the calling thread's last error and returns `st`.
hgs_status fail(hgs_status st, const std::string &msg);

#define HGS_HIP(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return ::hgs::fail(e_ == hipErrorOutOfMemory ? HGS_ENOMEM : HGS_EHIP,             \
                         std::string(#expr) + ": " + hipGetErrorString(e_));            \
  } while (0)

struct Scene {
  bool used = false;
  bool resident = false;
  SceneDev dev{};
  void *buf = nullptr;
};

struct StageEvent {
  int stage;
  hipEvent_t a, b;
};

// Options with defaults filled in, as the kernels take them.
DevOpts to_dev_opts(const hgs_opts *o);
// Validates camera c and fills d (view index `view`); false with a reason.
bool make_dev_cam(const hgs_camera &c, DevCam &d, int view, std::string &why);

}  // namespace hgs

struct hgs_ctx {
  int device = 0;
  std::vector<hgs::Scene> scenes;
  bool profile = false;
  std::vector<hgs::StageEvent> pending;
  std::vector<hipEvent_t> event_pool;
  double stage_ms[HGS_N_STAGES] = {0};
  int64_t stage_calls[HGS_N_STAGES] = {0};
};
