// The colour loss without any allocation: its three derivative maps live in
// one fixed device array instead of a pooled workspace, for callers that
// must not allocate (graph capture, serving loops, harnesses that forbid
// hipMalloc).  The kernels are the ones hgs_color_loss launches.
//
// The array's device address differs per GPU and is not its host-side name:
// it is resolved with hipGetSymbolAddress once per device, with that device
// current, when a context is created on it, and only that address is ever
// handed to kernels.

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "ctx_internal.h"

namespace hgs {

namespace {

constexpr int kMaxDevices = 64;

// Three maps of at most HGS_NOALLOC_MAX_ELEMS floats each (96 MiB per GPU).
static __device__ __align__(256) float scratch[3 * (size_t)HGS_NOALLOC_MAX_ELEMS];

std::mutex g_mu;
float *g_ptr[kMaxDevices] = {};

}  // namespace

// Resolves this device's copy of the array (device `device` must be
// current).  Called by hgs_create; idempotent.
hipError_t noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_ptr[device]) return hipSuccess;
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_ptr[device] = static_cast<float *>(p);
  return hipSuccess;
}

}  // namespace hgs

using namespace hgs;

extern "C" hgs_status hgs_color_loss_noalloc(hgs_ctx *ctx, int32_t n_views, int32_t height,
                                             int32_t width, const float *render_rgb,
                                             const float *target_rgb, double lambda_dssim,
                                             float *grad, double *losses, void *stream) {
  if (!ctx) return fail(HGS_EINVAL, "ctx is NULL");
  if (n_views < 0 || height < 0 || width < 0) return fail(HGS_EINVAL, "negative size");
  const int64_t planes = (int64_t)n_views * 3;
  const int64_t npx = planes * height * width;
  if (npx > HGS_NOALLOC_MAX_ELEMS)
    return fail(HGS_ECAPACITY, "n_views * 3 * height * width = " + std::to_string(npx) +
                                   " exceeds HGS_NOALLOC_MAX_ELEMS (" +
                                   std::to_string((long long)HGS_NOALLOC_MAX_ELEMS) + ")");
  if (npx > 0 && (!render_rgb || !target_rgb))
    return fail(HGS_EINVAL, "render_rgb and target_rgb are required");
  if (!(lambda_dssim >= 0.0 && lambda_dssim <= 1.0))
    return fail(HGS_EINVAL, "lambda_dssim must be in [0, 1]");
  if (losses && (reinterpret_cast<uintptr_t>(losses) & 7u))
    return fail(HGS_EINVAL, "losses must be 8-byte aligned");
  if (npx == 0) return HGS_OK;
  float *maps = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_mu);
    maps = ctx->device < kMaxDevices ? g_ptr[ctx->device] : nullptr;
  }
  if (!maps) return fail(HGS_ESTATE, "the fixed scratch array of this device is not resolved");
  HGS_HIP(hipSetDevice(ctx->device));
  hipStream_t s = (hipStream_t)stream;
  launch_ssim_fwd(planes, height, width, render_rgb, target_rgb, maps, maps + npx,
                  maps + 2 * npx, losses, ctx->n_cu, s);
  if (grad)
    launch_ssim_bwd(planes, height, width, render_rgb, target_rgb, maps, maps + npx,
                    maps + 2 * npx, lambda_dssim, grad, ctx->n_cu, s);
  HGS_HIP(hipGetLastError());
  return HGS_OK;
}
