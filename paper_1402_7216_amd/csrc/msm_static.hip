// Full evaluation without a caller workspace and without any device
// allocation: the workspace lives in a fixed-size array in this library's
// device data, one copy per GPU, for callers that cannot allocate (code under
// stream capture, serving loops, harnesses that forbid it).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "msm_plan.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB: a 1M-atom plan needs ~56 MiB
constexpr int kMaxDevices = 64;

// The workspace of msm_compute_static.  In host code this name stands for the
// host-side shadow of the variable, not a device address: kernels are only
// ever given the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

struct DeviceScratch {
  void* ptr = nullptr;       // device address of `scratch` on this device
  uint64_t plan_uid = 0;     // plan whose tables the array holds (0: none yet)
  uint64_t plan_gen = 0;     // that plan's tuning generation when they were written
};

std::mutex g_mu;
DeviceScratch g_dev[kMaxDevices];

}  // namespace

extern "C" {

msm_status msm_compute_static(const msm_plan* P, msm_stream_t stream, const float* x, const float* y,
                              const float* z, const float* q, float* fx, float* fy, float* fz,
                              float* phi, double* energy, double* virial) {
  if (!P) return fail(MSM_ERR_INVALID_ARG, "null plan");
  if (P->lay.total > kScratchBytes)
    return fail(MSM_ERR_UNSUPPORTED, "the plan's workspace (" + std::to_string(P->lay.total) +
                                         " bytes) exceeds the static array of msm_compute_static (" +
                                         std::to_string(kScratchBytes) + " bytes); use msm_compute");
  if (P->g.n_atoms > 0 && (!x || !y || !z || !q))
    return fail(MSM_ERR_INVALID_ARG, "null position or charge array");
  if (!((fx && fy && fz) || (!fx && !fy && !fz)))
    return fail(MSM_ERR_INVALID_ARG, "vector outputs must be all set or all null");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "current device");
  if (dev < 0 || dev >= kMaxDevices) return fail(MSM_ERR_UNSUPPORTED, "device index beyond 63");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::lock_guard<std::mutex> lock(g_mu);
  DeviceScratch& D = g_dev[dev];
  if (!D.ptr) {
    // once per device, with that device current: the device address of this
    // device's copy of the array
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "address of the static workspace");
    if (!ptr) return fail(MSM_ERR_HIP, "static workspace has no device address");
    D.ptr = ptr;
  }
  // the array keeps the last call's contents: (re)write the plan's tables and
  // descriptor unless they are this plan's, at its current tuning
  if (D.plan_uid != P->uid || D.plan_gen != P->tune_gen) {
    D.plan_uid = 0;
    const msm_status st = init_workspace(P, D.ptr, s);
    if (st != MSM_OK) return st;
    D.plan_uid = P->uid;
    D.plan_gen = P->tune_gen;
  }
  msm::LaunchGeom L = P->lg;
  L.sys = reinterpret_cast<const msm::SysDesc*>(static_cast<char*>(D.ptr) + P->lay.off[msm::kSecDesc]);
  const msm::Io io{x, y, z, q, fx, fy, fz, phi, energy, virial, nullptr};
  // every stage in order on the caller's stream (no side streams or events)
  e = msm::launch_eval(msm::kModeForces, L, s, io, nullptr, nullptr);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return MSM_OK;
}

}  // extern "C"
