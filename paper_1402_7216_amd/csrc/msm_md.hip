// Time stepping on top of the force evaluation: velocity Verlet (Sec. 2.1,
// "Simulation loop") and the parareal iteration (Sec. "Parareal Method",
// eq. (parareal)), whose fine propagator advances every time slice of the
// window at once through one batched evaluation per force call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <string>
#include <vector>

#include "msm_plan.hpp"

namespace {

constexpr int kMdBlock = 256;

int md_blocks(int64_t n) {
  const int64_t b = (n + kMdBlock - 1) / kMdBlock;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 8192));
}

// v += c inv_m F (one half kick; c = dt/2 times the force-to-acceleration scale)
__global__ void __launch_bounds__(kMdBlock) k_kick(int64_t n, float c, float* __restrict__ vx,
                                                   float* __restrict__ vy, float* __restrict__ vz,
                                                   const float* __restrict__ fx, const float* __restrict__ fy,
                                                   const float* __restrict__ fz, const float* __restrict__ inv_m) {
  for (int64_t i = blockIdx.x * (int64_t)kMdBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kMdBlock) {
    const float s = c * inv_m[i];
    vx[i] = fmaf(s, fx[i], vx[i]);
    vy[i] = fmaf(s, fy[i], vy[i]);
    vz[i] = fmaf(s, fz[i], vz[i]);
  }
}

// r += dt v
__global__ void __launch_bounds__(kMdBlock) k_drift(int64_t n, float dt, float* __restrict__ x,
                                                    float* __restrict__ y, float* __restrict__ z,
                                                    const float* __restrict__ vx, const float* __restrict__ vy,
                                                    const float* __restrict__ vz) {
  for (int64_t i = blockIdx.x * (int64_t)kMdBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kMdBlock) {
    x[i] = fmaf(dt, vx[i], x[i]);
    y[i] = fmaf(dt, vy[i], y[i]);
    z[i] = fmaf(dt, vz[i], z[i]);
  }
}

// dst[r n + i] = src[i] for r < reps (charges and inverse masses of the slices)
__global__ void __launch_bounds__(kMdBlock) k_replicate(int64_t n, int reps, const float* __restrict__ src,
                                                        float* __restrict__ dst) {
  const int64_t total = n * reps;
  for (int64_t i = blockIdx.x * (int64_t)kMdBlock + threadIdx.x; i < total; i += (int64_t)gridDim.x * kMdBlock)
    dst[i] = src[i % n];
}

// Copy of one state (6 components of n values; component c of src at
// src + c * sstride, of dst at dst + c * dstride).
__global__ void __launch_bounds__(kMdBlock) k_copy_state(int64_t n, const float* __restrict__ src, int64_t sstride,
                                                         float* __restrict__ dst, int64_t dstride) {
  for (int64_t i = blockIdx.x * (int64_t)kMdBlock + threadIdx.x; i < 6 * n; i += (int64_t)gridDim.x * kMdBlock) {
    const int64_t c = i / n, j = i - c * n;
    dst[c * dstride + j] = src[c * sstride + j];
  }
}

__global__ void k_clear_word(unsigned* w) { *w = 0u; }

// The parareal correction of one time point (6 components of n values):
//   lambda_new = f + (g_new - g_old),  g_old <- g_new,
// and the largest position change |lambda_new - lambda_old| as the bits of a
// non-negative float (max is order-independent, so the atomic is
// deterministic).  When lambda's input state has not changed, g_new equals
// g_old bit for bit and lambda_new is f exactly.
__global__ void __launch_bounds__(kMdBlock) k_correct(int64_t n, const float* __restrict__ f, int64_t fstride,
                                                      const float* __restrict__ gnew, float* __restrict__ gold,
                                                      int64_t gstride, float* __restrict__ lam, int64_t lstride,
                                                      unsigned* __restrict__ resid) {
  float m = 0.f;
  for (int64_t i = blockIdx.x * (int64_t)kMdBlock + threadIdx.x; i < 6 * n; i += (int64_t)gridDim.x * kMdBlock) {
    const int64_t c = i / n, j = i - c * n;
    const float gn = gnew[c * n + j];
    float* gp = gold + c * gstride + j;
    const float v = f[c * fstride + j] + (gn - *gp);
    *gp = gn;
    float* lp = lam + c * lstride + j;
    if (c < 3) m = fmaxf(m, fabsf(v - *lp));
    *lp = v;
  }
  // block maximum, then one atomic per block
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  __shared__ float wm[kMdBlock / 64];
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kMdBlock / 64; ++w) m = fmaxf(m, wm[w]);
    wm[0] = m;
    atomicMax(resid, __float_as_uint(wm[0]));
  }
}

struct Forces {
  // F at the current positions into fx, fy, fz
  virtual msm_status eval(const float* x, const float* y, const float* z, float* fx, float* fy, float* fz) = 0;
  virtual ~Forces() = default;
};

struct PlanForces : Forces {
  const msm_plan* P;
  void* ws;
  size_t wsb;
  msm_stream_t s;
  const float* q;
  PlanForces(const msm_plan* P_, void* ws_, size_t wsb_, msm_stream_t s_, const float* q_)
      : P(P_), ws(ws_), wsb(wsb_), s(s_), q(q_) {}
  msm_status eval(const float* x, const float* y, const float* z, float* fx, float* fy, float* fz) override {
    return msm_compute(P, ws, wsb, s, x, y, z, q, fx, fy, fz, nullptr, nullptr, nullptr);
  }
};

struct BatchForces : Forces {
  const msm_batch* B;
  void* ws;
  size_t wsb;
  msm_stream_t s;
  const float* q;
  BatchForces(const msm_batch* B_, void* ws_, size_t wsb_, msm_stream_t s_, const float* q_)
      : B(B_), ws(ws_), wsb(wsb_), s(s_), q(q_) {}
  msm_status eval(const float* x, const float* y, const float* z, float* fx, float* fy, float* fz) override {
    return msm_batch_compute(B, ws, wsb, s, x, y, z, q, fx, fy, fz, nullptr, nullptr, nullptr);
  }
};

// n_steps velocity Verlet steps of dt over n values per component: forces at
// the start, then per step a half kick, a drift, forces at the new positions
// and a half kick.  f holds the forces at the final positions on return.
msm_status vv(Forces& F, hipStream_t s, int64_t n, int n_steps, double dt, double scale, float* x, float* y,
              float* z, float* vx, float* vy, float* vz, const float* inv_m, float* fx, float* fy, float* fz) {
  msm_status st = F.eval(x, y, z, fx, fy, fz);
  if (st != MSM_OK) return st;
  const float half = (float)(0.5 * dt * scale), fdt = (float)dt;
  const int nb = md_blocks(n);
  for (int k = 0; k < n_steps; ++k) {
    k_kick<<<nb, kMdBlock, 0, s>>>(n, half, vx, vy, vz, fx, fy, fz, inv_m);
    k_drift<<<nb, kMdBlock, 0, s>>>(n, fdt, x, y, z, vx, vy, vz);
    st = F.eval(x, y, z, fx, fy, fz);
    if (st != MSM_OK) return st;
    k_kick<<<nb, kMdBlock, 0, s>>>(n, half, vx, vy, vz, fx, fy, fz, inv_m);
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? MSM_OK : hip_fail(e, "velocity Verlet launch");
}

msm_status check_vv(int n_steps, double dt, double scale) {
  if (n_steps < 0) return fail(MSM_ERR_INVALID_ARG, "n_steps must be >= 0");
  if (!std::isfinite(dt) || !std::isfinite(scale) || !(scale > 0.0))
    return fail(MSM_ERR_INVALID_ARG, "dt must be finite and accel_scale finite and > 0");
  return MSM_OK;
}

msm_status check_arrays(std::initializer_list<const void*> ptrs) {
  for (const void* p : ptrs)
    if (!p) return fail(MSM_ERR_INVALID_ARG, "null array");
  return MSM_OK;
}

// parareal scratch layout (floats, each section 256-byte aligned)
struct PrLayout {
  size_t qb, imb, f, g, tmp, ff, gf, resid, total;
};

size_t up(size_t v) { return (v + 63) & ~size_t(63); }   // floats -> 256-byte multiples

PrLayout pr_layout(int64_t n, int64_t T) {
  PrLayout L{};
  size_t o = 0;
  L.qb = o;    o += up(T * n);
  L.imb = o;   o += up(T * n);
  L.f = o;     o += up(6 * T * n);
  L.g = o;     o += up(6 * T * n);
  L.tmp = o;   o += up(6 * n);
  L.ff = o;    o += up(3 * T * n);
  L.gf = o;    o += up(3 * n);
  L.resid = o; o += 64;
  L.total = o * sizeof(float);
  return L;
}

}  // namespace

extern "C" {

msm_status msm_vv_run(const msm_plan* P, void* ws, size_t ws_bytes, msm_stream_t stream, int32_t n_steps, double dt,
                      double accel_scale, float* x, float* y, float* z, const float* q, float* vx, float* vy,
                      float* vz, const float* inv_mass, float* fx, float* fy, float* fz) {
  if (!P) return fail(MSM_ERR_INVALID_ARG, "null plan");
  msm_status st = check_vv(n_steps, dt, accel_scale);
  if (st != MSM_OK) return st;
  if (P->g.n_atoms > 0) {
    st = check_arrays({x, y, z, q, vx, vy, vz, inv_mass, fx, fy, fz});
    if (st != MSM_OK) return st;
  }
  PlanForces F(P, ws, ws_bytes, stream, q);
  return vv(F, reinterpret_cast<hipStream_t>(stream), P->g.n_atoms, n_steps, dt, accel_scale, x, y, z, vx, vy, vz,
            inv_mass, fx, fy, fz);
}

msm_status msm_batch_vv_run(const msm_batch* B, void* ws, size_t ws_bytes, msm_stream_t stream, int32_t n_steps,
                            double dt, double accel_scale, float* x, float* y, float* z, const float* q, float* vx,
                            float* vy, float* vz, const float* inv_mass, float* fx, float* fy, float* fz) {
  if (!B) return fail(MSM_ERR_INVALID_ARG, "null batch");
  msm_status st = check_vv(n_steps, dt, accel_scale);
  if (st != MSM_OK) return st;
  int32_t n_sys = 0, off_last = 0;
  st = batch_shape(B, &n_sys, &off_last);
  if (st != MSM_OK) return st;
  if (off_last > 0) {
    st = check_arrays({x, y, z, q, vx, vy, vz, inv_mass, fx, fy, fz});
    if (st != MSM_OK) return st;
  }
  BatchForces F(B, ws, ws_bytes, stream, q);
  return vv(F, reinterpret_cast<hipStream_t>(stream), off_last, n_steps, dt, accel_scale, x, y, z, vx, vy, vz,
            inv_mass, fx, fy, fz);
}

msm_status msm_parareal_workspace_bytes(int32_t n_atoms, int32_t slices, size_t* bytes) {
  if (!bytes || n_atoms < 0 || slices < 1) return fail(MSM_ERR_INVALID_ARG, "bad size or null output");
  *bytes = pr_layout(n_atoms, slices).total;
  return MSM_OK;
}

msm_status msm_parareal_run(const msm_parareal_params* pp, const msm_batch* fine, void* fine_ws, size_t fine_ws_bytes,
                            const msm_plan* coarse, void* coarse_ws, size_t coarse_ws_bytes, void* ws,
                            size_t ws_bytes, msm_stream_t stream, const float* q, const float* inv_mass,
                            float* states, int32_t* iterations, float* residuals) {
  if (!pp || !fine || !coarse || !states || !iterations)
    return fail(MSM_ERR_INVALID_ARG, "null parameters, plan, batch, states or iterations");
  const int T = pp->slices;
  if (T < 1 || pp->steps_per_slice < 1 || pp->max_iter < 1 || pp->max_iter > T)
    return fail(MSM_ERR_INVALID_ARG, "need slices >= 1, steps_per_slice >= 1 and 1 <= max_iter <= slices");
  msm_status st = check_vv(pp->steps_per_slice, pp->dt, pp->accel_scale);
  if (st != MSM_OK) return st;
  if (!std::isfinite(pp->tol) || pp->tol < 0.0) return fail(MSM_ERR_INVALID_ARG, "tol must be finite and >= 0");
  if (pp->reserved != 0) return fail(MSM_ERR_INVALID_ARG, "reserved field must be zero");
  const int64_t n = coarse->g.n_atoms;
  int32_t n_sys = 0, total = 0;
  st = batch_shape(fine, &n_sys, &total);
  if (st != MSM_OK) return st;
  if (n_sys != T || (int64_t)total != n * T)
    return fail(MSM_ERR_INVALID_ARG, "the fine batch must hold `slices` systems of the coarse plan's atom count");
  if (n > 0) {
    st = check_arrays({q, inv_mass});
    if (st != MSM_OK) return st;
  }
  const PrLayout L = pr_layout(n, T);
  if (!ws || ws_bytes < L.total) return fail(MSM_ERR_WORKSPACE, "parareal workspace missing or too small");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  float* W = static_cast<float*>(ws);
  float *qb = W + L.qb, *imb = W + L.imb, *f = W + L.f, *g = W + L.g, *tmp = W + L.tmp, *ff = W + L.ff,
        *gf = W + L.gf;
  unsigned* resid = reinterpret_cast<unsigned*>(W + L.resid);
  const int64_t ls = (int64_t)(T + 1) * n;       // component stride of `states` ([6][T + 1][n])
  const int64_t fs = (int64_t)T * n;             // component stride of f and g ([6][T][n])
  auto lam = [&](int t) { return states + (int64_t)t * n; };
  auto blocks6 = md_blocks(6 * n);
  const int spl = pp->steps_per_slice;
  PlanForces G(coarse, coarse_ws, coarse_ws_bytes, stream, q);
  BatchForces Fb(fine, fine_ws, fine_ws_bytes, stream, qb);
  auto coarse_step = [&](float* st6) {   // G over one slice, in place on a [6][n] state
    return vv(G, s, n, spl, pp->dt, pp->accel_scale, st6, st6 + n, st6 + 2 * n, st6 + 3 * n, st6 + 4 * n,
              st6 + 5 * n, inv_mass, gf, gf + n, gf + 2 * n);
  };
  auto data_flags = [&]() -> msm_status {
    int32_t fl = 0;
    msm_status r = msm_status_query(coarse, coarse_ws, stream, &fl);
    if (r != MSM_OK) return r;
    return msm_batch_status(fine, fine_ws, stream, nullptr);
  };
  *iterations = 0;
  if (n == 0) return MSM_OK;
  k_replicate<<<md_blocks(T * n), kMdBlock, 0, s>>>(n, T, q, qb);
  k_replicate<<<md_blocks(T * n), kMdBlock, 0, s>>>(n, T, inv_mass, imb);
  // initial coarse sweep: lambda_{t+1} = g_{t+1} = G(lambda_t)
  for (int t = 0; t < T; ++t) {
    k_copy_state<<<blocks6, kMdBlock, 0, s>>>(n, lam(t), ls, tmp, n);
    st = coarse_step(tmp);
    if (st != MSM_OK) return st;
    k_copy_state<<<blocks6, kMdBlock, 0, s>>>(n, tmp, n, g + (int64_t)t * n, fs);
    k_copy_state<<<blocks6, kMdBlock, 0, s>>>(n, tmp, n, lam(t + 1), ls);
  }
  for (int k = 0; k < pp->max_iter; ++k) {
    // fine propagation of every slice's start state at once (one batched
    // evaluation per force call): f_t = F(lambda_t), t = 0 .. T - 1
    k_copy_state<<<md_blocks(6 * fs), kMdBlock, 0, s>>>(fs, states, ls, f, fs);   // rows t < T of each component
    st = vv(Fb, s, fs, spl, pp->dt, pp->accel_scale, f, f + fs, f + 2 * fs, f + 3 * fs, f + 4 * fs, f + 5 * fs,
            imb, ff, ff + fs, ff + 2 * fs);
    if (st != MSM_OK) return st;
    // sequential coarse sweep with the correction; slices t < k are final
    k_clear_word<<<1, 1, 0, s>>>(resid);
    for (int t = k; t < T; ++t) {
      k_copy_state<<<blocks6, kMdBlock, 0, s>>>(n, lam(t), ls, tmp, n);
      st = coarse_step(tmp);
      if (st != MSM_OK) return st;
      k_correct<<<blocks6, kMdBlock, 0, s>>>(n, f + (int64_t)t * n, fs, tmp, g + (int64_t)t * n, fs, lam(t + 1),
                                              ls, resid);
    }
    unsigned rbits = 0;
    hipError_t e = hipMemcpyAsync(&rbits, resid, sizeof(unsigned), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "read parareal residual");
    st = data_flags();
    if (st != MSM_OK) return st;
    float r;
    std::memcpy(&r, &rbits, sizeof r);
    if (residuals) residuals[k] = r;
    *iterations = k + 1;
    if (r <= (float)pp->tol) break;
  }
  return MSM_OK;
}

}  // extern "C"
