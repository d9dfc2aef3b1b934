// gfx950 kernels of the multilevel summation method (thesis Sec. 2.3).
//
// Forward chain on one stream:
//   zero -> bin_count -> scan -> bin_scatter -> bin_place        link cells (Sec. 2.1)
//   short_range                                                   u^short, F^short
//   anterpolate -> restrict (k = 0..l-2)                          q^0 .. q^{l-1}
//   lattice (all k <= l-2 in one launch) + top (FP64)             u^{k,cut}
//   prolong (k = l-2..0)                                          u^k
//   interpolate_assemble -> reduce                                phi, F, E, virial
//
// Every per-atom and per-node value is a gather in a fixed order, so results
// are bitwise reproducible.  All arithmetic is float32 except the top-level
// sum and the energy / virial reductions (float64).
#include "msm_internal.hpp"

namespace msm {
namespace {

constexpr int kBlock = 256;
constexpr int kWave = 64;

// --------------------------------------------------------------------------
// Grid coordinates.  t = (x - lo)/h; f = floor(t) clamped to [0, floor(len/h)];
// r = t - f computed as fma(-f, h, x - lo) / h so the offset keeps full
// relative precision even far from the origin.
// --------------------------------------------------------------------------
__device__ __forceinline__ void grid_coord(float x, float lo, float h, float inv_h, int fmax, int& f,
                                           float& r) {
  float d = x - lo;
  int fi = (int)floorf(d * inv_h);
  fi = min(max(fi, 0), fmax);
  f = fi;
  r = fmaf(-(float)fi, h, d) * inv_h;
}

// --------------------------------------------------------------------------
// One-dimensional basis Phi (nodal basis of Sec. 2.3), C1 numerical Hermite.
// Piece p covers |u| in [p, p+1]; factored forms keep FP32 relative accuracy.
//   cubic:   p0 (1-t)(1+t-3t^2/2)          p1 -(t-1)(2-t)^2/2
//   quintic: p0 (1-t^2)(2-t)(6+3t-5t^2)/12 p1 (1-t)(2-t)(3-t)(4+9t-5t^2)/24
//            p2 (t-1)(t-2)(t-3)^2(4-t)/24
// --------------------------------------------------------------------------
template <int ORDER>
__device__ __forceinline__ void piece(int p, float t, float& v, float& d);

template <>
__device__ __forceinline__ void piece<4>(int p, float t, float& v, float& d) {
  if (p == 0) {
    float A = 1.f - t, B = 1.f + t - 1.5f * t * t;
    v = A * B;
    d = -B + A * (1.f - 3.f * t);
  } else {
    float A = t - 1.f, B = 2.f - t;
    v = -0.5f * A * B * B;
    d = -0.5f * (B * B - 2.f * A * B);
  }
}

template <>
__device__ __forceinline__ void piece<6>(int p, float t, float& v, float& d) {
  if (p == 0) {
    float A = 1.f - t * t, B = 2.f - t, C = 6.f + 3.f * t - 5.f * t * t;
    v = A * B * C * (1.f / 12.f);
    d = (-2.f * t * B * C - A * C + A * B * (3.f - 10.f * t)) * (1.f / 12.f);
  } else if (p == 1) {
    float A = 1.f - t, B = 2.f - t, C = 3.f - t, D = 4.f + 9.f * t - 5.f * t * t;
    v = A * B * C * D * (1.f / 24.f);
    d = (-(B * C * D) - A * C * D - A * B * D + A * B * C * (9.f - 10.f * t)) * (1.f / 24.f);
  } else {
    float A = t - 1.f, B = t - 2.f, E = t - 3.f, D = 4.f - t;
    float C = E * E;
    v = A * B * C * D * (1.f / 24.f);
    d = (B * C * D + A * C * D + 2.f * A * B * E * D - A * B * C) * (1.f / 24.f);
  }
}

// Weights w[s] = Phi(r + H - 1 - s) and dw[s] = dPhi/dr for the ORDER nodes
// f - (H-1) .. f + H of an atom with offset r in [0, 1).  The piece of each s
// is fixed, so there is no data-dependent branch.
template <int ORDER>
__device__ __forceinline__ void basis(float r, float* w, float* dw) {
  constexpr int H = ORDER / 2;
#pragma unroll
  for (int s = 0; s < ORDER; ++s) {
    float v, d;
    if (s <= H - 1) {
      piece<ORDER>(H - 1 - s, (float)(H - 1 - s) + r, v, d);
      w[s] = v;
      dw[s] = d;
    } else {
      piece<ORDER>(s - H, (float)(s - H + 1) - r, v, d);
      w[s] = v;
      dw[s] = -d;
    }
  }
}

// Phi(u) for an arbitrary argument (used by the node-centric gather).
template <int ORDER>
__device__ __forceinline__ float phi_any(float u) {
  float t = fabsf(u), v, d;
  if (ORDER == 4) {
    if (t >= 2.f) return 0.f;
    piece<4>(t <= 1.f ? 0 : 1, t, v, d);
  } else {
    if (t >= 3.f) return 0.f;
    piece<6>(t <= 1.f ? 0 : (t <= 2.f ? 1 : 2), t, v, d);
  }
  return v;
}

// --------------------------------------------------------------------------
// Link cells (Sec. 2.1): counting sort of atoms by cell, stable in input order.
// --------------------------------------------------------------------------
__global__ void k_zero(int* __restrict__ counts, int* __restrict__ cursor, int n_cells,
                       int* __restrict__ status) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= n_cells) counts[i] = 0;
  if (i < n_cells) cursor[i] = 0;
  if (i < 64) status[i] = 0;
}

__device__ __forceinline__ int cell_index(const Geom& g, float x, float y, float z) {
  int c[3];
  float p[3] = {x, y, z};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    float t = (p[d] - g.lo_f[d]) * g.inv_cs[d];
    t = fminf(fmaxf(t, 0.f), (float)(g.nc[d] - 1));   // NaN -> 0
    c[d] = min((int)t, g.nc[d] - 1);
  }
  return (c[2] * g.nc[1] + c[1]) * g.nc[0] + c[0];
}

__global__ void k_bin_count(Geom g, const float* __restrict__ x, const float* __restrict__ y,
                            const float* __restrict__ z, const float* __restrict__ q,
                            int* __restrict__ counts, int* __restrict__ cell_of,
                            int* __restrict__ status) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n_atoms) return;
  float px = x[i], py = y[i], pz = z[i], pq = q[i];
  int flags = 0;
  if (!(isfinite(px) && isfinite(py) && isfinite(pz) && isfinite(pq))) {
    flags |= kFlagNonFinite;
  } else {
    double p[3] = {(double)px, (double)py, (double)pz};
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (p[d] < g.lo[d] || p[d] > g.hi[d]) flags |= kFlagOutOfBox;
  }
  if (flags) atomicOr(status, flags);
  int c = cell_index(g, px, py, pz);
  cell_of[i] = c;
  atomicAdd(&counts[c], 1);
}

// Exclusive scan of counts[0..n) into start[0..n] by one block of 1024 threads.
__global__ void __launch_bounds__(1024) k_scan(const int* __restrict__ counts, int* __restrict__ start,
                                               int n) {
  __shared__ int part[1024];
  int t = threadIdx.x;
  int chunk = (n + 1023) / 1024;
  int b = t * chunk, e = min(b + chunk, n);
  int s = 0;
  for (int i = b; i < e; ++i) s += counts[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int v = (t >= off) ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - s;
  for (int i = b; i < e; ++i) {
    start[i] = run;
    run += counts[i];
  }
  if (t == 1023) start[n] = part[1023];
}

__global__ void k_bin_scatter(Geom g, const int* __restrict__ cell_of, const int* __restrict__ start,
                              int* __restrict__ cursor, int* __restrict__ tmp) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n_atoms) return;
  int c = cell_of[i];
  tmp[start[c] + atomicAdd(&cursor[c], 1)] = i;
}

// Final slot of each atom = cell start + number of atoms of the same cell with a
// smaller input index (a stable order independent of the scatter's atomics).
// Also flags coincident atoms and writes sanitised, box-clamped coordinates so
// every later kernel stays inside the grid even for bad input.
__global__ void k_bin_place(Geom g, const float* __restrict__ x, const float* __restrict__ y,
                            const float* __restrict__ z, const float* __restrict__ q,
                            const int* __restrict__ cell_of, const int* __restrict__ start,
                            const int* __restrict__ tmp, float4* __restrict__ sorted,
                            int* __restrict__ perm, int* __restrict__ status) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.n_atoms) return;
  int i = tmp[s];
  int c = cell_of[i];
  int b = start[c], e = start[c + 1];
  float px = x[i], py = y[i], pz = z[i], pq = q[i];
  int dst = s;
  if (e - b <= kRankCap) {
    int rank = 0;
    bool coincident = false;
    for (int t = b; t < e; ++t) {
      int j = tmp[t];
      rank += (j < i);
      if (j != i && x[j] == px && y[j] == py && z[j] == pz) coincident = true;
    }
    dst = b + rank;
    if (coincident) atomicOr(status, kFlagCoincident);
  }
  float hi[3] = {(float)g.hi[0], (float)g.hi[1], (float)g.hi[2]};
  px = fminf(fmaxf(px, g.lo_f[0]), hi[0]);
  py = fminf(fmaxf(py, g.lo_f[1]), hi[1]);
  pz = fminf(fmaxf(pz, g.lo_f[2]), hi[2]);
  if (!isfinite(pq)) pq = 0.f;
  sorted[dst] = make_float4(px, py, pz, pq);
  perm[dst] = i;
}

// --------------------------------------------------------------------------
// Short-range part (itemised algorithm, first sentence; eq. msmgrid g*):
//   phi_i^s = sum_j q_j g*(r_ij),  F_i^s = -q_i sum_j q_j g*'(r_ij) (r_i - r_j)/r_ij
//   g*(r) = 1/r - gamma(r/a)/a,  g*'(r)/r = -1/r^3 - gamma'(r/a)/(a^2 r)
// One work item = a run of run_w cells along x in one cell row; its atoms are
// contiguous in sorted order.  Lanes hold i atoms; j atoms are read with
// wave-uniform loads (scalar cache).  The (2 reach + 1)^2 neighbour rows are
// split over the 4 waves of the block and the partial sums added in a fixed
// order through LDS.
// --------------------------------------------------------------------------
template <int M>
__global__ void __launch_bounds__(kBlock) k_short(Geom g, const float4* __restrict__ sorted,
                                                  const int* __restrict__ start,
                                                  float4* __restrict__ fshort) {
  __shared__ float4 red[kBlock];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = threadIdx.x / kWave;
  const int run = blockIdx.x % g.runs_x;
  const int row = blockIdx.x / g.runs_x;
  const int cy = row % g.nc[1], cz = row / g.nc[1];
  const int cx0 = run * g.run_w;
  const int cx1 = min(cx0 + g.run_w, g.nc[0]) - 1;
  const int rowbase = (cz * g.nc[1] + cy) * g.nc[0];
  const int ib = start[rowbase + cx0], ie = start[rowbase + cx1 + 1];
  const int R = g.reach, side = 2 * R + 1;
  const int jx0 = max(cx0 - R, 0), jx1 = min(cx1 + R, g.nc[0] - 1);
  const float a2 = g.a2, inv_a2 = g.inv_a2;

  for (int ic = ib; ic < ie; ic += kWave) {
    const int i = ic + lane;
    float4 pi = (i < ie) ? sorted[i] : make_float4(3.0e30f, 3.0e30f, 3.0e30f, 0.f);
    float ax = 0.f, ay = 0.f, az = 0.f, ap = 0.f;
    for (int rr = wave; rr < side * side; rr += kBlock / kWave) {
      const int jy = cy + rr % side - R, jz = cz + rr / side - R;
      if (jy < 0 || jz < 0 || jy >= g.nc[1] || jz >= g.nc[2]) continue;
      const int jb = (jz * g.nc[1] + jy) * g.nc[0];
      const int j0 = start[jb + jx0], j1 = start[jb + jx1 + 1];
      for (int j = j0; j < j1; ++j) {
        const float4 pj = sorted[j];
        const float dx = pi.x - pj.x, dy = pi.y - pj.y, dz = pi.z - pj.z;
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        if (r2 < a2 && r2 > 0.f) {
          // hardware reciprocal square root plus one Newton step (the raw
          // instruction's error is biased, which would bias the energy)
          float ri = __builtin_amdgcn_rsqf(r2);
          ri = fmaf(0.5f * ri, fmaf(-r2 * ri, ri, 1.f), ri);
          const float ri2 = ri * ri;
          const float s = r2 * inv_a2;
          float gm = g.gcoef[M], dg = g.dcoef[M];
#pragma unroll
          for (int k = M - 1; k >= 0; --k) gm = fmaf(gm, s, g.gcoef[k]);
#pragma unroll
          for (int k = M - 1; k >= 1; --k) dg = fmaf(dg, s, g.dcoef[k]);
          const float gs = ri - gm;                    // g*(r)
          const float fr = fmaf(ri, ri2, dg);          // -g*'(r)/r
          ap = fmaf(pj.w, gs, ap);
          const float wq = pj.w * fr;
          ax = fmaf(wq, dx, ax);
          ay = fmaf(wq, dy, ay);
          az = fmaf(wq, dz, az);
        }
      }
    }
    red[threadIdx.x] = make_float4(ax, ay, az, ap);
    __syncthreads();
    if (wave == 0 && i < ie) {
      float4 s0 = red[lane], s1 = red[lane + 64], s2 = red[lane + 128], s3 = red[lane + 192];
      float qi = pi.w;
      float4 o;
      o.x = qi * (((s0.x + s1.x) + s2.x) + s3.x);
      o.y = qi * (((s0.y + s1.y) + s2.y) + s3.y);
      o.z = qi * (((s0.z + s1.z) + s2.z) + s3.z);
      o.w = ((s0.w + s1.w) + s2.w) + s3.w;
      fshort[i] = o;
    }
    __syncthreads();
  }
}

// --------------------------------------------------------------------------
// Anterpolation (itemised algorithm): q^0_mu = sum_j phi^0_mu(r_j) q_j, as a
// gather per level-0 node over the atoms of the cells its support touches.
// --------------------------------------------------------------------------
template <int ORDER>
__global__ void __launch_bounds__(kBlock) k_anterp(Geom g, const float4* __restrict__ sorted,
                                                   const int* __restrict__ start,
                                                   float* __restrict__ qgrid) {
  constexpr int H = ORDER / 2;
  const Level L = g.lv[0];
  int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= L.count) return;
  int mu[3] = {node % L.n[0] + L.lo[0], (node / L.n[0]) % L.n[1] + L.lo[1],
               node / (L.n[0] * L.n[1]) + L.lo[2]};
  // atoms touching mu have floor index in [mu - H, mu + H - 1]: positions in
  // [lo + (mu - H) h, lo + (mu + H) h); widen by a small margin for rounding
  int c0[3], c1[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    float xl = ((float)(mu[d] - H) - 0.01f) * g.h, xh = ((float)(mu[d] + H) + 0.01f) * g.h;
    c0[d] = min(g.nc[d] - 1, max(0, (int)floorf(fmaxf(xl, 0.f) * g.inv_cs[d])));
    c1[d] = max(c0[d], min(g.nc[d] - 1, (int)floorf(fmaxf(xh, 0.f) * g.inv_cs[d])));
  }
  float acc = 0.f;
  for (int cz = c0[2]; cz <= c1[2]; ++cz)
    for (int cy = c0[1]; cy <= c1[1]; ++cy) {
      int rb = (cz * g.nc[1] + cy) * g.nc[0];
      int jb = start[rb + c0[0]], je = start[rb + c1[0] + 1];
      for (int j = jb; j < je; ++j) {
        float4 p = sorted[j];
        float pp[3] = {p.x, p.y, p.z};
        float w = p.w;
        bool in = true;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          int f;
          float r;
          grid_coord(pp[d], g.lo_f[d], g.h, g.inv_h, g.fmax[d], f, r);
          int sidx = mu[d] - (f - (H - 1));
          in = in && (sidx >= 0) && (sidx < ORDER);
          w *= phi_any<ORDER>(r + (float)(H - 1 - sidx));
        }
        if (in) acc += w;
      }
    }
  qgrid[L.off + node] = acc;
}

// --------------------------------------------------------------------------
// Restriction (itemised algorithm): q^{k+1}_mu = sum_nu Phi(nu/2 - mu)^3 q^k_nu.
// Only offsets j = nu - 2 mu with Phi(j/2) != 0 are visited (given as lists).
// --------------------------------------------------------------------------
struct RestrictTaps {
  int n;
  int j[12];
  float w[12];
};

__global__ void __launch_bounds__(kBlock) k_restrict(Geom g, int k, RestrictTaps taps,
                                                     float* __restrict__ grid) {
  const Level F = g.lv[k], C = g.lv[k + 1];
  int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= C.count) return;
  int mx = node % C.n[0] + C.lo[0], my = (node / C.n[0]) % C.n[1] + C.lo[1],
      mz = node / (C.n[0] * C.n[1]) + C.lo[2];
  const float* fin = grid + F.off;
  float acc = 0.f;
  for (int a = 0; a < taps.n; ++a) {
    int vz = 2 * mz + taps.j[a] - F.lo[2];
    if (vz < 0 || vz >= F.n[2]) continue;
    float wz = taps.w[a];
    for (int b = 0; b < taps.n; ++b) {
      int vy = 2 * my + taps.j[b] - F.lo[1];
      if (vy < 0 || vy >= F.n[1]) continue;
      float wyz = taps.w[b] * wz;
      const float* rowp = fin + ((size_t)vz * F.n[1] + vy) * F.n[0];
      float racc = 0.f;
      for (int c = 0; c < taps.n; ++c) {
        int vx = 2 * mx + taps.j[c] - F.lo[0];
        if (vx < 0 || vx >= F.n[0]) continue;
        racc = fmaf(taps.w[c], rowp[vx], racc);
      }
      acc = fmaf(wyz, racc, acc);
    }
  }
  grid[C.off + node] = acc;
}

// --------------------------------------------------------------------------
// Lattice cutoff (itemised algorithm) for every level k <= l-2 in one launch:
//   u^{k,cut}_mu = sum_{|n| < 2a/h} g^k(2^k h |n|) q^k_{mu+n} = 2^-k sum W(n) q^k_{mu+n}
// with W(n) = g^0(h|n|) from the stencil table (rows of taps along z).
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_lattice(Geom g, const StencilRow* __restrict__ rows,
                                                    int n_rows, const float* __restrict__ wts,
                                                    const float* __restrict__ qgrid,
                                                    float* __restrict__ ucut, int n_lattice_nodes) {
  int gid = blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= n_lattice_nodes) return;
  int k = 0;
  while (k + 1 < g.levels - 1 && gid >= g.lv[k + 1].off) ++k;
  const Level L = g.lv[k];
  int node = gid - L.off;
  int mx = node % L.n[0], my = (node / L.n[0]) % L.n[1], mz = node / (L.n[0] * L.n[1]);
  const float* qk = qgrid + L.off;
  float acc = 0.f;
  for (int r = 0; r < n_rows; ++r) {
    StencilRow row = rows[r];
    int vx = mx + row.nx, vy = my + row.ny;
    if (vx < 0 || vy < 0 || vx >= L.n[0] || vy >= L.n[1]) continue;
    int z0 = max(-row.zr, -mz), z1 = min(row.zr, L.n[2] - 1 - mz);
    const float* col = qk + (size_t)vy * L.n[0] + vx;
    const float* w = wts + row.woff + row.zr;
    float racc = 0.f;
    for (int nz = z0; nz <= z1; ++nz)
      racc = fmaf(w[nz], col[(size_t)(mz + nz) * L.n[0] * L.n[1]], racc);
    acc += racc;
  }
  ucut[gid] = ldexpf(acc, -k);
}

// --------------------------------------------------------------------------
// Top level (itemised algorithm), float64: u^{l-1}_mu = sum over every node nu
// of g^{l-1}(2^{l-1} h |mu - nu|) q^{l-1}_nu, from a table T[|dx|][|dy|][|dz|].
// --------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_top(Geom g, const double* __restrict__ T,
                                                const float* __restrict__ qgrid,
                                                float* __restrict__ ucut, float* __restrict__ u) {
  const Level L = g.lv[g.levels - 1];
  int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= L.count) return;
  int mx = node % L.n[0], my = (node / L.n[0]) % L.n[1], mz = node / (L.n[0] * L.n[1]);
  const float* qt = qgrid + L.off;
  double acc = 0.0;
  for (int vz = 0; vz < L.n[2]; ++vz) {
    int dz = abs(mz - vz);
    for (int vy = 0; vy < L.n[1]; ++vy) {
      int dy = abs(my - vy);
      const double* trow = T + ((size_t)dz * L.n[1] + dy) * L.n[0];
      const float* qrow = qt + ((size_t)vz * L.n[1] + vy) * L.n[0];
      for (int vx = 0; vx < L.n[0]; ++vx) acc = fma(trow[abs(mx - vx)], (double)qrow[vx], acc);
    }
  }
  ucut[L.off + node] = (float)acc;
  u[L.off + node] = (float)acc;
}

// --------------------------------------------------------------------------
// Prolongation (itemised algorithm):
//   u^k_mu = u^{k,cut}_mu + sum_nu Phi(mu/2 - nu)^3 u^{k+1}_nu, |mu - 2 nu| <= order - 1.
// pw[j + order - 1] = Phi(j/2).
// --------------------------------------------------------------------------
struct ProlongW {
  float w[11];
};

__global__ void __launch_bounds__(kBlock) k_prolong(Geom g, int k, ProlongW pw,
                                                    const float* __restrict__ ucut,
                                                    float* __restrict__ u) {
  const Level F = g.lv[k], C = g.lv[k + 1];
  int node = blockIdx.x * blockDim.x + threadIdx.x;
  if (node >= F.count) return;
  int m[3] = {node % F.n[0] + F.lo[0], (node / F.n[0]) % F.n[1] + F.lo[1],
              node / (F.n[0] * F.n[1]) + F.lo[2]};
  const int R = g.order - 1;
  int v0[3], v1[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    // nu with |m - 2 nu| <= R  ->  nu in [ceil((m - R)/2), floor((m + R)/2)]
    int lo = m[d] - R, hi = m[d] + R;
    int a = (lo >= 0) ? (lo + 1) / 2 : -((-lo) / 2);
    int b = (hi >= 0) ? hi / 2 : -((-hi + 1) / 2);
    v0[d] = max(a, C.lo[d]);
    v1[d] = min(b, C.lo[d] + C.n[d] - 1);
  }
  const float* uc = u + C.off;
  float acc = 0.f;
  for (int vz = v0[2]; vz <= v1[2]; ++vz) {
    float wz = pw.w[m[2] - 2 * vz + R];
    for (int vy = v0[1]; vy <= v1[1]; ++vy) {
      float wyz = wz * pw.w[m[1] - 2 * vy + R];
      const float* rowp = uc + ((size_t)(vz - C.lo[2]) * C.n[1] + (vy - C.lo[1])) * C.n[0] - C.lo[0];
      float racc = 0.f;
      for (int vx = v0[0]; vx <= v1[0]; ++vx) racc = fmaf(pw.w[m[0] - 2 * vx + R], rowp[vx], racc);
      acc = fmaf(wyz, racc, acc);
    }
  }
  u[F.off + node] = ucut[F.off + node] + acc;
}

// --------------------------------------------------------------------------
// Interpolation (itemised algorithm) and assembly (potential display, force as
// minus gradient):  phi_i^L = sum_mu phi^0_mu(r_i) u^0_mu,  grad phi_i^L,
//   phi_i = ke (phi^s + phi^L - q_i gamma(0)/a),  F_i = ke (F^s - q_i grad phi^L).
// Per-block float64 partials of E = 1/2 sum q_i phi_i and W = sum (r_i - lo) F_i.
// --------------------------------------------------------------------------
template <int ORDER>
__global__ void __launch_bounds__(kBlock) k_interp(Geom g, const float4* __restrict__ sorted,
                                                   const int* __restrict__ perm,
                                                   const float4* __restrict__ fshort,
                                                   const float* __restrict__ u,
                                                   float* __restrict__ fx, float* __restrict__ fy,
                                                   float* __restrict__ fz, float* __restrict__ phi,
                                                   double* __restrict__ partials, int n_partials) {
  constexpr int H = ORDER / 2;
  __shared__ double red[10][kBlock / kWave];
  const Level L = g.lv[0];
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  double e = 0.0, vir[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) vir[t] = 0.0;
  if (s < g.n_atoms) {
    float4 p = sorted[s];
    float pp[3] = {p.x, p.y, p.z};
    float w[3][ORDER], dw[3][ORDER];
    int base[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int f;
      float r;
      grid_coord(pp[d], g.lo_f[d], g.h, g.inv_h, g.fmax[d], f, r);
      basis<ORDER>(r, w[d], dw[d]);
      base[d] = f - (H - 1) - L.lo[d];
    }
    const float* u0 = u + L.off;
    float pl = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
    for (int sz = 0; sz < ORDER; ++sz) {
      float py_ = 0.f, gxy = 0.f, gyy = 0.f;
#pragma unroll
      for (int sy = 0; sy < ORDER; ++sy) {
        const float* rowp = u0 + ((size_t)(base[2] + sz) * L.n[1] + (base[1] + sy)) * L.n[0] + base[0];
        float vx = 0.f, dvx = 0.f;
#pragma unroll
        for (int sx = 0; sx < ORDER; ++sx) {
          float uv = rowp[sx];
          vx = fmaf(w[0][sx], uv, vx);
          dvx = fmaf(dw[0][sx], uv, dvx);
        }
        py_ = fmaf(w[1][sy], vx, py_);
        gxy = fmaf(w[1][sy], dvx, gxy);
        gyy = fmaf(dw[1][sy], vx, gyy);
      }
      pl = fmaf(w[2][sz], py_, pl);
      gx = fmaf(w[2][sz], gxy, gx);
      gy = fmaf(w[2][sz], gyy, gy);
      gz = fmaf(dw[2][sz], py_, gz);
    }
    gx *= g.inv_h;
    gy *= g.inv_h;
    gz *= g.inv_h;
    float4 fs = fshort[s];
    double qd = (double)p.w;
    double ph = g.ke * ((double)fs.w + (double)pl - qd * (double)g.self);
    float ofx = (float)(g.ke * ((double)fs.x - qd * (double)gx));
    float ofy = (float)(g.ke * ((double)fs.y - qd * (double)gy));
    float ofz = (float)(g.ke * ((double)fs.z - qd * (double)gz));
    int i = perm[s];
    if (fx) {
      fx[i] = ofx;
      fy[i] = ofy;
      fz[i] = ofz;
    }
    if (phi) phi[i] = (float)ph;
    e = 0.5 * qd * ph;
    double rr[3] = {(double)p.x - g.lo[0], (double)p.y - g.lo[1], (double)p.z - g.lo[2]};
    double ff[3] = {(double)ofx, (double)ofy, (double)ofz};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) vir[3 * a + b] = rr[a] * ff[b];
  }
  // fixed-order block reduction: butterfly within the wave, then waves in order
  double vals[10];
  vals[0] = e;
#pragma unroll
  for (int t = 0; t < 9; ++t) vals[t + 1] = vir[t];
#pragma unroll
  for (int t = 0; t < 10; ++t) {
    double v = vals[t];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    vals[t] = v;
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == 0)
#pragma unroll
    for (int t = 0; t < 10; ++t) red[t][wave] = vals[t];
  __syncthreads();
  if (threadIdx.x < 10) {
    double v = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) v += red[threadIdx.x][w];
    partials[(size_t)threadIdx.x * n_partials + blockIdx.x] = v;
  }
}

// Sum the per-block partials in a fixed order (one block).
__global__ void __launch_bounds__(kBlock) k_reduce(const double* __restrict__ partials, int n_partials,
                                                   double* __restrict__ energy,
                                                   double* __restrict__ virial) {
  __shared__ double red[kBlock];
  for (int t = 0; t < 10; ++t) {
    double v = 0.0;
    for (int b = threadIdx.x; b < n_partials; b += kBlock) v += partials[(size_t)t * n_partials + b];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int off = kBlock / 2; off >= 1; off >>= 1) {
      if (threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      if (t == 0) {
        if (energy) energy[0] = red[0];
      } else if (virial) {
        virial[t - 1] = red[0];
      }
    }
    __syncthreads();
  }
}

inline int blocks_for(int n, int b = kBlock) { return (n + b - 1) / b; }

}  // namespace

int interp_partials(const Geom& g) { return std::max(1, blocks_for(g.n_atoms)); }

hipError_t launch_forward(const Geom& g, const DevPtrs& d, int n_rows, int n_partials,
                          const int* restrict_j, const float* restrict_w, int n_restrict,
                          const float* prolong_w, hipStream_t s, const float* x, const float* y,
                          const float* z, const float* q, float* fx, float* fy, float* fz,
                          float* phi, double* energy, double* virial, hipEvent_t* ev) {
  const int n = g.n_atoms;
  auto mark = [&](int stage) {
    if (ev) (void)hipEventRecord(ev[stage], s);
  };
  mark(kStageBin);
  k_zero<<<blocks_for(std::max(g.n_cells + 1, 64)), kBlock, 0, s>>>(d.counts, d.cursor, g.n_cells,
                                                                   d.status);
  if (n > 0) {
    k_bin_count<<<blocks_for(n), kBlock, 0, s>>>(g, x, y, z, q, d.counts, d.cell_of, d.status);
    k_scan<<<1, 1024, 0, s>>>(d.counts, d.cell_start, g.n_cells);
    k_bin_scatter<<<blocks_for(n), kBlock, 0, s>>>(g, d.cell_of, d.cell_start, d.cursor, d.tmp);
    k_bin_place<<<blocks_for(n), kBlock, 0, s>>>(g, x, y, z, q, d.cell_of, d.cell_start, d.tmp,
                                                 d.sorted, d.perm, d.status);
    mark(kStageShort);
    int items = g.runs_x * g.nc[1] * g.nc[2];
    if (g.m == 1)
      k_short<1><<<items, kBlock, 0, s>>>(g, d.sorted, d.cell_start, d.fshort);
    else if (g.m == 2)
      k_short<2><<<items, kBlock, 0, s>>>(g, d.sorted, d.cell_start, d.fshort);
    else if (g.m == 3)
      k_short<3><<<items, kBlock, 0, s>>>(g, d.sorted, d.cell_start, d.fshort);
    else if (g.m == 4)
      k_short<4><<<items, kBlock, 0, s>>>(g, d.sorted, d.cell_start, d.fshort);
    else if (g.m == 5)
      k_short<5><<<items, kBlock, 0, s>>>(g, d.sorted, d.cell_start, d.fshort);
    else if (g.m == 6)
      k_short<6><<<items, kBlock, 0, s>>>(g, d.sorted, d.cell_start, d.fshort);
    else
      k_short<7><<<items, kBlock, 0, s>>>(g, d.sorted, d.cell_start, d.fshort);
  } else {
    k_scan<<<1, 1024, 0, s>>>(d.counts, d.cell_start, g.n_cells);
    mark(kStageShort);
  }
  mark(kStageAnterp);
  const Level& L0 = g.lv[0];
  if (g.order == 4)
    k_anterp<4><<<blocks_for(L0.count), kBlock, 0, s>>>(g, d.sorted, d.cell_start, d.qgrid);
  else
    k_anterp<6><<<blocks_for(L0.count), kBlock, 0, s>>>(g, d.sorted, d.cell_start, d.qgrid);
  mark(kStageRestrict);
  RestrictTaps rt{};
  rt.n = n_restrict;
  for (int t = 0; t < n_restrict; ++t) {
    rt.j[t] = restrict_j[t];
    rt.w[t] = restrict_w[t];
  }
  for (int k = 0; k + 1 < g.levels; ++k)
    k_restrict<<<blocks_for(g.lv[k + 1].count), kBlock, 0, s>>>(g, k, rt, d.qgrid);
  mark(kStageLattice);
  if (g.levels > 1) {
    int n_lat = g.lv[g.levels - 1].off;   // every node below the top level
    k_lattice<<<blocks_for(n_lat), kBlock, 0, s>>>(g, d.rows, n_rows, d.weights, d.qgrid, d.ucut,
                                                   n_lat);
  }
  mark(kStageTop);
  k_top<<<blocks_for(g.lv[g.levels - 1].count), kBlock, 0, s>>>(g, d.top, d.qgrid, d.ucut, d.u);
  mark(kStageProlong);
  ProlongW pw{};
  for (int t = 0; t < 2 * g.order - 1; ++t) pw.w[t] = prolong_w[t];
  for (int k = g.levels - 2; k >= 0; --k)
    k_prolong<<<blocks_for(g.lv[k].count), kBlock, 0, s>>>(g, k, pw, d.ucut, d.u);
  mark(kStageInterp);
  if (n > 0) {
    if (g.order == 4)
      k_interp<4><<<blocks_for(n), kBlock, 0, s>>>(g, d.sorted, d.perm, d.fshort, d.u, fx, fy, fz,
                                                   phi, d.partials, n_partials);
    else
      k_interp<6><<<blocks_for(n), kBlock, 0, s>>>(g, d.sorted, d.perm, d.fshort, d.u, fx, fy, fz,
                                                   phi, d.partials, n_partials);
  }
  mark(kStageReduce);
  if (energy || virial) {
    // with no atoms there are no partials and k_reduce writes zeros
    k_reduce<<<1, kBlock, 0, s>>>(d.partials, n > 0 ? n_partials : 0, energy, virial);
  }
  mark(kStageCount);
  return hipGetLastError();
}

}  // namespace msm
