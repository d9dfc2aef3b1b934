// gfx950 kernels of the multilevel summation method (thesis Sec. 2.3).
//
// One evaluation:
//   bin_count -> scan -> bin_scatter -> bin_place                 link cells (Sec. 2.1)
//   short_range                        (side stream)              u^short, F^short
//   anterpolate                                                   q^0
//   lattice, level 0                   (side stream)              u^{0,cut}
//   restrict (k = 0..l-2) -> lattice, levels 1..l-2 -> top (FP64) q^k, u^{k,cut}
//   prolong (every level, one launch)                             u^k
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


// A copy of the block's system descriptor in LDS (one round of 16-byte loads
// by the block, then a barrier).  Kernels that walk the level and tile tables
// with data-dependent indices read them from here: a chain of dependent scalar
// loads from the descriptor in global memory costs hundreds of cycles a link.
static_assert(sizeof(SysDesc) % 16 == 0, "descriptor copied in 16-byte words");
__device__ __forceinline__ const SysDesc& stage_desc(const SysDesc& src, SysDesc* dst) {
  const int4* __restrict__ s4 = reinterpret_cast<const int4*>(&src);
  int4* d4 = reinterpret_cast<int4*>(dst);
  for (int i = threadIdx.x; i < (int)(sizeof(SysDesc) / 16); i += blockDim.x) d4[i] = s4[i];
  __syncthreads();
  return *dst;
}

// Quotient and remainder of 0 <= i < 2^20 by 0 < d <= 2^10 with a float
// reciprocal (inv_d = 1/d rounded): (i + 1/2)/d lies at least 1/(2d) away from
// an integer, far more than the rounding error of (i + 1/2) * inv_d, so the
// truncation is exact.  Replaces the long integer-division sequence for
// runtime divisors in index arithmetic.
__device__ __forceinline__ int fdiv(int i, int d, float inv_d, int& rem) {
  const int q = (int)(((float)i + 0.5f) * inv_d);
  rem = i - q * d;
  return q;
}

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
// Counts are zero on entry: the workspace is initialised that way (for the
// cells of every reach a re-tune may select) and the scan clears them (with
// the scatter cursors and the status word) after reading.
__global__ void k_zero_counts(KArgs A) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  const int i = blk * blockDim.x + threadIdx.x;
  if (i <= S.g.max_cells) S.d.counts[i] = 0;
}

template <class G>
__device__ __forceinline__ int cell_coord(const G& g, float p, int d) {
  float t = (p - g.lo_f[d]) * g.inv_cs[d];
  t = fminf(fmaxf(t, 0.f), (float)(g.nc[d] - 1));   // NaN -> 0
  return min((int)t, g.nc[d] - 1);
}

// Coordinates as the kernels take them: a periodic plan maps each into
// [lo, lo + len), in double precision so the float32 result is the image
// rounded once (an atom inside the box keeps its coordinate; the result may
// round up to lo + len, which the cell and grid clamps absorb); free space
// keeps it.
template <class G>
__device__ __forceinline__ float wrap_coord(const G& g, float p, int d) {
  if (!g.periodic) return p;
  const double t = (double)p - g.lo[d];
  return (float)(g.lo[d] + (t - g.len[d] * floor(t / g.len[d])));
}

// The coordinate binning stores for an atom (wrapped, then clamped to the box).
__device__ __forceinline__ float sorted_coord(const Geom& g, float p, int d) {
  return fminf(fmaxf(wrap_coord(g, p, d), g.lo_f[d]), (float)g.hi[d]);
}

// An image of coordinate p shifted by s box edges, placed as the short-range
// pass stages it (shift added in double precision, rounded once).
__device__ __forceinline__ float shifted(float p, double s) { return (float)((double)p + s); }

__device__ __forceinline__ int cell_index(const Geom& g, float x, float y, float z) {
  return (cell_coord(g, wrap_coord(g, z, 2), 2) * g.nc[1] + cell_coord(g, wrap_coord(g, y, 1), 1)) * g.nc[0] +
         cell_coord(g, wrap_coord(g, x, 0), 0);
}

// Runs of equal cells among the lanes of a wave (consecutive input atoms —
// the sites of one molecule — often share a cell): a lane heads a run when
// its left neighbour (among the active lanes) has another cell.  Returns the
// run's length for its head (0 for the other lanes) and, in head, the lane
// of the run's head.  The whole wave must call it (inactive lanes pass
// active = false).
__device__ __forceinline__ int cell_run(int c, bool active, int& head) {
  const int lane = threadIdx.x & (kWave - 1);
  const int left = __shfl_up(c, 1);
  const unsigned long long act = __ballot(active);
  const bool starts = active && (lane == 0 || !((act >> (lane - 1)) & 1ull) || left != c);
  const unsigned long long heads = __ballot(starts);
  const unsigned long long upto = heads & (lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1ull));
  head = upto ? 63 - __clzll(upto) : lane;
  if (!starts) return 0;
  // the run ends at the next head or at the first inactive lane after it
  const unsigned long long stop = (heads | ~act) & (lane == kWave - 1 ? 0ull : ~((2ull << lane) - 1ull));
  const int end = stop ? __ffsll(stop) - 1 : kWave;
  return end - lane;
}

__global__ void k_bin_count(KArgs A) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  const Geom& g = S.g;
  if (g.bin_blocks || g.bin_row_blocks || g.binr_blocks) return;
  const int i = blk * blockDim.x + threadIdx.x;
  const bool active = i < g.n_atoms;
  int c = -1;
  if (active) {
    const float* x = A.io.x + S.atom_off;
    const float* y = A.io.y + S.atom_off;
    const float* z = A.io.z + S.atom_off;
    c = cell_index(g, x[i], y[i], z[i]);
    S.d.cell_of[i] = c;
  }
  int head;
  const int run = cell_run(c, active, head);
  if (run > 0) atomicAdd(&S.d.counts[c], run);
}

// Exclusive scan of counts[0..n) into start[0..n] in two launches over tiles
// of kScanTile cells (1024 threads, 4 cells each): k_scan_tiles writes each
// tile's total; k_scan_apply adds the totals of the earlier tiles (a fixed-
// order block sum), scans its tile, writes start[], and clears the counts and
// cursors (and, block 0, the status words) for this call.
constexpr int kScanThreads = kScanTile / 4;

// Block-wide sum of one int per thread (wave butterflies, then the waves in order).
__device__ __forceinline__ int block_sum_1024(int v, int* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  int t = 0;
#pragma unroll
  for (int w = 0; w < kScanThreads / kWave; ++w) t += red[w];
  return t;
}

__device__ __forceinline__ int4 load_counts4(const int* counts, int c, int n) {
  if (c + 3 < n) return *reinterpret_cast<const int4*>(counts + c);
  int4 v = make_int4(0, 0, 0, 0);
  if (c < n) v.x = counts[c];
  if (c + 1 < n) v.y = counts[c + 1];
  if (c + 2 < n) v.z = counts[c + 2];
  return v;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(KArgs A) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  if (S.g.bin_blocks || S.g.bin_row_blocks || S.g.binr_blocks) return;  // binned by another path
  __shared__ int red[kScanThreads / kWave];
  const int n = S.g.n_cells;
  const int4 v = load_counts4(S.d.counts, blk * kScanTile + 4 * (int)threadIdx.x, n);
  const int t = block_sum_1024(v.x + v.y + v.z + v.w, red);
  if (threadIdx.x == 0) S.d.scan[blk] = t;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_apply(KArgs A) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  if (S.g.bin_blocks || S.g.bin_row_blocks || S.g.binr_blocks) return;
  __shared__ int red[kScanThreads / kWave];
  __shared__ int wsum[kScanThreads / kWave];
  int* __restrict__ counts = S.d.counts;
  int* __restrict__ start = S.d.cell_start;
  int* __restrict__ cursor = S.d.cursor;
  const int n = S.g.n_cells;
  const int t = threadIdx.x;
  const int c = blk * kScanTile + 4 * t;
  const int4 v = load_counts4(counts, c, n);
  int before = 0;
  for (int b = t; b < blk; b += kScanThreads) before += S.d.scan[b];
  const int offset = block_sum_1024(before, red);
  // exclusive scan of the thread sums: within the wave, then over the waves
  const int own = v.x + v.y + v.z + v.w;
  const int lane = t & (kWave - 1), wv = t / kWave;
  int inc = own;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int u = __shfl_up(inc, off);
    if (lane >= off) inc += u;
  }
  if (lane == kWave - 1) wsum[wv] = inc;
  __syncthreads();
  int run = offset + inc - own;
  for (int w = 0; w < wv; ++w) run += wsum[w];
  const int e[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (c + u < n) {
      start[c + u] = run;
      run += e[u];
      counts[c + u] = 0;
      cursor[c + u] = 0;
    }
  if (c < n && c + 4 >= n) start[n] = run;           // the thread holding the last cell
  if (blk == 0 && t < 64) S.d.status[t] = 0;
}

// Scatter into cell segments in arrival order (atomic cursors); the atom's
// index and raw coordinates travel together so the next pass reads each
// segment contiguously.
__global__ void k_bin_scatter(KArgs A) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  if (S.g.bin_blocks || S.g.bin_row_blocks || S.g.binr_blocks) return;
  const int i = blk * blockDim.x + threadIdx.x;
  const bool active = i < S.g.n_atoms;
  const int* __restrict__ cell_of = S.d.cell_of;
  const int* __restrict__ start = S.d.cell_start;
  int* __restrict__ cursor = S.d.cursor;
  int* __restrict__ tmp = S.d.tmp;
  float4* __restrict__ tmp4 = S.d.fshort;   // coordinate copies until k_bin_place
  const int c = active ? cell_of[i] : -1;
  // one cursor atomic per run of equal cells; the run's lanes take
  // consecutive slots after the head's
  int head;
  const int run = cell_run(c, active, head);
  int base = 0;
  if (run > 0) base = start[c] + atomicAdd(&cursor[c], run);
  base = __shfl(base, head);
  if (!active) return;
  const float* x = A.io.x + S.atom_off;
  const float* y = A.io.y + S.atom_off;
  const float* z = A.io.z + S.atom_off;
  const float* q = A.io.q + S.atom_off;
  const float4 p = make_float4(x[i], y[i], z[i], q[i]);
  const int slot = base + ((int)(threadIdx.x & (kWave - 1)) - head);
  if ((unsigned)slot >= (unsigned)S.g.n_atoms) return;   // only a corrupted workspace gets here
  tmp[slot] = i;
  tmp4[slot] = p;
}

// Final slot of each atom = cell start + number of atoms of the same cell with
// a smaller input index (a stable order independent of the scatter's atomics).
// Also validates the input (non-finite, outside the box, coincident atoms) and
// writes sanitised, box-clamped coordinates so every later kernel stays inside
// the grid even for bad input.
__global__ void k_bin_place(KArgs A) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  const Geom& g = S.g;
  const int s = blk * blockDim.x + threadIdx.x;
  if (s >= g.n_atoms || g.bin_blocks || g.bin_row_blocks || g.binr_blocks) return;
  const int* __restrict__ cell_of = S.d.cell_of;
  const int* __restrict__ start = S.d.cell_start;
  const int* __restrict__ tmp = S.d.tmp;
  const float4* __restrict__ tmp4 = S.d.fshort;
  float4* __restrict__ sorted = S.d.sorted;
  int* __restrict__ perm = S.d.perm;
  int* __restrict__ status = S.d.status;
  const int i = tmp[s];
  if ((unsigned)i >= (unsigned)g.n_atoms) return;       // only a corrupted workspace gets here
  const float4 p = tmp4[s];
  const int c = cell_of[i];
  const int b = start[c], e = start[c + 1];
  int flags = 0;
  if (!(isfinite(p.x) && isfinite(p.y) && isfinite(p.z) && isfinite(p.w))) {
    flags |= kFlagNonFinite;
  } else {
    const double pd[3] = {(double)p.x, (double)p.y, (double)p.z};
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (!g.periodic && (pd[d] < g.lo[d] || pd[d] > g.hi[d])) flags |= kFlagOutOfBox;
  }
  int dst = s;
  if (s == b && e - b > kRankCap) atomicOr(status + kStatusUnranked, 1);
  if (0 <= b && b <= e && e <= g.n_atoms && e - b <= kRankCap) {
    int rank = 0;
#pragma unroll 4
    for (int t = b; t < e; ++t) {
      const int j = tmp[t];
      const float4 o = tmp4[t];
      rank += (j < i);
      if (j != i && o.x == p.x && o.y == p.y && o.z == p.z) flags |= kFlagCoincident;
    }
    dst = b + rank;
  }
  if (flags) atomicOr(status, flags);
  const float hx = (float)g.hi[0], hy = (float)g.hi[1], hz = (float)g.hi[2];
  float4 o;
  o.x = fminf(fmaxf(wrap_coord(g, p.x, 0), g.lo_f[0]), hx);
  o.y = fminf(fmaxf(wrap_coord(g, p.y, 1), g.lo_f[1]), hy);
  o.z = fminf(fmaxf(wrap_coord(g, p.z, 2), g.lo_f[2]), hz);
  o.w = isfinite(p.w) ? p.w : 0.f;
  sorted[dst] = o;
  perm[dst] = i;
}

// --------------------------------------------------------------------------
// Link cells in two kernels (systems whose cell counts fit in LDS).  Block b
// owns atoms [b kBinChunk, (b+1) kBinChunk).  k_bin_hist writes each block's
// cell counts; k_bin_sort gives every atom the slot
//   start[c] + (atoms of cell c in earlier blocks) + (atoms of cell c in this
//   block with a smaller input index),
// the same stable order as the four-kernel path, validates the input and
// writes the sorted, box-clamped atoms.  Coincident atoms are flagged by the
// short-range pass on this path.
// --------------------------------------------------------------------------
constexpr int kBinThreads = 1024;
constexpr int kBinPerThread = kBinChunk / kBinThreads;

__global__ void __launch_bounds__(kBinThreads) k_bin_hist(KArgs A) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  const Geom& g = S.g;
  extern __shared__ int hist[];
  const int nc = g.n_cells;
  for (int c = threadIdx.x; c < nc; c += kBinThreads) hist[c] = 0;
  if (blk == 0 && threadIdx.x < 64) S.d.status[threadIdx.x] = 0;
  __syncthreads();
  const float* x = A.io.x + S.atom_off;
  const float* y = A.io.y + S.atom_off;
  const float* z = A.io.z + S.atom_off;
  const int i0 = blk * kBinChunk;
#pragma unroll
  for (int u = 0; u < kBinPerThread; ++u) {
    const int i = i0 + u * kBinThreads + threadIdx.x;
    if (i < g.n_atoms) {
      const int c = cell_index(g, x[i], y[i], z[i]);
      S.d.cell_of[i] = c;
      atomicAdd(&hist[c], 1);
    }
  }
  __syncthreads();
  const int nc4 = (nc + 3) & ~3;                     // rows padded for 16-byte loads
  int* out = S.d.bin_hist + (size_t)blk * nc4;
  for (int c = threadIdx.x; c < nc4; c += kBinThreads) out[c] = c < nc ? hist[c] : 0;
}

__global__ void __launch_bounds__(kBinThreads) k_bin_sort(KArgs A) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  const Geom& g = S.g;
  extern __shared__ int lds[];
  const int nc = g.n_cells, nb = g.bin_blocks;
  int* base = lds;                 // [nc] first global slot of this block's atoms of cell c
  int* cur = base + nc;            // [nc] atoms of cell c in earlier blocks, then a cursor
  int* loc = cur + nc;             // [nc] first local slot of this block's atoms of cell c
  int* lidx = loc + nc;            // [kBinChunk] this block's atom indices grouped by cell
  int2* part = reinterpret_cast<int2*>(lidx + kBinChunk);   // [kBinThreads]
  const int t = threadIdx.x;
  // this thread's atoms (loads in flight during the scans)
  const float* x = A.io.x + S.atom_off;
  const float* y = A.io.y + S.atom_off;
  const float* z = A.io.z + S.atom_off;
  const float* q = A.io.q + S.atom_off;
  const int i0 = blk * kBinChunk;
  int cc[kBinPerThread];
  float4 p[kBinPerThread];
#pragma unroll
  for (int u = 0; u < kBinPerThread; ++u) {
    const int i = i0 + u * kBinThreads + t;
    cc[u] = -1;
    p[u] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (i < g.n_atoms) {
      cc[u] = S.d.cell_of[i];
      p[u] = make_float4(x[i], y[i], z[i], q[i]);
    }
  }
  // per cell: atoms over all blocks, in earlier blocks, in this block.
  // Thread t owns cells [t k, t k + k), k = 4 or 8 (rows of the block
  // histogram are padded to a multiple of 4, read 4 cells per load); the
  // loads of all its cells are in flight together, blocks taken 8 at a time.
  const int4* __restrict__ bh4 = reinterpret_cast<const int4*>(S.d.bin_hist);
  constexpr int kMaxK = kBinMaxCells / kBinThreads;
  const int nc4 = (nc + 3) & ~3, row4 = nc4 / 4;
  const int k = ((nc4 + kBinThreads - 1) / kBinThreads + 3) & ~3;
  const int c0 = min(t * k, nc), c1 = min(c0 + k, nc);
  const bool has = c0 < c1;
  int tot[kMaxK], pre[kMaxK], own[kMaxK];
#pragma unroll
  for (int u4 = 0; u4 < kMaxK / 4; ++u4) {
    const int4 v = (has && 4 * u4 < k && c0 + 4 * u4 < nc4) ? bh4[(size_t)blk * row4 + c0 / 4 + u4]
                                                             : make_int4(0, 0, 0, 0);
    own[4 * u4] = v.x;
    own[4 * u4 + 1] = v.y;
    own[4 * u4 + 2] = v.z;
    own[4 * u4 + 3] = v.w;
  }
#pragma unroll
  for (int u = 0; u < kMaxK; ++u) tot[u] = pre[u] = 0;
  for (int b0 = 0; b0 < nb; b0 += 8) {
    int4 v[8][kMaxK / 4];
#pragma unroll
    for (int w = 0; w < 8; ++w)
#pragma unroll
      for (int u4 = 0; u4 < kMaxK / 4; ++u4)
        v[w][u4] = (has && b0 + w < nb && 4 * u4 < k && c0 + 4 * u4 < nc4)
                       ? bh4[(size_t)(b0 + w) * row4 + c0 / 4 + u4]
                       : make_int4(0, 0, 0, 0);
#pragma unroll
    for (int w = 0; w < 8; ++w)
#pragma unroll
      for (int u4 = 0; u4 < kMaxK / 4; ++u4) {
        const int e[4] = {v[w][u4].x, v[w][u4].y, v[w][u4].z, v[w][u4].w};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          tot[4 * u4 + c] += e[c];
          pre[4 * u4 + c] += (b0 + w < blk) ? e[c] : 0;
        }
      }
  }
#pragma unroll
  for (int u = 0; u < kMaxK; ++u)
    if (c0 + u >= c1) tot[u] = pre[u] = own[u] = 0;   // padding cells
  // exclusive scans of the totals and of this block's counts
  int2 sum = make_int2(0, 0);
#pragma unroll
  for (int u = 0; u < kMaxK; ++u) {
    sum.x += tot[u];
    sum.y += own[u];
  }
  // inclusive scan of the thread sums: within each wave by shuffles, then
  // over the wave totals
  const int lane = t & (kWave - 1), wv = t / kWave;
  int2 inc = sum;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int vx = __shfl_up(inc.x, off), vy = __shfl_up(inc.y, off);
    if (lane >= off) {
      inc.x += vx;
      inc.y += vy;
    }
  }
  if (lane == kWave - 1) part[wv] = inc;
  __syncthreads();
  constexpr int kWaves = kBinThreads / kWave;
  if (t < kWave) {                                    // scan of the wave totals by wave 0
    int2 v = (t < kWaves) ? part[t] : make_int2(0, 0);
    const int2 own_total = v;
#pragma unroll
    for (int off = 1; off < kWaves; off <<= 1) {
      const int vx = __shfl_up(v.x, off), vy = __shfl_up(v.y, off);
      if (t >= off) {
        v.x += vx;
        v.y += vy;
      }
    }
    if (t < kWaves) part[kWaves + 1 + t] = make_int2(v.x - own_total.x, v.y - own_total.y);
    if (t == kWaves - 1) part[kWaves] = v;            // grand totals
  }
  __syncthreads();
  const int2 wpre = part[kWaves + 1 + wv];
  int run = wpre.x + inc.x - sum.x, lrun = wpre.y + inc.y - sum.y;
#pragma unroll
  for (int u = 0; u < kMaxK; ++u) {
    const int c = c0 + u;
    if (c < c1) {
      if (blk == 0) S.d.cell_start[c] = run;
      base[c] = run + pre[u];
      loc[c] = lrun;
      cur[c] = 0;
      run += tot[u];
      lrun += own[u];
    }
  }
  if (blk == 0 && t == kBinThreads - 1) S.d.cell_start[nc] = part[kWaves].x;
  __syncthreads();
  // group this block's atoms by cell in LDS (arrival order), then rank each
  // by input index within its cell
#pragma unroll
  for (int u = 0; u < kBinPerThread; ++u)
    if (cc[u] >= 0) lidx[loc[cc[u]] + atomicAdd(&cur[cc[u]], 1)] = i0 + u * kBinThreads + t;
  __syncthreads();
  int flags = 0;
#pragma unroll
  for (int u = 0; u < kBinPerThread; ++u) {
    if (cc[u] < 0) continue;
    const int i = i0 + u * kBinThreads + t;
    const int c = cc[u], l0 = loc[c], n = cur[c];
    int rank = 0;
    for (int j = 0; j < n; ++j) rank += (lidx[l0 + j] < i);
    const float4 pi = p[u];
    if (!(isfinite(pi.x) && isfinite(pi.y) && isfinite(pi.z) && isfinite(pi.w))) {
      flags |= kFlagNonFinite;
    } else {
      const double pd[3] = {(double)pi.x, (double)pi.y, (double)pi.z};
#pragma unroll
      for (int d = 0; d < 3; ++d)
        if (!g.periodic && (pd[d] < g.lo[d] || pd[d] > g.hi[d])) flags |= kFlagOutOfBox;
    }
    float4 o;
    o.x = fminf(fmaxf(wrap_coord(g, pi.x, 0), g.lo_f[0]), (float)g.hi[0]);
    o.y = fminf(fmaxf(wrap_coord(g, pi.y, 1), g.lo_f[1]), (float)g.hi[1]);
    o.z = fminf(fmaxf(wrap_coord(g, pi.z, 2), g.lo_f[2]), (float)g.hi[2]);
    o.w = isfinite(pi.w) ? pi.w : 0.f;
    S.d.sorted[base[c] + rank] = o;
    S.d.perm[base[c] + rank] = i;
  }
  if (flags) atomicOr(S.d.status, flags);
}

// --------------------------------------------------------------------------
// Link cells in one kernel (systems of at most kBinRowAtoms atoms).  Cells are
// numbered (cz ny + cy) nx + cx, so the cell row r = cz ny + cy holds the
// cells [r nx, (r + 1) nx).  Block b of B owns the rows [b R / B, (b + 1) R / B)
// of the R rows.  Every block walks all atoms of its system, each of its 16
// waves over a contiguous range of 64-atom chunks: it counts the atoms of
// earlier rows, counts per wave the atoms of each cell it owns, and lists in
// LDS (in input order) the wave's atoms that fall in its rows.  A prefix over
// the cells and the waves gives each (wave, cell) its first slot, and each
// wave places its listed atoms.  The order is the one of the other binning
// paths (cell, then input index), reached without any pass across blocks.
// Validation flags of a block's atoms go to its own status word.
// --------------------------------------------------------------------------
constexpr int kBRWaves = 16;
constexpr int kBRThreads = kBRWaves * kWave;
constexpr int kBRUnroll = 8;   // chunks of a wave whose loads are in flight together

__global__ void __launch_bounds__(kBRThreads) k_bin_rows(KArgs A) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  const Geom& g = S.g;
  extern __shared__ int lds[];
  // every descriptor field the kernel uses, read before its first store (the
  // compiler cannot keep later reads of the descriptor in scalar registers)
  const int n = g.n_atoms, nb = g.bin_row_blocks, nx = g.nc[0], ny = g.nc[1], nz = g.nc[2];
  const float lo0 = g.lo_f[0], lo1 = g.lo_f[1], lo2 = g.lo_f[2];
  const float iv0 = g.inv_cs[0], iv1 = g.inv_cs[1], iv2 = g.inv_cs[2];
  const double blo0 = g.lo[0], blo1 = g.lo[1], blo2 = g.lo[2];
  const double bhi0 = g.hi[0], bhi1 = g.hi[1], bhi2 = g.hi[2];
  const bool per = g.periodic != 0;
  const double ln0 = g.len[0], ln1 = g.len[1], ln2 = g.len[2];
  int* const status = S.d.status;
  int* const cell_start = S.d.cell_start;
  float4* const sorted = S.d.sorted;
  int* const perm = S.d.perm;
  const float* x = A.io.x + S.atom_off;
  const float* y = A.io.y + S.atom_off;
  const float* z = A.io.z + S.atom_off;
  const float* q = A.io.q + S.atom_off;
  const int rows = ny * nz;
  // (B <= kBinRowMaxBlocks and R <= B kBinRowCells: the products fit in 32 bits)
  const int r0 = (int)((unsigned)(blk * rows) / (unsigned)nb);
  const int r1 = (int)((unsigned)((blk + 1) * rows) / (unsigned)nb);
  const int own = (r1 - r0) * nx;                  // cells of the block: local index (r - r0) nx + cx
  int* cnt = lds;                                  // [kBRWaves][own] counts, then first slots
  int* red = cnt + kBRWaves * own;                 // [2 kBRWaves]
  unsigned short* list = reinterpret_cast<unsigned short*>(red + 2 * kBRWaves);   // [chunks * 64]
  const int t = threadIdx.x, lane = t & (kWave - 1);
  const int w = __builtin_amdgcn_readfirstlane(t / kWave);   // wave-uniform, in a scalar register
  const int nch = (n + kWave - 1) / kWave;
  const int cb = w * nch / kBRWaves, ce = (w + 1) * nch / kBRWaves;
  // whole batches of kBRUnroll chunks inside the atom range
  auto full = [&](int c0) { return c0 + kBRUnroll <= ce && (c0 + kBRUnroll) * kWave <= n; };
  // the first batch's loads are issued before the LDS is cleared and the
  // block meets at the barrier
  float fy[kBRUnroll], fz[kBRUnroll];
  const bool first = full(cb);
  if (first) {
#pragma unroll
    for (int u = 0; u < kBRUnroll; ++u) {
      fy[u] = y[(cb + u) * kWave + lane];
      fz[u] = z[(cb + u) * kWave + lane];
    }
  }
  for (int c = t; c < kBRWaves * own; c += kBRThreads) cnt[c] = 0;
  if (blk == 0 && t < 64) status[t] = 0;
  __syncthreads();
  int* wc = cnt + w * own;
  unsigned short* wl = list + cb * kWave;
  // cell coordinates as cell_index computes them, with the geometry in
  // registers (one median-of-three clamps to [0, mx], a NaN lands on 0 as
  // there; the final min of cell_index never changes a clamped value)
  const float mx0 = (float)(nx - 1), mx1 = (float)(ny - 1), mx2 = (float)(nz - 1);
  auto coord = [](float p, float lo, float iv, float mx) {
    return (int)__builtin_amdgcn_fmed3f((p - lo) * iv, 0.f, mx);
  };
  // periodic plans: the coordinate mapped into the box first (wrap_coord)
  auto wr = [&](float p, double lo, double ln) {
    if (!per) return p;
    const double t = (double)p - lo;
    return (float)(lo + (t - ln * floor(t / ln)));
  };
  auto local_cell = [&](float px, float py, float pz) {
    return (coord(wr(pz, blo2, ln2), lo2, iv2, mx2) * ny + coord(wr(py, blo1, ln1), lo1, iv1, mx1) - r0) * nx +
           coord(wr(px, blo0, ln0), lo0, iv0, mx0);
  };
  const unsigned span = (unsigned)(r1 - r0);
  int below = 0, len = 0;                          // wave-uniform
  // one chunk: count the atoms of earlier rows, list the block's own
  auto chunk = [&](int i, bool live, float py, float pz) {
    const int r = coord(wr(pz, blo2, ln2), lo2, iv2, mx2) * ny + coord(wr(py, blo1, ln1), lo1, iv1, mx1);
    below += __popcll(__ballot(live && r < r0));
    const bool mine = live && (unsigned)(r - r0) < span;
    const unsigned long long m = __ballot(mine);
    if (m) {
      if (mine) {
        const int before = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
        wl[len + before] = (unsigned short)i;
      }
      len += __popcll(m);
    }
  };
  int c = cb;
  if (first) {
#pragma unroll
    for (int u = 0; u < kBRUnroll; ++u) chunk((c + u) * kWave + lane, true, fy[u], fz[u]);
    c += kBRUnroll;
  }
  // the other whole batches: loads at fixed offsets, all in flight
  for (; full(c); c += kBRUnroll) {
    const int i0 = c * kWave + lane;
    float py[kBRUnroll], pz[kBRUnroll];
#pragma unroll
    for (int u = 0; u < kBRUnroll; ++u) {
      py[u] = y[i0 + u * kWave];
      pz[u] = z[i0 + u * kWave];
    }
#pragma unroll
    for (int u = 0; u < kBRUnroll; ++u) chunk(i0 + u * kWave, true, py[u], pz[u]);
  }
  for (; c < ce; ++c) {
    const int i = c * kWave + lane;
    const bool live = i < n;
    const int il = live ? i : n - 1;
    chunk(i, live, y[il], z[il]);
  }
  // per-wave counts of the listed atoms' cells; the first 64 listed atoms
  // stay in registers for the placement
  float4 p0 = make_float4(0.f, 0.f, 0.f, 0.f);
  int lc0 = -1;
  for (int e0 = 0; e0 < len; e0 += kWave) {
    const bool act = e0 + lane < len;
    const int i = act ? (int)wl[e0 + lane] : 0;
    const float4 pi = make_float4(x[i], y[i], z[i], q[i]);
    const int lc = act ? local_cell(pi.x, pi.y, pi.z) : -1;
    if (act) atomicAdd(&wc[lc], 1);
    if (e0 == 0) {
      p0 = pi;
      lc0 = lc;
    }
  }
  // first slot of every (wave, cell): atoms of earlier rows, of earlier cells
  // of the block, and of the same cell in earlier waves
  if (lane == 0) red[w] = below;
  __syncthreads();
  int v16[kBRWaves];
#pragma unroll
  for (int v = 0; v < kBRWaves; ++v) v16[v] = red[v];
  int base = 0;
#pragma unroll
  for (int v = 0; v < kBRWaves; ++v) base += v16[v];
  int tot = 0;
  if (t < own) {
#pragma unroll
    for (int v = 0; v < kBRWaves; ++v) v16[v] = cnt[v * own + t];
#pragma unroll
    for (int v = 0; v < kBRWaves; ++v) {
      const int e = v16[v];
      v16[v] = tot;
      tot += e;
    }
  }
  int inc = tot;                                   // inclusive scan over the cells (own <= threads)
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int v = __shfl_up(inc, off);
    if (lane >= off) inc += v;
  }
  if (lane == kWave - 1) red[kBRWaves + w] = inc;
  __syncthreads();
  int pre = 0;
#pragma unroll
  for (int v = 0; v < kBRWaves; ++v) {
    const int e = red[kBRWaves + v];
    pre += v < w ? e : 0;
  }
  const int start = base + pre + inc - tot;
  if (t < own) {
#pragma unroll
    for (int v = 0; v < kBRWaves; ++v) cnt[v * own + t] = v16[v] + start;
    cell_start[r0 * nx + t] = start;
  }
  if (blk == nb - 1 && t == 0) cell_start[rows * nx] = n;
  __syncthreads();
  // place the listed atoms: slot = first slot of (wave, cell) + atoms of the
  // same cell listed earlier by the wave
  int flags = 0;
  for (int e0 = 0; e0 < len; e0 += kWave) {
    const bool act = e0 + lane < len;
    const int i = act ? (int)wl[e0 + lane] : 0;
    float4 pi = p0;
    int lc = lc0;
    if (e0 > 0) {
      pi = make_float4(x[i], y[i], z[i], q[i]);
      lc = act ? local_cell(pi.x, pi.y, pi.z) : -1;
    }
    int rank = 0;
    for (unsigned long long b = __ballot(act); b; b &= b - 1) {
      const int j = __builtin_ctzll(b);
      const int lj = __builtin_amdgcn_readlane(lc, j);
      rank += (j < lane && lj == lc) ? 1 : 0;
    }
    if (act) {
      const int slot = wc[lc] + rank;
      atomicAdd(&wc[lc], 1);
      if (!(isfinite(pi.x) && isfinite(pi.y) && isfinite(pi.z) && isfinite(pi.w))) {
        flags |= kFlagNonFinite;
      } else {
        const double px = pi.x, py = pi.y, pz = pi.z;
        if (!per && (px < blo0 || px > bhi0 || py < blo1 || py > bhi1 || pz < blo2 || pz > bhi2))
          flags |= kFlagOutOfBox;
      }
      float4 o;
      o.x = fminf(fmaxf(wr(pi.x, blo0, ln0), lo0), (float)bhi0);
      o.y = fminf(fmaxf(wr(pi.y, blo1, ln1), lo1), (float)bhi1);
      o.z = fminf(fmaxf(wr(pi.z, blo2, ln2), lo2), (float)bhi2);
      o.w = isfinite(pi.w) ? pi.w : 0.f;
      sorted[slot] = o;
      perm[slot] = i;
    }
  }
  // the block's flags: wave ORs by ballot, then over the waves
  const int wf = (__ballot(flags & kFlagOutOfBox) ? kFlagOutOfBox : 0) |
                 (__ballot(flags & kFlagNonFinite) ? kFlagNonFinite : 0);
  if (lane == 0) red[w] = wf;
  __syncthreads();
  if (t == 0) {
    int f = 0;
#pragma unroll
    for (int v = 0; v < kBRWaves; ++v) f |= red[v];
    status[64 + blk] = f;
  }
}

// --------------------------------------------------------------------------
// Link cells of a large system in four kernels, by cell row first: the cells
// are numbered (cz ny + cy) nx + cx, so a cell row r = cz ny + cy is a
// contiguous range of cells.
//   k_binr_count   per block of kBinRChunk atoms: LDS counts of the rows, one
//                  global add per row into counts[]
//   k_binr_scan    row starts (exclusive scan of counts[]); clears counts[]
//                  and the row cursors for the scatter and the next call
//   k_binr_scatter the atoms into their row's segment (LDS counts give every
//                  block a range per row; order inside it is arbitrary)
//   k_binr_sort    one block per row: counting sort of the row's atoms by x
//                  cell, each atom ranked in its cell by input index (the
//                  order of the other binning paths), validation, the sorted
//                  and box-clamped atoms and the row's cell starts.
// The row starts live in the scan array.
// --------------------------------------------------------------------------
constexpr int kBRCThreads = 1024;
constexpr int kBRCPer = kBinRChunk / kBRCThreads;
constexpr int kBRSThreads = 256;
static_assert(kBinRSortCap % kBRSThreads == 0 && kBinRSortCap <= kRankCap, "a cached row ranks every cell");
static_assert(kBinRSortCap <= 65536 && kBinRowsMax <= 65536, "16-bit x cells and positions");

__device__ __forceinline__ int cell_row(const Geom& g, float y, float z) {
  return cell_coord(g, wrap_coord(g, z, 2), 2) * g.nc[1] + cell_coord(g, wrap_coord(g, y, 1), 1);
}

// Exclusive scan of a[0, n) in place by the block's NT threads (thread t
// takes a contiguous run of ceil(n / NT) entries); returns the total.
template <int NT>
__device__ int block_exclusive_scan(int* a, int n, int* wsum) {
  constexpr int NW = NT / kWave;
  const int t = threadIdx.x, lane = t & (kWave - 1), wv = t / kWave;
  const int per = (n + NT - 1) / NT;
  const int b = min(t * per, n), e = min(b + per, n);
  int own = 0;
  for (int i = b; i < e; ++i) own += a[i];
  int inc = own;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int u = __shfl_up(inc, off);
    if (lane >= off) inc += u;
  }
  if (lane == kWave - 1) wsum[wv] = inc;
  __syncthreads();
  int run = inc - own, total = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const int v = wsum[w];
    run += w < wv ? v : 0;
    total += v;
  }
  for (int i = b; i < e; ++i) {
    const int v = a[i];
    a[i] = run;
    run += v;
  }
  __syncthreads();
  return total;
}

__global__ void __launch_bounds__(kBRCThreads) k_binr_count(KArgs A) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  const Geom& g = S.g;
  if (!g.binr_blocks) return;
  __shared__ int hist[kBinRowsMax];
  const int rows = g.nc[1] * g.nc[2];
  for (int r = threadIdx.x; r < rows; r += kBRCThreads) hist[r] = 0;
  __syncthreads();
  const float* y = A.io.y + S.atom_off;
  const float* z = A.io.z + S.atom_off;
  const int i0 = blk * kBinRChunk;
  float py[kBRCPer], pz[kBRCPer];
#pragma unroll
  for (int u = 0; u < kBRCPer; ++u) {
    const int i = i0 + u * kBRCThreads + threadIdx.x;
    py[u] = i < g.n_atoms ? y[i] : 0.f;
    pz[u] = i < g.n_atoms ? z[i] : 0.f;
  }
#pragma unroll
  for (int u = 0; u < kBRCPer; ++u)
    if (i0 + u * kBRCThreads + (int)threadIdx.x < g.n_atoms) atomicAdd(&hist[cell_row(g, py[u], pz[u])], 1);
  __syncthreads();
  int* __restrict__ counts = S.d.counts;
  for (int r = threadIdx.x; r < rows; r += kBRCThreads) {
    const int c = hist[r];
    if (c) atomicAdd(&counts[r], c);
  }
}

__global__ void __launch_bounds__(kBRCThreads) k_binr_scan(KArgs A) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  const Geom& g = S.g;
  if (!g.binr_blocks) return;
  __shared__ int wsum[kBRCThreads / kWave];
  __shared__ int st[kBinRowsMax];
  const int rows = g.nc[1] * g.nc[2];
  int* __restrict__ counts = S.d.counts;
  int* __restrict__ row_start = S.d.scan;
  int* __restrict__ cursor = S.d.cursor;
  for (int r = threadIdx.x; r < rows; r += kBRCThreads) {
    st[r] = counts[r];
    counts[r] = 0;
    cursor[r] = 0;
  }
  if (threadIdx.x < 64) S.d.status[threadIdx.x] = 0;
  __syncthreads();
  const int total = block_exclusive_scan<kBRCThreads>(st, rows, wsum);
  for (int r = threadIdx.x; r < rows; r += kBRCThreads) row_start[r] = st[r];
  if (threadIdx.x == 0) {
    row_start[rows] = total;
    S.d.cell_start[g.n_cells] = total;
  }
}

__global__ void __launch_bounds__(kBRCThreads) k_binr_scatter(KArgs A) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  const Geom& g = S.g;
  if (!g.binr_blocks) return;
  __shared__ int hist[kBinRowsMax];
  __shared__ int base[kBinRowsMax];
  const int rows = g.nc[1] * g.nc[2], n = g.n_atoms;
  for (int r = threadIdx.x; r < rows; r += kBRCThreads) hist[r] = 0;
  __syncthreads();
  const float* x = A.io.x + S.atom_off;
  const float* y = A.io.y + S.atom_off;
  const float* z = A.io.z + S.atom_off;
  const float* q = A.io.q + S.atom_off;
  const int i0 = blk * kBinRChunk;
  float4 p[kBRCPer];
  int rr[kBRCPer];
#pragma unroll
  for (int u = 0; u < kBRCPer; ++u) {
    const int i = i0 + u * kBRCThreads + threadIdx.x;
    p[u] = i < g.n_atoms ? make_float4(x[i], y[i], z[i], q[i]) : make_float4(0.f, 0.f, 0.f, 0.f);
  }
#pragma unroll
  for (int u = 0; u < kBRCPer; ++u) {
    const int i = i0 + u * kBRCThreads + threadIdx.x;
    rr[u] = -1;
    if (i < g.n_atoms) {
      rr[u] = cell_row(g, p[u].y, p[u].z);
      atomicAdd(&hist[rr[u]], 1);
    }
  }
  __syncthreads();
  // this block's range in every row it touches, then its counts become cursors
  const int* __restrict__ row_start = S.d.scan;
  int* __restrict__ cursor = S.d.cursor;
  for (int r = threadIdx.x; r < rows; r += kBRCThreads) {
    const int c = hist[r];
    if (c) base[r] = row_start[r] + atomicAdd(&cursor[r], c);
    hist[r] = 0;
  }
  __syncthreads();
  int* __restrict__ tmp = S.d.tmp;
  float4* __restrict__ tmp4 = S.d.fshort;   // coordinate copies until k_binr_sort
#pragma unroll
  for (int u = 0; u < kBRCPer; ++u)
    if (rr[u] >= 0) {
      const int slot = base[rr[u]] + atomicAdd(&hist[rr[u]], 1);
      if ((unsigned)slot < (unsigned)n) {                 // only a corrupted workspace fails this
        tmp[slot] = i0 + u * kBRCThreads + threadIdx.x;
        tmp4[slot] = p[u];
      }
    }
}

// The binning geometry in registers: kernels that store to global memory in
// a loop would otherwise reload every descriptor field after each store (the
// compiler cannot rule out that the store changed it).
struct BinGeo {
  float lo_f[3], inv_cs[3];
  double lo[3], hi[3], len[3];
  int nc[3];
  int periodic;
};

__device__ __forceinline__ BinGeo bin_geo(const Geom& s) {
  BinGeo b;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    b.lo_f[d] = s.lo_f[d];
    b.inv_cs[d] = s.inv_cs[d];
    b.lo[d] = s.lo[d];
    b.hi[d] = s.hi[d];
    b.len[d] = s.len[d];
    b.nc[d] = s.nc[d];
  }
  b.periodic = s.periodic;
  return b;
}

// One validated, box-clamped atom of the row binning at its final slot;
// returns its validation flags.
__device__ __forceinline__ int binr_place(const BinGeo& g, const float4 p, int i, int dst, float4* sorted, int* perm) {
  int flags = 0;
  if (!(isfinite(p.x) && isfinite(p.y) && isfinite(p.z) && isfinite(p.w))) {
    flags |= kFlagNonFinite;
  } else if (!g.periodic) {
    const double pd[3] = {(double)p.x, (double)p.y, (double)p.z};
#pragma unroll
    for (int d = 0; d < 3; ++d)
      if (pd[d] < g.lo[d] || pd[d] > g.hi[d]) flags |= kFlagOutOfBox;
  }
  float4 o;
  o.x = fminf(fmaxf(wrap_coord(g, p.x, 0), g.lo_f[0]), (float)g.hi[0]);
  o.y = fminf(fmaxf(wrap_coord(g, p.y, 1), g.lo_f[1]), (float)g.hi[1]);
  o.z = fminf(fmaxf(wrap_coord(g, p.z, 2), g.lo_f[2]), (float)g.hi[2]);
  o.w = isfinite(p.w) ? p.w : 0.f;
  sorted[dst] = o;
  perm[dst] = i;
  return flags;
}

__global__ void __launch_bounds__(kBRSThreads) k_binr_sort(KArgs A) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  if (!S.g.binr_blocks) return;
  const BinGeo g = bin_geo(S.g);
  extern __shared__ int lds[];
  __shared__ int wsum[kBRSThreads / kWave];
  __shared__ int bflags;
  const int nx = g.nc[0], n = S.g.n_atoms;
  const int ints = (2 * (nx + 1) + 3) & ~3;
  int* lstart = lds;                                   // [nx + 1] x-cell counts, then starts
  int* lcur = lds + nx + 1;                            // [nx + 1] cursors of the bucket fill
  // a row of at most kBinRSortCap atoms, in bucket (x cell) order
  float4* bpos = reinterpret_cast<float4*>(lds + ints);                 // [cap] coordinates and charge
  int* bid = reinterpret_cast<int*>(bpos + kBinRSortCap);               // [cap] input indices
  unsigned short* bcx = reinterpret_cast<unsigned short*>(bid + kBinRSortCap);   // [cap] x cells
  const int* __restrict__ row_start = S.d.scan;
  const int* __restrict__ tmp = S.d.tmp;
  const float4* __restrict__ tmp4 = S.d.fshort;
  int* __restrict__ gord = S.d.cell_of;                // bucket order of a row too long for the LDS
  const int r = blk;
  const int rs = row_start[r], re = row_start[r + 1];
  if (rs < 0 || re < rs || re > n) return;             // only a corrupted workspace gets here
  const int cnt = re - rs;
  const bool cached = cnt <= kBinRSortCap;
  constexpr int kPer = kBinRSortCap / kBRSThreads;     // atoms per thread of a cached row
  for (int c = threadIdx.x; c <= nx; c += kBRSThreads) {
    lstart[c] = 0;
    lcur[c] = 0;
  }
  if (threadIdx.x == 0) bflags = 0;
  // a cached row's atoms stay in registers until the bucket fill
  float4 mp[kPer];
  int mid[kPer], mcx[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int t = u * kBRSThreads + threadIdx.x;
    mcx[u] = -1;
    mp[u] = make_float4(0.f, 0.f, 0.f, 0.f);
    mid[u] = 0;
    if (cached && t < cnt) {
      mp[u] = tmp4[rs + t];
      mid[u] = tmp[rs + t];
      mcx[u] = cell_coord(g, wrap_coord(g, mp[u].x, 0), 0);
    }
  }
  __syncthreads();
  if (cached) {
#pragma unroll
    for (int u = 0; u < kPer; ++u)
      if (mcx[u] >= 0) atomicAdd(&lstart[mcx[u]], 1);
  } else {
    for (int t = threadIdx.x; t < cnt; t += kBRSThreads) atomicAdd(&lstart[cell_coord(g, wrap_coord(g, tmp4[rs + t].x, 0), 0)], 1);
  }
  __syncthreads();
  block_exclusive_scan<kBRSThreads>(lstart, nx, wsum);
  if (threadIdx.x == 0) lstart[nx] = cnt;
  __syncthreads();
  int* __restrict__ cell_start = S.d.cell_start;
  for (int c = threadIdx.x; c < nx; c += kBRSThreads) cell_start[r * nx + c] = rs + lstart[c];
  int flags = 0;
  float4* __restrict__ sorted = S.d.sorted;
  int* __restrict__ perm = S.d.perm;
  if (cached) {
    // buckets by x cell (arrival order), then every atom ranked by input
    // index among its cell's members (contiguous in LDS); coincident atoms
    // share a cell.  A cached row is shorter than kRankCap.
#pragma unroll
    for (int u = 0; u < kPer; ++u)
      if (mcx[u] >= 0) {
        const int slot = lstart[mcx[u]] + atomicAdd(&lcur[mcx[u]], 1);
        bpos[slot] = mp[u];
        bid[slot] = mid[u];
        bcx[slot] = (unsigned short)mcx[u];
      }
    __syncthreads();
    for (int k = threadIdx.x; k < cnt; k += kBRSThreads) {
      const int cx = bcx[k], b = lstart[cx], e = lstart[cx + 1];
      const int i = bid[k];
      const float4 p = bpos[k];
      int rank = 0;
      for (int k2 = b; k2 < e; ++k2) {
        rank += (bid[k2] < i);
        const float4 o = bpos[k2];
        if (k2 != k && o.x == p.x && o.y == p.y && o.z == p.z) flags |= kFlagCoincident;
      }
      flags |= binr_place(g, p, i, rs + b + rank, sorted, perm);
    }
  } else {
    // a long row: bucket order as row positions in global scratch; an atom
    // of a cell longer than kRankCap stays at its arrival slot (as in the
    // four kernels over the cells)
    for (int t = threadIdx.x; t < cnt; t += kBRSThreads) {
      const float4 p = tmp4[rs + t];
      const int cx = cell_coord(g, wrap_coord(g, p.x, 0), 0);
      const int slot = lstart[cx] + atomicAdd(&lcur[cx], 1);
      gord[rs + slot] = t;
      if (lstart[cx + 1] - lstart[cx] > kRankCap) {
        flags |= binr_place(g, p, tmp[rs + t], rs + slot, sorted, perm);
        if (slot == lstart[cx]) atomicOr(S.d.status + kStatusUnranked, 1);
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += kBRSThreads) {
      const float4 p = tmp4[rs + t];
      const int i = tmp[rs + t];
      const int cx = cell_coord(g, wrap_coord(g, p.x, 0), 0);
      const int b = lstart[cx], e = lstart[cx + 1];
      if (e - b > kRankCap) continue;
      int rank = 0;
      for (int k = b; k < e; ++k) {
        const int u = gord[rs + k];
        rank += (tmp[rs + u] < i);
        if (u != t) {
          const float4 o = tmp4[rs + u];
          if (o.x == p.x && o.y == p.y && o.z == p.z) flags |= kFlagCoincident;
        }
      }
      flags |= binr_place(g, p, i, rs + b + rank, sorted, perm);
    }
  }
  if (flags) atomicOr(&bflags, flags);
  __syncthreads();
  if (threadIdx.x == 0 && bflags) atomicOr(S.d.status, bflags);
}

// --------------------------------------------------------------------------
// Short-range part (itemised algorithm, first sentence; eq. msmgrid g*):
//   phi_i^s = sum_j q_j g*(r_ij),  F_i^s = -q_i sum_j q_j g*'(r_ij) (r_i - r_j)/r_ij
//   g*(r) = 1/r - gamma(r/a)/a,  g*'(r)/r = -1/r^3 - gamma'(r/a)/(a^2 r)
// Work items: the atoms of a cell row are contiguous in sorted order (x
// cells, then input order) and are cut into 64-atom chunks, one atom per lane.
// The neighbour atoms of a chunk lie in the (2 reach + 1)^2 cell rows around
// it (y, z offsets up to reach).  For each such row every lane cuts its own
// window: with d the distance of the atom to the row in (y, z), only x cells
// within sqrt(a^2 - d^2) of the atom can hold partners, a contiguous range of
// sorted atoms.  A wave stages the union of its lanes' windows in LDS (one
// coalesced load per 256 atoms) and each lane walks its own range (gathered
// LDS reads).  In free space a row and its mirror row are walked as one unit
// (both unions staged, each lane's two windows back to back), which evens out
// the lanes' walk lengths; the units are dealt to the block's 4 waves by
// expected window length (fixed per plan); the waves' partial sums meet in
// LDS and are added in wave order.
// --------------------------------------------------------------------------
constexpr int kShortThreads = kShortWaves * kWave;
constexpr int kShortSeg = 256;                   // j atoms a wave stages at a time (one row)
constexpr int kShortBuf = 312;                   // entries of a wave's staging buffer (a row pair; 4 waves x 312 x 16 B: 8 blocks per CU)
static_assert(kShortBuf >= kShortSeg + 4 && kShortSeg % kWave == 0, "short-range staging sizes");

__device__ __forceinline__ int cell_x(const Geom& g, float x) {
  float t = (x - g.lo_f[0]) * g.inv_cs[0];
  t = fminf(fmaxf(t, 0.f), (float)(g.nc[0] - 1));   // NaN -> 0
  return min((int)t, g.nc[0] - 1);
}

// Minimum / maximum over the 64 lanes of a wave (every lane active), returned
// in a scalar register, with DPP moves instead of LDS permutes: row_shr 1, 2,
// 4, 8 leave the extreme of each 16-lane row in its lane 15, row_bcast 15 and
// row_bcast 31 carry it across the rows into lane 63.
__device__ __forceinline__ int wave_min_s(int v) {
  v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x111, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x112, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x114, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x118, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x142, 0xa, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(INT_MAX, v, 0x143, 0xc, 0xf, false));
  return __builtin_amdgcn_readlane(v, 63);
}

__device__ __forceinline__ int wave_max_s(int v) {
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x111, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x112, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x114, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x118, 0xf, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x142, 0xa, 0xf, false));
  v = max(v, __builtin_amdgcn_update_dpp(INT_MIN, v, 0x143, 0xc, 0xf, false));
  return __builtin_amdgcn_readlane(v, 63);
}

// Sum over the 64 lanes of a wave (every lane active) in a fixed order, the
// same DPP pattern on the two halves of each double; the total is in lane 63.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_shift_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double wave_sum_d63(double v) {
  v += dpp_shift_d<0x111, 0xf>(v);
  v += dpp_shift_d<0x112, 0xf>(v);
  v += dpp_shift_d<0x114, 0xf>(v);
  v += dpp_shift_d<0x118, 0xf>(v);
  v += dpp_shift_d<0x142, 0xa>(v);
  v += dpp_shift_d<0x143, 0xc>(v);
  return v;
}

// A launch takes the work items [n lo_pm / 1000, n hi_pm / 1000) of each system.
// binom(-1/2, j): the coefficients of the Taylor polynomial of s^{-1/2} about
// s = 1 in powers of (s - 1) (exact dyadic rationals).
constexpr float binom_half(int j) {
  double v = 1.0;
  for (int i = 0; i < j; ++i) v *= (-0.5 - i) / (i + 1);
  return (float)v;
}

// erfc(x) for the Wolf pair function from ex = exp(-x^2): erfc(x) exp(x^2) is
// a polynomial in t = 1 / (1 + x/2) whose coefficients ec the plan fits (in
// double, rounded to float one at a time with the rest refitted); t takes the
// hardware reciprocal and one Newton step (the raw instruction's error is
// biased, as for the reciprocal square root).
__device__ __forceinline__ float wolf_erfc(const float* ec, float x, float ex) {
  const float d = fmaf(0.5f, x, 1.f);
  float t = __builtin_amdgcn_rcpf(d);
  t = fmaf(t, fmaf(-d, t, 1.f), t);
  float p = ec[kWolfTerms - 1];
#pragma unroll
  for (int k = kWolfTerms - 2; k >= 0; --k) p = fmaf(p, t, ec[k]);
  return p * ex;
}

// KIND selects the pair function: the MSM short-range kernel g* (gamma of
// degree M), or a cheap pair method on its own with e(r) and -e'(r)/r
//   plain cutoff     e = 1/r                                -e'/r = 1/r^3
//   shifted force    e = 1/r + r pk1 - 2 pk0                -e'/r = (1/r^2 - pk1)/r
//                    (pk0 = 1/rc, pk1 = 1/rc^2)
//   Wolf             e = erfc(pk0 r)/r - pk1                -e'/r = (erfc(pk0 r)/r + pk2 exp(-alpha^2 r^2))/r^2
//                    (pk0 = alpha, pk1 = erfc(alpha rc)/rc, pk2 = 2 alpha/sqrt(pi), pk3 = -alpha^2 log2(e), so that
//                    exp(-alpha^2 r^2) = 2^(pk3 r^2), the hardware exp2 (which may flush results
//                    below 2^-126 to zero: there erfc(alpha r) < 1e-38); erfc from the plan's
//                    polynomial and that one exponential)
// PER: periodic plans (the neighbour rows and x windows wrap around the box,
// the atoms of a wrapped image staged shifted by the box edges); a template
// flag so the free-space kernel keeps its registers.
// The lane's x window in the free-space neighbour row of offsets code r
// ((oy + R) | (oz + R) << 4) around cell row (cy, cz): the sorted atoms of the
// x cells within sqrt(aw^2 - d^2) of the atom, d its distance to the row in
// (y, z); empty (lo > hi) outside the box, for a dead lane or a row beyond aw.
__device__ __forceinline__ void row_window(const Geom& g, const int* start, int cy, int cz, int r, int R,
                                           const float4& pi, bool live, float aw, int& lo, int& hi) {
  lo = 0x7fffffff;
  hi = -1;
  const int jy = cy + (r & 15) - R, jz = cz + (r >> 4) - R;
  if (!live || jy < 0 || jz < 0 || jy >= g.nc[1] || jz >= g.nc[2]) return;
  const float ylo = g.lo_f[1] + (float)jy * g.cs[1], zlo = g.lo_f[2] + (float)jz * g.cs[2];
  const float dyw = fmaxf(fmaxf(ylo - pi.y, pi.y - (ylo + g.cs[1])), 0.f);
  const float dzw = fmaxf(fmaxf(zlo - pi.z, pi.z - (zlo + g.cs[2])), 0.f);
  const float d2 = fmaf(dyw, dyw, dzw * dzw);
  if (!(d2 < aw * aw)) return;
  const float e = sqrtf(aw * aw - d2) + 1e-4f * aw;
  const int jrow = (jz * g.nc[1] + jy) * g.nc[0];
  lo = start[jrow + cell_x(g, pi.x - e)];
  hi = start[jrow + cell_x(g, pi.x + e) + 1];
}

// Four staged j atoms against the lane's atom pi: the pair function of KIND
// for each one with 0 < r^2 < a^2, added to the lane's sums.
template <int M, bool FORCES, int KIND>
__device__ __forceinline__ void short_pairs4(const float4* jp, const float4& pi, unsigned a2m1, float inv_a,
                                             float inv_a2, const float* dc, const float* pk, const float* ec,
                                             float& ax, float& ay, float& az, float& ap) {
  float4 pj[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) pj[v] = jp[v];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const float dx = pi.x - pj[v].x, dy = pi.y - pj[v].y, dz = pi.z - pj[v].z;
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    // one predicate (non-short-circuit), so a single branch per pair
    // 0 < r2 < a2 as one unsigned compare of the bit patterns (r2 >= +0)
    if (__float_as_uint(r2) - 1u < a2m1) {
      // hardware reciprocal square root plus one Newton step (the raw
      // instruction's error is biased, which would bias the energy)
      float ri = __builtin_amdgcn_rsqf(r2);
      ri = fmaf(0.5f * ri, fmaf(-r2 * ri, ri, 1.f), ri);
      const float qj = pj[v].w;
      if (KIND == kPairMsm) {
        // g*(r) = 1/r - gamma(r/a)/a with gamma the Taylor polynomial of
        // s^{-1/2} in t = s - 1, s = (r/a)^2: exact coefficients and
        // every term of one sign, then one rounding for the difference.
        // (Horner in r^2 with the rounded coefficients c_k / a^{2k+1}
        // leaves a fixed bias in every pair that does not average out
        // over the pairs of rigid molecules.)
        const float t = fmaf(r2, inv_a2, -1.f);
        float gm = binom_half(M);
#pragma unroll
        for (int k = M - 1; k >= 0; --k) gm = fmaf(gm, t, binom_half(k));
        ap = fmaf(qj, fmaf(-gm, inv_a, ri), ap);
        // gamma'(r/a)/(a^2 r) as a polynomial in r^2
        float dg = dc[M];
#pragma unroll
        for (int k = M - 1; k >= 1; --k) dg = fmaf(dg, r2, dc[k]);
        if (FORCES) {
          const float wq = qj * fmaf(ri, ri * ri, dg);  // q_j (-g*'(r)/r)
          ax = fmaf(wq, dx, ax);
          ay = fmaf(wq, dy, ay);
          az = fmaf(wq, dz, az);
        }
      } else {
        float e, fr;                                     // e(r), -e'(r)/r
        if (KIND == kPairCutoff) {
          e = ri;
          fr = ri * ri * ri;
        } else if (KIND == kPairShiftedForce) {
          e = ri + fmaf(r2 * ri, pk[1], -2.f * pk[0]);
          fr = ri * fmaf(ri, ri, -pk[1]);
        } else {
          const float ex = __builtin_amdgcn_exp2f(pk[3] * r2);
          const float er = wolf_erfc(ec, pk[0] * (r2 * ri), ex);
          e = fmaf(er, ri, -pk[1]);
          fr = ri * ri * fmaf(er, ri, pk[2] * ex);
        }
        ap = fmaf(qj, e, ap);
        if (FORCES) {
          const float wq = qj * fr;
          ax = fmaf(wq, dx, ax);
          ay = fmaf(wq, dy, ay);
          az = fmaf(wq, dz, az);
        }
      }
    }
  }
}

template <int M, bool FORCES, int KIND, bool PER>
// Eight 4-wave blocks per CU (LDS 20 KB each): 8 waves per SIMD, so at most 64
// registers per lane.
__global__ void __launch_bounds__(kShortThreads, 8) k_short(KArgs A, int lo_pm, int hi_pm) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  const Geom& g = S.g;
  const float4* __restrict__ sorted = S.d.sorted;
  const int* __restrict__ start = S.d.cell_start;
  float4* __restrict__ fshort = S.d.fshort;
  // staged j atoms of each wave (one row segment, or a row pair) with 4
  // far-away uncharged entries after each row: a lane reads 4 entries at a
  // time, and every entry past its window fails the cutoff test (same-row
  // atoms beyond the window lie farther than a)
  __shared__ float4 jbuf[kShortWaves][kShortBuf];
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int n_items = g.row_items * g.nc[1] * g.nc[2];
  const float a2 = g.a2, aw = g.a_win;
  const unsigned a2m1 = __float_as_uint(a2) - 1u;
  // Constants of the pair terms, copied into registers once: left to the
  // compiler they are reloaded from the descriptor inside the pair loop (a
  // global load and wait per pair).  The force polynomial's coefficients go to
  // vector registers (its first FMA would otherwise read two scalars), 1/a and
  // 1/a^2 to scalar registers.
  float dc[M + 1];
#pragma unroll
  for (int k = 0; k <= M; ++k) {
    float v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(g.dr[k]));
    dc[k] = v;
  }
  const float inv_a = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(g.inv_a)));
  const float inv_a2 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(g.inv_a2f)));
  float pk[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    float v;
    asm volatile("v_mov_b32 %0, %1" : "=v"(v) : "s"(g.pk[k]));
    pk[k] = v;
  }
  float ec[kWolfTerms];
  if (KIND == kPairWolf) {
#pragma unroll
    for (int k = 0; k < kWolfTerms; ++k)
      ec[k] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(g.ec[k])));
  }
  float4* jb = jbuf[wave];
  const int R = g.reach;
  // coincident atoms: the one- and two-kernel binnings leave them to this
  // pass, and so does every periodic plan (atoms one box edge apart coincide
  // once wrapped, which binning's comparison of the inputs does not see); the
  // other binnings compare the atoms of each cell themselves, except in cells
  // longer than kRankCap (status word 1 then set)
  const bool coin = PER || g.bin_blocks || g.bin_row_blocks || S.d.status[kStatusUnranked] != 0;
  const int centre = coin ? (R | (R << 4)) : -1;      // the row of offsets (0, 0)
  // the launch has g.short_blocks blocks; work items are strided over them
  const int item_lo = (int)((long long)n_items * lo_pm / 1000);
  const int item_hi = (int)((long long)n_items * hi_pm / 1000);
  for (int item = item_lo + blk; item < item_hi; item += g.short_blocks) {
    const int row = item / g.row_items, kk = item - row * g.row_items;
    const int cy = row % g.nc[1], cz = row / g.nc[1];
    const int rowbase = (cz * g.nc[1] + cy) * g.nc[0];
    const int rb = start[rowbase], re = start[rowbase + g.nc[0]];
    for (int ic = rb + kk * kWave; ic < re; ic += g.row_items * kWave) {
      const int ie = min(ic + kWave, re);
      const int i = ic + lane;
      const bool live = i < ie;
      const float4 pi = live ? sorted[i] : make_float4(0.f, 0.f, 0.f, 0.f);
      // ap: sum q_j g*(r) (MSM) or sum q_j e(r) (pair methods)
      float ax = 0.f, ay = 0.f, az = 0.f, ap = 0.f;
      bool coincident = false;
      for (int q = 0; q < kShortRowsPerWave; ++q) {
        const int r0 = g.short_rows[wave][q];
        if (r0 == 0xff) break;
        const int r1 = g.short_pair[wave][q];
        // a free-space row and its mirror walked together when both staged
        // unions fit the wave's buffer: [0, LA) row A, 4 far entries, [LA + 4,
        // E) row B, 4 far entries.  A lane walks its A window (its count
        // rounded up to 4: the entries past it are A atoms beyond a or far
        // entries), then its B window, then far entries (index clamped to E),
        // for the wave's longest such walk.
        if (!PER && r1 != 0xff) {
          int loA, hiA, loB, hiB;
          row_window(g, start, cy, cz, r0, R, pi, live, aw, loA, hiA);
          row_window(g, start, cy, cz, r1, R, pi, live, aw, loB, hiB);
          const int uA0 = wave_min_s(loA), uA1 = wave_max_s(hiA);
          const int uB0 = wave_min_s(loB), uB1 = wave_max_s(hiB);
          const int LA = max(uA1 - uA0, 0), LB = max(uB1 - uB0, 0);
          if (LA + LB + 8 <= kShortBuf) {
            const int E = LA + 4 + LB;
#pragma unroll
            for (int v = 0; v < (kShortBuf + kWave - 1) / kWave; ++v) {
              const int sj = v * kWave + lane;
              if (sj < E + 4) {
                float4 pj = make_float4(3e30f, 3e30f, 3e30f, 0.f);
                if (sj < LA) pj = sorted[uA0 + sj];
                else if (sj >= LA + 4 && sj < E) pj = sorted[uB0 + (sj - LA - 4)];
                jb[sj] = pj;
              }
            }
            const int nA = hiA > loA ? hiA - loA : 0, nB = hiB > loB ? hiB - loB : 0;
            const int a0A = nA > 0 ? loA - uA0 : 0;
            const int a0B = LA + 4 + (nB > 0 ? loB - uB0 : 0);
            const int c4A = (nA + 3) & ~3;
            const int T = wave_max_s(c4A + nB);
            for (int t0 = 0; t0 < T; t0 += 4) {
              const int idx = t0 < c4A ? a0A + t0 : min(a0B + (t0 - c4A), E);
              short_pairs4<M, FORCES, KIND>(jb + idx, pi, a2m1, inv_a, inv_a2, dc, pk, ec, ax, ay, az, ap);
            }
            continue;
          }
        }
        // otherwise the unit's rows one at a time, in segments of kShortSeg
        for (int h = 0; h < 2; ++h) {
        const int r = h ? r1 : r0;
        if (r == 0xff) break;
        const int oy = (r & 15) - R, oz = (r >> 4) - R;
        int jy = cy + oy, jz = cz + oz;
        // periodic plans: the row's image, its atoms shifted by (sx, sy, sz)
        double sy = 0.0, sz = 0.0;
        if (PER) {
          const int wy = ((jy % g.nc[1]) + g.nc[1]) % g.nc[1], wz = ((jz % g.nc[2]) + g.nc[2]) % g.nc[2];
          sy = (double)((jy - wy) / g.nc[1]) * g.len[1];
          sz = (double)((jz - wz) / g.nc[2]) * g.len[2];
          jy = wy;
          jz = wz;
        } else if (jy < 0 || jz < 0 || jy >= g.nc[1] || jz >= g.nc[2]) {
          continue;
        }
        // this lane's window in the row
        const float ylo = g.lo_f[1] + (float)jy * g.cs[1] + (float)sy, zlo = g.lo_f[2] + (float)jz * g.cs[2] + (float)sz;
        const float dyw = fmaxf(fmaxf(ylo - pi.y, pi.y - (ylo + g.cs[1])), 0.f);
        const float dzw = fmaxf(fmaxf(zlo - pi.z, pi.z - (zlo + g.cs[2])), 0.f);
        const float d2 = fmaf(dyw, dyw, dzw * dzw);
        const int jrow = (jz * g.nc[1] + jy) * g.nc[0];
        // x images: 0 the row itself; periodic plans also take its atoms near
        // the upper end shifted by -len (image 1) and those near the lower end
        // shifted by +len (image 2) when the lane's reach crosses a box face
        for (int img = 0; img < (PER ? 3 : 1); ++img) {
        const double sx = img == 0 ? 0.0 : (img == 1 ? -g.len[0] : g.len[0]);
        int lo = 0x7fffffff, hi = -1;
        if (live && d2 < aw * aw) {
          const float e = sqrtf(aw * aw - d2) + 1e-4f * aw;
          if (img == 0) {
            lo = start[jrow + cell_x(g, pi.x - e)];
            hi = start[jrow + cell_x(g, pi.x + e) + 1];
          } else if (img == 1 && pi.x - e < g.lo_f[0]) {
            lo = start[jrow + cell_x(g, pi.x - e + g.len_f[0])];
            hi = start[jrow + g.nc[0]];
          } else if (img == 2 && pi.x + e > g.lo_f[0] + g.len_f[0]) {
            lo = start[jrow];
            hi = start[jrow + cell_x(g, pi.x + e - g.len_f[0]) + 1];
          }
        }
        const int u0 = wave_min_s(lo), u1 = wave_max_s(hi);
        for (int s0 = u0; s0 < u1; s0 += kShortSeg) {
          // stage the union of the windows, 256 atoms at a time
#pragma unroll
          for (int v = 0; v < kShortSeg / kWave; ++v) {
            const int j = s0 + v * kWave + lane;
            float4 pj = make_float4(3e30f, 3e30f, 3e30f, 0.f);
            if (j < u1) {
              pj = sorted[j];
              if (PER) {
                pj.x = shifted(pj.x, sx);
                pj.y = shifted(pj.y, sy);
                pj.z = shifted(pj.z, sz);
              }
            }
            jb[v * kWave + lane] = pj;
          }
          if (lane < 4) jb[kShortSeg + lane] = make_float4(3e30f, 3e30f, 3e30f, 0.f);
          // this lane's part of the staged segment: [a0, a0 + n) (n = 0 keeps a0 = 0)
          const int lo_s = max(lo, s0) - s0, hi_s = min(hi, s0 + kShortSeg) - s0;
          const int n = (hi > lo && hi_s > lo_s) ? hi_s - lo_s : 0;
          const int a0 = n > 0 ? lo_s : 0;
          const int b0 = a0 + n;
          const int nmax = wave_max_s(n);
          if (r == centre && img == 0) {
            // the centre row holds the atom's own cell: any other atom at
            // distance zero is a coincident pair
            int zeros = 0;
            for (int t = 0; t < n; ++t) {
              const float4 pj = jb[a0 + t];
              zeros += (pi.x == pj.x && pi.y == pj.y && pi.z == pj.z);
            }
            coincident |= zeros > ((i >= s0 + a0 && i < s0 + b0) ? 1 : 0);
          }
          for (int t0 = 0; t0 < nmax; t0 += 4)
            short_pairs4<M, FORCES, KIND>(jb + min(a0 + t0, kShortSeg), pi, a2m1, inv_a, inv_a2, dc, pk, ec, ax, ay, az, ap);
        }
        }
        }
      }
      if (coincident) atomicOr(S.d.status, kFlagCoincident);
      // the waves' partial sums meet in the staging buffers (all waves are done with them)
      float4* red = &jbuf[0][0];                       // kShortWaves x kWave entries
      __syncthreads();
      red[wave * kWave + lane] = make_float4(ax, ay, az, ap);
      __syncthreads();
      if (wave == 0 && live) {
        float4 t = red[lane];
#pragma unroll
        for (int w = 1; w < kShortWaves; ++w) {
          const float4 v = red[w * kWave + lane];
          t.x += v.x;
          t.y += v.y;
          t.z += v.z;
          t.w += v.w;
        }
        const float qi = pi.w;
        fshort[i] = make_float4(qi * t.x, qi * t.y, qi * t.z, t.w);
      }
      __syncthreads();
    }
  }
}

// --------------------------------------------------------------------------
// Anterpolation (itemised algorithm): q^0_mu = sum_j phi^0_mu(r_j) q_j.
// An atom whose level-0 floor index is f touches the ORDER nodes f .. f +
// ORDER - 1 (level-local indices) per dimension.  Block b owns a node tile
// [n0, n0 + T) per dimension and processes exactly the atoms whose f lies in
// it, so every atom is visited once; their contributions land in a private LDS
// region of T + ORDER - 1 nodes per dimension as 2^-36 fixed-point integers
// (integer sums do not depend on the order of the atomics, so the result is
// bitwise reproducible).  The block writes its region as int64 partials and
// k_anterp_gather adds, for every node, the partials of the (at most two per
// dimension) tiles whose regions hold it, in tile order.
// --------------------------------------------------------------------------
constexpr double kFix = 68719476736.0;            // 2^36
constexpr double kInvFix = 1.0 / 68719476736.0;
constexpr int kAThreads = 256;

// round(v 2^36) as a 64-bit integer from float arithmetic: v 16 = hi + frac
// with hi = floor(v 16) and frac in [0, 1) (both exact); frac 2^32 is exact
// and rounded to the nearest integer.  frac is at most 1 - 2^-24 (the largest
// float below 1), so the rounding never reaches 2^32 and needs no carry.
// Valid for |v| < 2^27.
__device__ __forceinline__ unsigned long long fixed36(float v) {
  const float a = v * 16.f;
  const float hi = floorf(a);
  const float lo = rintf((a - hi) * 4294967296.f);
  return ((unsigned long long)(unsigned)(int)hi << 32) + (unsigned long long)(unsigned)lo;
}

// The same integer from s = v 2^36 (exact in float32) for |v| < 2^15, in three
// instructions: s + 1.5 2^52 in float64 is rounded once, to the nearest
// integer (doubles in [2^52, 2^53) are spaced 1 apart; ties to even as above),
// and since |s| < 2^51 its bit pattern is that of 1.5 2^52
// (0x4338000000000000) plus the integer.  Taking the constant's pattern off
// leaves the integer (its low word is 0, so only the high word changes).
__device__ __forceinline__ unsigned long long fixed36_scaled(float s) {
  const double t = (double)s + 6755399441055744.0;
  return (unsigned long long)__double_as_longlong(t) - 0x4338000000000000ull;
}

// Whether the tile with corner n0 (floor indices) and extent T owns the atom
// at p; f receives its tile-local floor indices.
template <int ORDER>
__device__ __forceinline__ bool owned(const Geom& g, const float4 p, const int* n0, const int* T, int* f) {
  const float pp[3] = {p.x, p.y, p.z};
  bool own = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    float r;
    grid_coord(pp[d], g.lo_f[d], g.h, g.inv_h, g.fmax[d], f[d], r);
    f[d] -= n0[d];
    own = own && f[d] >= 0 && f[d] < T[d];
  }
  return own;
}

// One owned atom's ORDER^3 contributions to the tile's region (ex x ey x ...
// nodes, x fastest) as 2^-36 fixed-point LDS atomics.
template <int ORDER>
__device__ __forceinline__ void anterp_scatter(const Geom& g, const float4 p, const int* n0, const int* T,
                                               int ex, int ey, unsigned long long* acc) {
  const float pp[3] = {p.x, p.y, p.z};
  int f[3];
  float r[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    grid_coord(pp[d], g.lo_f[d], g.h, g.inv_h, g.fmax[d], f[d], r[d]);
    f[d] -= n0[d];
  }
  float w[3][ORDER], dw[3][ORDER];
#pragma unroll
  for (int d = 0; d < 3; ++d) basis<ORDER>(r[d], w[d], dw[d]);
  // |Phi| <= 1, so every contribution of a charge below 2^15 in magnitude
  // takes the short conversion, with 2^36 folded into the charge (scaling by
  // a power of two commutes with the rounding of the products)
  if (fabsf(p.w) < 32768.f) {
    const float qs = p.w * (float)kFix;
#pragma unroll
    for (int sz = 0; sz < ORDER; ++sz) {
      const float qz = qs * w[2][sz];
#pragma unroll
      for (int sy = 0; sy < ORDER; ++sy) {
        const float qyz = qz * w[1][sy];
        unsigned long long* rowp = acc + ((f[2] + sz) * ey + (f[1] + sy)) * ex + f[0];
#pragma unroll
        for (int sx = 0; sx < ORDER; ++sx) atomicAdd(rowp + sx, fixed36_scaled(qyz * w[0][sx]));
      }
    }
  } else {
#pragma unroll
    for (int sz = 0; sz < ORDER; ++sz) {
      const float qz = p.w * w[2][sz];
#pragma unroll
      for (int sy = 0; sy < ORDER; ++sy) {
        const float qyz = qz * w[1][sy];
        unsigned long long* rowp = acc + ((f[2] + sz) * ey + (f[1] + sy)) * ex + f[0];
#pragma unroll
        for (int sx = 0; sx < ORDER; ++sx) atomicAdd(rowp + sx, fixed36(qyz * w[0][sx]));
      }
    }
  }
}

static_assert(kAThreads == 256, "bank_order() deals 256 entries to 8 half-waves");

// The queue entry thread t takes in a scatter round of `count` entries (-1:
// none).  The entries are sorted by the LDS bank pair of their region corner
// (corner node mod 32: a 64-bit accumulator spans two of the 64 banks) and
// dealt so that the 32 lanes of a half-wave take entries about count/32
// apart in that order, mostly one per bank pair: every atomic of the
// half-wave then hits distinct banks, and atoms with the same corner (same
// addresses) fall in different instructions.  Any order gives the same
// integer sums.
template <int ORDER>
__device__ __forceinline__ int bank_order(const Geom& g, const float4* queue, int count, const int* n0, int ex,
                                          int ey, int* bcount, unsigned short* border) {
  const int t = threadIdx.x;
  if (t < 32) bcount[t] = 0;
  __syncthreads();
  int bucket = -1, pos = 0;
  if (t < count) {
    const float4 p = queue[t];
    const float pp[3] = {p.x, p.y, p.z};
    int f[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      float r;
      grid_coord(pp[d], g.lo_f[d], g.h, g.inv_h, g.fmax[d], f[d], r);
      f[d] -= n0[d];
    }
    bucket = ((f[2] * ey + f[1]) * ex + f[0]) & 31;
    pos = atomicAdd(&bcount[bucket], 1);
  }
  __syncthreads();
  if (t < kWave) {                                      // exclusive scan of the 32 bucket sizes
    const int v = t < 32 ? bcount[t] : 0;
    int inc = v;
#pragma unroll
    for (int off = 1; off < 32; off <<= 1) {
      const int u = __shfl_up(inc, off);
      if (t >= off) inc += u;
    }
    if (t < 32) bcount[t] = inc - v;
  }
  __syncthreads();
  if (bucket >= 0) border[bcount[bucket] + pos] = (unsigned short)t;
  __syncthreads();
  const int j = (t & 31) * (kAThreads / 32) + (t >> 5);
  return j < count ? (int)border[j] : -1;
}

template <int ORDER>
__global__ void __launch_bounds__(kAThreads) k_anterp(KArgs A) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  const Geom& g = S.g;
  const float4* __restrict__ sorted = S.d.sorted;
  const int* __restrict__ start = S.d.cell_start;
  extern __shared__ unsigned long long acc[];
  __shared__ int row_beg[64], row_pre[65];
  // owned atoms wait here until a whole round of them (one per thread) is
  // there, so the scatter runs with every lane busy (about a third of the
  // candidates lie in the margin cells and belong to other tiles)
  __shared__ float4 queue[2 * kAThreads];
  __shared__ int bcount[32];
  __shared__ unsigned short border[kAThreads];
  __shared__ int wcount[kAThreads / kWave];
  __shared__ int qlen;
  if (threadIdx.x == 0) qlen = 0;
  const int T[3] = {g.at[0], g.at[1], g.at[2]};
  const int ex = T[0] + ORDER - 1, ey = T[1] + ORDER - 1;
  const int ext = g.at_ext;
  const int bx = blk % g.atn[0], by = (blk / g.atn[0]) % g.atn[1], bz = blk / (g.atn[0] * g.atn[1]);
  const int n0[3] = {bx * T[0], by * T[1], bz * T[2]};
  for (int i = threadIdx.x; i < ext; i += kAThreads) acc[i] = 0ull;
  // the tile's atoms lie at box-relative positions [n0 h, (n0 + T) h) (the
  // last tile also takes atoms on the upper box face); candidate cells cover
  // that range with a margin for the rounding of cell and floor indices
  int c0[3], c1[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const float xl = ((float)n0[d] - 0.01f) * g.h, xh = ((float)(n0[d] + T[d]) + 0.01f) * g.h;
    c0[d] = min(g.nc[d] - 1, max(0, (int)floorf(fmaxf(xl, 0.f) * g.inv_cs[d])));
    c1[d] = max(c0[d], min(g.nc[d] - 1, (int)floorf(fmaxf(xh, 0.f) * g.inv_cs[d])));
    if (n0[d] + T[d] > g.fmax[d]) c1[d] = g.nc[d] - 1;
  }
  // candidate atoms: the contiguous sorted ranges of the cell rows in
  // [c0, c1], taken 64 rows at a time; prefix sums over a chunk's rows let
  // every thread walk one flat index space
  const int nry = c1[1] - c0[1] + 1, nrows = nry * (c1[2] - c0[2] + 1);
  for (int rc0 = 0; rc0 < nrows; rc0 += 64) {
    const int nr = min(64, nrows - rc0);
    __syncthreads();                                   // previous chunk is done with the table
    if (threadIdx.x < nr) {
      const int rr = rc0 + threadIdx.x;
      const int cy = c0[1] + rr % nry, cz = c0[2] + rr / nry;
      const int rb = (cz * g.nc[1] + cy) * g.nc[0];
      row_beg[threadIdx.x] = start[rb + c0[0]];
      row_pre[threadIdx.x + 1] = start[rb + c1[0] + 1] - start[rb + c0[0]];
    }
    if (threadIdx.x == 0) row_pre[0] = 0;
    __syncthreads();
    if (threadIdx.x < kWave) {                         // inclusive scan of the row lengths by wave 0
      int v = (int)threadIdx.x < nr ? row_pre[threadIdx.x + 1] : 0;
#pragma unroll
      for (int off = 1; off < kWave; off <<= 1) {
        const int u = __shfl_up(v, off);
        if ((int)threadIdx.x >= off) v += u;
      }
      if ((int)threadIdx.x < nr) row_pre[threadIdx.x + 1] = v;
    }
    __syncthreads();
    const int ncand = row_pre[nr];
    int row = 0;
    for (int t0 = 0; t0 < ncand; t0 += kAThreads) {
      // candidates of this round: the owned ones join the queue
      const int t = t0 + (int)threadIdx.x;
      float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
      bool own = false;
      if (t < ncand) {
        while (row_pre[row + 1] <= t) ++row;
        p = sorted[row_beg[row] + (t - row_pre[row])];
        int f[3];
        own = owned<ORDER>(g, p, n0, T, f);
      }
      const unsigned long long m = __ballot(own);
      const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
      if (lane == 0) wcount[wave] = __popcll(m);
      __syncthreads();
      int total = qlen, base = qlen;
#pragma unroll
      for (int w = 0; w < kAThreads / kWave; ++w) {
        base += w < wave ? wcount[w] : 0;
        total += wcount[w];
      }
      if (own) queue[base + __popcll(m & ((1ull << lane) - 1))] = p;
      __syncthreads();
      if (total >= kAThreads) {
        // a full round: one queued atom per thread (in bank order), then the
        // rest to the front
        const int e = bank_order<ORDER>(g, queue, kAThreads, n0, ex, ey, bcount, border);
        anterp_scatter<ORDER>(g, queue[e], n0, T, ex, ey, acc);
        const int rest = total - kAThreads;
        const float4 v = (int)threadIdx.x < rest ? queue[kAThreads + threadIdx.x] : make_float4(0.f, 0.f, 0.f, 0.f);
        __syncthreads();
        if ((int)threadIdx.x < rest) queue[threadIdx.x] = v;
        total = rest;
      }
      if (threadIdx.x == 0) qlen = total;
      __syncthreads();
    }
  }
  {
    const int e = bank_order<ORDER>(g, queue, qlen, n0, ex, ey, bcount, border);
    if (e >= 0) anterp_scatter<ORDER>(g, queue[e], n0, T, ex, ey, acc);
  }
  __syncthreads();
  long long* __restrict__ out = S.d.ant_part + (size_t)blk * ext;
  for (int i = threadIdx.x; i < ext; i += kAThreads) out[i] = (long long)acc[i];
}

// q^0 of every level-0 node: the sum, in tile order, of the partials of the
// tiles whose private regions hold the node.
template <int ORDER>
__global__ void __launch_bounds__(kBlock) k_anterp_gather(KArgs A) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  const Geom& g = S.g;
  const Level L = g.lv[0];
  const int node = blk * kBlock + threadIdx.x;
  if (node >= L.count) return;
  const float inv_n0 = 1.f / (float)L.n[0], inv_n1 = 1.f / (float)L.n[1];
  int m[3];
  m[2] = fdiv(fdiv(node, L.n[0], inv_n0, m[0]), L.n[1], inv_n1, m[1]);
  int t0[3], t1[3];
  bool any = true;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    // position from the first node of tile 0's region (node -(ORDER/2 - 1);
    // a periodic level also has ghost nodes below it, which no region holds)
    m[d] += L.lo[d] + ORDER / 2 - 1;
    any = any && m[d] >= 0;
    // tiles t with t T <= m < (t + 1) T + ORDER - 1, clipped to the tiles that exist
    t1[d] = min(m[d] / g.at[d], g.atn[d] - 1);
    t0[d] = max(0, (m[d] - (ORDER - 1)) / g.at[d]);
    if (m[d] < ORDER - 1) t0[d] = 0;
  }
  if (!any) {
    S.d.qgrid[L.off + node] = 0.f;
    return;
  }
  const int ex = g.at[0] + ORDER - 1, ey = g.at[1] + ORDER - 1;
  const long long* __restrict__ part = S.d.ant_part;
  long long sum = 0;
  for (int tz = t0[2]; tz <= t1[2]; ++tz)
    for (int ty = t0[1]; ty <= t1[1]; ++ty)
      for (int tx = t0[0]; tx <= t1[0]; ++tx) {
        const int tile = (tz * g.atn[1] + ty) * g.atn[0] + tx;
        const int lx = m[0] - tx * g.at[0], ly = m[1] - ty * g.at[1], lz = m[2] - tz * g.at[2];
        sum += part[(size_t)tile * g.at_ext + (lz * ey + ly) * ex + lx];
      }
  S.d.qgrid[L.off + node] = (float)((double)sum * kInvFix);
}

// --------------------------------------------------------------------------
// Restriction (itemised algorithm): q^{k+1}_mu = sum_nu Phi(nu/2 - mu)^3 q^k_nu.
// Only offsets j = nu - 2 mu with Phi(j/2) != 0 are visited (given as lists).
// --------------------------------------------------------------------------
// Phi at half-integers, evaluated at compile time from the piecewise forms
// above: the weights of restriction (nu = 2 mu + j) and prolongation.  Phi
// vanishes at non-zero integers, so only j = 0 and odd j contribute.
constexpr double phi_half(int order, int j) {
  const double t = (j < 0 ? -j : j) * 0.5;
  if (order == 4) {
    if (t <= 1.0) return (1.0 - t) * (1.0 + t - 1.5 * t * t);
    if (t <= 2.0) return -0.5 * (t - 1.0) * (2.0 - t) * (2.0 - t);
    return 0.0;
  }
  if (t <= 1.0) return (1.0 - t * t) * (2.0 - t) * (6.0 + 3.0 * t - 5.0 * t * t) / 12.0;
  if (t <= 2.0) return (1.0 - t) * (2.0 - t) * (3.0 - t) * (4.0 + 9.0 * t - 5.0 * t * t) / 24.0;
  if (t <= 3.0) return (t - 1.0) * (t - 2.0) * (t - 3.0) * (t - 3.0) * (4.0 - t) / 24.0;
  return 0.0;
}

template <int ORDER>
struct Dyadic {
  static constexpr int R = ORDER - 1;          // largest |j| with a non-zero weight
  static constexpr int NT = ORDER + 1;         // taps: 0 and the ORDER odd j in [-R, R]
  // tap offsets and weights, ascending j
  static constexpr int j(int t) { return t < ORDER / 2 ? 2 * t - R : (t == ORDER / 2 ? 0 : 2 * (t - ORDER / 2) - 1); }
  static constexpr float w(int t) { return (float)phi_half(ORDER, j(t)); }
  // odd fine index m: coarse nu = (m - R)/2 + i, i < ORDER, weight Phi((R - 2i)/2)
  static_assert(j(0) == -R && j(ORDER / 2) == 0 && j(ORDER) == R, "tap offsets");
  static constexpr float wodd(int i) { return (float)phi_half(ORDER, R - 2 * i); }
};

// One block = 4 x 4 x 4 coarse nodes (small tiles: more blocks, each a short
// round of loads; 8 x 8 x 4 took 16.4 us for the three launches on water24k
// against 13.6 us); the fine nodes they read are staged in
// LDS by all kRThreads threads (one round of loads), all threads form the
// x-direction row sums, then one thread per coarse node combines its rows.
constexpr int kRX = 4, kRY = 4, kRZ = 4;
constexpr int kRThreads = 1024;

template <int ORDER>
__global__ void __launch_bounds__(kRThreads) k_restrict(KArgs A, int k) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  const Geom& g = S.g;
  float* __restrict__ grid = S.d.qgrid;
  using D = Dyadic<ORDER>;
  constexpr int R = D::R;
  constexpr int FX = 2 * kRX - 1 + 2 * R, FY = 2 * kRY - 1 + 2 * R, FZ = 2 * kRZ - 1 + 2 * R;
  __shared__ float fine[FX * FY * FZ];
  __shared__ float xs[FZ * FY * kRX];                  // x-pass row sums
  const Level F = g.lv[k], C = g.lv[k + 1];
  const int ntx = (C.n[0] + kRX - 1) / kRX, nty = (C.n[1] + kRY - 1) / kRY;
  const int bx = blk % ntx, by = (blk / ntx) % nty, bz = blk / (ntx * nty);
  const int c0x = bx * kRX, c0y = by * kRY, c0z = bz * kRZ;          // level-local coarse origin
  // absolute fine index of local fine (0,0,0): 2 (C.lo + c0) - R
  const int f0x = 2 * (C.lo[0] + c0x) - R, f0y = 2 * (C.lo[1] + c0y) - R, f0z = 2 * (C.lo[2] + c0z) - R;
  const float* fin = grid + F.off;
  constexpr int nfine = FX * FY * FZ;
  for (int i0 = 0; i0 < nfine; i0 += 8 * kRThreads) {    // 8 loads in flight per thread
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * kRThreads + threadIdx.x;
      v[u] = 0.f;
      if (i < nfine) {
        const int lx = i % FX, ly = (i / FX) % FY, lz = i / (FX * FY);
        const int vx = f0x + lx - F.lo[0], vy = f0y + ly - F.lo[1], vz = f0z + lz - F.lo[2];
        if (vx >= 0 && vx < F.n[0] && vy >= 0 && vy < F.n[1] && vz >= 0 && vz < F.n[2])
          v[u] = fin[((size_t)vz * F.n[1] + vy) * F.n[0] + vx];
      }
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * kRThreads + threadIdx.x;
      if (i < nfine) fine[i] = v[u];
    }
  }
  __syncthreads();
  // x pass over every staged (z, y) fine row, by all threads:
  //   xs[lz][ly][tx] = sum_c w_c fine[lz][ly][2 tx + R + j_c]      (c ascending)
  constexpr int nxs = FZ * FY * kRX;
  for (int i = threadIdx.x; i < nxs; i += kRThreads) {
    const int tx = i % kRX, row = i / kRX;             // row = lz * FY + ly
    const float* rowp = fine + row * FX + 2 * tx + R;
    float r[D::NT];
#pragma unroll
    for (int c = 0; c < D::NT; ++c) r[c] = rowp[D::j(c)];
    float racc = 0.f;
#pragma unroll
    for (int c = 0; c < D::NT; ++c) racc = fmaf(D::w(c), r[c], racc);
    xs[i] = racc;
  }
  __syncthreads();
  if (threadIdx.x >= kRX * kRY * kRZ) return;
  const int tx = threadIdx.x % kRX, ty = (threadIdx.x / kRX) % kRY, tz = threadIdx.x / (kRX * kRY);
  const int mx = c0x + tx, my = c0y + ty, mz = c0z + tz;
  if (tz >= kRZ || mx >= C.n[0] || my >= C.n[1] || mz >= C.n[2]) return;
  // then sum_{a, b} (w_b w_a) xs[2 tz + R + j_a][2 ty + R + j_b][tx] (a, then b
  // ascending): the operations of the direct triple sum, in its order
  float r[D::NT][D::NT];
#pragma unroll
  for (int a = 0; a < D::NT; ++a)
#pragma unroll
    for (int b = 0; b < D::NT; ++b)
      r[a][b] = xs[((2 * tz + D::j(a) + R) * FY + (2 * ty + D::j(b) + R)) * kRX + tx];
  float acc = 0.f;
#pragma unroll
  for (int a = 0; a < D::NT; ++a)
#pragma unroll
    for (int b = 0; b < D::NT; ++b) acc = fmaf(D::w(b) * D::w(a), r[a][b], acc);
  grid[C.off + ((size_t)mz * C.n[1] + my) * C.n[0] + mx] = acc;
}

// --------------------------------------------------------------------------
// Top level (itemised algorithm), float64: u^{l-1}_mu = sum over every node nu
// of g^{l-1}(2^{l-1} h |mu - nu|) q^{l-1}_nu, from a table T[|dx|][|dy|][|dz|].
// One wave per output node: lanes stride over the input nodes, then a fixed
// butterfly sums the 64 lane partials.  Runs as extra blocks of the coarse
// lattice-cutoff launch (same inputs ready) or, with the untiled lattice
// kernel, as its own launch.
// --------------------------------------------------------------------------
// Periodic plans: the outputs and inputs are the nodes of one period (the
// ghost copies are filled afterwards) and T holds the image sum K at the node
// offsets (mu - nu) modulo the period.
__device__ __forceinline__ void top_node_periodic(const SysDesc& S, const Level& L, int mx, int my, int mz,
                                                  int lane) {
  const double* __restrict__ T = S.d.top;
  const int G = S.g.ghost;
  const int p0 = L.per[0], p1 = L.per[1], p2 = L.per[2];
  mx -= G;
  my -= G;
  mz -= G;
  if (mx < 0 || my < 0 || mz < 0 || mx >= p0 || my >= p1 || mz >= p2) return;
  const float* qt = S.d.qgrid + L.off;
  const int count = p0 * p1 * p2;
  const float inv_p0 = 1.f / (float)p0, inv_p1 = 1.f / (float)p1;
  double acc = 0.0;
  for (int v0 = lane; v0 < count; v0 += 4 * kWave) {
    double t[4];
    float qv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int v = v0 + u * kWave;
      t[u] = 0.0;
      qv[u] = 0.f;
      if (v < count) {
        int vx, vy;
        const int vz = fdiv(fdiv(v, p0, inv_p0, vx), p1, inv_p1, vy);
        const int dx = mx - vx + (mx < vx ? p0 : 0), dy = my - vy + (my < vy ? p1 : 0);
        const int dz = mz - vz + (mz < vz ? p2 : 0);
        t[u] = T[((size_t)dz * p1 + dy) * p0 + dx];
        qv[u] = qt[((size_t)(vz + G) * L.n[1] + (vy + G)) * L.n[0] + (vx + G)];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = fma(t[u], (double)qv[u], acc);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) {
    const size_t node = ((size_t)(mz + G) * L.n[1] + (my + G)) * L.n[0] + (mx + G);
    S.d.ucut[L.off + node] = (float)acc;
    S.d.u[L.off + node] = (float)acc;
  }
}

__device__ __forceinline__ void top_node(const SysDesc& S, int node, int lane) {
  const Geom& g = S.g;
  const double* __restrict__ T = S.d.top;
  const Level L = g.lv[g.levels - 1];
  if (node >= L.count) return;
  const float inv_n0 = 1.f / (float)L.n[0], inv_n1 = 1.f / (float)L.n[1];
  int mx, my;
  const int mz = fdiv(fdiv(node, L.n[0], inv_n0, mx), L.n[1], inv_n1, my);
  if (g.periodic) {
    top_node_periodic(S, L, mx, my, mz, lane);
    return;
  }
  const float* qt = S.d.qgrid + L.off;
  double acc = 0.0;
  for (int v0 = lane; v0 < L.count; v0 += 4 * kWave) {     // 4 table and charge loads in flight
    double t[4];
    float qv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int v = v0 + u * kWave;
      t[u] = 0.0;
      qv[u] = 0.f;
      if (v < L.count) {
        int vx, vy;
        const int vz = fdiv(fdiv(v, L.n[0], inv_n0, vx), L.n[1], inv_n1, vy);
        t[u] = T[((size_t)abs(mz - vz) * L.n[1] + abs(my - vy)) * L.n[0] + abs(mx - vx)];
        qv[u] = qt[v];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) acc = fma(t[u], (double)qv[u], acc);
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) {
    S.d.ucut[L.off + node] = (float)acc;
    S.d.u[L.off + node] = (float)acc;
  }
}

// --------------------------------------------------------------------------
// Ghost nodes of a periodic level: the nodes outside one period (indices from
// -ghost up) stand for nodes of the period.  fold: every node of the period
// adds what its ghost images received (anterpolation spreads the atoms near a
// face onto them), images in a fixed order; fill: every ghost node takes the
// value of its node in the period.  One thread per node of the level (one
// system: periodic plans are not batched).
// --------------------------------------------------------------------------
enum GhostGrid : int { kGhostQ = 0, kGhostU = 1 };

__global__ void __launch_bounds__(kBlock) k_ghost(KArgs A, int level, int which, int fold) {
  const SysDesc& S = A.sys[0];
  const Geom& g = S.g;
  const Level L = g.lv[level];
  const int node = (int)blockIdx.x * kBlock + (int)threadIdx.x;
  if (node >= L.count) return;
  float* grid = (which == kGhostQ ? S.d.qgrid : S.d.u) + L.off;
  const int G = g.ghost;
  const int mx = node % L.n[0], my = (node / L.n[0]) % L.n[1], mz = node / (L.n[0] * L.n[1]);
  const int ix = mx - G, iy = my - G, iz = mz - G;
  const int p0 = L.per[0], p1 = L.per[1], p2 = L.per[2];
  const bool inside = ix >= 0 && iy >= 0 && iz >= 0 && ix < p0 && iy < p1 && iz < p2;
  auto at = [&](int x, int y, int z) { return ((size_t)(z + G) * L.n[1] + (y + G)) * L.n[0] + (x + G); };
  if (fold) {
    if (!inside) return;
    // images x + j p of this node inside the level's nodes [-G, p + G)
    auto jlo = [G](int x, int p) { return -((x + G) / p); };
    auto jhi = [G](int x, int p) { return (p + G - 1 - x) / p; };
    float v = grid[node];
    for (int jz = jlo(iz, p2); jz <= jhi(iz, p2); ++jz)
      for (int jy = jlo(iy, p1); jy <= jhi(iy, p1); ++jy)
        for (int jx = jlo(ix, p0); jx <= jhi(ix, p0); ++jx)
          if (jx || jy || jz) v += grid[at(ix + jx * p0, iy + jy * p1, iz + jz * p2)];
    grid[node] = v;
  } else if (!inside) {
    const int wx = ((ix % p0) + p0) % p0, wy = ((iy % p1) + p1) % p1, wz = ((iz % p2) + p2) % p2;
    grid[node] = grid[at(wx, wy, wz)];
  }
}

__global__ void __launch_bounds__(kBlock) k_top(KArgs A) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  const int node = __builtin_amdgcn_readfirstlane((blk * (int)blockDim.x + (int)threadIdx.x) / kWave);
  top_node(S, node, threadIdx.x & (kWave - 1));
}

// Blocks of a lattice-cutoff launch of a system.  part 0: the level-0 tiles;
// part 1: the coarse tiles (levels 1 .. l-2) then kLatWaves top-level nodes
// per block; part 2: every tile then the top level (one launch when level 0
// has no stream of its own).  first = first tile block of the part.
__device__ __forceinline__ int lattice_tile_blocks(const LatLaunch& P, int part, int& first) {
  const LatTile& t = P.t[P.n - 1];
  const int total = t.block0 + t.ntx * t.nty * t.ntz * t.groups;
  const int b1 = P.n > 1 ? P.t[1].block0 : total;
  first = (part == 1) ? b1 : 0;
  return (part == 0) ? b1 : (part == 1 ? total - b1 : total);
}

// --------------------------------------------------------------------------
// Lattice cutoff (itemised algorithm) for every level k <= l-2 in one launch:
//   u^{k,cut}_mu = sum_{|n| < 2a/h} g^k(2^k h |n|) q^k_{mu+n} = 2^-k sum W(n) q^k_{mu+n}
// with W(n) = g^0(h|n|) from the stencil table (rows of taps along z).
// --------------------------------------------------------------------------
// part 0: the nodes of level 0; part 1: the nodes of levels 1 .. l-2;
// part 2: both.
__global__ void __launch_bounds__(kBlock) k_lattice(KArgs A, int part) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  const Geom& g = S.g;
  const StencilRow* __restrict__ rows = S.d.rows;
  const int n_rows = S.n_rows;
  const float* __restrict__ wts = S.d.weights;
  const float* __restrict__ qgrid = S.d.qgrid;
  float* __restrict__ ucut = S.d.ucut;
  const int first = (part == 1) ? g.lv[1].off : 0;
  const int end = (part == 0) ? g.lv[1].off : g.lv[g.levels - 1].off;   // the top level is not included
  int gid = first + blk * blockDim.x + threadIdx.x;
  if (gid >= end) return;
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
// Lattice cutoff, windowed (same sum as k_lattice).  One block = one output
// tile of one level: xl lanes along x (B consecutive outputs each, kept in
// registers), ty along y, tz along z.  The block stages its whole input
// window ((tz + 2H) x (ty + 2H) x (xl B + 2H), zero outside the grid) in LDS
// once, together with the stencil in compact form, then its 8 waves split a
// flat list of stencil rows with no further barriers.
//
// Compact stencil: W depends on |n| only, so a row (nz, ny) with taps
// nx in [-xr, xr] stores W for nx = 0..xr, shared by nz and -nz; and rows
// (nz, +ny), (nz, -ny) are processed together by adding their inputs first
// (one FMA chain for both).
// --------------------------------------------------------------------------

template <int B, int XR, bool PAIR>
__device__ __forceinline__ void row_win(float* acc, const float* a, const float* b,
                                        const float* wrow) {
  // taps in groups of 4: each group reads the 4 window values (and weights) it
  // adds to the window, and the scheduler keeps the groups apart, so a lane
  // holds about B + 8 values instead of the whole row (8 waves per SIMD fit)
  constexpr int NT = 2 * XR + 1;
  float v[B + 2 * XR];
#pragma unroll
  for (int j = 0; j < B - 1; ++j) v[j] = PAIR ? a[j] + b[j] : a[j];
#pragma unroll
  for (int t0 = 0; t0 < NT; t0 += 4) {
    float w[4];
#pragma unroll
    for (int t = t0; t < t0 + 4 && t < NT; ++t) {
      v[t + B - 1] = PAIR ? a[t + B - 1] + b[t + B - 1] : a[t + B - 1];
      w[t - t0] = wrow[t < XR ? XR - t : t - XR];
    }
#pragma unroll
    for (int t = t0; t < t0 + 4 && t < NT; ++t)
#pragma unroll
      for (int bb = 0; bb < B; ++bb) acc[bb] = fmaf(w[t - t0], v[bb + t], acc[bb]);
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <int B, bool PAIR>
__device__ __forceinline__ void row_win_dispatch(int xr, float* acc, const float* a, const float* b,
                                                 const float* w) {
  switch (xr) {
    case 0: row_win<B, 0, PAIR>(acc, a, b, w); break;
    case 1: row_win<B, 1, PAIR>(acc, a, b, w); break;
    case 2: row_win<B, 2, PAIR>(acc, a, b, w); break;
    case 3: row_win<B, 3, PAIR>(acc, a, b, w); break;
    case 4: row_win<B, 4, PAIR>(acc, a, b, w); break;
    case 5: row_win<B, 5, PAIR>(acc, a, b, w); break;
    case 6: row_win<B, 6, PAIR>(acc, a, b, w); break;
    case 7: row_win<B, 7, PAIR>(acc, a, b, w); break;
    case 8: row_win<B, 8, PAIR>(acc, a, b, w); break;
    case 9: row_win<B, 9, PAIR>(acc, a, b, w); break;
    case 10: row_win<B, 10, PAIR>(acc, a, b, w); break;
    case 11: row_win<B, 11, PAIR>(acc, a, b, w); break;
    case 12: row_win<B, 12, PAIR>(acc, a, b, w); break;
    case 13: row_win<B, 13, PAIR>(acc, a, b, w); break;
    case 14: row_win<B, 14, PAIR>(acc, a, b, w); break;
    case 15: row_win<B, 15, PAIR>(acc, a, b, w); break;
    default: row_win<B, 16, PAIR>(acc, a, b, w); break;
  }
}

// part 0: the tiles of level 0; part 1: the tiles of levels 1 .. l-2 and the
// top level; part 2: every tile and the top level.
template <int B, int W>
__global__ void __launch_bounds__(W * kWave, B <= 6 ? 8 : 4) k_lattice_win(KArgs A, int part) {
  constexpr int kLatWaves = W, kLatThreads = W * kWave;
  int blk;
  const SysDesc& S = sys_of(A, blk, false);
  const Geom& g = S.g;
  const LatLaunch& P = S.lat;
  {
    int first;
    const int nl = lattice_tile_blocks(P, part, first);
    if (blk >= nl) {                                    // a top-level block (no barriers)
      top_node(S, (blk - nl) * kLatWaves + (int)(threadIdx.x / kWave), threadIdx.x & (kWave - 1));
      return;
    }
    blk += first;
  }
  const int4* __restrict__ rows_g = S.d.rows_c;
  const float* __restrict__ wc_g = S.d.weights_c;
  const float* __restrict__ qgrid = S.d.qgrid;
  float* __restrict__ ucut = S.d.ucut;
  extern __shared__ float4 lds4[];
  int4* rows = reinterpret_cast<int4*>(lds4);
  float* wc = reinterpret_cast<float*>(lds4 + P.n_rows);
  float* win = wc + P.n_wc;
  int bid = blk, li = 0;
  while (li + 1 < P.n && bid >= P.t[li + 1].block0) ++li;
  const LatTile T = P.t[li];
  const Level Lv = g.lv[T.level];
  bid -= T.block0;
  // block = (tile, row group); the group's rows have nz in [nz_lo, nz_hi]
  const int G = T.groups;
  const int grp = bid % G;
  const int tile = bid / G;
  const int r_lo = P.grp[G][grp], r_hi = P.grp[G][grp + 1];
  const int nz_lo = r_lo < r_hi ? rows_g[r_lo].x : 0, nz_hi = r_lo < r_hi ? rows_g[r_hi - 1].x : 0;
  const int bx = tile % T.ntx, by = (tile / T.ntx) % T.nty, bz = tile / (T.ntx * T.nty);
  const int H = P.H;
  const int x0 = bx * T.xl * B, y0 = by * T.ty, z0 = bz * T.tz;
  // window: planes z0 + nz_lo .. z0 + tz - 1 + nz_hi, rows y0 - H .., columns x0 - H ..
  const int WX = T.xl * B + 2 * H, PY = T.ty + 2 * H, WZ = T.tz + nz_hi - nz_lo, PX = T.px, PP = T.pp;
  const float* qk = qgrid + Lv.off;
  const int NX = Lv.n[0], NY = Lv.n[1], NZ = Lv.n[2];

  for (int i = threadIdx.x; i < P.n_rows; i += kLatThreads) rows[i] = rows_g[i];
  for (int i = threadIdx.x; i < P.n_wc; i += kLatThreads) wc[i] = wc_g[i];
  // the window in runs of 4 consecutive x (index arithmetic and the y, z
  // bounds once per run), 2 runs per thread at a time: 8 loads in flight
  const int WXq = (WX + 3) >> 2;
  const int nq = WZ * PY * WXq;                        // < 2^16 (bounded by the LDS budget)
  const float inv_wq = 1.f / (float)WXq, inv_py = 1.f / (float)PY;
  for (int i0 = 0; i0 < nq; i0 += 2 * kLatThreads) {
    float v[2][4];
    int dst[2], nx4[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int i = i0 + u * kLatThreads + threadIdx.x;
      dst[u] = -1;
      nx4[u] = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e) v[u][e] = 0.f;
      if (i < nq) {
        int xq, yy;
        const int zz = fdiv(fdiv(i, WXq, inv_wq, xq), PY, inv_py, yy);
        const int xx = 4 * xq;
        dst[u] = zz * PP + yy * PX + xx;
        nx4[u] = min(4, WX - xx);
        const int gx = x0 - H + xx, gy = y0 - H + yy, gz = z0 + nz_lo + zz;
        if (gy >= 0 && gy < NY && gz >= 0 && gz < NZ) {
          const float* src = qk + ((size_t)gz * NY + gy) * NX;
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (e < nx4[u] && gx + e >= 0 && gx + e < NX) v[u][e] = src[gx + e];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (dst[u] >= 0 && e < nx4[u]) win[dst[u] + e] = v[u][e];
  }
  __syncthreads();

  const int lane = threadIdx.x & (kWave - 1);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int xi = lane % T.xl, yi = (lane / T.xl) % T.ty, zi = lane / (T.xl * T.ty);
  const bool active = zi < T.tz;
  const float* base = win + (zi - nz_lo) * PP + (yi + H) * PX + xi * B + H;
  double tot[B];
  float acc[B];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    tot[b] = 0.0;
    acc[b] = 0.f;
  }
  int cnt = 0;
  int4 row = (r_lo + wave < r_hi) ? rows[r_lo + wave] : make_int4(0, 0, 0, 0);
  for (int r = r_lo + wave; r < r_hi; r += kLatWaves) {
    const int4 cur = row;
    if (r + kLatWaves < r_hi) row = rows[r + kLatWaves];           // next descriptor in flight
    const int nz = __builtin_amdgcn_readfirstlane(cur.x);
    const int ny = __builtin_amdgcn_readfirstlane(cur.y);
    const int xr = __builtin_amdgcn_readfirstlane(cur.z);
    const int wo = __builtin_amdgcn_readfirstlane(cur.w);
    if (active) {
      const float* a = base + nz * PP + ny * PX - xr;
      if (ny == 0) {
        row_win_dispatch<B, false>(xr, acc, a, a, wc + wo);
      } else {
        const float* b = base + nz * PP - ny * PX - xr;
        row_win_dispatch<B, true>(xr, acc, a, b, wc + wo);
      }
    }
    if (++cnt == 4) {                                  // float32 groups of 4 rows, float64 total
#pragma unroll
      for (int b = 0; b < B; ++b) {
        tot[b] += (double)acc[b];
        acc[b] = 0.f;
      }
      cnt = 0;
    }
  }
#pragma unroll
  for (int b = 0; b < B; ++b) tot[b] += (double)acc[b];
  __syncthreads();                                     // window no longer needed
  double* red = reinterpret_cast<double*>(lds4);
#pragma unroll
  for (int b = 0; b < B; ++b) red[((size_t)wave * kWave + lane) * B + b] = tot[b];
  __syncthreads();
  // every thread sums one output over the waves (in wave order)
  for (int o = threadIdx.x; o < kWave * B; o += kLatThreads) {
    const int l = o / B, b = o - l * B;
    const int lxi = l % T.xl, lyi = (l / T.xl) % T.ty, lzi = l / (T.xl * T.ty);
    const int x = x0 + lxi * B + b, y = y0 + lyi, z = z0 + lzi;
    if (lzi >= T.tz || x >= NX || y >= NY || z >= NZ) continue;
    double r[kLatWaves];
#pragma unroll
    for (int w = 0; w < kLatWaves; ++w) r[w] = red[((size_t)w * kWave + l) * B + b];
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kLatWaves; ++w) v += r[w];
    const size_t node = ((size_t)z * NY + y) * NX + x;
    if (G == 1)
      ucut[Lv.off + node] = (float)ldexp(v, -T.level);
    else
      S.d.lat_part[T.part0 + (size_t)grp * Lv.count + node] = v;
  }
}

// u^{k,cut} at node `node` of level k (level-local index): the stored value,
// or, where the level's lattice tiles were split into row groups, the sum of
// the groups' float64 partials in group order (with `store`, written back into
// u^{k,cut} so the grid is complete after the prolongation).  The partials are
// loaded together.
__device__ __forceinline__ float ucut_value(const SysDesc& S, int k, int node, bool store) {
  const Level& L = S.g.lv[k];
  const int off = L.off;
  float* __restrict__ ucut = S.d.ucut;
  const int groups = (S.lat.b == 0 || k >= S.lat.n) ? 1 : S.lat.t[k].groups;
  if (groups == 1) return ucut[off + node];
  const size_t cnt = (size_t)L.count;
  const double* __restrict__ part = S.d.lat_part + S.lat.t[k].part0 + node;
  double pv[kLatMaxGroups];
#pragma unroll
  for (int gi = 0; gi < kLatMaxGroups; ++gi) pv[gi] = (gi < groups) ? part[(size_t)gi * cnt] : 0.0;
  double v = 0.0;
#pragma unroll
  for (int gi = 0; gi < kLatMaxGroups; ++gi)
    if (gi < groups) v += pv[gi];
  const float u = (float)ldexp(v, -k);
  if (store) ucut[off + node] = u;
  return u;
}

// --------------------------------------------------------------------------
// Prolongation (itemised algorithm):
//   u^k_mu = u^{k,cut}_mu + sum_nu Phi(mu/2 - nu)^3 u^{k+1}_nu, |mu - 2 nu| <= order - 1.
// Per dimension, an even fine index m reads only nu = m/2 (weight Phi(0) = 1);
// an odd one reads the ORDER coarse nodes nu = (m - R)/2 + i.
//
// Every level in one launch.  The blocks own 8 x 8 x 8 node tiles of every
// level below the top (level 0 first).  A block of level k rebuilds in LDS the
// coarser potentials its tile reads: the top grid over a box of nodes, then
// levels l-2 .. k+1 each over the box the next finer box reads, and finally
// writes u^k (and the completed u^{k,cut}) of its tile.  A box (o, e) of
// level j reads the level-(j+1) box (ceil((o - R)/2), (e - 1 + 2R)/2 + 2),
// which never exceeds 2R + 3 nodes per side.  Every rebuilt value is computed
// by the same operations as at its owner, so the results equal those of a
// level-by-level pass while the blocks need no other block's output.
// --------------------------------------------------------------------------
constexpr int kPX = 8, kPY = 8, kPZ = 8;
constexpr int kPThreads = kPX * kPY * kPZ;          // one thread per node of a tile

__host__ __device__ inline int prolong_tiles(const Level& F) {
  return ((F.n[0] + kPX - 1) / kPX) * ((F.n[1] + kPY - 1) / kPY) * ((F.n[2] + kPZ - 1) / kPZ);
}

__device__ __forceinline__ int ceil_half(int v) { return v >= 0 ? (v + 1) / 2 : -((-v) / 2); }

// Prolongation weights along one dimension for the absolute fine index m:
// first coarse node (local to a box starting at c0) and ORDER taps.  An odd m
// takes its ORDER weights from nu = (m - R)/2; an even m the weight 1 at
// nu = m/2 among zeros from nu = (m - R + 1)/2 (zero taps leave the sums
// unchanged, and all of them lie inside the box).
template <int ORDER>
__device__ __forceinline__ int prolong_taps(int m, int c0, float* w) {
  using D = Dyadic<ORDER>;
  constexpr int R = D::R;
  constexpr int E0 = (R - 1) / 2;                      // tap of nu = m/2 for even m
  const bool odd = (m & 1) != 0;
#pragma unroll
  for (int i = 0; i < ORDER; ++i) w[i] = odd ? D::wodd(i) : (i == E0 ? 1.f : 0.f);
  return (odd ? (m - R) / 2 : (m - R + 1) / 2) - c0;   // exact halves of even numbers
}

// The prolongation of a coarse box (co, ce) in cs onto the fine box (fo, fe)
// in two passes.  x pass: for every coarse (z, y) row and fine x, the row sum
//   xs[zc][yc][xf] = sum_a wx_a cs[zc][yc][bx + a]          (a ascending)
// into xs (ce[2] x ce[1] x fe[0], x fastest); then, per fine node,
//   sum_{c, b} (wz_c wy_b) xs[bz + c][by + b][xf]            (c, then b ascending)
// in prolong_yz.  The order of operations is that of the direct triple sum.
template <int ORDER>
__device__ __forceinline__ void prolong_x(const float* cs, const int* co, const int* ce, const int* fo,
                                          const int* fe, float* xs) {
  const int n = ce[2] * ce[1] * fe[0];
  const float inv_x = 1.f / (float)fe[0];
  for (int i = threadIdx.x; i < n; i += kPThreads) {
    int xf;
    const int row = fdiv(i, fe[0], inv_x, xf);         // zc * ce[1] + yc
    float w[ORDER];
    const int bx = prolong_taps<ORDER>(fo[0] + xf, co[0], w);
    const float* rowp = cs + row * ce[0] + bx;
    float r[ORDER];
#pragma unroll
    for (int a = 0; a < ORDER; ++a) r[a] = rowp[a];
    float racc = 0.f;
#pragma unroll
    for (int a = 0; a < ORDER; ++a) racc = fmaf(w[a], r[a], racc);
    xs[i] = racc;
  }
}

template <int ORDER>
__device__ __forceinline__ float prolong_yz(const float* xs, const int* co, const int* ce, const int* fe,
                                            const int* m, int xf) {
  float wy[ORDER], wz[ORDER];
  const int by = prolong_taps<ORDER>(m[1], co[1], wy);
  const int bz = prolong_taps<ORDER>(m[2], co[2], wz);
  const float* base = xs + (bz * ce[1] + by) * fe[0] + xf;
  float r[ORDER][ORDER];                               // every read in flight before the sums
#pragma unroll
  for (int c = 0; c < ORDER; ++c)
#pragma unroll
    for (int b = 0; b < ORDER; ++b) r[c][b] = base[(c * ce[1] + b) * fe[0]];
  float acc = 0.f;
#pragma unroll
  for (int c = 0; c < ORDER; ++c)
#pragma unroll
    for (int b = 0; b < ORDER; ++b) acc = fmaf(wz[c] * wy[b], r[c][b], acc);
  return acc;
}

// Box of level j read (through levels k+1 .. j-1) by the tile (to, (kPX, kPY, kPZ))
// of level k: origin (absolute) and extents.  Uniform arithmetic.
template <int R>
__device__ __forceinline__ void box_of(int k, int j, const int* to, int* o, int* e) {
  o[0] = to[0];
  o[1] = to[1];
  o[2] = to[2];
  e[0] = kPX;
  e[1] = kPY;
  e[2] = kPZ;
  for (int i = k; i < j; ++i) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      o[d] = ceil_half(o[d] - R);
      e[d] = (e[d] - 1 + 2 * R) / 2 + 2;
    }
  }
}

// LDS of one block: a box of up to (2R + 3)^3 nodes, padded to a whole number
// of block-wide rounds, for each level above the block's own, and one more for
// the x-pass sums (dynamic shared memory, sized for the launch's deepest system).
__host__ __device__ constexpr int prolong_box(int order) {
  return ((2 * order + 1) * (2 * order + 1) * (2 * order + 1) + kPThreads - 1) / kPThreads * kPThreads;
}

// Few waves per SIMD (one launch of a few hundred blocks): registers are spent
// on loads in flight instead of occupancy.
//
// With ONE set the launch covers the tiles of level `level` only and reads the
// finished u^{level+1} from global memory (written by the launch of the level
// above), so nothing is rebuilt: for large grids, where a level-0 block would
// otherwise rebuild several (2R + 3)^3 boxes for its 8^3 nodes, the per-level
// launches do each level's work once.  Results are the same either way.
template <int ORDER, bool ONE>
__global__ void __launch_bounds__(kPThreads) __attribute__((amdgpu_waves_per_eu(1, 2)))
k_prolong(KArgs A, int level) {
  int blk;
  __shared__ __align__(16) SysDesc sdesc;
  const SysDesc& S = stage_desc(sys_of(A, blk), &sdesc);
  const Geom& g = S.g;
  float* __restrict__ u = S.d.u;
  constexpr int R = Dyadic<ORDER>::R;
  constexpr int BOX = prolong_box(ORDER);              // (2R + 3)^3 rounded up to kPThreads
  constexpr int SL = BOX / kPThreads;                     // nodes per thread and box
  constexpr int LV = SL >= 9 ? 1 : 9 / SL;             // boxes per round of loads
  extern __shared__ float pbox[];                      // box of level j at pbox + (j - k - 1) * BOX
  const int top = g.levels - 1;
  // level and tile of this block
  int k = 0, t = blk;
  if (ONE) {
    k = level;
  } else {
    while (k + 1 < top && t >= prolong_tiles(g.lv[k])) {
      t -= prolong_tiles(g.lv[k]);
      ++k;
    }
  }
  float* __restrict__ xs = pbox + (ONE ? 1 : top - k) * BOX;     // x-pass sums of the box being built
  const Level F = g.lv[k];
  const int ntx = (F.n[0] + kPX - 1) / kPX, nty = (F.n[1] + kPY - 1) / kPY;
  const int bx = t % ntx, by = (t / ntx) % nty, bz = t / (ntx * nty);
  const int to[3] = {F.lo[0] + bx * kPX, F.lo[1] + by * kPY, F.lo[2] + bz * kPZ};   // absolute
  const int tx = threadIdx.x % kPX, ty = (threadIdx.x / kPX) % kPY, tz = threadIdx.x / (kPX * kPY);
  const int fx = bx * kPX + tx, fy = by * kPY + ty, fz = bz * kPZ + tz;          // level-local
  const bool inside = fx < F.n[0] && fy < F.n[1] && fz < F.n[2];
  const int node = (fz * F.n[1] + fy) * F.n[0] + fx;
  const float own = inside ? ucut_value(S, k, node, false) : 0.f;   // stored with u^k at the end
  // Fill the boxes, LV of them per round of loads: u^{l-1} for the top box,
  // u^{j,cut} for the others (the sum of the partials in group order where
  // grouped), zero outside the grids.  Every load of a round is issued before
  // the first sum; the per-level choices are uniform branches.
  const int nlev = ONE ? 1 : top - k;
  for (int j0 = 0; j0 < nlev; j0 += LV) {
    float fv[LV][SL];
    double pv[LV][SL][kLatMaxGroups];
    bool ok[LV][SL];
    int ng[LV];
#pragma unroll
    for (int lv = 0; lv < LV; ++lv) {
      ng[lv] = 0;
      if (j0 + lv >= nlev) continue;
      const int j = k + 1 + j0 + lv;
      int o[3], e[3];
      box_of<R>(k, j, to, o, e);
      const Level J = g.lv[j];
      const int groups = (ONE || j == top || S.lat.b == 0 || j >= S.lat.n) ? 1 : S.lat.t[j].groups;
      ng[lv] = groups;
      const float inv_e0 = 1.f / (float)e[0], inv_e01 = 1.f / (float)(e[0] * e[1]);
      int jn[SL];
#pragma unroll
      for (int sl = 0; sl < SL; ++sl) {
        const int li = sl * kPThreads + threadIdx.x;
        int lx, ly;
        const int lz = fdiv(li, e[0] * e[1], inv_e01, ly);
        ly = fdiv(ly, e[0], inv_e0, lx);
        const int vx = o[0] + lx - J.lo[0], vy = o[1] + ly - J.lo[1], vz = o[2] + lz - J.lo[2];
        ok[lv][sl] = lz < e[2] && vx >= 0 && vx < J.n[0] && vy >= 0 && vy < J.n[1] && vz >= 0 && vz < J.n[2];
        jn[sl] = J.off + (ok[lv][sl] ? (vz * J.n[1] + vy) * J.n[0] + vx : 0);
      }
      if (groups == 1) {
        const float* __restrict__ src = (ONE || j == top) ? u : S.d.ucut;   // finished u, or u^{j,cut}
#pragma unroll
        for (int sl = 0; sl < SL; ++sl) fv[lv][sl] = src[jn[sl]];
      } else {
        const double* __restrict__ part = S.d.lat_part + S.lat.t[j].part0 - J.off;
        const size_t cnt = (size_t)J.count;
#pragma unroll
        for (int gi = 0; gi < kLatMaxGroups; ++gi)
          if (gi < groups)
#pragma unroll
            for (int sl = 0; sl < SL; ++sl) pv[lv][sl][gi] = part[gi * cnt + jn[sl]];
      }
    }
#pragma unroll
    for (int lv = 0; lv < LV; ++lv) {
      if (j0 + lv >= nlev) continue;
      const int j = k + 1 + j0 + lv;
#pragma unroll
      for (int sl = 0; sl < SL; ++sl) {
        float v;
        if (ng[lv] == 1) {
          v = fv[lv][sl];
        } else {
          double d = 0.0;
#pragma unroll
          for (int gi = 0; gi < kLatMaxGroups; ++gi)
            if (gi < ng[lv]) d += pv[lv][sl][gi];
          v = (float)ldexp(d, -j);
        }
        pbox[(j0 + lv) * BOX + sl * kPThreads + threadIdx.x] = ok[lv][sl] ? v : 0.f;
      }
    }
  }
  __syncthreads();
  // levels top-1 .. k+1 in place: u^j = u^{j,cut} + prolongation of u^{j+1}
  for (int j = ONE ? k : top - 1; j > k; --j) {
    const Level J = g.lv[j];
    int jo[3], je[3], co[3], ce[3];
    box_of<R>(k, j, to, jo, je);
    box_of<R>(k, j + 1, to, co, ce);
    float* __restrict__ fine = pbox + (j - k - 1) * BOX;
    prolong_x<ORDER>(fine + BOX, co, ce, jo, je, xs);
    __syncthreads();
    const int nb = je[0] * je[1] * je[2];
    const float inv_e0 = 1.f / (float)je[0], inv_e01 = 1.f / (float)(je[0] * je[1]);
    for (int i = threadIdx.x; i < nb; i += kPThreads) {
      int lx, ly;
      const int lz = fdiv(i, je[0] * je[1], inv_e01, ly);
      ly = fdiv(ly, je[0], inv_e0, lx);
      const int m[3] = {jo[0] + lx, jo[1] + ly, jo[2] + lz};
      const int vx = m[0] - J.lo[0], vy = m[1] - J.lo[1], vz = m[2] - J.lo[2];
      if (vx >= 0 && vx < J.n[0] && vy >= 0 && vy < J.n[1] && vz >= 0 && vz < J.n[2])
        fine[i] = fine[i] + prolong_yz<ORDER>(xs, co, ce, je, m, lx);
    }
    __syncthreads();
  }
  {
    int co[3], ce[3];
    const int te[3] = {kPX, kPY, kPZ};
    box_of<R>(k, k + 1, to, co, ce);
    prolong_x<ORDER>(pbox, co, ce, to, te, xs);
    __syncthreads();
    if (!inside) return;
    const int m[3] = {to[0] + tx, to[1] + ty, to[2] + tz};
    u[F.off + (size_t)node] = own + prolong_yz<ORDER>(xs, co, ce, te, m, tx);
  }
  if (!(S.lat.b == 0 || k >= S.lat.n) && S.lat.t[k].groups > 1) S.d.ucut[F.off + (size_t)node] = own;
}

// Fixed-order block reduction of one energy and (with vir_on) 9 virial values
// per thread (DPP sum within the wave, then the waves in order) into the
// block's slot of the float64 partials (component t at t * n_partials + blk).
__device__ __forceinline__ void block_partials(double e, const double* vir, double* partials, int n_partials,
                                               int blk, bool vir_on) {
  __shared__ double red[10][kBlock / kWave];
  const int nv = vir_on ? 10 : 1;
  double vals[10];
  vals[0] = e;
#pragma unroll
  for (int t = 0; t < 9; ++t) vals[t + 1] = vir[t];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int t = 0; t < 10; ++t)
    if (t < nv) {
      const double v = wave_sum_d63(vals[t]);
      if (lane == kWave - 1) red[t][wave] = v;
    }
  __syncthreads();
  if (threadIdx.x < nv) {
    double v = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) v += red[threadIdx.x][w];
    partials[(size_t)threadIdx.x * n_partials + blk] = v;
  }
}

// --------------------------------------------------------------------------
// Interpolation (itemised algorithm) and assembly (potential display, force as
// minus gradient):  phi_i^L = sum_mu phi^0_mu(r_i) u^0_mu,  grad phi_i^L,
//   phi_i = ke (phi^s + phi^L - q_i gamma(0)/a),  F_i = ke (F^s - q_i grad phi^L).
// Per-block float64 partials of E = 1/2 sum q_i phi_i and W = sum (r_i - lo) F_i.
// --------------------------------------------------------------------------
// MODE 0: forces and potentials, plus per-block energy/virial partials.
// MODE 1: gradients of the energy scaled by *gscale: fx..fz receive
//         gscale dE/dr = -gscale F, phi receives gscale dE/dq = gscale phi.
// Bonded exclusions (pairs left out of the Coulomb sum).  For the atom with
// local input index i: the sums over its listed partners j of q_j / r and of
// q_j (r_i - r_j) / r^3, from the caller's float32 inputs.  A list entry out
// of range (start not within [0, nnz], a partner outside this system) sets
// kFlagBadExclusion and ends the atom's list.
// r_i - r_j of a listed pair.  Periodic plans: from the coordinates binning
// stores, at the image of j nearest to i, placed as the short-range pass
// stages it, so the pair's term comes out bit for bit as that pass added it.
__device__ __forceinline__ void pair_disp(const Geom& g, const Io& io, int gi, int gj, float& dx, float& dy,
                                          float& dz) {
  if (!g.periodic) {
    dx = io.x[gi] - io.x[gj];
    dy = io.y[gi] - io.y[gj];
    dz = io.z[gi] - io.z[gj];
    return;
  }
  const float pi[3] = {io.x[gi], io.y[gi], io.z[gi]}, pj[3] = {io.x[gj], io.y[gj], io.z[gj]};
  float d[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float wi = sorted_coord(g, pi[c], c), wj = sorted_coord(g, pj[c], c);
    const double s = g.len[c] * (double)rintf((wi - wj) * g.inv_len_f[c]);
    d[c] = wi - shifted(wj, s);
  }
  dx = d[0];
  dy = d[1];
  dz = d[2];
}

struct ExclSums {
  float p = 0.f, x = 0.f, y = 0.f, z = 0.f;
};

__device__ __forceinline__ bool excl_range(const SysDesc& S, int i, int& b, int& e) {
  const int gi = S.atom_off + i;
  b = S.d.excl_start[gi];
  e = S.d.excl_start[gi + 1];
  if (b < 0 || e < b || (long long)e > S.d.excl_nnz) {
    atomicOr(S.d.status, kFlagBadExclusion);
    return false;
  }
  return true;
}

__device__ __forceinline__ bool excl_partner(const SysDesc& S, int k, int& j) {
  j = S.d.excl_idx[k];
  if ((unsigned)(j - S.atom_off) >= (unsigned)S.g.n_atoms) {
    atomicOr(S.d.status, kFlagBadExclusion);
    return false;
  }
  return true;
}

__device__ ExclSums coulomb_exclusions(const SysDesc& S, const Io& io, int i) {
  ExclSums r;
  int b, e;
  if (!S.d.excl_start || !excl_range(S, i, b, e)) return r;
  const int gi = S.atom_off + i;
  for (int k = b; k < e; ++k) {
    int j;
    if (!excl_partner(S, k, j)) break;
    float dx, dy, dz;
    pair_disp(S.g, io, gi, j, dx, dy, dz);
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    if (!(r2 > 0.f)) continue;
    const float ri = 1.f / sqrtf(r2);
    const float qj = io.q[j];
    r.p = fmaf(qj, ri, r.p);
    const float w = qj * ri * ri * ri;
    r.x = fmaf(w, dx, r.x);
    r.y = fmaf(w, dy, r.y);
    r.z = fmaf(w, dz, r.z);
  }
  return r;
}

// The same sums for a cheap pair method: q_j e(r) and q_j (-e'(r)/r) (r_i -
// r_j) over the listed partners that the short-range pass counted (0 < r^2
// < rc^2 decided in float32 as there), with its pair functions.
__device__ ExclSums pair_exclusions(const SysDesc& S, const Io& io, int i) {
  ExclSums r;
  int b, e;
  if (!S.d.excl_start || !excl_range(S, i, b, e)) return r;
  const Geom& g = S.g;
  const int gi = S.atom_off + i;
  for (int k = b; k < e; ++k) {
    int j;
    if (!excl_partner(S, k, j)) break;
    float dx, dy, dz;
    pair_disp(g, io, gi, j, dx, dy, dz);
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    if (!(r2 > 0.f && r2 < g.a2)) continue;
    const float ri = 1.f / sqrtf(r2);
    float ev, fr;
    if (g.pair == kPairCutoff) {
      ev = ri;
      fr = ri * ri * ri;
    } else if (g.pair == kPairShiftedForce) {
      ev = ri + fmaf(r2 * ri, g.pk[1], -2.f * g.pk[0]);
      fr = ri * fmaf(ri, ri, -g.pk[1]);
    } else {
      const float ex = __builtin_amdgcn_exp2f(g.pk[3] * r2);
      const float er = wolf_erfc(g.ec, g.pk[0] * (r2 * ri), ex);
      ev = fmaf(er, ri, -g.pk[1]);
      fr = ri * ri * fmaf(er, ri, g.pk[2] * ex);
    }
    const float qj = io.q[j];
    r.p = fmaf(qj, ev, r.p);
    const float w = qj * fr;
    r.x = fmaf(w, dx, r.x);
    r.y = fmaf(w, dy, r.y);
    r.z = fmaf(w, dz, r.z);
  }
  return r;
}

constexpr int kInterpBox = 2048;   // nodes of u^0 one wave stages in LDS (8 KB)
constexpr int kInterpStageAtoms = 65536;   // systems from this size stage u^0 in LDS

template <int ORDER, int MODE>
__global__ void __launch_bounds__(kBlock) k_interp(KArgs A) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  const Geom& g = S.g;
  const float4* __restrict__ sorted = S.d.sorted;
  const int* __restrict__ perm = S.d.perm;
  const float4* __restrict__ fshort = S.d.fshort;
  const float* __restrict__ u = S.d.u;
  float* __restrict__ fx = A.io.fx ? A.io.fx + S.atom_off : nullptr;
  float* __restrict__ fy = A.io.fy ? A.io.fy + S.atom_off : nullptr;
  float* __restrict__ fz = A.io.fz ? A.io.fz + S.atom_off : nullptr;
  float* __restrict__ phi = A.io.phi ? A.io.phi + S.atom_off : nullptr;
  double* __restrict__ partials = S.d.partials;
  const int n_partials = S.n_partials;
  const double* __restrict__ gscale = A.io.gscale ? A.io.gscale + S.index : nullptr;
  constexpr int H = ORDER / 2;
  const Level L = g.lv[0];
  const int s = blk * blockDim.x + threadIdx.x;
  const bool live = s < g.n_atoms;
  double e = 0.0, vir[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) vir[t] = 0.0;
  // Every lane of the block takes part in the staging below (a lane past the
  // last atom takes that atom's place and discards its result).
  const float4 p = g.n_atoms > 0 ? sorted[live ? s : g.n_atoms - 1] : make_float4(0.f, 0.f, 0.f, 0.f);
  const float pp[3] = {p.x, p.y, p.z};
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
  // sum_{sx,sy,sz} w_x w_y w_z u and its three partial derivatives over the
  // ORDER^3 nodes from src (the node base of this atom), rows sy apart, planes sz
  float pl = 0.f, gx = 0.f, gy = 0.f, gz = 0.f;
  auto gather = [&](const float* src, int sy_stride, int sz_stride) {
#pragma unroll ORDER == 4 ? ORDER : 1
    for (int sz = 0; sz < ORDER; ++sz) {
      float py_ = 0.f, gxy = 0.f, gyy = 0.f;
#pragma unroll
      for (int sy = 0; sy < ORDER; ++sy) {
        const float* rowp = src + sz * sz_stride + sy * sy_stride;
        float vx = 0.f, dvx = 0.f;
#pragma unroll
        for (int sx = 0; sx < ORDER; ++sx) {
          const float uv = rowp[sx];
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
  };
  // The atoms of one link-cell row are consecutive in sorted order and close
  // together, so the nodes they read form a small box of u^0: the lanes of a
  // row stage their box in the wave's LDS slice with coalesced loads, then
  // every lane reads its ORDER^3 nodes from there.  A wave whose atoms span
  // several rows takes them one row at a time; a row whose box exceeds the
  // slice reads u^0 directly.
  __shared__ float stage[kBlock / kWave][kInterpBox];
  const int lane = threadIdx.x & (kWave - 1);
  float* box = stage[threadIdx.x / kWave];
  const int row = cell_coord(g, p.z, 2) * g.nc[1] + cell_coord(g, p.y, 1);
  const float* u0 = u + L.off;
  const int n0 = L.n[0], n01 = L.n[0] * L.n[1];
  // (a system of fewer than kInterpStageAtoms atoms reads u^0 directly: its
  // grid stays in the L2 and the staging round only adds latency)
  if (g.n_atoms < kInterpStageAtoms) {
    if (live) gather(u0 + (size_t)base[2] * n01 + (size_t)base[1] * n0 + base[0], n0, n01);
  }
  for (unsigned long long pending = g.n_atoms < kInterpStageAtoms ? 0ull : __ballot(live); pending;) {
    const int lead = __ffsll((long long)pending) - 1;
    const int grow = __builtin_amdgcn_readlane(row, lead);
    const bool mine = ((pending >> lane) & 1ull) && row == grow;
    pending &= ~__ballot(mine);
    int lo3[3], ext[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo3[d] = wave_min_s(mine ? base[d] : INT_MAX);
      ext[d] = wave_max_s(mine ? base[d] : INT_MIN) - lo3[d] + ORDER;
    }
    const int vol = ext[0] * ext[1] * ext[2];
    // the box lies in the grid (every base does), checked before any load
    const bool inside = lo3[0] >= 0 && lo3[1] >= 0 && lo3[2] >= 0 && lo3[0] + ext[0] <= L.n[0] &&
                        lo3[1] + ext[1] <= L.n[1] && lo3[2] + ext[2] <= L.n[2];
    if (inside && vol <= kInterpBox) {
      const float inv0 = 1.f / (float)ext[0], inv1 = 1.f / (float)ext[1];
      const float* corner = u0 + (size_t)lo3[2] * n01 + (size_t)lo3[1] * n0 + lo3[0];
      // 16 loads per lane in flight at a time
      for (int i0 = 0; i0 < vol; i0 += 16 * kWave) {
        float v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const int i = i0 + k * kWave + lane;
          v[k] = 0.f;
          if (i < vol) {
            int xx, yy;
            const int zz = fdiv(fdiv(i, ext[0], inv0, xx), ext[1], inv1, yy);
            v[k] = corner[zz * n01 + yy * n0 + xx];
          }
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
          const int i = i0 + k * kWave + lane;
          if (i < vol) box[i] = v[k];
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (mine)
        gather(box + ((base[2] - lo3[2]) * ext[1] + (base[1] - lo3[1])) * ext[0] + (base[0] - lo3[0]), ext[0],
               ext[0] * ext[1]);
      // the next row's staging overwrites the slice
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else if (mine) {
      gather(u0 + (size_t)base[2] * n01 + (size_t)base[1] * n0 + base[0], n0, n01);
    }
  }
  if (live) {
    gx *= g.inv_h;
    gy *= g.inv_h;
    gz *= g.inv_h;
    float4 fs = fshort[s];
    // excluded pairs lose their whole Coulomb term q_i q_j / r (the short-range
    // part and the smooth part the grids carry)
    const ExclSums ex = coulomb_exclusions(S, A.io, perm[s]);
    gx += ex.x;
    gy += ex.y;
    gz += ex.z;
    fs.w -= ex.p;
    double qd = (double)p.w;
    double ph = g.ke * ((double)fs.w + (double)pl - qd * (double)g.self);
    if (MODE == 1) {
      const double gsc = *gscale;
      const int i = perm[s];
      if (fx) {
        fx[i] = (float)(-gsc * g.ke * ((double)fs.x - qd * (double)gx));
        fy[i] = (float)(-gsc * g.ke * ((double)fs.y - qd * (double)gy));
        fz[i] = (float)(-gsc * g.ke * ((double)fs.z - qd * (double)gz));
      }
      if (phi) phi[i] = (float)(gsc * ph);
    } else {
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
  }
  // gradient mode has no reductions: every thread of the block leaves here
  if (MODE == 1) return;
  block_partials(e, vir, partials, n_partials, blk, A.io.virial != nullptr);
}

// Assembly of a cheap pair method evaluated on its own (no grids):
//   phi_i = ke (phi_i^pair - q_i self),  F_i = ke F_i^pair,
// with self = -2 s (s the method's self-energy coefficient), plus per-block
// float64 partials of E = 1/2 sum q_i phi_i and W = sum (r_i - lo) F_i.
__global__ void __launch_bounds__(kBlock) k_pair_finish(KArgs A) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  const Geom& g = S.g;
  float* __restrict__ fx = A.io.fx ? A.io.fx + S.atom_off : nullptr;
  float* __restrict__ fy = A.io.fy ? A.io.fy + S.atom_off : nullptr;
  float* __restrict__ fz = A.io.fz ? A.io.fz + S.atom_off : nullptr;
  float* __restrict__ phi = A.io.phi ? A.io.phi + S.atom_off : nullptr;
  const int s = blk * blockDim.x + threadIdx.x;
  double e = 0.0, vir[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) vir[t] = 0.0;
  if (s < g.n_atoms) {
    const float4 p = S.d.sorted[s];
    float4 fs = S.d.fshort[s];
    const int i = S.d.perm[s];
    // excluded pairs lose the method's own pair term
    const ExclSums ex = pair_exclusions(S, A.io, i);
    fs.x -= p.w * ex.x;
    fs.y -= p.w * ex.y;
    fs.z -= p.w * ex.z;
    fs.w -= ex.p;
    const double qd = (double)p.w;
    const double ph = g.ke * ((double)fs.w - qd * (double)g.self);
    const float of[3] = {(float)(g.ke * (double)fs.x), (float)(g.ke * (double)fs.y), (float)(g.ke * (double)fs.z)};
    if (fx) {
      fx[i] = of[0];
      fy[i] = of[1];
      fz[i] = of[2];
    }
    if (phi) phi[i] = (float)ph;
    e = 0.5 * qd * ph;
    const double rr[3] = {(double)p.x - g.lo[0], (double)p.y - g.lo[1], (double)p.z - g.lo[2]};
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) vir[3 * a + b] = rr[a] * (double)of[b];
  }
  block_partials(e, vir, S.d.partials, S.n_partials, blk, A.io.virial != nullptr);
}

// Energy without prolongation or interpolation (grid form):
//   E = 1/2 sum_i q_i phi_i^s + 1/2 sum_k <q^k, u^{k,cut}> - gamma(0)/(2a) sum_i q_i^2,
// since 1/2 q^0.u^0 = 1/2 sum_k <q^k, u^{k,cut}> when prolongation is the
// transpose of restriction.  One float64 partial per block.
__global__ void __launch_bounds__(kBlock) k_energy_terms(KArgs A) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  const Geom& g = S.g;
  const float4* __restrict__ sorted = S.d.sorted;
  const float4* __restrict__ fshort = S.d.fshort;
  const float* __restrict__ qgrid = S.d.qgrid;
  double* __restrict__ partials = S.d.partials;
  __shared__ double red[kBlock / kWave];
  const int stride = S.n_partials * blockDim.x;
  double e = 0.0;
  for (int i = blk * blockDim.x + threadIdx.x; i < g.n_atoms; i += stride) {
    const double q = (double)sorted[i].w;
    const double ex = S.d.excl_start ? (double)coulomb_exclusions(S, A.io, S.d.perm[i]).p : 0.0;
    e += 0.5 * q * ((double)fshort[i].w - ex - q * (double)g.self);
  }
  for (int k = 0; k < g.levels; ++k) {
    const Level& L = g.lv[k];
    for (int m = blk * blockDim.x + threadIdx.x; m < L.count; m += stride) {
      if (g.periodic) {                     // the nodes of one period only (ghosts are copies)
        const int mx = m % L.n[0] - g.ghost, my = (m / L.n[0]) % L.n[1] - g.ghost;
        const int mz = m / (L.n[0] * L.n[1]) - g.ghost;
        if (mx < 0 || my < 0 || mz < 0 || mx >= L.per[0] || my >= L.per[1] || mz >= L.per[2]) continue;
      }
      e += 0.5 * (double)qgrid[L.off + m] * (double)ucut_value(S, k, m, true);
    }
  }
  e *= g.ke;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) e += __shfl_xor(e, off);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if (lane == 0) red[wave] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) v += red[w];
    partials[blk] = v;
  }
}

// Sum the per-block partials in a fixed order (one block): each thread adds
// its strided share, then a DPP sum per wave and the 4 waves in order.
__global__ void __launch_bounds__(kBlock) k_reduce(KArgs A, int with_virial) {
  int blk;
  const SysDesc& S = sys_of(A, blk);
  const double* __restrict__ partials = S.d.partials;
  const int n_partials = S.g.n_atoms > 0 ? S.n_partials : 0;
  double* __restrict__ energy = A.io.energy ? A.io.energy + S.index : nullptr;
  double* __restrict__ virial = (with_virial && A.io.virial) ? A.io.virial + 9 * (size_t)S.index : nullptr;
  // the virial partials exist only when the evaluation asked for the virial
  const int nv = A.io.virial ? 10 : 1;
  __shared__ double red[10][kBlock / kWave];
  double acc[10];
#pragma unroll
  for (int t = 0; t < 10; ++t) acc[t] = 0.0;
  if (nv == 1) {
    // energy only: 8 loads per thread in flight, added in index order
    for (int b0 = threadIdx.x; b0 < n_partials; b0 += 8 * kBlock) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = b0 + u * kBlock < n_partials ? partials[b0 + u * kBlock] : 0.0;
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[0] += v[u];
    }
  } else {
    for (int b = threadIdx.x; b < n_partials; b += kBlock) {
      double v[10];
#pragma unroll
      for (int t = 0; t < 10; ++t) v[t] = partials[(size_t)t * n_partials + b];
#pragma unroll
      for (int t = 0; t < 10; ++t) acc[t] += v[t];
    }
  }
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int t = 0; t < 10; ++t)
    if (t < nv) {
      const double v = wave_sum_d63(acc[t]);
      if (lane == kWave - 1) red[t][wave] = v;
    }
  __syncthreads();
  if (threadIdx.x < nv) {
    double v = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) v += red[threadIdx.x][w];
    if (threadIdx.x == 0) {
      if (energy) energy[0] = v;
    } else if (virial) {
      virial[threadIdx.x - 1] = v;
    }
  }
}

inline int blocks_for(int n, int b = kBlock) { return (n + b - 1) / b; }

}  // namespace

int interp_partials(const Geom& g) { return std::max(1, blocks_for(g.n_atoms)); }

SysBlocks system_blocks(const Geom& g, const LatLaunch& lat, int n_partials) {
  SysBlocks b{};
  b.zero = blocks_for(g.max_cells + 1);
  b.scan = (g.bin_blocks == 0 && g.bin_row_blocks == 0 && g.binr_blocks == 0)
               ? (g.n_cells + kScanTile - 1) / kScanTile : 0;
  b.rchunk = g.binr_blocks;
  b.rscan = g.binr_blocks > 0 ? 1 : 0;
  b.rsort = g.binr_blocks > 0 ? g.nc[1] * g.nc[2] : 0;
  b.atoms = g.n_atoms > 0 ? blocks_for(g.n_atoms) : 0;
  b.bin = g.bin_blocks;
  b.binrow = g.bin_row_blocks;
  b.shortr = g.n_atoms > 0 ? g.short_blocks : 0;
  const Level& L0 = g.lv[0];
  b.anterp = g.atn[0] * g.atn[1] * g.atn[2];
  b.agather = blocks_for(L0.count);
  for (int k = 0; k + 1 < g.levels; ++k) {
    const Level& C = g.lv[k + 1];
    b.restrict_[k] = ((C.n[0] + kRX - 1) / kRX) * ((C.n[1] + kRY - 1) / kRY) * ((C.n[2] + kRZ - 1) / kRZ);
    b.prolong += prolong_tiles(g.lv[k]);
  }
  // lattice cutoff in two launches: level 0, and levels 1 .. l-2
  if (g.levels > 1) {
    if (lat.b > 0) {
      const LatTile& t = lat.t[lat.n - 1];
      const int total = t.block0 + t.ntx * t.nty * t.ntz * t.groups;
      b.lattice0 = lat.n > 1 ? lat.t[1].block0 : total;
      b.lattice = total - b.lattice0;
    } else {
      b.lattice0 = blocks_for(g.lv[1].off);
      b.lattice = blocks_for(g.lv[g.levels - 1].off - g.lv[1].off);
    }
  }
  const int top_nodes = g.lv[g.levels - 1].count;
  b.lattice_all = b.lattice0 + b.lattice;
  if (g.levels > 1 && lat.b > 0) {
    const int tb = (top_nodes + lat.waves - 1) / lat.waves;  // top level rides in the coarse launch
    b.lattice += tb;
    b.lattice_all += tb;
    b.top = 0;
  } else {
    b.top = blocks_for(top_nodes * kWave);
  }
  b.energy = n_partials;
  return b;
}

int prolong_level_blocks(const Geom& g, int k) { return prolong_tiles(g.lv[k]); }

hipError_t launch_init(const LaunchGeom& L, hipStream_t s) {
  if (L.zero.blocks > 0) k_zero_counts<<<L.zero.blocks, kBlock, 0, s>>>(KArgs{L.sys, L.zero.map, Io{}});
  return hipGetLastError();
}

hipError_t launch_eval(int mode, const LaunchGeom& L, hipStream_t s, const Io& io, hipEvent_t* ev,
                       const Concurrency* cc, bool live) {
  const bool forces = (mode != kModeEnergy);
  auto args = [&](const StageGrid& sg) { return KArgs{L.sys, sg.map, io}; };
  // in-order timing: one event at every stage boundary on s
  auto mark = [&](int stage) {
    if (ev && !live) (void)hipEventRecord(ev[stage], s);
  };
  // live timing: a begin and an end event around each slot's launches, on the
  // stream they run on; slots without work get an empty interval on s
  bool recorded[kLiveSlots] = {};
  auto beg = [&](int slot, hipStream_t st) {
    if (ev && live) (void)hipEventRecord(ev[slot], st);
  };
  auto end = [&](int slot, hipStream_t st) {
    if (ev && live) {
      (void)hipEventRecord(ev[kLiveSlots + slot], st);
      recorded[slot] = true;
    }
  };
  auto finish = [&]() {
    for (int slot = 0; slot < kLiveSlots; ++slot)
      if (ev && live && !recorded[slot]) {
        beg(slot, s);
        end(slot, s);
      }
    return hipGetLastError();
  };
  // fork: `side` waits for everything enqueued on s so far
  auto fork = [&](const SideStream& side) {
    (void)hipEventRecord(side.fork, s);
    (void)hipStreamWaitEvent(side.stream, side.fork, 0);
  };
  auto join = [&](const SideStream& side) { (void)hipStreamWaitEvent(s, side.join, 0); };
  const bool concurrent = (cc != nullptr && (ev == nullptr || live));   // in-order timing runs in order
  const bool have_atoms = L.atoms.blocks > 0;

  mark(kStageBin);
  beg(kStageBin, s);
  if (L.bin4) {
    if (have_atoms) k_bin_count<<<L.atoms.blocks, kBlock, 0, s>>>(args(L.atoms));
    k_scan_tiles<<<L.scan.blocks, kScanThreads, 0, s>>>(args(L.scan));
    k_scan_apply<<<L.scan.blocks, kScanThreads, 0, s>>>(args(L.scan));
    if (have_atoms) {
      k_bin_scatter<<<L.atoms.blocks, kBlock, 0, s>>>(args(L.atoms));
      k_bin_place<<<L.atoms.blocks, kBlock, 0, s>>>(args(L.atoms));
    }
  }
  if (L.bin.blocks > 0) {
    const int hist_lds = kBinMaxCells * (int)sizeof(int);
    const int sort_lds = (3 * kBinMaxCells + kBinChunk + 2 * kBinThreads) * (int)sizeof(int);
    (void)hipFuncSetAttribute((const void*)k_bin_hist, hipFuncAttributeMaxDynamicSharedMemorySize, hist_lds);
    (void)hipFuncSetAttribute((const void*)k_bin_sort, hipFuncAttributeMaxDynamicSharedMemorySize, sort_lds);
    k_bin_hist<<<L.bin.blocks, kBinThreads, hist_lds, s>>>(args(L.bin));
    k_bin_sort<<<L.bin.blocks, kBinThreads, sort_lds, s>>>(args(L.bin));
  }
  if (L.binrow.blocks > 0) {
    (void)hipFuncSetAttribute((const void*)k_bin_rows, hipFuncAttributeMaxDynamicSharedMemorySize, L.binrow_lds);
    k_bin_rows<<<L.binrow.blocks, kBRThreads, L.binrow_lds, s>>>(args(L.binrow));
  }
  if (L.rchunk.blocks > 0) {
    k_binr_count<<<L.rchunk.blocks, kBRCThreads, 0, s>>>(args(L.rchunk));
    k_binr_scan<<<L.rscan.blocks, kBRCThreads, 0, s>>>(args(L.rscan));
    k_binr_scatter<<<L.rchunk.blocks, kBRCThreads, 0, s>>>(args(L.rchunk));
    (void)hipFuncSetAttribute((const void*)k_binr_sort, hipFuncAttributeMaxDynamicSharedMemorySize, L.rsort_lds);
    k_binr_sort<<<L.rsort.blocks, kBRSThreads, L.rsort_lds, s>>>(args(L.rsort));
  }
  end(kStageBin, s);

  // short-range pairs: on their own stream (forked after binning,
  // anterpolation or the coarse lattice cutoff), joined before interpolation
  mark(kStageShort);
  const bool short_side =
      concurrent && L.streams >= 2 && have_atoms && L.shortr.blocks > 0 && L.pair == kPairMsm;
  // with a side stream, the work items [0, split) start at short_after and the
  // rest after the lattice cutoff
  const int split = (short_side && L.short_split > 0 && L.short_split < 1000) ? L.short_split : 1000;
  int short_part = 0;
  auto launch_short = [&](int lo_pm, int hi_pm) {
    if (!(have_atoms && L.shortr.blocks > 0) || lo_pm >= hi_pm) return;
    hipStream_t ss = s;
    if (short_side) {
      fork(cc->shortr);
      ss = cc->shortr.stream;
    }
    const int slot = short_part++ == 0 ? kStageShort : kSlotShort2;
    beg(slot, ss);
    const KArgs A = args(L.shortr);
    const int nb = L.shortr.blocks;
#define MSM_SHORT_P(MM, FF, KK)                                                        \
  do {                                                                                 \
    if (L.short_periodic)                                                              \
      k_short<MM, FF, KK, true><<<nb, kShortThreads, 0, ss>>>(A, lo_pm, hi_pm);         \
    else                                                                               \
      k_short<MM, FF, KK, false><<<nb, kShortThreads, 0, ss>>>(A, lo_pm, hi_pm);        \
  } while (0)
#define MSM_SHORT(MM)                                                          \
  do {                                                                         \
    if (forces)                                                                \
      MSM_SHORT_P(MM, true, kPairMsm);                                         \
    else                                                                       \
      MSM_SHORT_P(MM, false, kPairMsm);                                        \
  } while (0)
    if (L.pair == kPairCutoff)
      MSM_SHORT_P(1, true, kPairCutoff);
    else if (L.pair == kPairShiftedForce)
      MSM_SHORT_P(1, true, kPairShiftedForce);
    else if (L.pair == kPairWolf)
      MSM_SHORT_P(1, true, kPairWolf);
    else
    switch (L.m) {
      case 1: MSM_SHORT(1); break;
      case 2: MSM_SHORT(2); break;
      case 3: MSM_SHORT(3); break;
      case 4: MSM_SHORT(4); break;
      case 5: MSM_SHORT(5); break;
      case 6: MSM_SHORT(6); break;
      default: MSM_SHORT(7); break;
    }
#undef MSM_SHORT
#undef MSM_SHORT_P
    end(slot, ss);
    if (short_side) (void)hipEventRecord(cc->shortr.join, ss);
  };
  const int short_at = short_side ? L.short_after : 1;
  if (short_at == 1) launch_short(0, split);

  if (L.pair != kPairMsm) {
    // a cheap pair method on its own: no grids
    for (int st = kStageAnterp; st <= kStageInterp; ++st) mark(st);
    beg(kStageInterp, s);
    if (have_atoms) k_pair_finish<<<L.atoms.blocks, kBlock, 0, s>>>(args(L.atoms));
    end(kStageInterp, s);
    mark(kStageReduce);
    beg(kStageReduce, s);
    if (io.energy || io.virial) k_reduce<<<L.one.blocks, kBlock, 0, s>>>(args(L.one), 1);
    end(kStageReduce, s);
    mark(kStageCount);
    return finish();
  }

  mark(kStageAnterp);
  beg(kStageAnterp, s);
  if (L.order == 4) {
    (void)hipFuncSetAttribute((const void*)k_anterp<4>, hipFuncAttributeMaxDynamicSharedMemorySize, L.anterp_lds);
    k_anterp<4><<<L.anterp.blocks, kAThreads, L.anterp_lds, s>>>(args(L.anterp));
    k_anterp_gather<4><<<L.agather.blocks, kBlock, 0, s>>>(args(L.agather));
  } else {
    (void)hipFuncSetAttribute((const void*)k_anterp<6>, hipFuncAttributeMaxDynamicSharedMemorySize, L.anterp_lds);
    k_anterp<6><<<L.anterp.blocks, kAThreads, L.anterp_lds, s>>>(args(L.anterp));
    k_anterp_gather<6><<<L.agather.blocks, kBlock, 0, s>>>(args(L.agather));
  }
  // periodic: ghost copies of level k's grid of `which` (fold: gather them first)
  const KArgs one_sys{L.sys, nullptr, io};
  auto ghosts = [&](int k, int which, int fold) {
    if (L.periodic && L.ghost_blocks[k] > 0) k_ghost<<<L.ghost_blocks[k], kBlock, 0, s>>>(one_sys, k, which, fold);
  };
  ghosts(0, kGhostQ, 1);
  ghosts(0, kGhostQ, 0);
  end(kStageAnterp, s);
  if (short_at == 2) launch_short(0, split);

  // lattice cutoff of one part (0: level 0, 1: levels 1 .. l-2 and the top,
  // 2: all of them) on stream `ls`
  auto lattice = [&](const StageGrid& sg, int part, hipStream_t ls) {
    if (sg.blocks == 0) return;
    const KArgs A = args(sg);
    const int nb = sg.blocks;
#define MSM_LAT(BB, WW)                                                                                      \
  do {                                                                                                      \
    (void)hipFuncSetAttribute((const void*)k_lattice_win<BB, WW>, hipFuncAttributeMaxDynamicSharedMemorySize, \
                              L.lat_lds);                                                                   \
    k_lattice_win<BB, WW><<<nb, WW * kWave, L.lat_lds, ls>>>(A, part);                                       \
  } while (0)
    const bool few = L.lat_waves == kLatWavesFew;
    if (L.lat_b == 4) {
      if (few) MSM_LAT(4, kLatWavesFew); else MSM_LAT(4, kLatWavesMany);
    } else if (L.lat_b == 6) {
      if (few) MSM_LAT(6, kLatWavesFew); else MSM_LAT(6, kLatWavesMany);
    } else if (L.lat_b == 8) {
      if (few) MSM_LAT(8, kLatWavesFew); else MSM_LAT(8, kLatWavesMany);
    } else {
      k_lattice<<<nb, kBlock, 0, ls>>>(A, part);
    }
#undef MSM_LAT
  };
  // level 0 needs only the anterpolated charges: it overlaps the coarse chain
  const bool lat0_side = concurrent && L.streams >= 3 && L.lattice0.blocks > 0;
  if (lat0_side) {
    fork(cc->lattice0);
    beg(kSlotLattice0, cc->lattice0.stream);
    lattice(L.lattice0, 0, cc->lattice0.stream);
    end(kSlotLattice0, cc->lattice0.stream);
    (void)hipEventRecord(cc->lattice0.join, cc->lattice0.stream);
  }

  mark(kStageRestrict);
  beg(kStageRestrict, s);
  for (int k = 0; k + 1 < L.max_levels; ++k) {
    const StageGrid& sg = L.restrict_[k];
    if (sg.blocks == 0) continue;
    if (L.order == 4)
      k_restrict<4><<<sg.blocks, kRThreads, 0, s>>>(args(sg), k);
    else
      k_restrict<6><<<sg.blocks, kRThreads, 0, s>>>(args(sg), k);
    ghosts(k + 1, kGhostQ, 0);
  }
  end(kStageRestrict, s);
  mark(kStageLattice);
  beg(kStageLattice, s);
  if (lat0_side)
    lattice(L.lattice, 1, s);
  else
    lattice(L.lattice_all, 2, s);                      // every level (and the top) in one launch
  end(kStageLattice, s);
  if (short_at == 3) launch_short(0, split);
  launch_short(split, 1000);
  mark(kStageTop);
  beg(kStageTop, s);
  if (L.top.blocks > 0) k_top<<<L.top.blocks, kBlock, 0, s>>>(args(L.top));
  end(kStageTop, s);

  if (mode == kModeEnergy) {
    mark(kStageProlong);
    mark(kStageInterp);
    if (lat0_side) join(cc->lattice0);
    if (short_side) join(cc->shortr);
    mark(kStageReduce);
    beg(kStageReduce, s);
    k_energy_terms<<<L.energy.blocks, kBlock, 0, s>>>(args(L.energy));
    k_reduce<<<L.one.blocks, kBlock, 0, s>>>(args(L.one), 0);
    end(kStageReduce, s);
    mark(kStageCount);
    return finish();
  }

  mark(kStageProlong);
  if (lat0_side) join(cc->lattice0);                 // u^0 adds the level-0 cutoff potential
  beg(kStageProlong, s);
  if (L.prolong.blocks > 0 && L.prolong_split) {
    // one launch per level, coarse to fine (a single system: no block tables)
    const int lds = 2 * prolong_box(L.order) * (int)sizeof(float);             // one box + x-pass sums
    for (int k = L.max_levels - 2; k >= 0; --k) {
      const int nb = L.prolong_level[k];
      if (nb == 0) continue;
      ghosts(k + 1, kGhostU, 0);
      const KArgs A{L.sys, nullptr, io};
      if (L.order == 4)
        k_prolong<4, true><<<nb, kPThreads, lds, s>>>(A, k);
      else
        k_prolong<6, true><<<nb, kPThreads, lds, s>>>(A, k);
    }
  } else if (L.prolong.blocks > 0) {
    const int lds = L.max_levels * prolong_box(L.order) * (int)sizeof(float);   // boxes + x-pass sums
    if (L.order == 4) {
      (void)hipFuncSetAttribute((const void*)k_prolong<4, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                lds);
      k_prolong<4, false><<<L.prolong.blocks, kPThreads, lds, s>>>(args(L.prolong), 0);
    } else {
      (void)hipFuncSetAttribute((const void*)k_prolong<6, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                lds);
      k_prolong<6, false><<<L.prolong.blocks, kPThreads, lds, s>>>(args(L.prolong), 0);
    }
  }
  ghosts(0, kGhostU, 0);
  end(kStageProlong, s);
  mark(kStageInterp);
  if (short_side) join(cc->shortr);
  beg(kStageInterp, s);
  if (have_atoms) {
    const KArgs A = args(L.atoms);
    const int nb = L.atoms.blocks;
    if (mode == kModeGradient) {
      if (L.order == 4)
        k_interp<4, 1><<<nb, kBlock, 0, s>>>(A);
      else
        k_interp<6, 1><<<nb, kBlock, 0, s>>>(A);
    } else {
      if (L.order == 4)
        k_interp<4, 0><<<nb, kBlock, 0, s>>>(A);
      else
        k_interp<6, 0><<<nb, kBlock, 0, s>>>(A);
    }
  }
  end(kStageInterp, s);
  mark(kStageReduce);
  beg(kStageReduce, s);
  if (mode == kModeForces && (io.energy || io.virial)) k_reduce<<<L.one.blocks, kBlock, 0, s>>>(args(L.one), 1);
  end(kStageReduce, s);
  mark(kStageCount);
  return finish();
}

}  // namespace msm
