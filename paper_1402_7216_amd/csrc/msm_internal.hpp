// Internal declarations of libmsm: geometry descriptors passed to the gfx950
// kernels by value, workspace section indices and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/msm.h"

namespace msm {

constexpr int kMaxLevels = 12;
constexpr int kShortWaves = 4;           // waves of a short-range block (they split the neighbour rows)
constexpr int kShortRowsPerWave = 24;    // neighbour rows one wave can take
constexpr int kMaxOrder = 6;
constexpr int kMaxTopNodes = 1 << 17;     // all-pairs FP64 top level stays below ~1e10 pair terms
constexpr int kRankCap = 2048;            // cells longer than this keep scatter order (see bin_place)
constexpr int kBinChunk = 2048;           // atoms per block of the two-kernel binning
constexpr int kXSub = 4;                  // link cells are this many times finer along x
constexpr int kBinMaxCells = 8192;        // cells the two-kernel binning keeps in LDS
constexpr int kBinMaxHist = 1 << 20;      // block histogram entries of the two-kernel binning
constexpr int kBinRowAtoms = 32768;       // atoms per system at most for the one-kernel binning
constexpr int kBinRChunk = 8192;          // atoms per block of the row binning's count and scatter
constexpr int kBinRowsMax = 8192;         // cell rows of a system at most for the row binning
constexpr int kBinRSortCap = 1024;        // atoms of a cell row the row binning's sort keeps in LDS
constexpr int kBinRowCells = 512;         // cells one block of the one-kernel binning owns at most
constexpr int kBinRowMaxBlocks = 256;     // blocks of the one-kernel binning per system at most
constexpr int kStatusWords = 64 + kBinRowMaxBlocks;   // [0]: flags; [64 + b]: flags of binning block b
constexpr int kStatusUnranked = 1;        // status word: some cell kept its scatter order (not checked for
                                          // coincident atoms by binning)
constexpr int kScanTile = 4096;           // cells per block of the four-kernel binning's scan
constexpr int kXcds = 8;                  // accelerator dies of the chip, each with its own L2
constexpr int kProlongSplitTiles = 1000;  // level-0 prolongation tiles from which each level gets its own launch

enum DeviceFlag : int { kFlagOutOfBox = 1, kFlagNonFinite = 2, kFlagCoincident = 4, kFlagBadExclusion = 8 };

// Pair function of the short-range pass: the MSM short-range kernel g*, or one
// of the cheap pair methods evaluated on their own (values of msm_pair_kind).
enum PairKind : int { kPairMsm = 0, kPairCutoff = 1, kPairShiftedForce = 2, kPairWolf = 3 };
constexpr int kWolfTerms = 11;            // terms of the Wolf pair method's erfc polynomial

struct Level {
  int lo[3];     // lowest node index per dimension
  int n[3];      // node count per dimension
  int off;       // first node of this level in the concatenated grid arrays
  int count;     // n[0] * n[1] * n[2]
  int per[3];    // periodic plans: nodes of one period (interior 0 .. per - 1; the
                 // others, lo = -ghost and up, are ghost copies); 0 for free space
};

// Everything the kernels need to know about one system.  Plain data, passed
// by value as a kernel argument.
struct Geom {
  int n_atoms;
  int order, half;                 // interpolation order, order / 2
  int levels;
  int total_nodes;
  float h, inv_h;                  // finest spacing and its reciprocal
  float lo_f[3];                   // box corner (float) = grid origin
  double lo[3], hi[3];             // exact box bounds for the in-box test
  int periodic;                    // 1: the box repeats in every direction
  int ghost;                       // periodic: ghost nodes on each side of every level
  float len_f[3], inv_len_f[3];    // periodic: box edges and their reciprocals
  double len[3];                   // periodic: box edges (images are placed in double precision)
  int fmax[3];                     // largest level-0 floor index floor(len / h)
  // link cells
  int nc[3];
  int n_cells;
  int max_cells;                   // cells of the finest reach any tuning may select (sizes the cell arrays)
  int bin_blocks;                  // blocks of the two-kernel binning (0: another binning)
  int bin_row_blocks;              // blocks of the one-kernel binning (0: another binning)
  int binr_blocks;                 // blocks (kBinRChunk atoms each) of the row binning (0: another binning)
  int reach;                       // neighbour cell rows per side in y and z
  float inv_cs[3];                 // 1 / cell edge
  float cs[3];                     // cell edge (x cells are kXSub times finer than y, z)
  float a_win;                     // cutoff with a margin, for the short-range x windows
  unsigned char short_rows[kShortWaves][kShortRowsPerWave]; // neighbour rows of each short-range wave:
                                                           // (oy + reach) | (oz + reach) << 4, 0xff
                                                           // ends a list
  unsigned char short_pair[kShortWaves][kShortRowsPerWave]; // the row walked together with short_rows
                                                           // (its mirror (-oy, -oz)), 0xff: none
  int item_chunks;                 // short-range 64-atom chunks of a cell row per work item
  int row_items;                   // short-range work items per cell row (chunks interleaved)
  int short_blocks;                // blocks of the short-range launch (work items strided over them)
  // short-range constants
  float a2;                        // cutoff^2
  float inv_a2;                    // 1 / a^2
  float inv_a;                     // 1 / a
  float inv_a2f;                   // 1 / a^2 (float)
  float dr[8];                     // 2 k c_k / a^(2k+1)   (gamma'(r/a)/(a^2 r) = sum_{k>=1} dr[k] r^2(k-1))
  int at[3];                       // anterpolation node tile (level-0 nodes per dimension)
  int atn[3];                      // anterpolation tiles per dimension (they own floor indices 0..fmax)
  int at_ext;                      // nodes of a tile's private region (at[d] + order - 1 per dimension)
  int pair;                        // 0: MSM; else the cheap pair method evaluated alone (kPair*)
  float pk[4];                     // constants of the pair method (see k_short)
  float ec[kWolfTerms];            // Wolf: erfc(x) exp(x^2) as a polynomial in t = 1 / (1 + x/2) (coefficients of t^0..)
  int m;                           // smoothing degree
  float self;                      // gamma(0) / a
  double ke;                       // energy prefactor
  Level lv[kMaxLevels];
};

// Lattice-cutoff stencil: rows (nx, ny) of taps nz in [-zr, zr].
struct StencilRow {
  int nx, ny, zr, woff;
};

// Windowed lattice-cutoff launch: one tile shape per sub-top level.  A tile's
// stencil rows may be split into `groups` contiguous ranges of nz, one block
// each; each such block then writes float64 partial sums per node, which the
// consumers of u^{k,cut} add in group order.
struct LatTile {
  int level;
  int xl, ty, tz;          // lanes along x (B outputs each), y, z
  int ntx, nty, ntz;       // tiles per dimension
  int block0;              // first block of this level
  int px;                  // padded LDS row pitch of the window (floats)
  int pp;                  // padded LDS plane pitch of the window (floats)
  int groups;              // row groups per tile (1: the block writes u^{k,cut} itself)
  int part0;               // first float64 partial of this level (groups * nodes of the level)
};

constexpr int kLatMaxHalo = 16;          // windowed kernel handles stencil half-widths up to this
constexpr int kLatMaxLds = 150 * 1024;   // LDS budget of one windowed block (bytes)
constexpr int kLatWavesFew = 8;          // waves per windowed block for grids of many tiles
constexpr int kLatWavesMany = 16;        // and for grids of few tiles (their totals meet in LDS)
constexpr int kLatWavesTiles = 1024;     // level-0 tiles from which the smaller blocks are used
constexpr int kLatMaxGroups = 8;         // row groups per tile

struct LatLaunch {
  int b;                   // outputs per lane along x (template), 0 = use the untiled kernel
  int n;                   // levels in the launch
  int H;                   // stencil half-width in nodes
  int lds_bytes;           // dynamic LDS per block
  int n_rows;              // compact rows (nz in [-H, H], ny >= 0)
  int n_wc;                // compact weights (floats, each row padded to a multiple of 4)
  int n_part;              // float64 partials of every grouped level
  int waves;               // waves per block (kLatWavesFew or kLatWavesMany)
  // first compact row of group g when a tile has G groups: grp[G][g], g <= G
  short grp[kLatMaxGroups + 1][kLatMaxGroups + 1];
  LatTile t[kMaxLevels];
};

// Workspace sections (in order).  Offsets are 256-byte aligned.
enum Section : int {
  kSecQGrid = 0,      // float[total_nodes]
  kSecUCut = 1,       // float[total_nodes]
  kSecU = 2,          // float[total_nodes]
  kSecSorted = 3,     // float4[n]
  kSecPerm = 4,       // int[n]
  kSecShort = 5,      // float4[n]
  kSecStatus,         // int[kStatusWords]
  kSecCounts,         // int[n_cells + 1]
  kSecCellStart,      // int[n_cells + 1]
  kSecCursor,         // int[n_cells]
  kSecCellOf,         // int[n]
  kSecTmp,            // int[n]
  kSecBinHist,        // int[bin_blocks * n_cells]: per-block cell counts (two-kernel binning)
  kSecScan,           // int[scan tiles]: cell counts per tile of the four-kernel binning's scan
  kSecAntPart,        // int64[anterpolation tiles * at_ext]: fixed-point private regions of the tiles
  kSecRows,           // StencilRow[n_rows]
  kSecWeights,        // float[n_weights]
  kSecRowsC,          // int4[n_rows]: compact rows (nz, ny >= 0, xr, weight offset)
  kSecWeightsC,       // float[n_wc]: W(nx, ny, |nz|) for nx = 0..xr per compact row
  kSecTop,            // double[top table]
  kSecPartials,       // double[10 * n_partials]: energy, then 9 virial components
  kSecLatPart,        // double[]: row-group partials of the lattice cutoff
  kSecDesc,           // SysDesc: this workspace's descriptor (pointers into it)
  kSecCount
};

struct Layout {
  size_t off[kSecCount];
  size_t bytes[kSecCount];
  size_t total;
};

// Device code sees the workspace pointers in the global address space, so
// every access through them is a global (not a flat) memory operation: flat
// operations also count as LDS operations, and a kernel waiting for an LDS
// result would wait for every flat load in flight.  The layout is the same.
#if defined(__HIP_DEVICE_COMPILE__)
#define MSM_GLOBAL __attribute__((address_space(1)))
#else
#define MSM_GLOBAL
#endif

struct DevPtrs {
  MSM_GLOBAL float* qgrid;
  MSM_GLOBAL float* ucut;
  MSM_GLOBAL float* u;
  MSM_GLOBAL float4* sorted;
  MSM_GLOBAL int* perm;
  MSM_GLOBAL float4* fshort;
  MSM_GLOBAL int* status;
  MSM_GLOBAL int* counts;
  MSM_GLOBAL int* cell_start;
  MSM_GLOBAL int* cursor;
  MSM_GLOBAL int* cell_of;
  MSM_GLOBAL int* tmp;
  MSM_GLOBAL int* bin_hist;
  MSM_GLOBAL int* scan;
  MSM_GLOBAL long long* ant_part;
  MSM_GLOBAL const StencilRow* rows;
  MSM_GLOBAL const int4* rows_c;
  MSM_GLOBAL const float* weights_c;
  MSM_GLOBAL const float* weights;
  MSM_GLOBAL const double* top;
  MSM_GLOBAL double* partials;
  MSM_GLOBAL double* lat_part;
  // bonded exclusions (caller's arrays, null: none): partners of the atom with
  // global input index g are excl_idx[excl_start[g] .. excl_start[g + 1])
  MSM_GLOBAL const int* excl_start;
  MSM_GLOBAL const int* excl_idx;
  long long excl_nnz;
};

// Stages of one evaluation, in launch order (for optional event timing).
enum Stage : int {
  kStageBin = 0, kStageShort, kStageAnterp, kStageRestrict, kStageLattice, kStageTop,
  kStageProlong, kStageInterp, kStageReduce, kStageCount
};
// Live timing slots: the stages, the second short-range launch (when its work
// is split) and the level-0 lattice cutoff on its side stream.
enum LiveSlot : int { kSlotShort2 = kStageCount, kSlotLattice0, kLiveSlots };
constexpr int kProfileEvents = 2 * kLiveSlots;   // enough for either timing mode

// Everything one system's kernels read, resident in device memory (one entry
// per system of a batch; a plain plan has one).
struct alignas(16) SysDesc {
  Geom g;
  DevPtrs d;
  LatLaunch lat;
  int atom_off;        // first atom of this system in the caller's arrays
  int index;           // slot of this system's energy, virial (x9) and gradient scale
  int n_partials;      // float64 partial slots (= interpolation blocks)
  int n_rows;          // full stencil rows (untiled lattice kernel)
};

// Caller buffers of one evaluation (kernel arguments): base pointers; a
// system's atoms start at atom_off and its scalars sit at index.
struct Io {
  const float* x;
  const float* y;
  const float* z;
  const float* q;
  float* fx;
  float* fy;
  float* fz;
  float* phi;
  double* energy;
  double* virial;
  const double* gscale;
};

// Kernel arguments shared by every stage: the descriptors, an optional
// block -> (system, block of that system) table for batched launches, and
// the caller's buffers.
struct KArgs {
  const SysDesc* sys;
  const int2* map;
  Io io;
};

// The dispatcher hands workgroups to the kXcds dies in turn (workgroup b to
// die b mod kXcds).  Numbering the logical blocks so that each die runs one
// contiguous range of them keeps neighbouring tiles, which read the same atoms
// and grid nodes, behind one L2 instead of fetching every input into all
// eight.  A bijection of [0, n) for any n.
__host__ __device__ inline int xcd_block(int b, int n) {
  const int x = b % kXcds, i = b / kXcds, per = n / kXcds, rem = n % kXcds;
  return x * per + (x < rem ? x : rem) + i;
}

// remap false keeps the dispatcher's round-robin over the dies: for launches
// whose blocks differ in cost (the lattice cutoff holds every level's tiles
// and the top-level blocks), contiguous ranges per die would load the dies
// unevenly.
__device__ inline const SysDesc& sys_of(const KArgs& a, int& blk, bool remap = true) {
  const int b = remap ? xcd_block((int)blockIdx.x, (int)gridDim.x) : (int)blockIdx.x;
  if (a.map) {
    const int2 m = a.map[b];
    blk = m.y;
    return a.sys[m.x];
  }
  blk = b;
  return a.sys[0];
}

// Host view of one launch sequence: block counts per stage (summed over the
// systems of a batch) and the matching block tables (null for one system).
struct StageGrid {
  int blocks = 0;
  const int2* map = nullptr;
};

struct LaunchGeom {
  const SysDesc* sys = nullptr;      // device array of n_sys descriptors
  int n_sys = 1;
  int order = 4;                     // common to every system of a launch
  int m = 2;
  int pair = kPairMsm;               // pair method (common to every system of a launch)
  int lat_b = 0;                     // windowed lattice outputs per lane, 0 = untiled kernel
  int lat_waves = kLatWavesMany;     // waves per windowed lattice block
  int lat_lds = 0;                   // dynamic LDS of the windowed kernel
  int max_levels = 1;
  int streams = 3;                   // 1: in order; 2: short range on a side stream; 3: also level-0 lattice
  int short_after = 1;               // side-stream short range starts after 1: binning, 2: anterpolation,
                                     // 3: the coarse lattice cutoff
  int short_split = 1000;            // per mille of its work items started there (the rest after the
                                     // lattice cutoff)
  StageGrid zero, atoms, one, shortr, anterp, top, energy;
  StageGrid scan;                    // tiles of the four-kernel binning's cell-count scan
  StageGrid agather;                 // level-0 nodes (gather of the anterpolation partials)
  int anterp_lds = 0;                // dynamic LDS of the anterpolation (largest system)
  bool prolong_split = false;        // one prolongation launch per level (one large system)
  int prolong_level[kMaxLevels] = {};   // prolongation tiles of each level below the top
  StageGrid bin;                     // two-kernel binning (systems with bin_blocks > 0)
  StageGrid binrow;                  // one-kernel binning (systems with bin_row_blocks > 0)
  StageGrid rchunk;                  // row binning: count and scatter (systems with binr_blocks > 0)
  StageGrid rscan;                   // row binning: one block per system
  StageGrid rsort;                   // row binning: one block per cell row
  int rsort_lds = 0;                 // dynamic LDS of the row binning's sort (largest system)
  bool periodic = false;             // periodic grids: ghost folds and fills between the stages
  bool short_periodic = false;       // periodic short range (MSM or pair plans)
  int ghost_blocks[kMaxLevels] = {}; // blocks of a ghost fill of each level (one system)
  int binrow_lds = 0;                // dynamic LDS of the one-kernel binning (largest system)
  bool bin4 = true;                  // some system uses the four-kernel binning
  StageGrid lattice0;                // lattice cutoff of level 0
  StageGrid lattice;                 // lattice cutoff of levels 1 .. l-2 (with the top level)
  StageGrid lattice_all;             // every level in one launch (no level-0 side stream)
  StageGrid restrict_[kMaxLevels];   // level k -> k+1
  StageGrid prolong;                 // every level k+1 -> k, one launch
};

// Per-stage block counts of one system.
struct SysBlocks {
  int zero, atoms, bin, binrow, shortr, anterp, lattice0, lattice, lattice_all, top, energy, scan;
  int agather;
  int rchunk, rscan, rsort;          // row binning
  int restrict_[kMaxLevels];
  int prolong;                       // tiles of every level below the top
};
SysBlocks system_blocks(const Geom& g, const LatLaunch& lat, int n_partials);
int prolong_level_blocks(const Geom& g, int k);   // prolongation tiles of level k

// Dynamic LDS of the one-kernel binning for one system: per-wave counts of the
// cells a block owns, scan scratch, and a 16-bit list entry per atom.
inline int bin_rows_lds(const Geom& g) {
  if (g.bin_row_blocks == 0) return 0;
  const int rows = g.nc[1] * g.nc[2];
  const int own = (rows + g.bin_row_blocks - 1) / g.bin_row_blocks * g.nc[0];
  const int chunks = (g.n_atoms + 63) / 64;
  return 16 * own * 4 + 2 * 16 * 4 + chunks * 64 * 2;
}

// Dynamic LDS of the row binning's sort for one system: x-cell starts and
// cursors, then (for rows of at most kBinRSortCap atoms) the row's atoms,
// input indices and x cells in bucket order.
inline int binr_sort_lds(const Geom& g) {
  if (g.binr_blocks == 0) return 0;
  const int ints = (2 * (g.nc[0] + 1) + 3) & ~3;
  return ints * 4 + kBinRSortCap * (16 + 4 + 2);
}

// Dynamic LDS of the anterpolation of one system: its tile's private region
// as 64-bit fixed-point accumulators.
inline int anterp_lds(const Geom& g) { return g.at_ext * 8; }

// What one evaluation produces.
enum Mode : int {
  kModeForces = 0,     // forces, potentials, energy, virial
  kModeEnergy = 1,     // energy only (grid form; no prolongation or interpolation)
  kModeGradient = 2    // gscale * dE/dr into fx..fz, gscale * dE/dq into phi
};

// A side stream with the events that fork work onto it and join it back.
struct SideStream {
  hipStream_t stream = nullptr;
  hipEvent_t fork = nullptr;
  hipEvent_t join = nullptr;
};

// Side streams of one evaluation: the short-range pass, and the level-0
// lattice cutoff (which needs only the anterpolated charges, so it overlaps
// the restriction chain, the coarse lattice levels, the top level and the
// coarse prolongations).
struct Concurrency {
  SideStream shortr;
  SideStream lattice0;
};

// Enqueues one evaluation (of every system of L) on `s` and returns the first
// HIP error.  cc (nullable): side streams for the concurrent branches, each
// joined back before its result is needed.  ev (nullable): timing events.
// With live false, kStageCount + 1 events recorded at the stage boundaries,
// and the evaluation runs in order on `s`; with live true, the schedule is
// kept and ev[slot] / ev[kLiveSlots + slot] bracket the launches of each
// LiveSlot on the stream they run on.
hipError_t launch_eval(int mode, const LaunchGeom& L, hipStream_t s, const Io& io, hipEvent_t* ev,
                       const Concurrency* cc, bool live = false);

int interp_partials(const Geom& g);      // number of FP64 partial slots the forward pass uses

// Workspace initialisation on the device (clears the cell counters).
hipError_t launch_init(const LaunchGeom& L, hipStream_t s);

}  // namespace msm
