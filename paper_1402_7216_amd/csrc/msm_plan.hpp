// Host-side state of libmsm shared by the single-system API (msm_api.hip) and
// the batch API (msm_batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <set>
#include <string>
#include <vector>

#include "msm_internal.hpp"

using msm::Geom;
using msm::Layout;

// Side streams and fork/join events of the concurrent branches of an evaluation.
struct AuxStreams {
  msm::Concurrency cc;
  int device = -1;
};

struct msm_plan {
  msm_params p;
  msm_pair_params pp{};                      // parameters of a pair-method plan (g.pair != 0)
  Geom g;
  std::vector<msm::StencilRow> rows;         // full stencil rows (untiled lattice kernel)
  std::vector<int4> rows_c;                  // compact rows of the windowed kernel
  std::vector<float> weights_c;              // compact weights of the windowed kernel
  std::vector<float> weights;                // full stencil weights
  std::vector<double> top;                   // FP64 top-level kernel table
  int n_partials = 1;
  int bin2_blocks = 0;                       // blocks of the two-kernel binning where it is possible
  bool prefer_bin2 = false;                  // two-kernel binning over one kernel where both work (batches)
  int lat_waves = 0;                         // waves per lattice block: 0 by the level-0 tiles (batches: 16)
  int max_cells = 0;                         // link cells of the finest cell reach (sizes the cell sections)
  long long max_bin_hist = 0;                // two-kernel histogram entries of any cell reach
  msm::LatLaunch lat;
  int lat_tables = 0;                        // LDS bytes of the compact stencil tables
  int lat_part_max = 0;                      // lattice row-group partials of the largest tuning
  int short_cap = 0;                         // short-range blocks (0: one per work item)
  int streams = 3;                           // stream layout of an evaluation (msm_tuning.streams)
  int short_after = 1;                       // start of the side-stream short range (msm_tuning.short_after)
  int short_split = 1000;                    // per mille of it started there (msm_tuning.short_split)
  uint64_t tune_gen = 0;                     // bumped by every tuning change (graphs record it)
  uint64_t uid = 0;                          // unique over the process (never reused)
  const int32_t* excl_start = nullptr;       // bonded exclusions (device arrays of the caller)
  const int32_t* excl_idx = nullptr;
  int64_t excl_nnz = 0;
  Layout lay;
  msm::SysDesc desc;                         // host copy; device pointers filled per workspace
  msm::LaunchGeom lg;                        // stage grids of one evaluation (descriptor set per call)
  std::set<const void*> ready;               // workspaces initialised for this plan
  // optional stage timing (diagnostics); mutable state of an otherwise fixed plan
  int profile = 0;                           // 0 off, 1 stages in order, 2 live schedule
  bool profiled = false;                     // an evaluation was timed since profiling was enabled
  hipEvent_t ev[msm::kProfileEvents] = {};
  AuxStreams aux;
};

// A captured evaluation.  Its launch grids, kernel templates and LDS sizes are
// those of the tuning in effect at capture; `owner_gen` points at the tuning
// generation of the plan or batch it was captured from, and a replay after a
// tuning change is refused.
struct msm_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const uint64_t* owner_gen = nullptr;
  uint64_t gen = 0;
};

msm_status fail(msm_status s, const std::string& msg);
msm_status hip_fail(hipError_t e, const char* what);
hipError_t ensure_aux(AuxStreams& a);
void destroy_aux(AuxStreams& a);

// Upload a plan's tables and descriptor into workspace ws and clear its cell
// counters (stream s; synchronises).
msm_status init_workspace(const msm_plan* P, void* ws, hipStream_t s);
// Device pointers of a workspace's sections.
msm::DevPtrs dev_ptrs(const msm_plan* P, void* ws);
// Device flags of the last evaluation of plan P in workspace ws: status word 0
// ORed with the words of the one-kernel binning's blocks (synchronous copy).
hipError_t read_flags(const msm_plan* P, const char* ws, int32_t* flags);
// Recompute the host descriptor and stage grids after a tuning change.
void refresh_launch(msm_plan* P);
// Link cells of reach 2, 3 or 4 (edge a / reach along y and z), with the
// short-range rows, work items and binning path they imply.
void set_cell_geometry(msm_plan* P, int reach);
int default_reach(int n_atoms);

// Number of systems and total atom count of a batch (the concatenated arrays'
// length).
msm_status batch_shape(const msm_batch* B, int32_t* n_sys, int32_t* total_atoms);
// Apply tuning knobs (zero fields keep the current value).  Host-side only;
// the caller re-uploads descriptors.
void retune(msm_plan* P, const msm_tuning& t);
// Waves per windowed lattice block for every later tile choice (0: by the
// level-0 tile count); re-chooses the current tiles.  Host-side only.
void set_lattice_waves(msm_plan* P, int waves);
// Reject knob values outside their documented ranges.
msm_status check_tuning(const msm_tuning* t);
// Capture the work `launch` enqueues on a private stream into an instantiated graph.
template <class F>
msm_status capture_graph(F launch, const uint64_t* owner_gen, msm_graph** out) {
  *out = nullptr;
  msm_graph* G = new (std::nothrow) msm_graph();
  if (!G) return fail(MSM_ERR_INVALID_ARG, "out of host memory");
  G->owner_gen = owner_gen;
  G->gen = *owner_gen;
  hipStream_t cs = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
  if (e != hipSuccess) {
    delete G;
    return hip_fail(e, "create capture stream");
  }
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    hipError_t le = launch(cs);
    e = hipStreamEndCapture(cs, &G->graph);
    if (le != hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&G->exec, G->graph, nullptr, nullptr, 0);
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess) {
    if (G->exec) (void)hipGraphExecDestroy(G->exec);
    if (G->graph) (void)hipGraphDestroy(G->graph);
    delete G;
    return hip_fail(e, "capture evaluation graph");
  }
  *out = G;
  return MSM_OK;
}
