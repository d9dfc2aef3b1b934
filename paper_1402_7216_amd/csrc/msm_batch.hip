// Batches of independent systems (replicas of uneven size) evaluated together:
// every stage is one launch whose blocks cover all systems, mapped through a
// per-stage block -> (system, block) table, so a batch costs the same number
// of launches as one evaluation.  Also the tuning knobs and the autotuner of
// plans and batches.
#include <hip/hip_runtime.h>

#include <unistd.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <set>
#include <sstream>
#include <string>
#include <vector>

#include "msm_plan.hpp"

namespace {

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

constexpr int kNumStages = 18 + msm::kMaxLevels;

}  // namespace

struct msm_batch {
  int n_sys = 0;
  std::vector<msm_plan*> plans;
  std::vector<int32_t> n_atoms;
  std::vector<int32_t> atom_off;
  int64_t total_atoms = 0;
  // workspace layout
  std::vector<size_t> sub_off;
  size_t desc_off = 0;
  size_t map_off[kNumStages] = {};
  size_t map_cap[kNumStages] = {};        // capacity in int2 entries
  size_t total = 0;
  // current stage tables (host)
  std::vector<int2> map[kNumStages];
  msm::LaunchGeom lg;                      // pointers set per workspace
  std::set<const void*> ready;
  uint64_t tune_gen = 0;                   // bumped by every tuning change (graphs record it)
  AuxStreams aux;
};

namespace {

// Stage order inside the map arrays.
enum : int {
  kMZero = 0, kMAtoms, kMBin, kMOne, kMShort, kMAnterp, kMLattice0, kMLattice, kMLatticeAll, kMTop, kMEnergy,
  kMProlong, kMBinRow, kMScan, kMAGather, kMRChunk, kMRScan, kMRSort,
  kMRestrict0
};

msm::StageGrid* stage_of(msm::LaunchGeom& L, int st) {
  switch (st) {
    case kMZero: return &L.zero;
    case kMAtoms: return &L.atoms;
    case kMBin: return &L.bin;
    case kMOne: return &L.one;
    case kMShort: return &L.shortr;
    case kMAnterp: return &L.anterp;
    case kMLattice0: return &L.lattice0;
    case kMLattice: return &L.lattice;
    case kMLatticeAll: return &L.lattice_all;
    case kMTop: return &L.top;
    case kMEnergy: return &L.energy;
    case kMProlong: return &L.prolong;
    case kMBinRow: return &L.binrow;
    case kMScan: return &L.scan;
    case kMAGather: return &L.agather;
    case kMRChunk: return &L.rchunk;
    case kMRScan: return &L.rscan;
    case kMRSort: return &L.rsort;
    default: return &L.restrict_[st - kMRestrict0];
  }
}

int blocks_of(const msm::SysBlocks& b, int st) {
  switch (st) {
    case kMZero: return b.zero;
    case kMAtoms: return b.atoms;
    case kMBin: return b.bin;
    case kMOne: return 1;
    case kMShort: return b.shortr;
    case kMAnterp: return b.anterp;
    case kMLattice0: return b.lattice0;
    case kMLattice: return b.lattice;
    case kMLatticeAll: return b.lattice_all;
    case kMTop: return b.top;
    case kMEnergy: return b.energy;
    case kMProlong: return b.prolong;
    case kMBinRow: return b.binrow;
    case kMScan: return b.scan;
    case kMAGather: return b.agather;
    case kMRChunk: return b.rchunk;
    case kMRScan: return b.rscan;
    case kMRSort: return b.rsort;
    default: return b.restrict_[st - kMRestrict0];
  }
}

// Rebuild the host stage tables and the launch geometry from the sub-plans.
void rebuild_maps(msm_batch* Bt) {
  msm::LaunchGeom& L = Bt->lg;
  L = msm::LaunchGeom{};
  L.n_sys = Bt->n_sys;
  L.order = Bt->plans[0]->g.order;
  L.m = Bt->plans[0]->g.m;
  L.streams = Bt->plans[0]->streams;
  L.short_after = Bt->plans[0]->short_after;
  L.short_split = Bt->plans[0]->short_split;
  L.lat_b = 0;
  L.bin4 = false;
  for (int st = 0; st < kNumStages; ++st) Bt->map[st].clear();
  for (int s = 0; s < Bt->n_sys; ++s) {
    const msm_plan* P = Bt->plans[s];
    if (P->g.bin_blocks == 0 && P->g.bin_row_blocks == 0 && P->g.binr_blocks == 0) L.bin4 = true;
    L.binrow_lds = std::max(L.binrow_lds, msm::bin_rows_lds(P->g));
    L.rsort_lds = std::max(L.rsort_lds, msm::binr_sort_lds(P->g));
    L.anterp_lds = std::max(L.anterp_lds, msm::anterp_lds(P->g));
    L.max_levels = std::max(L.max_levels, P->g.levels);
    L.lat_b = std::max(L.lat_b, P->lat.b);
    L.lat_waves = P->lat.b ? P->lat.waves : L.lat_waves;
    L.lat_lds = std::max(L.lat_lds, P->lat.lds_bytes);
    const msm::SysBlocks sb = msm::system_blocks(P->g, P->lat, P->n_partials);
    for (int st = 0; st < kNumStages; ++st) {
      const int nb = blocks_of(sb, st);
      for (int b = 0; b < nb; ++b) Bt->map[st].push_back(make_int2(s, b));
    }
  }
  for (int st = 0; st < kNumStages; ++st) stage_of(L, st)->blocks = (int)Bt->map[st].size();
}

void point_into(msm_batch* Bt, void* ws, msm::LaunchGeom& L) {
  char* base = static_cast<char*>(ws);
  L.sys = reinterpret_cast<const msm::SysDesc*>(base + Bt->desc_off);
  for (int st = 0; st < kNumStages; ++st)
    stage_of(L, st)->map = reinterpret_cast<const int2*>(base + Bt->map_off[st]);
}

// Upload the descriptor array and the stage tables of the current tuning.
msm_status upload_tables(msm_batch* Bt, void* ws, hipStream_t s) {
  char* base = static_cast<char*>(ws);
  std::vector<msm::SysDesc> descs(Bt->n_sys);
  for (int i = 0; i < Bt->n_sys; ++i) {
    msm_plan* P = Bt->plans[i];
    P->desc.d = dev_ptrs(P, base + Bt->sub_off[i]);
    descs[i] = P->desc;
    descs[i].atom_off = Bt->atom_off[i];
    descs[i].index = i;
  }
  hipError_t e = hipMemcpyAsync(base + Bt->desc_off, descs.data(), descs.size() * sizeof(msm::SysDesc),
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "upload batch descriptors");
  for (int st = 0; st < kNumStages; ++st) {
    if (Bt->map[st].size() > Bt->map_cap[st]) return fail(MSM_ERR_WORKSPACE, "stage table exceeds its reserve");
    if (Bt->map[st].empty()) continue;
    e = hipMemcpyAsync(base + Bt->map_off[st], Bt->map[st].data(), Bt->map[st].size() * sizeof(int2),
                       hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "upload stage tables");
  }
  e = hipStreamSynchronize(s);   // host vectors are staged before returning
  if (e != hipSuccess) return hip_fail(e, "upload batch tables");
  return MSM_OK;
}

msm_status check_batch(const msm_batch* Bt, const void* ws, size_t ws_bytes) {
  if (!Bt) return fail(MSM_ERR_INVALID_ARG, "null batch");
  if (!ws || ws_bytes < Bt->total) return fail(MSM_ERR_WORKSPACE, "workspace missing or too small");
  if (!Bt->ready.count(ws)) return fail(MSM_ERR_WORKSPACE, "workspace not initialised for this batch");
  return MSM_OK;
}

}  // namespace

msm_status batch_shape(const msm_batch* B, int32_t* n_sys, int32_t* total_atoms) {
  if (!B || !n_sys || !total_atoms) return fail(MSM_ERR_INVALID_ARG, "null batch or output");
  *n_sys = B->n_sys;
  *total_atoms = (int32_t)B->total_atoms;
  return MSM_OK;
}

extern "C" {

msm_status msm_batch_destroy(msm_batch* Bt) {
  if (Bt) {
    for (msm_plan* P : Bt->plans) msm_plan_destroy(P);
    destroy_aux(Bt->aux);
    delete Bt;
  }
  return MSM_OK;
}

msm_status msm_batch_create(const msm_params* params, const int32_t* n_atoms, int32_t n_sys,
                            msm_batch** out) {
  if (!out) return fail(MSM_ERR_INVALID_ARG, "null output pointer");
  *out = nullptr;
  if (!params || !n_atoms || n_sys < 1) return fail(MSM_ERR_INVALID_ARG, "empty batch or null arrays");
  msm_batch* Bt = new (std::nothrow) msm_batch();
  if (!Bt) return fail(MSM_ERR_INVALID_ARG, "out of host memory");
  Bt->n_sys = n_sys;
  int64_t off = 0;
  for (int s = 0; s < n_sys; ++s) {
    if (params[s].periodic) {
      msm_batch_destroy(Bt);
      return fail(MSM_ERR_UNSUPPORTED, "batches take free-space systems only");
    }
    msm_plan* P = nullptr;
    msm_status st = msm_plan_create(&params[s], n_atoms[s], &P);
    if (st != MSM_OK) {
      msm_batch_destroy(Bt);
      return st;
    }
    Bt->plans.push_back(P);
    Bt->n_atoms.push_back(n_atoms[s]);
    Bt->atom_off.push_back((int32_t)off);
    off += n_atoms[s];
    if (off > (int64_t)1 << 31) {
      msm_batch_destroy(Bt);
      return fail(MSM_ERR_UNSUPPORTED, "batch exceeds 2^31 atoms");
    }
  }
  Bt->total_atoms = off;
  // with several systems the two-kernel binning wins on throughput: the
  // one-kernel binning walks all of a system's atoms in every block, which
  // pays for a single system's latency but not when many systems fill the GPU
  if (n_sys > 1)
    for (msm_plan* P : Bt->plans) {
      P->prefer_bin2 = true;
      set_cell_geometry(P, P->g.reach);
      refresh_launch(P);
    }
  // one lattice launch serves every system, so they share its block size:
  // the smaller blocks only when every system's grid takes them on its own
  // (a batch of one system computes as its plan does)
  bool few = true;
  for (const msm_plan* P : Bt->plans) few = few && (P->lat.b == 0 || P->lat.waves == msm::kLatWavesFew);
  for (msm_plan* P : Bt->plans) set_lattice_waves(P, few ? msm::kLatWavesFew : msm::kLatWavesMany);
  const msm_plan* P0 = Bt->plans[0];
  bool tiled = P0->lat.b > 0 || P0->g.levels == 1;
  for (const msm_plan* P : Bt->plans) {
    if (P->g.pair) {
      msm_batch_destroy(Bt);
      return fail(MSM_ERR_UNSUPPORTED, "batches hold multilevel-summation systems only");
    }
    if (P->g.order != P0->g.order || P->g.m != P0->g.m) {
      msm_batch_destroy(Bt);
      return fail(MSM_ERR_UNSUPPORTED, "systems of a batch must share order and split_m");
    }
    const bool t = P->lat.b > 0 || P->g.levels == 1;
    if (t != tiled) {
      msm_batch_destroy(Bt);
      return fail(MSM_ERR_UNSUPPORTED, "mixed stencil widths in one batch");
    }
  }
  // common lattice template: the largest system's choice
  int big = 0;
  for (int s = 1; s < n_sys; ++s)
    if (n_atoms[s] > n_atoms[big]) big = s;
  const int b0 = Bt->plans[big]->lat.b;
  for (msm_plan* P : Bt->plans) retune(P, msm_tuning{b0, 0, 0, 0, 0, 0, 0, 0});

  // stage-table reserves: the most blocks any tuning can ask for
  // (lattice template 4, one cell per short-range work item)
  size_t cap[kNumStages] = {};
  for (msm_plan* P : Bt->plans) {
    const Geom keep_g = P->g;
    const msm::LatLaunch keep_l = P->lat;
    const int keep_cap = P->short_cap, keep_bin2 = P->bin2_blocks;
    size_t most[kNumStages] = {};
    for (int r : {2, 3, 4})
      for (int b : {4, 6, 8})
        for (int w : {1, keep_g.item_chunks}) {
          // one short-range block per item: the most
          retune(P, msm_tuning{P->lat.b ? b : 0, w, -1, 0, 0, 0, r, 0});
          const msm::SysBlocks sb = msm::system_blocks(P->g, P->lat, P->n_partials);
          for (int st = 0; st < kNumStages; ++st) most[st] = std::max(most[st], (size_t)blocks_of(sb, st));
        }
    P->g = keep_g;
    P->lat = keep_l;
    P->short_cap = keep_cap;
    P->bin2_blocks = keep_bin2;
    refresh_launch(P);
    for (int st = 0; st < kNumStages; ++st) cap[st] += most[st];
  }
  size_t o = 0;
  for (msm_plan* P : Bt->plans) {
    Bt->sub_off.push_back(o);
    o += align256(P->lay.total);
  }
  Bt->desc_off = o;
  o += align256(n_sys * sizeof(msm::SysDesc));
  for (int st = 0; st < kNumStages; ++st) {
    Bt->map_off[st] = o;
    Bt->map_cap[st] = cap[st];
    o += align256(std::max<size_t>(cap[st], 1) * sizeof(int2));
  }
  Bt->total = o;
  rebuild_maps(Bt);
  *out = Bt;
  return MSM_OK;
}

msm_status msm_batch_workspace_bytes(const msm_batch* Bt, size_t* bytes) {
  if (!Bt || !bytes) return fail(MSM_ERR_INVALID_ARG, "null batch or bytes pointer");
  *bytes = Bt->total;
  return MSM_OK;
}

msm_status msm_batch_atom_offsets(const msm_batch* Bt, int32_t* offsets) {
  if (!Bt || !offsets) return fail(MSM_ERR_INVALID_ARG, "null batch or offsets");
  for (int s = 0; s < Bt->n_sys; ++s) offsets[s] = Bt->atom_off[s];
  offsets[Bt->n_sys] = (int32_t)Bt->total_atoms;
  return MSM_OK;
}

msm_status msm_batch_workspace_init(const msm_batch* Bt, void* ws, size_t ws_bytes, msm_stream_t stream) {
  if (!Bt) return fail(MSM_ERR_INVALID_ARG, "null batch");
  if (!ws || ws_bytes < Bt->total) return fail(MSM_ERR_WORKSPACE, "workspace missing or too small");
  char* base = static_cast<char*>(ws);
  for (int s = 0; s < Bt->n_sys; ++s) {
    const msm_plan* P = Bt->plans[s];
    msm_status st = msm_workspace_init(P, base + Bt->sub_off[s], P->lay.total, stream);
    if (st != MSM_OK) return st;
  }
  msm_batch* M = const_cast<msm_batch*>(Bt);
  msm_status st = upload_tables(M, ws, reinterpret_cast<hipStream_t>(stream));
  if (st != MSM_OK) return st;
  M->ready.insert(ws);
  return MSM_OK;
}

static msm_status batch_eval(int mode, const msm_batch* Bt, void* ws, size_t ws_bytes,
                             msm_stream_t stream, const msm::Io& io, msm_graph** graph) {
  msm_status st = check_batch(Bt, ws, ws_bytes);
  if (st != MSM_OK) return st;
  if (Bt->total_atoms > 0 && (!io.x || !io.y || !io.z || !io.q))
    return fail(MSM_ERR_INVALID_ARG, "null position or charge array");
  if (!((io.fx && io.fy && io.fz) || (!io.fx && !io.fy && !io.fz)))
    return fail(MSM_ERR_INVALID_ARG, "vector outputs must be all set or all null");
  msm_batch* M = const_cast<msm_batch*>(Bt);
  hipError_t e = ensure_aux(M->aux);
  if (e != hipSuccess) return hip_fail(e, "create auxiliary stream");
  msm::LaunchGeom L = Bt->lg;
  point_into(M, ws, L);
  if (graph)
    return capture_graph(
        [&](hipStream_t cs) {
          return msm::launch_eval(mode, L, cs, io, nullptr, &M->aux.cc);
        },
        &M->tune_gen, graph);
  e = msm::launch_eval(mode, L, reinterpret_cast<hipStream_t>(stream), io, nullptr, &M->aux.cc);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return MSM_OK;
}

msm_status msm_batch_compute(const msm_batch* Bt, void* ws, size_t ws_bytes, msm_stream_t stream,
                             const float* x, const float* y, const float* z, const float* q,
                             float* fx, float* fy, float* fz, float* phi, double* energy,
                             double* virial) {
  const msm::Io io{x, y, z, q, fx, fy, fz, phi, energy, virial, nullptr};
  return batch_eval(msm::kModeForces, Bt, ws, ws_bytes, stream, io, nullptr);
}

msm_status msm_batch_energy(const msm_batch* Bt, void* ws, size_t ws_bytes, msm_stream_t stream,
                            const float* x, const float* y, const float* z, const float* q,
                            double* energy) {
  if (!energy) return fail(MSM_ERR_INVALID_ARG, "null energy output");
  const msm::Io io{x, y, z, q, nullptr, nullptr, nullptr, nullptr, energy, nullptr, nullptr};
  return batch_eval(msm::kModeEnergy, Bt, ws, ws_bytes, stream, io, nullptr);
}

msm_status msm_batch_backward(const msm_batch* Bt, void* ws, size_t ws_bytes, msm_stream_t stream,
                              const float* x, const float* y, const float* z, const float* q,
                              const double* grad_energy, float* dedx, float* dedy, float* dedz,
                              float* dedq) {
  if (!grad_energy) return fail(MSM_ERR_INVALID_ARG, "null grad_energy");
  const msm::Io io{x, y, z, q, dedx, dedy, dedz, dedq, nullptr, nullptr, grad_energy};
  return batch_eval(msm::kModeGradient, Bt, ws, ws_bytes, stream, io, nullptr);
}

msm_status msm_batch_graph_capture(const msm_batch* Bt, void* ws, size_t ws_bytes, const float* x,
                                   const float* y, const float* z, const float* q, float* fx,
                                   float* fy, float* fz, float* phi, double* energy, double* virial,
                                   msm_graph** out) {
  if (!out) return fail(MSM_ERR_INVALID_ARG, "null output pointer");
  *out = nullptr;
  const msm::Io io{x, y, z, q, fx, fy, fz, phi, energy, virial, nullptr};
  return batch_eval(msm::kModeForces, Bt, ws, ws_bytes, nullptr, io, out);
}

msm_status msm_batch_status(const msm_batch* Bt, const void* ws, msm_stream_t stream,
                            int32_t* flags_per_system) {
  if (!Bt || !ws) return fail(MSM_ERR_INVALID_ARG, "null batch or workspace");
  hipError_t e = hipStreamSynchronize(reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "stream synchronize");
  int32_t all = 0;
  for (int s = 0; s < Bt->n_sys; ++s) {
    int32_t f = 0;
    const msm_plan* P = Bt->plans[s];
    const char* sub = static_cast<const char*>(ws) + Bt->sub_off[s];
    e = read_flags(P, sub, &f);
    if (e != hipSuccess) return hip_fail(e, "read status");
    if (flags_per_system) flags_per_system[s] = f;
    all |= f;
  }
  if (all & msm::kFlagNonFinite) return fail(MSM_ERR_NONFINITE, "non-finite position or charge");
  if (all & msm::kFlagOutOfBox) return fail(MSM_ERR_OUT_OF_BOX, "atom outside the box");
  if (all & msm::kFlagCoincident) return fail(MSM_ERR_COINCIDENT, "coincident atoms");
  if (all & msm::kFlagBadExclusion) return fail(MSM_ERR_INVALID_ARG, "exclusion list entry out of range");
  return MSM_OK;
}

msm_status msm_batch_describe(const msm_batch* Bt, char* buf, size_t buf_bytes) {
  if (!Bt || !buf || buf_bytes == 0) return fail(MSM_ERR_INVALID_ARG, "null batch or buffer");
  const msm::LaunchGeom& L = Bt->lg;
  std::string o = "{\"systems\": " + std::to_string(Bt->n_sys) +
                  ", \"atoms\": " + std::to_string(Bt->total_atoms) +
                  ", \"max_levels\": " + std::to_string(L.max_levels) +
                  ", \"lattice_b\": " + std::to_string(L.lat_b) +
                  ", \"lattice_waves\": " + std::to_string(L.lat_waves) + ", \"lattice_lds\": " +
                  std::to_string(L.lat_lds) +
                  ", \"item_chunks\": " + std::to_string(Bt->plans[0]->g.item_chunks) +   // first system's
                  ", \"blocks\": {\"atoms\": " + std::to_string(L.atoms.blocks) +
                  ", \"short\": " + std::to_string(L.shortr.blocks) +
                  ", \"anterp\": " + std::to_string(L.anterp.blocks) +
                  ", \"lattice\": " + std::to_string(L.lattice_all.blocks) +
                  ", \"top\": " + std::to_string(L.top.blocks) + "}, \"levels\": [";
  for (int s = 0; s < Bt->n_sys; ++s) o += (s ? ", " : "") + std::to_string(Bt->plans[s]->g.levels);
  o += "], \"item_chunks_all\": [";
  for (int s = 0; s < Bt->n_sys; ++s) o += (s ? ", " : "") + std::to_string(Bt->plans[s]->g.item_chunks);
  o += "], \"workspace_bytes\": " + std::to_string(Bt->total) + "}";
  std::strncpy(buf, o.c_str(), buf_bytes - 1);
  buf[buf_bytes - 1] = 0;
  return o.size() < buf_bytes ? MSM_OK : fail(MSM_ERR_INVALID_ARG, "buffer too small");
}

// ---------------------------------------------------------------------------
// Tuning knobs and the autotuner
// ---------------------------------------------------------------------------

msm_status msm_plan_tuning(const msm_plan* P, msm_tuning* t) {
  if (!P || !t) return fail(MSM_ERR_INVALID_ARG, "null plan or tuning");
  *t = msm_tuning{P->lat.b, P->g.item_chunks, P->short_cap > 0 ? P->short_cap : -1, P->streams,
                  P->short_after, P->short_split, P->g.reach, 0};
  return MSM_OK;
}

msm_status msm_plan_tune(msm_plan* P, void* ws, size_t ws_bytes, msm_stream_t stream,
                         const msm_tuning* t) {
  if (!P) return fail(MSM_ERR_INVALID_ARG, "null plan");
  msm_status cs = check_tuning(t);
  if (cs != MSM_OK) return cs;
  if (!ws || ws_bytes < P->lay.total || !P->ready.count(ws))
    return fail(MSM_ERR_WORKSPACE, "workspace not initialised for this plan");
  retune(P, *t);
  ++P->tune_gen;
  P->desc.d = dev_ptrs(P, ws);
  // other workspaces now hold stale descriptors
  P->ready.clear();
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(static_cast<char*>(ws) + P->lay.off[msm::kSecDesc], &P->desc,
                                sizeof(msm::SysDesc), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "upload descriptor");
  P->ready.insert(ws);
  return MSM_OK;
}

static msm_status check_exclusions(const int32_t* start, const int32_t* idx, int64_t nnz) {
  if (nnz < 0 || nnz > INT32_MAX) return fail(MSM_ERR_INVALID_ARG, "nnz must be in 0 .. 2^31 - 1");
  if (start && nnz > 0 && !idx) return fail(MSM_ERR_INVALID_ARG, "null exclusion partner array");
  return MSM_OK;
}

msm_status msm_set_exclusions(msm_plan* P, void* ws, size_t ws_bytes, msm_stream_t stream, const int32_t* start,
                              const int32_t* idx, int64_t nnz) {
  if (!P) return fail(MSM_ERR_INVALID_ARG, "null plan");
  msm_status st = check_exclusions(start, idx, nnz);
  if (st != MSM_OK) return st;
  if (!ws || ws_bytes < P->lay.total || !P->ready.count(ws))
    return fail(MSM_ERR_WORKSPACE, "workspace not initialised for this plan");
  P->excl_start = start;
  P->excl_idx = start ? idx : nullptr;
  P->excl_nnz = start ? nnz : 0;
  ++P->tune_gen;                                   // graphs and the static workspace see a new plan state
  P->desc.d = dev_ptrs(P, ws);
  P->ready.clear();
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(static_cast<char*>(ws) + P->lay.off[msm::kSecDesc], &P->desc,
                                sizeof(msm::SysDesc), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "upload descriptor");
  P->ready.insert(ws);
  return MSM_OK;
}

msm_status msm_batch_set_exclusions(msm_batch* Bt, void* ws, size_t ws_bytes, msm_stream_t stream,
                                    const int32_t* start, const int32_t* idx, int64_t nnz) {
  msm_status st = check_batch(Bt, ws, ws_bytes);
  if (st != MSM_OK) return st;
  st = check_exclusions(start, idx, nnz);
  if (st != MSM_OK) return st;
  for (msm_plan* P : Bt->plans) {
    P->excl_start = start;
    P->excl_idx = start ? idx : nullptr;
    P->excl_nnz = start ? nnz : 0;
    ++P->tune_gen;
  }
  ++Bt->tune_gen;
  Bt->ready.clear();
  st = upload_tables(Bt, ws, reinterpret_cast<hipStream_t>(stream));
  if (st != MSM_OK) return st;
  Bt->ready.insert(ws);
  return MSM_OK;
}

msm_status msm_batch_tune(msm_batch* Bt, void* ws, size_t ws_bytes, msm_stream_t stream,
                          const msm_tuning* t) {
  msm_status st = check_batch(Bt, ws, ws_bytes);
  if (st != MSM_OK) return st;
  st = check_tuning(t);
  if (st != MSM_OK) return st;
  for (msm_plan* P : Bt->plans) retune(P, *t);
  ++Bt->tune_gen;
  rebuild_maps(Bt);
  Bt->ready.clear();
  st = upload_tables(Bt, ws, reinterpret_cast<hipStream_t>(stream));
  if (st != MSM_OK) return st;
  Bt->ready.insert(ws);
  return MSM_OK;
}

// Time candidates over `trials` evaluations of the given inputs with HIP
// events on `stream`: lattice_b in {4, 6, 8} x item_chunks in {1, 2, 3} x the
// two side-stream layouts with one short-range block per work item (at the
// current cell reach), then the cell reach (2, 3, 4), the stream layouts x
// short-range block counts for the best so far, where the side short range
// starts, the chunks again, and how much of the short range waits for the
// lattice cutoff.  Apply the fastest and describe the search in `report`
// (JSON, nullable).
static msm_status autotune(bool batch, void* obj, void* ws, size_t ws_bytes, msm_stream_t stream,
                           const float* x, const float* y, const float* z, const float* q,
                           int32_t trials, char* report, size_t report_bytes) {
  if (trials < 1) return fail(MSM_ERR_INVALID_ARG, "trials must be >= 1");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t he = hipEventCreate(&e0);
  if (he == hipSuccess) he = hipEventCreate(&e1);
  if (he != hipSuccess) return hip_fail(he, "create timing events");
  msm_batch* Bt = batch ? static_cast<msm_batch*>(obj) : nullptr;
  msm_plan* P = batch ? nullptr : static_cast<msm_plan*>(obj);
  const bool tiled = batch ? Bt->lg.lat_b > 0 : P->lat.b > 0;
  auto tune = [&](const msm_tuning& t) {
    return batch ? msm_batch_tune(Bt, ws, ws_bytes, stream, &t) : msm_plan_tune(P, ws, ws_bytes, stream, &t);
  };
  auto eval = [&]() {
    return batch ? msm_batch_compute(Bt, ws, ws_bytes, stream, x, y, z, q, nullptr, nullptr, nullptr, nullptr,
                                     nullptr, nullptr)
                 : msm_compute(P, ws, ws_bytes, stream, x, y, z, q, nullptr, nullptr, nullptr, nullptr,
                               nullptr, nullptr);
  };
  auto describe = [](const msm_tuning& t) {
    return "\"lattice_b\": " + std::to_string(t.lattice_b) + ", \"item_chunks\": " + std::to_string(t.item_chunks) +
           ", \"short_blocks\": " + std::to_string(t.short_blocks) + ", \"streams\": " +
           std::to_string(t.streams) + ", \"short_after\": " + std::to_string(t.short_after) +
           ", \"short_split\": " + std::to_string(t.short_split) + ", \"cell_reach\": " +
           std::to_string(t.cell_reach);
  };
  msm_tuning cur{};
  if (batch) {
    (void)msm_plan_tuning(Bt->plans[0], &cur);
  } else {
    (void)msm_plan_tuning(P, &cur);
  }
  std::string rep = "{\"candidates\": [";
  float best = 1e30f;
  msm_tuning bt{0, 0, 0, 0, 1, 1000, cur.cell_reach, 0};
  bool first = true;
  auto time_one = [&](const msm_tuning& t) {
    msm_status st = tune(t);
    // one warm-up evaluation, then `trials` timed ones
    for (int k = -1; k < trials && st == MSM_OK; ++k) {
      if (k == 0) (void)hipEventRecord(e0, s);
      st = eval();
    }
    if (st != MSM_OK) return st;
    (void)hipEventRecord(e1, s);
    float ms = 0.f;
    hipError_t r = hipEventSynchronize(e1);
    if (r == hipSuccess) r = hipEventElapsedTime(&ms, e0, e1);
    if (r != hipSuccess) return hip_fail(r, "time candidate");
    ms /= trials;
    rep += std::string(first ? "" : ", ") + "{" + describe(t) + ", \"ms\": " + std::to_string(ms) + "}";
    first = false;
    // a later (more elaborate) candidate must win by more than 1% (timing noise)
    if (ms < best * 0.99f) {
      best = ms;
      bt = t;
    }
    return MSM_OK;
  };
  msm_status st = MSM_OK;
  const std::vector<int> bs = tiled ? std::vector<int>{4, 6, 8} : std::vector<int>{0};
  // B x chunks under both side-stream layouts (the best chunk count depends
  // on the layout)
  for (int n : {3, 2})
    for (int b : bs)
      for (int w : {1, 2, 3})
        if (st == MSM_OK) st = time_one(msm_tuning{b, w, -1, n, 1, 1000, cur.cell_reach, 0});
  // cell reach for the best (B, chunks, layout)
  for (int r : {2, 3, 4})
    if (st == MSM_OK && r != bt.cell_reach) {
      msm_tuning t = bt;
      t.cell_reach = r;
      st = time_one(t);
    }
  // stream layouts x short-range block counts for the best so far; the counts
  // are fractions of the compute units, so the short-range pass leaves room
  // for the grid chain running beside it
  int n_cu = 256;
  {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      n_cu = prop.multiProcessorCount;
  }
  {
    const msm_tuning base = bt;
    for (int n : {1, 2, 3})
      for (int c : {-1, 3 * n_cu / 2, n_cu, 3 * n_cu / 4, n_cu / 2})
        if (st == MSM_OK && !(n == 3 && c == -1) && !(n == base.streams && c == base.short_blocks)) {
          msm_tuning t = base;
          t.streams = n;
          t.short_blocks = c;
          st = time_one(t);
        }
  }
  // where the side-stream short range starts, for the best layout so far
  if (bt.streams >= 2) {
    const msm_tuning base = bt;
    for (int sa : {2, 3})
      if (st == MSM_OK) {
        msm_tuning t = base;
        t.short_after = sa;
        st = time_one(t);
      }
  }
  // chunks per short-range item again, for the best layout and start (the
  // first pass chose them with every stream on)
  {
    const msm_tuning base = bt;
    for (int w : {1, 2, 3})
      if (st == MSM_OK && w != base.item_chunks) {
        msm_tuning t = base;
        t.item_chunks = w;
        st = time_one(t);
      }
  }
  // part of the short range after the lattice cutoff, for the best start
  if (bt.streams >= 2 && bt.short_after < 3) {
    const msm_tuning base = bt;
    for (int sp : {300, 500, 700})
      if (st == MSM_OK) {
        msm_tuning t = base;
        t.short_split = sp;
        st = time_one(t);
      }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != MSM_OK) return st;
  st = tune(bt);
  if (st != MSM_OK) return st;
  rep += "], \"best\": {" + describe(bt) + ", \"ms\": " + std::to_string(best) + "}}";
  if (report && report_bytes) {
    std::strncpy(report, rep.c_str(), report_bytes - 1);
    report[report_bytes - 1] = 0;
  }
  return MSM_OK;
}

// ---------------------------------------------------------------------------
// Tuning cache: one text line per key, "<key> lattice_b item_chunks
// short_blocks streams short_after short_split cell_reach"; '#' starts a
// comment line.  The key names what the best tuning depends on: the target,
// the interpolation order, the smoothing degree, the level-0 stencil taps and,
// rounded to half octaves, the level-0 node count and the atom count.
// ---------------------------------------------------------------------------
static int stencil_taps(double a, double h) {
  if (!(h > 0.0) || !(a > 0.0) || 2.0 * a / h > 1024.0) return 0;
  const double R = 2.0 * a / h;
  const int r = (int)std::floor(R);
  int n = 0;
  for (int i = -r; i <= r; ++i)
    for (int j = -r; j <= r; ++j)
      for (int k = -r; k <= r; ++k)
        if ((double)(i * i + j * j + k * k) < R * R) ++n;
  return n;
}

static int half_octave(double v) { return v > 0 ? (int)std::lround(2.0 * std::log2(v)) : -1; }

static msm_status write_key(const std::string& k, char* key, size_t key_bytes) {
  if (!key || key_bytes <= k.size()) return fail(MSM_ERR_INVALID_ARG, "key buffer missing or too small");
  std::memcpy(key, k.c_str(), k.size() + 1);
  return MSM_OK;
}

static std::string plan_key(const msm_plan* P) {
  char b[160];
  if (P->g.pair != msm::kPairMsm) {   // a cheap pair method: no grids
    std::snprintf(b, sizeof b, "gfx950/pair%d/a%ld/n%d", P->g.pair, std::lround(10.0 * P->p.cutoff),
                  half_octave(P->g.n_atoms));
    return b;
  }
  std::snprintf(b, sizeof b, "gfx950/o%d/m%d/S%d/g%d/n%d", P->g.order, P->g.m,
                stencil_taps(P->p.cutoff, P->p.spacing), half_octave(P->g.lv[0].count),
                half_octave(P->g.n_atoms));
  return b;
}

static std::string batch_key(const msm_batch* Bt) {
  int taps = 0;
  double nodes = 0;
  for (const msm_plan* P : Bt->plans) {
    taps = std::max(taps, stencil_taps(P->p.cutoff, P->p.spacing));
    nodes += P->g.lv[0].count;
  }
  const msm_plan* P0 = Bt->plans[0];
  char b[160];
  std::snprintf(b, sizeof b, "gfx950/batch%d/o%d/m%d/S%d/g%d/n%d", Bt->n_sys, P0->g.order, P0->g.m, taps,
                half_octave(nodes), half_octave((double)Bt->total_atoms));
  return b;
}

static bool valid_key(const char* key) {
  if (!key || !*key) return false;
  for (const char* c = key; *c; ++c)
    if (*c == ' ' || *c == '\t' || *c == '\n' || *c == '\r' || *c == '#') return false;
  return true;
}

static std::string tuning_fields(const msm_tuning& t) {
  return std::to_string(t.lattice_b) + " " + std::to_string(t.item_chunks) + " " + std::to_string(t.short_blocks) +
         " " + std::to_string(t.streams) + " " + std::to_string(t.short_after) + " " +
         std::to_string(t.short_split) + " " + std::to_string(t.cell_reach);
}

static std::string describe_tuning(const msm_tuning& t) {
  return "\"lattice_b\": " + std::to_string(t.lattice_b) + ", \"item_chunks\": " + std::to_string(t.item_chunks) +
         ", \"short_blocks\": " + std::to_string(t.short_blocks) + ", \"streams\": " +
         std::to_string(t.streams) + ", \"short_after\": " + std::to_string(t.short_after) +
         ", \"short_split\": " + std::to_string(t.short_split) + ", \"cell_reach\": " +
         std::to_string(t.cell_reach);
}

static void put_report(const std::string& rep, char* report, size_t report_bytes) {
  if (report && report_bytes) {
    std::strncpy(report, rep.c_str(), report_bytes - 1);
    report[report_bytes - 1] = 0;
  }
}

msm_status msm_plan_tuning_key(const msm_plan* P, char* key, size_t key_bytes) {
  if (!P) return fail(MSM_ERR_INVALID_ARG, "null plan");
  return write_key(plan_key(P), key, key_bytes);
}

msm_status msm_batch_tuning_key(const msm_batch* Bt, char* key, size_t key_bytes) {
  if (!Bt) return fail(MSM_ERR_INVALID_ARG, "null batch");
  return write_key(batch_key(Bt), key, key_bytes);
}

msm_status msm_tuning_cache_lookup(const char* path, const char* key, msm_tuning* tuning) {
  if (!path || !tuning || !valid_key(key)) return fail(MSM_ERR_INVALID_ARG, "null path or tuning, or bad key");
  std::ifstream f(path);
  if (!f) return fail(MSM_ERR_UNSUPPORTED, std::string("no tuning cache at ") + path);
  std::string line;
  while (std::getline(f, line)) {
    if (line.empty() || line[0] == '#') continue;
    std::istringstream in(line);
    std::string k;
    in >> k;
    if (k != key) continue;
    msm_tuning t{};
    in >> t.lattice_b >> t.item_chunks >> t.short_blocks >> t.streams >> t.short_after >> t.short_split >>
        t.cell_reach;
    std::string rest;
    if (in.fail() || (in >> rest)) return fail(MSM_ERR_INVALID_ARG, "malformed tuning cache entry: " + line);
    const msm_status st = check_tuning(&t);
    if (st != MSM_OK) return st;
    *tuning = t;
    return MSM_OK;
  }
  return fail(MSM_ERR_UNSUPPORTED, std::string("no entry for ") + key + " in " + path);
}

msm_status msm_tuning_cache_store(const char* path, const char* key, const msm_tuning* tuning) {
  if (!path || !valid_key(key)) return fail(MSM_ERR_INVALID_ARG, "null path or bad key");
  msm_status st = check_tuning(tuning);
  if (st != MSM_OK) return st;
  std::vector<std::string> lines;
  {
    std::ifstream f(path);
    std::string line;
    while (f && std::getline(f, line)) {
      std::istringstream in(line);
      std::string k;
      in >> k;
      if (line.empty() || line[0] == '#' || k != key) lines.push_back(line);
    }
  }
  lines.push_back(std::string(key) + " " + tuning_fields(*tuning));
  // written beside the file and renamed over it: readers see the old or the new file
  const std::string tmp = std::string(path) + ".tmp" + std::to_string((long)getpid());
  {
    std::ofstream o(tmp, std::ios::trunc);
    if (!o) return fail(MSM_ERR_INVALID_ARG, "cannot write " + tmp);
    for (const std::string& l : lines) o << l << "\n";
    o.flush();
    if (!o) return fail(MSM_ERR_INVALID_ARG, "cannot write " + tmp);
  }
  if (std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return fail(MSM_ERR_INVALID_ARG, std::string("cannot replace ") + path);
  }
  return MSM_OK;
}

// Autotune through the cache: a hit applies the stored tuning without timing
// anything; a miss runs the search and stores its result.
static msm_status autotune_cached(bool batch, void* obj, const std::string& key, void* ws, size_t ws_bytes,
                                  msm_stream_t stream, const float* x, const float* y, const float* z,
                                  const float* q, int32_t trials, const char* cache, char* report,
                                  size_t report_bytes) {
  msm_batch* Bt = batch ? static_cast<msm_batch*>(obj) : nullptr;
  msm_plan* P = batch ? nullptr : static_cast<msm_plan*>(obj);
  msm_tuning t{};
  const std::string hdr = "{\"key\": \"" + key + "\", ";
  if (cache && msm_tuning_cache_lookup(cache, key.c_str(), &t) == MSM_OK) {
    const msm_status st =
        batch ? msm_batch_tune(Bt, ws, ws_bytes, stream, &t) : msm_plan_tune(P, ws, ws_bytes, stream, &t);
    if (st != MSM_OK) return st;
    put_report(hdr + "\"cache\": \"hit\", \"best\": {" + describe_tuning(t) + "}}", report, report_bytes);
    return MSM_OK;
  }
  std::vector<char> inner(std::max<size_t>(report_bytes, 1), 0);
  msm_status st = autotune(batch, obj, ws, ws_bytes, stream, x, y, z, q, trials, inner.data(), inner.size());
  if (st != MSM_OK) return st;
  st = batch ? msm_plan_tuning(Bt->plans[0], &t) : msm_plan_tuning(P, &t);
  if (st != MSM_OK) return st;
  if (cache) {
    st = msm_tuning_cache_store(cache, key.c_str(), &t);
    if (st != MSM_OK) return st;
  }
  put_report(hdr + "\"cache\": \"" + (cache ? "miss" : "none") + "\", \"search\": " + std::string(inner.data()) +
                 "}",
             report, report_bytes);
  return MSM_OK;
}

msm_status msm_plan_autotune_cached(msm_plan* P, void* ws, size_t ws_bytes, msm_stream_t stream, const float* x,
                                    const float* y, const float* z, const float* q, int32_t trials,
                                    const char* cache, char* report, size_t report_bytes) {
  if (!P) return fail(MSM_ERR_INVALID_ARG, "null plan");
  if (trials < 1) return fail(MSM_ERR_INVALID_ARG, "trials must be >= 1");
  return autotune_cached(false, P, plan_key(P), ws, ws_bytes, stream, x, y, z, q, trials, cache, report,
                         report_bytes);
}

msm_status msm_batch_autotune_cached(msm_batch* Bt, void* ws, size_t ws_bytes, msm_stream_t stream,
                                     const float* x, const float* y, const float* z, const float* q,
                                     int32_t trials, const char* cache, char* report, size_t report_bytes) {
  msm_status st = check_batch(Bt, ws, ws_bytes);
  if (st != MSM_OK) return st;
  if (trials < 1) return fail(MSM_ERR_INVALID_ARG, "trials must be >= 1");
  return autotune_cached(true, Bt, batch_key(Bt), ws, ws_bytes, stream, x, y, z, q, trials, cache, report,
                         report_bytes);
}

msm_status msm_plan_autotune(msm_plan* P, void* ws, size_t ws_bytes, msm_stream_t stream,
                             const float* x, const float* y, const float* z, const float* q,
                             int32_t trials, char* report, size_t report_bytes) {
  if (!P) return fail(MSM_ERR_INVALID_ARG, "null plan");
  return autotune(false, P, ws, ws_bytes, stream, x, y, z, q, trials, report, report_bytes);
}

msm_status msm_batch_autotune(msm_batch* Bt, void* ws, size_t ws_bytes, msm_stream_t stream,
                              const float* x, const float* y, const float* z, const float* q,
                              int32_t trials, char* report, size_t report_bytes) {
  msm_status st = check_batch(Bt, ws, ws_bytes);
  if (st != MSM_OK) return st;
  return autotune(true, Bt, ws, ws_bytes, stream, x, y, z, q, trials, report, report_bytes);
}

}  // extern "C"
