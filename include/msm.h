/*
 * msm.h -- C ABI of the MI355X (gfx950) multilevel summation method (MSM)
 * library, libmsm.so.
 *
 * The library evaluates the electrostatic energy, per-atom forces and per-atom
 * potentials of N point charges by the multilevel summation method as stated
 * in Sec. 2.3 "Multilevel Summation Method" of the thesis:
 *   - 1/r is split into a short-range part g* (zero beyond the cutoff a) and
 *     smooth parts g^0 .. g^{l-1} carried by grids of spacing 2^k h
 *     (eq. split, eq. msmgrid, Taylor smoothing gamma);
 *   - u_i^short = sum_j g*(r_i, r_j) q_j over link cells (Sec. 2.1, link cells);
 *   - anterpolation, restriction, lattice cutoff, top level, prolongation,
 *     interpolation (the itemised MSM algorithm of Sec. 2.3);
 *   - U_i ~ (u_i^short + u_i^long)/(4 pi eps0) (potential display) and
 *     F_i = -dU/dr_i (Sec. 2.1 "Simulation loop").
 * Free-space (non-periodic) boundaries; the self term q_i gamma(0)/a is
 * removed from every potential; no bonded exclusions.
 *
 * Conventions shared by every entry point:
 *   - Every call returns msm_status; nothing throws across the ABI.
 *     msm_last_error() gives a thread-local message for the last failure.
 *   - Pointers named "device" are HIP device pointers; "host" are host memory.
 *   - All device work is enqueued on the caller's stream; no entry point
 *     synchronises except msm_status_query.  No entry point allocates device
 *     memory: the caller owns every device buffer, including the workspace.
 *   - Atom arrays are structure-of-arrays, float32, length n_atoms, in the
 *     caller's atom order; outputs are written in the same order.
 *   - Data errors (non-finite input, atom outside the box, coincident atoms)
 *     are detected on the device and recorded in status words inside the
 *     workspace; msm_status_query reports them.  With such an error the
 *     outputs are undefined (but every kernel stays in bounds).
 */
#ifndef MSM_H
#define MSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* msm_stream_t;   /* a hipStream_t; NULL = default stream */

typedef enum {
  MSM_OK = 0,
  MSM_ERR_INVALID_ARG = -1,   /* bad parameter, size or pointer */
  MSM_ERR_OUT_OF_BOX = -2,    /* some atom lies outside [box_lo, box_lo + box_len] */
  MSM_ERR_NONFINITE = -3,     /* NaN or Inf in a position or charge */
  MSM_ERR_WORKSPACE = -4,     /* workspace missing, too small or not initialised */
  MSM_ERR_HIP = -5,           /* a HIP runtime call failed */
  MSM_ERR_UNSUPPORTED = -6,   /* valid request outside what this build supports */
  MSM_ERR_COINCIDENT = -7     /* two atoms at exactly the same position */
} msm_status;

/* Method parameters (thesis Sec. 2.3: cutoff a, finest spacing h, number of
 * levels l, interpolation degree p = order - 1, smoothing degree m). */
typedef struct {
  double cutoff;          /* a > 0, Angstrom: short-range cutoff, level k carries 2^k a */
  double spacing;         /* h > 0, Angstrom: finest grid spacing; level k has 2^k h */
  int32_t order;          /* 4 = cubic C1 basis, 6 = quintic C1 basis */
  int32_t split_m;        /* Taylor smoothing degree m (gamma has degree 2m); 0 -> order/2 */
  int32_t levels;         /* l >= 1 grid levels; 0 -> fewest levels whose top interior
                             spans at most 8 nodes per dimension (periodic: whose top
                             grid has at most 8 nodes per side, as far as the levels
                             halve) */
  int32_t periodic;       /* 0: free space (atoms must lie in [lo, lo + len]);
                             1: periodic boundaries, the box repeated in every direction
                             (atoms anywhere; box_len / spacing an integer, divisible by
                             2^(levels-1), and 2 cutoff <= box_len) */
  double box_lo[3];       /* box lower corner; also the grid origin */
  double box_len[3];      /* box edge lengths > 0; free space: atoms must lie in [lo, lo + len] */
  double coulomb_k;       /* prefactor 1/(4 pi eps0) in the caller's units; 0 -> 1 (e^2/A) */
} msm_params;

typedef struct msm_plan msm_plan;   /* host object; immutable after creation */

/* Create a plan for systems of exactly n_atoms atoms (n_atoms >= 0).
 * Thesis Sec. 2.3: the l grids of spacing 2^k h (nodal basis display), the
 * cutoff 2^k a carried by level k (eq. msmgrid), the interpolation degree p
 * and smoothing degree m of eq. (flop); Sec. 2.1 "Potentials" for the link
 * cells of the short-range sum.
 * Validates the parameters, derives the grid hierarchy (level k node mu sits
 * at box_lo + 2^k h mu; each level spans every node with a non-zero weight)
 * and the cell decomposition.  *out receives the plan (host memory owned by
 * the library; free with msm_plan_destroy).
 * Errors: MSM_ERR_INVALID_ARG, MSM_ERR_UNSUPPORTED (grid or stencil beyond
 * this build's limits).
 * periodic = 1 (the thesis evaluates free-space systems; Sec. "Calculation
 * of Long-Range Interactions" names periodic boundaries with the Fourier
 * methods): every sum runs over the atoms of the box and all their images.
 * Level k is a periodic grid of (box_len / spacing) / 2^k nodes per side,
 * stored with ghost copies on each side (msm_plan_info reports lo = -ghost
 * and the count with the ghosts); the pair sum takes each pair at its nearest
 * image (2 cutoff <= box_len); the top level sums its kernel over every image
 * in the Ewald convention (conducting boundary, uniform neutralising
 * background for a charged box).  Atoms may lie anywhere (each is taken at its
 * image in the box).  Batches take free-space systems only. */
msm_status msm_plan_create(const msm_params* params, int32_t n_atoms, msm_plan** out);
msm_status msm_plan_destroy(msm_plan* plan);

/* Cheap pair methods on their own: the coarse propagators the thesis proposes
 * beside MSM (Sec. 3.2 "Proposed Solutions": "Cutoff Method", "Wolf Summation
 * Method"; the smoothed cutoff method of Sec. 2.2).  The pair energy
 * q_i q_j e(r) is summed over the unordered pairs closer than rc:
 *   MSM_PAIR_CUTOFF          e(r) = 1/r
 *   MSM_PAIR_SHIFTED_FORCE   e(r) = 1/r - 1/rc + (r - rc)/rc^2 (smoothed cutoff:
 *                            energy and force vanish continuously at rc)
 *   MSM_PAIR_WOLF            e(r) = erfc(alpha r)/r - erfc(alpha rc)/rc, plus the
 *                            self energy -(erfc(alpha rc)/(2 rc) + alpha/sqrt(pi)) q_i^2
 * msm_pair_plan_create returns a plan for n_atoms atoms that works with
 * msm_workspace_bytes, msm_workspace_init, msm_compute (same outputs: forces
 * -dE/dr_i, potentials dE/dq_i, energy, virial), msm_compute_static,
 * msm_graph_capture, msm_status_query, msm_plan_describe, msm_plan_tune / msm_plan_autotune (the
 * cell knobs) and msm_plan_destroy; msm_energy and
 * msm_backward return MSM_ERR_UNSUPPORTED for it, and batches do not take it.
 * Pair arithmetic is float32 (erfcf, expf for Wolf), reductions float64. */
typedef enum { MSM_PAIR_CUTOFF = 1, MSM_PAIR_SHIFTED_FORCE = 2, MSM_PAIR_WOLF = 3 } msm_pair_kind;
typedef struct {
  int32_t kind;           /* msm_pair_kind */
  int32_t periodic;       /* 0: free space; 1: periodic boundaries (pairs at their nearest
                             image; 2 cutoff <= box_len) */
  double cutoff;          /* rc > 0, Angstrom */
  double alpha;           /* Wolf damping (1/Angstrom), >= 0; ignored by the other kinds */
  double box_lo[3];       /* box lower corner */
  double box_len[3];      /* box edge lengths > 0; atoms must lie in [lo, lo + len] */
  double coulomb_k;       /* prefactor 1/(4 pi eps0); 0 -> 1 */
} msm_pair_params;
msm_status msm_pair_plan_create(const msm_pair_params* params, int32_t n_atoms, msm_plan** out);

/* Grid hierarchy of a plan: *levels, and per level k the lowest node index
 * grid_lo[3k+d] and node count grid_n[3k+d] along dimension d (host arrays of
 * at least 3 * 16 entries). */
msm_status msm_plan_info(const msm_plan* plan, int32_t* levels, int32_t* grid_lo, int32_t* grid_n);

/* Human-readable JSON description of the plan's decomposition (levels, link
 * cells, stencil taps, lattice-cutoff tile shapes, workspace size) written
 * into the host buffer buf (NUL-terminated; MSM_ERR_INVALID_ARG if it does
 * not fit in buf_bytes). */
msm_status msm_plan_describe(const msm_plan* plan, char* buf, size_t buf_bytes);

/* Device workspace size in bytes for this plan (256-byte aligned sections). */
msm_status msm_workspace_bytes(const msm_plan* plan, size_t* bytes);

/* Initialise a workspace: uploads the lattice-cutoff stencil weights and the
 * FP64 top-level kernel table (computed on the host in double precision).
 * Must be called once per workspace before any evaluation; enqueued on
 * `stream`.  ws: device, at least msm_workspace_bytes bytes. */
msm_status msm_workspace_init(const msm_plan* plan, void* ws, size_t ws_bytes, msm_stream_t stream);

/* Full evaluation (energy, forces, potentials): the itemised MSM algorithm of
 * Sec. 2.3 (short-range part, anterpolation, restriction and lattice cutoff
 * per level, top level, prolongation, interpolation), the potential display
 * U_i ~ (u_i^short + u_i^long) / (4 pi eps0), and F_i = -dU/dr_i of Sec. 2.1
 * "Simulation loop".
 * x, y, z, q : device float32 [n_atoms]  positions (A) and charges (e)
 * fx, fy, fz : device float32 [n_atoms]  forces F_i = -dE/dr_i (nullable: all three or none)
 * phi        : device float32 [n_atoms]  potentials phi_i = dE/dq_i (nullable)
 * energy     : device float64 [1]        E = 1/2 sum_i q_i phi_i (nullable)
 * virial     : device float64 [9]        W_ab = sum_i (r_i - lo)_a F_i,b (nullable)
 * Energy and virial are reduced in float64 in a fixed order; all other
 * arithmetic is float32 except the top-level grid sum (float64).
 * Results are bitwise reproducible for identical inputs. */
msm_status msm_compute(const msm_plan* plan, void* ws, size_t ws_bytes, msm_stream_t stream,
                       const float* x, const float* y, const float* z, const float* q,
                       float* fx, float* fy, float* fz, float* phi, double* energy,
                       double* virial);

/* msm_compute without a caller workspace and without any device allocation,
 * for callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation).  Same arguments and
 * results as msm_compute minus ws/ws_bytes; every stage runs in order on
 * `stream`.  The workspace is a 64 MiB array in the library's device data,
 * one copy per GPU, held until the process ends; plans whose workspace
 * (msm_workspace_bytes) exceeds 64 MiB are rejected with MSM_ERR_UNSUPPORTED
 * before anything runs.  The array keeps the last call's contents: the first
 * call of a plan on a device (and the first after a re-tune, or after another
 * plan's call) uploads the plan's tables into it and synchronises `stream`.
 * All calls on one GPU share the array, so calls that overlap on one GPU (two
 * streams, two threads) race and give undefined results.  Data errors (non-
 * finite input, atoms outside the box, coincident atoms) are not reported on
 * this path; the kernels stay in bounds and the outputs are then undefined. */
msm_status msm_compute_static(const msm_plan* plan, msm_stream_t stream, const float* x,
                              const float* y, const float* z, const float* q, float* fx,
                              float* fy, float* fz, float* phi, double* energy, double* virial);

/* Energy only (Sec. 2.3 potential display, E = 1/2 sum_i q_i U_i): E as
 * msm_compute would return it, evaluated through the grid form
 * 1/2 sum_k <q^k, u^{k,cut}> of the long-range part (no prolongation,
 * interpolation or short-range forces).  energy: device float64 [1].
 * Nothing but the workspace is written; grid potentials are not kept for a
 * later backward pass (msm_backward recomputes them). */
msm_status msm_energy(const msm_plan* plan, void* ws, size_t ws_bytes, msm_stream_t stream,
                      const float* x, const float* y, const float* z, const float* q,
                      double* energy);

/* Backward pass of the energy (F_i = -dU/dr_i, Sec. 2.1 "Simulation loop";
 * the chain of Sec. 2.3 run as its adjoint): with g = *grad_energy (device float64 scalar,
 * read on the device, so no host synchronisation),
 *   dedx, dedy, dedz (device float32 [n], nullable all three) = g dE/dr_i = -g F_i
 *   dedq            (device float32 [n], nullable)            = g dE/dq_i =  g phi_i.
 * The grid chain is recomputed from x, y, z, q; interpolation is run in
 * gradient mode (it is the adjoint of anterpolation), and the short-range
 * pair terms supply their part.  E is a quadratic form in q with a symmetric
 * kernel, so phi_i is exactly dE/dq_i and F_i exactly -dE/dr_i. */
msm_status msm_backward(const msm_plan* plan, void* ws, size_t ws_bytes, msm_stream_t stream,
                        const float* x, const float* y, const float* z, const float* q,
                        const double* grad_energy, float* dedx, float* dedy, float* dedz,
                        float* dedq);

/* Synchronise `stream` and return the data-error status recorded by the last
 * evaluation on this workspace (MSM_OK, MSM_ERR_OUT_OF_BOX, MSM_ERR_NONFINITE
 * or MSM_ERR_COINCIDENT).  *device_flags (nullable) receives the raw bit set. */
msm_status msm_status_query(const msm_plan* plan, const void* ws, msm_stream_t stream,
                            int32_t* device_flags);

/* Graph of one full evaluation.  msm_graph_capture records the kernels of
 * msm_compute for these exact buffers (same argument meaning, device
 * pointers baked into the graph) into a HIP graph and instantiates it;
 * nothing is executed.  msm_graph_launch replays it on `stream`: each replay
 * is a complete evaluation of the current contents of x, y, z, q.  The plan,
 * workspace and buffers must outlive the graph; replays on one workspace
 * must not overlap.  A graph holds the launch grids, kernel variants and LDS
 * sizes of the tuning in effect when it was captured: after msm_plan_tune,
 * msm_plan_autotune, msm_batch_tune or msm_batch_autotune on its plan or
 * batch, msm_graph_launch refuses it (MSM_ERR_INVALID_ARG, nothing runs);
 * capture it again.  Free with msm_graph_destroy. */
typedef struct msm_graph msm_graph;
msm_status msm_graph_capture(const msm_plan* plan, void* ws, size_t ws_bytes, const float* x,
                             const float* y, const float* z, const float* q, float* fx, float* fy,
                             float* fz, float* phi, double* energy, double* virial, msm_graph** out);
msm_status msm_graph_launch(const msm_graph* graph, msm_stream_t stream);
msm_status msm_graph_destroy(msm_graph* graph);

/* Byte offset and size of an internal workspace section, for stage-by-stage
 * checks.  section: 0 level grids of charges q^k (float32, levels
 * concatenated, x fastest), 1 lattice-cutoff/top-level sums u^{k,cut}
 * (same layout), 2 prolongated potentials u^k (same layout), 3 cell-sorted
 * atoms (float4 x,y,z,q), 4 sorted-to-input permutation (int32), 5 short-range
 * results per sorted atom (float4 Fx,Fy,Fz,phi, without the prefactor). */
msm_status msm_workspace_section(const msm_plan* plan, int32_t section, size_t* offset, size_t* bytes);

/* Diagnostics: per-stage timing of msm_compute, for its 9 stages: binning,
 * short range, anterpolation, restriction, lattice cutoff, top level,
 * prolongation, interpolation, reduction.  enable: 0 off; 1 in order (every
 * stage runs on the caller's stream, with a HIP event at each stage
 * boundary, so a stage's time is its launches alone); 2 live (the tuned
 * stream layout is kept and each stage's launches are bracketed by two
 * events on the stream they run on, so a stage's time includes the slowdown
 * from the stages that overlap it).  Events are created on the current
 * device by the first enabling call.  msm_profile_read waits for the last
 * evaluation timed since profiling was enabled and writes the 9 stage
 * durations in milliseconds to ms[0..8] (host); it fails when no evaluation
 * was timed. */
msm_status msm_profile_enable(msm_plan* plan, int32_t enable);
msm_status msm_profile_read(const msm_plan* plan, float* ms, int32_t* n_stages);

/* ------------------------------------------------------------------------ */
/* Tuning knobs.  Results depend on them only through float32 summation
 * order.  In msm_plan_tune / msm_batch_tune a zero field keeps the current
 * value. */
typedef struct msm_tuning {
  int32_t lattice_b;     /* lattice-cutoff outputs per lane along x: 4, 6 or 8 */
  int32_t item_chunks;   /* short-range 64-atom chunks of a cell row per work item (>= 1) */
  int32_t short_blocks;  /* blocks the short-range work items are strided over
                            (> 0), or -1 for one block per work item */
  int32_t streams;       /* 1: every stage in order on the caller's stream;
                            2: the short-range pass on a side stream;
                            3: also the level-0 lattice cutoff on a side stream */
  int32_t short_after;   /* with a side stream, the short-range pass starts after
                            1: binning, 2: anterpolation, 3: the coarse lattice
                            cutoff (it then overlaps the prolongations) */
  int32_t short_split;   /* with a side stream: per mille (1 .. 1000) of the
                            short-range work items that start at short_after; the
                            others start after the lattice cutoff (so they
                            overlap the prolongation rather than the lattice
                            cutoff); 1000: all of them */
  int32_t cell_reach;    /* link cells of edge a / cell_reach along y and z
                            (2, 3 or 4; x cells are 4 times finer): finer cells
                            cut the short-range candidates beyond the cutoff */
  int32_t reserved;      /* must be zero */
} msm_tuning;

/* Apply tuning knobs to a plan and re-upload its descriptor to ws (other
 * workspaces of the plan must be initialised again).  msm_plan_autotune times
 * candidates over `trials` evaluations of the given device inputs on `stream`
 * with HIP events: lattice_b (4, 6, 8) x item_chunks (1, 2, 3) x streams
 * (2, 3) first, then the stream layout x short-range block counts, then the
 * short-range start, the chunks per item again and the split; it applies the
 * fastest (a later candidate replaces the best so far only when faster by more
 * than 1%) and writes a JSON report (nullable) of the search.  *current
 * (msm_plan_tuning, nullable) receives the tuning in effect. */
msm_status msm_plan_tune(msm_plan* plan, void* ws, size_t ws_bytes, msm_stream_t stream,
                         const msm_tuning* tuning);
msm_status msm_plan_tuning(const msm_plan* plan, msm_tuning* current);
msm_status msm_plan_autotune(msm_plan* plan, void* ws, size_t ws_bytes, msm_stream_t stream,
                             const float* x, const float* y, const float* z, const float* q,
                             int32_t trials, char* report, size_t report_bytes);

/* Tuning cache (host files, no device work).  A cache is a text file with one
 * line per key: "<key> lattice_b item_chunks short_blocks streams short_after
 * short_split cell_reach" ('#' starts a comment line).  A key names what the
 * best tuning depends on: target (gfx950), interpolation order, smoothing
 * degree, level-0 stencil taps and, rounded to half octaves, the level-0 node
 * count and the atom count; a batch key adds the system count and uses the
 * largest stencil and the totals.  msm_*_tuning_key writes the key (with its
 * terminating zero) to key[key_bytes]; it fails when the buffer is too small.
 * msm_tuning_cache_lookup: MSM_OK with *tuning filled when the entry exists,
 * MSM_ERR_UNSUPPORTED when the file or the entry does not (*tuning
 * untouched), MSM_ERR_INVALID_ARG for a malformed or out-of-range entry.
 * msm_tuning_cache_store adds or replaces the key's entry; the file is
 * written beside the old one and renamed over it, so concurrent readers see
 * one or the other.  Keys contain no white space and no '#'.
 * msm_plan_autotune_cached / msm_batch_autotune_cached: with a cache entry
 * for the plan's key, apply it without timing anything; otherwise run the
 * autotuner and store its result (cache null: autotune, store nothing).  The
 * JSON report gives the key, "cache": "hit" | "miss" | "none", and the
 * applied tuning or the search. */
msm_status msm_plan_tuning_key(const msm_plan* plan, char* key, size_t key_bytes);
msm_status msm_tuning_cache_lookup(const char* path, const char* key, msm_tuning* tuning);
msm_status msm_tuning_cache_store(const char* path, const char* key, const msm_tuning* tuning);
msm_status msm_plan_autotune_cached(msm_plan* plan, void* ws, size_t ws_bytes, msm_stream_t stream,
                                    const float* x, const float* y, const float* z, const float* q,
                                    int32_t trials, const char* cache, char* report, size_t report_bytes);

/* ------------------------------------------------------------------------ */
/* Batches: n_sys independent systems (replicas of uneven size) evaluated
 * together.  Every stage is one launch covering all systems, so a batch costs
 * the launches of a single evaluation.  System s has params[s] and n_atoms[s]
 * atoms; its atoms occupy [off[s], off[s] + n_atoms[s]) of the concatenated
 * SoA arrays, off = exclusive prefix sum of n_atoms (msm_batch_atom_offsets
 * writes off[0..n_sys]).  All systems must share order and split_m.
 * Outputs: per-atom arrays concatenated like the inputs; energy[n_sys] and
 * virial[9 n_sys] (float64, device); grad_energy[n_sys] for the backward. */
typedef struct msm_batch msm_batch;
msm_status msm_batch_create(const msm_params* params, const int32_t* n_atoms, int32_t n_sys,
                            msm_batch** out);
msm_status msm_batch_destroy(msm_batch* batch);
msm_status msm_batch_workspace_bytes(const msm_batch* batch, size_t* bytes);
msm_status msm_batch_atom_offsets(const msm_batch* batch, int32_t* offsets);
msm_status msm_batch_workspace_init(const msm_batch* batch, void* ws, size_t ws_bytes,
                                    msm_stream_t stream);
msm_status msm_batch_compute(const msm_batch* batch, void* ws, size_t ws_bytes, msm_stream_t stream,
                             const float* x, const float* y, const float* z, const float* q,
                             float* fx, float* fy, float* fz, float* phi, double* energy,
                             double* virial);
msm_status msm_batch_energy(const msm_batch* batch, void* ws, size_t ws_bytes, msm_stream_t stream,
                            const float* x, const float* y, const float* z, const float* q,
                            double* energy);
msm_status msm_batch_backward(const msm_batch* batch, void* ws, size_t ws_bytes, msm_stream_t stream,
                              const float* x, const float* y, const float* z, const float* q,
                              const double* grad_energy, float* dedx, float* dedy, float* dedz,
                              float* dedq);
/* Graph of one batched evaluation (replay with msm_graph_launch). */
msm_status msm_batch_graph_capture(const msm_batch* batch, void* ws, size_t ws_bytes, const float* x,
                                   const float* y, const float* z, const float* q, float* fx,
                                   float* fy, float* fz, float* phi, double* energy, double* virial,
                                   msm_graph** out);
/* Synchronise and OR the data-error flags of every system (per-system raw
 * flags into flags_per_system[n_sys], nullable). */
msm_status msm_batch_status(const msm_batch* batch, const void* ws, msm_stream_t stream,
                            int32_t* flags_per_system);
msm_status msm_batch_describe(const msm_batch* batch, char* buf, size_t buf_bytes);
/* Tuning of every system of the batch (same knobs as msm_plan_tune; the
 * short-range block count applies per system). */
msm_status msm_batch_tune(msm_batch* batch, void* ws, size_t ws_bytes, msm_stream_t stream,
                          const msm_tuning* tuning);
msm_status msm_batch_autotune(msm_batch* batch, void* ws, size_t ws_bytes, msm_stream_t stream,
                              const float* x, const float* y, const float* z, const float* q,
                              int32_t trials, char* report, size_t report_bytes);
msm_status msm_batch_tuning_key(const msm_batch* batch, char* key, size_t key_bytes);
msm_status msm_batch_autotune_cached(msm_batch* batch, void* ws, size_t ws_bytes, msm_stream_t stream,
                                     const float* x, const float* y, const float* z, const float* q,
                                     int32_t trials, const char* cache, char* report, size_t report_bytes);

/* ------------------------------------------------------------------------ */
/* Bonded exclusions: pairs whose Coulomb interaction is left out of the sum
 * (atoms with bonded interactions are excluded from eq. (coulomb), Sec.
 * "Calculation of Long-Range Interactions").  Per-atom partner lists in CSR form over input indices:
 * the partners of atom g are idx[start[g] .. start[g + 1]) (device int32;
 * start has one entry per atom plus one; every pair listed from both sides;
 * nnz = start[n]).  For a batch the indices are global (into the
 * concatenated arrays) and a system's atoms may only list atoms of the same
 * system.  The library keeps the pointers: the arrays must stay valid and
 * unchanged while evaluations on ws use them; start = null removes the
 * exclusions.  Like a tuning change, the call re-uploads the descriptor to ws
 * (other workspaces must be initialised again) and refuses later replays of
 * graphs captured before it.  Effect on an MSM plan: every excluded pair loses
 * q_i q_j / r_ij from the energy, q_j / r_ij from phi_i and the matching
 * Coulomb force, i.e. its short-range term and the exact smooth part the grids
 * approximate (so an excluded pair keeps the grid's approximation error of that
 * smooth part); on a pair-method plan it loses the method's own pair term when
 * the short-range pass counted the pair.  Entries out of range are reported
 * through the data-error status as MSM_ERR_INVALID_ARG. */
msm_status msm_set_exclusions(msm_plan* plan, void* ws, size_t ws_bytes, msm_stream_t stream,
                              const int32_t* start, const int32_t* idx, int64_t nnz);
msm_status msm_batch_set_exclusions(msm_batch* batch, void* ws, size_t ws_bytes, msm_stream_t stream,
                                    const int32_t* start, const int32_t* idx, int64_t nnz);

/* ------------------------------------------------------------------------ */
/* Time stepping (Sec. 2.1 "Simulation loop": velocity Verlet; Sec. "Parareal
 * Method", eq. (parareal)).
 *
 * msm_vv_run / msm_batch_vv_run: n_steps velocity Verlet steps of dt on the
 * plan's (or batch's concatenated) atoms, forces from the plan or batch (any
 * plan: MSM or a cheap pair method).  Per step: v += (dt/2) s F / m; r += dt v;
 * F at the new r; v += (dt/2) s F / m, with s = accel_scale (the factor that
 * turns force / mass in the caller's units into acceleration, e.g. 0.138935
 * A/fs^2 per e^2/A^2/amu with coulomb_k = 1) and inv_mass = 1/m per atom.
 * Forces are evaluated at the start positions first (n_steps + 1 evaluations
 * in all).  x, y, z, vx, vy, vz (device) are updated in place; fx, fy, fz
 * (device) receive the forces at the final positions.  All work is enqueued
 * on `stream`; the data-error flags (msm_status_query / msm_batch_status)
 * are those of the last evaluation.
 *
 * msm_parareal_run: one computational window of the parareal iteration.
 * State lambda_t = (x, y, z, vx, vy, vz) of every atom at time points t = 0 ..
 * T (T = slices), stored in `states` (device, float, [6][T + 1][n]: component
 * c of time t at states + (c (T + 1) + t) n); the caller fills t = 0.  The
 * fine propagator F and the coarse G each take steps_per_slice velocity
 * Verlet steps of dt; F's forces come from `fine`, a batch of T systems with
 * the coarse plan's atom count (normally T copies of the MSM plan's
 * parameters), which advances all T slices together (one batched evaluation
 * per force call), and G's from `coarse` (one system, e.g. a cutoff or Wolf
 * pair plan).  Initial sweep: lambda_{t+1} = G(lambda_t).  Iteration k (0 ..
 * max_iter - 1): f_t = F(lambda_t) for every t < T at once, then for t = k ..
 * T - 1 in order lambda_{t+1} = f_t + (G(lambda_t) - g_t) with g_t the
 * previous G(lambda_t) (slices before k are final).  A slice whose start
 * state did not change gets f_t bit for bit, so after k iterations the first k
 * slices equal k sequential fine propagations exactly.  The iteration stops
 * after the first k whose largest position change max |lambda^{k+1} -
 * lambda^k| is <= tol (A), or after max_iter (<= T) iterations.
 * residuals (host, nullable, max_iter floats) receives those changes and
 * *iterations (host) the iterations run.  ws (device, >=
 * msm_parareal_workspace_bytes) is scratch.  q and inv_mass (device, n).
 * Synchronises once per iteration (to read the change); data errors of the
 * fine batch or the coarse plan are returned then. */
typedef struct {
  int32_t slices;           /* T >= 1 */
  int32_t steps_per_slice;  /* >= 1 */
  double dt;                /* time step */
  double accel_scale;       /* > 0 */
  int32_t max_iter;         /* 1 .. slices */
  int32_t reserved;         /* must be zero */
  double tol;               /* >= 0, A */
} msm_parareal_params;
msm_status msm_vv_run(const msm_plan* plan, void* ws, size_t ws_bytes, msm_stream_t stream, int32_t n_steps,
                      double dt, double accel_scale, float* x, float* y, float* z, const float* q, float* vx,
                      float* vy, float* vz, const float* inv_mass, float* fx, float* fy, float* fz);
msm_status msm_batch_vv_run(const msm_batch* batch, void* ws, size_t ws_bytes, msm_stream_t stream,
                            int32_t n_steps, double dt, double accel_scale, float* x, float* y, float* z,
                            const float* q, float* vx, float* vy, float* vz, const float* inv_mass, float* fx,
                            float* fy, float* fz);
msm_status msm_parareal_workspace_bytes(int32_t n_atoms, int32_t slices, size_t* bytes);
msm_status msm_parareal_run(const msm_parareal_params* params, const msm_batch* fine, void* fine_ws,
                            size_t fine_ws_bytes, const msm_plan* coarse, void* coarse_ws, size_t coarse_ws_bytes,
                            void* ws, size_t ws_bytes, msm_stream_t stream, const float* q, const float* inv_mass,
                            float* states, int32_t* iterations, float* residuals);

const char* msm_status_string(msm_status status);
const char* msm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MSM_H */
