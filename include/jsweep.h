/*
 * jsweep: data-driven discrete-ordinates transport sweeps on one AMD
 * Instinct MI355X (gfx950).  C ABI.
 *
 * The library implements the sweep path of JSweep (Yan, Yang, Zhang, Mo,
 * "A Patch-centric Data-driven Approach for Parallel Sweeps on Large-scale
 * Meshes", arXiv 1803.09876):
 *
 *   - the sweep dependency graph G = (V, E) whose vertices are (cell,
 *     direction) pairs and whose edges carry angular flux from an upwind
 *     cell to a downwind cell (Sec. V-A), with counts of upwind
 *     neighbours per vertex (Listing 1, init) and cycles removed before
 *     sweeping (appendix, sweep workflow step 1);
 *   - a data-driven sweep of all directions at once: a vertex is computed
 *     as soon as all of its upwind vertices are (Listing 1, compute;
 *     patch-angle parallelism, Sec. V-B);
 *   - source iteration around the sweep (appendix algorithm "Source
 *     iterative Sn solver": scattering source, sweeps, error reduction).
 *
 * The transport problem is steady, mono-group, with isotropic scattering:
 *   Omega . grad psi + sigma_t psi = sigma_s phi + q,  phi = sum_m w_m psi_m,
 * with sum_m w_m = 1, discretised with the step (upwind, piecewise
 * constant) scheme on triangles (2D), tetrahedra or hexahedra (3D):
 *   psi_{K,m} = (V_K s_{K,m} + sum_{inflow f} a_f psi_up)
 *             / (sigma_t,K V_K + sum_{outflow f} a_f),   a_f = |Omega_m . S_f|,
 * where S_f is the vector area of face f.  The paper leaves the spatial
 * scheme, the weight normalisation and the cycle rule open; the choices
 * are documented with each entry point.
 *
 * Conventions
 *   - All functions return JSWEEP_OK (0) or a negative error code; the
 *     thread-local detail is available from jsweep_last_error().  No C++
 *     exception crosses this interface.
 *   - Mesh and quadrature inputs to jsweep_build_graph are HOST pointers,
 *     borrowed for the call; the library copies what it keeps.
 *   - Problem data and results of jsweep_sweep / jsweep_solve /
 *     jsweep_solve_batch are DEVICE pointers (e.g. torch tensor
 *     data_ptr() on ROCm), caller-allocated, unless a function says
 *     otherwise.  Arrays indexed by (direction, cell) are stored
 *     direction-major: element m * n_cells + K.
 *   - hip_stream is a hipStream_t (NULL = the default stream).  Sweeps are
 *     stream-ordered; solves synchronise the stream once per outer
 *     iteration to read the residual.
 *   - One graph must not be used by two calls at the same time (its work
 *     lists, flux and scratch arrays are shared by every call on it).
 */
#ifndef JSWEEP_H
#define JSWEEP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define JSWEEP_OK 0
#define JSWEEP_E_INVALID_ARG (-1)   /* bad pointer, size or flag */
#define JSWEEP_E_MESH (-2)          /* non-positive volume, face shared by >2 cells, bad ids */
#define JSWEEP_E_QUADRATURE (-3)    /* weights not summing to 1, |Omega| != 1 */
#define JSWEEP_E_CYCLE (-4)         /* dependency cycle while lagging is disabled */
#define JSWEEP_E_DEVICE (-5)        /* HIP runtime error (detail in jsweep_last_error) */
#define JSWEEP_E_OOM (-6)           /* device or host allocation failed */
#define JSWEEP_E_STALLED (-7)       /* sweep watchdog fired: no progress within the time limit */
#define JSWEEP_E_NOT_CONVERGED (-8) /* iteration limit reached; outputs and stats are still written */
#define JSWEEP_E_PLACEMENT (-9)     /* a work-list sweep workgroup ran on another XCD than its stream
                                       (the hand-offs need each stream on one XCD); outputs undefined */

/* ---- cell types ---------------------------------------------------------
 * JSWEEP_TRI (2D): local edge j is the edge opposite vertex j.
 * JSWEEP_TET (3D): local face j is the face opposite vertex j.
 * JSWEEP_HEX (3D): corner c (0..7) sits at lattice offset
 *   (c>>2 & 1, c>>1 & 1, c & 1); local faces are -x, +x, -y, +y, -z, +z. */
#define JSWEEP_TRI 3
#define JSWEEP_TET 4
#define JSWEEP_HEX 8

/* ---- build flags ---------------------------------------------------- */
#define JSWEEP_DEBUG_NO_LAG 0x1u   /* report cycles as JSWEEP_E_CYCLE instead of lagging */
#define JSWEEP_HOST_PTRS 0x2u      /* jsweep_graph_export: output buffers are host memory */
/* bits 8-15 of the build flags: the work-list priority (below), e.g.
 * JSWEEP_PRIORITY_FLAGS(JSWEEP_PRIORITY_SLBD | JSWEEP_PRIORITY_ANGLE_MAJOR) */
#define JSWEEP_PRIORITY_FLAGS(p) (((uint32_t)(p) & 0xffu) << 8)

/* ---- work-list priorities (paper Sec. V-D, "Optimization: Priority
 * Strategy") ------------------------------------------------------------
 * The data-driven sweep takes the chunks (clusters of <= 64 vertices of one
 * level and direction, the coarsened graph of Sec. V-E) of each stream in a
 * fixed order: the order in which a ready queue ordered by the priority
 * would release them (Kahn's algorithm on the chunk graph, ties broken by
 * level order).  Every order is topological, so every priority gives
 * bit-identical fluxes; only the schedule changes.
 *   BFS   breadth first: level, then direction;
 *   LDCP  longest distance on the critical path: the longest chunk path to
 *         a sink of the graph first;
 *   SLBD  shortest local boundary distance: the chunk with the shortest
 *         such path (closest to the outflow boundary) first, a depth-first
 *         variant;
 *   PACED level / (the direction's level count): every direction of a
 *         stream reaches its last level at the end of the stream, the
 *         deepest ones in more, smaller steps (with BFS the deepest
 *         direction of a stream runs alone at the end, with LDCP at the
 *         start); a pacing of the paper's BFS by each angle's critical path
 *         (the default);
 *   ANGLE_MAJOR (OR-ed with one of the above): prior(a) * C + prior(p) with
 *         a large C, i.e. the chunk's direction ranks first (ascending), the
 *         strategy only among chunks of one direction.
 *   ANGLE_WEIGHT(k) (OR-ed with one of the above, k = 1..7, not with
 *         ANGLE_MAJOR): the same combined rank with a finite C, the largest
 *         level count of the stream's directions divided by k (rounded up);
 *         prior(a) is the direction's rank in its stream (streams hold
 *         contiguous direction ranges) and prior(p) the strategy's key (for
 *         BFS the level).  About k directions of a stream are then under
 *         way at once, each in a different phase of its sweep: fewer sweep
 *         fronts at a time than BFS across all directions, so the scattered
 *         per-cell reads stay in cache, with more parallelism than one
 *         direction at a time.
 * With a priority other than BFS or PACED the DIRECTION_LDS strategy is not
 * used (its program lookup needs each level's chunks together). */
#define JSWEEP_PRIORITY_BFS 1
#define JSWEEP_PRIORITY_LDCP 2
#define JSWEEP_PRIORITY_SLBD 3
#define JSWEEP_PRIORITY_PACED 4
#define JSWEEP_PRIORITY_ANGLE_MAJOR 0x10
#define JSWEEP_PRIORITY_ANGLE_WEIGHT(k) (((uint32_t)(k) & 7u) << 5)
#define JSWEEP_PRIORITY_ANGLE_WEIGHT_OF(p) ((int)(((uint32_t)(p) >> 5) & 7u))

/* ---- solve modes ---------------------------------------------------- */
#define JSWEEP_FP64 0              /* FP64 source iteration */
#define JSWEEP_FP32_REFINED 1      /* FP32 correction sweeps inside an FP64 residual loop */
#define JSWEEP_WARM_START 0x100    /* OR-ed into mode: psi holds the initial iterate */

typedef struct {
    int32_t dim;                   /* 2 or 3 */
    int32_t cell_type;             /* JSWEEP_TRI (dim 2), JSWEEP_TET or JSWEEP_HEX (dim 3) */
    int64_t n_vertices;
    const double *coords;          /* [n_vertices * dim], row-major */
    int64_t n_cells;
    const int64_t *cell_vertices;  /* [n_cells * cell_type], vertex ids in [0, n_vertices) */
} jsweep_mesh;

typedef struct {
    int32_t n_dirs;
    const double *omega;           /* [n_dirs * 3] unit directions; 2D streams with (x, y) */
    const double *weight;          /* [n_dirs], positive, summing to 1 (checked to 1e-12) */
} jsweep_quadrature;

typedef struct jsweep_graph_s *jsweep_graph;   /* opaque, owned by the library */

/* Sweep strategies.
 * DATA_DRIVEN: a persistent kernel over all directions at once; vertices of
 *   a level-ordered work list run as soon as their upwind vertices are done
 *   (the level-ordered flux array holds an empty marker, or in FP64 solves
 *   whose inputs all have the sign bit clear, i.e. hold no negative value,
 *   -0.0 or NaN, the previous sweep's sign tag, until a flux is written;
 *   waiting vertices poll it).
 * DIRECTION: one workgroup per direction walks that direction's levels with
 *   a workgroup barrier between levels; directions run side by side.
 * DIRECTION_LDS: as DIRECTION, with the recent fluxes of the direction in an
 *   LDS window and the per-vertex data streamed one level ahead; for graphs
 *   whose consecutive levels hold at most 16384 (FP64) / 32768 (FP32)
 *   vertices together and at most 2048 levels
 *   (otherwise DIRECTION is used).
 * PATCH: the paper's patch-program form (Sec. V-A, V-B): cells are cut into
 *   spatial patches (Morton order of the cell centres); one wavefront runs a
 *   patch of one direction as a task, its vertices level by level out of
 *   LDS.  The paper's patch programs are re-entrant: a patch whose cells and
 *   another patch's wait on each other is computed in several visits.  The
 *   visits are fixed when the program is built, by running each direction's
 *   graph patch by patch on the host (the patch with the lowest-level ready
 *   cell next, as far as the kernel's per-task budget allows); each visit is
 *   a task, and the task graph is acyclic.  A task enters its stream's
 *   ready queue when the last of its upstream tasks completes, and
 *   wavefronts take tasks from the queues.  The program is built on the
 *   first PATCH sweep; FP64 sweeps only (FP32 sweeps use DATA_DRIVEN);
 *   graphs above 2^26 (cell, direction) pairs or whose tasks exceed the
 *   kernel's LDS limits fall back to DATA_DRIVEN. */
/* AUTO (and no strategy set) is DATA_DRIVEN for a single graph; the
 * batched solve sweeps the union of the instances' work lists with the
 * DATA_DRIVEN kernel, compacting the list to the instances still iterating
 * whenever their work falls below half of the listed work (DATA_DRIVEN for
 * a batch: the full list every sweep; DIRECTION, DIRECTION_LDS: the
 * batched direction kernels). */
#define JSWEEP_STRATEGY_AUTO 0
#define JSWEEP_STRATEGY_DATA_DRIVEN 1
#define JSWEEP_STRATEGY_DIRECTION 2
#define JSWEEP_STRATEGY_DIRECTION_LDS 3
#define JSWEEP_STRATEGY_PATCH 4

/* Launch tuning of the sweep kernels; 0 in a field = default or the value
 * chosen by jsweep_autotune.  The knobs a batched sweep is usually tuned
 * by map onto these fields: cells per workgroup = 64 * waves_per_block (a
 * wavefront works on one chunk of up to 64 cells); queue depth =
 * chunks_per_ticket (the chunks a wavefront holds from one ticket, plus one
 * whose program it prefetches); directions in flight = the angle weight k
 * of the priority (JSWEEP_PRIORITY_ANGLE_WEIGHT, about k directions of a
 * stream at once; 0 = all of them); the batch is always every instance in
 * one launch. */
typedef struct {
    int32_t waves_per_block;       /* 64-lane wavefronts per workgroup (1..16) */
    int32_t blocks_per_cu;         /* DATA_DRIVEN: resident workgroups per CU (at most 4, and occupancy) */
    int32_t inner_sweeps;          /* FP32-refined: maximum inner sweeps per outer residual */
    int32_t chunks_per_ticket;     /* DATA_DRIVEN: work-list chunks a wavefront takes per atomic ticket */
    int32_t strategy;              /* JSWEEP_STRATEGY_* */
    int32_t priority;              /* JSWEEP_PRIORITY_* (0: keep the graph's work-list order); a
                                      different one rebuilds the graph's work list on first use */
} jsweep_params;

typedef struct {
    int32_t outer_iters;           /* FP64 residual evaluations */
    int32_t sweeps;                /* transport sweeps (all directions) */
    double residual;               /* final rho = ||r|| / ||q|| */
    double seconds;                /* wall time of the solve */
    int64_t lagged_edges;
    int32_t max_levels;
    int32_t history_len;           /* entries written to residual_history */
    double *residual_history;      /* caller-provided host buffer or NULL */
    int32_t history_capacity;      /* its length */
    int32_t reserved;
} jsweep_solve_stats;

/* Build the per-direction sweep graph of a mesh on the current device.
 *
 * Computes, on the GPU: unique faces and their vector areas S_f (oriented
 * from the lower to the higher cell id, outward on the boundary), cell
 * volumes, for every direction the upwind edges (Omega . S_f > 0: lower ->
 * higher cell; < 0: the reverse; == 0: no edge and no flux), in-degrees
 * (counts of upwind neighbours, Listing 1 init) and longest-path levels;
 * the level-ordered cell lists drive the sweep.  Geometry and graph
 * arithmetic is IEEE FP64 without contraction, so the graph is a pure
 * function of the inputs.
 *
 * Cycles (the paper excludes them and removes them beforehand, appendix
 * workflow step 1): inside every non-trivial strongly connected component
 * of a direction's graph, edges from a higher to a lower cell id are
 * lagged: they are not counted in the in-degree and carry the previous
 * iterate.  With JSWEEP_DEBUG_NO_LAG a cycle is an error instead.
 *
 * mesh, quad: host pointers (copied).  flags: JSWEEP_DEBUG_NO_LAG, and a
 * work-list priority as JSWEEP_PRIORITY_FLAGS(p) (default PACED).
 * out: receives the handle (NULL on error).
 * Errors: E_INVALID_ARG, E_MESH, E_QUADRATURE, E_CYCLE, E_DEVICE, E_OOM.
 * Limits: n_cells * faces_per_cell < 2^31; 3D meshes need n_vertices < 2^21
 * and 2D meshes n_vertices < 2^32 (face keys); n_dirs <= 4096. */
int jsweep_build_graph(const jsweep_mesh *mesh, const jsweep_quadrature *quad, uint32_t flags,
                       jsweep_graph *out);

/* Sizes of a built graph (any pointer may be NULL): cells, directions,
 * lagged edges (the appendix workflow's step 1, cycle elimination, as the
 * lag rule above reads it) and the largest level count of any direction
 * (the depth of the longest dependency chain of the sweep, Sec. II-C). */
int jsweep_graph_info(jsweep_graph g, int64_t *n_cells, int32_t *n_dirs, int64_t *n_lagged,
                      int32_t *max_levels);

/* The sweep program of a graph (any pointer may be NULL): *slots = its
 * inflow slots per vertex (the largest number of inflow faces of any
 * vertex, at most the faces per cell); *block_slots = how many of those
 * slots the FP64 work-list sweep reads from the chunk blocks instead of the
 * program arrays (0: it reads the full program); *packed = 1 when the
 * work-list sweeps read the upwind positions packed, three 21-bit
 * distances back from the vertex's own position in one 8-byte word, with
 * the few that do not fit (lagged faces, far upwind vertices) in the chunk
 * blocks.  Graphs with more than 3 slots get a compact program of 3 slots
 * per vertex when every work-list chunk has at most 7 further (vertex,
 * slot) pairs; graphs with at most 3 slots get packed positions when every
 * chunk has at most 12 codes that do not fit.  The sweep's results do not
 * depend on which program it reads. */
int jsweep_program_info(jsweep_graph g, int32_t *slots, int32_t *block_slots, int32_t *packed);

/* Export direction dir's graph (Sec. II-C: the sweep of one angle is a
 * topological traversal of this DAG; Listing 1's count is the in-degree):
 * in-degree [n_cells], level [n_cells], level pointers [n_levels + 1] and
 * cells ordered by (level, id) [n_cells].  Buffers are caller-allocated, device memory unless flags has
 * JSWEEP_HOST_PTRS; any may be NULL.  n_levels receives the level count
 * of the direction (size lvl_ptr accordingly; call once with lvl_ptr NULL
 * to learn it). */
int jsweep_graph_export(jsweep_graph g, int32_t dir, int32_t *indeg, int32_t *level, int64_t *lvl_ptr,
                        int64_t *lvl_cells, int32_t *n_levels, uint32_t flags);

/* Export the lagged edges (host buffers of length n_lagged, any may be
 * NULL), sorted by (direction, downwind cell, downwind local face):
 * direction, upwind cell, downwind cell, downwind cell's local face. */
int jsweep_graph_lagged(jsweep_graph g, int32_t *dir, int64_t *up, int64_t *down, int32_t *face);

/* One FP64 transport sweep of every direction (Listing 1 semantics: a
 * vertex runs when its upwind count is satisfied).
 *   sigma_t [n_cells]     total cross section (> 0)
 *   source  [n_cells]     isotropic source s (already including scattering)
 *   psi     [n_dirs*n_cells] in: previous iterate (read only on lagged
 *                         edges); out: the new angular flux
 *   phi     [n_cells]     out: sum_m w_m psi_m in ascending m (may be NULL)
 *   psi_boundary          isotropic inflow on boundary faces (0 = vacuum)
 * All device pointers; stream-ordered on hip_stream.
 * Errors: E_INVALID_ARG, E_STALLED (watchdog; psi is then undefined),
 * E_DEVICE. */
int jsweep_sweep(jsweep_graph g, const double *sigma_t, const double *source, double *psi, double *phi,
                 double psi_boundary, void *hip_stream);

/* jsweep_sweep for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results and errors as jsweep_sweep, and it calls no
 * hipMalloc, hipFree or other allocating routine: the per-cell V s of the
 * sweep is staged in a fixed device array of the library (64 MiB, so at
 * most 8,388,608 cells; larger graphs are rejected with
 * JSWEEP_E_INVALID_ARG), which every GPU the library runs on holds until
 * the process ends, and the graph's own arrays were allocated when it was
 * built.  The data-driven strategy only (a graph pinned to another strategy
 * with jsweep_set_params, or being traced, is rejected with
 * JSWEEP_E_INVALID_ARG); no kernel timing is recorded.  Every call on one
 * GPU shares that GPU's array: calls that overlap on one GPU (from two
 * threads or on two streams) race.  The graph must live on the current
 * device. */
int jsweep_sweep_noalloc(jsweep_graph g, const double *sigma_t, const double *source, double *psi, double *phi,
                         double psi_boundary, void *hip_stream);

/* Source iteration to a residual (appendix algorithm: scattering source,
 * sweeps, error reduction).  Each outer step evaluates in FP64
 *   r_{K,m} = q_K + sigma_s,K phi_K - (L psi)_{K,m} / V_K
 * with the full (un-lagged) streaming operator L and stops once
 * rho = ||r|| / ||q|| <= tol, where ||x||^2 = sum_K V_K sum_m w_m x_{K,m}^2
 * and ||q||^2 = sum_K V_K q_K^2 (rho = ||r|| when q = 0); tol = 0 runs
 * exactly max_iter sweeps.  After a plain FP64 sweep r is evaluated through
 * the identity the sweep satisfies (sigma_s times the change of phi plus
 * the lagged-face differences), which equals the operator form up to
 * rounding.
 *   mode JSWEEP_FP64: plain source iteration, one FP64 sweep per outer step.
 *   mode JSWEEP_FP32_REFINED: iterative refinement; the correction
 *     (L - sigma_s W) dpsi = r is approximated by up to inner_sweeps FP32
 *     source iterations, then psi += dpsi and phi = sum w psi in FP64.
 *   OR JSWEEP_WARM_START: psi holds the initial iterate (else psi = 0).
 * sigma_t, sigma_s, q: device [n_cells]; phi: device [n_cells] out;
 * psi: device [n_dirs*n_cells] (out, and in with WARM_START) or NULL;
 * params may be NULL; stats (host) may be NULL.
 * Errors: E_INVALID_ARG, E_NOT_CONVERGED (results and stats written),
 * E_STALLED, E_DEVICE, E_OOM. */
int jsweep_solve(jsweep_graph g, const double *sigma_t, const double *sigma_s, const double *q,
                 double psi_boundary, int32_t mode, double tol, int32_t max_iter, const jsweep_params *params,
                 double *phi, double *psi, jsweep_solve_stats *stats, void *hip_stream);

/* Multigroup source iteration (the appendix form of the transport
 * equation, with a flux per ordinate and energy group and isotropic
 * scattering from every group into every group; appendix algorithm "Source
 * iterative Sn solver": 2.1 scattering source and coupling terms, 2.2 sweeps
 * of every angle and energy, 2.3 error reduction):
 *   Omega_m . grad psi_{m,g} + sigma_t,g psi_{m,g}
 *       = q_g + sum_{g'} sigma_s,g'->g phi_{g'},   phi_g = sum_m w_m psi_{m,g}.
 * Jacobi over groups: each iteration takes every group's source from the
 * previous iterate of all groups (sum over g' ascending), then sweeps every
 * (direction, group) in one launch of the data-driven kernel (the groups
 * share the graph and its sweep program), then phi_g (ascending m) and
 *   rho = sqrt(sum_g sum_K V_K sum_m w_m r_{K,m,g}^2) / sqrt(sum_g sum_K V_K q_{K,g}^2)
 * with r the residual of the full (un-lagged) operator.  Stops once
 * rho <= tol (tol = 0: exactly max_iter iterations).  FP64 throughout.
 *   n_groups        1 .. 8
 *   sigma_t, q      device [n_groups * n_cells], group-major
 *   sigma_s         device [n_groups * n_groups * n_cells]: the cross
 *                   section from group g' into group g of cell K at
 *                   (g' * n_groups + g) * n_cells + K
 *   phi             device [n_groups * n_cells] (out)
 *   psi             device [n_groups * n_dirs * n_cells] (out) or NULL
 * Starts from psi = 0.  Errors as jsweep_solve. */
int jsweep_solve_groups(jsweep_graph g, int32_t n_groups, const double *sigma_t, const double *sigma_s, const double *q,
                        double psi_boundary, double tol, int32_t max_iter, const jsweep_params *params, double *phi,
                        double *psi, jsweep_solve_stats *stats, void *hip_stream);

/* One problem instance of a batch (device pointers as in jsweep_solve). */
typedef struct {
    const double *sigma_t, *sigma_s, *q;
    double psi_boundary;
    double *phi;
    double *psi;                   /* may be NULL */
} jsweep_problem;

/* Solve n independent problems, each on its own graph, together: every
 * sweep of the batch is one persistent kernel launch over all instances
 * (patch-angle parallelism across instances), and each outer step of the
 * batch is replayed from a captured HIP graph.  Instances stop
 * individually at their own residual.  stats: host array [n] or NULL.
 * Errors as jsweep_solve (E_NOT_CONVERGED if any instance missed tol). */
int jsweep_solve_batch(int32_t n, const jsweep_graph *graphs, const jsweep_problem *problems, int32_t mode,
                       double tol, int32_t max_iter, const jsweep_params *params, jsweep_solve_stats *stats,
                       void *hip_stream);

/* Pick launch parameters for these graphs by timing candidate
 * configurations of the sweep kernel on the device (the paper tunes its
 * run-time hyper-parameters, patch size and clustering, by measurement,
 * Sec. VI; here the workgroup shape, chunks per ticket, kernel strategy and
 * for FP32-refined solves the inner sweep count) (uses scratch problem
 * data, no caller buffers).  The result is cached in memory and, when the
 * environment variable JSWEEP_TUNE_CACHE names a file, in that JSON file
 * keyed by (cell type, size bucket, direction count, mode, device). */
int jsweep_autotune(int32_t n, const jsweep_graph *graphs, int32_t mode, jsweep_params *out);

/* Launch parameters of a graph's sweeps: the ones jsweep_sweep uses and
 * jsweep_solve uses when its params argument is NULL (the same slot
 * jsweep_autotune fills).  p == NULL returns the graph to the defaults
 * (the work-list order stays as it is).  A nonzero p->priority reorders the
 * work list now (paper Sec. V-D). */
int jsweep_set_params(jsweep_graph g, const jsweep_params *p);

/* The PATCH strategy's program of a graph, built now if it was not yet
 * (hip_stream as for the other calls).  out[6] (host): 1 if the strategy
 * applies to this graph (else 0, and PATCH sweeps run DATA_DRIVEN), tasks,
 * rounds, halo entries, task dependencies, visits beyond one per (patch,
 * direction). */
int jsweep_patch_info(jsweep_graph g, void *hip_stream, int64_t *out);

/* Kernel timing of the sweep launches on a graph: while enabled, the
 * library records a HIP event pair around every launch of the sweep kernel
 * (on the launch stream); a batched solve's data-driven launches over the
 * union of its instances are recorded on its first instance's graph.  jsweep_profile_read synchronises on those
 * events and returns the number of launches and their summed duration in
 * milliseconds since the last reset (reset != 0 clears them afterwards). */
int jsweep_profile(jsweep_graph g, int32_t enable);
int jsweep_profile_read(jsweep_graph g, int32_t reset, int64_t *launches, double *total_ms);

/* Tracing of the data-driven sweep (the paper's runtime breakdown into
 * scheduling, waiting and computing).  While enabled, every sweep records,
 * per work-list chunk, three s_memrealtime stamps (100 MHz, low 32 bits):
 * when a wavefront took the chunk (issued the loads of its program), when
 * every upwind flux of its vertices had arrived, and when it had issued the
 * stores of its own fluxes.  Tracing runs a variant of the kernel that
 * writes the stamps.
 * jsweep_trace_read (host buffers, any may be NULL) returns the chunk count,
 * the stamps of the last traced sweep [3 * n_chunks], per chunk (direction,
 * vertex count, level) [3 * n_chunks], and the coarsened graph as CSR
 * (deps_ptr [n_chunks + 1], deps [deps_ptr[n_chunks]]).  When the last
 * traced sweep ran the PATCH kernel, the units are its tasks instead: the
 * stamps are those of the task, and the per-unit triple is (direction,
 * vertex count, rounds); the CSR lists the upstream tasks. */
int jsweep_trace(jsweep_graph g, int32_t enable);
int jsweep_trace_read(jsweep_graph g, int64_t *n_chunks, uint32_t *stamps, int32_t *chunk_info, int32_t *deps_ptr,
                      int32_t *deps);

void jsweep_graph_destroy(jsweep_graph g);

const char *jsweep_error_string(int code);
const char *jsweep_last_error(void);   /* thread-local detail of the last failure */

#ifdef __cplusplus
}
#endif
#endif /* JSWEEP_H */
