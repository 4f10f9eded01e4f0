// Internal declarations of the jsweep library (gfx950).
#pragma once
#include <cstring>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <initializer_list>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "../../include/jsweep.h"

namespace jsw {

// ---------------------------------------------------------------------------
// errors: thrown inside the library, turned into status codes at the ABI
// ---------------------------------------------------------------------------
struct Error {
    int code;
    std::string msg;
};
[[noreturn]] void fail(int code, const std::string &msg);
void hip_check(hipError_t e, const char *what, const char *file, int line);
#define JSW_HIP(x) ::jsw::hip_check((x), #x, __FILE__, __LINE__)
void set_last_error(const std::string &msg);

// ---------------------------------------------------------------------------
// device memory owned by the library
// ---------------------------------------------------------------------------
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    explicit DevBuf(size_t n) { alloc(n); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t n);
    void release();
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// ---------------------------------------------------------------------------
// per-cell records read by the sweep: outward vector areas of the local
// faces, volume, sigma_t * V (filled per problem) and neighbour codes.
// Neighbour code: >= 0 interior neighbour id, -1 boundary, <= -2 interior
// neighbour (-code - 2) through a face that is lagged in some direction.
// ---------------------------------------------------------------------------
template <class R, int NF, int DIM>
struct alignas(16) CellRec {
    R S[NF][DIM];
    R V;
    R sigV;
    int32_t nbr[NF];
};

__host__ __device__ constexpr int faces_of(int ctype) { return ctype == JSWEEP_TRI ? 3 : ctype == JSWEEP_TET ? 4 : 6; }

// Sweep work unit: up to 64 cells of one direction and one level, one
// wavefront lane each.  a = direction | (count - 1) << 16, b = offset of
// the first cell in the direction's level-ordered cell list.
struct Chunk {
    uint32_t a, b;
};

// Chunk block, kBlock int32 words: [0, 64) the chunk's cells (-1 past the
// end), [64] Chunk::a, [65] the number of upwind chunks (-1: more than
// kBlockDeps, see the CSR lists), [66] Chunk::b (the first position),
// [67, 67 + kBlockDeps) the upwind chunks.  Lane l of a wavefront reads
// words l and 64 + l (l < 32); the work-list sweep uses words 0 - 66 (it
// waits on the upwind fluxes themselves, not on the upwind chunks).
constexpr int kBlock = 96;
constexpr int kBlockDeps = kBlock - 67;
// Compact FP64 program of the work-list sweep (graphs with more than
// kCompactSlots inflow slots): kCompactSlots slots per lane in the program
// arrays, and the few further slots as at most kBlockExtra entries in the
// chunk block: [65] the entry count, [67 + 4 e, 71 + 4 e) entry e = (lane |
// slot << 8, code, low and high words of a_f).  These words replace the
// inline upwind chunks, which the work-list sweep does not read.
constexpr int kCompactSlots = 3;
constexpr int kBlockExtra = 7;
// Packed codes (graphs with at most 3 inflow slots and no compact entries):
// the 3 slot codes of a lane in one 64-bit word, 21 bits per slot: the
// distance back from the vertex's own level position to the upwind one
// (1 .. kPkMaxDelta), or kPkNoFace / kPkBound (-1, psi_b) / kPkEsc.  An
// escaped code (a lagged face, or an upwind vertex further back) is an
// entry of the chunk block: [65] the entry count, [70 + 2 e, 72 + 2 e)
// entry e = (lane | slot << 8, the int32 code), at most kPkEscMax of them
// (words 67 - 69 stay free for the batched sweep's direction base).
// Graph::dd_state bits of a level-position array holding sign-tagged FP64
// fluxes, and whether their tag (the sign bit) is set
constexpr int kDdTagged = 1 << 16;
constexpr int kDdTagSet = 1 << 17;
constexpr int kPkBits = 21;
constexpr uint32_t kPkMask = (1u << kPkBits) - 1u;
constexpr uint32_t kPkNoFace = kPkMask;
constexpr uint32_t kPkBound = kPkMask - 1u;
constexpr uint32_t kPkEsc = kPkMask - 2u;
constexpr uint32_t kPkMaxDelta = kPkMask - 3u;
constexpr int kPkEscMax = 12;

// Sweep program: per chunk lane (index c * 64 + lane, stride S = 64 *
// n_chunks) the vertex's inflow faces in local face order, ns slots each:
// code >= 0 position of the upwind vertex in the direction's level order,
// -1 boundary (psi_b), <= -2 lagged edge -(e + 2),
// kNoFace empty; coefficient a_f = |Omega . S_f| (FP64 and FP32 copies);
// and den = sigma_t V + sum of outflow a_f in local face order (refreshed
// when sigma_t changes).
constexpr int32_t kNoFace = INT32_MIN;

// Index of the lagged edge u -> v of direction m in the (m, v, u)-sorted
// lists, or -1 when that edge is not lagged.
__device__ inline int64_t lag_index(const uint64_t *lag_mv, const int32_t *lag_u, int64_t n_lag, int m, int64_t v,
                                    int64_t u) {
    uint64_t key = ((uint64_t)(uint32_t)m << 32) | (uint64_t)v;
    int64_t lo = 0, hi = n_lag;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (lag_mv[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    for (; lo < n_lag && lag_mv[lo] == key; ++lo)
        if (lag_u[lo] == u) return lo;
    return -1;
}

// The work list is split into kStreams streams (a direction belongs to one
// stream); on MI355X stream x runs on XCD x.
constexpr int kStreams = 8;

// Device status word bits (Graph::status[0]): a sweep wavefront's watchdog
// fired, or a workgroup found itself on another XCD than its stream's.
constexpr int32_t kStatusStalled = 1;
constexpr int32_t kStatusPlacement = 2;

// XCD (accelerator complex die) the calling wavefront runs on: the XCC_ID
// hardware register (hwreg 20, bits 3:0) of gfx94x / gfx950.
__device__ __forceinline__ int xcc_id() {
    return (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 0xfu);
}

// The work-list sweeps hand fluxes from producer to consumer through the L2
// of one XCD, so every workgroup of a stream (ids congruent mod kStreams)
// must run on the same XCD.  The dispatcher deals workgroups round robin
// over the XCDs, which keeps ids congruent mod 8 together; which XCD a
// stream lands on is not fixed (dispatches have been seen with workgroup b
// on an XCD other than b mod 8), and nothing else needs it.  Each stream
// has a slot next to its ticket, reset to kNoXcc before every sweep: the
// first wavefront of the stream records its XCD there, every later one
// compares.  A wavefront on another XCD takes no work and raises
// kStatusPlacement (every waiting wavefront sees it and ends) instead of
// leaving its stream's consumers to the watchdog.  Returns true when the
// wavefront is where the hand-offs need it.
constexpr uint32_t kNoXcc = 0xffffffffu;
constexpr int kXccSlot = 8;              // word of a stream's ticket block holding its XCD
__device__ __forceinline__ bool check_stream_placement(uint32_t *slot, int32_t *status) {
    const uint32_t x = (uint32_t)xcc_id();
    uint32_t prev = kNoXcc;
    if ((threadIdx.x & 63) == 0) prev = atomicCAS(slot, kNoXcc, x);
    prev = __builtin_amdgcn_readfirstlane(prev);
    if (prev == kNoXcc || prev == x) return true;
    if ((threadIdx.x & 63) == 0) atomicOr(status, kStatusPlacement);
    return false;
}

// Patch-task sweep program (built on the first sweep that uses it).  The
// cells are cut into patches of consecutive Morton rank; a task is one visit
// of a patch in one direction (a patch may need several visits when its
// cells and another patch's wait on each other).  Per direction, positions
// run task by task (tasks in ticket order), by level within a task; a task's
// levels are split into rounds of at most 64 vertices.  Codes (kPatch*
// limits below): >= 0 LDS slot of the upwind flux (the task's own vertices
// first, then its halo), -1 boundary, kNoFace empty.  A halo entry >= 0 is
// an upwind position of another task of the direction, < 0 the lagged edge
// -(h + 1).
constexpr int kPatchSlots = 512;         // task vertices + halo entries
constexpr int kPatchCells = 256;         // vertices of a task
constexpr int kPatchHalo = 256;          // halo entries of a task
constexpr int kPatchRounds = 64;         // rounds of a task
constexpr int kPatchDesc = 16;           // descriptor words per task
struct PatchProg {
    bool built = false, ok = false;      // ok: every task fits the limits above
    int P = 0;                           // cells per patch
    int ns = 0;                          // inflow slots per vertex
    int64_t n_tasks = 0, n_rounds = 0, n_halo = 0, n_dep = 0;
    int64_t revisits = 0;                // visits beyond one per (patch, direction)
    std::vector<int64_t> stream_off_h;
    DevBuf stream_off;                   // [kStreams + 1] int64 task offsets of the streams
    DevBuf desc;                         // [n_tasks * kPatchDesc] int32: q0, m, n, rounds, round0, halo, halo0,
                                         //   deps, dep0, downstream tasks, down0
    DevBuf round;                        // [n_rounds] int32 offset in the task | (count - 1) << 16
    DevBuf halo;                         // [n_halo] int32
    DevBuf dep;                          // [n_dep] int32 upstream tasks
    DevBuf cell;                         // [nd*nc] int32 vertex at each position
    DevBuf code;                         // [ns * nd*nc] int32
    DevBuf a64;                          // [ns * nd*nc] double
    DevBuf den64;                        // [nd*nc] double
    bool den64_ok = false;
    DevBuf psi;                          // [nd*nc] double fluxes by position (halo source)
    DevBuf down;                         // [n_dep] int32 downstream tasks (ranges in the descriptors)
    DevBuf cnt;                          // [n_tasks] int32 upstream tasks not yet complete
    DevBuf slot;                         // [n_tasks] uint32 ready queues, stream by stream
    DevBuf qctl;                         // [32 * kStreams] uint32 queue heads and tails
    DevBuf nsrc;                         // [kStreams] int32 tasks without upstream tasks
    int epoch = 0;
};

// ---------------------------------------------------------------------------
// graph handle
// ---------------------------------------------------------------------------
struct Graph {
    uint64_t uid = 0;                    // unique per built graph (process-wide counter)
    uint32_t prog_version = 0;           // bumped whenever the work list or program is rebuilt
    int device = 0;
    int n_cu = 0;
    int priority = JSWEEP_PRIORITY_PACED;  // order of the work list (JSWEEP_PRIORITY_*)
    int dim = 3, ctype = JSWEEP_TET, nfpc = 4;
    int64_t nv = 0, nc = 0, nf = 0;
    int nd = 0;
    std::vector<double> omega_h, weight_h;
    DevBuf omega64, omega32, weight;     // [nd*3] double / float, [nd] double
    DevBuf rec64, rec32;                 // cell records (rec32 built on first FP32 use)
    DevBuf vol;                          // [nc] double
    DevBuf level;                        // [nd*nc] int32
    DevBuf lvl_cells;                    // [nd*nc] int32, per direction by (level, id)
    std::vector<int64_t> lvl_off_h;      // [nd+1] start of each direction's lvl_ptr block
    std::vector<int64_t> lvl_ptr_h;      // concatenated per-direction level pointers
    std::vector<int32_t> nlev_h;         // [nd]
    DevBuf lvl_ptr_d, lvl_off_d;         // device copies of the level pointers
    std::vector<int32_t> lvl_chunk_h;    // first chunk of each (direction, level), indexed like lvl_ptr_h
    DevBuf lvl_chunk_d;
    int64_t max_w = 0, max_w2 = 0;       // widest level; widest pair of consecutive levels
    int max_levels = 0;
    DevBuf chunks;                       // [n_chunks] Chunk: per stream, ordered by (level, direction)
    DevBuf cblk;                         // [n_chunks * kBlock] int32 chunk blocks (see kBlock)
    int64_t n_chunks = 0;
    DevBuf stream_off;                   // [kStreams + 1] int64 chunk offsets of the streams
    std::vector<int64_t> stream_off_h;
    std::vector<int32_t> dir_stream_h;   // [nd] stream of each direction
    DevBuf dep_ptr, dep;                 // coarsened graph: upwind chunks of every chunk (CSR)
    int64_t n_dep = 0;
    int ns = 0;                          // sweep program: inflow slots per vertex
    DevBuf pcode, pa64, pa32;            // [ns * S] int32 / double / float (pa32 on first FP32 use)
    DevBuf pcode3, pa3;                  // [kCompactSlots * S] compact FP64 program (see kCompactSlots)
    DevBuf pk;                           // [S] packed codes (see kPkBits), or empty
    int ns_x = 0;                        // slots past kCompactSlots in the blocks; 0: no compact program
    DevBuf pden64, pden32;               // [S] double / float
    DevBuf sig_last;                     // [nc] sigma_t the denominators were built for
    bool den64_ok = false, den32_ok = false;
    DevBuf psi_pos;                      // [nd*nc] fluxes of the running sweep in level order (LDS-window sweeps)
    DevBuf dd_pos[2];                    // [nd*nc] alternating level-order flux arrays of the work-list sweep
    int dd_state[2] = {0, 0};            // element size | groups << 8 of the markers each array holds (0: unknown),
                                         // or | kDdTagged (| kDdTagSet) for sign-tagged FP64 fluxes
    int dd_cur = 0;                      // array of the next work-list sweep
    DevBuf pvol64, pvol32;               // [64 n_chunks] cell volume in program order (ring sweep)
    DevBuf vsc;                          // [nc] V s (or {V, s}) of the running sweep, per cell
    DevBuf posi;                         // [nd*nc] int32 level position of every vertex
    DevBuf mrank;                        // [nc] int32 rank of every cell in the Morton order of the vertex averages
    DevBuf status;                       // [4] int32 device status words (watchdog)
    // lagged edges, sorted by (direction, downwind cell, upwind cell)
    int64_t n_lag = 0;
    std::vector<int32_t> lag_m_h, lag_face_h;
    std::vector<int64_t> lag_u_h, lag_v_h;
    DevBuf lag_mv;                       // [n_lag] uint64  m << 32 | v
    DevBuf lag_u;                        // [n_lag] int32
    DevBuf lag_val64, lag_val32;         // previous-iterate snapshots
    DevBuf lag_a;                        // [n_lag] double |Omega . S| of the lagged face
    DevBuf lag_cptr;                     // [nc + 1] int32: each downwind cell's lagged-edge groups (n_lag > 0)
    DevBuf lag_cgrp;                     // int32 first edge of every (direction, downwind cell) group, by cell
    // scratch reused across solves
    DevBuf scratch_a, scratch_b, scratch_c, scratch_d;
    int grid_waves64 = 0, grid_waves32 = 0;   // persistent grid sizes
    jsweep_params tuned{};               // set by jsweep_autotune
    bool has_tuned = false;
    // per-chunk time stamps of the last sweep (jsweep_trace)
    bool trace = false;
    int trace_units = 0;                 // units of the last traced sweep: 0 work-list chunks, 1 patch tasks
    DevBuf trace_buf;
    PatchProg pp;                        // patch-task sweep program
    // kernel timing (jsweep_profile)
    bool profile = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_events;
    ~Graph() {
        for (auto &e : prof_events) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    }
};

// build steps (geometry.hip, dag.hip)
void build_geometry(Graph &g, const jsweep_mesh &mesh, hipStream_t s);
void build_dag(Graph &g, bool lag_cycles, hipStream_t s);
// whether the work list keeps the chunks of every (direction, level)
// together (what the LDS-window kernels read a level's program from)
inline bool levels_contiguous(const Graph &g) {
    return g.priority == JSWEEP_PRIORITY_BFS || g.priority == JSWEEP_PRIORITY_PACED;
}
// reorder the work list by a priority (JSWEEP_PRIORITY_*), rebuilding what
// is kept in chunk order
void set_priority(Graph &g, int priority, hipStream_t s);
void build_rec32(Graph &g, hipStream_t s);

// sweep launch (sweep.hip)
struct SweepSrc {
    const void *cell;        // [nc] isotropic part of the source (Real), may be null
    const void *dir;         // [nd*nc] per-direction part (float, FP32 path only), may be null
};
void refresh_sigma(Graph &g, const double *sigma_t, bool fp32, hipStream_t s);
// sweep-program denominators from the records' sigma_t V, where not valid
void ensure_den(Graph &g, bool fp32, hipStream_t s);
// prepared: g.vsc already holds V s of src_cell for this sweep (FP64, or
// one float per cell in FP32) and the data-driven kernel's tickets are zero
// (the FP64 solve prepares the next sweep in its residual kernels, the FP32
// correction solve in k_dphi).  nonneg: the caller has checked that every
// input of the sweep (source, cross sections, boundary and lagged values)
// is non-negative, so every flux is: the data-driven sweep then tags its
// fluxes by sign instead of writing empty markers, and readers of its
// level-position array mask the sign bit (last_sweep_keep)
void launch_sweep64(Graph &g, const double *src_cell, double *psi, double psi_b, const jsweep_params *p, hipStream_t s,
                    bool prepared = false, bool nonneg = false);
void launch_sweep32(Graph &g, const float *src_dir, const float *src_cell, float *psi, const jsweep_params *p,
                    hipStream_t s, bool prepared = false);
// The data-driven sweep always leaves its fluxes in level-position order
// (flux of cell K in direction m at m nc + posi[m nc + K]) in one of the
// graph's two level-position arrays; psi == null to those launchers skips
// the cell-order copy.  This returns the array the last data-driven sweep
// filled (double or float by that sweep's precision).
void *last_sweep_pos(Graph &g);
// The bits to keep of each FP64 flux read from last_sweep_pos: all, or all
// but the sign bit when that sweep tagged its fluxes by sign
uint64_t last_sweep_keep(const Graph &g);
// Whether every element of the given device arrays (pointer, length; null
// pointers skipped) has its sign bit clear and is not NaN (-0.0 and NaN
// count as negative); one synchronisation
bool all_nonnegative(std::initializer_list<std::pair<const double *, int64_t>> arrays, hipStream_t s);
// A direction of a union of graphs swept by one launch of the data-driven
// kernel (the batched solve): where its arrays start.  pos_base: its first
// level position in the union's level-position arrays; psi_row: the
// instance's cell-order fluxes of this direction (or null); cell_off: the
// instance's first cell in the union's per-cell arrays (cell ids in the
// union's chunk blocks are global); src_row: the instance's per-direction
// FP32 source of this direction, by level position (or null); inst: the
// instance.
struct DirRow {
    int64_t pos_base;
    int64_t cell_off;
    void *psi_row;
    const float *src_row;
    double psi_b;                        // the instance's boundary inflow
    int32_t inst;
    int32_t pad;
};

// Multigroup FP64 sweep: groups (<= kMaxGroups) energy groups of one graph
// in one launch of the data-driven kernel.  The caller has prepared
// g.vsc as V s per (group, cell) [groups * nc] and zeroed the stream
// tickets; den [groups][64 n_chunks] holds each group's denominators and
// lag_val [groups][n_lag] each group's previous-iterate lagged values.
// psi: [groups][nd][nc] cell-order fluxes (out).
constexpr int kMaxGroups = 8;
struct GroupSweep {
    int groups;
    const double *den;
    const double *lag_val;
    double psi_b;
    bool nonneg;                         // every input non-negative (see launch_sweep64)
};
void launch_sweep_groups(Graph &g, double *psi, const GroupSweep &mg, const jsweep_params *p, hipStream_t s);
// FP64 data-driven sweep whose per-cell V s goes to vs_buf (8 n_cells bytes,
// device) instead of a graph buffer: allocates nothing (the graph's flux
// arrays are allocated when it is built)
void launch_sweep64_staged(Graph &g, const double *src_cell, double *psi, double psi_b, void *vs_buf, hipStream_t s);
int check_sweep_status(Graph &g, hipStream_t s);   // JSWEEP_OK, JSWEEP_E_STALLED or JSWEEP_E_PLACEMENT
int persistent_waves(Graph &g, bool fp32, const jsweep_params *p, int *waves_per_block, int groups = 0,
                     bool sg = false);
int sweep_strategy(const Graph &g, const jsweep_params *p);

// patch-task sweep (patch.hip): program built on first use; false when the
// graph does not fit the patch limits (the caller then uses another kernel)
bool patch_ready(Graph &g, hipStream_t s);
void patch_den(Graph &g, hipStream_t s);
void launch_patch64(Graph &g, const double *src_cell, double *psi, double psi_b, const jsweep_params *p,
                    hipStream_t s, bool prepared = false);

// Batched data-driven sweep (sweep.hip): the work lists of several graphs
// merged into one, so that every instance and direction of a batch is
// swept by one launch of the data-driven kernel.  Stream x of the union
// holds the chunks of stream x of every instance, ordered by (level,
// instance, chunk) -- a topological order of every instance at once.  Cell
// ids in the union's chunk blocks are global (the instance's first cell
// added), direction fields are global directions (the instance's first
// direction added), lagged-edge codes index the union's lagged-value array;
// each global direction's row (DirRow) gives its arrays.  The structure
// depends only on the graphs' programs and is cached (one batch at a
// time); denominators, rows and sources are refreshed per solve.
struct UnionSweep {
    std::vector<uint64_t> key;           // (uid, program version) of every instance, then the precision
    bool fp32 = false;
    int n = 0, ns = 0, n_cu = 0, total_dirs = 0;
    int64_t n_chunks = 0, C = 0, A = 0, LG = 0;
    std::vector<int64_t> coff, aoff, loff;        // per instance: first cell, vertex, lagged edge
    std::vector<int32_t> dir_off;                 // per instance: first global direction
    std::vector<int64_t> stream_off_h;
    DevBuf uinst, uchunk, isrc, cblk, pcode, pa, pden, stream_off, rows, status, lag, vs, pk;
    DevBuf pos[2];
    int pos_state[2] = {0, 0}, cur = 0;   // element size of the empty markers each array holds (0: none)
    // The compacted list: the chunks of the instances still iterating, in
    // the same order and layout as the full list (program stride 64 *
    // n_chunks); launch() walks it while `compacted`.  Its launches keep
    // the markers of the listed chunks only, so going back to the full list
    // (expand) refills them on its next launch.
    DevBuf c_cblk, c_pcode, c_pa, c_pden, c_pk, c_stream_off, c_flag, c_scan, c_tmp;
    int64_t c_chunks = 0;
    bool compacted = false;
    void compact(const int32_t *active, hipStream_t s);
    void expand();
    Graph *prof = nullptr;               // the batch's first graph: its jsweep_profile records the launches
    void build(int n, Graph *const *graphs, bool fp32, hipStream_t s);
    void refresh_den(Graph *const *graphs, hipStream_t s);
    // rows: per instance its cell-order flux array (psi_row base), FP32
    // per-direction source (src_row base, or null) and boundary inflow
    void set_rows(Graph *const *graphs, void *const *psi, const float *const *src_dir, const double *psi_b,
                  hipStream_t s);
    // the current level-position array holds the empty marker (before a
    // capture: the captured launches keep the alternation consistent)
    void fill_current(hipStream_t s);
    void launch(const int32_t *active, int waves_per_block, hipStream_t s);
    // the level-position array the last launch filled (instance i's flux
    // of direction m and cell K at aoff[i] + m nc + posi[m nc + K])
    const void *last_pos() const { return pos[1 - cur].p; }
    int check_status(hipStream_t s);
};
// packed codes (kPkBits) of a 3-slot program into pk [64 * n_chunks], with
// the escaped codes as entries of the chunk blocks; false (pk unusable)
// when a chunk has more than kPkEscMax escaped codes
bool pack_codes(int32_t *cblk, int64_t n_chunks, int ns, const int32_t *code, uint64_t *pk, hipStream_t s);
// the cached union of these graphs (rebuilt when any of them changed)
UnionSweep &union_for(int n, Graph *const *graphs, bool fp32, hipStream_t s);
// drops the cached union if it holds this graph
void union_forget(uint64_t uid);
uint64_t next_graph_uid();

// batched sweep over an ensemble of graphs: one workgroup per
// (instance, direction), one launch (sweep.hip)
struct BatchSweep {
    DevBuf inst, task_inst, task_dir;
    int64_t n_tasks = 0;
    int threads = 256;
    bool fp32 = false;
    bool ring = false;                   // LDS-window kernel (every instance fits its limits)
    // strategy: JSWEEP_STRATEGY_DIRECTION forces the plain direction kernel;
    // otherwise the LDS-window kernel is used where every instance fits it
    void setup(int32_t n, Graph *const *graphs, bool fp32, const void *const *src_cell, const float *const *src_dir,
               void *const *psi, const double *psi_b, int threads, int strategy, hipStream_t s);
    void launch(const int32_t *active, hipStream_t s);
};

// solve (solve.hip)
int solve(Graph &g, const double *sigma_t, const double *sigma_s, const double *q, double psi_b, int32_t mode,
          double tol, int32_t max_iter, const jsweep_params *params, double *phi, double *psi,
          jsweep_solve_stats *stats, hipStream_t s);
void scalar_flux(Graph &g, const double *psi, double *phi, hipStream_t s);
void lag_snapshot64(Graph &g, const double *psi, hipStream_t s);
// jsweep_sweep without device allocation (noalloc.hip)
int sweep_noalloc(Graph &g, const double *sigma_t, const double *source, double *psi, double *phi, double psi_b,
                  hipStream_t s);
int64_t noalloc_max_cells();
int solve_groups(Graph &g, int G, const double *sigma_t, const double *sigma_s, const double *q, double psi_b,
                 double tol, int32_t max_iter, const jsweep_params *params, double *phi, double *psi,
                 jsweep_solve_stats *stats, hipStream_t s);
int solve_batch(int32_t n, Graph *const *graphs, const jsweep_problem *problems, int32_t mode, double tol,
                int32_t max_iter, const jsweep_params *params, jsweep_solve_stats *stats, hipStream_t s);

int autotune(int32_t n, Graph *const *graphs, int32_t mode, jsweep_params *out);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace jsw
