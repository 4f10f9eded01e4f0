// Persistent data-driven transport sweep (gfx950).
//
// Work list: chunks of up to 64 vertices (cell, direction) of one level of
// one direction.  Directions are dealt to kStreams streams; within a stream
// the chunks follow a priority order that is a topological order of all of
// the stream's directions at once (by default PACED: level over the
// direction's level count), so every direction is in flight together
// (patch-angle parallelism, paper Sec. V-B).
//
// Coarsened graph (paper Sec. V-E): a chunk is a cluster of vertices and the
// work list is ordered by the clusters' graph (the union of their vertices'
// upwind edges, lagged edges excluded).  Clusters of one level of an acyclic
// graph give an acyclic coarsened graph (Theorem 1), and every upwind chunk
// of a chunk comes earlier in its stream.  A chunk starts as soon as the
// upwind fluxes of its own vertices are complete, which implies nothing
// about the rest of the upwind chunks: the wait is per vertex, the order per
// cluster.
//
// Data: a chunk's lanes read the sweep program (common.hpp) at c * 64 +
// lane -- inflow-face codes (packed where they fit) and coefficients,
// denominator -- as coalesced streams; the scattered accesses are the
// cell's V s and the upwind fluxes (and the cell-order flux store when a
// caller asks for one).  Cell records are not read at all.
//
// Execution: a persistent grid of a few workgroups per CU.  A running
// wavefront takes chunks of its stream (workgroup id mod kStreams, which is
// also the XCD the workgroup runs on) with atomic tickets, polls the upwind
// fluxes of its vertices until all of them are there, then computes one
// vertex per lane and stores the fluxes.  While it polls, the program of
// its next chunk is already on the way, and the ticket after that too, so
// a chunk costs the wavefront one memory round trip when its inputs are
// ready.  Only running wavefronts hold chunks, every wavefront walks its
// stream in order, and what it holds beyond the chunk it works on comes
// later in the stream; so the first unfinished chunk of a stream is always
// being worked on and has all of its inputs: the sweep cannot deadlock on
// an acyclic graph however many workgroups are resident.  A watchdog turns
// anything else into an error instead of a hang.
//
// Completion.  The level-ordered flux array is its own completion flag:
// before a sweep every entry holds an empty marker (a signalling-NaN bit
// pattern that no arithmetic produces), and a flux is ready once its entry
// holds anything else.  Two such arrays alternate between sweeps; while a
// sweep fills one, it writes the marker into the same entries of the other,
// so the next sweep starts from an empty array without a separate pass.  A
// consumer therefore waits on the data it needs with the loads that fetch
// it, and a producer publishes with the store of the value itself: one
// memory round trip per dependency instead of a flag poll, a flux load and
// a store acknowledgement.  Every entry is one naturally aligned 4- or
// 8-byte store and load, so a reader sees either the marker or the whole
// value.  FP64 sweeps whose fluxes are all non-negative carry a tag in the
// sign bit instead and write no markers (kSignBit).
//
// Memory ordering across compute units.  Every hand-off stays inside one
// XCD: a chunk's upwind chunks are in its own stream, and the workgroups of
// a stream (ids congruent mod 8) are dispatched to the same XCD (workgroups
// go round robin over the XCDs of the partition, and 1, 2, 4 or 8 XCDs all
// divide 8), whose L2 is then the point of coherence.  Producers store with ordinary (L1
// write-through) stores; consumers poll with device-scope loads, which
// bypass L1 and read L2.  No L2 writeback or invalidate is needed.  Within a
// kernel the L2s of different XCDs are not coherent for these accesses (a
// plain store on one XCD was never seen by device-scope polls on another in
// a two-wavefront test, while a same-XCD hand-off took 0.2 us), so the
// stream-to-XCD pinning is what makes the hand-off work; between kernels
// the runtime's cache maintenance makes every result visible.
#include <cstring>

#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <cstdlib>
#include <limits>

#include <rocprim/device/device_scan.hpp>

#include "common.hpp"

namespace jsw {

template <class Real>
struct SweepArgs {
    const int32_t *cblk;                     // [n_chunks * kBlock] chunk blocks
    int64_t nc;
    int64_t stride;                          // 64 * n_chunks: program slot stride
    const int32_t *pcode;                    // [ns * stride]
    const uint64_t *pk;                      // [stride] packed codes (NS <= 3), or null: pcode
    const Real *pa;                          // [ns * stride]
    const Real *pden;                        // [stride]
    const void *vs;                          // [nc] V s per cell (float in the FP32 sweep)
    const float *src_dir;                    // [nd*nc] or null (FP32 path)
    Real *psi;                               // [nd*nc] by cell
    Real *psi_pos;                           // [nd*nc] by level position: this sweep's fluxes (upwind reads)
    Real *pos_next;                          // [nd*nc] the other level-position array, emptied for the next sweep
    int32_t *status;                         // [0]: stalled flag
    uint32_t *tickets;                       // per-stream counters, 128 B apart
    const int64_t *stream_off;               // [kStreams + 1] chunk range of each stream
    const Real *lag_val;
    Real psi_b;
    int32_t grab;                            // chunks taken per ticket
    uint32_t nap;                            // s_sleep units between input polls
    uint32_t backoff;                        // the pause doubles every 8 polls, at most this many times
    uint64_t watchdog_ticks;
    uint32_t *stamps;                        // tracing: [3 * n_chunks] or null
    // energy groups swept together (multigroup kernels, NG > 1): the
    // level-position arrays, the lagged values and V s keep the groups of
    // one entry adjacent (entry e of group g at e n_groups + g), so that one
    // segment holds a face's upwind fluxes of every group; the cell-order
    // fluxes and the denominators are group-major, at these strides
    int32_t n_groups;
    int64_t gs_pos;                          // psi (cell order): nd * nc
    int64_t gs_den;                          // pden: stride (64 * n_chunks)
    // union of several graphs (batched sweep): a chunk's direction field is
    // a global direction whose row locates its arrays; null for one graph
    const DirRow *rows;
    const int32_t *active;                   // per instance: chunks of inactive ones only empty their entries
    uint64_t tag;                            // sign-tagged sweeps: this sweep's sign bit (kSignBit or 0)
};

template <class T>
__device__ __forceinline__ T ld_coherent(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Empty marker of the level-position flux arrays: signalling NaNs, which
// no arithmetic result equals (a NaN result is always quiet)
constexpr uint64_t kEmpty64 = 0x7ff5a5a5a5a5a5a5ull;
constexpr uint32_t kEmpty32 = 0x7fa5a5a5u;
template <class Real>
__device__ __forceinline__ Real empty_marker() {
    if constexpr (sizeof(Real) == 8) return __builtin_bit_cast(double, kEmpty64);
    else return __builtin_bit_cast(float, kEmpty32);
}
__device__ __forceinline__ bool is_empty(double v) { return __builtin_bit_cast(uint64_t, v) == kEmpty64; }
__device__ __forceinline__ bool is_empty(float v) { return __builtin_bit_cast(uint32_t, v) == kEmpty32; }

// Sign-tagged fluxes (FP64 sweeps of solves whose inputs are all
// non-negative, so that every flux is): a stored flux carries the sweep's
// tag in its sign bit, and the tag alternates between the sweeps that fill
// one array.  A value the array's previous sweep left there, and the empty
// marker (sign bit clear; an array holding markers is next filled with the
// sign bit set), read as not yet computed, so no sweep writes markers for
// the next one.  Readers take the magnitude.
constexpr uint64_t kSignBit = 0x8000000000000000ull;
__device__ __forceinline__ double with_tag(double v, uint64_t tag) {
    return __builtin_bit_cast(double, (__builtin_bit_cast(uint64_t, v) & ~kSignBit) | tag);
}
__device__ __forceinline__ double untag(double v) {
    return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, v) & ~kSignBit);
}
template <bool SG, class Real>
__device__ __forceinline__ bool not_ready(Real v, uint64_t tag) {
    if constexpr (SG) return (__builtin_bit_cast(uint64_t, v) & kSignBit) != tag;
    else return is_empty(v);
}

template <class Real>
__global__ void k_fill_empty(Real *p, int64_t n) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) p[i] = empty_marker<Real>();
}

// Omega . S of local face j, evaluated left to right.  The FP32 path takes
// the FP64 value whenever the FP32 result is too close to zero for its sign
// to be certain, so both paths agree on which faces are inflow/outflow.
template <class Real, int NF, int DIM>
__device__ __forceinline__ Real face_dot(const CellRec<Real, NF, DIM> &r, int j, const Real *om,
                                         const CellRec<double, NF, DIM> *rec64, int64_t K, const double *om64) {
    Real d = om[0] * r.S[j][0] + om[1] * r.S[j][1];
    if constexpr (DIM == 3) d = d + om[2] * r.S[j][2];
    if constexpr (sizeof(Real) == 4) {
        float mag = fabsf(om[0] * r.S[j][0]) + fabsf(om[1] * r.S[j][1]);
        if constexpr (DIM == 3) mag = mag + fabsf(om[2] * r.S[j][2]);
        if (fabsf(d) <= 2e-6f * mag) {
            const double *S = rec64[K].S[j];
            double e = om64[0] * S[0] + om64[1] * S[1];
            if constexpr (DIM == 3) e = e + om64[2] * S[2];
            d = (float)e;
            if (e != 0.0 && d == 0.0) d = e > 0.0 ? 1e-38f : -1e-38f;
        }
    }
    return d;
}

// A chunk's part of the sweep program as one lane holds it
template <class Real, int NS, int NG = 1>
struct LaneProg {
    int32_t item;                            // cell, or -1 past the chunk's end
    int32_t w2;                              // descriptor word (lanes 0 .. 31)
    Real den[NG];                            // one denominator per energy group
    int32_t code[NS];
    uint64_t pk;                             // packed codes, decoded into code[] when the chunk starts
    Real af[NS];
};

template <bool PK, class Real, int NS, int NG>
__device__ __forceinline__ void load_prog(const SweepArgs<Real> &a, int64_t c, int lane, LaneProg<Real, NS, NG> &P) {
    // read once per sweep: streamed past the caches (non-temporal), which
    // leaves L2 to the fluxes being handed off and merged
    const int32_t *blk = a.cblk + c * kBlock;
    P.item = __builtin_nontemporal_load(blk + lane);
    P.w2 = lane < 32 ? __builtin_nontemporal_load(blk + 64 + lane) : -1;
    const int64_t idx = c * 64 + lane;
#pragma unroll
    for (int g = 0; g < NG; ++g)
        P.den[g] = (g == 0 || g < a.n_groups) ? __builtin_nontemporal_load(a.pden + g * a.gs_den + idx) : Real(1);
    if constexpr (PK) {
        P.pk = __builtin_nontemporal_load(a.pk + idx);
    } else {
#pragma unroll
        for (int j = 0; j < NS; ++j) P.code[j] = __builtin_nontemporal_load(a.pcode + j * a.stride + idx);
    }
#pragma unroll
    for (int j = 0; j < NS; ++j) P.af[j] = __builtin_nontemporal_load(a.pa + j * a.stride + idx);
}

// code[] of a chunk whose program came packed: the upwind level position
// is the vertex's own one minus the stored distance; escaped codes are
// entries of the chunk block, which the descriptor lanes already hold
template <class Real, int NS, int NG>
__device__ __forceinline__ void unpack_codes(LaneProg<Real, NS, NG> &P, int64_t pos0, int lane) {
    static_assert(NS <= 3, "packed codes hold 3 slots");
#pragma unroll
    for (int j = 0; j < NS; ++j) {
        const uint32_t f = (uint32_t)(P.pk >> (kPkBits * j)) & kPkMask;
        P.code[j] = f == kPkNoFace ? kNoFace : f == kPkBound ? -1 : (int32_t)(pos0 + lane - (int64_t)f);
    }
    const int ne = __builtin_amdgcn_readlane(P.w2, 1);
    for (int e = 0; e < ne; ++e) {
        const uint32_t w0 = (uint32_t)__builtin_amdgcn_readlane(P.w2, 6 + 2 * e);
        const int32_t cd = __builtin_amdgcn_readlane(P.w2, 7 + 2 * e);
        if (lane == (int)(w0 & 63u)) {
#pragma unroll
            for (int j = 0; j < NS; ++j)
                if ((int)(w0 >> 8) == j) P.code[j] = cd;
        }
    }
}

// Multigroup FP64 kernels with an even group count store an entry's
// groups two at a time
typedef double Dbl2 __attribute__((ext_vector_type(2)));
template <class Real, int NG>
constexpr bool kPairStores = NG > 1 && NG % 2 == 0 && sizeof(Real) == 8;

// Keeps values in registers up to this point.  A store's data and address
// registers may only be reused once the store has completed; values kept
// live until the next chunk's poll has waited for everything (and with it
// for these stores) leave the compiler no store to wait for earlier.
template <class T>
__device__ __forceinline__ void keep_live(const T &v) {
    asm volatile("" ::"v"(v));
}

// NS: inflow slots per vertex in the program arrays (the program's ns, up to
// the faces per cell, or kCompactSlots for the compact program); NSX: slots
// past NS that the compact program keeps in the chunk blocks (0: none);
// TRACE: record take / ready / done stamps per chunk; NG: energy groups
// swept per chunk (multigroup: a.n_groups <= NG groups share the chunk's
// program, each with its own denominator, source and fluxes); PK: the
// upwind positions come packed (a.pk, see kPkBits); SG: the fluxes are
// sign-tagged with a.tag (see kSignBit) and no empty markers are written.
template <class Real, int NS, int NSX, bool TRACE, int NG = 1, bool PK = false, bool SG = false>
__global__ void k_sweep(SweepArgs<Real> a) {
    constexpr int NX = NSX > 0 ? NSX : 1;
    static_assert(NG == 1 || (NSX == 0 && sizeof(Real) == 8), "multigroup sweeps read the full FP64 program");
    static_assert(!PK || (NS <= 3 && NSX == 0), "packed codes hold 3 slots and no compact entries");
    static_assert(!SG || (sizeof(Real) == 8 && !TRACE), "sign tags are FP64 untraced work-list sweeps");
    const int lane = threadIdx.x & 63;
    const int stream = (int)(blockIdx.x % kStreams);
    // a wavefront off its stream's XCD takes no chunk (it holds nothing
    // anyone waits for) and raises the placement flag
    if (!check_stream_placement(a.tickets + 32 * stream + kXccSlot, a.status)) return;
    const int64_t first = a.stream_off[stream];
    const int64_t per_stream = a.stream_off[stream + 1] - first;
    const int ng = NG == 1 ? 1 : a.n_groups;
    // tickets: each is a range of a.grab consecutive chunks of the stream.
    // A wavefront holds its current chunk, the next one (whose program is
    // loaded while the current one waits for its inputs) and one requested
    // range beyond that, so neither the ticket nor the program load is a
    // round trip of its own.
    uint32_t *ticket = a.tickets + 32 * stream;
    uint32_t nxt = 0;
    if (lane == 0) nxt = atomicAdd(ticket, (uint32_t)a.grab);
    int64_t t = (int64_t)__builtin_amdgcn_readfirstlane(nxt);
    int64_t t_end = t + a.grab;
    if (lane == 0) nxt = atomicAdd(ticket, (uint32_t)a.grab);
    if (t >= per_stream) return;
    LaneProg<Real, NS, NG> P;
    load_prog<PK>(a, first + t, lane, P);
    uint32_t t_take = (uint32_t)__builtin_amdgcn_s_memrealtime();
    int64_t pend = (int64_t)__builtin_amdgcn_readfirstlane(nxt);   // start of the requested range
    __builtin_amdgcn_s_waitcnt(0);   // the loop starts with nothing in flight
    // the previous chunk's stores: value and addresses (kept live, see keep_live)
    Real out = Real(0);
    Real *at_pos = nullptr, *at_cell = nullptr, *at_next = nullptr;
    uint32_t t_done = 0, t_ready = 0;
    // every lane stays in this loop until the wavefront leaves it as a whole
    // (tickets, the input poll and abort are wave-uniform)
    while (true) {
        const int64_t c = first + t;
        // next chunk: the rest of this range, else the requested range (and
        // a new request, read back once this chunk's loads have returned)
        int64_t tn = t + 1, tn_end = t_end;
        const bool request = tn == t_end;
        if (request) {
            tn = pend;
            tn_end = tn + a.grab;
            if (lane == 0) nxt = atomicAdd(ticket, (uint32_t)a.grab);
        }
        LaneProg<Real, NS, NG> Pn;
        uint32_t tn_take = 0;
        if (tn < per_stream) {
            load_prog<PK>(a, first + tn, lane, Pn);
            tn_take = (uint32_t)__builtin_amdgcn_s_memrealtime();
        }
        const uint32_t hdr = (uint32_t)__builtin_amdgcn_readfirstlane(P.w2);
        const int64_t pos0 = (int64_t)(uint32_t)__builtin_amdgcn_readlane(P.w2, 2);
        const int m = (int)(hdr & 0xffffu);
        if constexpr (PK) unpack_codes(P, pos0, lane);
        bool active = P.item >= 0;
        const int64_t K = active ? (int64_t)P.item : 0;
        // where direction m's arrays start: m nc for one graph, the
        // direction's row for a union of graphs
        int64_t base = (int64_t)m * a.nc;
        Real *cell_row = a.psi ? a.psi + base : nullptr;
        int64_t cell_k = K;
        const float *src_row = a.src_dir ? a.src_dir + base : nullptr;
        Real psi_b = a.psi_b;
        // union of graphs: the direction's first level position and the
        // instance come with the chunk block (words 67 - 69), so the polls
        // below need nothing else; the rest of the direction's row (output
        // and source rows) is only used after them.  Whether the instance
        // still iterates is loaded together with the first poll.
        int act_flag = 1;
        if (a.rows) {
            base = (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readlane(P.w2, 4) << 32) |
                             (uint64_t)(uint32_t)__builtin_amdgcn_readlane(P.w2, 3));
            const int inst = __builtin_amdgcn_readlane(P.w2, 5);
            if (a.active) act_flag = a.active[inst];
            const DirRow row = a.rows[m];
            cell_row = static_cast<Real *>(row.psi_row);
            cell_k = K - row.cell_off;
            src_row = row.src_row;
            psi_b = (Real)row.psi_b;
        }
        const int64_t own = base + pos0 + lane;
        // entry stride of the level-position, lagged-value and V s arrays
        // (the groups of an entry adjacent)
        const int64_t gm = NG > 1 ? (int64_t)ng : 1;
        // V s of the cell (one gather of the cell's groups; in FP32 one
        // float, to which the per-direction source, V r, is added after the
        // poll, so that nothing waits for these loads before it)
        Real num[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) num[g] = Real(0);
        float vs32 = 0.0f;
        float sd32 = 0.0f;
        if (active) {
            if constexpr (sizeof(Real) == 8) {
                const double *vk = reinterpret_cast<const double *>(a.vs) + K * gm;
                if constexpr (kPairStores<Real, NG>) {
                    if (ng == NG) {
#pragma unroll
                        for (int h = 0; h < NG / 2; ++h) {
                            const Dbl2 x = reinterpret_cast<const Dbl2 *>(vk)[h];
                            num[2 * h] = x.x;
                            num[2 * h + 1] = x.y;
                        }
                    } else {
#pragma unroll
                        for (int g = 0; g < NG; ++g)
                            if (g < ng) num[g] = vk[g];
                    }
                } else {
#pragma unroll
                    for (int g = 0; g < NG; ++g)
                        if (g < ng) num[g] = vk[g];
                }
            } else {
                vs32 = reinterpret_cast<const float *>(a.vs)[K];
                if (src_row) sd32 = __builtin_nontemporal_load(src_row + pos0 + lane);   // read once per sweep
            }
        }
        // upwind fluxes: interior and lagged ones are loaded together (one
        // device-scope load per slot and group, issued only by the lanes
        // whose slot has such a face).  The loads are repeated until no
        // interior slot of any lane holds the empty marker; polls that keep
        // failing back off.
        const Real *from[NS];
        bool want[NS];
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            const int32_t cd = P.code[j];
            const bool lagged = cd <= -2 && cd != kNoFace;
            want[j] = cd >= 0 || lagged;
            from[j] = cd >= 0 ? a.psi_pos + (base + cd) * gm
                      : lagged ? a.lag_val + (-(int64_t)cd - 2) * gm
                               : a.psi_pos + own * gm;
        }
        // the compact program's further slots: the chunk's few entries
        // (descriptor lanes 3 ..) go to their lanes
        int32_t code_x[NX];
        Real af_x[NX], val_x[NX];
        const Real *from_x[NX];
        int nx = 0;
#pragma unroll
        for (int k = 0; k < NX; ++k) {
            code_x[k] = kNoFace;
            af_x[k] = Real(0);
            val_x[k] = Real(0);
            from_x[k] = a.psi_pos + own;
        }
        if constexpr (NSX > 0) {
            nx = __builtin_amdgcn_readlane(P.w2, 1);
            for (int e = 0; e < nx; ++e) {
                const uint32_t w0 = (uint32_t)__builtin_amdgcn_readlane(P.w2, 3 + 4 * e);
                const int32_t cd = __builtin_amdgcn_readlane(P.w2, 4 + 4 * e);
                const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane(P.w2, 5 + 4 * e);
                const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane(P.w2, 6 + 4 * e);
                if (lane == (int)(w0 & 63u)) {
                    const int k = (int)(w0 >> 8) - NS;
#pragma unroll
                    for (int kk = 0; kk < NX; ++kk)
                        if (k == kk) {
                            code_x[kk] = cd;
                            af_x[kk] = (Real)__builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
                        }
                }
            }
#pragma unroll
            for (int k = 0; k < NX; ++k) {
                const int32_t cd = code_x[k];
                const bool lagged = cd <= -2 && cd != kNoFace;
                from_x[k] = cd >= 0 ? a.psi_pos + base + cd : lagged ? a.lag_val + (-(int64_t)cd - 2) : a.psi_pos + own;
            }
        }
        Real val[NG][NS];
        uint64_t t0 = 0;
        for (uint32_t spin = 0;; ++spin) {
            bool ok = true;
            if (active) {
#pragma unroll
                for (int g = 0; g < NG; ++g)
                    if (g < ng) {
#pragma unroll
                        for (int j = 0; j < NS; ++j) val[g][j] = want[j] ? ld_coherent(from[j] + g) : Real(0);
                    }
                if constexpr (NSX > 0) {
                    if (nx > 0) {
#pragma unroll
                        for (int k = 0; k < NX; ++k) val_x[k] = ld_coherent(from_x[k]);
                    }
                }
#pragma unroll
                for (int g = 0; g < NG; ++g)
                    if (g < ng) {
#pragma unroll
                        for (int j = 0; j < NS; ++j) ok = ok && !(P.code[j] >= 0 && not_ready<SG>(val[g][j], a.tag));
                    }
#pragma unroll
                for (int k = 0; k < NX; ++k) ok = ok && !(code_x[k] >= 0 && not_ready<SG>(val_x[k], a.tag));
            }
            if (!__builtin_amdgcn_readfirstlane(act_flag)) break;   // an instance that no longer iterates
            if (__all(ok)) break;
            if (spin == 0) t0 = __builtin_amdgcn_s_memrealtime();
            if ((spin & 7) == 7) {
                bool stop = ld_coherent(a.status) != 0;
                if (!stop && __builtin_amdgcn_s_memrealtime() - t0 > a.watchdog_ticks) {
                    if (lane == 0) atomicOr(a.status, kStatusStalled);
                    stop = true;
                }
                // the wavefront ends here (no barrier in this kernel); an
                // end of program instead of a jump to the loop's exit keeps
                // this path's loads in flight out of the loop's other paths
                if (__any(stop)) __builtin_amdgcn_endpgm();
            }
            const uint32_t naps = a.nap << min(spin >> 3, a.backoff);
            for (uint32_t z = 0; z < naps; ++z) __builtin_amdgcn_s_sleep(1);
        }
        // every load issued so far has returned, and with them the previous
        // chunk's stores (the poll waited for them, on every path): said
        // explicitly, so that nothing after this chunk's stores waits for
        // them (memory counters retire in order)
        __builtin_amdgcn_s_waitcnt(0);
        keep_live(out);
        keep_live(at_pos);
        keep_live(at_cell);
        keep_live(at_next);
        if constexpr (TRACE) {
            keep_live(t_ready);
            keep_live(t_done);
        }
        t_ready = (uint32_t)__builtin_amdgcn_s_memrealtime();
        if (request) pend = (int64_t)__builtin_amdgcn_readfirstlane(nxt);
        if (!__builtin_amdgcn_readfirstlane(act_flag)) {
            // a chunk of an instance that no longer iterates computes
            // nothing; it only empties its entries of the next sweep's array
            // (the instance may iterate again then)
            if (active) __builtin_nontemporal_store(empty_marker<Real>(), a.pos_next + own);
            active = false;
        }
        at_pos = a.psi_pos + own * gm;
        at_cell = cell_row ? cell_row + cell_k : nullptr;
        at_next = a.pos_next + own * gm;
        Real og[NG];
        if constexpr (SG) {
#pragma unroll
            for (int g = 0; g < NG; ++g)
#pragma unroll
                for (int j = 0; j < NS; ++j) val[g][j] = untag(val[g][j]);
#pragma unroll
            for (int k = 0; k < NX; ++k) val_x[k] = untag(val_x[k]);
        }
        if (active) {
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                if (g >= ng) continue;
                Real ng_num = num[g];
                if constexpr (sizeof(Real) == 4) ng_num = src_row ? sd32 + vs32 : vs32;
                // step-scheme balance, inflow faces in local face order
#pragma unroll
                for (int j = 0; j < NS; ++j) {
                    const int32_t cd = P.code[j];
                    const bool lagged = cd <= -2 && cd != kNoFace;
                    const Real v = (cd >= 0 || lagged) ? val[g][j] : (cd == -1 ? psi_b : Real(0));
                    if (cd != kNoFace) ng_num = ng_num + P.af[j] * v;
                }
                if constexpr (NSX > 0) {
#pragma unroll
                    for (int k = 0; k < NX; ++k) {
                        const int32_t cd = code_x[k];
                        const bool lagged = cd <= -2 && cd != kNoFace;
                        const Real v = (cd >= 0 || lagged) ? val_x[k] : (cd == -1 ? psi_b : Real(0));
                        if (cd != kNoFace) ng_num = ng_num + af_x[k] * v;
                    }
                }
                Real o = ng_num / P.den[g];
                // a NaN carrying the marker's bits (never produced by
                // arithmetic) would read as not yet computed
                if (is_empty(o)) o = std::numeric_limits<Real>::quiet_NaN();
                // the cell-order copy (when the caller wants one) is read
                // only after the kernel
                if (cell_row) at_cell[g * a.gs_pos] = o;
                if constexpr (SG) o = with_tag(o, a.tag);
                // the level-order store publishes the flux
                if constexpr (kPairStores<Real, NG>) {
                    og[g] = o;   // stored below, two groups at a time
                } else {
                    at_pos[g] = o;
                    if constexpr (!SG) __builtin_nontemporal_store(empty_marker<Real>(), at_next + g);   // read in the next sweep
                }
                if (g == 0) out = o;
            }
            if constexpr (kPairStores<Real, NG>) {
                // an entry's groups are adjacent: with every group slot in
                // use they are 16-byte aligned pairs, each published by one
                // 16-byte store (its 8-byte halves are written whole)
                if (ng == NG) {
#pragma unroll
                    for (int h = 0; h < NG / 2; ++h) {
                        reinterpret_cast<Dbl2 *>(at_pos)[h] = Dbl2{og[2 * h], og[2 * h + 1]};
                        if constexpr (!SG)
                            __builtin_nontemporal_store(Dbl2{empty_marker<Real>(), empty_marker<Real>()},
                                                        reinterpret_cast<Dbl2 *>(at_next) + h);
                    }
                } else {
#pragma unroll
                    for (int g = 0; g < NG; ++g)
                        if (g < ng) {
                            at_pos[g] = og[g];
                            if constexpr (!SG) __builtin_nontemporal_store(empty_marker<Real>(), at_next + g);
                        }
                }
            }
        }
        if constexpr (TRACE) {
            t_done = (uint32_t)__builtin_amdgcn_s_memrealtime();
            if (lane == 0) {
                a.stamps[3 * c] = t_take;
                a.stamps[3 * c + 1] = t_ready;
                a.stamps[3 * c + 2] = t_done;
            }
        }
        if (tn >= per_stream) break;
        t = tn;
        t_end = tn_end;
        P = Pn;
        t_take = tn_take;
    }
}

// ---------------------------------------------------------------------------
// Direction-parallel sweep: one workgroup per direction walks the
// direction's levels in order, all lanes of the workgroup sharing each
// level's vertices, with a workgroup barrier between levels.  Upwind fluxes
// were written by the same workgroup (same compute unit) at an earlier
// level, so they are read back through the compute unit's own L1/L2 and no
// vertex ever waits on another compute unit.  The levels are a topological
// order of the direction's graph, so the sweep needs no flags at all; many
// directions (and batch instances) run side by side, one per compute unit.
// ---------------------------------------------------------------------------
template <class Real, int NF, int DIM>
struct DirArgs {
    const CellRec<Real, NF, DIM> *rec;
    const CellRec<double, NF, DIM> *rec64;
    const int32_t *lvl_cells;
    const int64_t *lvl_ptr;                  // concatenated level pointers
    const int64_t *lvl_off;                  // [nd + 1] block of each direction
    int64_t nc;
    const Real *omega;
    const double *omega64;
    const Real *src_cell;
    const float *src_dir;
    Real *psi;
    const uint64_t *lag_mv;
    const int32_t *lag_u;
    const Real *lag_val;
    int64_t n_lag;
    Real psi_b;
};

// Sweep of direction m by one workgroup: the lanes share each level's
// vertices; a barrier separates levels.
template <class Real, int NF, int DIM>
__device__ void sweep_direction(const DirArgs<Real, NF, DIM> &a, int m) {
    const int64_t base = (int64_t)m * a.nc;
    const int64_t *ptr = a.lvl_ptr + a.lvl_off[m];
    const int nlev = (int)(a.lvl_off[m + 1] - a.lvl_off[m] - 1);
    const Real om[3] = {a.omega[3 * m], a.omega[3 * m + 1], DIM == 3 ? a.omega[3 * m + 2] : Real(0)};
    const double *om64 = a.omega64 + 3 * m;
    for (int L = 0; L < nlev; ++L) {
        const int64_t end = ptr[L + 1];
        for (int64_t i = ptr[L] + threadIdx.x; i < end; i += blockDim.x) {
            const int64_t K = a.lvl_cells[base + i];
            const CellRec<Real, NF, DIM> r = a.rec[K];
            Real s = Real(0);
            if (a.src_cell) s = a.src_cell[K];
            // the FP32 correction source per direction comes as V r
            Real num = r.V * s;
            if (a.src_dir) num = num + (Real)a.src_dir[base + i];
            Real den = r.sigV;
#pragma unroll
            for (int j = 0; j < NF; ++j) {
                const Real d = face_dot(r, j, om, a.rec64, K, om64);
                if (d > Real(0)) den = den + d;
                else if (d < Real(0)) {
                    const int32_t code = r.nbr[j];
                    Real up;
                    if (code == -1) up = a.psi_b;
                    else {
                        const int32_t u = code <= -2 ? -code - 2 : code;
                        const int64_t e = code <= -2 ? lag_index(a.lag_mv, a.lag_u, a.n_lag, m, K, u) : -1;
                        up = e >= 0 ? a.lag_val[e] : a.psi[base + u];
                    }
                    num = num + (-d) * up;
                }
            }
            a.psi[base + K] = num / den;
        }
        __syncthreads();
    }
}

template <class Real, int NF, int DIM>
__global__ void __launch_bounds__(1024) k_sweep_dir(DirArgs<Real, NF, DIM> a) {
    sweep_direction(a, (int)blockIdx.x);
}

// Batched sweep: one workgroup per (instance, direction) task of an
// ensemble of independent graphs, all in one launch.  Instances may differ
// in cell type; a task of a converged instance returns at once.
template <class Real>
struct BatchInst {
    const void *rec;
    const void *rec64;
    const int32_t *lvl_cells;
    const int64_t *lvl_ptr;
    const int64_t *lvl_off;
    int64_t nc;
    const Real *omega;
    const double *omega64;
    const Real *src_cell;
    const float *src_dir;
    Real *psi;
    const uint64_t *lag_mv;
    const int32_t *lag_u;
    const Real *lag_val;
    int64_t n_lag;
    Real psi_b;
    int32_t ctype;
    int32_t nd;
};

template <class Real, int NF, int DIM>
__device__ void batch_task(const BatchInst<Real> &b, int m) {
    DirArgs<Real, NF, DIM> a;
    a.rec = static_cast<const CellRec<Real, NF, DIM> *>(b.rec);
    a.rec64 = static_cast<const CellRec<double, NF, DIM> *>(b.rec64);
    a.lvl_cells = b.lvl_cells;
    a.lvl_ptr = b.lvl_ptr;
    a.lvl_off = b.lvl_off;
    a.nc = b.nc;
    a.omega = b.omega;
    a.omega64 = b.omega64;
    a.src_cell = b.src_cell;
    a.src_dir = b.src_dir;
    a.psi = b.psi;
    a.lag_mv = b.lag_mv;
    a.lag_u = b.lag_u;
    a.lag_val = b.lag_val;
    a.n_lag = b.n_lag;
    a.psi_b = b.psi_b;
    sweep_direction(a, m);
}

template <class Real>
__global__ void __launch_bounds__(1024) k_sweep_batch(const BatchInst<Real> *inst, const int32_t *task_inst,
                                                     const int32_t *task_dir, const int32_t *active) {
    const int i = task_inst[blockIdx.x];
    if (i < 0 || !active[i]) return;
    const BatchInst<Real> &b = inst[i];
    const int m = task_dir[blockIdx.x];
    if (b.ctype == JSWEEP_TRI) batch_task<Real, 3, 2>(b, m);
    else if (b.ctype == JSWEEP_TET) batch_task<Real, 4, 3>(b, m);
    else batch_task<Real, 6, 3>(b, m);
}

// ticket counters back to zero before a sweep
__global__ void k_reset_tickets(uint32_t *t) {
    if (threadIdx.x < kStreams) {
        t[32 * threadIdx.x] = 0u;
        t[32 * threadIdx.x + kXccSlot] = kNoXcc;
    }
}

static uint64_t watchdog_ticks() {
    const char *e = std::getenv("JSWEEP_WATCHDOG_MS");
    double ms = e ? std::atof(e) : 4000.0;
    if (!(ms > 0)) ms = 4000.0;
    return (uint64_t)(ms * 1e5);   // s_memrealtime runs at 100 MHz
}

// sg: sign-tagged fluxes (FP64, untraced)
template <class Real, int NS, int NSX = 0, bool PK = false>
static const void *kernel_ptr(bool trace, bool sg = false) {
    if constexpr (sizeof(Real) == 8) {
        if (sg) return reinterpret_cast<const void *>(&k_sweep<Real, NS, NSX, false, 1, PK, true>);
    }
    return trace ? reinterpret_cast<const void *>(&k_sweep<Real, NS, NSX, true, 1, PK>)
                 : reinterpret_cast<const void *>(&k_sweep<Real, NS, NSX, false, 1, PK>);
}

// pk: the program's upwind positions are packed (at most 3 slots)
template <class Real>
static const void *sweep_kernel_t(int ns, bool trace, bool pk = false, bool sg = false) {
    if (pk) {
        switch (ns) {
        case 1: return kernel_ptr<Real, 1, 0, true>(trace, sg);
        case 2: return kernel_ptr<Real, 2, 0, true>(trace, sg);
        case 3: return kernel_ptr<Real, 3, 0, true>(trace, sg);
        default: fail(JSWEEP_E_DEVICE, "packed codes with more than 3 slots");
        }
    }
    switch (ns) {
    case 1: return kernel_ptr<Real, 1>(trace, sg);
    case 2: return kernel_ptr<Real, 2>(trace, sg);
    case 3: return kernel_ptr<Real, 3>(trace, sg);
    case 4: return kernel_ptr<Real, 4>(trace, sg);
    case 5: return kernel_ptr<Real, 5>(trace, sg);
    default: return kernel_ptr<Real, 6>(trace, sg);
    }
}

// the FP64 sweep of a graph with a compact program reads kCompactSlots
// slots from the arrays and ns_x from the chunk blocks
static bool use_compact(const Graph &g, bool fp32) { return !fp32 && g.ns_x > 0; }

// the work-list sweeps read packed upwind positions where the graph has
// them (programs of at most 3 slots without compact entries)
static bool use_packed(const Graph &g, bool fp32, int groups) {
    (void)groups;
    return g.pk.p && g.ns <= 3 && !use_compact(g, fp32);
}

// multigroup FP64 kernels: NG groups per chunk, full program (its upwind
// positions packed where the graph has them)
template <int NS, int NG, bool PK>
static const void *group_kernel_ptr(bool sg) {
    return sg ? reinterpret_cast<const void *>(&k_sweep<double, NS, 0, false, NG, PK, true>)
              : reinterpret_cast<const void *>(&k_sweep<double, NS, 0, false, NG, PK>);
}
template <int NG>
static const void *sweep_kernel_groups(int ns, bool pk, bool sg) {
    if (pk) {
        switch (ns) {
        case 1: return group_kernel_ptr<1, NG, true>(sg);
        case 2: return group_kernel_ptr<2, NG, true>(sg);
        case 3: return group_kernel_ptr<3, NG, true>(sg);
        default: fail(JSWEEP_E_DEVICE, "packed codes with more than 3 slots");
        }
    }
    switch (ns) {
    case 1: return group_kernel_ptr<1, NG, false>(sg);
    case 2: return group_kernel_ptr<2, NG, false>(sg);
    case 3: return group_kernel_ptr<3, NG, false>(sg);
    case 4: return group_kernel_ptr<4, NG, false>(sg);
    case 5: return group_kernel_ptr<5, NG, false>(sg);
    default: return group_kernel_ptr<6, NG, false>(sg);
    }
}

// groups = 0: the single-group sweep (compact program where the graph has
// one); groups >= 1: the multigroup sweep over that many groups, which
// reads the full program; sg: sign-tagged fluxes (FP64, untraced: the
// caller checks)
static const void *sweep_kernel(const Graph &g, bool fp32, bool trace = false, int groups = 0, bool sg = false) {
    const int ns = g.ns;
    if (ns < 1 || ns > 6) fail(JSWEEP_E_DEVICE, "sweep program with an unsupported number of inflow slots");
    if (groups >= 1) {
        if (fp32 || trace) fail(JSWEEP_E_INVALID_ARG, "multigroup sweeps are FP64 and untraced");
        if (groups == 1) return sweep_kernel_t<double>(ns, false, use_packed(g, false, 1), sg);
        const bool pk = use_packed(g, false, groups);
        if (groups <= 2) return sweep_kernel_groups<2>(ns, pk, sg);
        if (groups <= 4) return sweep_kernel_groups<4>(ns, pk, sg);
        if (groups <= kMaxGroups) return sweep_kernel_groups<kMaxGroups>(ns, pk, sg);
        fail(JSWEEP_E_INVALID_ARG, "too many energy groups");
    }
    if (use_compact(g, fp32)) {
        static_assert(kCompactSlots == 3, "compact kernels are instantiated for 3 program slots");
        switch (g.ns_x) {
        case 1: return kernel_ptr<double, 3, 1>(trace, sg);
        case 2: return kernel_ptr<double, 3, 2>(trace, sg);
        default: return kernel_ptr<double, 3, 3>(trace, sg);
        }
    }
    const bool pk = use_packed(g, fp32, groups);
    return fp32 ? sweep_kernel_t<float>(ns, trace, pk) : sweep_kernel_t<double>(ns, trace, pk, sg);
}

constexpr int kMaxSweepBlocksPerCU = 4;

int persistent_waves(Graph &g, bool fp32, const jsweep_params *p, int *waves_per_block, int groups, bool sg) {
    // default (measured on 0.3M- to 6.6M-chunk graphs): one workgroup per
    // CU, of eight wavefronts for graphs above a million chunks (more
    // requests in flight; ten or more poll more than they gain), of five
    // below
    const int wpb_default = g.n_chunks >= (int64_t)1000000 ? 8 : 5;
    int wpb = (p && p->waves_per_block > 0) ? p->waves_per_block
              : (g.has_tuned && g.tuned.waves_per_block > 0 ? g.tuned.waves_per_block : wpb_default);
    if (wpb > 16) wpb = 16;
    // the occupancy query is answered once per (kernel, workgroup size):
    // it is not free, and a tolerance-driven solve launches one sweep at a
    // time, waiting for the last
    static std::mutex occ_mu;
    static std::map<std::pair<const void *, int>, int> occ_seen;
    const void *kern = sweep_kernel(g, fp32, false, groups, sg);
    int occ = 0;
    {
        std::lock_guard<std::mutex> lock(occ_mu);
        auto it = occ_seen.find({kern, wpb});
        if (it != occ_seen.end()) {
            occ = it->second;
        } else {
            JSW_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 64 * wpb, 0));
            occ_seen[{kern, wpb}] = occ;
        }
    }
    if (occ < 1) occ = 1;
    // at most kMaxSweepBlocksPerCU workgroups per CU: every waiting
    // wavefront polls its vertices' upwind fluxes, and with all resident
    // wavefronts polling (measured on 5.3M-cell graphs) the polls crowd out
    // the loads and stores of the chunks that could run
    int bpc = (p && p->blocks_per_cu > 0) ? p->blocks_per_cu
              : (g.has_tuned && g.tuned.blocks_per_cu > 0 ? g.tuned.blocks_per_cu : 1);
    if (bpc > kMaxSweepBlocksPerCU) bpc = kMaxSweepBlocksPerCU;
    if (bpc > occ) bpc = occ;
    *waves_per_block = wpb;
    return bpc * g.n_cu * wpb;
}

// cell volume of every program slot (0 past a chunk's end), FP64 or rounded
// to FP32 as in the FP32 sweep
template <class Real>
__global__ void k_pvol(const int32_t *cblk, int64_t stride, const double *vol, Real *pvol) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= stride) return;
    const int32_t K = cblk[(idx >> 6) * kBlock + (idx & 63)];
    pvol[idx] = K < 0 ? Real(0) : (Real)vol[K];
}

// Packed codes of chunk c (one 64-lane workgroup per chunk): the distance
// of every slot's upwind position back from the lane's own, or a reserved
// value; escaped codes go to the chunk block as entries (lane | slot << 8,
// code), and *too_many is set when a chunk has more than kPkEscMax.  The
// largest distance kept can be lowered for tests (max_delta).
__global__ void k_pack_codes(int32_t *blk, int64_t n_chunks, int ns, const int32_t *code, uint64_t *pk,
                             uint32_t max_delta, int32_t *too_many) {
    const int64_t c = blockIdx.x;
    const int lane = threadIdx.x;
    if (c >= n_chunks) return;
    const int64_t S = 64 * n_chunks, idx = c * 64 + lane;
    int32_t *b = blk + c * kBlock;
    const int64_t pos = (int64_t)b[66] + lane;
    const int cnt = (int)((uint32_t)b[64] >> 16) + 1;
    uint64_t v = 0;
    int n = 0;
    for (int j = 0; j < 3; ++j) {
        const int32_t cd = (j < ns && lane < cnt) ? code[j * S + idx] : kNoFace;
        uint32_t f = kPkEsc;
        if (cd == kNoFace) f = kPkNoFace;
        else if (cd == -1) f = kPkBound;
        else if (cd >= 0 && pos - cd >= 1 && pos - cd <= (int64_t)max_delta) f = (uint32_t)(pos - cd);
        v |= (uint64_t)f << (kPkBits * j);
        const bool esc = f == kPkEsc;
        const uint64_t mask = __ballot(esc);
        const int e = n + __popcll(mask & ((1ull << lane) - 1ull));
        if (esc && e < kPkEscMax) {
            b[70 + 2 * e] = lane | (j << 8);
            b[71 + 2 * e] = cd;
        }
        n += __popcll(mask);
    }
    pk[idx] = v;
    if (lane == 0) {
        b[65] = n;
        if (n > kPkEscMax) atomicOr(too_many, 1);
    }
}

bool pack_codes(int32_t *cblk, int64_t n_chunks, int ns, const int32_t *code, uint64_t *pk, hipStream_t s) {
    if (ns > 3 || n_chunks <= 0) return false;
    uint32_t max_delta = kPkMaxDelta;
    if (const char *e = std::getenv("JSWEEP_PACK_MAX_DELTA")) {
        const long v = std::atol(e);
        if (v >= 1 && v < (long)kPkMaxDelta) max_delta = (uint32_t)v;
    }
    DevBuf flag(4);
    JSW_HIP(hipMemsetAsync(flag.p, 0, 4, s));
    k_pack_codes<<<(unsigned)n_chunks, 64, 0, s>>>(cblk, n_chunks, ns, code, pk, max_delta, flag.as<int32_t>());
    JSW_HIP(hipGetLastError());
    int32_t too_many = 0;
    JSW_HIP(hipMemcpyAsync(&too_many, flag.p, 4, hipMemcpyDeviceToHost, s));
    JSW_HIP(hipStreamSynchronize(s));
    return too_many == 0;
}

// V s per cell for the FP64 sweep (the same product the balance takes),
// and for the FP32 sweep rounded from the FP64 product (one 4-byte gather
// per vertex instead of V and s)
__global__ void k_vs64(const double *vol, const double *src, int64_t nc, double *vs) {
    int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (K < nc) vs[K] = src ? vol[K] * src[K] : vol[K] * 0.0;
}
__global__ void k_vs32(const double *vol, const float *src, int64_t nc, float *vs) {
    int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (K < nc) vs[K] = src ? (float)(vol[K] * (double)src[K]) : 0.0f;
}

// vs_buf: where the per-cell V s of this sweep is staged (null: the
// graph's own buffer, allocated on first use); a caller-provided buffer
// also keeps the launch free of HIP event creation (no profiling); nonneg:
// every flux of this sweep is non-negative (the caller checked its inputs):
// an FP64 sweep of the full program then tags its fluxes by sign instead of
// writing empty markers (see kSignBit)
template <class Real>
static void launch_persistent(Graph &g, const Real *src_cell, const float *src_dir, Real *psi, Real psi_b,
                              const jsweep_params *p, hipStream_t s, bool prepared = false,
                              const GroupSweep *mg = nullptr, void *vs_buf = nullptr, bool nonneg = false) {
    const bool f32 = sizeof(Real) == 4;
    const int G = mg ? mg->groups : 1;
    if (mg && (f32 || !prepared)) fail(JSWEEP_E_DEVICE, "multigroup sweeps are FP64 with a prepared source");
    if (!mg && !(f32 ? g.den32_ok : g.den64_ok)) fail(JSWEEP_E_DEVICE, "sweep program denominators not built");
    SweepArgs<Real> a;
    a.cblk = g.cblk.as<int32_t>();
    a.nc = g.nc;
    a.stride = 64 * g.n_chunks;
    const bool compact = use_compact(g, f32) && !mg;   // multigroup kernels read the full program
    a.pcode = compact ? g.pcode3.as<int32_t>() : g.pcode.as<int32_t>();
    a.pk = use_packed(g, f32, mg ? G : 0) ? g.pk.as<uint64_t>() : nullptr;
    a.pa = reinterpret_cast<const Real *>(compact ? g.pa3.p : f32 ? g.pa32.p : g.pa64.p);
    a.pden = reinterpret_cast<const Real *>(f32 ? g.pden32.p : g.pden64.p);
    void *vs = vs_buf;
    if (!vs) {
        if (!prepared && g.vsc.bytes < (size_t)(8 * g.nc)) g.vsc.alloc(8 * g.nc);
        vs = g.vsc.p;
    }
    if (!prepared) {
        const int gb = (int)ceil_div(g.nc, 256);
        if (f32)
            k_vs32<<<gb, 256, 0, s>>>(g.vol.as<double>(), reinterpret_cast<const float *>(src_cell), g.nc,
                                     static_cast<float *>(vs));
        else
            k_vs64<<<gb, 256, 0, s>>>(g.vol.as<double>(), reinterpret_cast<const double *>(src_cell), g.nc,
                                     static_cast<double *>(vs));
        JSW_HIP(hipGetLastError());
    }
    a.vs = vs;
    a.src_dir = src_dir;
    a.psi = psi;
    // groups: group g's fluxes, denominators and lagged values follow group
    // 0's at these strides
    a.n_groups = G;
    a.gs_pos = g.nc * g.nd;
    a.gs_den = a.stride;
    if (mg) a.pden = reinterpret_cast<const Real *>(mg->den);
    // the two level-position arrays alternate.  A marker sweep needs the
    // empty marker of its precision in the first G nc nd entries of its
    // array (every group of every position; the previous sweep of that
    // precision left it so, otherwise it is filled here) and empties the
    // other array for the next sweep.  A sign-tagged sweep needs its array
    // to hold markers or the fluxes of its own previous G-group tagged
    // sweep, and takes the other tag; it writes no markers.  State (see
    // Graph::dd_state): element size | G << 8, plus the tag bits.
    const bool sg = nonneg && !f32 && !g.trace && !vs_buf;
    const int want = (int)sizeof(Real) | (G << 8);
    const size_t need_bytes = (size_t)8 * g.nc * g.nd * G;
    for (int i = 0; i < 2; ++i)
        if (g.dd_pos[i].bytes < need_bytes) {
            g.dd_pos[i].alloc(need_bytes);
            g.dd_state[i] = 0;
        }
    const int cur = g.dd_cur;
    const int st = g.dd_state[cur];
    bool fill = !(!(st & kDdTagged) && (st & 0xff) == (int)sizeof(Real) && ((st >> 8) & 0xff) >= G);
    bool tag_set = true;   // markers (sign bit clear) never carry a set tag
    if (sg && (st & kDdTagged) && ((st >> 8) & 0xff) == G) {
        tag_set = !(st & kDdTagSet);
        fill = false;
    }
    if (fill && g.nc * g.nd > 0) {
        const int64_t n = g.nc * g.nd * G;
        k_fill_empty<Real><<<(int)std::min<int64_t>(ceil_div(n, 256), 8192), 256, 0, s>>>(g.dd_pos[cur].as<Real>(), n);
        JSW_HIP(hipGetLastError());
    }
    a.psi_pos = g.dd_pos[cur].as<Real>();
    a.pos_next = g.dd_pos[1 - cur].as<Real>();
    if (sg) {
        a.tag = tag_set ? kSignBit : 0;
        g.dd_state[cur] = kDdTagged | (tag_set ? kDdTagSet : 0) | (G << 8) | 8;   // the other array's state stands
    } else {
        a.tag = 0;
        g.dd_state[cur] = 0;
        g.dd_state[1 - cur] = want;
    }
    g.dd_cur = 1 - cur;
    a.status = g.status.as<int32_t>();
    a.lag_val = reinterpret_cast<const Real *>(mg ? mg->lag_val : f32 ? g.lag_val32.p : g.lag_val64.p);
    a.tickets = reinterpret_cast<uint32_t *>(g.status.as<char>() + 128);
    a.stream_off = g.stream_off.as<int64_t>();
    // defaults (measured): one chunk per ticket for graphs of a few hundred
    // thousand chunks, where the critical path dominates; three for graphs
    // above a million chunks
    a.grab = (p && p->chunks_per_ticket > 0) ? p->chunks_per_ticket
             : (g.has_tuned && g.tuned.chunks_per_ticket > 0 ? g.tuned.chunks_per_ticket
                                                              : (g.n_chunks < (int64_t)1000000 ? 1 : 3));
    a.psi_b = psi_b;
    a.watchdog_ticks = watchdog_ticks();
    a.stamps = g.trace ? g.trace_buf.as<uint32_t>() : nullptr;
    a.rows = nullptr;
    a.active = nullptr;
    if (g.trace) g.trace_units = 0;
    {
        const char *e = std::getenv("JSWEEP_POLL_NAP");
        a.nap = e ? (uint32_t)std::max(1, std::atoi(e)) : 1u;
        const char *b = std::getenv("JSWEEP_POLL_BACKOFF");
        a.backoff = b ? (uint32_t)std::min(4, std::max(0, std::atoi(b))) : 3u;
    }
    int wpb = 4;
    int waves = persistent_waves(g, f32, p, &wpb, mg ? G : 0, sg);
    int64_t need = std::max<int64_t>(1, g.n_chunks);
    if (waves > need) waves = (int)((need + wpb - 1) / wpb * wpb);
    int blocks = std::max(waves / wpb, kStreams);
    if (!prepared) k_reset_tickets<<<1, 64, 0, s>>>(a.tickets);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    const bool prof = g.profile && !vs_buf;
    if (prof) {
        JSW_HIP(hipEventCreate(&ev0));
        JSW_HIP(hipEventCreate(&ev1));
        JSW_HIP(hipEventRecord(ev0, s));
    }
    void *args[] = {&a};
    if (mg) a.stamps = nullptr;
    JSW_HIP(hipLaunchKernel(sweep_kernel(g, f32, a.stamps != nullptr, mg ? G : 0, sg), dim3(blocks), dim3(64 * wpb),
                            args, 0, s));
    if (prof) {
        JSW_HIP(hipEventRecord(ev1, s));
        g.prof_events.push_back({ev0, ev1});
    }
}

template <class Real, int NF, int DIM>
static void launch_dir(Graph &g, const Real *src_cell, const float *src_dir, Real *psi, Real psi_b,
                       const jsweep_params *p, hipStream_t s) {
    DirArgs<Real, NF, DIM> a;
    a.rec = sizeof(Real) == 8 ? reinterpret_cast<const CellRec<Real, NF, DIM> *>(g.rec64.p)
                              : reinterpret_cast<const CellRec<Real, NF, DIM> *>(g.rec32.p);
    a.rec64 = g.rec64.as<CellRec<double, NF, DIM>>();
    a.lvl_cells = g.lvl_cells.as<int32_t>();
    a.lvl_ptr = g.lvl_ptr_d.as<int64_t>();
    a.lvl_off = g.lvl_off_d.as<int64_t>();
    a.nc = g.nc;
    a.omega = sizeof(Real) == 8 ? reinterpret_cast<const Real *>(g.omega64.p) : reinterpret_cast<const Real *>(g.omega32.p);
    a.omega64 = g.omega64.as<double>();
    a.src_cell = src_cell;
    a.src_dir = src_dir;
    a.psi = psi;
    a.lag_mv = g.lag_mv.as<uint64_t>();
    a.lag_u = g.lag_u.as<int32_t>();
    a.lag_val = sizeof(Real) == 8 ? reinterpret_cast<const Real *>(g.lag_val64.p) : reinterpret_cast<const Real *>(g.lag_val32.p);
    a.n_lag = g.n_lag;
    a.psi_b = psi_b;
    int threads = (p && p->waves_per_block > 0) ? 64 * p->waves_per_block
                  : (g.has_tuned && g.tuned.waves_per_block > 0 ? 64 * g.tuned.waves_per_block : 0);
    if (threads <= 0) threads = g.nd <= g.n_cu ? 1024 : (g.nd <= 2 * g.n_cu ? 512 : 256);
    threads = std::min(1024, std::max(64, threads));
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (g.profile) {
        JSW_HIP(hipEventCreate(&ev0));
        JSW_HIP(hipEventCreate(&ev1));
        JSW_HIP(hipEventRecord(ev0, s));
    }
    hipLaunchKernelGGL((k_sweep_dir<Real, NF, DIM>), dim3(g.nd), dim3(threads), 0, s, a);
    JSW_HIP(hipGetLastError());
    if (g.profile) {
        JSW_HIP(hipEventRecord(ev1, s));
        g.prof_events.push_back({ev0, ev1});
    }
}

// ---------------------------------------------------------------------------
// Direction-parallel sweep with an LDS window (graphs whose levels are
// narrow): one 1024-lane workgroup per direction walks the levels in order,
// reading the sweep program as coalesced streams one level ahead of the
// compute.  The fluxes of the most recent kRing level positions live in an
// LDS ring indexed by position; an upwind value further back (rare) is read
// from the level-ordered copy in memory, which holds every level completed
// two levels earlier (a level's stores are issued at the start of the next
// level and complete at that level's barrier).  Every level therefore costs
// a barrier and LDS traffic instead of cross-CU hand-offs.
// Requirements (checked by the launcher): two consecutive levels fit in the
// ring and the level table fits in LDS.
// ---------------------------------------------------------------------------
constexpr int kRingThreads = 1024;
constexpr int kRingMaxLev = 2048;
template <class Real>
constexpr int ring_size() { return sizeof(Real) == 8 ? 16384 : 32768; }

template <class Real>
struct RingArgs {
    const int64_t *lvl_ptr;                  // concatenated level pointers (positions)
    const int64_t *lvl_off;                  // [nd + 1]
    const int32_t *lvl_chunk;                // first chunk of each (direction, level)
    const int32_t *lvl_cells;                // [nd*nc]
    int64_t nc;
    int64_t stride;                          // program slot stride
    int32_t ns;                              // program slots (the batched kernel reads up to its NS)
    const int32_t *pcode;
    const Real *pa;
    const Real *pden;
    const Real *pvol;                        // [stride] cell volume, program order
    const Real *src_cell;                    // [nc] isotropic source, or null
    const float *src_dir;                    // [nd*nc] by position, or null
    Real *psi;                               // [nd*nc] by cell
    Real *psi_pos;                           // [nd*nc] by position
    const Real *lag_val;
    Real psi_b;
};

template <class Real, int NS>
struct RingItem {
    Real den, V, sd;                         // sd: per-direction source part (FP32 path)
    int32_t K;
    int32_t code[NS];
    uint64_t pk;                             // packed codes, decoded into code[] when the chunk starts
    Real af[NS];
};

// one pass: vertices [s0 + off, s0 + off + n) of a level whose first chunk
// is c0; lane t takes vertices t, t + T, ...  With DYN, slots at or past
// a.ns are empty.
template <class Real, int NS, int ITEMS, int T, bool DYN>
__device__ __forceinline__ void ring_load(const RingArgs<Real> &a, int64_t base, int64_t s0, int off, int n,
                                          int64_t c0, RingItem<Real, NS> (&it)[ITEMS]) {
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int i = off + (int)threadIdx.x + k * T;
        if (i < off + n) {
            const int64_t idx = (c0 + (i >> 6)) * 64 + (i & 63);
            it[k].den = a.pden[idx];
            it[k].K = a.lvl_cells[base + s0 + i];
#pragma unroll
            for (int j = 0; j < NS; ++j) {
                if (!DYN || j < a.ns) {
                    it[k].code[j] = a.pcode[j * a.stride + idx];
                    it[k].af[j] = a.pa[j * a.stride + idx];
                } else {
                    it[k].code[j] = kNoFace;
                    it[k].af[j] = Real(0);
                }
            }
            it[k].V = a.pvol[idx];
            it[k].sd = Real(0);
            if constexpr (sizeof(Real) == 4) {
                if (a.src_dir) it[k].sd = a.src_dir[base + s0 + i];
            }
        }
    }
}

// A level is processed in passes of at most T * ITEMS vertices (its
// vertices are independent); the next pass's data is loaded while the
// current one computes.  After every pass: all loads and stores complete,
// then a barrier.  A pass's fluxes are stored at the start of the next
// pass, so values of levels two or more back are always readable from
// memory; the ring (R entries) holds the previous level and the current one.
template <class Real, int NS, int ITEMS, int T, int R, int MAXLEV, bool DYN>
__device__ __forceinline__ void ring_direction(const RingArgs<Real> &a, int m, Real *ring, int32_t *lp, int32_t *lc) {
    constexpr int P = T * ITEMS;
    const int64_t base = (int64_t)m * a.nc;
    const int64_t off0 = a.lvl_off[m];
    const int nlev = (int)(a.lvl_off[m + 1] - off0 - 1);
    for (int i = threadIdx.x; i <= nlev; i += T) {
        lp[i] = (int32_t)a.lvl_ptr[off0 + i];
        lc[i] = i < nlev ? a.lvl_chunk[off0 + i] : 0;
    }
    __syncthreads();
    if (nlev <= 0) return;
    RingItem<Real, NS> cur[ITEMS], nxt[ITEMS];
    Real prev_v[ITEMS];
    int32_t prev_K[ITEMS];
    int64_t prev_s = -1;      // first position of the stored-but-not-yet-written pass
    int prev_n = 0;
    // pass cursor: level L, vertices [off, off + n)
    int L = 0, off = 0;
    int n = min(P, lp[1] - lp[0]);
    ring_load<Real, NS, ITEMS, T, DYN>(a, base, lp[0], 0, n, lc[0], cur);
    while (true) {
        const int64_t s0 = lp[L];
        const int w = lp[L + 1] - lp[L];
        // this pass's isotropic source: a gather from a per-cell array,
        // issued first so that it returns ahead of the next pass's loads
        Real sc[ITEMS];
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int i = off + (int)threadIdx.x + k * T;
            sc[k] = (a.src_cell && i < off + n) ? a.src_cell[cur[k].K] : Real(0);
        }
        // the previous pass's fluxes to memory
        if (prev_s >= 0) {
#pragma unroll
            for (int k = 0; k < ITEMS; ++k) {
                const int i = (int)threadIdx.x + k * T;
                if (i < prev_n) {
                    a.psi_pos[base + prev_s + i] = prev_v[k];
                    a.psi[base + prev_K[k]] = prev_v[k];
                }
            }
        }
        // the next pass
        int nL = L, noff = off + n;
        if (noff >= w) { nL = L + 1; noff = 0; }
        int nn = 0;
        if (nL < nlev) {
            nn = min(P, lp[nL + 1] - lp[nL] - noff);
            ring_load<Real, NS, ITEMS, T, DYN>(a, base, lp[nL], noff, nn, lc[nL], nxt);
        }
        // this pass: positions [e - R, s0) of the direction are in the ring
        const int64_t lo = s0 + w - R;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) {
            const int i = off + (int)threadIdx.x + k * T;
            if (i < off + n) {
                const RingItem<Real, NS> &it = cur[k];
                // V s, evaluated as in the other sweep kernels
                Real num;
                if constexpr (sizeof(Real) == 8) num = it.V * sc[k];
                else num = a.src_dir ? it.V * sc[k] + it.sd : it.V * sc[k];   // sd: V r
#pragma unroll
                for (int j = 0; j < NS; ++j) {
                    const int32_t cd = it.code[j];
                    if (cd == kNoFace) continue;
                    Real v;
                    if (cd >= 0) v = cd >= lo ? ring[cd & (R - 1)] : ld_coherent(a.psi_pos + base + cd);
                    else if (cd == -1) v = a.psi_b;
                    else v = a.lag_val[-(int64_t)cd - 2];
                    num = num + it.af[j] * v;
                }
                const Real v = num / it.den;
                ring[(s0 + i) & (R - 1)] = v;
                prev_v[k] = v;
                prev_K[k] = it.K;
            }
        }
        prev_s = s0 + off;
        prev_n = n;
        // every load and store of this pass complete (the previous pass's
        // fluxes are now readable from memory), then the ring
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (nL >= nlev) break;
#pragma unroll
        for (int k = 0; k < ITEMS; ++k) cur[k] = nxt[k];
        L = nL;
        off = noff;
        n = nn;
    }
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        const int i = (int)threadIdx.x + k * T;
        if (i < prev_n) {
            a.psi_pos[base + prev_s + i] = prev_v[k];
            a.psi[base + prev_K[k]] = prev_v[k];
        }
    }
}

template <class Real, int NS, int ITEMS>
__global__ void __launch_bounds__(kRingThreads) k_sweep_ring(RingArgs<Real> a) {
    constexpr int R = ring_size<Real>();
    __shared__ Real ring[R];
    __shared__ int32_t lp[kRingMaxLev + 1], lc[kRingMaxLev + 1];
    ring_direction<Real, NS, ITEMS, kRingThreads, R, kRingMaxLev, false>(a, blockIdx.x, ring, lp, lc);
}

// Batched form: one 256-lane workgroup per (instance, direction), a 32 KB
// ring and a 1024-level table, so several tasks share a compute unit.
constexpr int kBRingThreads = 256;
constexpr int kBRingMaxLev = 1024;
constexpr int kBRingNS = 6;
template <class Real>
constexpr int bring_size() { return sizeof(Real) == 8 ? 4096 : 8192; }

template <class Real>
__global__ void __launch_bounds__(kBRingThreads) k_sweep_batch_ring(const RingArgs<Real> *inst, const int32_t *task_inst,
                                                                   const int32_t *task_dir, const int32_t *active) {
    constexpr int R = bring_size<Real>();
    __shared__ Real ring[R];
    __shared__ int32_t lp[kBRingMaxLev + 1], lc[kBRingMaxLev + 1];
    const int i = task_inst[blockIdx.x];
    if (i < 0 || !active[i]) return;
    ring_direction<Real, kBRingNS, 2, kBRingThreads, R, kBRingMaxLev, true>(inst[i], task_dir[blockIdx.x], ring, lp,
                                                                           lc);
}

// vertices per lane and pass for the ring kernel (0: not applicable to
// this graph): two consecutive levels must fit in the ring and the level
// table in LDS; two per lane unless the inflow slots need the registers
static int ring_items(const Graph &g, bool f32) {
    const int64_t R = f32 ? ring_size<float>() : ring_size<double>();
    // the ring reads a level's program from its consecutive chunks, which
    // the BFS and PACED work lists keep together
    if (!levels_contiguous(g)) return 0;
    if (g.max_w2 > R || g.max_levels > kRingMaxLev || g.ns < 1 || g.ns > 6) return 0;
    return (!f32 && g.ns >= 6) ? 1 : 2;
}

template <class Real, int NS>
static const void *ring_kernel_ns(int items) {
    if (items == 1) return reinterpret_cast<const void *>(&k_sweep_ring<Real, NS, 1>);
    return reinterpret_cast<const void *>(&k_sweep_ring<Real, NS, 2>);
}

template <class Real>
static const void *ring_kernel(int ns, int items) {
    switch (ns) {
    case 1: return ring_kernel_ns<Real, 1>(items);
    case 2: return ring_kernel_ns<Real, 2>(items);
    case 3: return ring_kernel_ns<Real, 3>(items);
    case 4: return ring_kernel_ns<Real, 4>(items);
    case 5: return ring_kernel_ns<Real, 5>(items);
    default: return ring_kernel_ns<Real, 6>(items);
    }
}

// arguments of the ring sweep for one graph (builds the program-order
// volumes and the level-ordered flux copy on first use)
template <class Real>
static RingArgs<Real> ring_args(Graph &g, const Real *src_cell, const float *src_dir, Real *psi, Real psi_b,
                                hipStream_t s) {
    const bool f32 = sizeof(Real) == 4;
    if (!(f32 ? g.den32_ok : g.den64_ok)) fail(JSWEEP_E_DEVICE, "sweep program denominators not built");
    const int64_t S = 64 * g.n_chunks;
    DevBuf &pv = f32 ? g.pvol32 : g.pvol64;
    if (!pv.p) {
        pv.alloc((f32 ? 4 : 8) * (size_t)S);
        k_pvol<Real><<<(unsigned)ceil_div(S, 256), 256, 0, s>>>(g.cblk.as<int32_t>(), S, g.vol.as<double>(), pv.as<Real>());
        JSW_HIP(hipGetLastError());
    }
    RingArgs<Real> a;
    a.lvl_ptr = g.lvl_ptr_d.as<int64_t>();
    a.lvl_off = g.lvl_off_d.as<int64_t>();
    a.lvl_chunk = g.lvl_chunk_d.as<int32_t>();
    a.lvl_cells = g.lvl_cells.as<int32_t>();
    a.nc = g.nc;
    a.stride = S;
    a.ns = g.ns;
    a.pcode = g.pcode.as<int32_t>();
    a.pa = reinterpret_cast<const Real *>(f32 ? g.pa32.p : g.pa64.p);
    a.pden = reinterpret_cast<const Real *>(f32 ? g.pden32.p : g.pden64.p);
    a.pvol = pv.as<Real>();
    a.src_cell = src_cell;
    a.src_dir = src_dir;
    a.psi = psi;
    if (g.psi_pos.bytes < (size_t)(8 * g.nc * g.nd)) g.psi_pos.alloc(8 * g.nc * g.nd);
    a.psi_pos = g.psi_pos.as<Real>();
    a.lag_val = reinterpret_cast<const Real *>(f32 ? g.lag_val32.p : g.lag_val64.p);
    a.psi_b = psi_b;
    return a;
}

template <class Real>
static void launch_ring(Graph &g, const Real *src_cell, const float *src_dir, Real *psi, Real psi_b, hipStream_t s) {
    const bool f32 = sizeof(Real) == 4;
    const int items = ring_items(g, f32);
    if (!items) fail(JSWEEP_E_DEVICE, "ring sweep not applicable to this graph");
    RingArgs<Real> a = ring_args<Real>(g, src_cell, src_dir, psi, psi_b, s);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (g.profile) {
        JSW_HIP(hipEventCreate(&ev0));
        JSW_HIP(hipEventCreate(&ev1));
        JSW_HIP(hipEventRecord(ev0, s));
    }
    void *args[] = {&a};
    JSW_HIP(hipLaunchKernel(ring_kernel<Real>(g.ns, items), dim3(g.nd), dim3(kRingThreads), args, 0, s));
    if (g.profile) {
        JSW_HIP(hipEventRecord(ev1, s));
        g.prof_events.push_back({ev0, ev1});
    }
}

// Sweep strategy: the requested or tuned one, else the data-driven
// persistent kernel, which keeps many levels of every direction in flight
// (the direction kernels, with a barrier per level, are slower on every
// graph measured).
int sweep_strategy(const Graph &g, const jsweep_params *p) {
    int st = (p && p->strategy > 0) ? p->strategy : (g.has_tuned && g.tuned.strategy > 0 ? g.tuned.strategy : 0);
    if (st == JSWEEP_STRATEGY_DATA_DRIVEN || st == JSWEEP_STRATEGY_DIRECTION || st == JSWEEP_STRATEGY_PATCH) return st;
    if (st == JSWEEP_STRATEGY_DIRECTION_LDS) return ring_items(g, false) ? st : JSWEEP_STRATEGY_DIRECTION;
    return JSWEEP_STRATEGY_DATA_DRIVEN;
}

template <class Real, int NF, int DIM>
static void launch_impl(Graph &g, const Real *src_cell, const float *src_dir, Real *psi, Real psi_b,
                        const jsweep_params *p, hipStream_t s, bool prepared = false, bool nonneg = false) {
    const int st = sweep_strategy(g, p);
    if constexpr (sizeof(Real) == 8) {
        if (st == JSWEEP_STRATEGY_PATCH && patch_ready(g, s)) {
            launch_patch64(g, src_cell, psi, psi_b, p, s, prepared);
            return;
        }
    }
    if (st == JSWEEP_STRATEGY_DIRECTION_LDS && ring_items(g, sizeof(Real) == 4)) launch_ring<Real>(g, src_cell, src_dir, psi, psi_b, s);
    else if (st == JSWEEP_STRATEGY_DIRECTION || st == JSWEEP_STRATEGY_DIRECTION_LDS)
        launch_dir<Real, NF, DIM>(g, src_cell, src_dir, psi, psi_b, p, s);
    else launch_persistent<Real>(g, src_cell, src_dir, psi, psi_b, p, s, prepared, nullptr, nullptr, nonneg);
}

void launch_sweep64(Graph &g, const double *src_cell, double *psi, double psi_b, const jsweep_params *p, hipStream_t s,
                    bool prepared, bool nonneg) {
    if (g.ctype == JSWEEP_TRI) launch_impl<double, 3, 2>(g, src_cell, nullptr, psi, psi_b, p, s, prepared, nonneg);
    else if (g.ctype == JSWEEP_TET) launch_impl<double, 4, 3>(g, src_cell, nullptr, psi, psi_b, p, s, prepared, nonneg);
    else launch_impl<double, 6, 3>(g, src_cell, nullptr, psi, psi_b, p, s, prepared, nonneg);
}

void *last_sweep_pos(Graph &g) { return g.dd_pos[1 - g.dd_cur].p; }

uint64_t last_sweep_keep(const Graph &g) { return (g.dd_state[1 - g.dd_cur] & kDdTagged) ? ~kSignBit : ~0ull; }

void launch_sweep64_staged(Graph &g, const double *src_cell, double *psi, double psi_b, void *vs_buf, hipStream_t s) {
    if (sweep_strategy(g, nullptr) != JSWEEP_STRATEGY_DATA_DRIVEN)
        fail(JSWEEP_E_INVALID_ARG, "the staged sweep runs the data-driven strategy only");
    if (g.trace) fail(JSWEEP_E_INVALID_ARG, "the staged sweep does not trace");
    launch_persistent<double>(g, src_cell, nullptr, psi, psi_b, nullptr, s, false, nullptr, vs_buf);
}

void launch_sweep_groups(Graph &g, double *psi, const GroupSweep &mg, const jsweep_params *p, hipStream_t s) {
    launch_persistent<double>(g, nullptr, nullptr, psi, mg.psi_b, p, s, true, &mg, nullptr, mg.nonneg);
}

void launch_sweep32(Graph &g, const float *src_dir, const float *src_cell, float *psi, const jsweep_params *p,
                    hipStream_t s, bool prepared) {
    if (g.ctype == JSWEEP_TRI) launch_impl<float, 3, 2>(g, src_cell, src_dir, psi, 0.0f, p, s, prepared);
    else if (g.ctype == JSWEEP_TET) launch_impl<float, 4, 3>(g, src_cell, src_dir, psi, 0.0f, p, s, prepared);
    else launch_impl<float, 6, 3>(g, src_cell, src_dir, psi, 0.0f, p, s, prepared);
}

int check_sweep_status(Graph &g, hipStream_t s) {
    int32_t st = 0;
    JSW_HIP(hipMemcpyAsync(&st, g.status.p, 4, hipMemcpyDeviceToHost, s));
    JSW_HIP(hipStreamSynchronize(s));
    if (st == 0) return JSWEEP_OK;
    const int rc = (st & kStatusPlacement) ? JSWEEP_E_PLACEMENT : JSWEEP_E_STALLED;
    set_last_error(rc == JSWEEP_E_PLACEMENT ? "a sweep workgroup ran on another XCD than the workgroups of its stream"
                                            : "a sweep wavefront's watchdog fired (status word " + std::to_string(st) + ")");
    // a stalled sweep leaves the level-position arrays and the task slots
    // in an unknown state: start over
    g.dd_state[0] = g.dd_state[1] = 0;
    if (g.pp.slot.p) JSW_HIP(hipMemsetAsync(g.pp.slot.p, 0, g.pp.slot.bytes, s));
    JSW_HIP(hipMemsetAsync(g.status.p, 0, 64, s));
    JSW_HIP(hipStreamSynchronize(s));
    g.pp.epoch = 0;
    return rc;
}

// Host side of the batched sweep: the instance table and the task list are
// built once per batch solve (BatchSweep) and the launch is a single kernel.
template <class Real>
static void fill_inst(Graph &g, BatchInst<Real> &b, const Real *src_cell, const float *src_dir, Real *psi, Real psi_b) {
    b.rec = sizeof(Real) == 8 ? g.rec64.p : g.rec32.p;
    b.rec64 = g.rec64.p;
    b.lvl_cells = g.lvl_cells.as<int32_t>();
    b.lvl_ptr = g.lvl_ptr_d.as<int64_t>();
    b.lvl_off = g.lvl_off_d.as<int64_t>();
    b.nc = g.nc;
    b.omega = sizeof(Real) == 8 ? reinterpret_cast<const Real *>(g.omega64.p) : reinterpret_cast<const Real *>(g.omega32.p);
    b.omega64 = g.omega64.as<double>();
    b.src_cell = src_cell;
    b.src_dir = src_dir;
    b.psi = psi;
    b.lag_mv = g.lag_mv.as<uint64_t>();
    b.lag_u = g.lag_u.as<int32_t>();
    b.lag_val = sizeof(Real) == 8 ? reinterpret_cast<const Real *>(g.lag_val64.p) : reinterpret_cast<const Real *>(g.lag_val32.p);
    b.n_lag = g.n_lag;
    b.psi_b = psi_b;
    b.ctype = g.ctype;
    b.nd = g.nd;
}

// Launch order of the (instance, direction) tasks; index b runs on XCD
// b % kStreams.  All directions of an instance go to one XCD, so they share
// its L2 (the instance's cell records, volumes and sources are read by every
// direction); instances are dealt to the XCDs by estimated cost, costliest
// first, onto the least loaded XCD; within an XCD the costliest tasks start
// first.  Cost of a task: its rounds of T vertices over the direction's
// levels.  Slots left over where the XCDs' task counts differ hold -1.
static void batch_order(int32_t n, Graph *const *graphs, int T, DevBuf &task_inst, DevBuf &task_dir,
                        int64_t &n_tasks, hipStream_t s) {
    struct Task {
        int64_t cost;
        int32_t inst, dir;
    };
    std::vector<std::vector<Task>> per(n);
    std::vector<std::pair<int64_t, int32_t>> inst_cost(n);
    for (int i = 0; i < n; ++i) {
        const Graph &g = *graphs[i];
        int64_t tot = 0;
        for (int m = 0; m < g.nd; ++m) {
            const int64_t *ptr = g.lvl_ptr_h.data() + g.lvl_off_h[m];
            const int nlev = (int)(g.lvl_off_h[m + 1] - g.lvl_off_h[m] - 1);
            int64_t c = 1;
            for (int L = 0; L < nlev; ++L) c += ceil_div(ptr[L + 1] - ptr[L], T);
            per[i].push_back(Task{c, i, m});
            tot += c;
        }
        inst_cost[i] = {tot, i};
    }
    std::vector<std::vector<Task>> q(kStreams);
    std::stable_sort(inst_cost.begin(), inst_cost.end(), [](const auto &a, const auto &b) { return a.first > b.first; });
    std::vector<int64_t> load(kStreams, 0);
    for (const auto &ic : inst_cost) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[x] += ic.first;
        q[x].insert(q[x].end(), per[ic.second].begin(), per[ic.second].end());
    }
    size_t len = 0;
    for (auto &v : q) {
        std::stable_sort(v.begin(), v.end(), [](const Task &a, const Task &b) { return a.cost > b.cost; });
        len = std::max(len, v.size());
    }
    n_tasks = (int64_t)len * kStreams;
    std::vector<int32_t> ti(n_tasks, -1), td(n_tasks, 0);
    for (int x = 0; x < kStreams; ++x)
        for (size_t k = 0; k < q[x].size(); ++k) {
            ti[k * kStreams + x] = q[x][k].inst;
            td[k * kStreams + x] = q[x][k].dir;
        }
    task_inst.alloc(4 * std::max<int64_t>(1, n_tasks));
    task_dir.alloc(4 * std::max<int64_t>(1, n_tasks));
    JSW_HIP(hipMemcpyAsync(task_inst.p, ti.data(), 4 * n_tasks, hipMemcpyHostToDevice, s));
    JSW_HIP(hipMemcpyAsync(task_dir.p, td.data(), 4 * n_tasks, hipMemcpyHostToDevice, s));
    JSW_HIP(hipStreamSynchronize(s));   // the host tables go out of scope
}

void BatchSweep::setup(int32_t n, Graph *const *graphs, bool fp32, const void *const *src_cell,
                       const float *const *src_dir, void *const *psi, const double *psi_b, int threads_, int strategy,
                       hipStream_t s) {
    this->fp32 = fp32;
    // the LDS-window kernel when every instance fits it
    ring = strategy != JSWEEP_STRATEGY_DIRECTION;
    const int64_t R = fp32 ? bring_size<float>() : bring_size<double>();
    for (int i = 0; i < n && ring; ++i) {
        const Graph &g = *graphs[i];
        ring = g.n_chunks > 0 && levels_contiguous(g) && g.max_w2 <= R && g.max_levels <= kBRingMaxLev && g.ns >= 1 && g.ns <= kBRingNS;
    }
    const int T = ring ? kBRingThreads * 2 : (threads_ > 0 ? std::min(1024, std::max(64, threads_)) : 256);
    batch_order(n, graphs, T, task_inst, task_dir, n_tasks, s);
    if (ring) {
        if (fp32) {
            std::vector<RingArgs<float>> h(n);
            for (int i = 0; i < n; ++i)
                h[i] = ring_args<float>(*graphs[i], (const float *)src_cell[i], src_dir[i], (float *)psi[i], (float)psi_b[i], s);
            inst.alloc(sizeof(RingArgs<float>) * n);
            JSW_HIP(hipMemcpyAsync(inst.p, h.data(), sizeof(RingArgs<float>) * n, hipMemcpyHostToDevice, s));
        } else {
            std::vector<RingArgs<double>> h(n);
            for (int i = 0; i < n; ++i)
                h[i] = ring_args<double>(*graphs[i], (const double *)src_cell[i], src_dir[i], (double *)psi[i], psi_b[i], s);
            inst.alloc(sizeof(RingArgs<double>) * n);
            JSW_HIP(hipMemcpyAsync(inst.p, h.data(), sizeof(RingArgs<double>) * n, hipMemcpyHostToDevice, s));
        }
        JSW_HIP(hipStreamSynchronize(s));   // host tables above go out of scope
        threads = kBRingThreads;
        return;
    }
    if (fp32) {
        std::vector<BatchInst<float>> h(n);
        for (int i = 0; i < n; ++i)
            fill_inst<float>(*graphs[i], h[i], (const float *)src_cell[i], src_dir[i], (float *)psi[i], (float)psi_b[i]);
        inst.alloc(sizeof(BatchInst<float>) * n);
        JSW_HIP(hipMemcpyAsync(inst.p, h.data(), sizeof(BatchInst<float>) * n, hipMemcpyHostToDevice, s));
        JSW_HIP(hipStreamSynchronize(s));
    } else {
        std::vector<BatchInst<double>> h(n);
        for (int i = 0; i < n; ++i)
            fill_inst<double>(*graphs[i], h[i], (const double *)src_cell[i], src_dir[i], (double *)psi[i], psi_b[i]);
        inst.alloc(sizeof(BatchInst<double>) * n);
        JSW_HIP(hipMemcpyAsync(inst.p, h.data(), sizeof(BatchInst<double>) * n, hipMemcpyHostToDevice, s));
        JSW_HIP(hipStreamSynchronize(s));
    }
    threads = threads_ > 0 ? std::min(1024, std::max(64, threads_)) : 256;
}
void BatchSweep::launch(const int32_t *active, hipStream_t s) {
    if (ring) {
        if (fp32)
            hipLaunchKernelGGL(k_sweep_batch_ring<float>, dim3((unsigned)n_tasks), dim3(kBRingThreads), 0, s,
                               inst.as<RingArgs<float>>(), task_inst.as<int32_t>(), task_dir.as<int32_t>(), active);
        else
            hipLaunchKernelGGL(k_sweep_batch_ring<double>, dim3((unsigned)n_tasks), dim3(kBRingThreads), 0, s,
                               inst.as<RingArgs<double>>(), task_inst.as<int32_t>(), task_dir.as<int32_t>(), active);
    } else if (fp32) {
        hipLaunchKernelGGL(k_sweep_batch<float>, dim3((unsigned)n_tasks), dim3(threads), 0, s,
                           inst.as<BatchInst<float>>(), task_inst.as<int32_t>(), task_dir.as<int32_t>(), active);
    } else {
        hipLaunchKernelGGL(k_sweep_batch<double>, dim3((unsigned)n_tasks), dim3(threads), 0, s,
                           inst.as<BatchInst<double>>(), task_inst.as<int32_t>(), task_dir.as<int32_t>(), active);
    }
    JSW_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Union of several graphs swept by one launch of the data-driven kernel
// (the batched solve; structure in common.hpp).
// ---------------------------------------------------------------------------
namespace {

struct UnionSrc {
    const int32_t *cblk;                 // the instance's chunk blocks
    const int32_t *pcode;                // its program (ns slots, stride S)
    const void *pa;
    const void *pden;
    int64_t S, coff, loff, aoff, nc;
    int32_t ns, dir_off;
};

std::mutex g_union_mu;
std::unique_ptr<UnionSweep> g_union[2];   // one per precision
std::atomic<uint64_t> g_uid{0};

// chunk block of union chunk u from chunk c of instance i: global cell ids
// and global direction
__global__ void k_union_block(const int32_t *uinst, const int32_t *uchunk, const UnionSrc *src, int64_t n,
                              int32_t *blk) {
    const int64_t u = blockIdx.x;
    const int lane = threadIdx.x;
    if (u >= n) return;
    const int inst = uinst[u];
    const UnionSrc r = src[inst];
    const int32_t *b = r.cblk + (int64_t)uchunk[u] * kBlock;
    int32_t *o = blk + u * kBlock;
    const int32_t K = b[lane];
    o[lane] = K >= 0 ? (int32_t)(K + r.coff) : -1;
    if (lane == 0) {
        const uint32_t w = (uint32_t)b[64];
        o[64] = (int32_t)(((w & 0xffffu) + (uint32_t)r.dir_off) | (w & 0xffff0000u));
    }
    if (lane == 1) o[65] = 0;
    if (lane == 2) o[66] = b[66];
    // the direction's first level position in the union (lo, hi) and the
    // instance: what the sweep needs before its polls
    if (lane == 3 || lane == 4) {
        const int m = (int)((uint32_t)b[64] & 0xffffu);
        const uint64_t pb = (uint64_t)(r.aoff + (int64_t)m * r.nc);
        o[67 + lane - 3] = (int32_t)(uint32_t)(lane == 3 ? pb : pb >> 32);
    }
    if (lane == 5) o[69] = (int32_t)inst;
}

// program of union chunk u: codes (lagged-edge codes moved to the union's
// lagged-value array; slots past the instance's ns empty), coefficients
// and denominators (DEN_ONLY: the denominators alone)
template <class Real, bool DEN_ONLY>
__global__ void k_union_prog(const int32_t *uinst, const int32_t *uchunk, const UnionSrc *src, int64_t n, int ns,
                             int32_t *pcode, Real *pa, Real *pden) {
    const int64_t u = blockIdx.x;
    const int lane = threadIdx.x;
    if (u >= n) return;
    const UnionSrc r = src[uinst[u]];
    const int64_t from = (int64_t)uchunk[u] * 64 + lane, to = u * 64 + lane, S = n * 64;
    pden[to] = static_cast<const Real *>(r.pden)[from];
    if (DEN_ONLY) return;
    for (int j = 0; j < ns; ++j) {
        int32_t cd = kNoFace;
        Real af = Real(0);
        if (j < r.ns) {
            cd = r.pcode[j * r.S + from];
            af = static_cast<const Real *>(r.pa)[j * r.S + from];
            if (cd <= -2 && cd != kNoFace) cd = (int32_t)(-((-(int64_t)cd - 2) + r.loff) - 2);
        }
        pcode[j * S + to] = cd;
        pa[j * S + to] = af;
    }
}

}  // namespace

uint64_t next_graph_uid() { return ++g_uid; }

void union_forget(uint64_t uid) {
    std::lock_guard<std::mutex> lock(g_union_mu);
    for (auto &u : g_union) {
        if (!u) continue;
        for (size_t i = 0; i + 1 < u->key.size(); ++i)
            if ((u->key[i] >> 24) == uid) {
                u.reset();
                break;
            }
    }
}

static std::vector<UnionSrc> union_sources(const UnionSweep &u, Graph *const *graphs) {
    std::vector<UnionSrc> src(u.n);
    for (int i = 0; i < u.n; ++i) {
        const Graph &g = *graphs[i];
        UnionSrc &r = src[i];
        r.cblk = g.cblk.as<int32_t>();
        r.pcode = g.pcode.as<int32_t>();
        r.pa = u.fp32 ? g.pa32.p : g.pa64.p;
        r.pden = u.fp32 ? g.pden32.p : g.pden64.p;
        r.S = 64 * g.n_chunks;
        r.coff = u.coff[i];
        r.loff = u.loff[i];
        r.aoff = u.aoff[i];
        r.nc = g.nc;
        r.ns = g.ns;
        r.dir_off = u.dir_off[i];
    }
    return src;
}

void UnionSweep::build(int n_, Graph *const *graphs, bool fp32_, hipStream_t s) {
    n = n_;
    fp32 = fp32_;
    n_cu = graphs[0]->n_cu;
    ns = 1;
    coff.assign(n + 1, 0);
    aoff.assign(n + 1, 0);
    loff.assign(n + 1, 0);
    dir_off.assign(n + 1, 0);
    for (int i = 0; i < n; ++i) {
        const Graph &g = *graphs[i];
        if (g.ns > 6) fail(JSWEEP_E_INVALID_ARG, "batched data-driven sweep: too many inflow slots");
        ns = std::max(ns, g.ns);
        coff[i + 1] = coff[i] + g.nc;
        aoff[i + 1] = aoff[i] + g.nc * g.nd;
        loff[i + 1] = loff[i] + g.n_lag;
        dir_off[i + 1] = dir_off[i] + g.nd;
    }
    C = coff[n];
    A = aoff[n];
    LG = loff[n];
    total_dirs = dir_off[n];
    if (total_dirs > 0xffff) fail(JSWEEP_E_INVALID_ARG, "batched data-driven sweep: more than 65535 directions in all");
    if (A >= ((int64_t)1 << 32) || C >= ((int64_t)1 << 31)) fail(JSWEEP_E_INVALID_ARG, "batched data-driven sweep: batch too large");
    // merged streams: every instance's chunks of stream x, ordered as the
    // PACED priority orders one graph's: by the level over the level count
    // of the chunk's (instance, direction), then (level, instance, chunk).
    // The key grows with the level within every (instance, direction), so
    // the order is topological; instances of every depth reach their last
    // levels together at the end of the stream, instead of the deepest
    // ones running alone after the others (as in plain level order)
    struct Item {
        int64_t key;
        int32_t level, inst, chunk;
    };
    std::vector<std::vector<Item>> per(kStreams);
    for (int i = 0; i < n; ++i) {
        const Graph &g = *graphs[i];
        std::vector<Chunk> ch(g.n_chunks);
        if (g.n_chunks) JSW_HIP(hipMemcpy(ch.data(), g.chunks.p, sizeof(Chunk) * g.n_chunks, hipMemcpyDeviceToHost));
        for (int64_t c = 0; c < g.n_chunks; ++c) {
            const int m = (int)(ch[c].a & 0xffffu);
            const int64_t *p = g.lvl_ptr_h.data() + g.lvl_off_h[m];
            const int L = (int)(std::upper_bound(p, p + g.nlev_h[m] + 1, (int64_t)ch[c].b) - p - 1);
            per[g.dir_stream_h[m]].push_back(Item{((int64_t)L << 32) / std::max(1, g.nlev_h[m]), L, i, (int32_t)c});
        }
    }
    std::vector<int32_t> hi, hc;
    stream_off_h.assign(kStreams + 1, 0);
    for (int x = 0; x < kStreams; ++x) {
        auto &v = per[x];
        std::sort(v.begin(), v.end(), [](const Item &a, const Item &b) {
            if (a.key != b.key) return a.key < b.key;
            if (a.level != b.level) return a.level < b.level;
            if (a.inst != b.inst) return a.inst < b.inst;
            return a.chunk < b.chunk;
        });
        stream_off_h[x] = (int64_t)hi.size();
        for (const Item &it : v) {
            hi.push_back(it.inst);
            hc.push_back(it.chunk);
        }
    }
    stream_off_h[kStreams] = (int64_t)hi.size();
    n_chunks = (int64_t)hi.size();
    if (n_chunks >= ((int64_t)1 << 31)) fail(JSWEEP_E_INVALID_ARG, "batched data-driven sweep: too many chunks");
    const int64_t S = 64 * std::max<int64_t>(1, n_chunks);
    uinst.alloc(4 * std::max<int64_t>(1, n_chunks));
    uchunk.alloc(4 * std::max<int64_t>(1, n_chunks));
    isrc.alloc(sizeof(UnionSrc) * n);
    cblk.alloc(4 * (size_t)kBlock * std::max<int64_t>(1, n_chunks));
    pcode.alloc(4 * (size_t)ns * S);
    pa.alloc((fp32 ? 4 : 8) * (size_t)ns * S);
    pden.alloc((fp32 ? 4 : 8) * (size_t)S);
    stream_off.alloc(8 * (kStreams + 1));
    rows.alloc(sizeof(DirRow) * std::max(1, total_dirs));
    status.alloc(128 + 32 * 4 * kStreams);
    lag.alloc((fp32 ? 4 : 8) * (size_t)std::max<int64_t>(1, LG));
    vs.alloc(8 * (size_t)std::max<int64_t>(1, C));
    for (int k = 0; k < 2; ++k) {
        pos[k].alloc(8 * (size_t)std::max<int64_t>(1, A));
        pos_state[k] = 0;
    }
    cur = 0;
    const std::vector<UnionSrc> src = union_sources(*this, graphs);
    if (n_chunks) {
        JSW_HIP(hipMemcpyAsync(uinst.p, hi.data(), 4 * n_chunks, hipMemcpyHostToDevice, s));
        JSW_HIP(hipMemcpyAsync(uchunk.p, hc.data(), 4 * n_chunks, hipMemcpyHostToDevice, s));
    }
    JSW_HIP(hipMemcpyAsync(isrc.p, src.data(), sizeof(UnionSrc) * n, hipMemcpyHostToDevice, s));
    JSW_HIP(hipMemcpyAsync(stream_off.p, stream_off_h.data(), 8 * (kStreams + 1), hipMemcpyHostToDevice, s));
    JSW_HIP(hipMemsetAsync(status.p, 0, status.bytes, s));
    if (n_chunks) {
        k_union_block<<<(unsigned)n_chunks, 64, 0, s>>>(uinst.as<int32_t>(), uchunk.as<int32_t>(), isrc.as<UnionSrc>(),
                                                        n_chunks, cblk.as<int32_t>());
        JSW_HIP(hipGetLastError());
        if (fp32)
            k_union_prog<float, false><<<(unsigned)n_chunks, 64, 0, s>>>(
                uinst.as<int32_t>(), uchunk.as<int32_t>(), isrc.as<UnionSrc>(), n_chunks, ns, pcode.as<int32_t>(),
                pa.as<float>(), pden.as<float>());
        else
            k_union_prog<double, false><<<(unsigned)n_chunks, 64, 0, s>>>(
                uinst.as<int32_t>(), uchunk.as<int32_t>(), isrc.as<UnionSrc>(), n_chunks, ns, pcode.as<int32_t>(),
                pa.as<double>(), pden.as<double>());
        JSW_HIP(hipGetLastError());
        // packed codes of the merged program (the union's own lagged
        // indices are escapes like any other)
        pk.release();
        if (ns <= 3) {
            pk.alloc(8 * (size_t)S);
            if (!pack_codes(cblk.as<int32_t>(), n_chunks, ns, pcode.as<int32_t>(), pk.as<uint64_t>(), s)) pk.release();
        }
    }
    JSW_HIP(hipStreamSynchronize(s));   // the host tables go out of scope
}

void UnionSweep::refresh_den(Graph *const *graphs, hipStream_t s) {
    if (!n_chunks) return;
    const std::vector<UnionSrc> src = union_sources(*this, graphs);
    JSW_HIP(hipMemcpyAsync(isrc.p, src.data(), sizeof(UnionSrc) * n, hipMemcpyHostToDevice, s));
    if (fp32)
        k_union_prog<float, true><<<(unsigned)n_chunks, 64, 0, s>>>(uinst.as<int32_t>(), uchunk.as<int32_t>(),
                                                                    isrc.as<UnionSrc>(), n_chunks, ns, nullptr,
                                                                    nullptr, pden.as<float>());
    else
        k_union_prog<double, true><<<(unsigned)n_chunks, 64, 0, s>>>(uinst.as<int32_t>(), uchunk.as<int32_t>(),
                                                                     isrc.as<UnionSrc>(), n_chunks, ns, nullptr,
                                                                     nullptr, pden.as<double>());
    JSW_HIP(hipGetLastError());
    JSW_HIP(hipStreamSynchronize(s));   // src goes out of scope
}

void UnionSweep::set_rows(Graph *const *graphs, void *const *psi, const float *const *src_dir, const double *psi_b,
                          hipStream_t s) {
    prof = graphs[0];
    std::vector<DirRow> h(std::max(1, total_dirs));
    const size_t word = fp32 ? 4 : 8;
    for (int i = 0; i < n; ++i) {
        const Graph &g = *graphs[i];
        for (int m = 0; m < g.nd; ++m) {
            DirRow &r = h[dir_off[i] + m];
            r.pos_base = aoff[i] + (int64_t)m * g.nc;
            r.cell_off = coff[i];
            r.psi_row = psi[i] ? static_cast<char *>(psi[i]) + word * (size_t)m * g.nc : nullptr;
            r.src_row = src_dir[i] ? src_dir[i] + (int64_t)m * g.nc : nullptr;
            r.psi_b = psi_b[i];
            r.inst = i;
            r.pad = 0;
        }
    }
    JSW_HIP(hipMemcpyAsync(rows.p, h.data(), sizeof(DirRow) * h.size(), hipMemcpyHostToDevice, s));
    JSW_HIP(hipStreamSynchronize(s));
}

// compaction of the union's list: flag[u] = the instance of chunk u still
// iterates; flag[n] = 0 (the scan's last entry is the compacted length)
__global__ void k_union_flags(const int32_t *uinst, const int32_t *active, int64_t n, int32_t *flag) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u < n) flag[u] = active[uinst[u]] ? 1 : 0;
    else if (u == n) flag[u] = 0;
}

__global__ void k_union_offsets(const int64_t *stream_off, const int32_t *scan, int64_t *c_stream_off) {
    const int x = threadIdx.x;
    if (x <= kStreams) c_stream_off[x] = scan[stream_off[x]];
}

// chunk u (one 64-lane workgroup) to its place scan[u] in the compacted
// list: its block and every program array of its lanes
template <class Real>
__global__ void k_union_gather(const int32_t *flag, const int32_t *scan, int64_t n, int ns, const int32_t *cblk,
                               const int32_t *pcode, const Real *pa, const Real *pden, const uint64_t *pk,
                               int32_t *c_cblk, int32_t *c_pcode, Real *c_pa, Real *c_pden, uint64_t *c_pk) {
    const int64_t u = blockIdx.x;
    const int lane = threadIdx.x;
    if (u >= n || !flag[u]) return;
    const int64_t v = scan[u], S = 64 * n;
    const int32_t *b = cblk + u * kBlock;
    int32_t *o = c_cblk + v * kBlock;
    o[lane] = b[lane];
    if (lane < kBlock - 64) o[64 + lane] = b[64 + lane];
    const int64_t from = u * 64 + lane, to = v * 64 + lane;
    for (int j = 0; j < ns; ++j) {
        c_pcode[j * S + to] = pcode[j * S + from];
        c_pa[j * S + to] = pa[j * S + from];
    }
    c_pden[to] = pden[from];
    if (pk) c_pk[to] = pk[from];
}

void UnionSweep::compact(const int32_t *active, hipStream_t s) {
    if (!n_chunks) return;
    const int64_t S = 64 * n_chunks;
    const size_t word = fp32 ? 4 : 8;
    if (!c_cblk.p) {
        c_cblk.alloc(4 * (size_t)kBlock * n_chunks);
        c_pcode.alloc(4 * (size_t)ns * S);
        c_pa.alloc(word * (size_t)ns * S);
        c_pden.alloc(word * (size_t)S);
        if (pk.p) c_pk.alloc(8 * (size_t)S);
        c_stream_off.alloc(8 * (kStreams + 1));
        c_flag.alloc(4 * (size_t)(n_chunks + 1));
        c_scan.alloc(4 * (size_t)(n_chunks + 1));
    }
    const unsigned gb = (unsigned)ceil_div(n_chunks + 1, 256);
    k_union_flags<<<gb, 256, 0, s>>>(uinst.as<int32_t>(), active, n_chunks, c_flag.as<int32_t>());
    JSW_HIP(hipGetLastError());
    size_t tb = 0;
    JSW_HIP(rocprim::exclusive_scan(nullptr, tb, c_flag.as<int32_t>(), c_scan.as<int32_t>(), 0, (size_t)(n_chunks + 1),
                                    rocprim::plus<int32_t>(), s));
    if (c_tmp.bytes < tb + 16) c_tmp.alloc(tb + 16);
    JSW_HIP(rocprim::exclusive_scan(c_tmp.p, tb, c_flag.as<int32_t>(), c_scan.as<int32_t>(), 0, (size_t)(n_chunks + 1),
                                    rocprim::plus<int32_t>(), s));
    k_union_offsets<<<1, 64, 0, s>>>(stream_off.as<int64_t>(), c_scan.as<int32_t>(), c_stream_off.as<int64_t>());
    JSW_HIP(hipGetLastError());
    if (fp32)
        k_union_gather<float><<<(unsigned)n_chunks, 64, 0, s>>>(
            c_flag.as<int32_t>(), c_scan.as<int32_t>(), n_chunks, ns, cblk.as<int32_t>(), pcode.as<int32_t>(),
            pa.as<float>(), pden.as<float>(), pk.p ? pk.as<uint64_t>() : nullptr, c_cblk.as<int32_t>(),
            c_pcode.as<int32_t>(), c_pa.as<float>(), c_pden.as<float>(), c_pk.p ? c_pk.as<uint64_t>() : nullptr);
    else
        k_union_gather<double><<<(unsigned)n_chunks, 64, 0, s>>>(
            c_flag.as<int32_t>(), c_scan.as<int32_t>(), n_chunks, ns, cblk.as<int32_t>(), pcode.as<int32_t>(),
            pa.as<double>(), pden.as<double>(), pk.p ? pk.as<uint64_t>() : nullptr, c_cblk.as<int32_t>(),
            c_pcode.as<int32_t>(), c_pa.as<double>(), c_pden.as<double>(), c_pk.p ? c_pk.as<uint64_t>() : nullptr);
    JSW_HIP(hipGetLastError());
    int64_t h = 0;
    JSW_HIP(hipMemcpyAsync(&h, c_stream_off.as<int64_t>() + kStreams, 8, hipMemcpyDeviceToHost, s));
    JSW_HIP(hipStreamSynchronize(s));
    c_chunks = h;
    compacted = true;
}

void UnionSweep::expand() {
    if (!compacted) return;
    compacted = false;
    // entries of chunks left out of the compacted launches hold fluxes
    pos_state[0] = pos_state[1] = 0;
}

void UnionSweep::fill_current(hipStream_t s) {
    const int want = fp32 ? 4 : 8;
    if (pos_state[cur] == want || A == 0) return;
    if (fp32)
        k_fill_empty<float><<<(int)std::min<int64_t>(ceil_div(A, 256), 8192), 256, 0, s>>>(pos[cur].as<float>(), A);
    else
        k_fill_empty<double><<<(int)std::min<int64_t>(ceil_div(A, 256), 8192), 256, 0, s>>>(pos[cur].as<double>(), A);
    JSW_HIP(hipGetLastError());
    pos_state[cur] = want;
}

template <class Real>
static void union_launch(UnionSweep &u, const int32_t *active, int waves_per_block, hipStream_t s) {
    // the full list, or the compacted one (same program stride)
    const bool c = u.compacted;
    const int64_t listed = c ? u.c_chunks : u.n_chunks;
    SweepArgs<Real> a;
    a.cblk = (c ? u.c_cblk : u.cblk).as<int32_t>();
    a.nc = 0;
    a.stride = 64 * u.n_chunks;
    a.pcode = (c ? u.c_pcode : u.pcode).as<int32_t>();
    a.pk = (u.pk.p && u.ns <= 3) ? (c ? u.c_pk : u.pk).as<uint64_t>() : nullptr;
    a.pa = (c ? u.c_pa : u.pa).as<Real>();
    a.pden = (c ? u.c_pden : u.pden).as<Real>();
    a.vs = u.vs.p;
    a.src_dir = nullptr;
    a.psi = nullptr;
    u.fill_current(s);
    a.psi_pos = u.pos[u.cur].as<Real>();
    a.pos_next = u.pos[1 - u.cur].as<Real>();
    u.pos_state[u.cur] = 0;
    u.pos_state[1 - u.cur] = (int)sizeof(Real);
    u.cur = 1 - u.cur;
    a.status = u.status.as<int32_t>();
    a.tickets = reinterpret_cast<uint32_t *>(u.status.as<char>() + 128);
    a.stream_off = (c ? u.c_stream_off : u.stream_off).as<int64_t>();
    a.lag_val = u.lag.as<Real>();
    a.psi_b = Real(0);
    a.grab = listed < (int64_t)1000000 ? 1 : 2;
    a.nap = 1;
    a.backoff = 3;
    a.watchdog_ticks = watchdog_ticks();
    a.stamps = nullptr;
    a.n_groups = 1;
    a.gs_pos = u.A;
    a.gs_den = a.stride;
    a.rows = u.rows.as<DirRow>();
    a.active = active;
    a.tag = 0;
    // default (measured on the 256-instance ensemble, time to 1e-8 with a
    // compacted list: 2 / 4 / 8 / 10 / 16 wavefronts 267 / 184 / 138 / 134
    // / 138 ms): the union's deepest instances need many chunks in flight
    const int wpb = waves_per_block > 0 ? std::min(16, waves_per_block) : 10;
    int64_t waves = (int64_t)u.n_cu * wpb;
    const int64_t need = std::max<int64_t>(1, listed);
    if (waves > need) waves = (need + wpb - 1) / wpb * wpb;
    const int blocks = (int)std::max<int64_t>(waves / wpb, kStreams);
    k_reset_tickets<<<1, 64, 0, s>>>(a.tickets);
    JSW_HIP(hipGetLastError());
    // kernel timing: recorded on the first instance's graph when its
    // profiling is on (not while a HIP graph is being recorded)
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    JSW_HIP(hipStreamIsCapturing(s, &cap));
    const bool prof = u.prof && u.prof->profile && cap == hipStreamCaptureStatusNone;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (prof) {
        JSW_HIP(hipEventCreate(&ev0));
        JSW_HIP(hipEventCreate(&ev1));
        JSW_HIP(hipEventRecord(ev0, s));
    }
    void *args[] = {&a};
    JSW_HIP(hipLaunchKernel(sweep_kernel_t<Real>(u.ns, false, a.pk != nullptr), dim3(blocks), dim3(64 * wpb), args, 0,
                            s));
    if (prof) {
        JSW_HIP(hipEventRecord(ev1, s));
        u.prof->prof_events.push_back({ev0, ev1});
    }
}

void UnionSweep::launch(const int32_t *active, int waves_per_block, hipStream_t s) {
    if (!n_chunks) return;
    if (fp32) union_launch<float>(*this, active, waves_per_block, s);
    else union_launch<double>(*this, active, waves_per_block, s);
}

int UnionSweep::check_status(hipStream_t s) {
    int32_t st = 0;
    JSW_HIP(hipMemcpyAsync(&st, status.p, 4, hipMemcpyDeviceToHost, s));
    JSW_HIP(hipStreamSynchronize(s));
    if (st == 0) return JSWEEP_OK;
    pos_state[0] = pos_state[1] = 0;
    JSW_HIP(hipMemsetAsync(status.p, 0, 64, s));
    JSW_HIP(hipStreamSynchronize(s));
    set_last_error(st & kStatusPlacement ? "a batched sweep workgroup ran on another XCD than its stream"
                                         : "a batched sweep wavefront's watchdog fired");
    return (st & kStatusPlacement) ? JSWEEP_E_PLACEMENT : JSWEEP_E_STALLED;
}

UnionSweep &union_for(int n, Graph *const *graphs, bool fp32, hipStream_t s) {
    std::vector<uint64_t> key(n + 1);
    for (int i = 0; i < n; ++i) key[i] = (graphs[i]->uid << 24) | (graphs[i]->prog_version & 0xffffffu);
    key[n] = fp32 ? 1 : 0;
    std::lock_guard<std::mutex> lock(g_union_mu);
    std::unique_ptr<UnionSweep> &slot = g_union[fp32 ? 1 : 0];
    if (!slot || slot->key != key) {
        slot.reset();   // free the old one first
        auto u = std::make_unique<UnionSweep>();
        u->build(n, graphs, fp32, s);
        u->key = key;
        slot = std::move(u);
    }
    slot->expand();   // every user starts from the full list
    return *slot;
}

}  // namespace jsw
