// Sweep dependency graph on the GPU: per (direction, cell) counts of
// upwind neighbours, longest-path levels by frontier propagation, the
// cycle-lag rule, the level-ordered cell lists and the sweep work list.
//
// A vertex is a (cell, direction) pair; an edge u -> v means v consumes
// the outgoing angular flux of u (paper Sec. V-A).  The count of a vertex
// is its number of upwind neighbours (Listing 1, init); vertices with count
// zero start the sweep, and a vertex's level is one more than the largest
// level among its upwind neighbours.
#include <cstring>

#include <algorithm>
#include <queue>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "common.hpp"

namespace jsw {

// ---------------------------------------------------------------------------
// lagged-edge lookup: lag_mv sorted by (m << 32 | v), ties by upwind cell
// ---------------------------------------------------------------------------
__device__ inline bool is_lagged(const uint64_t *lag_mv, const int32_t *lag_u, int64_t n_lag, int m, int64_t v,
                                 int64_t u) {
    return lag_index(lag_mv, lag_u, n_lag, m, v, u) >= 0;
}

// wavefront-aggregated append to a work list
__device__ inline void push_item(bool want, uint32_t item, uint32_t *list, uint32_t *count) {
    uint64_t mask = __ballot(want);
    if (!mask) return;
    int lane = threadIdx.x & 63;
    int leader = __ffsll((long long)mask) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(count, (uint32_t)__popcll(mask));
    base = __shfl(base, leader);
    if (want) list[base + __popcll(mask & ((1ull << lane) - 1))] = item;
}

template <int NF, int DIM>
__device__ inline double out_dot(const CellRec<double, NF, DIM> &r, int j, const double *om) {
    double d = om[0] * r.S[j][0] + om[1] * r.S[j][1];
    if constexpr (DIM == 3) d = d + om[2] * r.S[j][2];
    return d;
}

__device__ inline int64_t nbr_id(int32_t code) { return code <= -2 ? (int64_t)(-code - 2) : (int64_t)code; }

struct LagView {
    const uint64_t *mv;
    const int32_t *u;
    int64_t n;
};

// counts of non-lagged upwind neighbours; level 0 and the first frontier
template <int NF, int DIM>
__global__ void k_counts(const CellRec<double, NF, DIM> *rec, const double *omega, int64_t nc, int nd, LagView lag,
                         int32_t *cnt, int32_t *level, uint32_t *front, uint32_t *front_n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool push = false;
    if (i < nc * nd) {
        int m = (int)(i / nc);
        int64_t K = i - (int64_t)m * nc;
        const double om[3] = {omega[3 * m], omega[3 * m + 1], omega[3 * m + 2]};
        CellRec<double, NF, DIM> r = rec[K];
        int c = 0;
        for (int j = 0; j < NF; ++j) {
            int32_t code = r.nbr[j];
            if (code == -1) continue;
            if (out_dot(r, j, om) < 0.0) {
                if (code <= -2 && is_lagged(lag.mv, lag.u, lag.n, m, K, nbr_id(code))) continue;
                ++c;
            }
        }
        cnt[i] = c;
        level[i] = c == 0 ? 0 : -1;
        push = c == 0;
    }
    push_item(push, (uint32_t)i, front, front_n);
}

// one frontier step: release downwind neighbours of the vertices at level L
template <int NF, int DIM>
__global__ void k_level_step(const CellRec<double, NF, DIM> *rec, const double *omega, int64_t nc, LagView lag,
                             const uint32_t *front, uint32_t n_front, int32_t L, int32_t *cnt, int32_t *level,
                             uint32_t *next, uint32_t *next_n) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // every lane of a wavefront takes part in the aggregated pushes
    uint32_t item = t < n_front ? front[t] : 0;
    int m = (int)(item / nc);
    int64_t K = (int64_t)item - (int64_t)m * nc;
    CellRec<double, NF, DIM> r;
    double om[3] = {0, 0, 0};
    if (t < n_front) {
        r = rec[K];
        om[0] = omega[3 * m]; om[1] = omega[3 * m + 1]; om[2] = omega[3 * m + 2];
    }
    for (int j = 0; j < NF; ++j) {
        bool push = false;
        uint32_t w_item = 0;
        if (t < n_front) {
            int32_t code = r.nbr[j];
            if (code != -1 && out_dot(r, j, om) > 0.0) {
                int64_t w = nbr_id(code);
                bool lagged = code <= -2 && is_lagged(lag.mv, lag.u, lag.n, m, w, K);
                if (!lagged) {
                    w_item = (uint32_t)((int64_t)m * nc + w);
                    if (atomicSub(&cnt[w_item], 1) == 1) {
                        level[w_item] = L + 1;
                        push = true;
                    }
                }
            }
        }
        push_item(push, w_item, next, next_n);
    }
}

// backward trim of the unlevelled residue: out-counts towards residue
template <int NF, int DIM>
__global__ void k_trim_init(const CellRec<double, NF, DIM> *rec, const double *omega, int64_t nc, int nd,
                            int32_t *level, int32_t *ocnt, uint32_t *front, uint32_t *front_n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool push = false;
    if (i < nc * nd && level[i] == -1) {
        int m = (int)(i / nc);
        int64_t K = i - (int64_t)m * nc;
        const double om[3] = {omega[3 * m], omega[3 * m + 1], omega[3 * m + 2]};
        CellRec<double, NF, DIM> r = rec[K];
        int c = 0;
        for (int j = 0; j < NF; ++j) {
            int32_t code = r.nbr[j];
            if (code == -1 || !(out_dot(r, j, om) > 0.0)) continue;
            if (level[(int64_t)m * nc + nbr_id(code)] == -1) ++c;
        }
        ocnt[i] = c;
        push = c == 0;
    }
    push_item(push, (uint32_t)i, front, front_n);
}

// mark the seeds of a trim step as removed (level -2)
__global__ void k_trim_mark(const uint32_t *front, uint32_t n, int32_t *level) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) level[front[t]] = -2;
}

template <int NF, int DIM>
__global__ void k_trim_step(const CellRec<double, NF, DIM> *rec, const double *omega, int64_t nc,
                            const uint32_t *front, uint32_t n_front, int32_t *level, int32_t *ocnt, uint32_t *next,
                            uint32_t *next_n) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t item = t < n_front ? front[t] : 0;
    int m = (int)(item / nc);
    int64_t K = (int64_t)item - (int64_t)m * nc;
    CellRec<double, NF, DIM> r;
    double om[3] = {0, 0, 0};
    if (t < n_front) {
        r = rec[K];
        om[0] = omega[3 * m]; om[1] = omega[3 * m + 1]; om[2] = omega[3 * m + 2];
    }
    for (int j = 0; j < NF; ++j) {
        bool push = false;
        uint32_t u_item = 0;
        if (t < n_front) {
            int32_t code = r.nbr[j];
            if (code != -1 && out_dot(r, j, om) < 0.0) {
                u_item = (uint32_t)((int64_t)m * nc + nbr_id(code));
                if (level[u_item] == -1 && atomicSub(&ocnt[u_item], 1) == 1) {
                    level[u_item] = -2;
                    push = true;
                }
            }
        }
        push_item(push, u_item, next, next_n);
    }
}

// edges among the remaining residue vertices (those on or between cycles)
template <int NF, int DIM>
__global__ void k_core_edges(const CellRec<double, NF, DIM> *rec, const double *omega, int64_t nc, int nd,
                             const int32_t *level, uint32_t *edges, uint32_t *n_edges, uint32_t cap) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc * nd || level[i] != -1) return;
    int m = (int)(i / nc);
    int64_t K = i - (int64_t)m * nc;
    const double om[3] = {omega[3 * m], omega[3 * m + 1], omega[3 * m + 2]};
    CellRec<double, NF, DIM> r = rec[K];
    for (int j = 0; j < NF; ++j) {
        int32_t code = r.nbr[j];
        if (code == -1 || !(out_dot(r, j, om) < 0.0)) continue;
        int64_t u = nbr_id(code);
        if (level[(int64_t)m * nc + u] != -1) continue;
        uint32_t e = atomicAdd(n_edges, 1u);
        if (e < cap) {
            edges[3 * (int64_t)e] = (uint32_t)m;
            edges[3 * (int64_t)e + 1] = (uint32_t)u;
            edges[3 * (int64_t)e + 2] = (uint32_t)K;
        }
    }
}

// mark both records of a lagged face as lag candidates
template <int NF, int DIM>
__global__ void k_mark_lag(CellRec<double, NF, DIM> *rec, const uint64_t *lag_mv, const int32_t *lag_u, int64_t n) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    int64_t v = (int64_t)(lag_mv[e] & 0xffffffffull);
    int64_t u = lag_u[e];
    for (int j = 0; j < NF; ++j) {
        if (nbr_id(rec[v].nbr[j]) == u && rec[v].nbr[j] != -1) rec[v].nbr[j] = (int32_t)(-u - 2);
        if (nbr_id(rec[u].nbr[j]) == v && rec[u].nbr[j] != -1) rec[u].nbr[j] = (int32_t)(-v - 2);
    }
}

__global__ void k_level_keys(const int32_t *level, int64_t nc, int nd, int cell_bits, int lev_bits, uint64_t *keys) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc * nd) return;
    int m = (int)(i / nc);
    int64_t K = i - (int64_t)m * nc;
    keys[i] = ((uint64_t)m << (lev_bits + cell_bits)) | ((uint64_t)level[i] << cell_bits) | (uint64_t)K;
}

__global__ void k_level_bounds(const uint64_t *keys, int64_t nc, int nd, int cell_bits, int lev_bits, int32_t Lcap,
                               int32_t *lvl_cells, int64_t *starts, int32_t *nlev) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc * nd) return;
    uint64_t k = keys[i];
    uint64_t cmask = (1ull << cell_bits) - 1;
    lvl_cells[i] = (int32_t)(k & cmask);
    int m = (int)(k >> (lev_bits + cell_bits));
    int32_t L = (int32_t)((k >> cell_bits) & ((1ull << lev_bits) - 1));
    bool head = i == 0 || (keys[i - 1] >> cell_bits) != (k >> cell_bits);
    if (head) {
        starts[(int64_t)m * (Lcap + 1) + L] = i - (int64_t)m * nc;
        atomicMax(&nlev[m], L + 1);
    }
}

static int bits_for(int64_t n) {
    int b = 1;
    while ((1ll << b) < n) ++b;
    return b;
}

template <int NF, int DIM>
static int64_t run_levels(Graph &g, const LagView &lag, DevBuf &cnt, DevBuf &fa, DevBuf &fb, DevBuf &ctr,
                          int32_t *maxL, hipStream_t s) {
    using Rec = CellRec<double, NF, DIM>;
    const int64_t N = g.nc * g.nd;
    const int B = 256;
    uint32_t *counters = ctr.as<uint32_t>();
    JSW_HIP(hipMemsetAsync(counters, 0, 8, s));
    k_counts<NF, DIM><<<(int)ceil_div(N, B), B, 0, s>>>(g.rec64.as<Rec>(), g.omega64.as<double>(), g.nc, g.nd, lag,
                                                       cnt.as<int32_t>(), g.level.as<int32_t>(), fa.as<uint32_t>(),
                                                       counters);
    JSW_HIP(hipGetLastError());
    uint32_t n_front = 0;
    JSW_HIP(hipMemcpyAsync(&n_front, counters, 4, hipMemcpyDeviceToHost, s));
    JSW_HIP(hipStreamSynchronize(s));
    int64_t done = 0;
    int32_t L = 0;
    uint32_t *cur = fa.as<uint32_t>(), *nxt = fb.as<uint32_t>();
    while (n_front > 0) {
        done += n_front;
        JSW_HIP(hipMemsetAsync(counters + 1, 0, 4, s));
        k_level_step<NF, DIM><<<(int)ceil_div(n_front, B), B, 0, s>>>(g.rec64.as<Rec>(), g.omega64.as<double>(), g.nc,
                                                                     lag, cur, n_front, L, cnt.as<int32_t>(),
                                                                     g.level.as<int32_t>(), nxt, counters + 1);
        JSW_HIP(hipGetLastError());
        JSW_HIP(hipMemcpyAsync(&n_front, counters + 1, 4, hipMemcpyDeviceToHost, s));
        JSW_HIP(hipStreamSynchronize(s));
        if (n_front) ++L;
        std::swap(cur, nxt);
    }
    *maxL = L;
    return done;
}

// Tarjan's strongly connected components on a small host graph
static void tarjan_small(int n, const std::vector<std::vector<int>> &adj, std::vector<int> &comp, std::vector<int> &csize) {
    std::vector<int> idx(n, -1), low(n, 0), stk;
    std::vector<char> on(n, 0);
    std::vector<std::pair<int, size_t>> call;
    int counter = 0;
    comp.assign(n, -1);
    csize.clear();
    for (int s0 = 0; s0 < n; ++s0) {
        if (idx[s0] >= 0) continue;
        call.push_back({s0, 0});
        idx[s0] = low[s0] = counter++;
        stk.push_back(s0);
        on[s0] = 1;
        while (!call.empty()) {
            int v = call.back().first;
            size_t &it = call.back().second;
            if (it < adj[v].size()) {
                int w = adj[v][it++];
                if (idx[w] < 0) {
                    idx[w] = low[w] = counter++;
                    stk.push_back(w);
                    on[w] = 1;
                    call.push_back({w, 0});
                } else if (on[w]) {
                    low[v] = std::min(low[v], idx[w]);
                }
            } else {
                if (low[v] == idx[v]) {
                    int c = (int)csize.size(), sz = 0, w;
                    do { w = stk.back(); stk.pop_back(); on[w] = 0; comp[w] = c; ++sz; } while (w != v);
                    csize.push_back(sz);
                }
                call.pop_back();
                if (!call.empty()) low[call.back().first] = std::min(low[call.back().first], low[v]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// coarsened graph (paper Sec. V-E): clusters are the work-list chunks, and a
// chunk's in-edges are the distinct chunks holding its vertices' upwind
// neighbours (lagged edges excluded).  Every such chunk has a lower level,
// hence comes earlier in the stream: the coarsened graph is acyclic.
// ---------------------------------------------------------------------------
__global__ void k_chunk_pos(const Chunk *chunks, int64_t n_chunks, const int32_t *lvl_cells, int64_t nc, int32_t *pos) {
    int64_t c = blockIdx.x;
    int lane = threadIdx.x;
    if (c >= n_chunks) return;
    Chunk ch = chunks[c];
    int m = (int)(ch.a & 0xffffu), cnt = (int)(ch.a >> 16) + 1;
    if (lane < cnt) {
        int64_t base = (int64_t)m * nc;
        pos[base + lvl_cells[base + ch.b + lane]] = (int32_t)c;
    }
}

// Chunk block: everything a wavefront needs to start a chunk, in one
// contiguous record it reads in a single memory round trip: the cells
// (-1 past the end), the descriptor, and the upwind chunks inline when they
// fit (else the count is -1 and the CSR lists are used).
__global__ void k_chunk_block(const Chunk *chunks, int64_t n_chunks, const int32_t *lvl_cells, int64_t nc,
                              const int32_t *dep_ptr, const int32_t *dep, int32_t *blk) {
    int64_t c = blockIdx.x;
    int lane = threadIdx.x;
    if (c >= n_chunks) return;
    Chunk ch = chunks[c];
    int m = (int)(ch.a & 0xffffu), cnt = (int)(ch.a >> 16) + 1;
    int32_t *b = blk + c * kBlock;
    b[lane] = lane < cnt ? lvl_cells[(int64_t)m * nc + ch.b + lane] : -1;
    int32_t d0 = dep_ptr[c], nd = dep_ptr[c + 1] - d0;
    bool inl = nd <= kBlockDeps;
    if (lane == 0) b[64] = (int32_t)ch.a;
    if (lane == 1) b[65] = inl ? nd : -1;
    if (lane == 2) b[66] = (int32_t)ch.b;
    if (lane < kBlockDeps) b[67 + lane] = inl && lane < nd ? dep[d0 + lane] : -1;
}

// ---------------------------------------------------------------------------
// Sweep program (layout in common.hpp): the inflow faces of every chunk
// lane, classified exactly as in the graph (FP64 Omega . S, left to right),
// so the sweep reads coalesced per-lane streams instead of cell records.
// COUNT = true: the largest number of inflow faces of any vertex.
// ---------------------------------------------------------------------------
template <int NF, int DIM, bool COUNT>
__global__ void k_program(const int32_t *blk, int64_t n_chunks, const CellRec<double, NF, DIM> *rec,
                          const double *omega, LagView lag, const int32_t *posi, int64_t nc, int ns, int32_t *max_in,
                          int32_t *code, double *a) {
    const int64_t c = blockIdx.x;
    const int lane = threadIdx.x;
    if (c >= n_chunks) return;
    const int64_t S = 64 * n_chunks, idx = c * 64 + lane;
    const int32_t K = blk[c * kBlock + lane];
    const int m = (int)((uint32_t)blk[c * kBlock + 64] & 0xffffu);
    int n = 0;
    if (K >= 0) {
        const CellRec<double, NF, DIM> r = rec[K];
        const double om[3] = {omega[3 * m], omega[3 * m + 1], omega[3 * m + 2]};
        for (int j = 0; j < NF; ++j) {
            const double d = out_dot(r, j, om);
            if (!(d < 0.0)) continue;
            if (!COUNT) {
                const int32_t nb = r.nbr[j];
                int32_t cd = -1;
                if (nb != -1) {
                    const int64_t u = nbr_id(nb);
                    const int64_t e = nb <= -2 ? lag_index(lag.mv, lag.u, lag.n, m, K, u) : -1;
                    cd = e >= 0 ? (int32_t)(-(e + 2)) : posi[(int64_t)m * nc + u];
                }
                code[n * S + idx] = cd;
                a[n * S + idx] = -d;
            }
            ++n;
        }
    }
    if (COUNT) {
        if (n > 0) atomicMax(max_in, n);
    } else {
        for (int j = n; j < ns; ++j) {
            code[j * S + idx] = kNoFace;
            a[j * S + idx] = 0.0;
        }
    }
}

// Compact FP64 program (common.hpp): one 64-lane workgroup per chunk copies
// its lanes' first kCompactSlots slots and appends the rest, slot by slot
// and lane by lane, as entries of the chunk block; *too_many is set when a
// chunk has more than kBlockExtra of them.
__global__ void k_compact(int32_t *blk, int64_t n_chunks, int ns, const int32_t *code, const double *a,
                          int32_t *code3, double *a3, int32_t *too_many) {
    const int64_t c = blockIdx.x;
    const int lane = threadIdx.x;
    if (c >= n_chunks) return;
    const int64_t S = 64 * n_chunks, idx = c * 64 + lane;
    for (int j = 0; j < kCompactSlots; ++j) {
        code3[j * S + idx] = code[j * S + idx];
        a3[j * S + idx] = a[j * S + idx];
    }
    int32_t *b = blk + c * kBlock;
    int n = 0;
    for (int j = kCompactSlots; j < ns; ++j) {
        const int32_t cd = code[j * S + idx];
        const bool has = cd != kNoFace;
        const uint64_t mask = __ballot(has);
        const int e = n + __popcll(mask & ((1ull << lane) - 1ull));
        if (has && e < kBlockExtra) {
            const uint64_t bits = (uint64_t)__double_as_longlong(a[j * S + idx]);
            b[67 + 4 * e] = lane | (j << 8);
            b[68 + 4 * e] = cd;
            b[69 + 4 * e] = (int32_t)(uint32_t)bits;
            b[70 + 4 * e] = (int32_t)(uint32_t)(bits >> 32);
        }
        n += __popcll(mask);
    }
    if (lane == 0) {
        b[65] = n;
        if (n > kBlockExtra) atomicOr(too_many, 1);
    }
}

// packed codes of a program of at most 3 slots without compact entries
static void build_packed(Graph &g, hipStream_t s) {
    g.pk.release();
    if (g.ns > 3 || g.ns_x > 0 || !g.n_chunks) return;
    g.pk.alloc(8 * (size_t)(64 * g.n_chunks));
    if (!pack_codes(g.cblk.as<int32_t>(), g.n_chunks, g.ns, g.pcode.as<int32_t>(), g.pk.as<uint64_t>(), s))
        g.pk.release();
}

static void build_compact(Graph &g, hipStream_t s) {
    g.ns_x = 0;
    g.pcode3.release();
    g.pa3.release();
    if (g.ns <= kCompactSlots || !g.n_chunks) return;
    const int64_t nch = g.n_chunks, S = 64 * nch;
    g.pcode3.alloc(4 * (size_t)kCompactSlots * S);
    g.pa3.alloc(8 * (size_t)kCompactSlots * S);
    DevBuf flag(4);
    JSW_HIP(hipMemsetAsync(flag.p, 0, 4, s));
    k_compact<<<(unsigned)nch, 64, 0, s>>>(g.cblk.as<int32_t>(), nch, g.ns, g.pcode.as<int32_t>(), g.pa64.as<double>(),
                                           g.pcode3.as<int32_t>(), g.pa3.as<double>(), flag.as<int32_t>());
    JSW_HIP(hipGetLastError());
    int32_t too_many = 0;
    JSW_HIP(hipMemcpyAsync(&too_many, flag.p, 4, hipMemcpyDeviceToHost, s));
    JSW_HIP(hipStreamSynchronize(s));
    if (too_many) {
        g.pcode3.release();
        g.pa3.release();
        return;
    }
    g.ns_x = g.ns - kCompactSlots;
}

// coefficient of every lagged edge, from the program slot that names it
__global__ void k_lag_coef(const int32_t *code, const double *a, int64_t n, double *lag_a) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t cd = code[i];
    if (cd <= -2 && cd != kNoFace) lag_a[-(int64_t)cd - 2] = a[i];
}

__global__ void k_positions(const int32_t *lvl_cells, int64_t nc, int64_t n, int32_t *posi) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t m = i / nc;
    posi[m * nc + lvl_cells[i]] = (int32_t)(i - m * nc);
}

template <int NF, int DIM>
static void build_program(Graph &g, const LagView &lag, hipStream_t s) {
    using Rec = CellRec<double, NF, DIM>;
    const int64_t nch = g.n_chunks, S = 64 * nch;
    DevBuf mx(4);
    JSW_HIP(hipMemsetAsync(mx.p, 0, 4, s));
    k_program<NF, DIM, true><<<(unsigned)nch, 64, 0, s>>>(g.cblk.as<int32_t>(), nch, g.rec64.as<Rec>(),
                                                          g.omega64.as<double>(), lag, nullptr, g.nc, 0,
                                                          mx.as<int32_t>(), nullptr, nullptr);
    JSW_HIP(hipGetLastError());
    int32_t ns = 0;
    JSW_HIP(hipMemcpyAsync(&ns, mx.p, 4, hipMemcpyDeviceToHost, s));
    JSW_HIP(hipStreamSynchronize(s));
    g.ns = std::max(1, (int)ns);
    g.pcode.alloc(4 * (size_t)g.ns * S);
    g.pa64.alloc(8 * (size_t)g.ns * S);
    // position of every vertex in its direction's level order
    const int64_t N = g.nc * g.nd;
    g.posi.alloc(4 * N);
    DevBuf &posi = g.posi;
    k_positions<<<(unsigned)ceil_div(N, 256), 256, 0, s>>>(g.lvl_cells.as<int32_t>(), g.nc, N, posi.as<int32_t>());
    JSW_HIP(hipGetLastError());
    k_program<NF, DIM, false><<<(unsigned)nch, 64, 0, s>>>(g.cblk.as<int32_t>(), nch, g.rec64.as<Rec>(),
                                                           g.omega64.as<double>(), lag, posi.as<int32_t>(), g.nc,
                                                           g.ns, nullptr, g.pcode.as<int32_t>(), g.pa64.as<double>());
    JSW_HIP(hipGetLastError());
    g.pden64.alloc(8 * (size_t)S);
    g.den64_ok = g.den32_ok = false;
    if (g.n_lag) {
        g.lag_a.alloc(8 * g.n_lag);
        k_lag_coef<<<(unsigned)ceil_div((int64_t)g.ns * S, 256), 256, 0, s>>>(g.pcode.as<int32_t>(), g.pa64.as<double>(),
                                                                           (int64_t)g.ns * S, g.lag_a.as<double>());
        JSW_HIP(hipGetLastError());
    }
}

// one 64-lane workgroup per chunk: gather the upwind chunks of its
// vertices and keep the first occurrence of each; WRITE = 0 counts them
template <int NF, int DIM, bool WRITE>
__global__ void k_chunk_deps(const Chunk *chunks, int64_t n_chunks, const int32_t *lvl_cells,
                             const CellRec<double, NF, DIM> *rec, const double *omega, int64_t nc, LagView lag,
                             const int32_t *pos, int32_t *count, const int32_t *ptr, int32_t *dep) {
    __shared__ int32_t cand[64 * NF];
    int64_t c = blockIdx.x;
    int lane = threadIdx.x;
    Chunk ch = chunks[c];
    int m = (int)(ch.a & 0xffffu), cnt = (int)(ch.a >> 16) + 1;
    int64_t base = (int64_t)m * nc;
    for (int j = 0; j < NF; ++j) cand[lane * NF + j] = -1;
    if (lane < cnt) {
        int64_t K = lvl_cells[base + ch.b + lane];
        CellRec<double, NF, DIM> r = rec[K];
        const double om[3] = {omega[3 * m], omega[3 * m + 1], omega[3 * m + 2]};
        for (int j = 0; j < NF; ++j) {
            int32_t code = r.nbr[j];
            if (code == -1 || !(out_dot(r, j, om) < 0.0)) continue;
            int64_t u = nbr_id(code);
            if (code <= -2 && is_lagged(lag.mv, lag.u, lag.n, m, K, u)) continue;
            cand[lane * NF + j] = pos[base + u];
        }
    }
    __syncthreads();
    int32_t total = 0;
    for (int i0 = 0; i0 < 64 * NF; i0 += 64) {
        int i = i0 + lane;
        int32_t v = cand[i];
        bool keep = v >= 0;
        for (int k = 0; k < i && keep; ++k) keep = cand[k] != v;
        uint64_t mask = __ballot(keep);
        if (WRITE && keep) dep[ptr[c] + total + __popcll(mask & ((1ull << lane) - 1))] = v;
        total += __popcll(mask);
    }
    if (!WRITE && lane == 0) count[c] = total;
}

__global__ void k_exclusive_to_ptr(const int32_t *incl, int64_t n, int32_t *ptr) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) ptr[0] = 0;
    if (i < n) ptr[i + 1] = incl[i];
}

template <int NF, int DIM>
static void build_coarsened(Graph &g, const LagView &lag, hipStream_t s) {
    using Rec = CellRec<double, NF, DIM>;
    const int64_t N = g.nc * g.nd, nch = g.n_chunks;
    DevBuf pos(4 * N), count(4 * std::max<int64_t>(1, nch)), incl(4 * std::max<int64_t>(1, nch));
    g.dep_ptr.alloc(4 * (nch + 1));
    k_chunk_pos<<<(unsigned)nch, 64, 0, s>>>(g.chunks.as<Chunk>(), nch, g.lvl_cells.as<int32_t>(), g.nc, pos.as<int32_t>());
    JSW_HIP(hipGetLastError());
    k_chunk_deps<NF, DIM, false><<<(unsigned)nch, 64, 0, s>>>(g.chunks.as<Chunk>(), nch, g.lvl_cells.as<int32_t>(),
                                                              g.rec64.as<Rec>(), g.omega64.as<double>(), g.nc, lag,
                                                              pos.as<int32_t>(), count.as<int32_t>(), nullptr, nullptr);
    JSW_HIP(hipGetLastError());
    size_t tmp_bytes = 0;
    JSW_HIP(rocprim::inclusive_scan(nullptr, tmp_bytes, count.as<int32_t>(), incl.as<int32_t>(), (size_t)nch,
                                    rocprim::plus<int32_t>(), s));
    {
        DevBuf tmp(tmp_bytes + 16);
        JSW_HIP(rocprim::inclusive_scan(tmp.p, tmp_bytes, count.as<int32_t>(), incl.as<int32_t>(), (size_t)nch,
                                        rocprim::plus<int32_t>(), s));
    }
    k_exclusive_to_ptr<<<(int)ceil_div(nch, 256), 256, 0, s>>>(incl.as<int32_t>(), nch, g.dep_ptr.as<int32_t>());
    JSW_HIP(hipGetLastError());
    int32_t total = 0;
    JSW_HIP(hipMemcpyAsync(&total, incl.as<int32_t>() + (nch - 1), 4, hipMemcpyDeviceToHost, s));
    JSW_HIP(hipStreamSynchronize(s));
    g.n_dep = total;
    g.dep.alloc(4 * std::max<int64_t>(1, total));
    k_chunk_deps<NF, DIM, true><<<(unsigned)nch, 64, 0, s>>>(g.chunks.as<Chunk>(), nch, g.lvl_cells.as<int32_t>(),
                                                             g.rec64.as<Rec>(), g.omega64.as<double>(), g.nc, lag,
                                                             pos.as<int32_t>(), nullptr, g.dep_ptr.as<int32_t>(),
                                                             g.dep.as<int32_t>());
    JSW_HIP(hipGetLastError());
    g.cblk.alloc(4 * (size_t)kBlock * std::max<int64_t>(1, nch));
    k_chunk_block<<<(unsigned)nch, 64, 0, s>>>(g.chunks.as<Chunk>(), nch, g.lvl_cells.as<int32_t>(), g.nc,
                                               g.dep_ptr.as<int32_t>(), g.dep.as<int32_t>(), g.cblk.as<int32_t>());
    JSW_HIP(hipGetLastError());
    JSW_HIP(hipStreamSynchronize(s));
}

template <int NF, int DIM>
static void dag_impl(Graph &g, bool lag_cycles, hipStream_t s) {
    using Rec = CellRec<double, NF, DIM>;
    const int64_t nc = g.nc, N = nc * g.nd;
    const int B = 256;
    g.level.alloc(4 * N);
    DevBuf cnt(4 * N), fa(4 * N), fb(4 * N), ctr(16);
    LagView lag{nullptr, nullptr, 0};
    int32_t maxL = 0;
    int64_t done = run_levels<NF, DIM>(g, lag, cnt, fa, fb, ctr, &maxL, s);
    if (done < N) {
        // cycles: trim everything that is only downstream of a cycle, then
        // find the strongly connected components of the small remainder
        if (!lag_cycles) fail(JSWEEP_E_CYCLE, "the sweep graph has a cycle and lagging is disabled");
        uint32_t *counters = ctr.as<uint32_t>();
        JSW_HIP(hipMemsetAsync(counters, 0, 8, s));
        k_trim_init<NF, DIM><<<(int)ceil_div(N, B), B, 0, s>>>(g.rec64.as<Rec>(), g.omega64.as<double>(), nc, g.nd,
                                                              g.level.as<int32_t>(), cnt.as<int32_t>(),
                                                              fa.as<uint32_t>(), counters);
        JSW_HIP(hipGetLastError());
        uint32_t n_front = 0;
        JSW_HIP(hipMemcpyAsync(&n_front, counters, 4, hipMemcpyDeviceToHost, s));
        JSW_HIP(hipStreamSynchronize(s));
        uint32_t *cur = fa.as<uint32_t>(), *nxt = fb.as<uint32_t>();
        if (n_front) k_trim_mark<<<(int)ceil_div(n_front, B), B, 0, s>>>(cur, n_front, g.level.as<int32_t>());
        while (n_front > 0) {
            JSW_HIP(hipMemsetAsync(counters + 1, 0, 4, s));
            k_trim_step<NF, DIM><<<(int)ceil_div(n_front, B), B, 0, s>>>(g.rec64.as<Rec>(), g.omega64.as<double>(), nc,
                                                                        cur, n_front, g.level.as<int32_t>(),
                                                                        cnt.as<int32_t>(), nxt, counters + 1);
            JSW_HIP(hipGetLastError());
            JSW_HIP(hipMemcpyAsync(&n_front, counters + 1, 4, hipMemcpyDeviceToHost, s));
            JSW_HIP(hipStreamSynchronize(s));
            std::swap(cur, nxt);
        }
        uint32_t cap = (uint32_t)std::min<int64_t>(N * NF, (int64_t)1 << 28);
        DevBuf edges(12ull * cap);
        JSW_HIP(hipMemsetAsync(counters + 2, 0, 4, s));
        k_core_edges<NF, DIM><<<(int)ceil_div(N, B), B, 0, s>>>(g.rec64.as<Rec>(), g.omega64.as<double>(), nc, g.nd,
                                                               g.level.as<int32_t>(), edges.as<uint32_t>(),
                                                               counters + 2, cap);
        JSW_HIP(hipGetLastError());
        uint32_t ne = 0;
        JSW_HIP(hipMemcpyAsync(&ne, counters + 2, 4, hipMemcpyDeviceToHost, s));
        JSW_HIP(hipStreamSynchronize(s));
        if (ne > cap) fail(JSWEEP_E_OOM, "too many cyclic edges");
        std::vector<uint32_t> he(3ull * ne);
        if (ne) JSW_HIP(hipMemcpy(he.data(), edges.p, 12ull * ne, hipMemcpyDeviceToHost));
        // per direction: SCCs; lag u -> v with u > v inside a non-trivial one
        std::vector<size_t> order(ne);
        for (size_t e = 0; e < ne; ++e) order[e] = e;
        std::sort(order.begin(), order.end(), [&](size_t a, size_t b) { return he[3 * a] < he[3 * b]; });
        struct LagRec { uint32_t m; int64_t v, u; };
        std::vector<LagRec> lags;
        for (size_t a = 0; a < ne;) {
            size_t b = a;
            uint32_t m = he[3 * order[a]];
            while (b < ne && he[3 * order[b]] == m) ++b;
            std::vector<int64_t> ids;
            for (size_t e = a; e < b; ++e) { ids.push_back(he[3 * order[e] + 1]); ids.push_back(he[3 * order[e] + 2]); }
            std::sort(ids.begin(), ids.end());
            ids.erase(std::unique(ids.begin(), ids.end()), ids.end());
            auto loc = [&](int64_t x) { return (int)(std::lower_bound(ids.begin(), ids.end(), x) - ids.begin()); };
            std::vector<std::vector<int>> adj(ids.size());
            for (size_t e = a; e < b; ++e) adj[loc(he[3 * order[e] + 1])].push_back(loc(he[3 * order[e] + 2]));
            std::vector<int> comp, csize;
            tarjan_small((int)ids.size(), adj, comp, csize);
            for (size_t e = a; e < b; ++e) {
                int64_t u = he[3 * order[e] + 1], v = he[3 * order[e] + 2];
                int cu = comp[loc(u)], cv = comp[loc(v)];
                if (cu == cv && csize[cu] > 1 && u > v) lags.push_back({m, v, u});
            }
            a = b;
        }
        std::sort(lags.begin(), lags.end(), [](const LagRec &x, const LagRec &y) {
            if (x.m != y.m) return x.m < y.m;
            if (x.v != y.v) return x.v < y.v;
            return x.u < y.u;
        });
        g.n_lag = (int64_t)lags.size();
        if (g.n_lag == 0) fail(JSWEEP_E_DEVICE, "unlevelled vertices without a cycle");
        std::vector<uint64_t> mv(g.n_lag);
        std::vector<int32_t> uu(g.n_lag);
        for (int64_t e = 0; e < g.n_lag; ++e) {
            mv[e] = ((uint64_t)lags[e].m << 32) | (uint64_t)lags[e].v;
            uu[e] = (int32_t)lags[e].u;
        }
        g.lag_mv.alloc(8 * g.n_lag);
        g.lag_u.alloc(4 * g.n_lag);
        JSW_HIP(hipMemcpyAsync(g.lag_mv.p, mv.data(), 8 * g.n_lag, hipMemcpyHostToDevice, s));
        JSW_HIP(hipMemcpyAsync(g.lag_u.p, uu.data(), 4 * g.n_lag, hipMemcpyHostToDevice, s));
        k_mark_lag<NF, DIM><<<(int)ceil_div(g.n_lag, B), B, 0, s>>>(g.rec64.as<Rec>(), g.lag_mv.as<uint64_t>(),
                                                                   g.lag_u.as<int32_t>(), g.n_lag);
        JSW_HIP(hipGetLastError());
        g.lag_m_h.resize(g.n_lag);
        g.lag_u_h.resize(g.n_lag);
        g.lag_v_h.resize(g.n_lag);
        for (int64_t e = 0; e < g.n_lag; ++e) {
            g.lag_m_h[e] = (int32_t)lags[e].m;
            g.lag_u_h[e] = lags[e].u;
            g.lag_v_h[e] = lags[e].v;
        }
        // the (direction, downwind cell) groups of every downwind cell, in
        // ascending direction (compressed rows by cell)
        {
            std::vector<int32_t> ptr(nc + 1, 0), grp;
            for (int64_t e = 0; e < g.n_lag; ++e)
                if (e == 0 || mv[e - 1] != mv[e]) ++ptr[lags[e].v + 1];
            for (int64_t v = 0; v < nc; ++v) ptr[v + 1] += ptr[v];
            grp.resize(ptr[nc]);
            std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
            for (int64_t e = 0; e < g.n_lag; ++e)
                if (e == 0 || mv[e - 1] != mv[e]) grp[fill[lags[e].v]++] = (int32_t)e;
            // groups were visited in (m, v) order, so each cell's are in ascending m
            g.lag_cptr.alloc(4 * (nc + 1));
            g.lag_cgrp.alloc(4 * std::max<size_t>(1, grp.size()));
            JSW_HIP(hipMemcpyAsync(g.lag_cptr.p, ptr.data(), 4 * (nc + 1), hipMemcpyHostToDevice, s));
            if (!grp.empty())
                JSW_HIP(hipMemcpyAsync(g.lag_cgrp.p, grp.data(), 4 * grp.size(), hipMemcpyHostToDevice, s));
            JSW_HIP(hipStreamSynchronize(s));   // before the host vectors go
        }
        lag = LagView{g.lag_mv.as<uint64_t>(), g.lag_u.as<int32_t>(), g.n_lag};
        done = run_levels<NF, DIM>(g, lag, cnt, fa, fb, ctr, &maxL, s);
        if (done < N) fail(JSWEEP_E_DEVICE, "cycles remain after lagging");
        g.lag_val64.alloc(8 * g.n_lag);
        g.lag_val32.alloc(4 * g.n_lag);
    }
    cnt.release();
    fb.release();
    // level-ordered cell lists: sort (direction, level, cell) keys
    const int cell_bits = bits_for(nc + 1), lev_bits = bits_for((int64_t)maxL + 2), dir_bits = bits_for(g.nd + 1);
    if (cell_bits + lev_bits + dir_bits > 64) fail(JSWEEP_E_INVALID_ARG, "graph too large for 64-bit level keys");
    DevBuf keys(8 * N), keys2(8 * N);
    k_level_keys<<<(int)ceil_div(N, B), B, 0, s>>>(g.level.as<int32_t>(), nc, g.nd, cell_bits, lev_bits,
                                                   keys.as<uint64_t>());
    JSW_HIP(hipGetLastError());
    size_t tmp_bytes = 0;
    unsigned end_bit = (unsigned)(cell_bits + lev_bits + dir_bits);
    JSW_HIP(rocprim::radix_sort_keys(nullptr, tmp_bytes, keys.as<uint64_t>(), keys2.as<uint64_t>(), (size_t)N, 0u,
                                     end_bit, s));
    {
        DevBuf tmp(tmp_bytes + 16);
        JSW_HIP(rocprim::radix_sort_keys(tmp.p, tmp_bytes, keys.as<uint64_t>(), keys2.as<uint64_t>(), (size_t)N, 0u,
                                         end_bit, s));
    }
    keys.release();
    g.lvl_cells.alloc(4 * N);
    const int32_t Lcap = maxL + 1;
    DevBuf starts(8 * (int64_t)g.nd * (Lcap + 1)), nlev(4 * g.nd);
    JSW_HIP(hipMemsetAsync(nlev.p, 0, 4 * g.nd, s));
    k_level_bounds<<<(int)ceil_div(N, B), B, 0, s>>>(keys2.as<uint64_t>(), nc, g.nd, cell_bits, lev_bits, Lcap,
                                                     g.lvl_cells.as<int32_t>(), starts.as<int64_t>(), nlev.as<int32_t>());
    JSW_HIP(hipGetLastError());
    std::vector<int64_t> hstarts((size_t)g.nd * (Lcap + 1));
    g.nlev_h.resize(g.nd);
    JSW_HIP(hipMemcpyAsync(hstarts.data(), starts.p, starts.bytes, hipMemcpyDeviceToHost, s));
    JSW_HIP(hipMemcpyAsync(g.nlev_h.data(), nlev.p, 4 * g.nd, hipMemcpyDeviceToHost, s));
    JSW_HIP(hipStreamSynchronize(s));
    g.lvl_off_h.assign(g.nd + 1, 0);
    g.max_levels = 0;
    for (int m = 0; m < g.nd; ++m) {
        g.lvl_off_h[m + 1] = g.lvl_off_h[m] + g.nlev_h[m] + 1;
        g.max_levels = std::max(g.max_levels, g.nlev_h[m]);
    }
    g.lvl_ptr_h.resize(g.lvl_off_h[g.nd]);
    for (int m = 0; m < g.nd; ++m) {
        int64_t *p = g.lvl_ptr_h.data() + g.lvl_off_h[m];
        for (int L = 0; L < g.nlev_h[m]; ++L) p[L] = hstarts[(size_t)m * (Lcap + 1) + L];
        p[g.nlev_h[m]] = nc;
    }
    g.lvl_ptr_d.alloc(8 * g.lvl_ptr_h.size());
    g.lvl_off_d.alloc(8 * g.lvl_off_h.size());
    JSW_HIP(hipMemcpyAsync(g.lvl_ptr_d.p, g.lvl_ptr_h.data(), 8 * g.lvl_ptr_h.size(), hipMemcpyHostToDevice, s));
    JSW_HIP(hipMemcpyAsync(g.lvl_off_d.p, g.lvl_off_h.data(), 8 * g.lvl_off_h.size(), hipMemcpyHostToDevice, s));
    // sweep work list: chunks of <= 64 cells of one (level, direction).
    // Directions are dealt to kStreams streams in contiguous blocks (with
    // octant-major quadratures a block is an octant).  Within a stream the
    // (direction, level) groups of chunks follow the PACED priority: level
    // divided by the direction's level count, then level, then direction.
    // The key grows along every edge of a direction, so the order is
    // topological for every direction of the stream at once, and the
    // deepest direction is spread over the whole stream instead of running
    // alone at its end (as in level-then-direction order).
    g.dir_stream_h.resize(g.nd);
    for (int m = 0; m < g.nd; ++m) g.dir_stream_h[m] = (int32_t)(((int64_t)m * kStreams) / g.nd);
    std::vector<Chunk> ch;
    ch.reserve((size_t)(N / 64 + (int64_t)g.nd * g.max_levels));
    g.stream_off_h.assign(kStreams + 1, 0);
    g.lvl_chunk_h.assign(g.lvl_ptr_h.size(), 0);
    g.max_w = g.max_w2 = 0;
    struct Group {
        int64_t key;
        int32_t L, m;
    };
    std::vector<Group> grp;
    for (int sidx = 0; sidx < kStreams; ++sidx) {
        g.stream_off_h[sidx] = (int64_t)ch.size();
        grp.clear();
        for (int m = 0; m < g.nd; ++m)
            if (g.dir_stream_h[m] == sidx)
                for (int L = 0; L < g.nlev_h[m]; ++L) grp.push_back(Group{((int64_t)L << 32) / g.nlev_h[m], L, m});
        std::sort(grp.begin(), grp.end(), [](const Group &x, const Group &y) {
            if (x.key != y.key) return x.key < y.key;
            return x.L != y.L ? x.L < y.L : x.m < y.m;
        });
        for (const Group &gr : grp) {
            const int L = gr.L, m = gr.m;
            const int64_t *p = g.lvl_ptr_h.data() + g.lvl_off_h[m];
            g.lvl_chunk_h[g.lvl_off_h[m] + L] = (int32_t)ch.size();
            g.max_w = std::max(g.max_w, p[L + 1] - p[L]);
            g.max_w2 = std::max(g.max_w2, p[L + 1] - (L > 0 ? p[L - 1] : p[L]));
            for (int64_t o = p[L]; o < p[L + 1]; o += 64) {
                int64_t c = std::min<int64_t>(64, p[L + 1] - o);
                ch.push_back(Chunk{(uint32_t)m | ((uint32_t)(c - 1) << 16), (uint32_t)o});
            }
        }
    }
    g.priority = JSWEEP_PRIORITY_PACED;
    g.stream_off_h[kStreams] = (int64_t)ch.size();
    g.n_chunks = (int64_t)ch.size();
    if (g.n_chunks >= ((int64_t)1 << 31)) fail(JSWEEP_E_INVALID_ARG, "too many sweep chunks");
    g.lvl_chunk_d.alloc(4 * g.lvl_chunk_h.size());
    JSW_HIP(hipMemcpyAsync(g.lvl_chunk_d.p, g.lvl_chunk_h.data(), 4 * g.lvl_chunk_h.size(), hipMemcpyHostToDevice, s));
    g.chunks.alloc(sizeof(Chunk) * std::max<int64_t>(1, g.n_chunks));
    JSW_HIP(hipMemcpyAsync(g.chunks.p, ch.data(), sizeof(Chunk) * g.n_chunks, hipMemcpyHostToDevice, s));
    g.stream_off.alloc(8 * (kStreams + 1));
    JSW_HIP(hipMemcpyAsync(g.stream_off.p, g.stream_off_h.data(), 8 * (kStreams + 1), hipMemcpyHostToDevice, s));
    build_coarsened<NF, DIM>(g, lag, s);
    build_program<NF, DIM>(g, lag, s);
    build_compact(g, s);
    build_packed(g, s);
    // the work-list sweep's two level-position flux arrays (FP64 size) and
    // the sigma_t cache are allocated here, so that single-group sweeps
    // allocate nothing
    for (int i = 0; i < 2; ++i) g.dd_pos[i].alloc(8 * (size_t)std::max<int64_t>(1, N));
    g.sig_last.alloc(8 * g.nc + 64);
    g.den64_ok = g.den32_ok = false;
    g.dd_state[0] = g.dd_state[1] = 0;
    g.status.alloc(128 + 32 * 4 * 8);   // status words, then 8 ticket counters 128 B apart
    JSW_HIP(hipMemsetAsync(g.status.p, 0, g.status.bytes, s));
    JSW_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// Priority strategies (paper Sec. V-D): the order of the chunks of every
// stream, i.e. which ready cluster a wavefront takes next.  The paper ranks
// a (patch, angle) pair by prior(a) * C + prior(p) with a large C (angle
// first) and names three vertex / patch priorities: BFS, LDCP (longest
// distance on the critical path) and SLBD (shortest local boundary
// distance, a depth-first variant).  On the coarsened graph (chunks,
// Sec. V-E; acyclic by Theorem 1) the order is produced the way a priority
// ready queue releases work: Kahn's algorithm per stream, always taking the
// ready chunk of smallest key, so every order is topological and the sweep
// keeps its guarantee that a chunk's upwind chunks come earlier in its
// stream.  Keys (ties broken by the level order):
//   BFS   level, direction, position (the level order itself);
//   LDCP  the longest chunk path from the chunk to a sink, longest first;
//   SLBD  the same distance, shortest first (the chunk closest to the
//         outflow boundary of its direction: depth first);
//   PACED the level divided by the direction's level count: every
//         direction of a stream takes the whole stream to reach its last
//         level, the deepest ones in proportionally more, shorter steps,
//         instead of all starting together (BFS: the deepest direction of
//         the stream ends alone) or the deepest first (LDCP: it starts
//         alone);
//   ANGLE_MAJOR (OR-ed) the chunk's direction first, ascending;
//   ANGLE_WEIGHT(k) (OR-ed, k = 1..7) the paper's combined rank
//         prior(a) * C + prior(p) with a finite C: prior(a) is the
//         direction's rank in its stream, prior(p) the strategy's key (the
//         level for BFS) and C the stream's largest level count divided by
//         k, rounded up.  Direction r then starts about r / k of a sweep
//         after the stream's first one, so about k directions of a stream
//         are under way at any time, each in another phase of its sweep
//         (C = 0 is BFS across the directions, an unbounded C ANGLE_MAJOR).
//         Fewer directions at once means fewer sweep fronts, whose cells'
//         V s gathers then stay in the XCD's L2.
// Any topological order gives bit-identical fluxes (each flux is a pure
// function of its upwind fluxes); only the schedule changes.
// ---------------------------------------------------------------------------
static std::vector<int64_t> priority_order(const std::vector<Chunk> &ch, const std::vector<int32_t> &dptr,
                                           const std::vector<int32_t> &dep, const std::vector<int64_t> &stream_off,
                                           const std::vector<int32_t> &lev_of, const std::vector<int32_t> &dir_stream,
                                           const std::vector<int32_t> &nlev, int priority) {
    const int64_t n = (int64_t)ch.size();
    const int base = priority & 0xf;
    const bool angle = (priority & JSWEEP_PRIORITY_ANGLE_MAJOR) != 0;
    const int weight_k = JSWEEP_PRIORITY_ANGLE_WEIGHT_OF(priority);
    // per direction: rank within its stream; per stream: C
    const int nd = (int)dir_stream.size();
    std::vector<int64_t> rank(nd, 0), cw(kStreams, 0);
    {
        std::vector<int64_t> seen(kStreams, 0), maxlev(kStreams, 0);
        for (int m = 0; m < nd; ++m) {
            const int sidx = dir_stream[m];
            rank[m] = seen[sidx]++;
            maxlev[sidx] = std::max<int64_t>(maxlev[sidx], nlev[m]);
        }
        if (weight_k > 0)
            for (int sidx = 0; sidx < kStreams; ++sidx) cw[sidx] = (maxlev[sidx] + weight_k - 1) / weight_k;
    }
    // longest path (in chunks) to a sink: chunks are in a topological order,
    // so one reverse pass settles every chunk before its upwind chunks
    std::vector<int32_t> bl(n, 0);
    if (base == JSWEEP_PRIORITY_LDCP || base == JSWEEP_PRIORITY_SLBD)
        for (int64_t c = n - 1; c >= 0; --c)
            for (int32_t k = dptr[c]; k < dptr[c + 1]; ++k) bl[dep[k]] = std::max(bl[dep[k]], bl[c] + 1);
    // downstream lists and counts of upwind chunks
    std::vector<int32_t> cnt(n), uptr(n + 1, 0), down((size_t)dptr[n]);
    for (int64_t c = 0; c < n; ++c) {
        cnt[c] = dptr[c + 1] - dptr[c];
        for (int32_t k = dptr[c]; k < dptr[c + 1]; ++k) ++uptr[dep[k] + 1];
    }
    for (int64_t c = 0; c < n; ++c) uptr[c + 1] += uptr[c];
    {
        std::vector<int32_t> fill(uptr.begin(), uptr.end() - 1);
        for (int64_t c = 0; c < n; ++c)
            for (int32_t k = dptr[c]; k < dptr[c + 1]; ++k) down[fill[dep[k]]++] = (int32_t)c;
    }
    struct Key {
        int64_t a, b, c;
        bool operator>(const Key &o) const { return a != o.a ? a > o.a : b != o.b ? b > o.b : c > o.c; }
    };
    auto key = [&](int64_t c) {
        const int dm = (int)(ch[c].a & 0xffffu);
        const int64_t m = angle ? (int64_t)dm : 0;
        int64_t k = base == JSWEEP_PRIORITY_LDCP ? -(int64_t)bl[c] : base == JSWEEP_PRIORITY_SLBD ? bl[c] : 0;
        if (base == JSWEEP_PRIORITY_PACED) k = ((int64_t)lev_of[c] << 32) / std::max(1, nlev[dm]);
        if (weight_k > 0) {
            // finite angle weight: BFS ranks by level, the others by their
            // key (PACED's in level units)
            if (base == JSWEEP_PRIORITY_BFS) k = lev_of[c];
            if (base == JSWEEP_PRIORITY_PACED) k = (k * cw[dir_stream[dm]] * weight_k) >> 32;
            k += rank[dm] * cw[dir_stream[dm]];
        }
        return Key{m, k, c};
    };
    std::vector<int64_t> order;
    order.reserve(n);
    for (int sidx = 0; sidx < kStreams; ++sidx) {
        std::priority_queue<Key, std::vector<Key>, std::greater<Key>> ready;
        for (int64_t c = stream_off[sidx]; c < stream_off[sidx + 1]; ++c)
            if (cnt[c] == 0) ready.push(key(c));
        while (!ready.empty()) {
            const int64_t c = ready.top().c;
            ready.pop();
            order.push_back(c);
            for (int32_t k = uptr[c]; k < uptr[c + 1]; ++k)
                if (--cnt[down[k]] == 0) ready.push(key(down[k]));
        }
        if ((int64_t)order.size() != stream_off[sidx + 1])
            fail(JSWEEP_E_DEVICE, "coarsened graph of a stream is not acyclic");
    }
    return order;
}

template <int NF, int DIM>
static void reorder_impl(Graph &g, int priority, hipStream_t s) {
    const int64_t nch = g.n_chunks;
    std::vector<Chunk> ch(nch);
    std::vector<int32_t> dptr(nch + 1), dep((size_t)std::max<int64_t>(1, g.n_dep));
    JSW_HIP(hipMemcpyAsync(ch.data(), g.chunks.p, sizeof(Chunk) * nch, hipMemcpyDeviceToHost, s));
    JSW_HIP(hipMemcpyAsync(dptr.data(), g.dep_ptr.p, 4 * (nch + 1), hipMemcpyDeviceToHost, s));
    if (g.n_dep) JSW_HIP(hipMemcpyAsync(dep.data(), g.dep.p, 4 * (size_t)g.n_dep, hipMemcpyDeviceToHost, s));
    JSW_HIP(hipStreamSynchronize(s));
    // the level order first (every other order is computed from it, so the
    // result does not depend on the order the graph had before)
    std::vector<int64_t> back(nch);
    // level of a chunk (all of its vertices share it)
    std::vector<int32_t> lev_of(nch);
    {
        std::vector<int64_t> lv(nch);
        for (int64_t c = 0; c < nch; ++c) lv[c] = c;
        for (int64_t c = 0; c < nch; ++c) {
            const int m = (int)(ch[c].a & 0xffffu);
            const int64_t *p = g.lvl_ptr_h.data() + g.lvl_off_h[m];
            lev_of[c] = (int32_t)(std::upper_bound(p, p + g.nlev_h[m] + 1, (int64_t)ch[c].b) - p - 1);
        }
        std::stable_sort(lv.begin(), lv.end(), [&](int64_t x, int64_t y) {
            const int sx = g.dir_stream_h[ch[x].a & 0xffffu], sy = g.dir_stream_h[ch[y].a & 0xffffu];
            if (sx != sy) return sx < sy;
            if (lev_of[x] != lev_of[y]) return lev_of[x] < lev_of[y];
            const uint32_t mx = ch[x].a & 0xffffu, my = ch[y].a & 0xffffu;
            if (mx != my) return mx < my;
            return ch[x].b < ch[y].b;
        });
        back = lv;
    }
    bool identity = true;
    for (int64_t c = 0; c < nch && identity; ++c) identity = back[c] == c;
    if (!identity) {
        // deps in level-order indices
        std::vector<int64_t> inv(nch);
        for (int64_t c = 0; c < nch; ++c) inv[back[c]] = c;
        std::vector<Chunk> lch(nch);
        std::vector<int32_t> lptr(nch + 1, 0), ldep(dep.size());
        for (int64_t c = 0; c < nch; ++c) {
            const int64_t o = back[c];
            lch[c] = ch[o];
            lptr[c + 1] = lptr[c] + (dptr[o + 1] - dptr[o]);
            for (int32_t k = dptr[o], j = lptr[c]; k < dptr[o + 1]; ++k, ++j) ldep[j] = (int32_t)inv[dep[k]];
        }
        std::vector<int32_t> llev(nch);
        for (int64_t c = 0; c < nch; ++c) llev[c] = lev_of[back[c]];
        ch.swap(lch);
        dptr.swap(lptr);
        dep.swap(ldep);
        lev_of.swap(llev);
    }
    const std::vector<int64_t> order =
        priority_order(ch, dptr, dep, g.stream_off_h, lev_of, g.dir_stream_h, g.nlev_h, priority);
    std::vector<Chunk> out(nch);
    for (int64_t c = 0; c < nch; ++c) out[c] = ch[order[c]];
    // first chunk (in the new order) of every (direction, level)
    std::fill(g.lvl_chunk_h.begin(), g.lvl_chunk_h.end(), INT32_MAX);
    for (int64_t c = 0; c < nch; ++c) {
        const int m = (int)(out[c].a & 0xffffu);
        const int64_t *p = g.lvl_ptr_h.data() + g.lvl_off_h[m];
        const int L = (int)(std::upper_bound(p, p + g.nlev_h[m] + 1, (int64_t)out[c].b) - p - 1);
        int32_t &f = g.lvl_chunk_h[g.lvl_off_h[m] + L];
        f = std::min(f, (int32_t)c);
    }
    for (auto &f : g.lvl_chunk_h)
        if (f == INT32_MAX) f = 0;
    JSW_HIP(hipMemcpyAsync(g.lvl_chunk_d.p, g.lvl_chunk_h.data(), 4 * g.lvl_chunk_h.size(), hipMemcpyHostToDevice, s));
    JSW_HIP(hipMemcpyAsync(g.chunks.p, out.data(), sizeof(Chunk) * nch, hipMemcpyHostToDevice, s));
    JSW_HIP(hipStreamSynchronize(s));   // before the host vectors go
    const LagView lag{g.n_lag ? g.lag_mv.as<uint64_t>() : nullptr, g.n_lag ? g.lag_u.as<int32_t>() : nullptr, g.n_lag};
    build_coarsened<NF, DIM>(g, lag, s);
    build_program<NF, DIM>(g, lag, s);
    build_compact(g, s);
    build_packed(g, s);
    // everything kept in chunk order is rebuilt on its next use
    g.pa32.release();
    g.pden32.release();
    g.pvol64.release();
    g.pvol32.release();
    g.den64_ok = g.den32_ok = false;
    g.dd_state[0] = g.dd_state[1] = 0;
    g.priority = priority;
    ++g.prog_version;
    JSW_HIP(hipStreamSynchronize(s));
}

void set_priority(Graph &g, int priority, hipStream_t s) {
    const int base = priority & 0xf;
    if ((priority & ~(0xf | JSWEEP_PRIORITY_ANGLE_MAJOR | JSWEEP_PRIORITY_ANGLE_WEIGHT(7))) ||
        base < JSWEEP_PRIORITY_BFS || base > JSWEEP_PRIORITY_PACED)
        fail(JSWEEP_E_INVALID_ARG, "unknown work-list priority");
    if ((priority & JSWEEP_PRIORITY_ANGLE_MAJOR) && JSWEEP_PRIORITY_ANGLE_WEIGHT_OF(priority))
        fail(JSWEEP_E_INVALID_ARG, "ANGLE_MAJOR and a finite angle weight exclude each other");
    if (priority == g.priority || !g.n_chunks) {
        g.priority = priority;
        return;
    }
    if (g.ctype == JSWEEP_TRI) reorder_impl<3, 2>(g, priority, s);
    else if (g.ctype == JSWEEP_TET) reorder_impl<4, 3>(g, priority, s);
    else reorder_impl<6, 3>(g, priority, s);
}

void build_dag(Graph &g, bool lag_cycles, hipStream_t s) {
    if ((int64_t)g.nc * g.nd >= (int64_t)1 << 32) fail(JSWEEP_E_INVALID_ARG, "n_cells * n_dirs must be below 2^32");
    if (g.ctype == JSWEEP_TRI) dag_impl<3, 2>(g, lag_cycles, s);
    else if (g.ctype == JSWEEP_TET) dag_impl<4, 3>(g, lag_cycles, s);
    else dag_impl<6, 3>(g, lag_cycles, s);
}

}  // namespace jsw
