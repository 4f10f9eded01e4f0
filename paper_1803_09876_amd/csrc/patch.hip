// Patch-task sweep: the patch-program form of the sweep (Sec. V-A: the mesh
// cut into patches along a Morton space-filling curve, one program per
// (patch, direction); Sec. V-B: patch-angle parallelism, all directions'
// programs in flight at once).
//
// A task is one visit of one patch in one direction: the paper's patch
// program is re-entrant (a patch whose cells wait on another patch that in
// turn waits on it is computed in several goes), and the visits are fixed
// here ahead of the sweep by running the direction's graph sequentially on
// the host: the patch holding the lowest-level ready cell runs next, as far
// as it can go (every cell of it that becomes ready is taken along, in level
// order, until the kernel's rounds or halo budget is reached).  Cells
// of one visit form a task; visits in that order are a topological order of
// the task graph, so it is acyclic.  A task's vertices run on one wavefront,
// level by level (rounds of at most 64 vertices), with the fluxes of the task
// and of its halo (upwind vertices of other tasks, lagged values) held in
// LDS.
//
// Tasks run out of one ready queue per stream (XCD; a direction's tasks all
// belong to one stream): every task has a count of its upstream tasks, reset
// before each sweep; the tasks without any (the first of each stream, whose
// tasks are numbered by depth in the task graph) start in the queue, and a
// finishing task decrements the counts of its downstream tasks and appends
// those it completes.  A wavefront only ever takes a task whose inputs are
// final, so none waits while holding one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <functional>
#include <queue>
#include <cstdlib>
#include <thread>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/device/device_select.hpp>

#include "common.hpp"

namespace jsw {

namespace {

constexpr int kB = 256;

unsigned blocks_for(int64_t n) { return (unsigned)std::max<int64_t>(1, ceil_div(n, kB)); }

template <int NF, int DIM>
__device__ inline double pdot(const CellRec<double, NF, DIM> &r, int j, const double *om) {
    double d = om[0] * r.S[j][0] + om[1] * r.S[j][1];
    if constexpr (DIM == 3) d = d + om[2] * r.S[j][2];
    return d;
}

// Offset of this lane's c items in an array shared by all lanes of the
// grid: one atomic per wavefront.  Every lane of the wavefront must call it.
__device__ inline unsigned long long wave_reserve(unsigned long long *ctr, int c) {
    const int lane = threadIdx.x & 63;
    int x = c;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    unsigned long long base = 0;
    if (lane == 63 && x > 0) base = atomicAdd(ctr, (unsigned long long)x);
    base = __shfl(base, 63, 64);
    return base + (unsigned long long)(x - c);
}

// upwind cells of every vertex through non-lagged inflow faces (ns
// slots, -1 past the last), for the host's visit order
template <int NF, int DIM>
__global__ void k_pp_upwind(const CellRec<double, NF, DIM> *rec, const double *omega, int64_t nc, int64_t N, int ns,
                            const uint64_t *lag_mv, const int32_t *lag_u, int64_t n_lag, int32_t *up) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t m = i / nc, v = i - m * nc;
    const CellRec<double, NF, DIM> r = rec[v];
    const double om[3] = {omega[3 * m], omega[3 * m + 1], omega[3 * m + 2]};
    int k = 0;
    for (int j = 0; j < NF; ++j) {
        if (!(pdot(r, j, om) < 0.0)) continue;
        const int32_t nb = r.nbr[j];
        if (nb == -1) continue;
        const int64_t u = nb <= -2 ? (int64_t)(-nb - 2) : (int64_t)nb;
        if (nb <= -2 && lag_index(lag_mv, lag_u, n_lag, (int)m, v, u) >= 0) continue;
        if (k < ns) up[i * ns + k++] = (int32_t)u;
    }
    for (; k < ns; ++k) up[i * ns + k] = -1;
}

// task id of every vertex, by binary search in the sorted task keys
__global__ void k_pp_tid(const uint32_t *tkey, int64_t nc, int64_t N, const uint64_t *keys, int64_t n,
                         const int32_t *tid_of, const int32_t *posi, uint64_t *sort_key, int32_t *sort_val) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t m = i / nc;
    const uint64_t key = (uint64_t)m << 32 | tkey[i];
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    const int64_t t = tid_of[lo];
    // positions: by task, then by level position (level, then id)
    sort_key[i] = (uint64_t)m << 54 | (uint64_t)t << 27 | (uint64_t)posi[i];
    sort_val[i] = (int32_t)(i - m * nc);
}

// from the sorted position keys: the task at every position, the position
// of every vertex, task bounds and round starts
__global__ void k_pp_positions(const uint64_t *skey, const int32_t *cell, const int32_t *level, int64_t nc, int64_t N,
                               int32_t *ptid, int32_t *ppos, int32_t *tstart, int32_t *tend, int32_t *tdir,
                               int64_t *step_mark) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t m = i / nc, q = i - m * nc;
    const int32_t t = (int32_t)((skey[i] >> 27) & ((1ull << 27) - 1));
    ptid[i] = t;
    ppos[m * nc + cell[i]] = (int32_t)q;
    const bool first = q == 0 || (int32_t)((skey[i - 1] >> 27) & ((1ull << 27) - 1)) != t;
    const bool last = q == nc - 1 || (int32_t)((skey[i + 1] >> 27) & ((1ull << 27) - 1)) != t;
    if (first) { tstart[t] = (int32_t)q; tdir[t] = (int32_t)m; }
    if (last) tend[t] = (int32_t)(q + 1);
    const int32_t lv = level[m * nc + cell[i]];
    const bool step = first || level[m * nc + cell[i - 1]] != lv;
    step_mark[i] = step ? i : 0;
}

__global__ void k_pp_round_mark(const int64_t *step_start, int64_t N, int32_t *mark) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    mark[i] = ((i - step_start[i]) & 63) == 0 ? 1 : 0;
}

// round table (offset in the task | (count - 1) << 16) and the tasks' round
// ranges; ridx is the inclusive count of round starts
__global__ void k_pp_rounds(const int32_t *mark, const int32_t *ridx, const int32_t *ptid, const int32_t *tstart,
                            const int32_t *tend, int64_t nc, int64_t N, int32_t *rstart_abs, int32_t *round0,
                            int32_t *nround) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t m = i / nc, q = i - m * nc;
    const int32_t t = ptid[i];
    if (mark[i]) rstart_abs[ridx[i] - 1] = (int32_t)i;
    if (q == tstart[t]) round0[t] = ridx[i] - 1;
    if (q == tend[t] - 1) nround[t] = ridx[i];   // turned into a count below
}

__global__ void k_pp_round_table(const int32_t *rstart_abs, int64_t n_rounds, int64_t N, int64_t nc,
                                 const int32_t *ptid, const int32_t *tstart, const int32_t *tend, int32_t *round) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rounds) return;
    const int64_t i = rstart_abs[r];
    const int64_t m = i / nc, q = i - m * nc;
    const int32_t t = ptid[i];
    const int64_t end = std::min<int64_t>(r + 1 < n_rounds ? (int64_t)rstart_abs[r + 1] : N, m * nc + tend[t]);
    round[r] = (int32_t)(q - tstart[t]) | (int32_t)(end - i - 1) << 16;
}

// halo keys: task << 32 | upwind position (or 0x80000000 | lagged edge)
template <int NF, int DIM, bool WRITE>
__global__ void k_pp_halo(const CellRec<double, NF, DIM> *rec, const double *omega, int64_t nc, int64_t N,
                          const uint64_t *lag_mv, const int32_t *lag_u, int64_t n_lag, const int32_t *cell,
                          const int32_t *ptid, const int32_t *ppos, unsigned long long *ctr, uint64_t *out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < N;
    uint64_t e[NF];
    int c = 0;
    if (valid) {
        const int64_t m = i / nc, v = cell[i];
        const CellRec<double, NF, DIM> r = rec[v];
        const double om[3] = {omega[3 * m], omega[3 * m + 1], omega[3 * m + 2]};
        const uint64_t t = (uint64_t)(uint32_t)ptid[i];
        for (int j = 0; j < NF; ++j) {
            if (!(pdot(r, j, om) < 0.0)) continue;
            const int32_t nb = r.nbr[j];
            if (nb == -1) continue;
            const int64_t u = nb <= -2 ? (int64_t)(-nb - 2) : (int64_t)nb;
            const int64_t l = nb <= -2 ? lag_index(lag_mv, lag_u, n_lag, (int)m, v, u) : -1;
            if (l >= 0) {
                e[c++] = t << 32 | (0x80000000ull | (uint64_t)l);
            } else {
                const int32_t qu = ppos[m * nc + u];
                if (ptid[m * nc + qu] != (int32_t)t) e[c++] = t << 32 | (uint64_t)(uint32_t)qu;
            }
        }
    }
    const unsigned long long at = wave_reserve(ctr, c);
    if (WRITE)
        for (int k = 0; k < c; ++k) out[at + k] = e[k];
}

// per-task ranges of a list sorted by task (the task in the upper 32 bits)
__global__ void k_pp_ranges(const uint64_t *keys, int64_t n, int32_t *start, int32_t *count) {
    const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= n) return;
    const uint32_t t = (uint32_t)(keys[h] >> 32);
    if (h == 0 || (uint32_t)(keys[h - 1] >> 32) != t) start[t] = (int32_t)h;
    if (h == n - 1 || (uint32_t)(keys[h + 1] >> 32) != t) count[t] = (int32_t)(h + 1);   // end, made a count later
}

// halo entries as stored (position >= 0, lagged edge -(h + 1)) and the
// dependency keys task << 32 | upstream task (no dependency for lagged ones)
__global__ void k_pp_halo_out(const uint64_t *hk, int64_t n, const int32_t *tdir, const int32_t *ptid, int64_t nc,
                              int32_t *halo, uint64_t *dkey) {
    const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= n) return;
    const uint64_t k = hk[h];
    const uint32_t t = (uint32_t)(k >> 32), lo = (uint32_t)k;
    if (lo & 0x80000000u) {
        halo[h] = -(int32_t)(lo & 0x7fffffffu) - 1;
        dkey[h] = ~0ull;
    } else {
        halo[h] = (int32_t)lo;
        dkey[h] = (uint64_t)t << 32 | (uint32_t)ptid[(int64_t)tdir[t] * nc + lo];
    }
}

__global__ void k_pp_dep_out(const uint64_t *dk, int64_t n, int32_t *dep) {
    const int64_t h = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (h < n) dep[h] = (int32_t)(uint32_t)dk[h];
}

__device__ inline int64_t find_key(const uint64_t *k, int64_t lo, int64_t hi, uint64_t key) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (k[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// program codes and coefficients, inflow faces in local face order (the
// classification of the graph: FP64 Omega . S < 0)
template <int NF, int DIM>
__global__ void k_pp_code(const CellRec<double, NF, DIM> *rec, const double *omega, int64_t nc, int64_t N, int ns,
                          const uint64_t *lag_mv, const int32_t *lag_u, int64_t n_lag, const int32_t *cell,
                          const int32_t *ptid, const int32_t *ppos, const int32_t *tstart, const int32_t *tend,
                          const uint64_t *hk, const int32_t *hstart, const int32_t *hend, int32_t *code, double *a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t m = i / nc, v = cell[i];
    const CellRec<double, NF, DIM> r = rec[v];
    const double om[3] = {omega[3 * m], omega[3 * m + 1], omega[3 * m + 2]};
    const int32_t t = ptid[i];
    const int32_t q0 = tstart[t], n = tend[t] - q0;
    const int64_t h0 = hstart[t], h1 = hend[t];
    int k = 0;
    for (int j = 0; j < NF; ++j) {
        const double d = pdot(r, j, om);
        if (!(d < 0.0)) continue;
        const int32_t nb = r.nbr[j];
        int32_t cd = -1;
        if (nb != -1) {
            const int64_t u = nb <= -2 ? (int64_t)(-nb - 2) : (int64_t)nb;
            const int64_t l = nb <= -2 ? lag_index(lag_mv, lag_u, n_lag, (int)m, v, u) : -1;
            const uint64_t tt = (uint64_t)(uint32_t)t << 32;
            if (l >= 0) {
                cd = n + (int32_t)(find_key(hk, h0, h1, tt | (0x80000000ull | (uint64_t)l)) - h0);
            } else {
                const int32_t qu = ppos[m * nc + u];
                if (ptid[m * nc + qu] == t) cd = qu - q0;
                else cd = n + (int32_t)(find_key(hk, h0, h1, tt | (uint64_t)(uint32_t)qu) - h0);
            }
        }
        code[(int64_t)k * N + i] = cd;
        a[(int64_t)k * N + i] = -d;
        ++k;
    }
    for (; k < ns; ++k) {
        code[(int64_t)k * N + i] = kNoFace;
        a[(int64_t)k * N + i] = 0.0;
    }
}

__global__ void k_pp_desc(int64_t n_tasks, const int32_t *tstart, const int32_t *tend, const int32_t *tdir,
                          const int32_t *round0, const int32_t *nround, const int32_t *hstart, const int32_t *hend,
                          const int32_t *dstart, const int32_t *dend, int32_t *desc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tasks) return;
    int32_t *d = desc + t * kPatchDesc;
    d[0] = tstart[t];
    d[1] = tdir[t];
    d[2] = tend[t] - tstart[t];
    d[3] = nround[t] - round0[t];
    d[4] = round0[t];
    d[5] = hend[t] - hstart[t];
    d[6] = hstart[t];
    d[7] = dend[t] - dstart[t];
    d[8] = dstart[t];
    for (int k = 9; k < kPatchDesc; ++k) d[k] = 0;
}

// denominators in position order: sigma_t V + outflow a_f in local face
// order, as in the other sweep programs
template <int NF, int DIM>
__global__ void k_pp_den(const CellRec<double, NF, DIM> *rec, const double *omega, const int32_t *cell, int64_t nc,
                         int64_t N, double *den) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int64_t m = i / nc;
    const CellRec<double, NF, DIM> r = rec[cell[i]];
    const double om[3] = {omega[3 * m], omega[3 * m + 1], omega[3 * m + 2]};
    double dn = r.sigV;
    for (int j = 0; j < NF; ++j) {
        const double d = pdot(r, j, om);
        if (d > 0.0) dn = dn + d;
    }
    den[i] = dn;
}

__global__ void k_pp_vs(const double *vol, const double *src, int64_t nc, double *vs) {
    const int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (K < nc) vs[K] = src ? vol[K] * src[K] : vol[K] * 0.0;
}


// sort keys (optionally with values) in place through a scratch copy
template <class K, class V>
void sort_pairs(DevBuf &keys, DevBuf *vals, int64_t n, int end_bit, hipStream_t s) {
    if (n <= 0) return;
    DevBuf k2(sizeof(K) * n), v2(vals ? sizeof(V) * n : 1);
    size_t bytes = 0;
    if (vals) {
        JSW_HIP(rocprim::radix_sort_pairs(nullptr, bytes, keys.as<K>(), k2.as<K>(), vals->as<V>(), v2.as<V>(), (size_t)n,
                                          0u, (unsigned)end_bit, s));
        DevBuf tmp(bytes + 16);
        JSW_HIP(rocprim::radix_sort_pairs(tmp.p, bytes, keys.as<K>(), k2.as<K>(), vals->as<V>(), v2.as<V>(), (size_t)n,
                                          0u, (unsigned)end_bit, s));
        JSW_HIP(hipStreamSynchronize(s));
        *vals = std::move(v2);
    } else {
        JSW_HIP(rocprim::radix_sort_keys(nullptr, bytes, keys.as<K>(), k2.as<K>(), (size_t)n, 0u, (unsigned)end_bit, s));
        DevBuf tmp(bytes + 16);
        JSW_HIP(rocprim::radix_sort_keys(tmp.p, bytes, keys.as<K>(), k2.as<K>(), (size_t)n, 0u, (unsigned)end_bit, s));
        JSW_HIP(hipStreamSynchronize(s));
    }
    keys = std::move(k2);
}

// distinct keys of a sorted list, in place; returns their number
int64_t unique_sorted(DevBuf &keys, int64_t n, hipStream_t s) {
    if (n <= 0) return 0;
    DevBuf out(8 * n), cnt(8);
    size_t bytes = 0;
    JSW_HIP(rocprim::unique(nullptr, bytes, keys.as<uint64_t>(), out.as<uint64_t>(), cnt.as<unsigned long long>(),
                            (size_t)n, rocprim::equal_to<uint64_t>(), s));
    DevBuf tmp(bytes + 16);
    JSW_HIP(rocprim::unique(tmp.p, bytes, keys.as<uint64_t>(), out.as<uint64_t>(), cnt.as<unsigned long long>(),
                            (size_t)n, rocprim::equal_to<uint64_t>(), s));
    unsigned long long u = 0;
    JSW_HIP(hipMemcpyAsync(&u, cnt.p, 8, hipMemcpyDeviceToHost, s));
    JSW_HIP(hipStreamSynchronize(s));
    keys = std::move(out);
    return (int64_t)u;
}

template <class T>
std::vector<T> to_host(const DevBuf &b, int64_t n, hipStream_t s) {
    std::vector<T> h(std::max<int64_t>(0, n));
    if (n > 0) JSW_HIP(hipMemcpyAsync(h.data(), b.p, sizeof(T) * n, hipMemcpyDeviceToHost, s));
    JSW_HIP(hipStreamSynchronize(s));
    return h;
}

// cells per patch: Morton runs of whole lattice blocks where the mesh is a
// lattice (4 x 8 x 8 hexahedra, 32 cubes of 6 tetrahedra)
int patch_cells(int ctype) { return ctype == JSWEEP_HEX ? 256 : ctype == JSWEEP_TET ? 192 : 128; }

// Visits of one direction's patches (see the top of the file): up[v * ns +
// k] are v's upwind cells (-1 past the last), lev the levels, patch the
// patches.  Out: the visit of every cell and each visit's depth in the task
// graph (1 + the deepest upstream visit).
void visits(int64_t nc, int ns, const int32_t *up, const int32_t *lev, const int32_t *patch, int32_t npatch,
            uint32_t *visit, std::vector<int32_t> &depth) {
    std::vector<int32_t> indeg(nc, 0), dptr(nc + 1, 0), dn;
    for (int64_t v = 0; v < nc; ++v)
        for (int k = 0; k < ns; ++k) {
            const int32_t u = up[v * ns + k];
            if (u < 0) break;
            ++indeg[v];
            ++dptr[u + 1];
        }
    for (int64_t v = 0; v < nc; ++v) dptr[v + 1] += dptr[v];
    dn.resize(dptr[nc]);
    {
        std::vector<int32_t> fill(dptr.begin(), dptr.end() - 1);
        for (int64_t v = 0; v < nc; ++v)
            for (int k = 0; k < ns; ++k) {
                const int32_t u = up[v * ns + k];
                if (u < 0) break;
                dn[fill[u]++] = (int32_t)v;
            }
    }
    // ready cells per patch (linked lists) and their lowest level; the
    // patches with ready cells in a heap keyed by (lowest ready level,
    // patch), entries made stale by a later change are skipped when popped
    std::vector<int32_t> head(npatch, -1), nxt(nc, -1), cnt(npatch, 0), minlev(npatch, INT32_MAX);
    std::priority_queue<std::pair<int32_t, int32_t>, std::vector<std::pair<int32_t, int32_t>>, std::greater<>> ph;
    auto push = [&](int32_t w) {
        const int32_t p = patch[w];
        nxt[w] = head[p];
        head[p] = w;
        ++cnt[p];
        if (lev[w] < minlev[p]) {
            minlev[p] = lev[w];
            ph.push({minlev[p], p});
        }
    };
    for (int64_t v = 0; v < nc; ++v)
        if (indeg[v] == 0) push((int32_t)v);
    // a visit takes its ready cells in level order and stops before it
    // would exceed the kernel's rounds or halo budget (halo counted as
    // upwind references from outside the visit; lagged edges, which are not
    // in up, get the last quarter of the budget)
    std::priority_queue<std::pair<int32_t, int32_t>, std::vector<std::pair<int32_t, int32_t>>, std::greater<>> pq;
    std::fill(visit, visit + nc, UINT32_MAX);
    int64_t done = 0;
    uint32_t nv = 0;
    while (done < nc) {
        while (cnt[ph.top().second] == 0 || minlev[ph.top().second] != ph.top().first) ph.pop();
        const int32_t best = ph.top().second;
        ph.pop();
        const uint32_t t = nv++;
        for (int32_t v = head[best]; v >= 0; v = nxt[v]) pq.push({lev[v], v});
        head[best] = -1;
        cnt[best] = 0;
        minlev[best] = INT32_MAX;
        int rounds = 0, cur_lev = -1, cur_cnt = 0, ext = 0;
        while (!pq.empty()) {
            const int32_t l = pq.top().first, v = pq.top().second;
            const int add = (l != cur_lev || cur_cnt % 64 == 0) ? 1 : 0;
            int ev = 0;
            for (int k = 0; k < ns; ++k) {
                const int32_t u = up[v * ns + k];
                if (u < 0) break;
                ev += visit[u] != t;
            }
            if (rounds + add > kPatchRounds || ext + ev > kPatchHalo * 3 / 4) break;
            pq.pop();
            visit[v] = t;
            ++done;
            rounds += add;
            if (l != cur_lev) { cur_lev = l; cur_cnt = 0; }
            ++cur_cnt;
            ext += ev;
            for (int32_t k = dptr[v]; k < dptr[v + 1]; ++k) {
                const int32_t w = dn[k];
                if (--indeg[w] == 0) {
                    if (patch[w] == best) pq.push({lev[w], w});
                    else push(w);
                }
            }
        }
        while (!pq.empty()) {
            push(pq.top().second);
            pq.pop();
        }
    }
    // depth: visits were made in a topological order of the task graph
    std::vector<int32_t> off(nv + 1, 0), byv(nc);
    for (int64_t v = 0; v < nc; ++v) ++off[visit[v] + 1];
    for (uint32_t t = 0; t < nv; ++t) off[t + 1] += off[t];
    {
        std::vector<int32_t> fill(off.begin(), off.end() - 1);
        for (int64_t v = 0; v < nc; ++v) byv[fill[visit[v]]++] = (int32_t)v;
    }
    depth.assign(nv, 0);
    for (uint32_t t = 0; t < nv; ++t) {
        int32_t d = 0;
        for (int32_t k = off[t]; k < off[t + 1]; ++k) {
            const int32_t v = byv[k];
            for (int j = 0; j < ns; ++j) {
                const int32_t u = up[(int64_t)v * ns + j];
                if (u < 0) break;
                if (visit[u] != t) d = std::max(d, depth[visit[u]] + 1);
            }
        }
        depth[t] = d;
    }
}

template <int NF, int DIM>
void build_patch(Graph &g, hipStream_t s) {
    using Rec = CellRec<double, NF, DIM>;
    PatchProg &pp = g.pp;
    pp.built = true;
    pp.ok = false;
    const int64_t nc = g.nc, N = nc * g.nd;
    const int P = patch_cells(g.ctype);
    pp.P = P;
    const int64_t npatch = ceil_div(nc, P);
    // key widths: direction 10 bits, task id 27 bits, level position 27 bits
    // (the visit order is built on the host: graphs up to 2^26 vertices)
    if (g.nd > 1023 || nc >= (1ll << 27) || N >= (1ll << 26)) return;
    const Rec *rec = g.rec64.as<Rec>();
    const double *om = g.omega64.as<double>();
    const uint64_t *lmv = g.lag_mv.as<uint64_t>();
    const int32_t *lu = g.lag_u.as<int32_t>();
    // the visits of every direction, on the host (one thread per direction
    // at a time, directions spread over the host's cores)
    const int ns = g.ns;
    DevBuf dup(4 * (size_t)ns * N);
    k_pp_upwind<NF, DIM><<<blocks_for(N), kB, 0, s>>>(rec, om, nc, N, ns, lmv, lu, g.n_lag, dup.as<int32_t>());
    JSW_HIP(hipGetLastError());
    std::vector<int32_t> up_h = to_host<int32_t>(dup, (int64_t)ns * N, s);
    dup.release();
    std::vector<int32_t> lev_h = to_host<int32_t>(g.level, N, s);
    std::vector<int32_t> rank_h = to_host<int32_t>(g.mrank, nc, s);
    std::vector<int32_t> patch_h(nc);
    for (int64_t v = 0; v < nc; ++v) patch_h[v] = rank_h[v] / P;
    std::vector<uint32_t> tkey_h(N);
    std::vector<std::vector<int32_t>> depth_dir(g.nd);
    {
        std::atomic<int> next{0};
        auto work = [&]() {
            for (int m; (m = next.fetch_add(1)) < g.nd;)
                visits(nc, ns, up_h.data() + (int64_t)m * nc * ns, lev_h.data() + (int64_t)m * nc, patch_h.data(),
                       (int32_t)npatch, tkey_h.data() + (int64_t)m * nc, depth_dir[m]);
        };
        const int nth = (int)std::max(1u, std::min<unsigned>(16, std::thread::hardware_concurrency()));
        std::vector<std::thread> th;
        for (int k = 1; k < nth; ++k) th.emplace_back(work);
        work();
        for (auto &x : th) x.join();
    }
    DevBuf tkey(4 * N), ctr(8);
    JSW_HIP(hipMemcpyAsync(tkey.p, tkey_h.data(), 4 * N, hipMemcpyHostToDevice, s));
    std::vector<uint64_t> tk_h;                 // (m, visit) of every task, sorted
    std::vector<int32_t> tdepth;                // depth of each task in its direction's task graph
    pp.revisits = 0;
    for (int m = 0; m < g.nd; ++m) {
        const int64_t nv_m = (int64_t)depth_dir[m].size();
        for (int64_t t = 0; t < nv_m; ++t) {
            tk_h.push_back((uint64_t)m << 32 | (uint64_t)t);
            tdepth.push_back(depth_dir[m][t]);
        }
        std::vector<char> seen(npatch, 0);
        int64_t distinct = 0;
        for (int64_t v = 0; v < nc; ++v)
            if (!seen[patch_h[v]]) { seen[patch_h[v]] = 1; ++distinct; }
        pp.revisits += nv_m - distinct;
    }
    up_h.clear();
    up_h.shrink_to_fit();
    lev_h.clear();
    lev_h.shrink_to_fit();
    // task ids: by stream, then depth, direction and key
    const int64_t nt = (int64_t)tk_h.size();
    if (nt >= (1ll << 27)) return;
    std::vector<int64_t> order(nt);
    for (int64_t k = 0; k < nt; ++k) order[k] = k;
    auto stream_of = [&](int64_t k) { return g.dir_stream_h[tk_h[k] >> 32]; };
    std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
        const int sx = stream_of(x), sy = stream_of(y);
        if (sx != sy) return sx < sy;
        if (tdepth[x] != tdepth[y]) return tdepth[x] < tdepth[y];
        return tk_h[x] < tk_h[y];
    });
    std::vector<int32_t> tid_of(nt);
    pp.stream_off_h.assign(kStreams + 1, 0);
    for (int64_t r = 0; r < nt; ++r) {
        tid_of[order[r]] = (int32_t)r;
        ++pp.stream_off_h[stream_of(order[r]) + 1];
    }
    for (int k = 0; k < kStreams; ++k) pp.stream_off_h[k + 1] += pp.stream_off_h[k];
    pp.n_tasks = nt;
    DevBuf d_tk(8 * nt), d_tid(4 * nt);
    JSW_HIP(hipMemcpyAsync(d_tk.p, tk_h.data(), 8 * nt, hipMemcpyHostToDevice, s));
    JSW_HIP(hipMemcpyAsync(d_tid.p, tid_of.data(), 4 * nt, hipMemcpyHostToDevice, s));
    // positions
    DevBuf skey(8 * N), sval(4 * N);
    k_pp_tid<<<blocks_for(N), kB, 0, s>>>(tkey.as<uint32_t>(), nc, N, d_tk.as<uint64_t>(), nt, d_tid.as<int32_t>(),
                                          g.posi.as<int32_t>(), skey.as<uint64_t>(), sval.as<int32_t>());
    JSW_HIP(hipGetLastError());
    sort_pairs<uint64_t, int32_t>(skey, &sval, N, 64, s);
    pp.cell = std::move(sval);
    tkey.release();
    DevBuf ptid(4 * N), ppos(4 * N), tstart(4 * nt), tend(4 * nt), tdir(4 * nt), smark(8 * N);
    k_pp_positions<<<blocks_for(N), kB, 0, s>>>(skey.as<uint64_t>(), pp.cell.as<int32_t>(), g.level.as<int32_t>(), nc,
                                                N, ptid.as<int32_t>(), ppos.as<int32_t>(), tstart.as<int32_t>(),
                                                tend.as<int32_t>(), tdir.as<int32_t>(), smark.as<int64_t>());
    JSW_HIP(hipGetLastError());
    skey.release();
    // rounds: steps (levels of a task) cut into pieces of 64
    {
        DevBuf sstart(8 * N);
        size_t bytes = 0;
        JSW_HIP(rocprim::inclusive_scan(nullptr, bytes, smark.as<int64_t>(), sstart.as<int64_t>(), (size_t)N,
                                        rocprim::maximum<int64_t>(), s));
        DevBuf tmp(bytes + 16);
        JSW_HIP(rocprim::inclusive_scan(tmp.p, bytes, smark.as<int64_t>(), sstart.as<int64_t>(), (size_t)N,
                                        rocprim::maximum<int64_t>(), s));
        smark.release();
        DevBuf mark(4 * N), ridx(4 * N);
        k_pp_round_mark<<<blocks_for(N), kB, 0, s>>>(sstart.as<int64_t>(), N, mark.as<int32_t>());
        JSW_HIP(hipGetLastError());
        JSW_HIP(hipStreamSynchronize(s));
        sstart.release();
        bytes = 0;
        JSW_HIP(rocprim::inclusive_scan(nullptr, bytes, mark.as<int32_t>(), ridx.as<int32_t>(), (size_t)N,
                                        rocprim::plus<int32_t>(), s));
        DevBuf tmp2(bytes + 16);
        JSW_HIP(rocprim::inclusive_scan(tmp2.p, bytes, mark.as<int32_t>(), ridx.as<int32_t>(), (size_t)N,
                                        rocprim::plus<int32_t>(), s));
        int32_t nr = 0;
        JSW_HIP(hipMemcpyAsync(&nr, ridx.as<int32_t>() + (N - 1), 4, hipMemcpyDeviceToHost, s));
        JSW_HIP(hipStreamSynchronize(s));
        pp.n_rounds = nr;
        DevBuf rabs(4 * std::max(1, nr)), round0(4 * nt), nround(4 * nt);
        k_pp_rounds<<<blocks_for(N), kB, 0, s>>>(mark.as<int32_t>(), ridx.as<int32_t>(), ptid.as<int32_t>(),
                                                 tstart.as<int32_t>(), tend.as<int32_t>(), nc, N, rabs.as<int32_t>(),
                                                 round0.as<int32_t>(), nround.as<int32_t>());
        JSW_HIP(hipGetLastError());
        pp.round.alloc(4 * std::max(1, nr));
        k_pp_round_table<<<blocks_for(nr), kB, 0, s>>>(rabs.as<int32_t>(), nr, N, nc, ptid.as<int32_t>(),
                                                       tstart.as<int32_t>(), tend.as<int32_t>(), pp.round.as<int32_t>());
        JSW_HIP(hipGetLastError());
        // halo
        JSW_HIP(hipMemsetAsync(ctr.p, 0, 8, s));
        k_pp_halo<NF, DIM, false><<<blocks_for(N), kB, 0, s>>>(rec, om, nc, N, lmv, lu, g.n_lag, pp.cell.as<int32_t>(),
                                                               ptid.as<int32_t>(), ppos.as<int32_t>(),
                                                               ctr.as<unsigned long long>(), nullptr);
        JSW_HIP(hipGetLastError());
        unsigned long long nh = 0;
        JSW_HIP(hipMemcpyAsync(&nh, ctr.p, 8, hipMemcpyDeviceToHost, s));
        JSW_HIP(hipStreamSynchronize(s));
        DevBuf hk(8 * std::max<unsigned long long>(1, nh));
        JSW_HIP(hipMemsetAsync(ctr.p, 0, 8, s));
        k_pp_halo<NF, DIM, true><<<blocks_for(N), kB, 0, s>>>(rec, om, nc, N, lmv, lu, g.n_lag, pp.cell.as<int32_t>(),
                                                              ptid.as<int32_t>(), ppos.as<int32_t>(),
                                                              ctr.as<unsigned long long>(), hk.as<uint64_t>());
        JSW_HIP(hipGetLastError());
        sort_pairs<uint64_t, int32_t>(hk, nullptr, (int64_t)nh, 64, s);
        const int64_t nhu = unique_sorted(hk, (int64_t)nh, s);
        pp.n_halo = nhu;
        DevBuf hstart(4 * nt), hend(4 * nt), dstart(4 * nt), dend(4 * nt);
        JSW_HIP(hipMemsetAsync(hstart.p, 0, 4 * nt, s));
        JSW_HIP(hipMemsetAsync(hend.p, 0, 4 * nt, s));
        JSW_HIP(hipMemsetAsync(dstart.p, 0, 4 * nt, s));
        JSW_HIP(hipMemsetAsync(dend.p, 0, 4 * nt, s));
        pp.halo.alloc(4 * std::max<int64_t>(1, nhu));
        DevBuf dk(8 * std::max<int64_t>(1, nhu));
        if (nhu) {
            k_pp_ranges<<<blocks_for(nhu), kB, 0, s>>>(hk.as<uint64_t>(), nhu, hstart.as<int32_t>(), hend.as<int32_t>());
            k_pp_halo_out<<<blocks_for(nhu), kB, 0, s>>>(hk.as<uint64_t>(), nhu, tdir.as<int32_t>(), ptid.as<int32_t>(),
                                                         nc, pp.halo.as<int32_t>(), dk.as<uint64_t>());
            JSW_HIP(hipGetLastError());
        }
        // dependencies: distinct upstream tasks of the halo
        sort_pairs<uint64_t, int32_t>(dk, nullptr, nhu, 64, s);
        int64_t nd_ = unique_sorted(dk, nhu, s);
        if (nd_ > 0) {
            uint64_t last = 0;
            JSW_HIP(hipMemcpyAsync(&last, dk.as<uint64_t>() + nd_ - 1, 8, hipMemcpyDeviceToHost, s));
            JSW_HIP(hipStreamSynchronize(s));
            if (last == ~0ull) --nd_;
        }
        pp.n_dep = nd_;
        pp.dep.alloc(4 * std::max<int64_t>(1, nd_));
        if (nd_) {
            k_pp_ranges<<<blocks_for(nd_), kB, 0, s>>>(dk.as<uint64_t>(), nd_, dstart.as<int32_t>(), dend.as<int32_t>());
            k_pp_dep_out<<<blocks_for(nd_), kB, 0, s>>>(dk.as<uint64_t>(), nd_, pp.dep.as<int32_t>());
            JSW_HIP(hipGetLastError());
        }
        // codes and coefficients
        pp.ns = g.ns;
        pp.code.alloc(4 * (size_t)g.ns * N);
        pp.a64.alloc(8 * (size_t)g.ns * N);
        k_pp_code<NF, DIM><<<blocks_for(N), kB, 0, s>>>(rec, om, nc, N, g.ns, lmv, lu, g.n_lag, pp.cell.as<int32_t>(),
                                                        ptid.as<int32_t>(), ppos.as<int32_t>(), tstart.as<int32_t>(),
                                                        tend.as<int32_t>(), hk.as<uint64_t>(), hstart.as<int32_t>(),
                                                        hend.as<int32_t>(), pp.code.as<int32_t>(), pp.a64.as<double>());
        JSW_HIP(hipGetLastError());
        pp.desc.alloc(4 * kPatchDesc * nt);
        k_pp_desc<<<blocks_for(nt), kB, 0, s>>>(nt, tstart.as<int32_t>(), tend.as<int32_t>(), tdir.as<int32_t>(),
                                                round0.as<int32_t>(), nround.as<int32_t>(), hstart.as<int32_t>(),
                                                hend.as<int32_t>(), dstart.as<int32_t>(), dend.as<int32_t>(),
                                                pp.desc.as<int32_t>());
        JSW_HIP(hipGetLastError());
    }
    // limits of the kernel
    std::vector<int32_t> desc = to_host<int32_t>(pp.desc, kPatchDesc * nt, s);
    for (int64_t t = 0; t < nt; ++t) {
        const int32_t *d = desc.data() + t * kPatchDesc;
        if (d[2] > kPatchCells || d[5] > kPatchHalo || d[2] + d[5] > kPatchSlots || d[3] > kPatchRounds || d[2] < 1)
            return;
    }
    // downstream tasks of every task (the upstream lists reversed), and the
    // tasks without upstream tasks, which are the first of their stream
    {
        std::vector<int32_t> dep_h = to_host<int32_t>(pp.dep, pp.n_dep, s);
        std::vector<int32_t> dptr(nt + 1, 0), dn(std::max<int64_t>(1, pp.n_dep));
        for (int64_t t = 0; t < nt; ++t) {
            const int32_t *d = desc.data() + t * kPatchDesc;
            for (int32_t k = 0; k < d[7]; ++k) ++dptr[dep_h[d[8] + k] + 1];
        }
        for (int64_t t = 0; t < nt; ++t) dptr[t + 1] += dptr[t];
        std::vector<int32_t> fill(dptr.begin(), dptr.end() - 1);
        for (int64_t t = 0; t < nt; ++t) {
            const int32_t *d = desc.data() + t * kPatchDesc;
            for (int32_t k = 0; k < d[7]; ++k) dn[fill[dep_h[d[8] + k]]++] = (int32_t)t;
        }
        std::vector<int32_t> nsrc(kStreams, 0);
        for (int k = 0; k < kStreams; ++k) {
            int64_t t = pp.stream_off_h[k];
            while (t < pp.stream_off_h[k + 1] && desc[t * kPatchDesc + 7] == 0) ++t;
            nsrc[k] = (int32_t)(t - pp.stream_off_h[k]);
            for (; t < pp.stream_off_h[k + 1]; ++t)
                if (desc[t * kPatchDesc + 7] == 0) return;   // sources must lead their stream
        }
        for (int64_t t = 0; t < nt; ++t) {
            desc[t * kPatchDesc + 9] = dptr[t + 1] - dptr[t];
            desc[t * kPatchDesc + 10] = dptr[t];
        }
        JSW_HIP(hipMemcpyAsync(pp.desc.p, desc.data(), 4 * desc.size(), hipMemcpyHostToDevice, s));
        pp.down.alloc(4 * dn.size());
        JSW_HIP(hipMemcpyAsync(pp.down.p, dn.data(), 4 * dn.size(), hipMemcpyHostToDevice, s));
        pp.nsrc.alloc(4 * kStreams);
        JSW_HIP(hipMemcpyAsync(pp.nsrc.p, nsrc.data(), 4 * kStreams, hipMemcpyHostToDevice, s));
        JSW_HIP(hipStreamSynchronize(s));
    }
    if (nt >= (1ll << 24)) return;   // queue entries carry 24-bit task ids
    pp.stream_off.alloc(8 * (kStreams + 1));
    JSW_HIP(hipMemcpyAsync(pp.stream_off.p, pp.stream_off_h.data(), 8 * (kStreams + 1), hipMemcpyHostToDevice, s));
    pp.cnt.alloc(4 * std::max<int64_t>(nt, 1));
    pp.slot.alloc(4 * std::max<int64_t>(nt, 1));
    JSW_HIP(hipMemsetAsync(pp.slot.p, 0, pp.slot.bytes, s));
    pp.qctl.alloc(4 * 32 * kStreams);
    pp.psi.alloc(8 * N);
    pp.den64.alloc(8 * N);
    pp.den64_ok = false;
    pp.epoch = 0;
    JSW_HIP(hipStreamSynchronize(s));
    pp.ok = true;
}

template <int NF, int DIM>
void den_impl(Graph &g, hipStream_t s) {
    const int64_t N = g.nc * g.nd;
    k_pp_den<NF, DIM><<<blocks_for(N), kB, 0, s>>>(g.rec64.as<CellRec<double, NF, DIM>>(), g.omega64.as<double>(),
                                                   g.pp.cell.as<int32_t>(), g.nc, N, g.pp.den64.as<double>());
    JSW_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// the kernel
// ---------------------------------------------------------------------------
struct PatchArgs {
    const int32_t *desc, *round, *halo, *dep, *cell, *code;
    const double *pa, *pden;
    int64_t N, nc;
    const double *vs;
    double *psi, *ppsi;
    const double *lag_val;
    int32_t *cnt;          // upstream tasks not yet complete, per task
    uint32_t *slot;        // ready queue of every stream: epoch << 24 | task
    uint32_t *qctl;        // per stream (128 B apart): head, tail at +16
    const int32_t *down;   // downstream tasks (CSR through the descriptors)
    int32_t *status;
    const int64_t *stream_off;
    uint32_t epoch, nap;
    uint64_t watchdog_ticks;
    double psi_b;
    uint32_t *stamps;   // per task: taken, upstream complete, published (s_memrealtime), or null
};

template <class T>
__device__ __forceinline__ T ld_agent(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// LDS code of an inflow slot: an LDS slot, the boundary or no face
constexpr uint16_t kLdsBoundary = 0xffff, kLdsNoFace = 0xfffe;

// NS: inflow slots per vertex.  Tasks come out of the stream's ready queue
// (the paper's ready queues, Listing 1, at task granularity): a wavefront
// only ever takes a task whose upstream tasks are complete, and the last
// upstream task to finish appends it.
template <int NS>
__global__ void __launch_bounds__(64) k_sweep_patch(PatchArgs a) {
    constexpr int kCL = kPatchCells / 64, kHL = kPatchHalo / 64;
    __shared__ double sv[kPatchSlots];         // fluxes: the task's vertices, then its halo
    __shared__ double svs[kPatchCells];        // V s of the task's vertices
    __shared__ double sden[kPatchCells];
    __shared__ double sa[NS][kPatchCells];
    __shared__ uint16_t scode[NS][kPatchCells];
    __shared__ int32_t scell[kPatchCells];
    __shared__ int32_t srnd[kPatchRounds];
    const int lane = threadIdx.x;
    const int stream = (int)(blockIdx.x % kStreams);
    const int64_t first = a.stream_off[stream];
    const int64_t per_stream = a.stream_off[stream + 1] - first;
    const uint32_t epoch = a.epoch & 0xffu;
    uint32_t *qctl = a.qctl + 32 * stream;
    if (!check_stream_placement(qctl + kXccSlot, a.status)) return;   // takes no task
    while (true) {
        uint32_t hv = 0;
        if (lane == 0) hv = atomicAdd(qctl, 1u);
        const int64_t h = (int64_t)__builtin_amdgcn_readfirstlane(hv);
        if (h >= per_stream) break;
        const uint32_t t_take = (uint32_t)__builtin_amdgcn_s_memrealtime();
        // the h-th task to become ready in this stream
        uint32_t sl = 0;
        uint64_t t0 = 0;
        for (uint32_t spin = 0;; ++spin) {
            sl = __builtin_amdgcn_readfirstlane(ld_agent(a.slot + first + h));
            if ((sl >> 24) == epoch) break;
            if (spin == 0) t0 = __builtin_amdgcn_s_memrealtime();
            if ((spin & 7) == 7) {
                bool stop = ld_agent(a.status) != 0;
                if (!stop && __builtin_amdgcn_s_memrealtime() - t0 > a.watchdog_ticks) {
                    if (lane == 0) atomicOr(a.status, kStatusStalled);
                    stop = true;
                }
                if (__any(stop)) return;
            }
            for (uint32_t z = 0; z < a.nap; ++z) __builtin_amdgcn_s_sleep(1);
        }
        const int64_t t = sl & 0xffffffu;
        const uint32_t t_ready = (uint32_t)__builtin_amdgcn_s_memrealtime();
        const int32_t w = lane < kPatchDesc ? a.desc[t * kPatchDesc + lane] : 0;
        const int q0 = __builtin_amdgcn_readlane(w, 0), m = __builtin_amdgcn_readlane(w, 1);
        const int n = __builtin_amdgcn_readlane(w, 2), nr = __builtin_amdgcn_readlane(w, 3);
        const int r0 = __builtin_amdgcn_readlane(w, 4), nh = __builtin_amdgcn_readlane(w, 5);
        const int h0 = __builtin_amdgcn_readlane(w, 6), ndn = __builtin_amdgcn_readlane(w, 9);
        const int dn0 = __builtin_amdgcn_readlane(w, 10);
        const int64_t base = (int64_t)m * a.nc, qa = base + q0;
        // the whole task into LDS: program, vertices, rounds and halo, all
        // loads issued together (a task's positions are contiguous)
        {
            int32_t cl[kCL], cd[NS][kCL], hs[kHL];
            double af[NS][kCL], dn[kCL];
#pragma unroll
            for (int k = 0; k < kCL; ++k) {
                const bool in = lane + 64 * k < n;
                const int64_t q = qa + (in ? lane + 64 * k : 0);
                cl[k] = a.cell[q];
#pragma unroll
                for (int j = 0; j < NS; ++j) {
                    cd[j][k] = a.code[(int64_t)j * a.N + q];
                    af[j][k] = a.pa[(int64_t)j * a.N + q];
                }
                dn[k] = a.pden[q];
            }
            const int32_t rl = lane < nr ? a.round[r0 + lane] : 0;
#pragma unroll
            for (int k = 0; k < kHL; ++k) hs[k] = lane + 64 * k < nh ? a.halo[h0 + lane + 64 * k] : 0;
            double vl[kCL], hv2[kHL];
#pragma unroll
            for (int k = 0; k < kCL; ++k) vl[k] = a.vs[cl[k]];
#pragma unroll
            for (int k = 0; k < kHL; ++k)
                hv2[k] = lane + 64 * k >= nh ? 0.0
                         : hs[k] >= 0     ? ld_agent(a.ppsi + base + hs[k])
                                          : a.lag_val[-(int64_t)hs[k] - 1];
#pragma unroll
            for (int k = 0; k < kCL; ++k) {
                const int i = lane + 64 * k;
                if (i < n) {
                    scell[i] = cl[k];
                    svs[i] = vl[k];
                    sden[i] = dn[k];
#pragma unroll
                    for (int j = 0; j < NS; ++j) {
                        const int32_t c = cd[j][k];
                        scode[j][i] = c >= 0 ? (uint16_t)c : c == -1 ? kLdsBoundary : kLdsNoFace;
                        sa[j][i] = af[j][k];
                    }
                }
            }
            if (lane < nr) srnd[lane] = rl;
#pragma unroll
            for (int k = 0; k < kHL; ++k)
                if (lane + 64 * k < nh) sv[n + lane + 64 * k] = hv2[k];
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        // rounds, out of LDS only; the next round's program is read while
        // the current one computes (it does not depend on the fluxes)
        {
            struct Rd {
                uint16_t c[NS];
                double af[NS], den, num0;
                int i, cnt;
            };
            auto read_round = [&](int r, Rd &x) {
                const int32_t rd = srnd[r];
                x.cnt = (rd >> 16) + 1;
                x.i = (rd & 0xffff) + min(lane, x.cnt - 1);
#pragma unroll
                for (int j = 0; j < NS; ++j) {
                    x.c[j] = scode[j][x.i];
                    x.af[j] = sa[j][x.i];
                }
                x.den = sden[x.i];
                x.num0 = svs[x.i];
            };
            Rd cur, nxt;
            read_round(0, cur);
            for (int r = 0; r < nr; ++r) {
                double vv[NS];
#pragma unroll
                for (int j = 0; j < NS; ++j) vv[j] = sv[cur.c[j] < kLdsNoFace ? cur.c[j] : 0];
                read_round(min(r + 1, nr - 1), nxt);
                double num = cur.num0;
#pragma unroll
                for (int j = 0; j < NS; ++j) {
                    const double v = cur.c[j] == kLdsBoundary ? a.psi_b : vv[j];
                    const double acc = num + cur.af[j] * v;
                    num = cur.c[j] != kLdsNoFace ? acc : num;
                }
                const double res = num / cur.den;
                if (lane < cur.cnt) sv[cur.i] = res;
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                cur = nxt;
            }
        }
        // publish the fluxes by position; once they are complete, count
        // this task off every downstream task and queue those it completes
        for (int i = lane; i < n; i += 64) a.ppsi[qa + i] = sv[i];
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        for (int k = lane; k < ndn; k += 64) {
            const int32_t d = a.down[dn0 + k];
            if (atomicSub(a.cnt + d, 1) == 1) {
                const uint32_t pos = atomicAdd(qctl + 16, 1u);
                a.slot[first + pos] = epoch << 24 | (uint32_t)d;
            }
        }
        for (int i = lane; i < n; i += 64) a.psi[base + scell[i]] = sv[i];
        if (a.stamps && lane == 0) {
            a.stamps[3 * t] = t_take;
            a.stamps[3 * t + 1] = t_ready;
            a.stamps[3 * t + 2] = (uint32_t)__builtin_amdgcn_s_memrealtime();
        }
    }
}

// per sweep: dependency counts, the queues' heads and tails, and the
// sources (the first tasks of every stream) queued
__global__ void k_pp_reset(const int32_t *desc, int64_t n_tasks, const int64_t *stream_off, const int32_t *nsrc,
                           uint32_t epoch, int32_t *cnt, uint32_t *slot, uint32_t *qctl) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < kStreams) {
        qctl[32 * t] = 0u;
        qctl[32 * t + kXccSlot] = kNoXcc;
        qctl[32 * t + 16] = (uint32_t)nsrc[t];
    }
    if (t >= n_tasks) return;
    cnt[t] = desc[t * kPatchDesc + 7];
    int s = 0;
    while (s + 1 < kStreams && stream_off[s + 1] <= t) ++s;
    if (t - stream_off[s] < nsrc[s]) slot[t] = (epoch & 0xffu) << 24 | (uint32_t)t;
}

template <int NS>
const void *patch_kernel_ns() {
    return reinterpret_cast<const void *>(&k_sweep_patch<NS>);
}

const void *patch_kernel(int ns) {
    switch (ns) {
    case 1: return patch_kernel_ns<1>();
    case 2: return patch_kernel_ns<2>();
    case 3: return patch_kernel_ns<3>();
    case 4: return patch_kernel_ns<4>();
    case 5: return patch_kernel_ns<5>();
    default: return patch_kernel_ns<6>();
    }
}

uint64_t pp_watchdog_ticks() {
    const char *e = std::getenv("JSWEEP_WATCHDOG_MS");
    double ms = e ? std::atof(e) : 4000.0;
    if (!(ms > 0)) ms = 4000.0;
    return (uint64_t)(ms * 1e5);   // s_memrealtime runs at 100 MHz
}

}  // namespace

bool patch_ready(Graph &g, hipStream_t s) {
    if (!g.pp.built) {
        if (!g.posi.p || !g.mrank.p || g.ns < 1 || g.ns > 6) {
            g.pp.built = true;
            g.pp.ok = false;
        } else if (g.ctype == JSWEEP_TRI) build_patch<3, 2>(g, s);
        else if (g.ctype == JSWEEP_TET) build_patch<4, 3>(g, s);
        else build_patch<6, 3>(g, s);
    }
    return g.pp.ok;
}

void patch_den(Graph &g, hipStream_t s) {
    if (!g.pp.ok) return;
    if (g.ctype == JSWEEP_TRI) den_impl<3, 2>(g, s);
    else if (g.ctype == JSWEEP_TET) den_impl<4, 3>(g, s);
    else den_impl<6, 3>(g, s);
    g.pp.den64_ok = true;
}

void launch_patch64(Graph &g, const double *src_cell, double *psi, double psi_b, const jsweep_params *p,
                    hipStream_t s, bool prepared) {
    (void)p;
    PatchProg &pp = g.pp;
    if (!pp.ok) fail(JSWEEP_E_DEVICE, "patch program not available for this graph");
    if (!pp.den64_ok) patch_den(g, s);
    PatchArgs a;
    a.desc = pp.desc.as<int32_t>();
    a.round = pp.round.as<int32_t>();
    a.halo = pp.halo.as<int32_t>();
    a.dep = pp.dep.as<int32_t>();
    a.cell = pp.cell.as<int32_t>();
    a.code = pp.code.as<int32_t>();
    a.pa = pp.a64.as<double>();
    a.pden = pp.den64.as<double>();
    a.N = g.nc * g.nd;
    a.nc = g.nc;
    if (!prepared) {
        if (g.vsc.bytes < (size_t)(8 * g.nc)) g.vsc.alloc(8 * g.nc);
        k_pp_vs<<<blocks_for(g.nc), kB, 0, s>>>(g.vol.as<double>(), src_cell, g.nc, g.vsc.as<double>());
        JSW_HIP(hipGetLastError());
    }
    a.vs = g.vsc.as<double>();
    a.psi = psi;
    a.ppsi = pp.psi.as<double>();
    a.lag_val = g.lag_val64.as<double>();
    a.cnt = pp.cnt.as<int32_t>();
    a.slot = pp.slot.as<uint32_t>();
    a.qctl = pp.qctl.as<uint32_t>();
    a.down = pp.down.as<int32_t>();
    a.status = g.status.as<int32_t>();
    a.stream_off = pp.stream_off.as<int64_t>();
    pp.epoch = pp.epoch % 255 + 1;
    a.epoch = (uint32_t)pp.epoch;
    a.nap = 2;
    a.watchdog_ticks = pp_watchdog_ticks();
    a.psi_b = psi_b;
    a.stamps = nullptr;
    if (g.trace) {
        if (g.trace_buf.bytes < 12 * (size_t)pp.n_tasks) g.trace_buf.alloc(12 * (size_t)pp.n_tasks);
        a.stamps = g.trace_buf.as<uint32_t>();
        g.trace_units = 1;
    }
    const void *kern = patch_kernel(pp.ns);
    int occ = 0;
    JSW_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kern, 64, 0));
    if (occ < 1) occ = 1;
    int64_t blocks = (int64_t)occ * g.n_cu;
    blocks = std::min<int64_t>(blocks, std::max<int64_t>(pp.n_tasks, kStreams));
    blocks = std::max<int64_t>(blocks, kStreams);
    k_pp_reset<<<blocks_for(std::max<int64_t>(pp.n_tasks, kStreams)), kB, 0, s>>>(
        pp.desc.as<int32_t>(), pp.n_tasks, pp.stream_off.as<int64_t>(), pp.nsrc.as<int32_t>(), a.epoch,
        pp.cnt.as<int32_t>(), pp.slot.as<uint32_t>(), pp.qctl.as<uint32_t>());
    JSW_HIP(hipGetLastError());
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (g.profile) {
        JSW_HIP(hipEventCreate(&ev0));
        JSW_HIP(hipEventCreate(&ev1));
        JSW_HIP(hipEventRecord(ev0, s));
    }
    void *args[] = {&a};
    JSW_HIP(hipLaunchKernel(kern, dim3((unsigned)blocks), dim3(64), args, 0, s));
    if (g.profile) {
        JSW_HIP(hipEventRecord(ev1, s));
        g.prof_events.push_back({ev0, ev1});
    }
}

}  // namespace jsw
