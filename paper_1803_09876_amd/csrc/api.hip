// C ABI of the jsweep library: argument checks, handle lifetime, error
// codes.  No exception crosses this boundary.
#include <cstring>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <numeric>
#include <string>

#include "common.hpp"

namespace jsw {

static thread_local std::string t_last_error;

void set_last_error(const std::string &msg) { t_last_error = msg; }

[[noreturn]] void fail(int code, const std::string &msg) { throw Error{code, msg}; }

void hip_check(hipError_t e, const char *what, const char *file, int line) {
    if (e == hipSuccess) return;
    std::string msg = std::string(what) + " failed: " + hipGetErrorString(e) + " (" + file + ":" + std::to_string(line) + ")";
    if (e == hipErrorOutOfMemory) fail(JSWEEP_E_OOM, msg);
    fail(JSWEEP_E_DEVICE, msg);
}

void DevBuf::alloc(size_t n) {
    release();
    if (n == 0) n = 16;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();
        fail(JSWEEP_E_OOM, "hipMalloc of " + std::to_string(n) + " bytes failed");
    }
    bytes = n;
}

void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}

template <class F>
static int guarded(F &&f) {
    try {
        return f();
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return JSWEEP_E_OOM;
    } catch (...) {
        set_last_error("unexpected internal error");
        return JSWEEP_E_DEVICE;
    }
}

static Graph *G(jsweep_graph g) { return reinterpret_cast<Graph *>(g); }

static void check_quadrature(const jsweep_quadrature &q) {
    if (q.n_dirs <= 0 || q.n_dirs > 4096 || !q.omega || !q.weight) fail(JSWEEP_E_INVALID_ARG, "bad quadrature arguments");
    double sw = 0.0;
    for (int m = 0; m < q.n_dirs; ++m) {
        const double *o = q.omega + 3 * m;
        double n2 = o[0] * o[0] + o[1] * o[1] + o[2] * o[2];
        if (!(std::fabs(std::sqrt(n2) - 1.0) <= 1e-12)) fail(JSWEEP_E_QUADRATURE, "direction " + std::to_string(m) + " is not a unit vector");
        if (!(q.weight[m] > 0.0) || !std::isfinite(q.weight[m])) fail(JSWEEP_E_QUADRATURE, "weights must be positive");
        sw += q.weight[m];
    }
    if (!(std::fabs(sw - 1.0) <= 1e-12)) fail(JSWEEP_E_QUADRATURE, "weights must sum to 1");
}

// in-degree of every cell of one direction, recomputed from the records
template <int NF, int DIM>
__global__ void k_export_indeg(const CellRec<double, NF, DIM> *rec, const double *om, int64_t nc, int m,
                               const uint64_t *lag_mv, const int32_t *lag_u, int64_t n_lag, int32_t *out) {
    int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (K >= nc) return;
    CellRec<double, NF, DIM> r = rec[K];
    int c = 0;
    for (int j = 0; j < NF; ++j) {
        int32_t code = r.nbr[j];
        if (code == -1) continue;
        double d = om[0] * r.S[j][0] + om[1] * r.S[j][1];
        if constexpr (DIM == 3) d = d + om[2] * r.S[j][2];
        if (!(d < 0.0)) continue;
        if (code <= -2) {
            int64_t u = -code - 2;
            uint64_t key = ((uint64_t)(uint32_t)m << 32) | (uint64_t)K;
            bool lagged = false;
            for (int64_t e = 0; e < n_lag; ++e)
                if (lag_mv[e] == key && lag_u[e] == u) lagged = true;
            if (lagged) continue;
        }
        ++c;
    }
    out[K] = c;
}

__global__ void k_widen(const int32_t *in, int64_t n, int64_t *out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i];
}

}  // namespace jsw

using namespace jsw;

extern "C" {

int jsweep_build_graph(const jsweep_mesh *mesh, const jsweep_quadrature *quad, uint32_t flags, jsweep_graph *out) {
    return guarded([&]() -> int {
        if (!out) fail(JSWEEP_E_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (!mesh || !quad) fail(JSWEEP_E_INVALID_ARG, "mesh or quadrature is NULL");
        if (flags & ~(JSWEEP_DEBUG_NO_LAG | JSWEEP_PRIORITY_FLAGS(0xff))) fail(JSWEEP_E_INVALID_ARG, "unknown build flag");
        const int priority = (int)((flags >> 8) & 0xffu);
        const jsweep_mesh &M = *mesh;
        bool ok_type = (M.dim == 2 && M.cell_type == JSWEEP_TRI) ||
                       (M.dim == 3 && (M.cell_type == JSWEEP_TET || M.cell_type == JSWEEP_HEX));
        if (!ok_type) fail(JSWEEP_E_INVALID_ARG, "cell type does not match the dimension");
        if (M.n_cells <= 0 || M.n_vertices <= 0 || !M.coords || !M.cell_vertices)
            fail(JSWEEP_E_INVALID_ARG, "empty mesh or NULL arrays");
        if (M.n_cells * faces_of(M.cell_type) >= ((int64_t)1 << 31)) fail(JSWEEP_E_INVALID_ARG, "too many cells");
        if (M.dim == 3 && M.n_vertices >= ((int64_t)1 << 21)) fail(JSWEEP_E_INVALID_ARG, "3D meshes need fewer than 2^21 vertices");
        if (M.dim == 2 && M.n_vertices >= ((int64_t)1 << 32)) fail(JSWEEP_E_INVALID_ARG, "too many vertices");
        for (int64_t i = 0; i < M.n_vertices * M.dim; ++i)
            if (!std::isfinite(M.coords[i])) fail(JSWEEP_E_MESH, "non-finite vertex coordinate");
        check_quadrature(*quad);
        auto g = std::make_unique<Graph>();
        g->uid = next_graph_uid();
        JSW_HIP(hipGetDevice(&g->device));
        hipDeviceProp_t prop;
        JSW_HIP(hipGetDeviceProperties(&prop, g->device));
        g->n_cu = prop.multiProcessorCount;
        g->nd = quad->n_dirs;
        g->omega_h.assign(quad->omega, quad->omega + 3 * g->nd);
        if (M.dim == 2)
            for (int m = 0; m < g->nd; ++m) g->omega_h[3 * m + 2] = 0.0;
        g->weight_h.assign(quad->weight, quad->weight + g->nd);
        std::vector<float> om32(g->omega_h.begin(), g->omega_h.end());
        g->omega64.alloc(8 * 3 * g->nd);
        g->omega32.alloc(4 * 3 * g->nd);
        g->weight.alloc(8 * g->nd);
        hipStream_t s = nullptr;
        JSW_HIP(hipMemcpy(g->omega64.p, g->omega_h.data(), 8 * 3 * g->nd, hipMemcpyHostToDevice));
        JSW_HIP(hipMemcpy(g->omega32.p, om32.data(), 4 * 3 * g->nd, hipMemcpyHostToDevice));
        JSW_HIP(hipMemcpy(g->weight.p, g->weight_h.data(), 8 * g->nd, hipMemcpyHostToDevice));
        build_geometry(*g, M, s);
        build_dag(*g, !(flags & JSWEEP_DEBUG_NO_LAG), s);
        if (priority) set_priority(*g, priority, s);
        JSW_HIP(hipDeviceSynchronize());
        *out = reinterpret_cast<jsweep_graph>(g.release());
        return JSWEEP_OK;
    });
}

int jsweep_graph_info(jsweep_graph h, int64_t *n_cells, int32_t *n_dirs, int64_t *n_lagged, int32_t *max_levels) {
    return guarded([&]() -> int {
        if (!h) fail(JSWEEP_E_INVALID_ARG, "graph is NULL");
        Graph &g = *G(h);
        if (n_cells) *n_cells = g.nc;
        if (n_dirs) *n_dirs = g.nd;
        if (n_lagged) *n_lagged = g.n_lag;
        if (max_levels) *max_levels = g.max_levels;
        return JSWEEP_OK;
    });
}

int jsweep_program_info(jsweep_graph h, int32_t *slots, int32_t *block_slots, int32_t *packed) {
    return guarded([&]() -> int {
        if (!h) fail(JSWEEP_E_INVALID_ARG, "graph is NULL");
        Graph &g = *G(h);
        if (slots) *slots = g.ns;
        if (block_slots) *block_slots = g.ns_x;
        if (packed) *packed = g.pk.p ? 1 : 0;
        return JSWEEP_OK;
    });
}

int jsweep_graph_export(jsweep_graph h, int32_t dir, int32_t *indeg, int32_t *level, int64_t *lvl_ptr,
                        int64_t *lvl_cells, int32_t *n_levels, uint32_t flags) {
    return guarded([&]() -> int {
        if (!h) fail(JSWEEP_E_INVALID_ARG, "graph is NULL");
        Graph &g = *G(h);
        if (dir < 0 || dir >= g.nd) fail(JSWEEP_E_INVALID_ARG, "direction out of range");
        if (flags & ~JSWEEP_HOST_PTRS) fail(JSWEEP_E_INVALID_ARG, "unknown export flag");
        const bool host = flags & JSWEEP_HOST_PTRS;
        const int64_t nc = g.nc;
        const int B = 256;
        if (n_levels) *n_levels = g.nlev_h[dir];
        auto put = [&](void *dst, const void *dev, size_t bytes) {
            JSW_HIP(hipMemcpy(dst, dev, bytes, host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice));
        };
        if (indeg) {
            DevBuf tmp(4 * nc);
            const double *om = g.omega64.as<double>() + 3 * dir;
            int gb = (int)ceil_div(nc, B);
            if (g.ctype == JSWEEP_TRI)
                k_export_indeg<3, 2><<<gb, B>>>(g.rec64.as<CellRec<double, 3, 2>>(), om, nc, dir, g.lag_mv.as<uint64_t>(), g.lag_u.as<int32_t>(), g.n_lag, tmp.as<int32_t>());
            else if (g.ctype == JSWEEP_TET)
                k_export_indeg<4, 3><<<gb, B>>>(g.rec64.as<CellRec<double, 4, 3>>(), om, nc, dir, g.lag_mv.as<uint64_t>(), g.lag_u.as<int32_t>(), g.n_lag, tmp.as<int32_t>());
            else
                k_export_indeg<6, 3><<<gb, B>>>(g.rec64.as<CellRec<double, 6, 3>>(), om, nc, dir, g.lag_mv.as<uint64_t>(), g.lag_u.as<int32_t>(), g.n_lag, tmp.as<int32_t>());
            JSW_HIP(hipGetLastError());
            put(indeg, tmp.p, 4 * nc);
        }
        if (level) put(level, g.level.as<int32_t>() + (int64_t)dir * nc, 4 * nc);
        if (lvl_cells) {
            DevBuf tmp(8 * nc);
            k_widen<<<(int)ceil_div(nc, B), B>>>(g.lvl_cells.as<int32_t>() + (int64_t)dir * nc, nc, tmp.as<int64_t>());
            JSW_HIP(hipGetLastError());
            put(lvl_cells, tmp.p, 8 * nc);
        }
        if (lvl_ptr) {
            const int64_t *p = g.lvl_ptr_h.data() + g.lvl_off_h[dir];
            size_t bytes = 8 * (size_t)(g.nlev_h[dir] + 1);
            if (host) std::memcpy(lvl_ptr, p, bytes);
            else JSW_HIP(hipMemcpy(lvl_ptr, p, bytes, hipMemcpyHostToDevice));
        }
        JSW_HIP(hipDeviceSynchronize());
        return JSWEEP_OK;
    });
}

int jsweep_graph_lagged(jsweep_graph h, int32_t *dir, int64_t *up, int64_t *down, int32_t *face) {
    return guarded([&]() -> int {
        if (!h) fail(JSWEEP_E_INVALID_ARG, "graph is NULL");
        Graph &g = *G(h);
        // order by (direction, downwind cell, downwind local face)
        std::vector<int64_t> idx(g.n_lag);
        std::vector<int32_t> fc(g.n_lag, -1);
        if (g.n_lag) {
            // local face of the downwind cell: read the records back
            size_t rs = g.rec64.bytes / g.nc;
            std::vector<char> rec(rs);
            for (int64_t e = 0; e < g.n_lag; ++e) {
                JSW_HIP(hipMemcpy(rec.data(), g.rec64.as<char>() + rs * g.lag_v_h[e], rs, hipMemcpyDeviceToHost));
                // neighbour codes follow S[NF][DIM], V and sigV in the record
                const int NF = g.nfpc, DIM = g.dim;
                const int32_t *nbr = reinterpret_cast<const int32_t *>(rec.data() + sizeof(double) * (size_t)(NF * DIM + 2));
                for (int j = 0; j < NF; ++j) {
                    int64_t u = nbr[j] <= -2 ? -(int64_t)nbr[j] - 2 : nbr[j];
                    if (nbr[j] != -1 && u == g.lag_u_h[e]) fc[e] = j;
                }
            }
        }
        std::iota(idx.begin(), idx.end(), 0);
        std::sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) {
            if (g.lag_m_h[a] != g.lag_m_h[b]) return g.lag_m_h[a] < g.lag_m_h[b];
            if (g.lag_v_h[a] != g.lag_v_h[b]) return g.lag_v_h[a] < g.lag_v_h[b];
            return fc[a] < fc[b];
        });
        for (int64_t i = 0; i < g.n_lag; ++i) {
            int64_t e = idx[i];
            if (dir) dir[i] = g.lag_m_h[e];
            if (up) up[i] = g.lag_u_h[e];
            if (down) down[i] = g.lag_v_h[e];
            if (face) face[i] = fc[e];
        }
        return JSWEEP_OK;
    });
}

int jsweep_sweep(jsweep_graph h, const double *sigma_t, const double *source, double *psi, double *phi,
                 double psi_boundary, void *hip_stream) {
    return guarded([&]() -> int {
        if (!h || !sigma_t || !source || !psi) fail(JSWEEP_E_INVALID_ARG, "NULL argument");
        if (!std::isfinite(psi_boundary)) fail(JSWEEP_E_INVALID_ARG, "psi_boundary must be finite");
        Graph &g = *G(h);
        hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
        refresh_sigma(g, sigma_t, false, s);
        lag_snapshot64(g, psi, s);   // previous-iterate values on lagged edges
        launch_sweep64(g, source, psi, psi_boundary, nullptr, s);
        if (phi) scalar_flux(g, psi, phi, s);
        return check_sweep_status(g, s);
    });
}

int jsweep_sweep_noalloc(jsweep_graph h, const double *sigma_t, const double *source, double *psi, double *phi,
                         double psi_boundary, void *hip_stream) {
    return guarded([&]() -> int {
        if (!h || !sigma_t || !source || !psi) fail(JSWEEP_E_INVALID_ARG, "NULL argument");
        if (!std::isfinite(psi_boundary)) fail(JSWEEP_E_INVALID_ARG, "psi_boundary must be finite");
        return sweep_noalloc(*G(h), sigma_t, source, psi, phi, psi_boundary, reinterpret_cast<hipStream_t>(hip_stream));
    });
}

int jsweep_solve(jsweep_graph h, const double *sigma_t, const double *sigma_s, const double *q, double psi_boundary,
                 int32_t mode, double tol, int32_t max_iter, const jsweep_params *params, double *phi, double *psi,
                 jsweep_solve_stats *stats, void *hip_stream) {
    return guarded([&]() -> int {
        if (!h || !sigma_t || !sigma_s || !q || !phi) fail(JSWEEP_E_INVALID_ARG, "NULL argument");
        int prec = mode & 0xff;
        if ((prec != JSWEEP_FP64 && prec != JSWEEP_FP32_REFINED) || (mode & ~0x1ff))
            fail(JSWEEP_E_INVALID_ARG, "unknown mode");
        if ((mode & JSWEEP_WARM_START) && !psi) fail(JSWEEP_E_INVALID_ARG, "warm start needs psi");
        if (max_iter < 1 || !(tol >= 0.0) || !std::isfinite(psi_boundary)) fail(JSWEEP_E_INVALID_ARG, "bad tolerance or iteration limit");
        if (stats && stats->residual_history && stats->history_capacity < 0) fail(JSWEEP_E_INVALID_ARG, "bad history capacity");
        return solve(*G(h), sigma_t, sigma_s, q, psi_boundary, mode, tol, max_iter, params, phi, psi, stats,
                     reinterpret_cast<hipStream_t>(hip_stream));
    });
}

int jsweep_solve_groups(jsweep_graph h, int32_t n_groups, const double *sigma_t, const double *sigma_s, const double *q,
                        double psi_boundary, double tol, int32_t max_iter, const jsweep_params *params, double *phi,
                        double *psi, jsweep_solve_stats *stats, void *hip_stream) {
    return guarded([&]() -> int {
        if (!h || !sigma_t || !sigma_s || !q || !phi) fail(JSWEEP_E_INVALID_ARG, "NULL argument");
        if (n_groups < 1 || n_groups > kMaxGroups) fail(JSWEEP_E_INVALID_ARG, "group count out of range (1..8)");
        if (max_iter < 1 || !(tol >= 0.0) || !std::isfinite(psi_boundary)) fail(JSWEEP_E_INVALID_ARG, "bad tolerance or iteration limit");
        if (stats && stats->residual_history && stats->history_capacity < 0) fail(JSWEEP_E_INVALID_ARG, "bad history capacity");
        return solve_groups(*G(h), n_groups, sigma_t, sigma_s, q, psi_boundary, tol, max_iter, params, phi, psi, stats,
                            reinterpret_cast<hipStream_t>(hip_stream));
    });
}

int jsweep_solve_batch(int32_t n, const jsweep_graph *graphs, const jsweep_problem *problems, int32_t mode, double tol,
                       int32_t max_iter, const jsweep_params *params, jsweep_solve_stats *stats, void *hip_stream) {
    return guarded([&]() -> int {
        if (n <= 0 || !graphs || !problems) fail(JSWEEP_E_INVALID_ARG, "empty batch");
        int prec = mode & 0xff;
        if ((prec != JSWEEP_FP64 && prec != JSWEEP_FP32_REFINED) || (mode & ~0xff))
            fail(JSWEEP_E_INVALID_ARG, "unknown mode (warm start is not supported for batches)");
        if (max_iter < 1 || !(tol >= 0.0)) fail(JSWEEP_E_INVALID_ARG, "bad tolerance or iteration limit");
        std::vector<Graph *> gs(n);
        for (int i = 0; i < n; ++i) {
            if (!graphs[i]) fail(JSWEEP_E_INVALID_ARG, "NULL graph in batch");
            const jsweep_problem &p = problems[i];
            if (!p.sigma_t || !p.sigma_s || !p.q || !p.phi) fail(JSWEEP_E_INVALID_ARG, "NULL problem array");
            gs[i] = G(graphs[i]);
        }
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < i; ++k)
                if (gs[i] == gs[k]) fail(JSWEEP_E_INVALID_ARG, "a graph appears twice in one batch");
        return solve_batch(n, gs.data(), problems, mode, tol, max_iter, params, stats,
                           reinterpret_cast<hipStream_t>(hip_stream));
    });
}

int jsweep_autotune(int32_t n, const jsweep_graph *graphs, int32_t mode, jsweep_params *out) {
    return guarded([&]() -> int {
        if (n <= 0 || !graphs || !out) fail(JSWEEP_E_INVALID_ARG, "bad arguments");
        int prec = mode & 0xff;
        if (prec != JSWEEP_FP64 && prec != JSWEEP_FP32_REFINED) fail(JSWEEP_E_INVALID_ARG, "unknown mode");
        std::vector<Graph *> gs(n);
        for (int i = 0; i < n; ++i) {
            if (!graphs[i]) fail(JSWEEP_E_INVALID_ARG, "NULL graph");
            gs[i] = G(graphs[i]);
        }
        return autotune(n, gs.data(), mode, out);
    });
}

int jsweep_set_params(jsweep_graph h, const jsweep_params *p) {
    return guarded([&]() -> int {
        if (!h) fail(JSWEEP_E_INVALID_ARG, "graph is NULL");
        Graph &g = *G(h);
        if (p) {
            if (p->strategy < 0 || p->strategy > JSWEEP_STRATEGY_PATCH || p->waves_per_block < 0 ||
                p->blocks_per_cu < 0 || p->inner_sweeps < 0 || p->chunks_per_ticket < 0 || p->priority < 0)
                fail(JSWEEP_E_INVALID_ARG, "bad launch parameters");
            if (p->priority) set_priority(g, p->priority, nullptr);
            g.tuned = *p;
            g.has_tuned = true;
        } else {
            g.tuned = jsweep_params{};
            g.has_tuned = false;
        }
        return JSWEEP_OK;
    });
}

int jsweep_patch_info(jsweep_graph h, void *hip_stream, int64_t *out) {
    return guarded([&]() -> int {
        if (!h || !out) fail(JSWEEP_E_INVALID_ARG, "NULL argument");
        Graph &g = *G(h);
        const bool ok = patch_ready(g, reinterpret_cast<hipStream_t>(hip_stream));
        out[0] = ok ? 1 : 0;
        out[1] = g.pp.n_tasks;
        out[2] = g.pp.n_rounds;
        out[3] = g.pp.n_halo;
        out[4] = g.pp.n_dep;
        out[5] = g.pp.revisits;
        return JSWEEP_OK;
    });
}

int jsweep_profile(jsweep_graph h, int32_t enable) {
    return guarded([&]() -> int {
        if (!h) fail(JSWEEP_E_INVALID_ARG, "graph is NULL");
        G(h)->profile = enable != 0;
        return JSWEEP_OK;
    });
}

int jsweep_profile_read(jsweep_graph h, int32_t reset, int64_t *launches, double *total_ms) {
    return guarded([&]() -> int {
        if (!h) fail(JSWEEP_E_INVALID_ARG, "graph is NULL");
        Graph &g = *G(h);
        double ms = 0.0;
        for (auto &e : g.prof_events) {
            JSW_HIP(hipEventSynchronize(e.second));
            float t = 0.0f;
            JSW_HIP(hipEventElapsedTime(&t, e.first, e.second));
            ms += t;
        }
        if (launches) *launches = (int64_t)g.prof_events.size();
        if (total_ms) *total_ms = ms;
        if (reset) {
            for (auto &e : g.prof_events) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
            g.prof_events.clear();
        }
        return JSWEEP_OK;
    });
}

int jsweep_trace(jsweep_graph h, int32_t enable) {
    return guarded([&]() -> int {
        if (!h) fail(JSWEEP_E_INVALID_ARG, "graph is NULL");
        Graph &g = *G(h);
        g.trace = enable != 0;
        if (g.trace && g.trace_buf.bytes < 12 * (size_t)std::max<int64_t>(1, g.n_chunks)) {
            g.trace_buf.alloc(12 * (size_t)std::max<int64_t>(1, g.n_chunks));
            JSW_HIP(hipMemset(g.trace_buf.p, 0, g.trace_buf.bytes));
        }
        return JSWEEP_OK;
    });
}

int jsweep_trace_read(jsweep_graph h, int64_t *n_chunks, uint32_t *stamps, int32_t *chunk_info, int32_t *deps_ptr,
                      int32_t *deps) {
    return guarded([&]() -> int {
        if (!h) fail(JSWEEP_E_INVALID_ARG, "graph is NULL");
        Graph &g = *G(h);
        JSW_HIP(hipDeviceSynchronize());
        if (g.trace_units == 1) {
            // the last traced sweep ran the patch kernel: units are its tasks
            const int64_t nt = g.pp.n_tasks;
            if (n_chunks) *n_chunks = nt;
            if (stamps) JSW_HIP(hipMemcpy(stamps, g.trace_buf.p, 12 * (size_t)nt, hipMemcpyDeviceToHost));
            std::vector<int32_t> desc;
            if (chunk_info || deps_ptr) {
                desc.resize(kPatchDesc * (size_t)nt);
                JSW_HIP(hipMemcpy(desc.data(), g.pp.desc.p, 4 * desc.size(), hipMemcpyDeviceToHost));
            }
            if (chunk_info)
                for (int64_t t = 0; t < nt; ++t) {
                    chunk_info[3 * t] = desc[kPatchDesc * t + 1];
                    chunk_info[3 * t + 1] = desc[kPatchDesc * t + 2];
                    chunk_info[3 * t + 2] = desc[kPatchDesc * t + 3];
                }
            if (deps_ptr) {
                deps_ptr[0] = 0;
                for (int64_t t = 0; t < nt; ++t) deps_ptr[t + 1] = deps_ptr[t] + desc[kPatchDesc * t + 7];
            }
            if (deps && g.pp.n_dep) JSW_HIP(hipMemcpy(deps, g.pp.dep.p, 4 * (size_t)g.pp.n_dep, hipMemcpyDeviceToHost));
            return JSWEEP_OK;
        }
        if (n_chunks) *n_chunks = g.n_chunks;
        if (stamps) {
            if (!g.trace_buf.p) fail(JSWEEP_E_INVALID_ARG, "tracing was never enabled");
            JSW_HIP(hipMemcpy(stamps, g.trace_buf.p, 12 * (size_t)g.n_chunks, hipMemcpyDeviceToHost));
        }
        if (chunk_info) {
            std::vector<Chunk> ch(g.n_chunks);
            JSW_HIP(hipMemcpy(ch.data(), g.chunks.p, sizeof(Chunk) * g.n_chunks, hipMemcpyDeviceToHost));
            for (int64_t c = 0; c < g.n_chunks; ++c) {
                int m = (int)(ch[c].a & 0xffffu);
                chunk_info[3 * c] = m;
                chunk_info[3 * c + 1] = (int32_t)(ch[c].a >> 16) + 1;
                // level of the chunk: position in the direction's level pointers
                const int64_t *p = g.lvl_ptr_h.data() + g.lvl_off_h[m];
                chunk_info[3 * c + 2] = (int32_t)(std::upper_bound(p, p + g.nlev_h[m] + 1, (int64_t)ch[c].b) - p - 1);
            }
        }
        if (deps_ptr) JSW_HIP(hipMemcpy(deps_ptr, g.dep_ptr.p, 4 * (size_t)(g.n_chunks + 1), hipMemcpyDeviceToHost));
        if (deps) JSW_HIP(hipMemcpy(deps, g.dep.p, 4 * (size_t)g.n_dep, hipMemcpyDeviceToHost));
        return JSWEEP_OK;
    });
}

void jsweep_graph_destroy(jsweep_graph h) {
    if (!h) return;
    try {
        union_forget(G(h)->uid);
        delete G(h);
    } catch (...) {
    }
}

const char *jsweep_error_string(int code) {
    switch (code) {
    case JSWEEP_OK: return "success";
    case JSWEEP_E_INVALID_ARG: return "invalid argument";
    case JSWEEP_E_MESH: return "invalid mesh";
    case JSWEEP_E_QUADRATURE: return "invalid quadrature";
    case JSWEEP_E_CYCLE: return "dependency cycle (lagging disabled)";
    case JSWEEP_E_DEVICE: return "device error";
    case JSWEEP_E_OOM: return "out of memory";
    case JSWEEP_E_STALLED: return "sweep stalled (watchdog)";
    case JSWEEP_E_NOT_CONVERGED: return "not converged";
    case JSWEEP_E_PLACEMENT: return "sweep workgroup on another XCD than its stream";
    default: return "unknown error";
    }
}

const char *jsweep_last_error(void) { return t_last_error.c_str(); }

}  // extern "C"
