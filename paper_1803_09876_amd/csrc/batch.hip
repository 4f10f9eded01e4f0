// Batched source iteration over an ensemble of independent graphs, and the
// launch-parameter autotuner.
//
// Every sweep of the batch is one launch of the batched direction-parallel
// kernel (one workgroup per (instance, direction) task).  The FP64 residual,
// scalar flux, correction flux and refinement update run as single
// launches over the concatenated cells (or angular fluxes) of all
// instances.  Instances converge independently: a device flag per instance
// switches its work off.  In the FP32-refined mode the inner correction
// sweeps are recorded once into a HIP graph (lag snapshot, sweep, scalar
// correction flux -- kInnerBlock of them) and replayed.
#include <cstring>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <string>

#include "common.hpp"
#include "device.hpp"

namespace jsw {

constexpr int kB = 256;
constexpr int kInnerBlock = 2;   // inner sweeps per graph replay (the granularity of the inner stop)
// the batched solve's default sweeps the union of all work lists in one
// data-driven launch while at least this fraction of the cell-angle updates
// is still iterating (a union sweep walks every chunk), the direction
// kernels after that
constexpr double kUnionMinActive = 0.5;
// outer residual reduction an FP32 correction solve reliably achieves
constexpr double kFp32Floor = 4e-6;

struct BInst {
    const void *rec64;
    void *rec32;
    const double *omega, *w, *vol;
    const double *sigma_t, *sigma_s, *q;
    double *phi, *psi, *src, *dphi;
    float *r32, *dpsi, *g32;
    const uint64_t *lag_mv;
    const int32_t *lag_u;
    const int32_t *posi;
    const int32_t *lvl;      // [nd*nc] level-ordered cells (position -> cell)
    double *sig_last;                    // sigma_t of the last denominator build
    const double *lag_a;                 // |Omega . S| of the lagged faces
    double wsum;                         // sum of the weights
    double *lag64;
    float *lag32;
    void *vsu;                           // batched data-driven sweep: the instance's V s (FP64 or FP32)
                                         // (FP32) in the union's per-cell array, else null
    void *lagu;                          // and its lagged values in the union's array (FP64 / FP32), else null
    int64_t n_lag, nc;
    int32_t nd, ctype;
    double psi_b;
};

// instance of a global index in a concatenation (off: n + 1 prefix sums).
// The indices of a wavefront's lanes ascend with the lane, so the search is
// done once, wave-uniformly, for the first active lane's index, and every
// lane then steps over the (few) instance boundaries between the two.
__device__ inline int find_inst(const int64_t *off, int n, int64_t g) {
    const uint64_t gu = (uint64_t)g;
    const int64_t g0 = (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(gu >> 32)) << 32) |
                                 (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)gu));
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (off[mid] <= g0) lo = mid;
        else hi = mid;
    }
    while (lo + 1 < n && off[lo + 1] <= g) ++lo;
    return lo;
}

// acc[4 i + slot] += v for every lane of a wavefront (i < 0: nothing).  The
// lanes that share the first lane's instance are summed in registers and
// added with one atomic; lanes past an instance boundary add their own.
// Every lane of the wavefront must call it.
__device__ inline void acc_add(double *acc, int i, int slot, double v) {
    const int i0 = __builtin_amdgcn_readfirstlane(i);
    const bool mine = i == i0;
    double x = mine ? v : 0.0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x = x + __shfl_xor(x, off, 64);
    if ((threadIdx.x & 63) == 0 && i0 >= 0) atomicAdd(acc + 4 * i0 + slot, x);
    if (!mine && i >= 0) atomicAdd(acc + 4 * i + slot, v);
}

// sigma_t V into every instance's records (FP32 copies too); flags the
// instances whose sigma_t differs from the one their denominators were
// built for, keeping the new values
__global__ void k_b_sigma(const BInst *I, const int64_t *coff, int n, int64_t total, int32_t *changed) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int i = find_inst(coff, n, g);
    const BInst &b = I[i];
    const int64_t K = g - coff[i];
    const double st = b.sigma_t[K];
    if (__double_as_longlong(st) != __double_as_longlong(b.sig_last[K])) {
        b.sig_last[K] = st;
        changed[i] = 1;
    }
    if (b.ctype == JSWEEP_TRI) {
        auto *r64 = (CellRec<double, 3, 2> *)b.rec64 + K;
        double v = st * r64->V;
        r64->sigV = v;
        if (b.rec32) ((CellRec<float, 3, 2> *)b.rec32 + K)->sigV = (float)v;
    } else if (b.ctype == JSWEEP_TET) {
        auto *r64 = (CellRec<double, 4, 3> *)b.rec64 + K;
        double v = st * r64->V;
        r64->sigV = v;
        if (b.rec32) ((CellRec<float, 4, 3> *)b.rec32 + K)->sigV = (float)v;
    } else {
        auto *r64 = (CellRec<double, 6, 3> *)b.rec64 + K;
        double v = st * r64->V;
        r64->sigV = v;
        if (b.rec32) ((CellRec<float, 6, 3> *)b.rec32 + K)->sigV = (float)v;
    }
}

__global__ void k_b_zero(const BInst *I, const int64_t *off, int n, int64_t total, const int32_t *active, int what) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int i = find_inst(off, n, g);
    if (active && !active[i]) return;
    const BInst &b = I[i];
    const int64_t x = g - off[i];
    if (what == 0) b.psi[x] = 0.0;
    else {
        // 1: a correction solve; 2: the first solve from a zero iterate,
        // whose source is q itself (no per-direction part)
        b.dpsi[x] = 0.0f;
        if (what == 2) b.r32[x] = 0.0f;
        if (x < b.nc) {
            b.dphi[x] = 0.0;
            const double src = what == 2 ? b.q[x] : 0.0;
            b.g32[x] = (float)src;
            if (b.vsu) static_cast<float *>(b.vsu)[x] = (float)(b.vol[x] * src);
        }
    }
}

// ||q||^2 of every instance into acc[4 i + 1]
__global__ void k_b_qnorm(const BInst *I, const int64_t *coff, int n, int64_t total, double *acc) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int i = -1;
    double v = 0.0;
    if (g < total) {
        i = find_inst(coff, n, g);
        const BInst &b = I[i];
        const int64_t K = g - coff[i];
        v = b.vol[K] * (b.q[K] * b.q[K]);
    }
    acc_add(acc, i, 1, v);
}

__global__ void k_b_source(const BInst *I, const int64_t *coff, int n, int64_t total, const int32_t *active) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int i = find_inst(coff, n, g);
    if (!active[i]) return;
    const BInst &b = I[i];
    const int64_t K = g - coff[i];
    const double src = b.q[K] + b.sigma_s[K] * b.phi[K];
    b.src[K] = src;
    if (b.vsu) static_cast<double *>(b.vsu)[K] = b.vol[K] * src;
}

// an instance's FP64 flux of direction m, cell K: in its cell-order row, or
// (upos given) at its level position in the union's last level-position
// array, whose instance i entries start at aoff[i]
__device__ inline double b_flux(const BInst &b, const double *upos, int64_t base, int64_t m, int64_t K) {
    return upos ? upos[base + m * b.nc + b.posi[m * b.nc + K]] : b.psi[m * b.nc + K];
}

__global__ void k_b_lag(const BInst *I, const int64_t *loff, int n, int64_t total, const int32_t *active, int fp32,
                        const double *upos, const int64_t *aoff) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int i = find_inst(loff, n, g);
    if (!active[i]) return;
    const BInst &b = I[i];
    const int64_t e = g - loff[i];
    const int64_t m = (int64_t)(b.lag_mv[e] >> 32);
    if (fp32) {
        const float v = b.dpsi[m * b.nc + b.lag_u[e]];
        b.lag32[e] = v;
        if (b.lagu) static_cast<float *>(b.lagu)[e] = v;
    } else {
        const double v = b_flux(b, upos, upos ? aoff[i] : 0, m, b.lag_u[e]);
        b.lag64[e] = v;
        if (b.lagu) static_cast<double *>(b.lagu)[e] = v;
    }
}

// FP64 residual of every active instance; acc[4 i] += ||r||^2, acc[4 i + 1] += ||q||^2
__global__ void k_b_residual(const BInst *I, const int64_t *coff, int n, int64_t total, const int32_t *active,
                             int fp32, double *acc) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int i = g < total ? find_inst(coff, n, g) : -1;
    if (i >= 0 && !active[i]) i = -1;
    double rr = 0.0, qq = 0.0;
    if (i >= 0) {
        const BInst &b = I[i];
        const int64_t K = g - coff[i];
        // FP32 copy of r in cell order, in the correction buffer (free until
        // the correction solve); k_b_level_order puts it in level order
        float *r32 = fp32 ? b.dpsi : nullptr;
        double V;
        if (b.ctype == JSWEEP_TRI) {
            const CellRec<double, 3, 2> r = ((const CellRec<double, 3, 2> *)b.rec64)[K];
            rr = residual_cell(r, K, b.omega, b.w, b.psi, b.q[K], b.sigma_s[K], b.psi_b, b.nc, b.nd, b.phi, r32, nullptr);
            V = r.V;
        } else if (b.ctype == JSWEEP_TET) {
            const CellRec<double, 4, 3> r = ((const CellRec<double, 4, 3> *)b.rec64)[K];
            rr = residual_cell(r, K, b.omega, b.w, b.psi, b.q[K], b.sigma_s[K], b.psi_b, b.nc, b.nd, b.phi, r32, nullptr);
            V = r.V;
        } else {
            const CellRec<double, 6, 3> r = ((const CellRec<double, 6, 3> *)b.rec64)[K];
            rr = residual_cell(r, K, b.omega, b.w, b.psi, b.q[K], b.sigma_s[K], b.psi_b, b.nc, b.nd, b.phi, r32, nullptr);
            V = r.V;
        }
        qq = V * (b.q[K] * b.q[K]);
    }
    acc_add(acc, i, 0, rr);
    acc_add(acc, i, 1, qq);
}

// r of every active instance in level-position order from its cell-order
// copy: r32[m nc + p] = dpsi[m nc + lvl[m nc + p]]
__global__ void k_b_level_order(const BInst *I, const int64_t *aoff, int n, int64_t total, const int32_t *active) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int i = find_inst(aoff, n, g);
    if (!active[i]) return;
    const BInst &b = I[i];
    const int64_t x = g - aoff[i];
    const int64_t m = x / b.nc;
    b.r32[x] = b.dpsi[m * b.nc + b.lvl[x]];
}

// Residual of a plain FP64 source iteration from the sweep identity (as in
// the single-graph solve): phi' (ascending m), d = sigma_s (phi' - phi),
// acc[4 i] += W V d^2, acc[4 i + 1] += V q^2; then the lagged-edge terms.
// (upos: the fluxes are read at their level positions, see b_flux)
__global__ void k_b_phi_delta(const BInst *I, const int64_t *coff, int n, int64_t total, const int32_t *active,
                              double *acc, const double *upos, const int64_t *aoff) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int i = g < total ? find_inst(coff, n, g) : -1;
    if (i >= 0 && !active[i]) i = -1;
    double rr = 0.0, qq = 0.0;
    if (i >= 0) {
        const BInst &b = I[i];
        const int64_t K = g - coff[i];
        const double s = upos ? dir_sum_pos(b.w, upos + aoff[i], b.posi, b.nc, b.nd, K) : dir_sum(b.w, b.psi, b.nc, b.nd, K);
        const double d = b.sigma_s[K] * (s - b.phi[K]);
        b.phi[K] = s;
        b.dphi[K] = d;
        rr = b.wsum * (b.vol[K] * (d * d));
        qq = b.vol[K] * (b.q[K] * b.q[K]);
    }
    acc_add(acc, i, 0, rr);
    acc_add(acc, i, 1, qq);
}

// one thread per (direction, downwind cell) group of an instance's lagged
// edges: w_m V ((d + l)^2 - d^2) with l = sum a (psi'_u - psi_u) / V
__global__ void k_b_lag_residual(const BInst *I, const int64_t *loff, int n, int64_t total, const int32_t *active,
                                 double *acc, const double *upos, const int64_t *aoff) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int i = g < total ? find_inst(loff, n, g) : -1;
    if (i >= 0 && !active[i]) i = -1;
    double rr = 0.0;
    if (i >= 0) {
        const BInst &b = I[i];
        const int64_t e = g - loff[i];
        if (e == 0 || b.lag_mv[e - 1] != b.lag_mv[e]) {
            const uint64_t key = b.lag_mv[e];
            const int64_t m = (int64_t)(key >> 32), v = (int64_t)(key & 0xffffffffu);
            double l = 0.0;
            for (int64_t f = e; f < b.n_lag && b.lag_mv[f] == key; ++f)
                l = l + b.lag_a[f] * (b_flux(b, upos, upos ? aoff[i] : 0, m, b.lag_u[f]) - b.lag64[f]) / b.vol[v];
            const double d = b.dphi[v];
            rr = b.w[m] * (b.vol[v] * ((d + l) * (d + l) - d * d));
        }
    }
    acc_add(acc, i, 0, rr);
}

// correction flux dphi (FP64 sum of FP32 fluxes), FP32 scattering source,
// acc[4 i + 2] += ||dphi||^2, acc[4 i + 3] += ||sigma_s (dphi - dphi_prev)||^2
// (the correction equation's residual, as in the single-graph solve)
__global__ void k_b_dphi(const BInst *I, const int64_t *coff, int n, int64_t total, const int32_t *active,
                         const int32_t *with_q, double *acc) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int i = g < total ? find_inst(coff, n, g) : -1;
    if (i >= 0 && !active[i]) i = -1;
    double ss = 0.0, dd = 0.0;
    if (i >= 0) {
        const BInst &b = I[i];
        const int64_t K = g - coff[i];
        const double s = dir_sum(b.w, b.dpsi, b.nc, b.nd, K);
        const double old = b.dphi[K];
        b.dphi[K] = s;
        const double src = with_q[i] ? b.q[K] + b.sigma_s[K] * s : b.sigma_s[K] * s;
        b.g32[K] = (float)src;
        if (b.vsu) static_cast<float *>(b.vsu)[K] = (float)(b.vol[K] * src);
        ss = b.vol[K] * (s * s);
        const double d = b.sigma_s[K] * (s - old);
        dd = b.vol[K] * (d * d);
    }
    acc_add(acc, i, 2, ss);
    acc_add(acc, i, 3, dd);
}

__global__ void k_b_update(const BInst *I, const int64_t *aoff, int n, int64_t total, const int32_t *active) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int i = find_inst(aoff, n, g);
    if (!active[i]) return;
    const BInst &b = I[i];
    const int64_t x = g - aoff[i];
    b.psi[x] = b.psi[x] + (double)b.dpsi[x];
}

// the cell-order fluxes of the flagged instances from the union's last
// level-position array: psi[m nc + K] = upos[aoff[i] + m nc + posi[m nc + K]]
__global__ void k_b_cell_order(const BInst *I, const int64_t *aoff, int n, int64_t total, const int32_t *flag,
                               const double *upos) {
    int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int i = find_inst(aoff, n, g);
    if (!flag[i]) return;
    const BInst &b = I[i];
    const int64_t x = g - aoff[i];
    b.psi[x] = upos[aoff[i] + (x / b.nc) * b.nc + b.posi[x]];
}

__global__ void k_b_clear(double *acc, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) acc[i] = 0.0;
}

static void ensure(DevBuf &b, size_t bytes) {
    if (b.bytes < bytes) b.alloc(bytes);
}

static unsigned grid_for(int64_t total) { return (unsigned)std::max<int64_t>(1, ceil_div(total, kB)); }

int solve_batch(int32_t n, Graph *const *graphs, const jsweep_problem *problems, int32_t mode, double tol,
                int32_t max_iter, const jsweep_params *params, jsweep_solve_stats *stats, hipStream_t user_s) {
    auto t_start = std::chrono::steady_clock::now();
    // the batch runs on a stream of its own (the legacy default stream
    // cannot be captured into a graph), after the caller's stream's work
    JSW_HIP(hipStreamSynchronize(user_s));
    hipStream_t s = nullptr;
    JSW_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() { (void)hipStreamSynchronize(s); (void)hipStreamDestroy(s); }
    } stream_guard{s};
    const bool refined = (mode & 0xff) == JSWEEP_FP32_REFINED;
    std::vector<BInst> h(n);
    std::vector<int64_t> coff(n + 1, 0), aoff(n + 1, 0), loff(n + 1, 0);
    std::vector<const void *> src_cell(n);
    std::vector<const float *> src_dir(n);
    std::vector<void *> psi_sweep(n);
    std::vector<double> psi_b(n);
    for (int i = 0; i < n; ++i) {
        Graph &g = *graphs[i];
        const jsweep_problem &p = problems[i];
        const int64_t N = g.nc * g.nd;
        if (refined) build_rec32(g, s);
        BInst &b = h[i];
        b.rec64 = g.rec64.p;
        b.rec32 = refined ? g.rec32.p : nullptr;
        b.omega = g.omega64.as<double>();
        b.w = g.weight.as<double>();
        b.vol = g.vol.as<double>();
        b.sigma_t = p.sigma_t;
        b.sigma_s = p.sigma_s;
        b.q = p.q;
        b.phi = p.phi;
        if (p.psi) b.psi = p.psi;
        else { ensure(g.scratch_a, 8 * N); b.psi = g.scratch_a.as<double>(); }
        ensure(g.scratch_b, 8 * g.nc + 64);
        b.src = g.scratch_b.as<double>();
        if (refined) {
            ensure(g.scratch_c, 8 * N + 64);
            b.r32 = g.scratch_c.as<float>();
            b.dpsi = b.r32 + N;
            ensure(g.scratch_d, 16 * g.nc + 64);
            b.dphi = g.scratch_d.as<double>();
            b.g32 = reinterpret_cast<float *>(b.dphi + g.nc);
        } else {
            b.r32 = b.dpsi = b.g32 = nullptr;
            ensure(g.scratch_d, 8 * g.nc + 64);
            b.dphi = g.scratch_d.as<double>();   // sigma_s (phi' - phi) of the last iteration
        }
        b.lag_mv = g.lag_mv.as<uint64_t>();
        b.lag_u = g.lag_u.as<int32_t>();
        b.posi = g.posi.as<int32_t>();
        b.lvl = g.lvl_cells.as<int32_t>();
        if (!g.sig_last.p) {
            g.sig_last.alloc(8 * g.nc + 64);
            g.den64_ok = g.den32_ok = false;
        }
        b.sig_last = g.sig_last.as<double>();
        b.lag_a = g.lag_a.as<double>();
        b.wsum = 0.0;
        for (double x : g.weight_h) b.wsum += x;
        b.lag64 = g.lag_val64.as<double>();
        b.lag32 = g.lag_val32.as<float>();
        b.vsu = nullptr;
        b.lagu = nullptr;
        b.n_lag = g.n_lag;
        b.nc = g.nc;
        b.nd = g.nd;
        b.ctype = g.ctype;
        b.psi_b = p.psi_boundary;
        coff[i + 1] = coff[i] + g.nc;
        aoff[i + 1] = aoff[i] + N;
        loff[i + 1] = loff[i] + g.n_lag;
        if (refined) { src_cell[i] = b.g32; src_dir[i] = b.r32; psi_sweep[i] = b.dpsi; psi_b[i] = 0.0; }
        else { src_cell[i] = b.src; src_dir[i] = nullptr; psi_sweep[i] = b.psi; psi_b[i] = p.psi_boundary; }
    }
    DevBuf d_inst(sizeof(BInst) * n), d_coff(8 * (n + 1)), d_aoff(8 * (n + 1)), d_loff(8 * (n + 1));
    DevBuf d_active(4 * n), d_all(4 * n), d_acc(8 * 4 * n);
    JSW_HIP(hipMemcpyAsync(d_inst.p, h.data(), sizeof(BInst) * n, hipMemcpyHostToDevice, s));
    JSW_HIP(hipMemcpyAsync(d_coff.p, coff.data(), 8 * (n + 1), hipMemcpyHostToDevice, s));
    JSW_HIP(hipMemcpyAsync(d_aoff.p, aoff.data(), 8 * (n + 1), hipMemcpyHostToDevice, s));
    JSW_HIP(hipMemcpyAsync(d_loff.p, loff.data(), 8 * (n + 1), hipMemcpyHostToDevice, s));
    std::vector<int32_t> active(n, 1), inner_active(n, 1);
    JSW_HIP(hipMemcpyAsync(d_all.p, active.data(), 4 * n, hipMemcpyHostToDevice, s));
    const BInst *I = d_inst.as<BInst>();
    const int64_t C = coff[n], A = aoff[n], LG = loff[n];
    int threads = (params && params->waves_per_block > 0) ? 64 * params->waves_per_block : 256;
    // sigma_t V in the records of every instance and the sweep-program
    // denominators, rebuilt only where sigma_t changed (one kernel and one
    // read-back for the whole batch)
    {
        DevBuf d_changed(4 * n);
        JSW_HIP(hipMemsetAsync(d_changed.p, 0, 4 * n, s));
        k_b_sigma<<<grid_for(C), kB, 0, s>>>(I, d_coff.as<int64_t>(), n, C, d_changed.as<int32_t>());
        JSW_HIP(hipGetLastError());
        std::vector<int32_t> changed(n);
        JSW_HIP(hipMemcpyAsync(changed.data(), d_changed.p, 4 * n, hipMemcpyDeviceToHost, s));
        JSW_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < n; ++i) {
            if (changed[i]) graphs[i]->den64_ok = graphs[i]->den32_ok = graphs[i]->pp.den64_ok = false;
            ensure_den(*graphs[i], refined, s);
        }
    }
    // The sweep of every instance and direction.  DATA_DRIVEN: one launch
    // of the data-driven kernel over the union of the instances' work lists
    // (the chunks of converged instances are still walked, only to empty
    // their entries).  DIRECTION, DIRECTION_LDS: the batched direction
    // kernels (a converged instance's tasks return at once).  AUTO (the
    // default): the union launch, over a list compacted to the instances
    // still iterating each time their cell-angle updates fall below
    // kUnionMinActive of the list's (so at most half of the listed work
    // is ever walked in vain).
    const int strategy = params ? params->strategy : 0;
    const bool compacting = strategy == JSWEEP_STRATEGY_AUTO || strategy == JSWEEP_STRATEGY_PATCH;
    const bool use_union = compacting || strategy == JSWEEP_STRATEGY_DATA_DRIVEN;
    const bool use_dir = !use_union;
    BatchSweep sweep;
    UnionSweep *un = nullptr;
    // FP64 through the union: the fluxes stay in the union's level-position
    // arrays (no cell-order copy per sweep); the flux pass and the lagged
    // values read them at their level positions, and an instance's fluxes
    // are copied to its cell-order psi when it stops (a later launch writes
    // markers over them)
    const bool lo64 = use_union && !refined;
    if (use_union) {
        un = &union_for(n, graphs, refined, s);
        un->refresh_den(graphs, s);
        std::vector<void *> rows_psi(psi_sweep);
        if (lo64) std::fill(rows_psi.begin(), rows_psi.end(), nullptr);
        un->set_rows(graphs, rows_psi.data(), src_dir.data(), psi_b.data(), s);
        for (int i = 0; i < n; ++i) {
            BInst &b = h[i];
            b.vsu = static_cast<char *>(un->vs.p) + (refined ? 4 : 8) * (size_t)un->coff[i];
            b.lagu = static_cast<char *>(un->lag.p) + (refined ? 4 : 8) * (size_t)un->loff[i];
        }
        JSW_HIP(hipMemcpyAsync(d_inst.p, h.data(), sizeof(BInst) * n, hipMemcpyHostToDevice, s));
        JSW_HIP(hipStreamSynchronize(s));
    }
    if (use_dir)
        sweep.setup(n, graphs, refined, src_cell.data(), src_dir.data(), psi_sweep.data(), psi_b.data(),
                    threads, strategy, s);
    const int wpb = (params && params->waves_per_block > 0) ? params->waves_per_block : 0;
    std::vector<double> work(n);
    double all_work = 0.0;
    for (int i = 0; i < n; ++i) all_work += (work[i] = (double)graphs[i]->nc * graphs[i]->nd);
    // work of the instances in the union's current list
    double listed_work = all_work;
    DevBuf d_cflags(4 * n);   // the instances a compaction keeps (d_active stays the outer set)
    // compacts the union's list when its active work has halved; true
    // when it did (a recorded union launch then refers to the old list)
    auto maybe_compact = [&](const std::vector<int32_t> &act) {
        if (!un || !compacting) return false;
        double w = 0.0;
        for (int i = 0; i < n; ++i) w += act[i] ? work[i] : 0.0;
        if (w <= 0.0 || w >= kUnionMinActive * listed_work) return false;
        JSW_HIP(hipMemcpyAsync(d_cflags.p, act.data(), 4 * n, hipMemcpyHostToDevice, s));
        un->compact(d_cflags.as<int32_t>(), s);
        listed_work = w;
        return true;
    };
    auto launch_sweep = [&](const int32_t *act) {
        if (un) un->launch(act, wpb, s);
        else sweep.launch(act, s);
    };
    k_b_zero<<<grid_for(A), kB, 0, s>>>(I, d_aoff.as<int64_t>(), n, A, nullptr, 0);
    JSW_HIP(hipGetLastError());

    std::vector<int32_t> outer(n, 0), sweeps(n, 0), hist(n, 0);
    std::vector<double> rho(n, INFINITY), acc(4 * n), qnorm(n, 1.0), wsum(n, 0.0);
    for (int i = 0; i < n; ++i)
        for (double x : graphs[i]->weight_h) wsum[i] += x;
    auto record = [&](int i, double v) {
        if (stats && stats[i].residual_history && hist[i] < stats[i].history_capacity) stats[i].residual_history[hist[i]] = v;
        ++hist[i];
    };
    auto residuals = [&]() {
        k_b_clear<<<grid_for(4 * n), kB, 0, s>>>(d_acc.as<double>(), 4 * n);
        k_b_residual<<<grid_for(C), kB, 0, s>>>(I, d_coff.as<int64_t>(), n, C, d_active.as<int32_t>(), refined ? 1 : 0,
                                                d_acc.as<double>());
        JSW_HIP(hipGetLastError());
        if (refined) {
            k_b_level_order<<<grid_for(A), kB, 0, s>>>(I, d_aoff.as<int64_t>(), n, A, d_active.as<int32_t>());
            JSW_HIP(hipGetLastError());
        }
        JSW_HIP(hipMemcpyAsync(acc.data(), d_acc.p, 8 * 4 * n, hipMemcpyDeviceToHost, s));
        JSW_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < n; ++i) {
            if (!active[i]) continue;
            qnorm[i] = acc[4 * i + 1] > 0.0 ? std::sqrt(acc[4 * i + 1]) : 1.0;
            rho[i] = acc[4 * i + 1] > 0.0 ? std::sqrt(acc[4 * i]) / std::sqrt(acc[4 * i + 1]) : std::sqrt(acc[4 * i]);
            ++outer[i];
            record(i, rho[i]);
        }
    };
    auto push_active = [&](const std::vector<int32_t> &v) {
        JSW_HIP(hipMemcpyAsync(d_active.p, v.data(), 4 * n, hipMemcpyHostToDevice, s));
    };
    push_active(active);
    int rc = JSWEEP_OK;
    int total_sweeps = 0;
    if (!refined) {
        // phi of the zero iterate is zero; plain source iteration
        JSW_HIP(hipMemsetAsync(d_acc.p, 0, 8 * 4 * n, s));
        for (int i = 0; i < n; ++i) JSW_HIP(hipMemsetAsync(h[i].phi, 0, 8 * graphs[i]->nc, s));
        // level-order fluxes (lo64): the last union launch's array (null
        // before the first: the lagged values then come from the zero psi),
        // and the instances whose fluxes go to their cell-order psi
        const double *upos = nullptr;
        DevBuf d_copy(4 * n);
        std::vector<int32_t> copy(n, 0);
        auto copy_out = [&]() {
            bool anyc = false;
            for (int i = 0; i < n; ++i) anyc = anyc || copy[i];
            if (!anyc || !upos) return;
            JSW_HIP(hipMemcpyAsync(d_copy.p, copy.data(), 4 * n, hipMemcpyHostToDevice, s));
            k_b_cell_order<<<grid_for(A), kB, 0, s>>>(I, d_aoff.as<int64_t>(), n, A, d_copy.as<int32_t>(), upos);
            JSW_HIP(hipGetLastError());
            JSW_HIP(hipStreamSynchronize(s));   // copy is host memory of this scope
        };
        while (true) {
            bool any = false;
            for (int i = 0; i < n; ++i) any = any || active[i];
            if (!any) break;
            if (total_sweeps >= max_iter) { rc = JSWEEP_E_NOT_CONVERGED; break; }
            k_b_source<<<grid_for(C), kB, 0, s>>>(I, d_coff.as<int64_t>(), n, C, d_active.as<int32_t>());
            if (LG)
                k_b_lag<<<grid_for(LG), kB, 0, s>>>(I, d_loff.as<int64_t>(), n, LG, d_active.as<int32_t>(), 0, upos,
                                                    d_aoff.as<int64_t>());
            launch_sweep(d_active.as<int32_t>());
            if (lo64) upos = static_cast<const double *>(un->last_pos());
            ++total_sweeps;
            for (int i = 0; i < n; ++i) sweeps[i] += active[i];
            // residual from the sweep identity (one pass over psi)
            k_b_clear<<<grid_for(4 * n), kB, 0, s>>>(d_acc.as<double>(), 4 * n);
            k_b_phi_delta<<<grid_for(C), kB, 0, s>>>(I, d_coff.as<int64_t>(), n, C, d_active.as<int32_t>(),
                                                     d_acc.as<double>(), upos, d_aoff.as<int64_t>());
            if (LG)
                k_b_lag_residual<<<grid_for(LG), kB, 0, s>>>(I, d_loff.as<int64_t>(), n, LG, d_active.as<int32_t>(),
                                                             d_acc.as<double>(), upos, d_aoff.as<int64_t>());
            JSW_HIP(hipGetLastError());
            JSW_HIP(hipMemcpyAsync(acc.data(), d_acc.p, 8 * 4 * n, hipMemcpyDeviceToHost, s));
            JSW_HIP(hipStreamSynchronize(s));
            if (un) {
                const int st = un->check_status(s);
                if (st != JSWEEP_OK) return st;
            }
            for (int i = 0; i < n; ++i) {
                copy[i] = 0;
                if (!active[i]) continue;
                const double rr = std::max(acc[4 * i], 0.0);
                rho[i] = acc[4 * i + 1] > 0.0 ? std::sqrt(rr) / std::sqrt(acc[4 * i + 1]) : std::sqrt(rr);
                ++outer[i];
                record(i, rho[i]);
                if (tol > 0.0 && rho[i] <= tol) {
                    active[i] = 0;
                    copy[i] = lo64 && problems[i].psi != nullptr;
                }
            }
            copy_out();
            push_active(active);
            maybe_compact(active);
        }
        // the instances still iterating at the end
        for (int i = 0; i < n; ++i) copy[i] = lo64 && active[i] && problems[i].psi != nullptr;
        copy_out();
    } else {
        const int J = (params && params->inner_sweeps > 0) ? params->inner_sweeps : 400;
        DevBuf d_inner(4 * n), d_withq(4 * n);
        std::vector<int32_t> withq(n, 0);
        // record kInnerBlock inner sweeps once; replay them per block.
        // The union sweep's level-position arrays alternate within the
        // recorded block (kInnerBlock is even); the first holds the marker
        // before recording.
        static_assert(kInnerBlock % 2 == 0, "the recorded block keeps the level-position arrays' alternation");
        // one recorded block of inner sweeps, recorded again whenever the
        // union's list is compacted
        hipGraph_t graph_rec = nullptr;
        hipGraphExec_t exec = nullptr;
        struct GraphGuard {
            hipGraph_t *g; hipGraphExec_t *e;
            void reset() {
                if (*e) (void)hipGraphExecDestroy(*e);
                if (*g) (void)hipGraphDestroy(*g);
                *e = nullptr;
                *g = nullptr;
            }
            ~GraphGuard() { reset(); }
        } guard{&graph_rec, &exec};
        auto record_block = [&]() {
            guard.reset();
            if (un) un->fill_current(s);
            JSW_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
            for (int k = 0; k < kInnerBlock; ++k) {
                if (LG)
                    k_b_lag<<<grid_for(LG), kB, 0, s>>>(I, d_loff.as<int64_t>(), n, LG, d_inner.as<int32_t>(), 1, nullptr,
                                                        nullptr);
                launch_sweep(d_inner.as<int32_t>());
                // the norms read back after a replay are those of its last pass
                if (k == kInnerBlock - 1) k_b_clear<<<grid_for(4 * n), kB, 0, s>>>(d_acc.as<double>(), 4 * n);
                k_b_dphi<<<grid_for(C), kB, 0, s>>>(I, d_coff.as<int64_t>(), n, C, d_inner.as<int32_t>(),
                                                    d_withq.as<int32_t>(), d_acc.as<double>());
            }
            hipError_t ce = hipStreamEndCapture(s, &graph_rec);
            if (ce != hipSuccess) JSW_HIP(ce);
            JSW_HIP(hipGraphInstantiate(&exec, graph_rec, nullptr, nullptr, 0));
        };
        record_block();
        std::vector<double> prev_pred(n, INFINITY), target(n, 0.0);
        // From the zero iterate with no boundary inflow the residual is q
        // itself (rho = 1): the first solve is source iteration on the
        // problem, with no operator application (as in the single-graph
        // solve).
        bool from_zero = true;
        for (int i = 0; i < n; ++i) from_zero = from_zero && problems[i].psi_boundary == 0.0;
        while (true) {
            if (from_zero) {
                k_b_clear<<<grid_for(4 * n), kB, 0, s>>>(d_acc.as<double>(), 4 * n);
                k_b_qnorm<<<grid_for(C), kB, 0, s>>>(I, d_coff.as<int64_t>(), n, C, d_acc.as<double>());
                JSW_HIP(hipGetLastError());
                JSW_HIP(hipMemcpyAsync(acc.data(), d_acc.p, 8 * 4 * n, hipMemcpyDeviceToHost, s));
                JSW_HIP(hipStreamSynchronize(s));
                for (int i = 0; i < n; ++i) {
                    qnorm[i] = acc[4 * i + 1] > 0.0 ? std::sqrt(acc[4 * i + 1]) : 1.0;
                    rho[i] = acc[4 * i + 1] > 0.0 ? 1.0 : 0.0;
                    ++outer[i];
                    record(i, rho[i]);
                }
            } else {
                residuals();
            }
            for (int i = 0; i < n; ++i)
                if (tol > 0.0 && active[i] && rho[i] <= tol) active[i] = 0;
            push_active(active);
            // each outer step starts from the list of the instances still
            // iterating; within it, the list follows the inner iterations'
            // own stops
            if (un && compacting && un->compacted) {
                un->expand();
                listed_work = all_work;
                maybe_compact(active);
                record_block();
            } else if (maybe_compact(active)) {
                record_block();
            }
            bool any = false;
            for (int i = 0; i < n; ++i) any = any || active[i];
            if (!any) break;
            if (total_sweeps >= max_iter) { rc = JSWEEP_E_NOT_CONVERGED; break; }
            // inner FP32 source iteration on the correction of every active instance
            k_b_zero<<<grid_for(A), kB, 0, s>>>(I, d_aoff.as<int64_t>(), n, A, d_active.as<int32_t>(), from_zero ? 2 : 1);
            JSW_HIP(hipGetLastError());
            std::fill(withq.begin(), withq.end(), from_zero ? 1 : 0);
            JSW_HIP(hipMemcpyAsync(d_withq.p, withq.data(), 4 * n, hipMemcpyHostToDevice, s));
            from_zero = false;
            inner_active = active;
            // inner stop as in the single-graph solve: the predicted outer
            // residual below half the tolerance, below the FP32 floor of the
            // current residual, or no longer improving close to that floor
            for (int i = 0; i < n; ++i) {
                prev_pred[i] = INFINITY;
                target[i] = std::max(0.5 * tol, kFp32Floor * rho[i]);
            }
            for (int j = 0; j < J && total_sweeps < max_iter; j += kInnerBlock) {
                JSW_HIP(hipMemcpyAsync(d_inner.p, inner_active.data(), 4 * n, hipMemcpyHostToDevice, s));
                JSW_HIP(hipGraphLaunch(exec, s));
                total_sweeps += kInnerBlock;
                JSW_HIP(hipMemcpyAsync(acc.data(), d_acc.p, 8 * 4 * n, hipMemcpyDeviceToHost, s));
                JSW_HIP(hipStreamSynchronize(s));
                if (un) {
                    const int st = un->check_status(s);
                    if (st != JSWEEP_OK) return st;
                }
                bool more = false;
                for (int i = 0; i < n; ++i) {
                    if (!inner_active[i]) continue;
                    sweeps[i] += kInnerBlock;
                    // norms of the block's last pass
                    const double norm = acc[4 * i + 2];
                    const double pred = std::sqrt(wsum[i] * acc[4 * i + 3]) / qnorm[i];
                    const bool stalled = j > 0 && pred > 0.9 * prev_pred[i] && pred < 100.0 * kFp32Floor * rho[i];
                    if (norm == 0.0 || pred <= target[i] || stalled) inner_active[i] = 0;
                    else more = true;
                    prev_pred[i] = pred;
                }
                if (!more) break;
                if (maybe_compact(inner_active)) record_block();
            }
            k_b_update<<<grid_for(A), kB, 0, s>>>(I, d_aoff.as<int64_t>(), n, A, d_active.as<int32_t>());
            JSW_HIP(hipGetLastError());
        }
    }
    JSW_HIP(hipStreamSynchronize(s));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    for (int i = 0; i < n; ++i) {
        if (rho[i] > tol) rc = JSWEEP_E_NOT_CONVERGED;
        if (stats) {
            stats[i].outer_iters = outer[i];
            stats[i].sweeps = sweeps[i];
            stats[i].residual = rho[i];
            stats[i].seconds = secs;
            stats[i].lagged_edges = graphs[i]->n_lag;
            stats[i].max_levels = graphs[i]->max_levels;
            stats[i].history_len = std::min(hist[i], stats[i].history_capacity);
        }
    }
    return rc;
}

// ---------------------------------------------------------------------------
// autotuner: time candidate launch configurations of the sweep on scratch
// problem data and keep the fastest; results are cached in memory and, when
// JSWEEP_TUNE_CACHE names a file, in that JSON file.
// ---------------------------------------------------------------------------
static std::string tune_key(Graph *const *graphs, int32_t n, int32_t mode, const char *arch) {
    int64_t cells = 0;
    int dirs = 0, ct = 0;
    for (int i = 0; i < n; ++i) { cells += graphs[i]->nc; dirs = std::max(dirs, graphs[i]->nd); ct |= graphs[i]->ctype; }
    int bucket = 0;
    while ((1ll << bucket) < cells) ++bucket;
    char buf[160];
    std::snprintf(buf, sizeof buf, "%s/ct%d/cells2^%d/dirs%d/n%d/mode%d", arch, ct, bucket, dirs, n, mode & 0xff);
    return buf;
}

static std::map<std::string, jsweep_params> &tune_memory() {
    static std::map<std::string, jsweep_params> m;
    return m;
}

static bool cache_lookup(const std::string &key, jsweep_params *out) {
    auto &mem = tune_memory();
    auto it = mem.find(key);
    if (it != mem.end()) { *out = it->second; return true; }
    const char *path = std::getenv("JSWEEP_TUNE_CACHE");
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, f)) {
        char k[256];
        jsweep_params p{};
        if (std::sscanf(line, " \"%255[^\"]\": [%d, %d, %d, %d, %d]", k, &p.waves_per_block, &p.blocks_per_cu,
                        &p.inner_sweeps, &p.chunks_per_ticket, &p.strategy) == 6 && key == k) {
            *out = p;
            found = true;
        }
    }
    std::fclose(f);
    if (found) mem[key] = *out;
    return found;
}

static void cache_store(const std::string &key, const jsweep_params &p) {
    auto &mem = tune_memory();
    mem[key] = p;
    const char *path = std::getenv("JSWEEP_TUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "w");
    if (!f) return;
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (auto &kv : mem) {
        const jsweep_params &q = kv.second;
        std::fprintf(f, "  \"%s\": [%d, %d, %d, %d, %d]%s\n", kv.first.c_str(), q.waves_per_block, q.blocks_per_cu,
                     q.inner_sweeps, q.chunks_per_ticket, q.strategy, ++i < mem.size() ? "," : "");
    }
    std::fprintf(f, "}\n");
    std::fclose(f);
}

int autotune(int32_t n, Graph *const *graphs, int32_t mode, jsweep_params *out) {
    hipDeviceProp_t prop;
    JSW_HIP(hipGetDeviceProperties(&prop, graphs[0]->device));
    const std::string key = tune_key(graphs, n, mode, prop.gcnArchName);
    if (cache_lookup(key, out)) {
        for (int i = 0; i < n; ++i) { graphs[i]->tuned = *out; graphs[i]->has_tuned = true; }
        return JSWEEP_OK;
    }
    const bool fp32 = (mode & 0xff) == JSWEEP_FP32_REFINED;
    hipStream_t s = nullptr;
    // scratch problem: sigma_t = 1, source = 1, per graph
    std::vector<DevBuf> st(n), src(n), psi(n);
    std::vector<float *> src32(n);
    for (int i = 0; i < n; ++i) {
        Graph &g = *graphs[i];
        const int64_t N = g.nc * g.nd;
        st[i].alloc(8 * g.nc);
        src[i].alloc(8 * g.nc);
        psi[i].alloc((fp32 ? 4 : 8) * N);
        std::vector<double> ones(g.nc, 1.0);
        JSW_HIP(hipMemcpy(st[i].p, ones.data(), 8 * g.nc, hipMemcpyHostToDevice));
        if (fp32) {
            std::vector<float> f(g.nc, 1.0f);
            JSW_HIP(hipMemcpy(src[i].p, f.data(), 4 * g.nc, hipMemcpyHostToDevice));
        } else {
            JSW_HIP(hipMemcpy(src[i].p, ones.data(), 8 * g.nc, hipMemcpyHostToDevice));
        }
        refresh_sigma(g, st[i].as<double>(), fp32, s);
    }
    std::vector<jsweep_params> cands;
    const jsweep_params ring_probe{0, 0, 0, 0, JSWEEP_STRATEGY_DIRECTION_LDS, 0};
    if (n == 1) {
        // (waves per workgroup, workgroups per CU) x chunks per ticket,
        // around the defaults (5 waves and 1 chunk below a million chunks,
        // 8 waves and 3 chunks above)
        const int wb[6][2] = {{4, 1}, {5, 1}, {6, 1}, {8, 1}, {10, 1}, {4, 2}};
        for (const auto &w : wb)
            for (int grab : {1, 2, 3})
                cands.push_back(jsweep_params{w[0], w[1], 0, grab, JSWEEP_STRATEGY_DATA_DRIVEN, 0});
        for (int w : {4, 8, 16}) cands.push_back(jsweep_params{w, 0, 0, 0, JSWEEP_STRATEGY_DIRECTION, 0});
        if (sweep_strategy(*graphs[0], nullptr) == JSWEEP_STRATEGY_DIRECTION_LDS ||
            sweep_strategy(*graphs[0], &ring_probe) == JSWEEP_STRATEGY_DIRECTION_LDS)
            cands.push_back(ring_probe);
        // the patch-task kernel (FP64 sweeps only), where its program applies
        if (!fp32 && patch_ready(*graphs[0], s)) cands.push_back(jsweep_params{1, 0, 0, 0, JSWEEP_STRATEGY_PATCH, 0});
    } else {
        // the union of the instances' work lists in one data-driven launch,
        // and the batched direction kernels
        for (int w : {5, 6, 8, 10, 12}) cands.push_back(jsweep_params{w, 0, 0, 0, JSWEEP_STRATEGY_DATA_DRIVEN, 0});
        for (int w : {1, 2, 4, 8, 16}) cands.push_back(jsweep_params{w, 0, 0, 0, JSWEEP_STRATEGY_DIRECTION, 0});
        cands.push_back(ring_probe);
    }
    hipEvent_t e0, e1;
    JSW_HIP(hipEventCreate(&e0));
    JSW_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    jsweep_params best_p = cands[0];
    std::vector<int32_t> ones(n, 1);
    DevBuf d_active(4 * n);
    JSW_HIP(hipMemcpy(d_active.p, ones.data(), 4 * n, hipMemcpyHostToDevice));
    for (const jsweep_params &c : cands) {
        float ms = 0.0f;
        BatchSweep bs;
        UnionSweep *un = nullptr;
        if (n > 1) {
            std::vector<const void *> sc(n);
            std::vector<const float *> sd(n, nullptr);
            std::vector<void *> ps(n);
            std::vector<double> pb(n, 0.0);
            for (int i = 0; i < n; ++i) { sc[i] = src[i].p; ps[i] = psi[i].p; }
            if (c.strategy == JSWEEP_STRATEGY_DATA_DRIVEN) {
                un = &union_for(n, graphs, fp32, s);
                un->refresh_den(graphs, s);
                un->set_rows(graphs, ps.data(), sd.data(), pb.data(), s);
                // unit sources (V s = V, or {V, 1}) are as good as any for timing
                JSW_HIP(hipMemsetAsync(un->vs.p, 0, un->vs.bytes, s));
            } else {
                bs.setup(n, graphs, fp32, sc.data(), sd.data(), ps.data(), pb.data(), 64 * c.waves_per_block,
                         c.strategy, s);
            }
        }
        for (int rep = 0; rep < 3; ++rep) {
            JSW_HIP(hipEventRecord(e0, s));
            if (n == 1) {
                if (fp32) launch_sweep32(*graphs[0], nullptr, src[0].as<float>(), psi[0].as<float>(), &c, s);
                else launch_sweep64(*graphs[0], src[0].as<double>(), psi[0].as<double>(), 0.0, &c, s);
            } else if (un) {
                un->launch(d_active.as<int32_t>(), c.waves_per_block, s);
            } else {
                bs.launch(d_active.as<int32_t>(), s);
            }
            JSW_HIP(hipEventRecord(e1, s));
            JSW_HIP(hipEventSynchronize(e1));
            if (un) {
                const int st = un->check_status(s);
                if (st != JSWEEP_OK) fail(st, "batched sweep failed while tuning: " + std::string(jsweep_last_error()));
            }
            if (n == 1) {
                const int st = check_sweep_status(*graphs[0], s);
                if (st != JSWEEP_OK)
                    fail(st, "sweep failed while tuning (strategy " + std::to_string(c.strategy) + ", " +
                                 std::to_string(c.waves_per_block) + " waves per workgroup, " +
                                 std::to_string(c.blocks_per_cu) + " per CU, " + std::to_string(c.chunks_per_ticket) +
                                 " chunks per ticket, repetition " + std::to_string(rep) + "): " + jsweep_last_error());
            }
            float t = 0.0f;
            JSW_HIP(hipEventElapsedTime(&t, e0, e1));
            if (rep > 0) ms += t;
        }
        if (ms < best) { best = ms; best_p = c; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // for a batch the data-driven union is used through AUTO, which
    // compacts its list to the instances still iterating
    if (n > 1 && best_p.strategy == JSWEEP_STRATEGY_DATA_DRIVEN) best_p.strategy = JSWEEP_STRATEGY_AUTO;
    *out = best_p;
    cache_store(key, best_p);
    for (int i = 0; i < n; ++i) { graphs[i]->tuned = best_p; graphs[i]->has_tuned = true; }
    return JSWEEP_OK;
}

}  // namespace jsw
