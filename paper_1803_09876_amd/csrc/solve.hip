// Source iteration around the sweep (appendix algorithm "Source iterative
// Sn solver": update the scattering source, sweep every direction, reduce
// the error, repeat), in plain FP64 and as FP64 iterative refinement with
// FP32 correction sweeps.
#include <cstring>

#include <algorithm>
#include <chrono>
#include <cmath>

#include "common.hpp"
#include "device.hpp"

namespace jsw {

constexpr int kB = 256;
// outer residual reduction an FP32 correction solve reliably achieves
// (measured: 3e-6 to 1e-5 of the residual it corrects)
constexpr double kFp32Floor = 4e-6;

// sigma_t * V into the sweep records (FP64 product; FP32 records take it
// rounded)
template <int NF, int DIM>
__global__ void k_sigv(CellRec<double, NF, DIM> *r64, CellRec<float, NF, DIM> *r32, const double *sigma_t, int64_t nc) {
    int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (K >= nc) return;
    double v = sigma_t[K] * r64[K].V;
    r64[K].sigV = v;
    if (r32) r32[K].sigV = (float)v;
}

// flags a change of sigma_t since the last call (and keeps the new values)
__global__ void k_sig_changed(const double *sig, double *last, int64_t nc, int32_t *flag) {
    int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (K >= nc) return;
    const double v = sig[K];
    if (__double_as_longlong(v) != __double_as_longlong(last[K])) {
        last[K] = v;
        *flag = 1;
    }
}

// Sweep-program denominators, one per chunk lane: sigma_t V plus the
// outflow a_f in local face order (FP64; the FP32 copy sums the rounded
// terms in FP32).
template <int NF, int DIM, bool F32>
__global__ void k_den(const int32_t *blk, int64_t n_chunks, const CellRec<double, NF, DIM> *rec, const double *omega,
                      double *den64, float *den32) {
    const int64_t c = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= n_chunks) return;
    const int64_t idx = c * 64 + lane;
    const int32_t K = blk[c * kBlock + lane];
    if (K < 0) {
        if (F32) den32[idx] = 1.0f;
        else den64[idx] = 1.0;
        return;
    }
    const int m = (int)((uint32_t)blk[c * kBlock + 64] & 0xffffu);
    const CellRec<double, NF, DIM> r = rec[K];
    const double om[3] = {omega[3 * m], omega[3 * m + 1], omega[3 * m + 2]};
    double den = r.sigV;
    float den_f = (float)r.sigV;
    for (int j = 0; j < NF; ++j) {
        double d = om[0] * r.S[j][0] + om[1] * r.S[j][1];
        if constexpr (DIM == 3) d = d + om[2] * r.S[j][2];
        if (d > 0.0) {
            den = den + d;
            den_f = den_f + (float)d;
        }
    }
    if (F32) den32[idx] = den_f;
    else den64[idx] = den;
}

__global__ void k_narrow(const double *a, int64_t n, float *b) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

template <int NF, int DIM>
static void refresh_den(Graph &g, bool f32, hipStream_t s) {
    const int64_t nch = g.n_chunks;
    const unsigned gb = (unsigned)ceil_div(nch, 4);
    if (f32)
        k_den<NF, DIM, true><<<gb, 256, 0, s>>>(g.cblk.as<int32_t>(), nch, g.rec64.as<CellRec<double, NF, DIM>>(),
                                                g.omega64.as<double>(), nullptr, g.pden32.as<float>());
    else
        k_den<NF, DIM, false><<<gb, 256, 0, s>>>(g.cblk.as<int32_t>(), nch, g.rec64.as<CellRec<double, NF, DIM>>(),
                                                 g.omega64.as<double>(), g.pden64.as<double>(), nullptr);
    JSW_HIP(hipGetLastError());
}

void refresh_sigma(Graph &g, const double *sigma_t, bool fp32, hipStream_t s) {
    if (fp32) build_rec32(g, s);
    int gb = (int)ceil_div(g.nc, kB);
    void *r32 = fp32 ? g.rec32.p : nullptr;
    if (g.ctype == JSWEEP_TRI)
        k_sigv<3, 2><<<gb, kB, 0, s>>>(g.rec64.as<CellRec<double, 3, 2>>(), (CellRec<float, 3, 2> *)r32, sigma_t, g.nc);
    else if (g.ctype == JSWEEP_TET)
        k_sigv<4, 3><<<gb, kB, 0, s>>>(g.rec64.as<CellRec<double, 4, 3>>(), (CellRec<float, 4, 3> *)r32, sigma_t, g.nc);
    else
        k_sigv<6, 3><<<gb, kB, 0, s>>>(g.rec64.as<CellRec<double, 6, 3>>(), (CellRec<float, 6, 3> *)r32, sigma_t, g.nc);
    JSW_HIP(hipGetLastError());
    // sweep-program denominators: rebuilt only when sigma_t has changed
    if (!g.n_chunks) return;
    if (!g.sig_last.p) {
        g.sig_last.alloc(8 * g.nc + 64);
        g.den64_ok = g.den32_ok = false;
    }
    int32_t *flag = reinterpret_cast<int32_t *>(g.sig_last.as<char>() + 8 * g.nc);
    JSW_HIP(hipMemsetAsync(flag, 0, 4, s));
    k_sig_changed<<<gb, kB, 0, s>>>(sigma_t, g.sig_last.as<double>(), g.nc, flag);
    JSW_HIP(hipGetLastError());
    int32_t changed = 0;
    JSW_HIP(hipMemcpyAsync(&changed, flag, 4, hipMemcpyDeviceToHost, s));
    JSW_HIP(hipStreamSynchronize(s));
    if (changed) g.den64_ok = g.den32_ok = g.pp.den64_ok = false;
    ensure_den(g, fp32, s);
}

void ensure_den(Graph &g, bool fp32, hipStream_t s) {
    if (!g.n_chunks) return;
    auto run = [&](bool f32) {
        if (g.ctype == JSWEEP_TRI) refresh_den<3, 2>(g, f32, s);
        else if (g.ctype == JSWEEP_TET) refresh_den<4, 3>(g, f32, s);
        else refresh_den<6, 3>(g, f32, s);
    };
    if (!g.den64_ok) {
        run(false);
        g.den64_ok = true;
    }
    if (fp32 && !g.den32_ok) {
        const int64_t S = 64 * g.n_chunks;
        if (!g.pa32.p) {
            g.pa32.alloc(4 * (size_t)g.ns * S);
            k_narrow<<<(unsigned)ceil_div((int64_t)g.ns * S, kB), kB, 0, s>>>(g.pa64.as<double>(), (int64_t)g.ns * S,
                                                                            g.pa32.as<float>());
            JSW_HIP(hipGetLastError());
        }
        if (!g.pden32.p) g.pden32.alloc(4 * (size_t)S);
        run(true);
        g.den32_ok = true;
    }
}

// s_K = q_K + sigma_s,K phi_K
__global__ void k_source(const double *q, const double *sigma_s, const double *phi, int64_t nc, double *src) {
    int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (K < nc) src[K] = q[K] + sigma_s[K] * phi[K];
}

// phi_K = sum_m w_m psi_{K,m}, ascending m
__global__ void k_phi(const double *psi, const double *w, int64_t nc, int nd, double *phi) {
    int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (K >= nc) return;
    const double s = dir_sum(w, psi, nc, nd, K);
    phi[K] = s;
}

void scalar_flux(Graph &g, const double *psi, double *phi, hipStream_t s) {
    k_phi<<<(int)ceil_div(g.nc, kB), kB, 0, s>>>(psi, g.weight.as<double>(), g.nc, g.nd, phi);
    JSW_HIP(hipGetLastError());
}

// previous-iterate values on lagged edges (taken before a sweep overwrites)
template <class Real>
__global__ void k_lag_snapshot(const uint64_t *lag_mv, const int32_t *lag_u, int64_t n, const Real *psi, int64_t nc,
                               Real *val) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    int64_t m = (int64_t)(lag_mv[e] >> 32);
    val[e] = psi[m * nc + lag_u[e]];
}

template <class Real>
static void lag_snapshot(Graph &g, const Real *psi, hipStream_t s) {
    if (!g.n_lag) return;
    Real *val = sizeof(Real) == 8 ? (Real *)g.lag_val64.p : (Real *)g.lag_val32.p;
    k_lag_snapshot<Real><<<(int)ceil_div(g.n_lag, kB), kB, 0, s>>>(g.lag_mv.as<uint64_t>(), g.lag_u.as<int32_t>(),
                                                                  g.n_lag, psi, g.nc, val);
    JSW_HIP(hipGetLastError());
}

void lag_snapshot64(Graph &g, const double *psi, hipStream_t s) { lag_snapshot<double>(g, psi, s); }

// FP64 residual with the full (un-lagged) streaming operator, one cell per
// thread looping over directions (the cell record is read once per pass):
//   phi_K = sum_m w_m psi_{K,m}
//   r_{K,m} = q_K + sigma_s,K phi_K - (den psi_{K,m} - in_{K,m}) / V_K
// norms: acc[0] += V_K sum_m w_m r^2, acc[1] += V_K q_K^2.  Optionally stores
// r in FP32 (the correction-sweep source, in level-position order).
template <int NF, int DIM>
__global__ void k_residual(const CellRec<double, NF, DIM> *rec, const double *omega, const double *w, const double *psi,
                           const double *q, const double *sigma_s, double psi_b, int64_t nc, int nd, double *phi,
                           float *r32, const int32_t *posi, double *acc) {
    int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double rr = 0.0, qq = 0.0;
    if (K < nc) {
        const CellRec<double, NF, DIM> r = rec[K];
        rr = residual_cell(r, K, omega, w, psi, q[K], sigma_s[K], psi_b, nc, nd, phi, r32, posi);
        qq = r.V * (q[K] * q[K]);
    }
    block_add(rr, acc);
    block_add(qq, acc + 1);
}

// Lagged edges by downwind cell, for the residual kernels below.
struct LagCells {
    const int32_t *cptr;   // [nc + 1] groups of each cell
    const int32_t *cgrp;   // first edge of each (direction, cell) group
    const uint64_t *mv;    // [n] m << 32 | v, sorted
    const int32_t *u;      // [n] upwind cell
    const double *a;       // [n] |Omega . S| of the face
    double *val;           // [n] previous-iterate value on the edge
    int64_t n;
};

// Lagged in-edges of cell v: the un-lagged residual's extra term
// w_m V ((d + l)^2 - d^2) per direction m, l = sum a (psi_now - psi_prev) / V;
// the lagged values are replaced by the new iterate's for the next sweep
// (psi in cell order, or in level-position order when posi is given, its
// values masked by keep)
__device__ inline double lag_terms(const LagCells &L, const double *psi, const int32_t *posi, const double *w,
                                   int64_t nc, int64_t v, double V, double d, uint64_t keep) {
    double c = 0.0;
    for (int32_t gi = L.cptr[v]; gi < L.cptr[v + 1]; ++gi) {
        const int64_t e = L.cgrp[gi];
        const uint64_t key = L.mv[e];
        const int64_t m = (int64_t)(key >> 32);
        double l = 0.0;
        for (int64_t f = e; f < L.n && L.mv[f] == key; ++f) {
            const int64_t u = L.u[f];
            const double now = kept(psi[m * nc + (posi ? (int64_t)posi[m * nc + u] : u)], keep);
            l = l + L.a[f] * (now - L.val[f]) / V;
            L.val[f] = now;
        }
        c = c + w[m] * (V * ((d + l) * (d + l) - d * d));
    }
    return c;
}

// Set-up of the next sweep and status shared by the FP64 residual kernels:
// the sweep status next to the norms, zeroed next norms, stream tickets
__device__ inline void next_sweep_setup(int64_t t, const int32_t *status, double *acc, double *acc_next,
                                        uint32_t *tickets) {
    if (t == 0) acc[2] = (double)status[0];
    if (acc_next && t < 3) acc_next[t] = 0.0;
    if (t < kStreams) {
        tickets[32 * t] = 0u;
        tickets[32 * t + kXccSlot] = kNoXcc;
    }
}

// Residual of a plain FP64 source iteration without re-applying the
// operator.  The sweep solved, per vertex, den psi' - sum_in a psi'_up =
// V (q + sigma_s phi) with lagged faces on the previous iterate, so the
// un-lagged residual of psi' is exactly
//   r = sigma_s (phi' - phi) + sum over lagged in-faces a (psi'_u - psi_u) / V.
// k_phi_delta: phi' (ascending m), the isotropic part d = sigma_s (phi' -
// phi) and its norm W V d^2 (W = sum of the weights), and V q^2.  psi is
// the sweep's output in cell order, or (posi given) the level-ordered
// array the data-driven sweep filled, read through the level positions with
// only the bits in keep (see last_sweep_keep).
// The lagged in-faces of the cell add their terms (lag_terms), so that one
// kernel gives the whole residual norm.  It also prepares the next sweep:
// its source q + sigma_s phi', the product V s the sweep kernels read, the
// lagged values, zeroed next norms (acc_next, unless null) and tickets.
__global__ void k_phi_delta(const double *psi, const int32_t *posi, const double *w, double wsum, const double *q,
                            const double *sigma_s, const double *vol, int64_t nc, int nd, double *phi, double *acc,
                            double *src_next, double *vs_next, LagCells L, const int32_t *status, double *acc_next,
                            uint32_t *tickets, int64_t per_xcd, uint64_t keep) {
    const int64_t K = xcd_block(per_xcd) * blockDim.x + threadIdx.x;
    next_sweep_setup(K, status, acc, acc_next, tickets);
    double a = 0.0, b = 0.0;
    if (K < nc) {
        const double s = posi ? dir_sum_pos(w, psi, posi, nc, nd, K, keep) : dir_sum(w, psi, nc, nd, K);
        const double d = sigma_s[K] * (s - phi[K]);
        phi[K] = s;
        const double sn = q[K] + sigma_s[K] * s;
        src_next[K] = sn;
        vs_next[K] = vol[K] * sn;
        a = wsum * (vol[K] * (d * d));
        if (L.n > 0) a = a + lag_terms(L, psi, posi, w, nc, K, vol[K], d, keep);
        b = vol[K] * (q[K] * q[K]);
    }
    block_add(a, acc);
    block_add(b, acc + 1);
}

// k_phi_delta for two consecutive cells per thread (n_cells even), so that
// every direction's fluxes are read in 16-byte pieces; the same
// arithmetic per cell
__global__ void k_phi_delta2(const double *psi, const int32_t *posi, const double *w, double wsum, const double *q,
                             const double *sigma_s, const double *vol, int64_t nc, int nd, double *phi, double *acc,
                             double *src_next, double *vs_next, LagCells L, const int32_t *status, double *acc_next,
                             uint32_t *tickets, int64_t per_xcd, uint64_t keep) {
    const int64_t t = xcd_block(per_xcd) * blockDim.x + threadIdx.x;
    next_sweep_setup(t, status, acc, acc_next, tickets);
    const int64_t K = 2 * t;
    double a = 0.0, b = 0.0;
    if (K < nc) {
        double s[2];
        if (posi) dir_sum_pos2(w, psi, posi, nc, nd, K, s[0], s[1], keep);
        else dir_sum2(w, psi, nc, nd, K, s[0], s[1]);
        const double2 ph = *reinterpret_cast<const double2 *>(phi + K);
        const double2 ss = *reinterpret_cast<const double2 *>(sigma_s + K);
        const double2 qq = *reinterpret_cast<const double2 *>(q + K);
        const double2 vv = *reinterpret_cast<const double2 *>(vol + K);
        const double old[2] = {ph.x, ph.y}, sig[2] = {ss.x, ss.y}, qk[2] = {qq.x, qq.y}, vk[2] = {vv.x, vv.y};
        double d[2], sn[2];
        for (int i = 0; i < 2; ++i) {
            d[i] = sig[i] * (s[i] - old[i]);
            sn[i] = qk[i] + sig[i] * s[i];
            a = a + wsum * (vk[i] * (d[i] * d[i]));
            if (L.n > 0) a = a + lag_terms(L, psi, posi, w, nc, K + i, vk[i], d[i], keep);
            b = b + vk[i] * (qk[i] * qk[i]);
        }
        *reinterpret_cast<double2 *>(phi + K) = make_double2(s[0], s[1]);
        *reinterpret_cast<double2 *>(src_next + K) = make_double2(sn[0], sn[1]);
        *reinterpret_cast<double2 *>(vs_next + K) = make_double2(vk[0] * sn[0], vk[1] * sn[1]);
    }
    block_add(a, acc);
    block_add(b, acc + 1);
}

// ||q||^2 = sum_K V_K q_K^2
__global__ void k_qnorm(const double *q, const double *vol, int64_t nc, double *acc) {
    int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double a = 0.0;
    if (K < nc) a = vol[K] * (q[K] * q[K]);
    block_add(a, acc);
}

// delta-phi of a correction iterate (FP64 accumulation of FP32 fluxes), the
// FP32 scattering source sigma_s dphi for the next inner sweep, the
// V-weighted norm of dphi and that of sigma_s (dphi - dphi_prev): by the
// sweep identity the latter is the isotropic part of the correction
// equation's residual, i.e. of the outer residual once the correction is
// applied.  It also prepares the next inner sweep: the per-cell V s (one
// float, rounded from the FP64 product) the sweep kernel reads, the
// lagged-edge values of this iterate, zeroed
// accumulators (acc_next) and stream tickets.  CPT consecutive cells per
// thread (1, or 4 when n_cells is a multiple of 4 and dpsi 16-byte
// aligned: every direction's fluxes are then read in 16-byte pieces); each
// cell's sum over directions in ascending m either way.
// With posi (POS), dpsi is the level-ordered array the data-driven sweep
// filled and is read through the level positions (CPT 1 or 2).
template <int CPT, bool POS = false>
__global__ void k_dphi(const float *dpsi, const int32_t *posi, const double *w, const double *sigma_s,
                       const double *vol, int64_t nc, int nd, const double *q, double *dphi, float *g32,
                       const int32_t *status, double *acc, double *acc_next, float *vs, uint32_t *tickets,
                       const uint64_t *lag_mv, const int32_t *lag_u, int64_t n_lag, float *lag_val, int64_t per_xcd) {
    const int64_t t = xcd_block(per_xcd) * blockDim.x + threadIdx.x;
    if (t == 0) acc[2] = (double)status[0];
    if (t < 2) acc_next[t] = 0.0;
    if (t < kStreams) {
        tickets[32 * t] = 0u;
        tickets[32 * t + kXccSlot] = kNoXcc;
    }
    for (int64_t e = t; e < n_lag; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t m = (int64_t)(lag_mv[e] >> 32), u = lag_u[e];
        lag_val[e] = dpsi[m * nc + (POS ? (int64_t)posi[m * nc + u] : u)];
    }
    double a = 0.0, b = 0.0;
    const int64_t K0 = t * CPT;
    if (K0 < nc) {
        double sum[CPT];
        if constexpr (POS) {
            static_assert(CPT <= 2, "level-position gathers take one or two cells per thread");
            if constexpr (CPT == 1) sum[0] = dir_sum_pos(w, dpsi, posi, nc, nd, K0);
            else dir_sum_pos2(w, dpsi, posi, nc, nd, K0, sum[0], sum[1]);
        } else if constexpr (CPT == 1) {
            sum[0] = dir_sum(w, dpsi, nc, nd, K0);
        } else {
#pragma unroll
            for (int c = 0; c < CPT; ++c) sum[c] = 0.0;
            int m = 0;
            for (; m + 16 <= nd; m += 16) {
                float4 v[16];
#pragma unroll
                for (int k = 0; k < 16; ++k) v[k] = *reinterpret_cast<const float4 *>(dpsi + (int64_t)(m + k) * nc + K0);
#pragma unroll
                for (int k = 0; k < 16; ++k) {
                    const double wk = w[m + k];
                    sum[0] = sum[0] + wk * (double)v[k].x;
                    sum[1] = sum[1] + wk * (double)v[k].y;
                    sum[2] = sum[2] + wk * (double)v[k].z;
                    sum[3] = sum[3] + wk * (double)v[k].w;
                }
            }
            for (; m < nd; ++m) {
                const float4 v = *reinterpret_cast<const float4 *>(dpsi + (int64_t)m * nc + K0);
                const double wk = w[m];
                sum[0] = sum[0] + wk * (double)v.x;
                sum[1] = sum[1] + wk * (double)v.y;
                sum[2] = sum[2] + wk * (double)v.z;
                sum[3] = sum[3] + wk * (double)v.w;
            }
        }
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int64_t K = K0 + c;
            const double s = sum[c];
            const double old = dphi[K];
            dphi[K] = s;
            const double src = q ? q[K] + sigma_s[K] * s : sigma_s[K] * s;
            g32[K] = (float)src;
            vs[K] = (float)(vol[K] * src);
            a = a + vol[K] * (s * s);
            const double d = sigma_s[K] * (s - old);
            b = b + vol[K] * (d * d);
        }
    }
    block_add(a, acc);
    block_add(b, acc + 1);
}

// psi += dpsi (FP64); with posi, dpsi is in level-position order
__global__ void k_update(double *psi, const float *dpsi, const int32_t *posi, int64_t nc, int64_t n, int64_t per_xcd) {
    int64_t i = xcd_block(per_xcd) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t j = posi ? (i / nc) * nc + posi[i] : i;
    psi[i] = psi[i] + (double)dpsi[j];
}

// cell-order copy of level-ordered fluxes: psi[m nc + K] = pos[m nc + posi[m nc + K]]
// (the bits in keep)
__global__ void k_cell_order(const double *pos, const int32_t *posi, int64_t nc, int64_t n, double *psi,
                             int64_t per_xcd, uint64_t keep) {
    int64_t i = xcd_block(per_xcd) * blockDim.x + threadIdx.x;
    if (i < n) psi[i] = kept(pos[(i / nc) * nc + posi[i]], keep);
}

// r in level-position order from its cell-order copy:
//   r32[m nc + p] = rc[m nc + lvl_cells[m nc + p]].
// Workgroup b works on block (b mod 8) * per_xcd + b / 8, so each XCD takes
// one contiguous eighth of the entries and gathers every direction's
// cell-order values through its own L2.
__global__ void k_level_order(const float *rc, const int32_t *lvl_cells, int64_t nc, int64_t n, int64_t per_xcd,
                              float *r32) {
    const int64_t blk = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    const int64_t i = blk * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t m = i / nc;
    r32[i] = rc[m * nc + lvl_cells[i]];
}

// FP64 residual rho = ||r||_V / ||q||_V.  With r32, r is also stored in FP32
// in level-position order for the correction sweep: the residual kernel
// writes it in cell order into rc (n_cells * n_dirs floats, coalesced) and
// k_level_order permutes it, which costs far less than scattering 4-byte
// stores from the residual kernel.
static double residual(Graph &g, const double *psi, const double *q, const double *sigma_s, double psi_b, double *phi,
                       float *r32, float *rc, double *acc, hipStream_t s, double *qq = nullptr) {
    JSW_HIP(hipMemsetAsync(acc, 0, 16, s));
    int gb = (int)ceil_div(g.nc, kB);
    const double *om = g.omega64.as<double>(), *w = g.weight.as<double>();
    float *out = r32 ? rc : nullptr;
    if (g.ctype == JSWEEP_TRI)
        k_residual<3, 2><<<gb, kB, 0, s>>>(g.rec64.as<CellRec<double, 3, 2>>(), om, w, psi, q, sigma_s, psi_b, g.nc, g.nd, phi, out, nullptr, acc);
    else if (g.ctype == JSWEEP_TET)
        k_residual<4, 3><<<gb, kB, 0, s>>>(g.rec64.as<CellRec<double, 4, 3>>(), om, w, psi, q, sigma_s, psi_b, g.nc, g.nd, phi, out, nullptr, acc);
    else
        k_residual<6, 3><<<gb, kB, 0, s>>>(g.rec64.as<CellRec<double, 6, 3>>(), om, w, psi, q, sigma_s, psi_b, g.nc, g.nd, phi, out, nullptr, acc);
    JSW_HIP(hipGetLastError());
    const int64_t N = g.nc * g.nd;
    if (r32 && N > 0) {
        const int64_t per_xcd = ceil_div(ceil_div(N, kB), 8);
        k_level_order<<<(unsigned)(8 * per_xcd), kB, 0, s>>>(rc, g.lvl_cells.as<int32_t>(), g.nc, N, per_xcd, r32);
        JSW_HIP(hipGetLastError());
    }
    double h[2];
    JSW_HIP(hipMemcpyAsync(h, acc, 16, hipMemcpyDeviceToHost, s));
    JSW_HIP(hipStreamSynchronize(s));
    if (qq) *qq = h[1];
    return h[1] > 0.0 ? std::sqrt(h[0]) / std::sqrt(h[1]) : std::sqrt(h[0]);
}

static void ensure(DevBuf &b, size_t bytes) {
    if (b.bytes < bytes) b.alloc(bytes);
}

// sets *flag when an element has its sign bit set (a negative value or
// -0.0) or is NaN
__global__ void k_flag_negative(const double *x, int64_t n, int32_t *flag) {
    const int64_t step = (int64_t)gridDim.x * blockDim.x;
    bool neg = false;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
        const double v = x[i];
        neg = neg || !(v >= 0.0) || (__builtin_bit_cast(uint64_t, v) >> 63) != 0;
    }
    if (neg) atomicOr(flag, 1);
}

bool all_nonnegative(std::initializer_list<std::pair<const double *, int64_t>> arrays, hipStream_t s) {
    DevBuf flag(4);
    JSW_HIP(hipMemsetAsync(flag.p, 0, 4, s));
    for (const auto &x : arrays)
        if (x.first && x.second > 0) {
            k_flag_negative<<<(int)std::min<int64_t>(ceil_div(x.second, kB), 4096), kB, 0, s>>>(x.first, x.second,
                                                                                              flag.as<int32_t>());
            JSW_HIP(hipGetLastError());
        }
    int32_t h = 0;
    JSW_HIP(hipMemcpyAsync(&h, flag.p, 4, hipMemcpyDeviceToHost, s));
    JSW_HIP(hipStreamSynchronize(s));
    return h == 0;
}

int solve(Graph &g, const double *sigma_t, const double *sigma_s, const double *q, double psi_b, int32_t mode,
          double tol, int32_t max_iter, const jsweep_params *params, double *phi, double *psi_out,
          jsweep_solve_stats *stats, hipStream_t s) {
    auto t_start = std::chrono::steady_clock::now();
    if (params && params->priority && params->priority != g.priority) set_priority(g, params->priority, s);
    const bool refined = (mode & 0xff) == JSWEEP_FP32_REFINED;
    const bool warm = (mode & JSWEEP_WARM_START) != 0;
    const int64_t N = g.nc * g.nd;
    const bool zero_start = !warm || !psi_out;
    // With the data-driven kernel the sweeps keep their fluxes in level
    // order only (the graph's level-position arrays): the flux passes read
    // them through the level positions, and the caller's psi (cell order)
    // is written once at the end, so no sweep scatters a cell-order copy.
    // The FP64 source iteration then needs no cell-order psi at all until
    // that final copy; the FP32 refinement keeps psi (FP64, cell order) for
    // its residual and adds each correction to it through the positions.
    const bool lo = sweep_strategy(g, params) == JSWEEP_STRATEGY_DATA_DRIVEN;
    const bool need_psi = !lo || refined || (warm && psi_out);
    // scratch: psi (if the caller gives none), source / dphi, accumulators
    double *psi = nullptr;
    if (need_psi) {
        psi = psi_out;
        if (!psi) { ensure(g.scratch_a, 8 * N); psi = g.scratch_a.as<double>(); }
    }
    ensure(g.scratch_b, 8 * g.nc + 128);
    double *src = g.scratch_b.as<double>();
    double *acc = src + g.nc + 2;   // 16-byte aligned tail, 8 doubles
    if (((uintptr_t)acc & 15) != 0) acc += 1;
    if (zero_start && need_psi) JSW_HIP(hipMemsetAsync(psi, 0, 8 * N, s));
    refresh_sigma(g, sigma_t, refined, s);
    int outer = 0, sweeps = 0, hist = 0, rc = JSWEEP_OK;
    double rho = INFINITY;
    auto record = [&](double v) {
        if (stats && stats->residual_history && hist < stats->history_capacity) stats->residual_history[hist] = v;
        ++hist;
    };
    if (!refined) {
        // phi of the initial iterate
        if (zero_start && !need_psi) JSW_HIP(hipMemsetAsync(phi, 0, 8 * g.nc, s));
        else scalar_flux(g, psi, phi, s);
        double wsum = 0.0;
        for (double x : g.weight_h) wsum += x;
        const LagCells lagc{g.lag_cptr.as<int32_t>(), g.lag_cgrp.as<int32_t>(), g.lag_mv.as<uint64_t>(),
                            g.lag_u.as<int32_t>(), g.lag_a.as<double>(), g.lag_val64.as<double>(), g.n_lag};
        if (g.vsc.bytes < (size_t)(8 * g.nc)) g.vsc.alloc(8 * g.nc);
        uint32_t *tickets = reinterpret_cast<uint32_t *>(g.status.as<char>() + 128);
        // a fixed number of iterations (tol = 0) keeps every iteration's
        // norms on the device and reads them once at the end; otherwise two
        // accumulator sets alternate and are read after every sweep
        const bool fixed = !(tol > 0.0) && max_iter <= 65536;
        DevBuf norms(8 * 4 * (size_t)(fixed ? max_iter : 2));
        JSW_HIP(hipMemsetAsync(norms.p, 0, norms.bytes, s));
        // after the first sweep, the residual kernels prepare the next one
        // (source, V s, lagged values, tickets)
        bool prepared = false;
        // the flux pass takes two cells per thread when every array it
        // touches allows 16-byte accesses
        auto al16 = [](const void *p) { return ((uintptr_t)p & 15) == 0; };
        const bool pairs = g.nc % 2 == 0 && (lo || al16(psi)) && al16(phi) && al16(q) && al16(sigma_s) && al16(src) &&
                           al16(g.vol.p) && al16(g.vsc.p);
        const int32_t *posi = lo ? g.posi.as<int32_t>() : nullptr;
        // with every input non-negative (cross sections, source, boundary
        // inflow, the initial iterate) every flux of every sweep is, and the
        // data-driven sweeps tag their fluxes by sign.  Non-negative means
        // sign bit clear: a -0.0 input can make a flux -0.0, whose sign a
        // tagged store would not keep
        const bool nonneg = lo && psi_b >= 0.0 && !std::signbit(psi_b) &&
                            all_nonnegative({{sigma_t, g.nc}, {sigma_s, g.nc}, {q, g.nc}, {phi, g.nc},
                                             {g.n_lag ? psi : nullptr, N}}, s);
        while (true) {
            if (sweeps >= max_iter) { rc = JSWEEP_E_NOT_CONVERGED; break; }
            double *it_acc = norms.as<double>() + 4 * (fixed ? sweeps : (sweeps & 1));
            double *next_acc = fixed ? nullptr : norms.as<double>() + 4 * ((sweeps + 1) & 1);
            if (!prepared) {
                k_source<<<(int)ceil_div(g.nc, kB), kB, 0, s>>>(q, sigma_s, phi, g.nc, src);
                JSW_HIP(hipGetLastError());
                if (psi) lag_snapshot<double>(g, psi, s);
                else if (g.n_lag) JSW_HIP(hipMemsetAsync(g.lag_val64.p, 0, 8 * g.n_lag, s));
            }
            launch_sweep64(g, src, lo ? nullptr : psi, psi_b, params, s, prepared, nonneg);
            ++sweeps;
            // residual of the new iterate from the identity above (one
            // pass over the fluxes for phi; the lagged edges by their
            // downwind cells), and the set-up of the next sweep
            const double *flux = lo ? static_cast<const double *>(last_sweep_pos(g)) : psi;
            const uint64_t keep = lo ? last_sweep_keep(g) : ~0ull;
            const int64_t pxcd = xcd_per(ceil_div(pairs ? g.nc / 2 : g.nc, kB));
            if (pairs)
                k_phi_delta2<<<(unsigned)(8 * pxcd), kB, 0, s>>>(
                    flux, posi, g.weight.as<double>(), wsum, q, sigma_s, g.vol.as<double>(), g.nc, g.nd, phi, it_acc,
                    src, g.vsc.as<double>(), lagc, g.status.as<int32_t>(), next_acc, tickets, pxcd, keep);
            else
                k_phi_delta<<<(unsigned)(8 * pxcd), kB, 0, s>>>(
                    flux, posi, g.weight.as<double>(), wsum, q, sigma_s, g.vol.as<double>(), g.nc, g.nd, phi, it_acc,
                    src, g.vsc.as<double>(), lagc, g.status.as<int32_t>(), next_acc, tickets, pxcd, keep);
            JSW_HIP(hipGetLastError());
            prepared = true;
            if (fixed) continue;
            double h[3];
            JSW_HIP(hipMemcpyAsync(h, it_acc, 24, hipMemcpyDeviceToHost, s));
            JSW_HIP(hipStreamSynchronize(s));
            if (h[2] != 0.0) return check_sweep_status(g, s);
            rho = h[1] > 0.0 ? std::sqrt(std::max(h[0], 0.0)) / std::sqrt(h[1]) : std::sqrt(std::max(h[0], 0.0));
            ++outer;
            record(rho);
            if (rho <= tol) break;
        }
        if (fixed && sweeps > 0) {
            std::vector<double> h(4 * (size_t)sweeps);
            JSW_HIP(hipMemcpyAsync(h.data(), norms.p, 8 * h.size(), hipMemcpyDeviceToHost, s));
            JSW_HIP(hipStreamSynchronize(s));
            for (int k = 0; k < sweeps; ++k) {
                const double *x = h.data() + 4 * k;
                if (x[2] != 0.0) return check_sweep_status(g, s);
                rho = x[1] > 0.0 ? std::sqrt(std::max(x[0], 0.0)) / std::sqrt(x[1]) : std::sqrt(std::max(x[0], 0.0));
                ++outer;
                record(rho);
            }
        }
        // the caller's psi in cell order, once
        if (lo && psi_out && sweeps > 0) {
            const int64_t pxcd = xcd_per(ceil_div(N, kB));
            k_cell_order<<<(unsigned)(8 * pxcd), kB, 0, s>>>(static_cast<const double *>(last_sweep_pos(g)),
                                                            g.posi.as<int32_t>(), g.nc, N, psi_out, pxcd,
                                                            last_sweep_keep(g));
            JSW_HIP(hipGetLastError());
        }
    } else {
        ensure(g.scratch_c, 4 * N * 2 + 64);            // r32 and dpsi32
        float *r32 = g.scratch_c.as<float>();
        float *dpsi = r32 + N;
        ensure(g.scratch_d, 16 * g.nc + 64);           // dphi (double), g32 (float)
        double *dphi = g.scratch_d.as<double>();
        float *g32 = reinterpret_cast<float *>(dphi + g.nc);
        int J = (params && params->inner_sweeps > 0) ? params->inner_sweeps
                : (g.has_tuned && g.tuned.inner_sweeps > 0 ? g.tuned.inner_sweeps : 400);
        double wsum = 0.0;
        for (double x : g.weight_h) wsum += x;
        while (true) {
            // From a zero iterate with no boundary inflow the residual is
            // q itself (rho = 1), and the first correction solve is source
            // iteration on the problem itself: isotropic source q + sigma_s
            // dphi, no per-direction part, no operator application needed.
            const bool from_zero = outer == 0 && zero_start && psi_b == 0.0;
            double qq = 0.0;
            if (from_zero) {
                JSW_HIP(hipMemsetAsync(acc, 0, 8, s));
                k_qnorm<<<(int)ceil_div(g.nc, kB), kB, 0, s>>>(q, g.vol.as<double>(), g.nc, acc);
                JSW_HIP(hipGetLastError());
                JSW_HIP(hipMemcpyAsync(&qq, acc, 8, hipMemcpyDeviceToHost, s));
                JSW_HIP(hipStreamSynchronize(s));
                rho = qq > 0.0 ? 1.0 : 0.0;
            } else {
                rho = residual(g, psi, q, sigma_s, psi_b, phi, r32, dpsi, acc, s, &qq);   // dpsi is free until the inner solve
            }
            const double qn = qq > 0.0 ? std::sqrt(qq) : 1.0;
            ++outer;
            record(rho);
            if (tol > 0.0 && rho <= tol) break;
            if (sweeps >= max_iter) { rc = JSWEEP_E_NOT_CONVERGED; break; }
            // inner source iteration on the correction in FP32 (from zero)
            if (!lo) JSW_HIP(hipMemsetAsync(dpsi, 0, 4 * N, s));
            JSW_HIP(hipMemsetAsync(dphi, 0, 8 * g.nc, s));
            if (from_zero) {
                k_narrow<<<(int)ceil_div(g.nc, kB), kB, 0, s>>>(q, g.nc, g32);
                JSW_HIP(hipGetLastError());
            } else {
                JSW_HIP(hipMemsetAsync(g32, 0, 4 * g.nc, s));
            }
            // Inner stop: the outer residual the correction leaves behind is
            // predicted after every inner sweep from the correction
            // equation's residual (isotropic part; lagged faces left out)
            // and the inner loop stops once it is below half the tolerance,
            // or below what FP32 corrections resolve (a few 1e-6 of the
            // current residual), or stops improving close to that floor.
            // The outer loop then measures the true residual.
            const double target = std::max(0.5 * tol, kFp32Floor * rho);
            double prev_pred = INFINITY;
            int inner = 0;
            // the first inner sweep is set up here; each later one by the
            // k_dphi of the sweep before it (two accumulator sets alternate)
            if (g.vsc.bytes < (size_t)(8 * g.nc)) g.vsc.alloc(8 * g.nc);
            uint32_t *tickets = reinterpret_cast<uint32_t *>(g.status.as<char>() + 128);
            const bool quads = g.nc % 4 == 0 && ((uintptr_t)dpsi & 15) == 0;
            const int32_t *posi = lo ? g.posi.as<int32_t>() : nullptr;
            for (int j = 0; j < J && sweeps < max_iter; ++j) {
                double *a_cur = acc + 2 + 3 * (j & 1), *a_next = acc + 2 + 3 * ((j + 1) & 1);
                if (j == 0) {
                    if (lo) {
                        if (g.n_lag) JSW_HIP(hipMemsetAsync(g.lag_val32.p, 0, 4 * g.n_lag, s));
                    } else {
                        lag_snapshot<float>(g, dpsi, s);
                    }
                    JSW_HIP(hipMemsetAsync(a_cur, 0, 16, s));
                }
                launch_sweep32(g, from_zero ? nullptr : r32, g32, lo ? nullptr : dpsi, params, s, j > 0);
                ++sweeps;
                ++inner;
                const float *dflux = lo ? static_cast<const float *>(last_sweep_pos(g)) : dpsi;
                const int cpt = lo ? (g.nc % 2 == 0 ? 2 : 1) : (quads ? 4 : 1);
                auto dphi_kernel = lo ? (cpt == 2 ? k_dphi<2, true> : k_dphi<1, true>) : (quads ? k_dphi<4> : k_dphi<1>);
                const int64_t pxcd = xcd_per(ceil_div(g.nc, kB * cpt));
                dphi_kernel<<<(unsigned)(8 * pxcd), kB, 0, s>>>(
                    dflux, posi, g.weight.as<double>(), sigma_s, g.vol.as<double>(), g.nc, g.nd,
                    from_zero ? q : nullptr, dphi, g32, g.status.as<int32_t>(), a_cur, a_next, g.vsc.as<float>(),
                    tickets, g.lag_mv.as<uint64_t>(), g.lag_u.as<int32_t>(), g.n_lag, g.lag_val32.as<float>(), pxcd);
                JSW_HIP(hipGetLastError());
                double h[3];   // norm of dphi, correction residual, sweep status
                JSW_HIP(hipMemcpyAsync(h, a_cur, 24, hipMemcpyDeviceToHost, s));
                JSW_HIP(hipStreamSynchronize(s));
                if (h[2] != 0.0) return check_sweep_status(g, s);
                const double pred = std::sqrt(wsum * h[1]) / qn;
                if (h[0] == 0.0 || pred <= target) break;
                // stalled near the FP32 floor (slow contraction far above it
                // is ordinary source iteration and continues)
                if (j > 0 && pred > 0.9 * prev_pred && pred < 100.0 * kFp32Floor * rho) break;
                prev_pred = pred;
            }
            const int64_t pxcd = xcd_per(ceil_div(N, kB));
            if (lo) {
                if (inner > 0)
                    k_update<<<(unsigned)(8 * pxcd), kB, 0, s>>>(psi, static_cast<const float *>(last_sweep_pos(g)),
                                                                g.posi.as<int32_t>(), g.nc, N, pxcd);
            } else k_update<<<(unsigned)(8 * pxcd), kB, 0, s>>>(psi, dpsi, nullptr, g.nc, N, pxcd);
            JSW_HIP(hipGetLastError());
        }
    }
    JSW_HIP(hipStreamSynchronize(s));
    if (stats) {
        stats->outer_iters = outer;
        stats->sweeps = sweeps;
        stats->residual = rho;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        stats->lagged_edges = g.n_lag;
        stats->max_levels = g.max_levels;
        stats->history_len = std::min(hist, stats->history_capacity);
    }
    return rc;
}

}  // namespace jsw
