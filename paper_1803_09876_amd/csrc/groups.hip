// Multigroup source iteration (the appendix form of the transport
// equation: a flux per ordinate and energy group, collisions coupling every
// group into every other through an isotropic group-to-group scattering
// cross section; appendix algorithm "Source iterative Sn solver": step 2.1
// updates the scattering source and the coupling terms, step 2.2 sweeps
// every angle and every energy, step 2.3 reduces the error).
//
// Jacobi over groups: every group's source comes from the previous iterate
// of all groups, so the sweeps of every (direction, group) are independent
// and run in one launch of the data-driven kernel.  The groups share the
// sweep graph and its program (geometry and directions do not depend on the
// energy); each group has its own denominators (sigma_t,g), source and
// fluxes.  Layouts: sigma_t, q, phi [G][nc]; sigma_s [G][G][nc] with the
// cross section from g' into g at (g' G + g) nc + K; psi [G][nd][nc].
// Inside the solve the sweep's level-position fluxes, the lagged values and
// V s keep the groups of one entry adjacent (entry e of group g at e G + g):
// a face's upwind fluxes of every group are one memory segment.
#include <cstring>

#include <algorithm>
#include <chrono>
#include <cmath>

#include "common.hpp"
#include "device.hpp"

namespace jsw {

namespace {

constexpr int kB = 256;

// Denominators of every group, one per chunk lane: sigma_t,g V plus the
// outflow a_f in local face order.
template <int NF, int DIM>
__global__ void k_den_groups(const int32_t *blk, int64_t n_chunks, const CellRec<double, NF, DIM> *rec,
                             const double *omega, const double *sigma_t, int64_t nc, int G, double *den) {
    const int64_t c = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (c >= n_chunks) return;
    const int64_t S = 64 * n_chunks, idx = c * 64 + lane;
    const int32_t K = blk[c * kBlock + lane];
    if (K < 0) {
        for (int g = 0; g < G; ++g) den[g * S + idx] = 1.0;
        return;
    }
    const int m = (int)((uint32_t)blk[c * kBlock + 64] & 0xffffu);
    const CellRec<double, NF, DIM> r = rec[K];
    const double om[3] = {omega[3 * m], omega[3 * m + 1], omega[3 * m + 2]};
    double out_a[NF];
#pragma unroll
    for (int j = 0; j < NF; ++j) {
        double d = om[0] * r.S[j][0] + om[1] * r.S[j][1];
        if constexpr (DIM == 3) d = d + om[2] * r.S[j][2];
        out_a[j] = d;
    }
    for (int g = 0; g < G; ++g) {
        double d = sigma_t[g * nc + K] * r.V;
#pragma unroll
        for (int j = 0; j < NF; ++j)
            if (out_a[j] > 0.0) d = d + out_a[j];
        den[g * S + idx] = d;
    }
}

// Group sources s_{K,g} = q_{K,g} + sum over g' (ascending) of
// sigma_s,g'->g,K phi_{K,g'}, and V s for the sweep at K G + g; also zeroes
// the stream tickets of the sweep that follows.
__global__ void k_group_source(const double *q, const double *sigma_s, const double *phi, const double *vol,
                               int64_t nc, int G, double *vs, uint32_t *tickets) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < kStreams) {
        tickets[32 * t] = 0u;
        tickets[32 * t + kXccSlot] = kNoXcc;
    }
    if (t >= nc * G) return;
    const int64_t K = t / G;
    const int g = (int)(t - K * G);
    double v = q[(int64_t)g * nc + K];
    for (int gp = 0; gp < G; ++gp) v = v + sigma_s[((int64_t)gp * G + g) * nc + K] * phi[(int64_t)gp * nc + K];
    vs[t] = vol[K] * v;
}

// previous-iterate values on the lagged edges of every group, edge e of
// group g at e G + g
__global__ void k_group_lag_snapshot(const uint64_t *lag_mv, const int32_t *lag_u, int64_t n_lag, int G,
                                     const double *psi, int64_t nc, int64_t N, double *val) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_lag * G) return;
    const int64_t e = t / G, g = t - e * G;
    val[t] = psi[g * N + (int64_t)(lag_mv[e] >> 32) * nc + lag_u[e]];
}

// phi_{K,g} = sum_m w_m psi_{K,m,g}, ascending m
__global__ void k_group_phi(const double *psi, const double *w, int64_t nc, int nd, int G, double *phi) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nc * G) return;
    const int64_t g = t / nc, K = t - g * nc;
    phi[t] = dir_sum(w, psi + g * nc * nd, nc, nd, K);
}

// Residual of the multigroup equations with the full (un-lagged) streaming
// operator, one (group, cell) per thread over every direction:
//   r_{K,m,g} = s_{K,g} - (den_g psi_{K,m,g} - in_{K,m,g}) / V_K
// with s from the new phi of every group; norms acc[0] += V_K sum_m w_m r^2,
// acc[1] += V_K q_{K,g}^2.
template <int NF, int DIM>
__global__ void k_group_residual(const CellRec<double, NF, DIM> *rec, const double *omega, const double *w,
                                 const double *psi, const double *q, const double *sigma_s, const double *sigma_t,
                                 const double *phi, double psi_b, int64_t nc, int nd, int G, double *acc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double rr = 0.0, qq = 0.0;
    if (t < nc * G) {
        const int g = (int)(t / nc);
        const int64_t K = t - (int64_t)g * nc;
        const CellRec<double, NF, DIM> r = rec[K];
        double src = q[t];
        for (int gp = 0; gp < G; ++gp) src = src + sigma_s[((int64_t)gp * G + g) * nc + K] * phi[(int64_t)gp * nc + K];
        int64_t nb[NF];
#pragma unroll
        for (int j = 0; j < NF; ++j) nb[j] = r.nbr[j] <= -2 ? -(int64_t)r.nbr[j] - 2 : (int64_t)r.nbr[j];
        const double *pg = psi + (int64_t)g * nd * nc;
        const double sv = sigma_t[t] * r.V;
        double cell = 0.0;
        for (int m = 0; m < nd; ++m) {
            const double *om = omega + 3 * m;
            const double *pm = pg + (int64_t)m * nc;
            double in = 0.0, den = sv;
#pragma unroll
            for (int j = 0; j < NF; ++j) {
                double d = om[0] * r.S[j][0] + om[1] * r.S[j][1];
                if constexpr (DIM == 3) d = d + om[2] * r.S[j][2];
                if (d < 0.0) in = in + (-d) * (nb[j] < 0 ? psi_b : pm[nb[j]]);
                else if (d > 0.0) den = den + d;
            }
            const double res = src - (den * pm[K] - in) / r.V;
            cell = cell + w[m] * (res * res);
        }
        rr = r.V * cell;
        qq = r.V * (q[t] * q[t]);
    }
    block_add(rr, acc);
    block_add(qq, acc + 1);
}

// the G values of one level-position entry (groups adjacent; 16-byte
// aligned when G is even)
template <int G>
__device__ __forceinline__ void load_groups(const double *e, double (&v)[G]) {
    if constexpr (G % 2 == 0) {
#pragma unroll
        for (int h = 0; h < G / 2; ++h) {
            const double2 x = reinterpret_cast<const double2 *>(e)[h];
            v[2 * h] = x.x;
            v[2 * h + 1] = x.y;
        }
    } else {
#pragma unroll
        for (int g = 0; g < G; ++g) v[g] = e[g];
    }
}

// Graphs without lagged edges keep every group's fluxes in level order for
// the whole solve (as the single-group solve does).  First every group's
// new phi, one cell per thread: phi'_{K,g} = sum_m w_m psi at entry
// (m nc + posi[m nc + K]) G + g, each group's sum in ascending m; a
// direction's position is read once for all groups and the groups' fluxes
// are one segment (each read with the bits in keep, see last_sweep_keep).
// Then, per cell, the residual from the identity the
// sweep satisfies, which without lagged faces is isotropic:
//   r_{K,g} = sum over g' (ascending) of sigma_s,g'->g,K (phi'_{K,g'} - phi_{K,g'}),
// acc[0] += (sum_m w_m) V_K r^2 and acc[1] += V_K q_{K,g}^2 over the
// groups; phi then takes the new iterate.
template <int G>
__global__ void k_group_phi_pos(const double *pos, const int32_t *posi, const double *w, int64_t nc, int nd,
                                double *phin, int64_t per_xcd, uint64_t keep) {
    // each XCD takes a contiguous range of cells, so its gathers share its own L2
    const int64_t K = xcd_block(per_xcd) * blockDim.x + threadIdx.x;
    if (K >= nc) return;
    constexpr int B = G <= 2 ? 16 : G <= 4 ? 8 : 4;   // directions per batch
    double s[G];
#pragma unroll
    for (int g = 0; g < G; ++g) s[g] = 0.0;
    int32_t p[B];
    int m = 0;
    if (B <= nd) {
#pragma unroll
        for (int k = 0; k < B; ++k) p[k] = posi[(int64_t)k * nc + K];
    }
    for (; m + B <= nd; m += B) {
        double v[B][G];
#pragma unroll
        for (int k = 0; k < B; ++k) load_groups<G>(pos + ((int64_t)(m + k) * nc + p[k]) * G, v[k]);
        // the next batch's positions travel while these fluxes do
        if (m + 2 * B <= nd) {
#pragma unroll
            for (int k = 0; k < B; ++k) p[k] = posi[(int64_t)(m + B + k) * nc + K];
        }
        // masked only here, after the next positions' loads have been issued
#pragma unroll
        for (int k = 0; k < B; ++k)
#pragma unroll
            for (int g = 0; g < G; ++g) s[g] = s[g] + w[m + k] * kept(v[k][g], keep);
    }
    for (; m < nd; ++m) {
        double v[G];
        load_groups<G>(pos + ((int64_t)m * nc + posi[(int64_t)m * nc + K]) * G, v);
#pragma unroll
        for (int g = 0; g < G; ++g) s[g] = s[g] + w[m] * kept(v[g], keep);
    }
#pragma unroll
    for (int g = 0; g < G; ++g) phin[(int64_t)g * nc + K] = s[g];
}

template <int G>
void launch_group_phi_pos(const double *pos, const int32_t *posi, const double *w, int64_t nc, int nd, double *phin,
                          uint64_t keep, hipStream_t s) {
    const int64_t pxcd = xcd_per(ceil_div(nc, kB));
    k_group_phi_pos<G><<<(unsigned)(8 * pxcd), kB, 0, s>>>(pos, posi, w, nc, nd, phin, pxcd, keep);
    JSW_HIP(hipGetLastError());
}

void group_phi_pos(int G, const double *pos, const int32_t *posi, const double *w, int64_t nc, int nd, double *phin,
                   uint64_t keep, hipStream_t s) {
    static_assert(kMaxGroups == 8, "group_phi_pos is instantiated for 1 - 8 groups");
    switch (G) {
    case 1: launch_group_phi_pos<1>(pos, posi, w, nc, nd, phin, keep, s); break;
    case 2: launch_group_phi_pos<2>(pos, posi, w, nc, nd, phin, keep, s); break;
    case 3: launch_group_phi_pos<3>(pos, posi, w, nc, nd, phin, keep, s); break;
    case 4: launch_group_phi_pos<4>(pos, posi, w, nc, nd, phin, keep, s); break;
    case 5: launch_group_phi_pos<5>(pos, posi, w, nc, nd, phin, keep, s); break;
    case 6: launch_group_phi_pos<6>(pos, posi, w, nc, nd, phin, keep, s); break;
    case 7: launch_group_phi_pos<7>(pos, posi, w, nc, nd, phin, keep, s); break;
    default: launch_group_phi_pos<8>(pos, posi, w, nc, nd, phin, keep, s); break;
    }
}

__global__ void k_group_res(const double *phin, double wsum, const double *q, const double *sigma_s, const double *vol,
                            int64_t nc, int G, double *phi, double *acc) {
    const int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double rr = 0.0, qq = 0.0;
    if (K < nc) {
        const double v = vol[K];
        for (int g = 0; g < G; ++g) {
            double r = 0.0;
            for (int gp = 0; gp < G; ++gp)
                r = r + sigma_s[((int64_t)gp * G + g) * nc + K] * (phin[(int64_t)gp * nc + K] - phi[(int64_t)gp * nc + K]);
            rr = rr + wsum * (v * (r * r));
            const double qk = q[(int64_t)g * nc + K];
            qq = qq + v * (qk * qk);
        }
        for (int g = 0; g < G; ++g) phi[(int64_t)g * nc + K] = phin[(int64_t)g * nc + K];
    }
    block_add(rr, acc);
    block_add(qq, acc + 1);
}

// cell-order angular flux of every group from the level-ordered one:
// psi[g N + m nc + K] = pos[(m nc + posi[m nc + K]) G + g] (the bits in keep)
__global__ void k_group_cell_order(const double *pos, const int32_t *posi, int64_t nc, int64_t N, int G, double *psi,
                                   uint64_t keep) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= N * G) return;
    const int64_t g = t / N, i = t - g * N;
    psi[t] = kept(pos[((i / nc) * nc + posi[i]) * G + g], keep);
}

template <int NF, int DIM>
void launch_den(Graph &g, const double *sigma_t, int G, double *den, hipStream_t s) {
    k_den_groups<NF, DIM><<<(unsigned)ceil_div(g.n_chunks, 4), 256, 0, s>>>(
        g.cblk.as<int32_t>(), g.n_chunks, g.rec64.as<CellRec<double, NF, DIM>>(), g.omega64.as<double>(), sigma_t,
        g.nc, G, den);
    JSW_HIP(hipGetLastError());
}

template <int NF, int DIM>
void launch_residual(Graph &g, const double *psi, const double *q, const double *sigma_s, const double *sigma_t,
                     const double *phi, double psi_b, int G, double *acc, hipStream_t s) {
    k_group_residual<NF, DIM><<<(unsigned)ceil_div(g.nc * G, kB), kB, 0, s>>>(
        g.rec64.as<CellRec<double, NF, DIM>>(), g.omega64.as<double>(), g.weight.as<double>(), psi, q, sigma_s,
        sigma_t, phi, psi_b, g.nc, g.nd, G, acc);
    JSW_HIP(hipGetLastError());
}

}  // namespace

int solve_groups(Graph &g, int G, const double *sigma_t, const double *sigma_s, const double *q, double psi_b,
                 double tol, int32_t max_iter, const jsweep_params *params, double *phi, double *psi_out,
                 jsweep_solve_stats *stats, hipStream_t s) {
    auto t_start = std::chrono::steady_clock::now();
    if (G < 1 || G > kMaxGroups) fail(JSWEEP_E_INVALID_ARG, "group count out of range");
    if (params && params->priority && params->priority != g.priority) set_priority(g, params->priority, s);
    const int64_t nc = g.nc, N = nc * g.nd, S = 64 * g.n_chunks;
    // without lagged edges the fluxes stay in level order (no cell-order
    // copy per sweep; the residual from the sweep identity)
    const bool lo = g.n_lag == 0;
    double *psi = psi_out;
    if (!psi && !lo) {
        if (g.scratch_a.bytes < (size_t)(8 * N * G)) g.scratch_a.alloc(8 * N * G);
        psi = g.scratch_a.as<double>();
    }
    if (!lo) JSW_HIP(hipMemsetAsync(psi, 0, 8 * (size_t)N * G, s));
    double wsum = 0.0;
    for (double x : g.weight_h) wsum += x;
    DevBuf phin(lo ? 8 * (size_t)nc * G : 8);   // the new iterate's phi before the residual
    JSW_HIP(hipMemsetAsync(phi, 0, 8 * (size_t)nc * G, s));
    DevBuf den(8 * (size_t)std::max<int64_t>(1, S) * G), acc(64);
    DevBuf lag_val(8 * (size_t)std::max<int64_t>(1, g.n_lag) * G);
    if (g.vsc.bytes < (size_t)(8 * nc * G)) g.vsc.alloc(8 * nc * G);
    if (g.ctype == JSWEEP_TRI) launch_den<3, 2>(g, sigma_t, G, den.as<double>(), s);
    else if (g.ctype == JSWEEP_TET) launch_den<4, 3>(g, sigma_t, G, den.as<double>(), s);
    else launch_den<6, 3>(g, sigma_t, G, den.as<double>(), s);
    uint32_t *tickets = reinterpret_cast<uint32_t *>(g.status.as<char>() + 128);
    // with every input non-negative every flux is (phi starts from zero,
    // lagged values from earlier sweeps): the sweeps tag their fluxes by sign
    const bool nonneg = psi_b >= 0.0 && !std::signbit(psi_b) && all_nonnegative({{sigma_t, nc * G}, {sigma_s, nc * G * G}, {q, nc * G}}, s);
    const GroupSweep mg{G, den.as<double>(), lag_val.as<double>(), psi_b, nonneg};
    int it = 0, hist = 0, rc = JSWEEP_OK;
    double rho = INFINITY;
    while (true) {
        if (it >= max_iter) { rc = JSWEEP_E_NOT_CONVERGED; break; }
        k_group_source<<<(unsigned)ceil_div(std::max<int64_t>(nc * G, kStreams), kB), kB, 0, s>>>(
            q, sigma_s, phi, g.vol.as<double>(), nc, G, g.vsc.as<double>(), tickets);
        JSW_HIP(hipGetLastError());
        if (g.n_lag) {
            k_group_lag_snapshot<<<(unsigned)ceil_div(g.n_lag * G, kB), kB, 0, s>>>(
                g.lag_mv.as<uint64_t>(), g.lag_u.as<int32_t>(), g.n_lag, G, psi, nc, N, lag_val.as<double>());
            JSW_HIP(hipGetLastError());
        }
        launch_sweep_groups(g, lo ? nullptr : psi, mg, params, s);
        ++it;
        JSW_HIP(hipMemsetAsync(acc.p, 0, 16, s));
        if (lo) {
            group_phi_pos(G, static_cast<const double *>(last_sweep_pos(g)), g.posi.as<int32_t>(),
                          g.weight.as<double>(), nc, g.nd, phin.as<double>(), last_sweep_keep(g), s);
            k_group_res<<<(unsigned)ceil_div(nc, kB), kB, 0, s>>>(phin.as<double>(), wsum, q, sigma_s,
                                                                  g.vol.as<double>(), nc, G, phi, acc.as<double>());
            JSW_HIP(hipGetLastError());
        } else {
            k_group_phi<<<(unsigned)ceil_div(nc * G, kB), kB, 0, s>>>(psi, g.weight.as<double>(), nc, g.nd, G, phi);
            JSW_HIP(hipGetLastError());
            if (g.ctype == JSWEEP_TRI) launch_residual<3, 2>(g, psi, q, sigma_s, sigma_t, phi, psi_b, G, acc.as<double>(), s);
            else if (g.ctype == JSWEEP_TET) launch_residual<4, 3>(g, psi, q, sigma_s, sigma_t, phi, psi_b, G, acc.as<double>(), s);
            else launch_residual<6, 3>(g, psi, q, sigma_s, sigma_t, phi, psi_b, G, acc.as<double>(), s);
        }
        const int st = check_sweep_status(g, s);
        if (st != JSWEEP_OK) return st;
        double h[2];
        JSW_HIP(hipMemcpyAsync(h, acc.p, 16, hipMemcpyDeviceToHost, s));
        JSW_HIP(hipStreamSynchronize(s));
        rho = h[1] > 0.0 ? std::sqrt(h[0]) / std::sqrt(h[1]) : std::sqrt(h[0]);
        if (stats && stats->residual_history && hist < stats->history_capacity) stats->residual_history[hist] = rho;
        ++hist;
        if (tol > 0.0 && rho <= tol) break;
    }
    if (lo && psi_out && it > 0) {
        k_group_cell_order<<<(unsigned)ceil_div(N * G, kB), kB, 0, s>>>(
            static_cast<const double *>(last_sweep_pos(g)), g.posi.as<int32_t>(), nc, N, G, psi_out,
            last_sweep_keep(g));
        JSW_HIP(hipGetLastError());
    } else if (lo && psi_out) {
        JSW_HIP(hipMemsetAsync(psi_out, 0, 8 * (size_t)N * G, s));
    }
    JSW_HIP(hipStreamSynchronize(s));
    if (stats) {
        stats->outer_iters = it;
        stats->sweeps = it;
        stats->residual = rho;
        stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
        stats->lagged_edges = g.n_lag;
        stats->max_levels = g.max_levels;
        stats->history_len = std::min(hist, stats->history_capacity);
    }
    return rc;
}

}  // namespace jsw
