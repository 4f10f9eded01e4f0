// Device helpers shared by the solve kernels (single graph and batched).
#pragma once
#include "common.hpp"

namespace jsw {

// sum_m w_m x_{m, K} in ascending m (the order of the scalar flux), with the
// loads of sixteen directions issued together
template <class T>
__device__ inline double dir_sum(const double *w, const T *x, int64_t nc, int nd, int64_t K) {
    double s = 0.0;
    int m = 0;
    for (; m + 16 <= nd; m += 16) {
        T v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = x[(int64_t)(m + k) * nc + K];
#pragma unroll
        for (int k = 0; k < 16; ++k) s = s + w[m + k] * (double)v[k];
    }
    for (; m + 4 <= nd; m += 4) {
        T v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = x[(int64_t)(m + k) * nc + K];
#pragma unroll
        for (int k = 0; k < 4; ++k) s = s + w[m + k] * (double)v[k];
    }
    for (; m < nd; ++m) s = s + w[m] * (double)x[(int64_t)m * nc + K];
    return s;
}

// dir_sum of the two cells K and K + 1 (K and nc even), each direction's
// pair read as one 16-byte load; each sum in ascending m as in dir_sum
__device__ inline void dir_sum2(const double *w, const double *x, int64_t nc, int nd, int64_t K, double &s0,
                                double &s1) {
    s0 = 0.0;
    s1 = 0.0;
    int m = 0;
    for (; m + 16 <= nd; m += 16) {
        double2 v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = *reinterpret_cast<const double2 *>(x + (int64_t)(m + k) * nc + K);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            s0 = s0 + w[m + k] * v[k].x;
            s1 = s1 + w[m + k] * v[k].y;
        }
    }
    for (; m < nd; ++m) {
        const double2 v = *reinterpret_cast<const double2 *>(x + (int64_t)m * nc + K);
        s0 = s0 + w[m] * v.x;
        s1 = s1 + w[m] * v.y;
    }
}

// Logical block of an XCD-aware launch of 8 * per_xcd workgroups.  The
// dispatcher deals workgroups round robin over the 8 XCDs, so logical block
// (b mod 8) * per_xcd + b / 8 gives each XCD one contiguous eighth of the
// blocks, walked in order: gathers of neighbouring cells through the level
// positions then share L2 lines (in level order the cells of one level
// that lie in a range of ids are stored together).
__device__ inline int64_t xcd_block(int64_t per_xcd) {
    return (int64_t)(blockIdx.x & 7u) * per_xcd + (int64_t)(blockIdx.x >> 3);
}
inline int64_t xcd_per(int64_t blocks) { return (blocks + 7) / 8; }

// An FP64 flux read from a sweep's level-position array with only the
// bits in keep (all but the sign bit when that sweep tagged its fluxes by
// sign); FP32 fluxes are never tagged
__device__ __forceinline__ double kept(double v, uint64_t keep) {
    return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, v) & keep);
}
__device__ __forceinline__ float kept(float v, uint64_t) { return v; }

// dir_sum over the level-ordered fluxes of a sweep: the flux of cell K in
// direction m sits at m nc + posi[m nc + K].  Sixteen directions' positions
// are loaded together, then their fluxes, and the next sixteen positions
// are loaded while those fluxes travel (one round trip per batch instead
// of two); the sum runs in ascending m.
template <class T>
__device__ inline double dir_sum_pos(const double *w, const T *pos, const int32_t *posi, int64_t nc, int nd, int64_t K,
                                     uint64_t keep = ~0ull) {
    double s = 0.0;
    int m = 0;
    int32_t p[16];
    if (16 <= nd) {
#pragma unroll
        for (int k = 0; k < 16; ++k) p[k] = posi[(int64_t)k * nc + K];
    }
    for (; m + 16 <= nd; m += 16) {
        T v[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) v[k] = pos[(int64_t)(m + k) * nc + p[k]];
        if (m + 32 <= nd) {
#pragma unroll
            for (int k = 0; k < 16; ++k) p[k] = posi[(int64_t)(m + 16 + k) * nc + K];
        }
        // masked only here, after the next positions' loads have been
        // issued: nothing waits for the fluxes before that
#pragma unroll
        for (int k = 0; k < 16; ++k) s = s + w[m + k] * (double)kept(v[k], keep);
    }
    for (; m < nd; ++m) s = s + w[m] * (double)kept(pos[(int64_t)m * nc + posi[(int64_t)m * nc + K]], keep);
    return s;
}

// dir_sum_pos of the cells K and K + 1 (K and nc even): each direction's two
// positions are one 8-byte load
template <class T>
__device__ inline void dir_sum_pos2(const double *w, const T *pos, const int32_t *posi, int64_t nc, int nd, int64_t K,
                                    double &s0, double &s1, uint64_t keep = ~0ull) {
    s0 = 0.0;
    s1 = 0.0;
    int m = 0;
    constexpr int B = 16;   // directions per batch
    int2 p[B];
    if (B <= nd) {
#pragma unroll
        for (int k = 0; k < B; ++k) p[k] = *reinterpret_cast<const int2 *>(posi + (int64_t)k * nc + K);
    }
    for (; m + B <= nd; m += B) {
        T v0[B], v1[B];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            v0[k] = pos[(int64_t)(m + k) * nc + p[k].x];
            v1[k] = pos[(int64_t)(m + k) * nc + p[k].y];
        }
        // the next batch's positions travel while these fluxes do
        if (m + 2 * B <= nd) {
#pragma unroll
            for (int k = 0; k < B; ++k) p[k] = *reinterpret_cast<const int2 *>(posi + (int64_t)(m + B + k) * nc + K);
        }
#pragma unroll
        for (int k = 0; k < B; ++k) {
            s0 = s0 + w[m + k] * (double)kept(v0[k], keep);
            s1 = s1 + w[m + k] * (double)kept(v1[k], keep);
        }
    }
    for (; m < nd; ++m) {
        const int2 pm = *reinterpret_cast<const int2 *>(posi + (int64_t)m * nc + K);
        s0 = s0 + w[m] * (double)kept(pos[(int64_t)m * nc + pm.x], keep);
        s1 = s1 + w[m] * (double)kept(pos[(int64_t)m * nc + pm.y], keep);
    }
}

// One cell of the FP64 residual with the full (un-lagged) streaming
// operator, looping over directions:
//   phi_K = sum_m w_m psi_{K,m}
//   r_{K,m} = q_K + sigma_s,K phi_K - (den psi_{K,m} - in_{K,m}) / V_K
// Returns V_K sum_m w_m r^2 (and writes phi_K).  When r32 != null, V_K r
// (the correction sweep's per-direction source times the cell volume, as
// the balance takes it) is stored in FP32: at the vertex's level position
// posi[m nc + K] within direction m, or at m nc + K (cell order) when posi
// is null.
template <int NF, int DIM>
__device__ inline double residual_cell(const CellRec<double, NF, DIM> &r, int64_t K, const double *omega,
                                       const double *w, const double *psi, double q, double sigma_s, double psi_b,
                                       int64_t nc, int nd, double *phi, float *r32, const int32_t *posi) {
    int32_t nb[NF];
#pragma unroll
    for (int j = 0; j < NF; ++j) nb[j] = r.nbr[j] <= -2 ? -r.nbr[j] - 2 : r.nbr[j];
    const double ph = dir_sum(w, psi, nc, nd, K);
    phi[K] = ph;
    const double src = q + sigma_s * ph;
    // B directions' fluxes (own and neighbours) are loaded before any is
    // used: four, or three for hexahedra, whose records and neighbour
    // fluxes would otherwise not fit in 128 registers
    constexpr int B = NF >= 6 ? 3 : 4;
    double cell = 0.0;
    for (int m = 0; m < nd; m += B) {
        double own[B], up[B][NF];
#pragma unroll
        for (int k = 0; k < B; ++k) {
            const int mm = m + k < nd ? m + k : m;
            const double *pm = psi + (int64_t)mm * nc;
            own[k] = pm[K];
#pragma unroll
            for (int j = 0; j < NF; ++j) up[k][j] = nb[j] < 0 ? 0.0 : pm[nb[j]];
        }
#pragma unroll
        for (int k = 0; k < B; ++k) {
            if (m + k < nd) {
                const double *om = omega + 3 * (m + k);
                double in = 0.0, den = r.sigV;
#pragma unroll
                for (int j = 0; j < NF; ++j) {
                    double d = om[0] * r.S[j][0] + om[1] * r.S[j][1];
                    if constexpr (DIM == 3) d = d + om[2] * r.S[j][2];
                    if (d < 0.0) in = in + (-d) * (nb[j] < 0 ? psi_b : up[k][j]);
                    else if (d > 0.0) den = den + d;
                }
                const double res = src - (den * own[k] - in) / r.V;
                if (r32) {
                    const int64_t o = (int64_t)(m + k) * nc;
                    r32[o + (posi ? (int64_t)posi[o + K] : K)] = (float)(r.V * res);
                }
                cell = cell + w[m + k] * (res * res);
            }
        }
    }
    return r.V * cell;
}

// wavefront + workgroup sum, one atomic per workgroup
__device__ inline void block_add(double v, double *out) {
    __shared__ double red[16];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
        atomicAdd(out, t);
    }
}

}  // namespace jsw
