// Mesh geometry on the GPU: unique faces, canonical vector areas, volumes
// and the per-cell records read by the sweep.
//
// Every expression below is IEEE FP64 evaluated exactly as written (the
// library is compiled without floating-point contraction), so the face
// areas, and therefore the upwind signs Omega . S that define the sweep
// graph, are a pure function of the input coordinates.
#include <algorithm>
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "common.hpp"

namespace jsw {

// Local faces.  Triangle edge j and tetrahedron face j are opposite local
// vertex j; hexahedron faces are -x, +x, -y, +y, -z, +z with corner
// c = 4 bx + 2 by + bz, each listed in cyclic order around the face.
__constant__ int8_t kTriFace[3][2] = {{1, 2}, {2, 0}, {0, 1}};
__constant__ int8_t kTetFace[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
__constant__ int8_t kHexFace[6][4] = {{0, 1, 3, 2}, {4, 5, 7, 6}, {0, 1, 5, 4}, {2, 3, 7, 6}, {0, 2, 6, 4}, {1, 3, 7, 5}};

enum : int { kErrMesh = 1, kErrNonManifold = 2, kErrVolume = 4 };

template <int CT>
__device__ inline int face_verts(const int64_t *cells, int64_t K, int j, int64_t *v) {
    const int64_t *c = cells + K * CT;
    if constexpr (CT == JSWEEP_TRI) {
        v[0] = c[kTriFace[j][0]]; v[1] = c[kTriFace[j][1]];
        return 2;
    } else if constexpr (CT == JSWEEP_TET) {
        v[0] = c[kTetFace[j][0]]; v[1] = c[kTetFace[j][1]]; v[2] = c[kTetFace[j][2]];
        return 3;
    } else {
        for (int i = 0; i < 4; ++i) v[i] = c[kHexFace[j][i]];
        return 4;
    }
}

__device__ inline void sort_small(int64_t *v, int n) {
    for (int i = 1; i < n; ++i)
        for (int k = i; k > 0 && v[k - 1] > v[k]; --k) { int64_t t = v[k]; v[k] = v[k - 1]; v[k - 1] = t; }
}

// one key per (cell, local face): the sorted vertex ids packed into 64
// bits (2D: 2 x 32 bits; 3D: the three smallest ids x 21 bits; the fourth
// id of a quadrilateral is checked after sorting)
template <int CT>
__global__ void k_face_keys(const int64_t *cells, int64_t nc, int64_t nv, uint64_t *keys, uint32_t *vals,
                            int32_t *fourth, int *err) {
    constexpr int NF = faces_of(CT);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nc * NF) return;
    int64_t K = i / NF;
    int j = (int)(i % NF);
    int64_t v[4];
    int n = face_verts<CT>(cells, K, j, v);
    for (int k = 0; k < n; ++k)
        if (v[k] < 0 || v[k] >= nv) { atomicOr(err, kErrMesh); v[k] = 0; }
    sort_small(v, n);
    for (int k = 1; k < n; ++k)
        if (v[k] == v[k - 1]) atomicOr(err, kErrMesh);
    uint64_t key;
    if constexpr (CT == JSWEEP_TRI) key = ((uint64_t)v[0] << 32) | (uint64_t)v[1];
    else key = ((uint64_t)v[0] << 42) | ((uint64_t)v[1] << 21) | (uint64_t)v[2];
    keys[i] = key;
    vals[i] = (uint32_t)i;
    if constexpr (CT == JSWEEP_HEX) fourth[i] = (int32_t)v[3];
}

// head[i] = 1 where a new face starts in the sorted key list; validates
// that no face has more than two cells and that paired quads agree.
template <int CT>
__global__ void k_face_heads(const uint64_t *keys, const uint32_t *vals, const int32_t *fourth, int64_t n,
                             int32_t *head, int *err) {
    constexpr int NF = faces_of(CT);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    bool h = (i == 0) || keys[i] != keys[i - 1];
    head[i] = h ? 1 : 0;
    if (!h) {
        if (i >= 2 && keys[i - 2] == keys[i]) atomicOr(err, kErrNonManifold);
        if (vals[i] / NF == vals[i - 1] / NF) atomicOr(err, kErrMesh);
        if constexpr (CT == JSWEEP_HEX)
            if (fourth[vals[i]] != fourth[vals[i - 1]]) atomicOr(err, kErrMesh);
    }
}

// face id of every sorted position -> cell-face map and face-cell pairs;
// the first instance of a face (lowest cell id: the sort is stable and
// instances were numbered cell-major) owns the orientation
template <int CT>
__global__ void k_face_assign(const uint32_t *vals, const int32_t *fid_incl, const int32_t *head, int64_t n,
                              int32_t *cface, int64_t *fcell, uint32_t *first) {
    constexpr int NF = faces_of(CT);
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t f = fid_incl[i] - 1;
    uint32_t inst = vals[i];
    cface[inst] = f;
    int64_t K = inst / NF;
    if (head[i]) {
        fcell[2 * (int64_t)f] = K;
        first[f] = inst;
        bool paired = (i + 1 < n) && !head[i + 1];
        if (!paired) fcell[2 * (int64_t)f + 1] = -1;
    } else {
        fcell[2 * (int64_t)f + 1] = K;
    }
}

template <int DIM>
__device__ inline void load_x(const double *coords, int64_t v, double *x) {
    x[0] = coords[v * DIM];
    x[1] = coords[v * DIM + 1];
    x[2] = DIM == 3 ? coords[v * DIM + 2] : 0.0;
}

// Vector area of a unique face, oriented away from its lower cell:
//   edge a < b:        S = (y_b - y_a, -(x_b - x_a))
//   triangle a < b < c: S = 1/2 (x_b - x_a) x (x_c - x_a)
//   quadrilateral:     S = 1/2 (x_2 - x_0) x (x_3 - x_1), x_0 the smallest
//                      id, x_1 its smaller cyclic neighbour
// then flipped when it points towards the lower cell's reference point
// (the vertex opposite the face; the vertex centroid for a hexahedron).
template <int CT>
__global__ void k_face_geometry(const double *coords, const int64_t *cells, const uint32_t *first, int64_t nf,
                                double *Sx, double *Sy, double *Sz) {
    constexpr int NF = faces_of(CT);
    constexpr int DIM = CT == JSWEEP_TRI ? 2 : 3;
    int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    uint32_t inst = first[f];
    int64_t K = inst / NF;
    int j = (int)(inst % NF);
    int64_t cyc[4];
    int n = face_verts<CT>(cells, K, j, cyc);
    double S[3];
    int64_t smallest;
    if constexpr (CT == JSWEEP_TRI) {
        int64_t a = cyc[0] < cyc[1] ? cyc[0] : cyc[1];
        int64_t b = cyc[0] < cyc[1] ? cyc[1] : cyc[0];
        double xa[3], xb[3];
        load_x<2>(coords, a, xa);
        load_x<2>(coords, b, xb);
        S[0] = xb[1] - xa[1];
        S[1] = -(xb[0] - xa[0]);
        S[2] = 0.0;
        smallest = a;
    } else {
        double u[3], w[3];
        if constexpr (CT == JSWEEP_TET) {
            int64_t s[3] = {cyc[0], cyc[1], cyc[2]};
            sort_small(s, 3);
            double p0[3], p1[3], p2[3];
            load_x<3>(coords, s[0], p0);
            load_x<3>(coords, s[1], p1);
            load_x<3>(coords, s[2], p2);
            for (int d = 0; d < 3; ++d) { u[d] = p1[d] - p0[d]; w[d] = p2[d] - p0[d]; }
            smallest = s[0];
        } else {
            int i0 = 0;
            for (int i = 1; i < n; ++i)
                if (cyc[i] < cyc[i0]) i0 = i;
            int step = cyc[(i0 + 1) & 3] < cyc[(i0 + 3) & 3] ? 1 : 3;
            double q[4][3];
            for (int i = 0; i < 4; ++i) load_x<3>(coords, cyc[(i0 + step * i) & 3], q[i]);
            for (int d = 0; d < 3; ++d) { u[d] = q[2][d] - q[0][d]; w[d] = q[3][d] - q[1][d]; }
            smallest = cyc[i0];
        }
        S[0] = u[1] * w[2] - u[2] * w[1];
        S[1] = u[2] * w[0] - u[0] * w[2];
        S[2] = u[0] * w[1] - u[1] * w[0];
        S[0] = 0.5 * S[0];
        S[1] = 0.5 * S[1];
        S[2] = 0.5 * S[2];
    }
    double r[3];
    if constexpr (CT == JSWEEP_HEX) {
        r[0] = r[1] = r[2] = 0.0;
        for (int c = 0; c < 8; ++c) {
            double x[3];
            load_x<3>(coords, cells[K * 8 + c], x);
            r[0] = r[0] + x[0];
            r[1] = r[1] + x[1];
            r[2] = r[2] + x[2];
        }
        r[0] = r[0] * 0.125;
        r[1] = r[1] * 0.125;
        r[2] = r[2] * 0.125;
    } else {
        load_x<DIM>(coords, cells[K * CT + j], r);
    }
    double xa[3];
    load_x<DIM>(coords, smallest, xa);
    double dd0 = r[0] - xa[0], dd1 = r[1] - xa[1];
    double t = S[0] * dd0 + S[1] * dd1;
    if constexpr (DIM == 3) {
        double dd2 = r[2] - xa[2];
        t = t + S[2] * dd2;
    }
    if (t > 0.0) { S[0] = -S[0]; S[1] = -S[1]; S[2] = -S[2]; }
    Sx[f] = S[0];
    Sy[f] = S[1];
    Sz[f] = S[2];
}

// Per-cell record: outward areas (the lower cell of a face uses +S, the
// higher one exactly -S), neighbour ids and the volume
//   triangle 1/2 |u x v|, tetrahedron |u . (v x w)| / 6,
//   hexahedron 1/3 sum_f xbar_f . S_f^out  (xbar_f: face vertex average).
template <int CT>
__global__ void k_cell_records(const double *coords, const int64_t *cells, const int32_t *cface,
                               const int64_t *fcell, const double *Sx, const double *Sy, const double *Sz,
                               int64_t nc, CellRec<double, faces_of(CT), CT == JSWEEP_TRI ? 2 : 3> *rec,
                               double *vol, int *err) {
    constexpr int NF = faces_of(CT);
    constexpr int DIM = CT == JSWEEP_TRI ? 2 : 3;
    int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (K >= nc) return;
    CellRec<double, NF, DIM> r;
    double so[NF][3];
    for (int j = 0; j < NF; ++j) {
        int64_t f = cface[K * NF + j];
        bool lower = fcell[2 * f] == K;
        double sx = Sx[f], sy = Sy[f], sz = Sz[f];
        so[j][0] = lower ? sx : -sx;
        so[j][1] = lower ? sy : -sy;
        so[j][2] = lower ? sz : -sz;
        for (int d = 0; d < DIM; ++d) r.S[j][d] = so[j][d];
        int64_t nb = lower ? fcell[2 * f + 1] : fcell[2 * f];
        r.nbr[j] = (int32_t)nb;
    }
    const int64_t *c = cells + K * CT;
    double V;
    if constexpr (CT == JSWEEP_TRI) {
        double a[3], b[3], e[3];
        load_x<2>(coords, c[0], a);
        load_x<2>(coords, c[1], b);
        load_x<2>(coords, c[2], e);
        double ux = b[0] - a[0], uy = b[1] - a[1], vx = e[0] - a[0], vy = e[1] - a[1];
        V = 0.5 * fabs(ux * vy - uy * vx);
    } else if constexpr (CT == JSWEEP_TET) {
        double a[3], b[3], e[3], h[3], u[3], v[3], w[3], x[3];
        load_x<3>(coords, c[0], a);
        load_x<3>(coords, c[1], b);
        load_x<3>(coords, c[2], e);
        load_x<3>(coords, c[3], h);
        for (int d = 0; d < 3; ++d) { u[d] = b[d] - a[d]; v[d] = e[d] - a[d]; w[d] = h[d] - a[d]; }
        x[0] = v[1] * w[2] - v[2] * w[1];
        x[1] = v[2] * w[0] - v[0] * w[2];
        x[2] = v[0] * w[1] - v[1] * w[0];
        V = fabs(u[0] * x[0] + u[1] * x[1] + u[2] * x[2]) / 6.0;
    } else {
        double acc = 0.0;
        for (int j = 0; j < 6; ++j) {
            double xb[3] = {0.0, 0.0, 0.0};
            for (int i = 0; i < 4; ++i) {
                double p[3];
                load_x<3>(coords, c[kHexFace[j][i]], p);
                xb[0] = xb[0] + p[0];
                xb[1] = xb[1] + p[1];
                xb[2] = xb[2] + p[2];
            }
            xb[0] = xb[0] * 0.25;
            xb[1] = xb[1] * 0.25;
            xb[2] = xb[2] * 0.25;
            acc = acc + (xb[0] * so[j][0] + xb[1] * so[j][1] + xb[2] * so[j][2]);
        }
        V = acc / 3.0;
    }
    if (!(V > 0.0)) atomicOr(err, kErrVolume);
    r.V = V;
    r.sigV = 0.0;
    rec[K] = r;
    vol[K] = V;
}

// Morton code of every cell's vertex average on a 2^21 grid per axis over
// the mesh's bounding box (lo, 1 / extent), with the cell id as the value:
// sorted, it gives the space-filling-curve order the sweep patches are cut
// from.
__device__ inline uint64_t spread3(uint64_t x) {
    x &= 0x1fffffull;
    x = (x | x << 32) & 0x1f00000000ffffull;
    x = (x | x << 16) & 0x1f0000ff0000ffull;
    x = (x | x << 8) & 0x100f00f00f00f00full;
    x = (x | x << 4) & 0x10c30c30c30c30c3ull;
    x = (x | x << 2) & 0x1249249249249249ull;
    return x;
}

template <int CT>
__global__ void k_cell_morton(const double *coords, const int64_t *cells, int64_t nc, double lx, double ly,
                              double lz, double sx, double sy, double sz, uint64_t *keys, int32_t *vals) {
    constexpr int DIM = CT == JSWEEP_TRI ? 2 : 3;
    int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (K >= nc) return;
    double c[3] = {0.0, 0.0, 0.0};
    for (int v = 0; v < CT; ++v) {
        const int64_t p = cells[K * CT + v];
        for (int d = 0; d < DIM; ++d) c[d] += coords[p * DIM + d];
    }
    const double lo[3] = {lx, ly, lz}, sc[3] = {sx, sy, sz};
    uint64_t q[3] = {0, 0, 0};
    for (int d = 0; d < DIM; ++d) {
        double t = (c[d] / CT - lo[d]) * sc[d];
        t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
        q[d] = (uint64_t)(t * 2097151.0);
    }
    keys[K] = spread3(q[0]) << 2 | spread3(q[1]) << 1 | spread3(q[2]);
    vals[K] = (int32_t)K;
}

__global__ void k_rank_of(const int32_t *order, int64_t nc, int32_t *rank) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nc) rank[order[i]] = (int32_t)i;
}

template <int CT>
static void geometry_impl(Graph &g, const jsweep_mesh &mesh, hipStream_t s) {
    constexpr int NF = faces_of(CT);
    constexpr int DIM = CT == JSWEEP_TRI ? 2 : 3;
    const int64_t nc = mesh.n_cells, nv = mesh.n_vertices;
    const int64_t ninst = nc * NF;
    DevBuf d_coords(sizeof(double) * nv * DIM), d_cells(sizeof(int64_t) * nc * CT);
    JSW_HIP(hipMemcpyAsync(d_coords.p, mesh.coords, d_coords.bytes, hipMemcpyHostToDevice, s));
    JSW_HIP(hipMemcpyAsync(d_cells.p, mesh.cell_vertices, d_cells.bytes, hipMemcpyHostToDevice, s));
    DevBuf keys(8 * ninst), keys2(8 * ninst), vals(4 * ninst), vals2(4 * ninst);
    DevBuf fourth(CT == JSWEEP_HEX ? 4 * ninst : 4), err(sizeof(int));
    JSW_HIP(hipMemsetAsync(err.p, 0, sizeof(int), s));
    const int B = 256;
    int gi = (int)ceil_div(ninst, B);
    k_face_keys<CT><<<gi, B, 0, s>>>(d_cells.as<int64_t>(), nc, nv, keys.as<uint64_t>(), vals.as<uint32_t>(),
                                     fourth.as<int32_t>(), err.as<int>());
    JSW_HIP(hipGetLastError());
    size_t tmp_bytes = 0;
    const unsigned end_bit = CT == JSWEEP_TRI ? 64 : 63;
    JSW_HIP(rocprim::radix_sort_pairs(nullptr, tmp_bytes, keys.as<uint64_t>(), keys2.as<uint64_t>(),
                                      vals.as<uint32_t>(), vals2.as<uint32_t>(), (size_t)ninst, 0u, end_bit, s));
    DevBuf tmp(tmp_bytes + 16);
    JSW_HIP(rocprim::radix_sort_pairs(tmp.p, tmp_bytes, keys.as<uint64_t>(), keys2.as<uint64_t>(),
                                      vals.as<uint32_t>(), vals2.as<uint32_t>(), (size_t)ninst, 0u, end_bit, s));
    DevBuf head(4 * ninst), fid(4 * ninst);
    k_face_heads<CT><<<gi, B, 0, s>>>(keys2.as<uint64_t>(), vals2.as<uint32_t>(), fourth.as<int32_t>(), ninst,
                                      head.as<int32_t>(), err.as<int>());
    JSW_HIP(hipGetLastError());
    size_t scan_bytes = 0;
    JSW_HIP(rocprim::inclusive_scan(nullptr, scan_bytes, head.as<int32_t>(), fid.as<int32_t>(), (size_t)ninst,
                                    rocprim::plus<int32_t>(), s));
    DevBuf scan_tmp(scan_bytes + 16);
    JSW_HIP(rocprim::inclusive_scan(scan_tmp.p, scan_bytes, head.as<int32_t>(), fid.as<int32_t>(), (size_t)ninst,
                                    rocprim::plus<int32_t>(), s));
    int32_t nf32 = 0;
    int herr = 0;
    JSW_HIP(hipMemcpyAsync(&nf32, fid.as<int32_t>() + (ninst - 1), 4, hipMemcpyDeviceToHost, s));
    JSW_HIP(hipMemcpyAsync(&herr, err.p, 4, hipMemcpyDeviceToHost, s));
    JSW_HIP(hipStreamSynchronize(s));
    if (herr & kErrNonManifold) fail(JSWEEP_E_MESH, "a face is shared by more than two cells");
    if (herr) fail(JSWEEP_E_MESH, "invalid cell connectivity (vertex id out of range, repeated vertex or mismatched face)");
    const int64_t nf = nf32;
    g.nf = nf;
    DevBuf cface(4 * ninst), fcell(16 * nf), first(4 * nf);
    k_face_assign<CT><<<gi, B, 0, s>>>(vals2.as<uint32_t>(), fid.as<int32_t>(), head.as<int32_t>(), ninst,
                                       cface.as<int32_t>(), fcell.as<int64_t>(), first.as<uint32_t>());
    JSW_HIP(hipGetLastError());
    DevBuf Sx(8 * nf), Sy(8 * nf), Sz(8 * nf);
    k_face_geometry<CT><<<(int)ceil_div(nf, B), B, 0, s>>>(d_coords.as<double>(), d_cells.as<int64_t>(),
                                                           first.as<uint32_t>(), nf, Sx.as<double>(),
                                                           Sy.as<double>(), Sz.as<double>());
    JSW_HIP(hipGetLastError());
    g.rec64.alloc(sizeof(CellRec<double, NF, DIM>) * nc);
    g.vol.alloc(8 * nc);
    k_cell_records<CT><<<(int)ceil_div(nc, B), B, 0, s>>>(
        d_coords.as<double>(), d_cells.as<int64_t>(), cface.as<int32_t>(), fcell.as<int64_t>(), Sx.as<double>(),
        Sy.as<double>(), Sz.as<double>(), nc, g.rec64.as<CellRec<double, NF, DIM>>(), g.vol.as<double>(),
        err.as<int>());
    JSW_HIP(hipGetLastError());
    JSW_HIP(hipMemcpyAsync(&herr, err.p, 4, hipMemcpyDeviceToHost, s));
    JSW_HIP(hipStreamSynchronize(s));
    if (herr & kErrVolume) fail(JSWEEP_E_MESH, "a cell has a non-positive volume");
    if (herr) fail(JSWEEP_E_MESH, "invalid mesh");
    // Morton rank of every cell (patches of the patch sweep)
    double lo[3] = {0.0, 0.0, 0.0}, hi[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < DIM; ++d) { lo[d] = mesh.coords[d]; hi[d] = mesh.coords[d]; }
    for (int64_t i = 0; i < nv; ++i)
        for (int d = 0; d < DIM; ++d) {
            lo[d] = std::min(lo[d], mesh.coords[i * DIM + d]);
            hi[d] = std::max(hi[d], mesh.coords[i * DIM + d]);
        }
    double sc[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < DIM; ++d) sc[d] = hi[d] > lo[d] ? 1.0 / (hi[d] - lo[d]) : 0.0;
    DevBuf mk(8 * nc), mk2(8 * nc), mv(4 * nc), mv2(4 * nc);
    k_cell_morton<CT><<<(int)ceil_div(nc, B), B, 0, s>>>(d_coords.as<double>(), d_cells.as<int64_t>(), nc, lo[0],
                                                         lo[1], lo[2], sc[0], sc[1], sc[2], mk.as<uint64_t>(),
                                                         mv.as<int32_t>());
    JSW_HIP(hipGetLastError());
    size_t mt_bytes = 0;
    JSW_HIP(rocprim::radix_sort_pairs(nullptr, mt_bytes, mk.as<uint64_t>(), mk2.as<uint64_t>(), mv.as<int32_t>(),
                                      mv2.as<int32_t>(), (size_t)nc, 0u, 63u, s));
    DevBuf mt(mt_bytes + 16);
    JSW_HIP(rocprim::radix_sort_pairs(mt.p, mt_bytes, mk.as<uint64_t>(), mk2.as<uint64_t>(), mv.as<int32_t>(),
                                      mv2.as<int32_t>(), (size_t)nc, 0u, 63u, s));
    g.mrank.alloc(4 * nc);
    k_rank_of<<<(int)ceil_div(nc, B), B, 0, s>>>(mv2.as<int32_t>(), nc, g.mrank.as<int32_t>());
    JSW_HIP(hipGetLastError());
    JSW_HIP(hipStreamSynchronize(s));
}

void build_geometry(Graph &g, const jsweep_mesh &mesh, hipStream_t s) {
    g.dim = mesh.dim;
    g.ctype = mesh.cell_type;
    g.nfpc = faces_of(mesh.cell_type);
    g.nc = mesh.n_cells;
    g.nv = mesh.n_vertices;
    if (mesh.cell_type == JSWEEP_TRI) geometry_impl<JSWEEP_TRI>(g, mesh, s);
    else if (mesh.cell_type == JSWEEP_TET) geometry_impl<JSWEEP_TET>(g, mesh, s);
    else geometry_impl<JSWEEP_HEX>(g, mesh, s);
}

// FP32 copy of the records for the correction sweeps (areas and volume
// rounded to nearest; the sign pattern of Omega . S can differ from the
// FP64 graph only on faces that are numerically parallel to a direction,
// which the FP32 sweep treats exactly like the FP64 graph does because it
// takes inflow/outflow from the FP64 record's classification: see
// k_rec32 below).
template <int CT>
__global__ void k_rec32(const CellRec<double, faces_of(CT), CT == JSWEEP_TRI ? 2 : 3> *r64, int64_t nc,
                        CellRec<float, faces_of(CT), CT == JSWEEP_TRI ? 2 : 3> *r32) {
    constexpr int NF = faces_of(CT);
    constexpr int DIM = CT == JSWEEP_TRI ? 2 : 3;
    int64_t K = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (K >= nc) return;
    CellRec<double, NF, DIM> a = r64[K];
    CellRec<float, NF, DIM> b;
    for (int j = 0; j < NF; ++j) {
        for (int d = 0; d < DIM; ++d) b.S[j][d] = (float)a.S[j][d];
        b.nbr[j] = a.nbr[j];
    }
    b.V = (float)a.V;
    b.sigV = 0.0f;
    r32[K] = b;
}

void build_rec32(Graph &g, hipStream_t s) {
    if (g.rec32.p) return;
    const int B = 256;
    int gb = (int)ceil_div(g.nc, B);
    if (g.ctype == JSWEEP_TRI) {
        g.rec32.alloc(sizeof(CellRec<float, 3, 2>) * g.nc);
        k_rec32<JSWEEP_TRI><<<gb, B, 0, s>>>(g.rec64.as<CellRec<double, 3, 2>>(), g.nc, g.rec32.as<CellRec<float, 3, 2>>());
    } else if (g.ctype == JSWEEP_TET) {
        g.rec32.alloc(sizeof(CellRec<float, 4, 3>) * g.nc);
        k_rec32<JSWEEP_TET><<<gb, B, 0, s>>>(g.rec64.as<CellRec<double, 4, 3>>(), g.nc, g.rec32.as<CellRec<float, 4, 3>>());
    } else {
        g.rec32.alloc(sizeof(CellRec<float, 6, 3>) * g.nc);
        k_rec32<JSWEEP_HEX><<<gb, B, 0, s>>>(g.rec64.as<CellRec<double, 6, 3>>(), g.nc, g.rec32.as<CellRec<float, 6, 3>>());
    }
    JSW_HIP(hipGetLastError());
}

}  // namespace jsw
