/*
 * Oracle for the data-driven transport sweep: a plain, serial, FP64 CPU
 * implementation of what the sweep path computes.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  The product library never
 * links, includes or calls anything here, and this file includes nothing of
 * the product (the two share no code).
 *
 * What it computes (paper: JSweep, arXiv 1803.09876):
 *   - the sweep dependency graph: vertices are (cell, direction) pairs and an
 *     edge u -> v means v needs u's outgoing angular flux (Sec. V-A; the
 *     sweep as a topological traversal, Sec. I and II-C);
 *   - counts of upwind neighbours and a ready queue seeded with count-0
 *     vertices, drained in dependency order (Listing 1, init/compute);
 *   - source iteration: scattering source, sweeps of every direction, error
 *     reduction, repeated to a tolerance (appendix algorithm "Source
 *     iterative Sn solver", steps 1, 2.1-2.3);
 *   - cycle elimination before sweeping (appendix, sweep workflow step 1);
 *     the paper gives no rule, the reading used here is: inside each
 *     non-trivial strongly connected component keep edges from lower to
 *     higher cell id and lag the others (use the previous iterate there).
 *
 * The paper names no spatial scheme, quadrature normalisation, face
 * orientation or summation order.  The readings used (step upwind scheme,
 * weights summing to one, canonical face vector areas, local-face and
 * ascending-direction summation orders) are spelled out at each function.
 * Every floating-point expression is evaluated exactly as written, left to
 * right, and this file is compiled without FMA contraction.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_TRI 3
#define ORC_TET 4
#define ORC_HEX 8

#define ORC_OK 0
#define ORC_E_ARG -1
#define ORC_E_MESH -2
#define ORC_E_CYCLE -4
#define ORC_E_OOM -6

typedef struct {
    int dim, ctype, nvpc, nfpc;
    int64_t nv, nc, nf;
    double *coords;   /* [nv*dim] */
    int64_t *cells;   /* [nc*nvpc] */
    double *S;        /* [nf*3] canonical vector area (lower cell -> higher cell, or outward) */
    int64_t *fcell;   /* [nf*2] lower cell id, higher cell id or -1 on the boundary */
    int64_t *cface;   /* [nc*nfpc] unique face of each local face */
    double *vol;      /* [nc] */
    int nd;
    double *omega;    /* [nd*3] */
    int32_t *level;   /* [nd*nc] */
    int32_t *order;   /* [nd*nc] cells by (level, id) */
    int64_t *lvl_off; /* [nd+1] start of each direction's level pointer block */
    int64_t *lvl_ptr; /* per direction nlev+1 offsets */
    int32_t *nlev;    /* [nd] */
    int64_t nlag;     /* lagged edges sorted by (m, v, local face of v) */
    int32_t *lag_m, *lag_face;
    int64_t *lag_u, *lag_v;
} orc_graph;

/* ------------------------------------------------------------------ */
/* local faces                                                          */
/* ------------------------------------------------------------------ */

/* Triangle edge j is the edge opposite vertex j: (v1 v2), (v2 v0), (v0 v1).
 * Tetrahedron face j is the face opposite vertex j.
 * Hexahedron (corner c at offset (c>>2&1, c>>1&1, c&1)): faces -x, +x, -y,
 * +y, -z, +z, each listed in cyclic order around the quadrilateral. */
static const int TRI_F[3][2] = {{1, 2}, {2, 0}, {0, 1}};
static const int TET_F[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
static const int HEX_F[6][4] = {{0, 1, 3, 2}, {4, 5, 7, 6}, {0, 1, 5, 4},
                                {2, 3, 7, 6}, {0, 2, 6, 4}, {1, 3, 7, 5}};

static int nverts_of_face(int ctype) { return ctype == ORC_TRI ? 2 : ctype == ORC_TET ? 3 : 4; }

static void local_face_vertices(const orc_graph *g, int64_t K, int j, int64_t *out) {
    const int64_t *c = g->cells + K * g->nvpc;
    if (g->ctype == ORC_TRI) { out[0] = c[TRI_F[j][0]]; out[1] = c[TRI_F[j][1]]; }
    else if (g->ctype == ORC_TET) { for (int i = 0; i < 3; ++i) out[i] = c[TET_F[j][i]]; }
    else { for (int i = 0; i < 4; ++i) out[i] = c[HEX_F[j][i]]; }
}

static const double *X(const orc_graph *g, int64_t v) { return g->coords + v * g->dim; }

/* Reference point inside cell K used to orient faces of K: the vertex
 * opposite local face j (triangle, tetrahedron) or the vertex centroid
 * (hexahedron, corners summed in index order then scaled by 1/8). */
static void ref_point(const orc_graph *g, int64_t K, int j, double *p) {
    const int64_t *c = g->cells + K * g->nvpc;
    p[0] = p[1] = p[2] = 0.0;
    if (g->ctype != ORC_HEX) {
        const double *x = X(g, c[j]);
        for (int d = 0; d < g->dim; ++d) p[d] = x[d];
        return;
    }
    for (int v = 0; v < 8; ++v) {
        const double *x = X(g, c[v]);
        p[0] = p[0] + x[0]; p[1] = p[1] + x[1]; p[2] = p[2] + x[2];
    }
    p[0] = p[0] * 0.125; p[1] = p[1] * 0.125; p[2] = p[2] * 0.125;
}

/* ------------------------------------------------------------------ */
/* unique faces                                                         */
/* ------------------------------------------------------------------ */

typedef struct { int64_t key[4]; int64_t cell; int32_t j; } face_inst;

static int cmp_inst(const void *a, const void *b) {
    const face_inst *x = a, *y = b;
    for (int i = 0; i < 4; ++i) {
        if (x->key[i] < y->key[i]) return -1;
        if (x->key[i] > y->key[i]) return 1;
    }
    if (x->cell < y->cell) return -1;
    if (x->cell > y->cell) return 1;
    return 0;
}

static int cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return x < y ? -1 : x > y;
}

/* Vector area of a unique face from its global vertices.
 *   edge (a < b):           S = (y_b - y_a, -(x_b - x_a))
 *   triangle (a < b < c):   S = 1/2 (x_b - x_a) x (x_c - x_a)
 *   quadrilateral:          S = 1/2 (x_2 - x_0) x (x_3 - x_1) with x_0 the
 *     smallest id and x_1 the smaller of its two cyclic neighbours; this is
 *     the exact vector area of any surface spanning the four edges. */
static void face_area(const orc_graph *g, const int64_t *cyc, int nfv, double *S) {
    S[0] = S[1] = S[2] = 0.0;
    if (nfv == 2) {
        int64_t a = cyc[0] < cyc[1] ? cyc[0] : cyc[1], b = cyc[0] < cyc[1] ? cyc[1] : cyc[0];
        const double *xa = X(g, a), *xb = X(g, b);
        S[0] = xb[1] - xa[1];
        S[1] = -(xb[0] - xa[0]);
        return;
    }
    double p0[3], p1[3], p2[3], u[3], v[3];
    if (nfv == 3) {
        int64_t s[3] = {cyc[0], cyc[1], cyc[2]};
        qsort(s, 3, sizeof(int64_t), cmp_i64);
        memcpy(p0, X(g, s[0]), 24); memcpy(p1, X(g, s[1]), 24); memcpy(p2, X(g, s[2]), 24);
        for (int d = 0; d < 3; ++d) { u[d] = p1[d] - p0[d]; v[d] = p2[d] - p0[d]; }
    } else {
        int i0 = 0;
        for (int i = 1; i < 4; ++i) if (cyc[i] < cyc[i0]) i0 = i;
        int nx = (i0 + 1) % 4, pv = (i0 + 3) % 4;
        int step = cyc[nx] < cyc[pv] ? 1 : 3;
        int64_t q[4];
        for (int i = 0; i < 4; ++i) q[i] = cyc[(i0 + step * i) % 4];
        const double *x0 = X(g, q[0]), *x1 = X(g, q[1]), *x2 = X(g, q[2]), *x3 = X(g, q[3]);
        for (int d = 0; d < 3; ++d) { u[d] = x2[d] - x0[d]; v[d] = x3[d] - x1[d]; }
    }
    S[0] = u[1] * v[2] - u[2] * v[1];
    S[1] = u[2] * v[0] - u[0] * v[2];
    S[2] = u[0] * v[1] - u[1] * v[0];
    S[0] = 0.5 * S[0]; S[1] = 0.5 * S[1]; S[2] = 0.5 * S[2];
}

static double dot3(const double *a, const double *b, int dim) {
    double r = a[0] * b[0] + a[1] * b[1];
    if (dim == 3) r = r + a[2] * b[2];
    return r;
}

/* outward vector area of local face j of cell K */
static void outward(const orc_graph *g, int64_t K, int j, double *s) {
    int64_t f = g->cface[K * g->nfpc + j];
    const double *S = g->S + 3 * f;
    if (g->fcell[2 * f] == K) { s[0] = S[0]; s[1] = S[1]; s[2] = S[2]; }
    else { s[0] = -S[0]; s[1] = -S[1]; s[2] = -S[2]; }
}

static int build_faces(orc_graph *g) {
    int nfv = nverts_of_face(g->ctype);
    int64_t ninst = g->nc * g->nfpc;
    face_inst *inst = malloc(sizeof(face_inst) * (size_t)(ninst ? ninst : 1));
    if (!inst) return ORC_E_OOM;
    for (int64_t K = 0; K < g->nc; ++K)
        for (int j = 0; j < g->nfpc; ++j) {
            face_inst *p = inst + K * g->nfpc + j;
            int64_t v[4] = {-1, -1, -1, -1};
            local_face_vertices(g, K, j, v);
            qsort(v, nfv, sizeof(int64_t), cmp_i64);
            for (int i = 0; i < 4; ++i) p->key[i] = i < nfv ? v[i] : -1;
            p->cell = K; p->j = j;
        }
    qsort(inst, (size_t)ninst, sizeof(face_inst), cmp_inst);
    int64_t nf = 0;
    for (int64_t i = 0; i < ninst; ++i)
        if (i == 0 || memcmp(inst[i].key, inst[i - 1].key, sizeof inst[i].key) != 0) ++nf;
    g->nf = nf;
    g->S = calloc((size_t)(nf ? nf : 1) * 3, sizeof(double));
    g->fcell = malloc(sizeof(int64_t) * 2 * (size_t)(nf ? nf : 1));
    g->cface = malloc(sizeof(int64_t) * (size_t)(ninst ? ninst : 1));
    if (!g->S || !g->fcell || !g->cface) { free(inst); return ORC_E_OOM; }
    int64_t f = -1;
    for (int64_t i = 0; i < ninst; ++i) {
        int first = (i == 0 || memcmp(inst[i].key, inst[i - 1].key, sizeof inst[i].key) != 0);
        if (first) { ++f; g->fcell[2 * f] = inst[i].cell; g->fcell[2 * f + 1] = -1; }
        else {
            if (g->fcell[2 * f + 1] != -1) { free(inst); return ORC_E_MESH; } /* >2 cells share a face */
            if (inst[i].cell == g->fcell[2 * f]) { free(inst); return ORC_E_MESH; }
            g->fcell[2 * f + 1] = inst[i].cell; /* sorted by cell: this is the higher id */
        }
        g->cface[inst[i].cell * g->nfpc + inst[i].j] = f;
    }
    /* vector areas, oriented from the lower cell towards the higher cell
     * (outward from the only cell on the boundary) */
    for (int64_t i = 0; i < ninst; ++i) {
        int first = (i == 0 || memcmp(inst[i].key, inst[i - 1].key, sizeof inst[i].key) != 0);
        if (!first) continue;
        int64_t ff = g->cface[inst[i].cell * g->nfpc + inst[i].j];
        int64_t K = inst[i].cell;
        int64_t cyc[4];
        local_face_vertices(g, K, inst[i].j, cyc);
        double *S = g->S + 3 * ff;
        face_area(g, cyc, nfv, S);
        double r[3], xa[3] = {0, 0, 0}, d[3] = {0, 0, 0};
        ref_point(g, K, inst[i].j, r);
        const double *pa = X(g, inst[i].key[0]);
        for (int k = 0; k < g->dim; ++k) xa[k] = pa[k];
        for (int k = 0; k < g->dim; ++k) d[k] = r[k] - xa[k];
        if (dot3(S, d, g->dim) > 0.0) { S[0] = -S[0]; S[1] = -S[1]; S[2] = -S[2]; }
    }
    free(inst);
    return ORC_OK;
}

/* Cell volumes: triangle 1/2 |u x v|, tetrahedron |u . (v x w)| / 6,
 * hexahedron 1/3 sum_f xbar_f . S_f^out (divergence theorem, xbar_f the
 * vertex average of face f). */
static int build_volumes(orc_graph *g) {
    g->vol = malloc(sizeof(double) * (size_t)(g->nc ? g->nc : 1));
    if (!g->vol) return ORC_E_OOM;
    for (int64_t K = 0; K < g->nc; ++K) {
        const int64_t *c = g->cells + K * g->nvpc;
        double V;
        if (g->ctype == ORC_TRI) {
            const double *a = X(g, c[0]), *b = X(g, c[1]), *e = X(g, c[2]);
            double ux = b[0] - a[0], uy = b[1] - a[1], vx = e[0] - a[0], vy = e[1] - a[1];
            V = 0.5 * fabs(ux * vy - uy * vx);
        } else if (g->ctype == ORC_TET) {
            const double *a = X(g, c[0]), *b = X(g, c[1]), *e = X(g, c[2]), *h = X(g, c[3]);
            double u[3], v[3], w[3], x[3];
            for (int d = 0; d < 3; ++d) { u[d] = b[d] - a[d]; v[d] = e[d] - a[d]; w[d] = h[d] - a[d]; }
            x[0] = v[1] * w[2] - v[2] * w[1];
            x[1] = v[2] * w[0] - v[0] * w[2];
            x[2] = v[0] * w[1] - v[1] * w[0];
            V = fabs(u[0] * x[0] + u[1] * x[1] + u[2] * x[2]) / 6.0;
        } else {
            double acc = 0.0;
            for (int j = 0; j < 6; ++j) {
                double xb[3] = {0, 0, 0}, s[3];
                for (int i = 0; i < 4; ++i) {
                    const double *p = X(g, c[HEX_F[j][i]]);
                    xb[0] = xb[0] + p[0]; xb[1] = xb[1] + p[1]; xb[2] = xb[2] + p[2];
                }
                xb[0] = xb[0] * 0.25; xb[1] = xb[1] * 0.25; xb[2] = xb[2] * 0.25;
                outward(g, K, j, s);
                acc = acc + (xb[0] * s[0] + xb[1] * s[1] + xb[2] * s[2]);
            }
            V = acc / 3.0;
        }
        if (!(V > 0.0)) return ORC_E_MESH;
        g->vol[K] = V;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* dependency graph per direction                                       */
/* ------------------------------------------------------------------ */

/* d = Omega . S evaluated left to right; for cell K's local face j the
 * outward value is d (K is the lower cell / boundary cell) or exactly -d. */
static double face_d(const orc_graph *g, const double *om, int64_t f) {
    return dot3(om, g->S + 3 * f, g->dim);
}

static double out_d(const orc_graph *g, const double *om, int64_t K, int j, int64_t *nbr) {
    int64_t f = g->cface[K * g->nfpc + j];
    double d = face_d(g, om, f);
    if (g->fcell[2 * f] == K) { *nbr = g->fcell[2 * f + 1]; return d; }
    *nbr = g->fcell[2 * f];
    return -d;
}

/* is the in-edge of v through local face j lagged for direction m? */
static int is_lagged(const orc_graph *g, int m, int64_t v, int j) {
    int64_t lo = 0, hi = g->nlag;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        int64_t a = g->lag_m[mid], b = g->lag_v[mid], c = g->lag_face[mid];
        if (a < m || (a == m && (b < v || (b == v && c < j)))) lo = mid + 1;
        else hi = mid;
    }
    return lo < g->nlag && g->lag_m[lo] == m && g->lag_v[lo] == v && g->lag_face[lo] == j;
}

/* Tarjan's strongly connected components (iterative).  comp[v] receives
 * the component id; csize[c] its size. */
static int64_t tarjan(const orc_graph *g, const double *om, int64_t *comp, int64_t *csize) {
    int64_t n = g->nc;
    int64_t *idx = malloc(sizeof(int64_t) * n), *low = malloc(sizeof(int64_t) * n);
    int64_t *stk = malloc(sizeof(int64_t) * n), *cs_v = malloc(sizeof(int64_t) * n);
    int32_t *cs_j = malloc(sizeof(int32_t) * n);
    char *on = calloc((size_t)n, 1);
    int64_t counter = 0, sp = 0, ncomp = 0;
    for (int64_t i = 0; i < n; ++i) idx[i] = -1;
    for (int64_t s = 0; s < n; ++s) {
        if (idx[s] >= 0) continue;
        int64_t csp = 0;
        cs_v[csp] = s; cs_j[csp] = 0; ++csp;
        idx[s] = low[s] = counter++; stk[sp++] = s; on[s] = 1;
        while (csp > 0) {
            int64_t v = cs_v[csp - 1];
            int j = cs_j[csp - 1];
            if (j < g->nfpc) {
                cs_j[csp - 1] = j + 1;
                int64_t w;
                double d = out_d(g, om, v, j, &w);
                if (!(d > 0.0) || w < 0) continue;      /* not a downwind edge */
                if (idx[w] < 0) {
                    idx[w] = low[w] = counter++; stk[sp++] = w; on[w] = 1;
                    cs_v[csp] = w; cs_j[csp] = 0; ++csp;
                } else if (on[w] && idx[w] < low[v]) low[v] = idx[w];
            } else {
                if (low[v] == idx[v]) {
                    int64_t size = 0, w;
                    do { w = stk[--sp]; on[w] = 0; comp[w] = ncomp; ++size; } while (w != v);
                    csize[ncomp++] = size;
                }
                --csp;
                if (csp > 0) {
                    int64_t u = cs_v[csp - 1];
                    if (low[v] < low[u]) low[u] = low[v];
                }
            }
        }
    }
    free(idx); free(low); free(stk); free(cs_v); free(cs_j); free(on);
    return ncomp;
}

typedef struct { int32_t m, j; int64_t u, v; } lag_rec;

static int cmp_lag(const void *a, const void *b) {
    const lag_rec *x = a, *y = b;
    if (x->m != y->m) return x->m < y->m ? -1 : 1;
    if (x->v != y->v) return x->v < y->v ? -1 : 1;
    if (x->j != y->j) return x->j < y->j ? -1 : 1;
    return 0;
}

/* Kahn's algorithm on the non-lagged graph: level(v) = 0 when v has no
 * upwind neighbour, else 1 + the largest upwind level (longest path).
 * tie_seed == 0 drains the ready set in (level, id) order; otherwise the
 * next vertex is drawn at random from the ready set, which yields another
 * valid topological order.  Returns the number of vertices ordered. */
static int64_t kahn(const orc_graph *g, int m, int32_t *level, int32_t *order, uint64_t tie_seed) {
    const double *om = g->omega + 3 * m;
    int64_t n = g->nc;
    int32_t *cnt = calloc((size_t)n, sizeof(int32_t));
    int32_t *ready = malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    for (int64_t K = 0; K < n; ++K)
        for (int j = 0; j < g->nfpc; ++j) {
            int64_t w;
            double d = out_d(g, om, K, j, &w);
            if (d < 0.0 && w >= 0 && !is_lagged(g, m, K, j)) cnt[K]++;
        }
    int64_t head = 0, tail = 0, done = 0;
    for (int64_t K = 0; K < n; ++K) { level[K] = 0; if (cnt[K] == 0) ready[tail++] = (int32_t)K; }
    uint64_t st = tie_seed * 6364136223846793005ULL + 1442695040888963407ULL;
    while (head < tail) {
        int64_t pick = head;
        if (tie_seed) {
            st = st * 6364136223846793005ULL + 1442695040888963407ULL;
            pick = head + (int64_t)((st >> 33) % (uint64_t)(tail - head));
            int32_t t = ready[pick]; ready[pick] = ready[head]; ready[head] = t;
            pick = head;
        }
        int64_t v = ready[head++];
        order[done++] = (int32_t)v;
        for (int j = 0; j < g->nfpc; ++j) {
            int64_t w;
            double d = out_d(g, om, v, j, &w);
            if (!(d > 0.0) || w < 0) continue;
            /* the edge v -> w enters w through w's local face facing v */
            int jw = -1;
            for (int k = 0; k < g->nfpc; ++k)
                if (g->cface[w * g->nfpc + k] == g->cface[v * g->nfpc + j]) jw = k;
            if (is_lagged(g, m, w, jw)) continue;
            if (level[v] + 1 > level[w]) level[w] = level[v] + 1;
            if (--cnt[w] == 0) ready[tail++] = (int32_t)w;
        }
    }
    free(cnt); free(ready);
    return done;
}

static int build_dag(orc_graph *g, int lag_cycles) {
    int64_t n = g->nc;
    int nd = g->nd;
    /* 1. cycles: lag edges u -> v with u > v inside non-trivial SCCs */
    int64_t cap = 64, nl = 0;
    lag_rec *lags = malloc(sizeof(lag_rec) * cap);
    int64_t *comp = malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    int64_t *csize = malloc(sizeof(int64_t) * (size_t)(n ? n : 1));
    for (int m = 0; m < nd; ++m) {
        const double *om = g->omega + 3 * m;
        tarjan(g, om, comp, csize);
        for (int64_t v = 0; v < n; ++v) {
            if (csize[comp[v]] < 2) continue;
            for (int j = 0; j < g->nfpc; ++j) {
                int64_t u;
                double d = out_d(g, om, v, j, &u);
                if (!(d < 0.0) || u < 0) continue;          /* in-edge u -> v */
                if (comp[u] != comp[v] || u < v) continue;  /* kept edge */
                if (!lag_cycles) { free(lags); free(comp); free(csize); return ORC_E_CYCLE; }
                if (nl == cap) { cap *= 2; lags = realloc(lags, sizeof(lag_rec) * cap); }
                lags[nl].m = m; lags[nl].j = j; lags[nl].u = u; lags[nl].v = v; ++nl;
            }
        }
    }
    free(comp); free(csize);
    qsort(lags, (size_t)nl, sizeof(lag_rec), cmp_lag);
    g->nlag = nl;
    g->lag_m = malloc(sizeof(int32_t) * (size_t)(nl ? nl : 1));
    g->lag_face = malloc(sizeof(int32_t) * (size_t)(nl ? nl : 1));
    g->lag_u = malloc(sizeof(int64_t) * (size_t)(nl ? nl : 1));
    g->lag_v = malloc(sizeof(int64_t) * (size_t)(nl ? nl : 1));
    for (int64_t i = 0; i < nl; ++i) {
        g->lag_m[i] = lags[i].m; g->lag_face[i] = lags[i].j; g->lag_u[i] = lags[i].u; g->lag_v[i] = lags[i].v;
    }
    free(lags);
    /* 2. levels and the canonical (level, id) order per direction */
    g->level = malloc(sizeof(int32_t) * (size_t)nd * (size_t)(n ? n : 1));
    g->order = malloc(sizeof(int32_t) * (size_t)nd * (size_t)(n ? n : 1));
    g->nlev = malloc(sizeof(int32_t) * (size_t)(nd ? nd : 1));
    g->lvl_off = malloc(sizeof(int64_t) * (size_t)(nd + 1));
    if (!g->level || !g->order || !g->nlev || !g->lvl_off) return ORC_E_OOM;
    int32_t *tmp = malloc(sizeof(int32_t) * (size_t)(n ? n : 1));
    int64_t total = 0;
    for (int m = 0; m < nd; ++m) {
        int32_t *lev = g->level + (int64_t)m * n;
        if (kahn(g, m, lev, tmp, 0) != n) { free(tmp); return ORC_E_CYCLE; }
        int32_t L = 0;
        for (int64_t K = 0; K < n; ++K) if (lev[K] + 1 > L) L = lev[K] + 1;
        g->nlev[m] = L;
        g->lvl_off[m] = total;
        total += L + 1;
    }
    g->lvl_off[nd] = total;
    g->lvl_ptr = calloc((size_t)(total ? total : 1), sizeof(int64_t));
    for (int m = 0; m < nd; ++m) {
        int32_t *lev = g->level + (int64_t)m * n;
        int64_t *ptr = g->lvl_ptr + g->lvl_off[m];
        int32_t *ord = g->order + (int64_t)m * n;
        for (int64_t K = 0; K < n; ++K) ptr[lev[K] + 1]++;
        for (int32_t l = 0; l < g->nlev[m]; ++l) ptr[l + 1] += ptr[l];
        int64_t *fill = malloc(sizeof(int64_t) * (size_t)(g->nlev[m] + 1));
        memcpy(fill, ptr, sizeof(int64_t) * (size_t)(g->nlev[m] + 1));
        for (int64_t K = 0; K < n; ++K) ord[fill[lev[K]]++] = (int32_t)K;  /* ascending id within a level */
        free(fill);
    }
    free(tmp);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* public entry points                                                  */
/* ------------------------------------------------------------------ */

void orc_free(orc_graph *g) {
    if (!g) return;
    free(g->coords); free(g->cells); free(g->S); free(g->fcell); free(g->cface); free(g->vol);
    free(g->omega); free(g->level); free(g->order); free(g->lvl_off); free(g->lvl_ptr); free(g->nlev);
    free(g->lag_m); free(g->lag_face); free(g->lag_u); free(g->lag_v);
    free(g);
}

/* flags bit 0: refuse cycles (return ORC_E_CYCLE) instead of lagging */
int orc_build(int dim, int ctype, int64_t nv, const double *coords, int64_t nc, const int64_t *cells,
              int nd, const double *omega, int flags, orc_graph **out) {
    *out = NULL;
    if ((dim != 2 && dim != 3) || nv <= 0 || nc <= 0 || nd <= 0 || nc > 2147483647LL) return ORC_E_ARG;
    if (!((dim == 2 && ctype == ORC_TRI) || (dim == 3 && (ctype == ORC_TET || ctype == ORC_HEX)))) return ORC_E_ARG;
    orc_graph *g = calloc(1, sizeof(orc_graph));
    if (!g) return ORC_E_OOM;
    g->dim = dim; g->ctype = ctype; g->nv = nv; g->nc = nc; g->nd = nd;
    g->nvpc = ctype;
    g->nfpc = ctype == ORC_TRI ? 3 : ctype == ORC_TET ? 4 : 6;
    g->coords = malloc(sizeof(double) * (size_t)(nv * dim));
    g->cells = malloc(sizeof(int64_t) * (size_t)(nc * g->nvpc));
    g->omega = malloc(sizeof(double) * 3 * (size_t)nd);
    memcpy(g->coords, coords, sizeof(double) * (size_t)(nv * dim));
    memcpy(g->cells, cells, sizeof(int64_t) * (size_t)(nc * g->nvpc));
    memcpy(g->omega, omega, sizeof(double) * 3 * (size_t)nd);
    if (dim == 2) for (int m = 0; m < nd; ++m) g->omega[3 * m + 2] = 0.0;
    for (int64_t i = 0; i < nc * g->nvpc; ++i)
        if (cells[i] < 0 || cells[i] >= nv) { orc_free(g); return ORC_E_MESH; }
    int rc = build_faces(g);
    if (!rc) rc = build_volumes(g);
    if (!rc) rc = build_dag(g, !(flags & 1));
    if (rc) { orc_free(g); return rc; }
    *out = g;
    return ORC_OK;
}

void orc_sizes(const orc_graph *g, int64_t *out) {
    out[0] = g->nc; out[1] = g->nf; out[2] = g->nd; out[3] = g->nlag; out[4] = g->nfpc;
    int32_t L = 0;
    for (int m = 0; m < g->nd; ++m) if (g->nlev[m] > L) L = g->nlev[m];
    out[5] = L;
}

void orc_geometry(const orc_graph *g, double *S, int64_t *fcell, int64_t *cface, double *vol) {
    if (S) memcpy(S, g->S, sizeof(double) * 3 * (size_t)g->nf);
    if (fcell) memcpy(fcell, g->fcell, sizeof(int64_t) * 2 * (size_t)g->nf);
    if (cface) memcpy(cface, g->cface, sizeof(int64_t) * (size_t)(g->nc * g->nfpc));
    if (vol) memcpy(vol, g->vol, sizeof(double) * (size_t)g->nc);
}

/* per-direction export: in-degree (non-lagged interior in-edges), level,
 * level pointers (nlev+1 entries) and cells ordered by (level, id) */
int orc_dir(const orc_graph *g, int m, int32_t *indeg, int32_t *level, int64_t *lvl_ptr, int64_t *lvl_cells) {
    if (m < 0 || m >= g->nd) return ORC_E_ARG;
    int64_t n = g->nc;
    const double *om = g->omega + 3 * m;
    if (indeg)
        for (int64_t K = 0; K < n; ++K) {
            int32_t c = 0;
            for (int j = 0; j < g->nfpc; ++j) {
                int64_t w;
                double d = out_d(g, om, K, j, &w);
                if (d < 0.0 && w >= 0 && !is_lagged(g, m, K, j)) ++c;
            }
            indeg[K] = c;
        }
    if (level) memcpy(level, g->level + (int64_t)m * n, sizeof(int32_t) * (size_t)n);
    if (lvl_ptr) memcpy(lvl_ptr, g->lvl_ptr + g->lvl_off[m], sizeof(int64_t) * (size_t)(g->nlev[m] + 1));
    if (lvl_cells) for (int64_t i = 0; i < n; ++i) lvl_cells[i] = g->order[(int64_t)m * n + i];
    return g->nlev[m];
}

void orc_lagged(const orc_graph *g, int32_t *m, int64_t *u, int64_t *v, int32_t *face) {
    for (int64_t i = 0; i < g->nlag; ++i) {
        if (m) m[i] = g->lag_m[i];
        if (u) u[i] = g->lag_u[i];
        if (v) v[i] = g->lag_v[i];
        if (face) face[i] = g->lag_face[i];
    }
}

/* One transport sweep of direction m with the step upwind scheme:
 *   psi_K = num / den,
 *   num = V_K s_K + sum over inflow faces (local face order) of a_f psi_up
 *   den = sigma_t,K V_K + sum over outflow faces (local face order) of a_f
 * with a_f = |Omega . S_f|; an inflow boundary face brings psi_b, a lagged
 * in-edge brings the previous iterate psi_prev; faces with Omega . S = 0
 * carry nothing.  Cells are visited in the given topological order. */
static void sweep_dir(const orc_graph *g, int m, const int32_t *order, const double *sigma_t,
                      const double *src, double psi_b, const double *psi_prev, double *psi) {
    int64_t n = g->nc;
    const double *om = g->omega + 3 * m;
    double *pm = psi + (int64_t)m * n;
    const double *pp = psi_prev ? psi_prev + (int64_t)m * n : NULL;
    for (int64_t i = 0; i < n; ++i) {
        int64_t K = order[i];
        double num = g->vol[K] * src[K];
        double den = sigma_t[K] * g->vol[K];
        for (int j = 0; j < g->nfpc; ++j) {
            int64_t w;
            double d = out_d(g, om, K, j, &w);
            if (d < 0.0) {
                double a = -d, up;
                if (w < 0) up = psi_b;
                else if (g->nlag && is_lagged(g, m, K, j)) up = pp ? pp[w] : 0.0;
                else up = pm[w];
                num = num + a * up;
            } else if (d > 0.0) {
                den = den + d;
            }
        }
        pm[K] = num / den;
    }
}

/* Sweep all directions.  src is [nc] (isotropic) or [nd*nc] when
 * src_per_dir != 0.  tie_seed != 0 uses a random valid topological order
 * per direction (seeded) instead of the (level, id) order. */
int orc_sweep(const orc_graph *g, const double *sigma_t, const double *src, int src_per_dir, double psi_b,
              const double *psi_prev, double *psi, uint64_t tie_seed) {
    int64_t n = g->nc;
    int32_t *ord = malloc(sizeof(int32_t) * (size_t)n);
    int32_t *lev = malloc(sizeof(int32_t) * (size_t)n);
    for (int m = 0; m < g->nd; ++m) {
        const int32_t *o = g->order + (int64_t)m * n;
        if (tie_seed) { kahn(g, m, lev, ord, tie_seed + (uint64_t)m); o = ord; }
        sweep_dir(g, m, o, sigma_t, src_per_dir ? src + (int64_t)m * n : src, psi_b, psi_prev, psi);
    }
    free(ord); free(lev);
    return ORC_OK;
}

/* Sweep a subset of directions [m0, m1) only (the rest of psi untouched). */
int orc_sweep_dirs(const orc_graph *g, int m0, int m1, const double *sigma_t, const double *src, int src_per_dir,
                   double psi_b, const double *psi_prev, double *psi) {
    if (m0 < 0 || m1 > g->nd || m0 > m1) return ORC_E_ARG;
    for (int m = m0; m < m1; ++m)
        sweep_dir(g, m, g->order + (int64_t)m * g->nc, sigma_t, src_per_dir ? src + (int64_t)m * g->nc : src,
                  psi_b, psi_prev, psi);
    return ORC_OK;
}

/* Scalar flux phi_K = sum_m w_m psi_{K,m}, summed in ascending m. */
void orc_phi(const orc_graph *g, const double *w, const double *psi, double *phi) {
    for (int64_t K = 0; K < g->nc; ++K) {
        double s = 0.0;
        for (int m = 0; m < g->nd; ++m) s = s + w[m] * psi[(int64_t)m * g->nc + K];
        phi[K] = s;
    }
}

/* Residual of the discrete transport equation with the full (un-lagged)
 * streaming operator:
 *   r_{K,m} = q_K + sigma_s,K phi_K - (den psi_{K,m} - in_{K,m}) / V_K
 * with den as in the sweep and in_{K,m} the sum of a_f psi_up over all
 * inflow faces (boundary faces bring psi_b).  Returns
 * rho = ||r|| / ||q|| with ||x||^2 = sum_K V_K sum_m w_m x_{K,m}^2 and
 * ||q||^2 = sum_K V_K q_K^2 (rho = ||r|| when q = 0).  r may be NULL. */
double orc_residual(const orc_graph *g, const double *sigma_t, const double *sigma_s, const double *q, double psi_b,
                    const double *w, const double *psi, const double *phi, double *r) {
    int64_t n = g->nc;
    double rr = 0.0, qq = 0.0;
    for (int64_t K = 0; K < n; ++K) {
        double cell = 0.0;
        for (int m = 0; m < g->nd; ++m) {
            const double *om = g->omega + 3 * m;
            const double *pm = psi + (int64_t)m * n;
            double in = 0.0, den = sigma_t[K] * g->vol[K];
            for (int j = 0; j < g->nfpc; ++j) {
                int64_t nb;
                double d = out_d(g, om, K, j, &nb);
                if (d < 0.0) in = in + (-d) * (nb < 0 ? psi_b : pm[nb]);
                else if (d > 0.0) den = den + d;
            }
            double res = (q[K] + sigma_s[K] * phi[K]) - (den * pm[K] - in) / g->vol[K];
            if (r) r[(int64_t)m * n + K] = res;
            cell = cell + w[m] * (res * res);
        }
        rr = rr + g->vol[K] * cell;
        qq = qq + g->vol[K] * (q[K] * q[K]);
    }
    return qq > 0.0 ? sqrt(rr) / sqrt(qq) : sqrt(rr);
}

/* Source iteration from psi = phi = 0:
 *   s = q + sigma_s phi;  sweep every direction (lagged in-edges take the
 *   previous iterate);  phi = sum_m w_m psi_m;  rho = residual.
 * Stops after max_iter iterations or once rho <= tol (tol <= 0: run all).
 * hist (may be NULL) receives rho per iteration.  Returns iterations done. */
int orc_si(const orc_graph *g, const double *sigma_t, const double *sigma_s, const double *q, double psi_b,
           const double *w, int max_iter, double tol, double *psi, double *phi, double *hist) {
    int64_t n = g->nc, N = n * g->nd;
    double *s = malloc(sizeof(double) * (size_t)n);
    double *prev = g->nlag ? malloc(sizeof(double) * (size_t)N) : NULL;
    memset(psi, 0, sizeof(double) * (size_t)N);
    memset(phi, 0, sizeof(double) * (size_t)n);
    int it = 0;
    while (it < max_iter) {
        for (int64_t K = 0; K < n; ++K) s[K] = q[K] + sigma_s[K] * phi[K];
        if (prev) memcpy(prev, psi, sizeof(double) * (size_t)N);
        orc_sweep(g, sigma_t, s, 0, psi_b, prev, psi, 0);
        orc_phi(g, w, psi, phi);
        double rho = orc_residual(g, sigma_t, sigma_s, q, psi_b, w, psi, phi, NULL);
        if (hist) hist[it] = rho;
        ++it;
        if (tol > 0.0 && rho <= tol) break;
    }
    free(s); free(prev);
    return it;
}

/* ------------------------------------------------------------------ */
/* multigroup                                                           */
/* ------------------------------------------------------------------ */

/* Multigroup transport with isotropic scattering between energy groups
 * (the appendix form of the transport equation: a flux per ordinate m and
 * group g, collisions coupling every (m', g') into (m, g) through the
 * direction weights and a group-to-group scattering cross section):
 *   Omega_m . grad psi_{m,g} + sigma_t,g psi_{m,g}
 *       = q_g + sum_{g'} sigma_s,g'->g phi_{g'},   phi_g = sum_m w_m psi_{m,g}.
 * Layouts: sigma_t, q, phi [G][nc]; sigma_s [G][G][nc] with the cross
 * section from group g' into group g at (g' * G + g) * nc + K; psi
 * [G][nd][nc].  Every group uses the same sweep graph (the geometry and
 * the directions do not depend on the energy). */

/* Group source s_{K,g} = q_{K,g} + sum over g' (ascending) of
 * sigma_s,g'->g,K phi_{K,g'}. */
static void mg_source(const orc_graph *g, int G, const double *sigma_s, const double *q, const double *phi,
                      int grp, double *s) {
    int64_t n = g->nc;
    for (int64_t K = 0; K < n; ++K) {
        double v = q[(int64_t)grp * n + K];
        for (int gp = 0; gp < G; ++gp)
            v = v + sigma_s[((int64_t)gp * G + grp) * n + K] * phi[(int64_t)gp * n + K];
        s[K] = v;
    }
}

/* Residual of the multigroup equations with the full (un-lagged)
 * streaming operator:
 *   r_{K,m,g} = s_{K,g} - (den_g psi_{K,m,g} - in_{K,m,g}) / V_K
 * with s the group source above (from the given phi), den_g and in as in
 * the single-group residual with sigma_t,g.  Returns
 * rho = sqrt(sum_g sum_K V_K sum_m w_m r^2) / sqrt(sum_g sum_K V_K q_g^2)
 * (without the denominator when q = 0). */
double orc_mg_residual(const orc_graph *g, int G, const double *sigma_t, const double *sigma_s, const double *q,
                       double psi_b, const double *w, const double *psi, const double *phi) {
    int64_t n = g->nc, N = n * g->nd;
    double *s = malloc(sizeof(double) * (size_t)n);
    double rr = 0.0, qq = 0.0;
    for (int grp = 0; grp < G; ++grp) {
        mg_source(g, G, sigma_s, q, phi, grp, s);
        const double *st = sigma_t + (int64_t)grp * n;
        const double *pg = psi + (int64_t)grp * N;
        for (int64_t K = 0; K < n; ++K) {
            double cell = 0.0;
            for (int m = 0; m < g->nd; ++m) {
                const double *om = g->omega + 3 * m;
                const double *pm = pg + (int64_t)m * n;
                double in = 0.0, den = st[K] * g->vol[K];
                for (int j = 0; j < g->nfpc; ++j) {
                    int64_t nb;
                    double d = out_d(g, om, K, j, &nb);
                    if (d < 0.0) in = in + (-d) * (nb < 0 ? psi_b : pm[nb]);
                    else if (d > 0.0) den = den + d;
                }
                double res = s[K] - (den * pm[K] - in) / g->vol[K];
                cell = cell + w[m] * (res * res);
            }
            double qk = q[(int64_t)grp * n + K];
            rr = rr + g->vol[K] * cell;
            qq = qq + g->vol[K] * (qk * qk);
        }
    }
    free(s);
    return qq > 0.0 ? sqrt(rr) / sqrt(qq) : sqrt(rr);
}

/* Multigroup source iteration from psi = phi = 0, Jacobi over groups
 * (every group's source from the previous iterate of all groups, then the
 * sweeps of every direction and group):
 *   s_g = q_g + sum_g' sigma_s,g'->g phi_g';  sweep (m, g) for all m, g
 *   (lagged in-edges take the previous iterate of the same group);
 *   phi_g = sum_m w_m psi_{m,g};  rho = multigroup residual.
 * Stops after max_iter iterations or once rho <= tol (tol <= 0: run all);
 * hist (may be NULL) receives rho per iteration.  Returns iterations done. */
int orc_mg_si(const orc_graph *g, int G, const double *sigma_t, const double *sigma_s, const double *q, double psi_b,
              const double *w, int max_iter, double tol, double *psi, double *phi, double *hist) {
    int64_t n = g->nc, N = n * g->nd;
    double *s = malloc(sizeof(double) * (size_t)n * (size_t)G);
    double *prev = g->nlag ? malloc(sizeof(double) * (size_t)N) : NULL;
    memset(psi, 0, sizeof(double) * (size_t)N * (size_t)G);
    memset(phi, 0, sizeof(double) * (size_t)n * (size_t)G);
    int it = 0;
    while (it < max_iter) {
        for (int grp = 0; grp < G; ++grp) mg_source(g, G, sigma_s, q, phi, grp, s + (int64_t)grp * n);
        for (int grp = 0; grp < G; ++grp) {
            double *pg = psi + (int64_t)grp * N;
            if (prev) memcpy(prev, pg, sizeof(double) * (size_t)N);
            orc_sweep(g, sigma_t + (int64_t)grp * n, s + (int64_t)grp * n, 0, psi_b, prev, pg, 0);
            orc_phi(g, w, pg, phi + (int64_t)grp * n);
        }
        double rho = orc_mg_residual(g, G, sigma_t, sigma_s, q, psi_b, w, psi, phi);
        if (hist) hist[it] = rho;
        ++it;
        if (tol > 0.0 && rho <= tol) break;
    }
    free(s); free(prev);
    return it;
}
