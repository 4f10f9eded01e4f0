"""Seeded synthetic inputs for the data-driven transport sweep.

This module produces *inputs only*: vertex coordinates and cell connectivity
of meshes, discrete-ordinates quadratures (directions and weights) and
per-cell material data.  It contains none of the sweep method's arithmetic
(no face areas, volumes, dependency graphs, sweeps or iterations), so that
the oracle and the HIP path can both consume it without sharing any of the
computation they are compared on.

The mesh families stand in for the paper's workloads (structured cube meshes
and unstructured tetrahedral / triangular meshes, Sec. VI); the paper's own
benchmark meshes are not reproduced.

Conventions (stated here because the generated arrays depend on them):

* vertex coordinates are row-major ``[n_vertices, dim]`` float64;
* cells are ``[n_cells, verts_per_cell]`` int64;
* hexahedron corner ``c`` (0..7) sits at lattice offset
  ``(c >> 2 & 1, c >> 1 & 1, c & 1)`` along (x, y, z);
* lattice vertex ``(i, j, k)`` has id ``(i * (n + 1) + j) * (n + 1) + k``
  and lattice cube ``(i, j, k)`` has index ``(i * n + j) * n + k``;
* quadrature directions are unit 3-vectors; 2D problems keep the upper
  hemisphere (Omega_z > 0) and stream with (Omega_x, Omega_y);
  weights always sum to 1.

Random numbers come from ``numpy.random.default_rng`` (PCG64) with the seed
given by the caller; draws happen in a fixed order documented per function.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field
from functools import lru_cache

import numpy as np

GENERATOR_VERSION = 1

TRI, TET, HEX = 3, 4, 8


# --------------------------------------------------------------------------
# Quadrature: level-symmetric LQ_N
# --------------------------------------------------------------------------

def _double_factorial_odd(n: int) -> int:
    """(n-1)!! for even n >= 0 written as prod of odd numbers below n."""
    r = 1
    for k in range(1, n, 2):
        r *= k
    return r


def sphere_moment(a: int, b: int, c: int) -> float:
    """Exact average of Omega_x^a Omega_y^b Omega_z^c over the unit sphere
    (zero unless all exponents are even)."""
    if a % 2 or b % 2 or c % 2:
        return 0.0
    num = _double_factorial_odd(a) * _double_factorial_odd(b) * _double_factorial_odd(c)
    den = 1
    for k in range(1, a + b + c + 2, 2):
        den *= k
    return num / den


def _octant_points(N: int):
    """Index triples (i, j, k) >= 1 with i + j + k = N/2 + 2, lexicographic."""
    s = N // 2 + 2
    pts = []
    for i in range(1, N // 2 + 1):
        for j in range(1, N // 2 + 1):
            k = s - i - j
            if 1 <= k <= N // 2:
                pts.append((i, j, k))
    return pts


def _level_cosines(N: int, mu1: float) -> np.ndarray:
    n = N // 2
    mu2 = np.array([mu1 * mu1 + (i * 2.0 * (1.0 - 3.0 * mu1 * mu1)) / (N - 2) for i in range(n)])
    return np.sqrt(mu2)


def _moment_system(N: int, mu1: float):
    """Rows: even moments (2a,2b,2c), 2(a+b+c) <= N; columns: weight classes.
    Returns (A, rhs, classes, pts)."""
    pts = _octant_points(N)
    classes = sorted({tuple(sorted(p)) for p in pts})
    cls_idx = [classes.index(tuple(sorted(p))) for p in pts]
    mu = _level_cosines(N, mu1)
    rows, rhs = [], []
    for a in range(0, N // 2 + 1):
        for b in range(0, N // 2 + 1 - a):
            for c in range(0, N // 2 + 1 - a - b):
                row = np.zeros(len(classes))
                for p, ci in zip(pts, cls_idx):
                    row[ci] += mu[p[0] - 1] ** (2 * a) * mu[p[1] - 1] ** (2 * b) * mu[p[2] - 1] ** (2 * c)
                rows.append(row)
                rhs.append(sphere_moment(2 * a, 2 * b, 2 * c))
    return np.array(rows), np.array(rhs), classes, pts


# First level cosine: S4..S8 follow from exact integration of the even
# moments (solved below); S16 uses the commonly tabulated LQ16 value, with
# weights fitted to the even moments in the least-squares sense.
_MU1_GUESS = {4: 0.3500212, 6: 0.2666355, 8: 0.2182179, 12: 0.1672126, 16: 0.1389568}
_MU1_FIXED = {16: 0.1389568}


@lru_cache(maxsize=None)
def _lq_octant(N: int):
    """Solve for (mu1, class weights) of LQ_N; octant-normalised weights.

    For each trial mu1 the class weights are the least-squares fit of the
    even-moment system; mu1 minimises the remaining moment residual (for
    S4-S8 the minimum is an exact zero, i.e. all even moments up to degree N
    are integrated exactly).  S16 keeps the tabulated mu1."""
    from scipy.optimize import brentq, minimize_scalar

    def fit(mu1):
        A, rhs, classes, pts = _moment_system(N, mu1)
        w, *_ = np.linalg.lstsq(A, rhs, rcond=None)
        return A, rhs, w, classes, pts

    def resid(mu1):
        A, rhs, w, _, _ = fit(mu1)
        return float(np.linalg.norm(A @ w - rhs))

    if N in _MU1_FIXED:
        mu1 = _MU1_FIXED[N]
    else:
        guess = _MU1_GUESS[N]
        xs = np.linspace(guess * 0.98, guess * 1.02, 81)
        x0 = xs[int(np.argmin([resid(x) for x in xs]))]
        step = xs[1] - xs[0]
        res = minimize_scalar(resid, bounds=(x0 - step, x0 + step), method="bounded",
                              options={"xatol": 1e-14})
        mu1 = float(res.x)
        # polish on the signed residual component that crosses zero there
        lo, hi = mu1 - 1e-6, mu1 + 1e-6
        rlo = fit(lo)[0] @ fit(lo)[2] - fit(lo)[1]
        rhi = fit(hi)[0] @ fit(hi)[2] - fit(hi)[1]
        i = int(np.argmax(np.abs(rlo) + np.abs(rhi)))
        if rlo[i] * rhi[i] < 0:
            def comp(x):
                A, rhs, w, _, _ = fit(x)
                return float((A @ w - rhs)[i])
            mu1 = float(brentq(comp, lo, hi, xtol=1e-17, rtol=4 * np.finfo(float).eps))
    A, rhs, w, classes, pts = fit(mu1)
    return mu1, w, classes, pts


def quadrature(N: int, dim: int = 3):
    """Level-symmetric LQ_N quadrature.

    Returns ``(omega [n,3] float64, weight [n] float64)``; 3D has N(N+2)
    directions, 2D keeps the Omega_z > 0 half.  Directions are ordered by
    octant (sign bits of x, y, z with bit set for negative) and, within an
    octant, by the lexicographic level-index triple."""
    if N not in (2, 4, 6, 8, 12, 16):
        raise ValueError(f"unsupported S_N order {N}")
    if N == 2:
        mu1 = 1.0 / math.sqrt(3.0)
        classes, pts, w = [(1, 1, 1)], [(1, 1, 1)], np.array([1.0])
    else:
        mu1, w, classes, pts = _lq_octant(N)
    mu = _level_cosines(N, mu1) if N > 2 else np.array([mu1])
    om, wt = [], []
    for octant in range(8):
        sx = -1.0 if octant & 4 else 1.0
        sy = -1.0 if octant & 2 else 1.0
        sz = -1.0 if octant & 1 else 1.0
        if dim == 2 and sz < 0:
            continue
        for p in pts:
            v = np.array([sx * mu[p[0] - 1], sy * mu[p[1] - 1], sz * mu[p[2] - 1]])
            v = v / np.linalg.norm(v)
            om.append(v)
            wt.append(w[classes.index(tuple(sorted(p)))])
    om = np.array(om, dtype=np.float64)
    wt = np.array(wt, dtype=np.float64)
    wt = wt / wt.sum()
    return np.ascontiguousarray(om), np.ascontiguousarray(wt)


def octant_of(omega: np.ndarray) -> np.ndarray:
    """Octant index (bit 2: x<0, bit 1: y<0, bit 0: z<0) of each direction."""
    om = np.asarray(omega)
    return ((om[:, 0] < 0) * 4 + (om[:, 1] < 0) * 2 + (om[:, 2] < 0)).astype(np.int32)


# --------------------------------------------------------------------------
# Meshes
# --------------------------------------------------------------------------

@dataclass
class Mesh:
    dim: int
    cell_type: int
    coords: np.ndarray       # [nv, dim] float64
    cells: np.ndarray        # [nc, vpc] int64
    lattice_n: int = 0       # cubes per axis for lattice meshes, else 0
    parent_cube: np.ndarray | None = None  # lattice cube index of each cell

    @property
    def n_vertices(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_cells(self) -> int:
        return int(self.cells.shape[0])


def _lattice_vertices(n: int, jitter: float, rng) -> np.ndarray:
    """(n+1)^3 lattice on the unit cube; interior vertices moved by
    U[-jitter*h, +jitter*h] per coordinate (boundary vertices fixed)."""
    h = 1.0 / n
    g = np.arange(n + 1, dtype=np.float64) * h
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    if jitter > 0:
        d = rng.uniform(-jitter * h, jitter * h, size=xyz.shape)
        idx = np.arange(n + 1)
        I, J, K = np.meshgrid(idx, idx, idx, indexing="ij")
        interior = ((I > 0) & (I < n) & (J > 0) & (J < n) & (K > 0) & (K < n)).ravel()
        xyz[interior] += d[interior]
    return np.ascontiguousarray(xyz)


def _vid(n: int, i, j, k):
    return (i * (n + 1) + j) * (n + 1) + k


def hex_lattice(n: int, jitter: float = 0.0, seed: int = 0) -> Mesh:
    """n^3 hexahedra on the unit cube (vertex draw first, one rng stream)."""
    rng = np.random.default_rng(seed)
    xyz = _lattice_vertices(n, jitter, rng)
    idx = np.arange(n)
    I, J, K = np.meshgrid(idx, idx, idx, indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    cells = np.empty((n ** 3, 8), dtype=np.int64)
    for c in range(8):
        bx, by, bz = (c >> 2) & 1, (c >> 1) & 1, c & 1
        cells[:, c] = _vid(n, I + bx, J + by, K + bz)
    return Mesh(3, HEX, xyz, cells, n, np.arange(n ** 3, dtype=np.int64))


# Kuhn / Freudenthal split: one tetrahedron per permutation of the axes,
# walking from cube corner (0,0,0) to (1,1,1) one axis at a time.
_KUHN_PERMS = list(itertools.permutations(range(3)))


def kuhn_tets(n: int, jitter: float = 0.0, seed: int = 0) -> Mesh:
    """n^3 lattice cubes, each split into 6 tetrahedra around its main
    diagonal; conforming across cubes.  Cell order: cube-major, then the
    permutation index."""
    rng = np.random.default_rng(seed)
    xyz = _lattice_vertices(n, jitter, rng)
    idx = np.arange(n)
    I, J, K = np.meshgrid(idx, idx, idx, indexing="ij")
    base = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
    cells = np.empty((n ** 3, 6, 4), dtype=np.int64)
    for t, perm in enumerate(_KUHN_PERMS):
        off = np.zeros(3, dtype=np.int64)
        cells[:, t, 0] = _vid(n, base[:, 0], base[:, 1], base[:, 2])
        for s in range(3):
            off[perm[s]] += 1
            cells[:, t, s + 1] = _vid(n, base[:, 0] + off[0], base[:, 1] + off[1], base[:, 2] + off[2])
    parent = np.repeat(np.arange(n ** 3, dtype=np.int64), 6)
    return Mesh(3, TET, xyz, cells.reshape(-1, 4), n, parent)


def jittered_points_2d(nx: int, ny: int, jitter: float, rng) -> np.ndarray:
    """nx*ny lattice points on [0,1]^2; interior points moved by
    U[-jitter*h, jitter*h] per axis; edge points move only along their edge;
    the four corners stay fixed."""
    hx, hy = 1.0 / (nx - 1), 1.0 / (ny - 1)
    X, Y = np.meshgrid(np.arange(nx) * hx, np.arange(ny) * hy, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    dx = rng.uniform(-jitter * hx, jitter * hx, size=nx * ny)
    dy = rng.uniform(-jitter * hy, jitter * hy, size=nx * ny)
    I, J = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    I, J = I.ravel(), J.ravel()
    move_x = (I > 0) & (I < nx - 1)   # not on the left / right edge
    move_y = (J > 0) & (J < ny - 1)   # not on the bottom / top edge
    pts[move_x, 0] += dx[move_x]
    pts[move_y, 1] += dy[move_y]
    return np.ascontiguousarray(pts)


def delaunay_2d(nx: int, ny: int, jitter: float = 0.3, seed: int = 0) -> Mesh:
    """Delaunay triangulation (scipy / Qhull) of a jittered nx*ny point set."""
    from scipy.spatial import Delaunay

    rng = np.random.default_rng(seed)
    pts = jittered_points_2d(nx, ny, jitter, rng)
    tri = Delaunay(pts)
    if len(getattr(tri, "coplanar", [])) != 0:
        raise RuntimeError("Delaunay dropped points")
    cells = np.ascontiguousarray(tri.simplices.astype(np.int64))
    used = np.unique(cells)
    if used.size != pts.shape[0]:
        raise RuntimeError("Delaunay left points unused")
    return Mesh(2, TRI, pts, cells, 0, None)


# --------------------------------------------------------------------------
# Problems (mesh + quadrature + materials)
# --------------------------------------------------------------------------

@dataclass
class Problem:
    name: str
    mesh: Mesh
    omega: np.ndarray
    weight: np.ndarray
    sigma_t: np.ndarray
    sigma_s: np.ndarray
    q: np.ndarray
    psi_boundary: float = 0.0
    n_iter: int = 0              # source iterations for fixed-count parity runs
    tol: float = 1e-8
    meta: dict = field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        return self.mesh.n_cells

    @property
    def n_dirs(self) -> int:
        return int(self.omega.shape[0])


def delaunay_problem(seed: int = 1, nx: int = 40, ny: int = 50, sn: int = 4) -> Problem:
    """2D Delaunay of nx*ny jittered points, S_N 2D, sigma_t ~ U[0.5, 2],
    scattering ratio 0.5, q = 1, vacuum.  Draw order: coords, sigma_t."""
    rng = np.random.default_rng(seed)
    from scipy.spatial import Delaunay
    pts = jittered_points_2d(nx, ny, 0.3, rng)
    tri = Delaunay(pts)
    cells = np.ascontiguousarray(tri.simplices.astype(np.int64))
    if np.unique(cells).size != pts.shape[0]:
        raise RuntimeError("Delaunay left points unused")
    mesh = Mesh(2, TRI, pts, cells)
    nc = mesh.n_cells
    st = rng.uniform(0.5, 2.0, size=nc)
    om, w = quadrature(sn, 2)
    return Problem(f"delaunay{nx}x{ny}_s{sn}", mesh, om, w, st, 0.5 * st, np.ones(nc), 0.0, 20)


def hex_problem(seed: int = 2, n: int = 64, sn: int = 8, jitter: float = 0.15, c: float = 0.9) -> Problem:
    """Jittered n^3 hex lattice, S_N, sigma_t = exp(N(0, 0.5^2)) per cell,
    scattering ratio c, q = 1 in the central cubes [n/4, 3n/4)^3 else 0,
    vacuum.  Draw order: coords, sigma_t."""
    rng = np.random.default_rng(seed)
    xyz = _lattice_vertices(n, jitter, rng)
    base = hex_lattice(n, 0.0)
    mesh = Mesh(3, HEX, xyz, base.cells, n, base.parent_cube)
    nc = mesh.n_cells
    st = np.exp(rng.normal(0.0, 0.5, size=nc))
    idx = np.arange(n)
    I, J, K = np.meshgrid(idx, idx, idx, indexing="ij")
    lo, hi = n // 4, 3 * n // 4
    inside = ((I >= lo) & (I < hi) & (J >= lo) & (J < hi) & (K >= lo) & (K < hi)).ravel()
    q = inside.astype(np.float64)
    om, w = quadrature(sn, 3)
    return Problem(f"hex{n}_s{sn}", mesh, om, w, st, c * st, q, 0.0, 20)


def checkerboard_tet_problem(seed: int = 3, n: int = 96, sn: int = 8, blocks: int = 8) -> Problem:
    """Kuhn-split jittered n^3 lattice (jitter 0.15h), S_N, checkerboard of
    blocks^3 material blocks by parity of the block index: even -> sigma_t 1,
    c 0.5; odd -> sigma_t 10, c 0.99; q = 1; vacuum.  Draw order: coords."""
    mesh = kuhn_tets(n, 0.15, seed)
    cube = mesh.parent_cube
    i, j, k = cube // (n * n), (cube // n) % n, cube % n
    bsz = n // blocks
    odd = ((i // bsz + j // bsz + k // bsz) % 2).astype(bool)
    st = np.where(odd, 10.0, 1.0)
    c = np.where(odd, 0.99, 0.5)
    om, w = quadrature(sn, 3)
    return Problem(f"tetcheck{n}_s{sn}", mesh, om, w, st, c * st, np.ones(mesh.n_cells), 0.0, 20)


def lognormal_tet_problem(seed: int = 5, n: int = 60, sn: int = 16, c: float = 0.95, s: float = 1.0) -> Problem:
    """Kuhn-split jittered n^3 lattice (jitter 0.15h), S_N, sigma_t =
    exp(N(0, s^2)) per cell, scattering ratio c, q = 1, vacuum.
    Draw order: coords, sigma_t."""
    rng = np.random.default_rng(seed)
    xyz = _lattice_vertices(n, 0.15, rng)
    base = kuhn_tets(n, 0.0)
    mesh = Mesh(3, TET, xyz, base.cells, n, base.parent_cube)
    st = np.exp(rng.normal(0.0, s, size=mesh.n_cells))
    om, w = quadrature(sn, 3)
    return Problem(f"tetlogn{n}_s{sn}", mesh, om, w, st, c * st, np.ones(mesh.n_cells), 0.0, 20)


def ensemble(seed: int = 4, count: int = 256, min_cells: int = 500, max_cells: int = 50000):
    """Ensemble of independent problems.  Instance i uses its own stream
    ``default_rng([seed, i])`` and draws, in order: target size (log-uniform),
    S_N order from {4, 6, 8}, scattering ratio U[0, 0.95], coordinates,
    sigma_t ~ U[0.1, 5] per cell.  Even i: 2D Delaunay of a jittered
    sqrt(N/2)-per-side point lattice; odd i: Kuhn tets of an
    n = max(2, round((N/6)^(1/3))) lattice.  q = 1, vacuum."""
    from scipy.spatial import Delaunay
    out = []
    for i in range(count):
        rng = np.random.default_rng([seed, i])
        target = math.exp(rng.uniform(math.log(min_cells), math.log(max_cells)))
        sn = int(rng.choice([4, 6, 8]))
        c = float(rng.uniform(0.0, 0.95))
        if i % 2 == 0:
            side = max(3, int(round(math.sqrt(target / 2.0))) + 1)
            pts = jittered_points_2d(side, side, 0.3, rng)
            tri = Delaunay(pts)
            cells = np.ascontiguousarray(tri.simplices.astype(np.int64))
            mesh = Mesh(2, TRI, pts, cells)
            om, w = quadrature(sn, 2)
        else:
            n = max(2, int(round((target / 6.0) ** (1.0 / 3.0))))
            xyz = _lattice_vertices(n, 0.15, rng)
            base = kuhn_tets(n, 0.0)
            mesh = Mesh(3, TET, xyz, base.cells, n, base.parent_cube)
            om, w = quadrature(sn, 3)
        st = rng.uniform(0.1, 5.0, size=mesh.n_cells)
        out.append(Problem(f"ens{i}", mesh, om, w, st, c * st, np.ones(mesh.n_cells), 0.0, 0,
                           meta={"sn": sn, "c": c}))
    return out


@dataclass
class MultigroupProblem:
    """Multigroup inputs on one mesh and quadrature: sigma_t, q [G, nc] and
    the isotropic scattering cross sections sigma_s [G, G, nc] from group g'
    (first index) into group g (second index)."""
    name: str
    mesh: Mesh
    omega: np.ndarray
    weight: np.ndarray
    sigma_t: np.ndarray
    sigma_s: np.ndarray
    q: np.ndarray
    psi_boundary: float = 0.0

    @property
    def n_cells(self) -> int:
        return self.mesh.n_cells

    @property
    def n_dirs(self) -> int:
        return int(self.omega.shape[0])

    @property
    def n_groups(self) -> int:
        return int(self.sigma_t.shape[0])


def multigroup(base: Problem, groups: int = 4, seed: int = 7) -> MultigroupProblem:
    """Synthetic multigroup data on a single-group problem's mesh and
    quadrature (the paper's unstructured runs use 4 energy groups).
    Group g has sigma_t,g = f_g sigma_t with f = 0.5, 0.8, 1.2, 2.0, 3.0, ...
    (x1.5 per further group) and source q_g = q / 2^g.  Its scattering
    ratio is the base problem's c = sigma_s / sigma_t per cell; that total
    is shared between destinations in proportions 0.75 (same group), 0.20
    (next group, downscatter) and 0.05 (previous group, upscatter), each
    proportion times a per-cell factor U[0.8, 1.2], renormalised over the
    destinations that exist.  Draw order: one [G, 3, nc] array of factors."""
    rng = np.random.default_rng(seed)
    G, nc = int(groups), base.n_cells
    f = [0.5, 0.8, 1.2, 2.0]
    while len(f) < G:
        f.append(f[-1] * 1.5)
    c = np.where(base.sigma_t > 0, base.sigma_s / base.sigma_t, 0.0)
    fac = rng.uniform(0.8, 1.2, size=(G, 3, nc))
    st = np.stack([base.sigma_t * f[g] for g in range(G)])
    ss = np.zeros((G, G, nc))
    for g in range(G):
        share = np.zeros((3, nc))
        share[0] = 0.75 * fac[g, 0]
        if g + 1 < G:
            share[1] = 0.20 * fac[g, 1]
        if g - 1 >= 0:
            share[2] = 0.05 * fac[g, 2]
        share /= share.sum(axis=0)
        tot = c * st[g]
        ss[g, g] = tot * share[0]
        if g + 1 < G:
            ss[g, g + 1] = tot * share[1]
        if g - 1 >= 0:
            ss[g, g - 1] = tot * share[2]
    q = np.stack([base.q / (2.0 ** g) for g in range(G)])
    return MultigroupProblem(f"{base.name}_g{G}", base.mesh, base.omega, base.weight, st, ss, q, base.psi_boundary)


def config(k: int, scale: str = "full") -> Problem:
    """The five benchmark configurations (k = 1..5; 4 is ``ensemble``).

    ``scale='small'`` shrinks the 3D lattices so the oracle finishes in
    seconds while keeping each configuration's structure."""
    small = scale == "small"
    if k == 1:
        return delaunay_problem(1, 40, 50, 4)
    if k == 2:
        return hex_problem(2, 12 if small else 64, 8)
    if k == 3:
        return checkerboard_tet_problem(3, 16 if small else 96, 8, 8)
    if k == 5:
        return lognormal_tet_problem(5, 8 if small else 60, 16)
    raise ValueError("config 4 is an ensemble; use ensemble()")
