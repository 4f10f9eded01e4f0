"""Python access to the oracle (``oracle.c``): a plain serial FP64 CPU
implementation of the transport sweep path.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark; never by the product package.

``build()`` compiles ``oracle.c`` with gcc, without FMA contraction and
without host-specific instruction sets, into ``oracle/_build/liboracle.so``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_OUT_DIR = os.path.join(_HERE, "_build")
_LIB = os.path.join(_OUT_DIR, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle shared library; returns its path."""
    os.makedirs(_OUT_DIR, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build(force=False)
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.orc_build.argtypes = [i32, i32, i64, P, i64, P, i32, P, i32, ctypes.POINTER(P)]
    lib.orc_build.restype = i32
    lib.orc_free.argtypes = [P]
    lib.orc_sizes.argtypes = [P, P]
    lib.orc_geometry.argtypes = [P, P, P, P, P]
    lib.orc_dir.argtypes = [P, i32, P, P, P, P]
    lib.orc_dir.restype = i32
    lib.orc_lagged.argtypes = [P, P, P, P, P]
    lib.orc_sweep.argtypes = [P, P, P, i32, dbl, P, P, ctypes.c_uint64]
    lib.orc_sweep.restype = i32
    lib.orc_sweep_dirs.argtypes = [P, i32, i32, P, P, i32, dbl, P, P]
    lib.orc_sweep_dirs.restype = i32
    lib.orc_phi.argtypes = [P, P, P, P]
    lib.orc_residual.argtypes = [P, P, P, P, dbl, P, P, P, P]
    lib.orc_residual.restype = dbl
    lib.orc_si.argtypes = [P, P, P, P, dbl, P, i32, dbl, P, P, P]
    lib.orc_si.restype = i32
    lib.orc_mg_residual.argtypes = [P, i32, P, P, P, dbl, P, P, P]
    lib.orc_mg_residual.restype = dbl
    lib.orc_mg_si.argtypes = [P, i32, P, P, P, dbl, P, i32, dbl, P, P, P]
    lib.orc_mg_si.restype = i32
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    pass


class Graph:
    """Oracle graph: geometry, per-direction DAG, lag rule and levels."""

    def __init__(self, mesh, omega, refuse_cycles: bool = False):
        lib = _load()
        self._lib = lib
        self.dim, self.cell_type = mesh.dim, mesh.cell_type
        self.coords = _f64(mesh.coords)
        self.cells = np.ascontiguousarray(mesh.cells, dtype=np.int64)
        self.omega = _f64(omega).reshape(-1, 3)
        h = ctypes.c_void_p()
        rc = lib.orc_build(mesh.dim, mesh.cell_type, self.coords.shape[0], _p(self.coords),
                           self.cells.shape[0], _p(self.cells), self.omega.shape[0], _p(self.omega),
                           1 if refuse_cycles else 0, ctypes.byref(h))
        if rc != 0:
            raise OracleError(f"orc_build failed with code {rc}")
        self._h = h
        sz = np.zeros(6, dtype=np.int64)
        lib.orc_sizes(h, _p(sz))
        self.n_cells, self.n_faces, self.n_dirs, self.n_lagged, self.faces_per_cell, self.max_levels = map(int, sz)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.orc_free(h)
            self._h = None

    # -- exports -----------------------------------------------------------
    def geometry(self):
        S = np.zeros((self.n_faces, 3))
        fcell = np.zeros((self.n_faces, 2), dtype=np.int64)
        cface = np.zeros((self.n_cells, self.faces_per_cell), dtype=np.int64)
        vol = np.zeros(self.n_cells)
        self._lib.orc_geometry(self._h, _p(S), _p(fcell), _p(cface), _p(vol))
        return S, fcell, cface, vol

    def direction(self, m: int):
        n = self.n_cells
        indeg = np.zeros(n, dtype=np.int32)
        level = np.zeros(n, dtype=np.int32)
        lvl_cells = np.zeros(n, dtype=np.int64)
        nlev = int(self._lib.orc_dir(self._h, m, _p(indeg), _p(level), None, None))
        lvl_ptr = np.zeros(nlev + 1, dtype=np.int64)
        self._lib.orc_dir(self._h, m, None, None, _p(lvl_ptr), _p(lvl_cells))
        return indeg, level, lvl_ptr, lvl_cells

    def lagged(self):
        k = self.n_lagged
        m = np.zeros(k, dtype=np.int32)
        u = np.zeros(k, dtype=np.int64)
        v = np.zeros(k, dtype=np.int64)
        f = np.zeros(k, dtype=np.int32)
        self._lib.orc_lagged(self._h, _p(m), _p(u), _p(v), _p(f))
        return m, u, v, f

    # -- numerics ----------------------------------------------------------
    def sweep(self, sigma_t, source, psi_b: float = 0.0, psi_prev=None, tie_seed: int = 0):
        st = _f64(sigma_t)
        src = _f64(source)
        per_dir = 1 if src.size == self.n_cells * self.n_dirs and self.n_dirs > 1 else 0
        psi = np.zeros((self.n_dirs, self.n_cells))
        pp = None if psi_prev is None else _f64(psi_prev)
        self._lib.orc_sweep(self._h, _p(st), _p(src), per_dir, float(psi_b), _p(pp), _p(psi), int(tie_seed))
        return psi

    def sweep_dirs(self, m0, m1, sigma_t, source, psi_b=0.0, psi_prev=None, psi=None):
        st, src = _f64(sigma_t), _f64(source)
        per_dir = 1 if src.size == self.n_cells * self.n_dirs and self.n_dirs > 1 else 0
        if psi is None:
            psi = np.zeros((self.n_dirs, self.n_cells))
        pp = None if psi_prev is None else _f64(psi_prev)
        rc = self._lib.orc_sweep_dirs(self._h, m0, m1, _p(st), _p(src), per_dir, float(psi_b), _p(pp), _p(psi))
        if rc:
            raise OracleError(f"orc_sweep_dirs failed with code {rc}")
        return psi

    def phi(self, weight, psi):
        w, ps = _f64(weight), _f64(psi)
        out = np.zeros(self.n_cells)
        self._lib.orc_phi(self._h, _p(w), _p(ps), _p(out))
        return out

    def residual(self, sigma_t, sigma_s, q, weight, psi, phi, psi_b: float = 0.0, want_r: bool = False):
        st, ss, qq, w = _f64(sigma_t), _f64(sigma_s), _f64(q), _f64(weight)
        ps, ph = _f64(psi), _f64(phi)
        r = np.zeros((self.n_dirs, self.n_cells)) if want_r else None
        rho = self._lib.orc_residual(self._h, _p(st), _p(ss), _p(qq), float(psi_b), _p(w), _p(ps), _p(ph), _p(r))
        return (rho, r) if want_r else rho

    def source_iteration(self, sigma_t, sigma_s, q, weight, max_iter: int, tol: float = 0.0, psi_b: float = 0.0):
        st, ss, qq, w = _f64(sigma_t), _f64(sigma_s), _f64(q), _f64(weight)
        psi = np.zeros((self.n_dirs, self.n_cells))
        phi = np.zeros(self.n_cells)
        hist = np.zeros(max(1, max_iter))
        it = self._lib.orc_si(self._h, _p(st), _p(ss), _p(qq), float(psi_b), _p(w), int(max_iter), float(tol),
                              _p(psi), _p(phi), _p(hist))
        return psi, phi, hist[:it]

    # -- multigroup (arrays: sigma_t, q [G, nc]; sigma_s [G, G, nc] from g' (first index)
    #    into g (second); psi [G, nd, nc]; phi [G, nc]) -------------------------------
    def mg_residual(self, sigma_t, sigma_s, q, weight, psi, phi, psi_b: float = 0.0):
        st, ss, qq, w = _f64(sigma_t), _f64(sigma_s), _f64(q), _f64(weight)
        G = st.shape[0]
        return self._lib.orc_mg_residual(self._h, G, _p(st), _p(ss), _p(qq), float(psi_b), _p(w), _p(_f64(psi)),
                                         _p(_f64(phi)))

    def mg_source_iteration(self, sigma_t, sigma_s, q, weight, max_iter: int, tol: float = 0.0,
                            psi_b: float = 0.0):
        st, ss, qq, w = _f64(sigma_t), _f64(sigma_s), _f64(q), _f64(weight)
        G = st.shape[0]
        psi = np.zeros((G, self.n_dirs, self.n_cells))
        phi = np.zeros((G, self.n_cells))
        hist = np.zeros(max(1, max_iter))
        it = self._lib.orc_mg_si(self._h, G, _p(st), _p(ss), _p(qq), float(psi_b), _p(w), int(max_iter), float(tol),
                                 _p(psi), _p(phi), _p(hist))
        return psi, phi, hist[:it]


def graph_for(problem, refuse_cycles: bool = False) -> Graph:
    return Graph(problem.mesh, problem.omega, refuse_cycles)
