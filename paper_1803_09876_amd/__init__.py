"""jsweep: data-driven S_n transport sweeps on AMD Instinct MI355X (gfx950).

Thin Python binding of the C ABI declared in ``include/jsweep.h`` (same
entry-point names).  It only marshals arguments: every step of the sweep
path runs in the HIP library ``libjsweep.so`` built next to this file.
PyTorch supplies device memory and streams; problem arrays are CUDA (ROCm)
tensors.  The library must be built (``paper_1803_09876_amd.build``)
before import on a GPU machine; importing without it raises."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjsweep.so")

JSWEEP_OK = 0
JSWEEP_E_INVALID_ARG = -1
JSWEEP_E_MESH = -2
JSWEEP_E_QUADRATURE = -3
JSWEEP_E_CYCLE = -4
JSWEEP_E_DEVICE = -5
JSWEEP_E_OOM = -6
JSWEEP_E_STALLED = -7
JSWEEP_E_NOT_CONVERGED = -8
JSWEEP_E_PLACEMENT = -9

JSWEEP_TRI, JSWEEP_TET, JSWEEP_HEX = 3, 4, 8
JSWEEP_DEBUG_NO_LAG = 0x1
JSWEEP_HOST_PTRS = 0x2
JSWEEP_FP64 = 0
JSWEEP_FP32_REFINED = 1
JSWEEP_WARM_START = 0x100
JSWEEP_STRATEGY_AUTO, JSWEEP_STRATEGY_DATA_DRIVEN, JSWEEP_STRATEGY_DIRECTION = 0, 1, 2
JSWEEP_STRATEGY_DIRECTION_LDS = 3
JSWEEP_STRATEGY_PATCH = 4
JSWEEP_PRIORITY_BFS, JSWEEP_PRIORITY_LDCP, JSWEEP_PRIORITY_SLBD, JSWEEP_PRIORITY_PACED = 1, 2, 3, 4
JSWEEP_PRIORITY_ANGLE_MAJOR = 0x10


def JSWEEP_PRIORITY_ANGLE_WEIGHT(k: int) -> int:
    """Priority bits of the finite angle weight C = (largest level count of
    a stream) / k, k = 1..7 (OR-ed with BFS, LDCP or SLBD)."""
    return (int(k) & 7) << 5


def JSWEEP_PRIORITY_FLAGS(p: int) -> int:
    """Build flags selecting a work-list priority (bits 8-15)."""
    return (int(p) & 0xff) << 8

EXPORTED = [
    "jsweep_build_graph", "jsweep_graph_info", "jsweep_graph_export", "jsweep_graph_lagged", "jsweep_sweep",
    "jsweep_solve", "jsweep_solve_batch", "jsweep_autotune", "jsweep_profile", "jsweep_profile_read",
    "jsweep_trace", "jsweep_trace_read", "jsweep_graph_destroy", "jsweep_error_string", "jsweep_last_error",
    "jsweep_set_params", "jsweep_patch_info", "jsweep_program_info", "jsweep_solve_groups", "jsweep_sweep_noalloc",
]


class JsweepError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class _Mesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("cell_type", ctypes.c_int32), ("n_vertices", ctypes.c_int64),
                ("coords", ctypes.c_void_p), ("n_cells", ctypes.c_int64), ("cell_vertices", ctypes.c_void_p)]


class _Quad(ctypes.Structure):
    _fields_ = [("n_dirs", ctypes.c_int32), ("omega", ctypes.c_void_p), ("weight", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("waves_per_block", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("inner_sweeps", ctypes.c_int32), ("chunks_per_ticket", ctypes.c_int32),
                ("strategy", ctypes.c_int32), ("priority", ctypes.c_int32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class SolveStats(ctypes.Structure):
    _fields_ = [("outer_iters", ctypes.c_int32), ("sweeps", ctypes.c_int32), ("residual", ctypes.c_double),
                ("seconds", ctypes.c_double), ("lagged_edges", ctypes.c_int64), ("max_levels", ctypes.c_int32),
                ("history_len", ctypes.c_int32), ("residual_history", ctypes.c_void_p),
                ("history_capacity", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _Problem(ctypes.Structure):
    _fields_ = [("sigma_t", ctypes.c_void_p), ("sigma_s", ctypes.c_void_p), ("q", ctypes.c_void_p),
                ("psi_boundary", ctypes.c_double), ("phi", ctypes.c_void_p), ("psi", ctypes.c_void_p)]


_lib = None


def load_library(path: str | None = None):
    """Load libjsweep.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"libjsweep.so not built: {path} missing (run paper_1803_09876_amd.build)")
    lib = ctypes.CDLL(path)
    P, i32, i64, dbl, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint32
    lib.jsweep_build_graph.argtypes = [ctypes.POINTER(_Mesh), ctypes.POINTER(_Quad), u32, ctypes.POINTER(P)]
    lib.jsweep_graph_info.argtypes = [P, P, P, P, P]
    lib.jsweep_program_info.argtypes = [P, P, P, P]
    lib.jsweep_graph_export.argtypes = [P, i32, P, P, P, P, P, u32]
    lib.jsweep_graph_lagged.argtypes = [P, P, P, P, P]
    lib.jsweep_sweep.argtypes = [P, P, P, P, P, dbl, P]
    lib.jsweep_sweep_noalloc.argtypes = [P, P, P, P, P, dbl, P]
    lib.jsweep_solve.argtypes = [P, P, P, P, dbl, i32, dbl, i32, P, P, P, P, P]
    lib.jsweep_solve_batch.argtypes = [i32, P, P, i32, dbl, i32, P, P, P]
    lib.jsweep_solve_groups.argtypes = [P, i32, P, P, P, dbl, dbl, i32, P, P, P, P, P]
    lib.jsweep_autotune.argtypes = [i32, P, i32, P]
    lib.jsweep_set_params.argtypes = [P, P]
    lib.jsweep_patch_info.argtypes = [P, P, P]
    lib.jsweep_profile.argtypes = [P, i32]
    lib.jsweep_profile_read.argtypes = [P, i32, P, P]
    lib.jsweep_trace.argtypes = [P, i32]
    lib.jsweep_trace_read.argtypes = [P, P, P, P, P, P]
    lib.jsweep_graph_destroy.argtypes = [P]
    lib.jsweep_graph_destroy.restype = None
    lib.jsweep_error_string.argtypes = [ctypes.c_int]
    lib.jsweep_error_string.restype = ctypes.c_char_p
    lib.jsweep_last_error.argtypes = []
    lib.jsweep_last_error.restype = ctypes.c_char_p
    for name in ("jsweep_build_graph", "jsweep_graph_info", "jsweep_graph_export", "jsweep_graph_lagged",
                 "jsweep_sweep", "jsweep_sweep_noalloc", "jsweep_solve", "jsweep_solve_groups", "jsweep_solve_batch", "jsweep_autotune", "jsweep_profile",
                 "jsweep_profile_read", "jsweep_trace", "jsweep_trace_read", "jsweep_set_params",
                 "jsweep_patch_info", "jsweep_program_info"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int, allow=()):
    if rc == JSWEEP_OK or rc in allow:
        return rc
    lib = load_library()
    raise JsweepError(rc, f"{lib.jsweep_error_string(rc).decode()}: {lib.jsweep_last_error().decode()}")


def _ptr(t):
    """Device pointer of a CUDA tensor (None passes NULL)."""
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _f64(t, n=None):
    import torch
    if t is None:
        return None
    if t.dtype != torch.float64:
        raise TypeError("expected float64 tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return _ptr(t)


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Graph:
    """Handle of a built sweep graph (``jsweep_build_graph``)."""

    def __init__(self, handle, n_cells, n_dirs):
        self._h = handle
        self.n_cells = n_cells
        self.n_dirs = n_dirs

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            load_library().jsweep_graph_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def jsweep_build_graph(dim, cell_type, coords, cells, omega, weight, flags: int = 0) -> Graph:
    lib = load_library()
    coords = np.ascontiguousarray(coords, dtype=np.float64)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    omega = np.ascontiguousarray(omega, dtype=np.float64).reshape(-1, 3)
    weight = np.ascontiguousarray(weight, dtype=np.float64)
    mesh = _Mesh(int(dim), int(cell_type), coords.shape[0], coords.ctypes.data, cells.shape[0], cells.ctypes.data)
    quad = _Quad(omega.shape[0], omega.ctypes.data, weight.ctypes.data)
    h = ctypes.c_void_p()
    _check(lib.jsweep_build_graph(ctypes.byref(mesh), ctypes.byref(quad), int(flags), ctypes.byref(h)))
    return Graph(h, cells.shape[0], omega.shape[0])


def build_graph(mesh, omega, weight, flags: int = 0) -> Graph:
    """Convenience: build from an object with dim, cell_type, coords, cells."""
    return jsweep_build_graph(mesh.dim, mesh.cell_type, mesh.coords, mesh.cells, omega, weight, flags)


def jsweep_graph_info(g: Graph):
    lib = load_library()
    nc, nd, nl, ml = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32()
    _check(lib.jsweep_graph_info(g.handle, ctypes.byref(nc), ctypes.byref(nd), ctypes.byref(nl), ctypes.byref(ml)))
    return {"n_cells": nc.value, "n_dirs": nd.value, "n_lagged": nl.value, "max_levels": ml.value}


def jsweep_program_info(g: Graph):
    """Sweep program shape: inflow slots per vertex, how many of them the
    FP64 work-list sweep reads from the chunk blocks (0: full program), and
    whether the work-list sweeps read packed upwind positions."""
    lib = load_library()
    ns, nx, pk = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib.jsweep_program_info(g.handle, ctypes.byref(ns), ctypes.byref(nx), ctypes.byref(pk)))
    return {"slots": ns.value, "block_slots": nx.value, "packed": bool(pk.value)}


def jsweep_graph_export(g: Graph, direction: int, want=("indeg", "level", "lvl_ptr", "lvl_cells")):
    """Per-direction graph arrays as host numpy arrays:
    (indeg int32, level int32, lvl_ptr int64, lvl_cells int64); arrays not
    named in ``want`` are not exported and come back as None."""
    lib = load_library()
    n = g.n_cells
    nlev = ctypes.c_int32()
    _check(lib.jsweep_graph_export(g.handle, int(direction), None, None, None, None, ctypes.byref(nlev),
                                   JSWEEP_HOST_PTRS))
    indeg = np.zeros(n, dtype=np.int32) if "indeg" in want else None
    level = np.zeros(n, dtype=np.int32) if "level" in want else None
    lvl_ptr = np.zeros(nlev.value + 1, dtype=np.int64) if "lvl_ptr" in want else None
    lvl_cells = np.zeros(n, dtype=np.int64) if "lvl_cells" in want else None
    addr = lambda a: None if a is None else a.ctypes.data  # noqa: E731
    _check(lib.jsweep_graph_export(g.handle, int(direction), addr(indeg), addr(level), addr(lvl_ptr),
                                   addr(lvl_cells), None, JSWEEP_HOST_PTRS))
    return indeg, level, lvl_ptr, lvl_cells


def jsweep_graph_lagged(g: Graph):
    lib = load_library()
    k = jsweep_graph_info(g)["n_lagged"]
    m = np.zeros(k, dtype=np.int32)
    u = np.zeros(k, dtype=np.int64)
    v = np.zeros(k, dtype=np.int64)
    f = np.zeros(k, dtype=np.int32)
    _check(lib.jsweep_graph_lagged(g.handle, m.ctypes.data, u.ctypes.data, v.ctypes.data, f.ctypes.data))
    return m, u, v, f


def jsweep_sweep(g: Graph, sigma_t, source, psi, phi=None, psi_boundary: float = 0.0, stream=None):
    """One FP64 sweep of all directions; psi (in: previous iterate, out:
    new) is a [n_dirs, n_cells] float64 device tensor."""
    lib = load_library()
    n = g.n_cells
    _check(lib.jsweep_sweep(g.handle, _f64(sigma_t, n), _f64(source, n), _f64(psi, n * g.n_dirs),
                            _f64(phi, n) if phi is not None else None, float(psi_boundary), _stream(stream)))


def jsweep_sweep_noalloc(g: Graph, sigma_t, source, psi, phi=None, psi_boundary: float = 0.0, stream=None):
    """jsweep_sweep without device allocation (V s staged in the library's
    fixed device array; at most 8,388,608 cells)."""
    lib = load_library()
    n = g.n_cells
    _check(lib.jsweep_sweep_noalloc(g.handle, _f64(sigma_t, n), _f64(source, n), _f64(psi, n * g.n_dirs),
                                    _f64(phi, n) if phi is not None else None, float(psi_boundary), _stream(stream)))


def jsweep_solve(g: Graph, sigma_t, sigma_s, q, phi, psi=None, psi_boundary: float = 0.0, mode: int = JSWEEP_FP64,
                 tol: float = 1e-8, max_iter: int = 1000, params: Params | None = None, history: int = 0,
                 stream=None, allow_not_converged: bool = False):
    """Source iteration to rho <= tol; returns a stats dict."""
    lib = load_library()
    n = g.n_cells
    st = SolveStats()
    hist = np.zeros(max(history, 1))
    if history:
        st.residual_history = hist.ctypes.data
        st.history_capacity = history
    rc = lib.jsweep_solve(g.handle, _f64(sigma_t, n), _f64(sigma_s, n), _f64(q, n), float(psi_boundary), int(mode),
                          float(tol), int(max_iter), ctypes.byref(params) if params is not None else None,
                          _f64(phi, n), _f64(psi, n * g.n_dirs) if psi is not None else None, ctypes.byref(st),
                          _stream(stream))
    _check(rc, allow=(JSWEEP_E_NOT_CONVERGED,) if allow_not_converged else ())
    out = {k: getattr(st, k) for k in ("outer_iters", "sweeps", "residual", "seconds", "lagged_edges", "max_levels")}
    out["converged"] = rc == JSWEEP_OK
    if history:
        out["history"] = hist[:st.history_len].copy()
    return out


def jsweep_solve_groups(g: Graph, sigma_t, sigma_s, q, phi, psi=None, psi_boundary: float = 0.0, tol: float = 1e-8,
                        max_iter: int = 1000, params: Params | None = None, history: int = 0, stream=None,
                        allow_not_converged: bool = False):
    """Multigroup (Jacobi over groups) FP64 source iteration.  sigma_t, q,
    phi: [G, n_cells]; sigma_s: [G, G, n_cells] (from g' into g); psi:
    [G, n_dirs, n_cells] or None.  Returns a stats dict."""
    lib = load_library()
    n = g.n_cells
    G = int(sigma_t.shape[0]) if sigma_t.dim() == 2 else sigma_t.numel() // n
    st = SolveStats()
    hist = np.zeros(max(history, 1))
    if history:
        st.residual_history = hist.ctypes.data
        st.history_capacity = history
    rc = lib.jsweep_solve_groups(g.handle, G, _f64(sigma_t, G * n), _f64(sigma_s, G * G * n), _f64(q, G * n),
                                 float(psi_boundary), float(tol), int(max_iter),
                                 ctypes.byref(params) if params is not None else None, _f64(phi, G * n),
                                 _f64(psi, G * n * g.n_dirs) if psi is not None else None, ctypes.byref(st),
                                 _stream(stream))
    _check(rc, allow=(JSWEEP_E_NOT_CONVERGED,) if allow_not_converged else ())
    out = {k: getattr(st, k) for k in ("outer_iters", "sweeps", "residual", "seconds")}
    out["converged"] = rc == JSWEEP_OK
    if history:
        out["history"] = hist[:st.history_len].copy()
    return out


def jsweep_solve_batch(graphs, problems, mode: int = JSWEEP_FP32_REFINED, tol: float = 1e-8, max_iter: int = 1000,
                       params: Params | None = None, stream=None, allow_not_converged: bool = False):
    """problems: list of dicts with sigma_t, sigma_s, q, phi (tensors),
    optional psi and psi_boundary.  Returns a list of stats dicts."""
    lib = load_library()
    n = len(graphs)
    hs = (ctypes.c_void_p * n)(*[g.handle.value for g in graphs])
    ps = (_Problem * n)()
    for i, (g, p) in enumerate(zip(graphs, problems)):
        nc = g.n_cells
        ps[i].sigma_t = _f64(p["sigma_t"], nc).value
        ps[i].sigma_s = _f64(p["sigma_s"], nc).value
        ps[i].q = _f64(p["q"], nc).value
        ps[i].psi_boundary = float(p.get("psi_boundary", 0.0))
        ps[i].phi = _f64(p["phi"], nc).value
        ps[i].psi = _f64(p["psi"], nc * g.n_dirs).value if p.get("psi") is not None else None
    sts = (SolveStats * n)()
    rc = lib.jsweep_solve_batch(n, hs, ps, int(mode), float(tol), int(max_iter),
                                ctypes.byref(params) if params is not None else None, sts, _stream(stream))
    _check(rc, allow=(JSWEEP_E_NOT_CONVERGED,) if allow_not_converged else ())
    return [{k: getattr(s, k) for k in ("outer_iters", "sweeps", "residual", "seconds")} for s in sts]


def jsweep_autotune(graphs, mode: int = JSWEEP_FP32_REFINED) -> Params:
    lib = load_library()
    n = len(graphs)
    hs = (ctypes.c_void_p * n)(*[g.handle.value for g in graphs])
    out = Params()
    _check(lib.jsweep_autotune(n, hs, int(mode), ctypes.byref(out)))
    return out


def jsweep_set_params(g: Graph, params: Params | None):
    """Pin the launch parameters of the graph's sweeps (None: defaults)."""
    _check(load_library().jsweep_set_params(g.handle, ctypes.byref(params) if params is not None else None))


def jsweep_patch_info(g: Graph, stream=None):
    """The PATCH strategy's program (built on demand): dict of available,
    tasks, rounds, halo, deps, revisits."""
    out = np.zeros(6, dtype=np.int64)
    _check(load_library().jsweep_patch_info(g.handle, _stream(stream), out.ctypes.data))
    return {"available": bool(out[0]), "tasks": int(out[1]), "rounds": int(out[2]), "halo": int(out[3]),
            "deps": int(out[4]), "revisits": int(out[5])}


def jsweep_profile(g: Graph, enable: bool = True):
    _check(load_library().jsweep_profile(g.handle, 1 if enable else 0))


def jsweep_profile_read(g: Graph, reset: bool = True):
    """(launches, total kernel milliseconds) of the sweep kernel."""
    n, ms = ctypes.c_int64(), ctypes.c_double()
    _check(load_library().jsweep_profile_read(g.handle, 1 if reset else 0, ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def jsweep_trace(g: Graph, enable: bool = True):
    _check(load_library().jsweep_trace(g.handle, 1 if enable else 0))


def jsweep_trace_read(g: Graph):
    """Per-chunk stamps of the last traced sweep as a dict of numpy arrays:
    take, ready, done (100 MHz ticks), dir, count, level, deps_ptr, deps."""
    lib = load_library()
    n = ctypes.c_int64()
    _check(lib.jsweep_trace_read(g.handle, ctypes.byref(n), None, None, None, None))
    n = n.value
    stamps = np.zeros(3 * n, dtype=np.uint32)
    info = np.zeros(3 * n, dtype=np.int32)
    ptr = np.zeros(n + 1, dtype=np.int32)
    _check(lib.jsweep_trace_read(g.handle, None, None, None, ptr.ctypes.data, None))
    deps = np.zeros(max(1, int(ptr[-1])), dtype=np.int32)
    _check(lib.jsweep_trace_read(g.handle, None, stamps.ctypes.data, info.ctypes.data, None, deps.ctypes.data))
    st = stamps.reshape(n, 3).astype(np.int64)
    inf = info.reshape(n, 3)
    return {"take": st[:, 0], "ready": st[:, 1], "done": st[:, 2], "dir": inf[:, 0], "count": inf[:, 1],
            "level": inf[:, 2], "deps_ptr": ptr, "deps": deps[:int(ptr[-1])]}


def jsweep_error_string(code: int) -> str:
    return load_library().jsweep_error_string(int(code)).decode()


def jsweep_last_error() -> str:
    return load_library().jsweep_last_error().decode()


# short aliases
graph_info = jsweep_graph_info
program_info = jsweep_program_info
set_params = jsweep_set_params
patch_info = jsweep_patch_info
graph_export = jsweep_graph_export
graph_lagged = jsweep_graph_lagged
sweep = jsweep_sweep
sweep_noalloc = jsweep_sweep_noalloc
solve = jsweep_solve
solve_batch = jsweep_solve_batch
solve_groups = jsweep_solve_groups
autotune = jsweep_autotune
