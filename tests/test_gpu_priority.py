"""GPU: work-list priority strategies (paper Sec. V-D: BFS, LDCP, SLBD and
the (patch, angle) ranking prior(a) * C + prior(p), with an unbounded C
(angle-major) or a finite one, a fraction of the level count).

Every priority must give a topological order of each stream's coarsened
graph (checked on the traced work list) and, since a flux is a pure
function of its upwind fluxes, fluxes bit-identical to the level-order
sweep and to the oracle, for single sweeps and source iterations (lagged
edges included)."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import J, dev, host, need_gpu, rel_max

pytestmark = pytest.mark.gpu

PRIORITIES = [
    J.JSWEEP_PRIORITY_BFS, J.JSWEEP_PRIORITY_LDCP, J.JSWEEP_PRIORITY_SLBD,
    J.JSWEEP_PRIORITY_BFS | J.JSWEEP_PRIORITY_ANGLE_MAJOR,
    J.JSWEEP_PRIORITY_LDCP | J.JSWEEP_PRIORITY_ANGLE_MAJOR,
    J.JSWEEP_PRIORITY_SLBD | J.JSWEEP_PRIORITY_ANGLE_MAJOR,
    J.JSWEEP_PRIORITY_BFS | J.JSWEEP_PRIORITY_ANGLE_WEIGHT(1),
    J.JSWEEP_PRIORITY_BFS | J.JSWEEP_PRIORITY_ANGLE_WEIGHT(3),
    J.JSWEEP_PRIORITY_LDCP | J.JSWEEP_PRIORITY_ANGLE_WEIGHT(2),
    J.JSWEEP_PRIORITY_PACED,
    J.JSWEEP_PRIORITY_PACED | J.JSWEEP_PRIORITY_ANGLE_WEIGHT(5),
]


def _cases():
    return [
        ("hex12_s8_lagged", W.config(2, "small")),
        ("tetcheck16_s8", W.config(3, "small")),
        ("delaunay_s4", W.config(1)),
    ]


@pytest.fixture(scope="module")
def cases(oracle_mod):
    need_gpu()
    out = []
    for name, p in _cases():
        print(f"[case] {name} cells={p.n_cells} dirs={p.n_dirs}", flush=True)
        og = oracle_mod.graph_for(p)
        ref = og.sweep(p.sigma_t, p.q)
        psi_ref, phi_ref, _ = og.source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, 6)
        out.append((name, p, ref, psi_ref, phi_ref))
    return out


def _check_order(tr, n_dirs):
    """The traced work list is a topological order of every stream's chunk
    graph; returns the per-chunk (direction, level) arrays in list order."""
    ptr, deps = tr["deps_ptr"], tr["deps"]
    n = len(ptr) - 1
    down = np.repeat(np.arange(n), np.diff(ptr))
    assert len(deps) == 0 or (deps < down).all()          # upwind chunks come first
    stream = (tr["dir"] * 8) // n_dirs
    assert len(deps) == 0 or (stream[deps] == stream[down]).all()
    assert (np.diff(stream) >= 0).all()                    # streams stay contiguous
    return tr["dir"], tr["level"], stream


@pytest.mark.parametrize("priority", PRIORITIES)
def test_priority_sweeps_bit_identical(cases, priority):
    for name, p, ref, psi_ref, phi_ref in cases:
        g = J.build_graph(p.mesh, p.omega, p.weight, J.JSWEEP_PRIORITY_FLAGS(priority))
        try:
            J.jsweep_trace(g, True)
            psi = dev(np.zeros((p.n_dirs, p.n_cells)))
            J.sweep(g, dev(p.sigma_t), dev(p.q), psi)
            tr = J.jsweep_trace_read(g)
            J.jsweep_trace(g, False)
            got = host(psi)
            d, lev, stream = _check_order(tr, p.n_dirs)
            if priority & J.JSWEEP_PRIORITY_ANGLE_MAJOR:
                for s in np.unique(stream):
                    assert (np.diff(d[stream == s]) >= 0).all(), name     # direction first
            if priority == J.JSWEEP_PRIORITY_BFS:
                for s in np.unique(stream):
                    key = lev[stream == s].astype(np.int64) * 4096 + d[stream == s]
                    assert (np.diff(key) >= 0).all(), name                # level, then direction
            if priority == J.JSWEEP_PRIORITY_PACED:
                # level / (level count of the direction), then level order
                nlev = np.array([len(J.graph_export(g, m, want=("lvl_ptr",))[2]) - 1 for m in range(p.n_dirs)])
                for s in np.unique(stream):
                    ds, ls = d[stream == s].astype(np.int64), lev[stream == s].astype(np.int64)
                    frac = (ls << 32) // nlev[ds]
                    assert (np.diff(frac) >= 0).all(), name
            k = (priority >> 5) & 7
            if k and priority & 0xf == J.JSWEEP_PRIORITY_BFS:
                # rank * C + level, C = ceil(max levels of the stream / k):
                # Kahn's queue releases in this key whenever the key itself
                # is topological, which it is here (an upwind chunk of the
                # same direction has a lower level)
                # (ties of the key go by level, as in the level order)
                nlev = np.array([len(J.graph_export(g, m, want=("lvl_ptr",))[2]) - 1 for m in range(p.n_dirs)])
                for s in np.unique(stream):
                    sd = np.arange(p.n_dirs)[(np.arange(p.n_dirs) * 8) // p.n_dirs == s]
                    C = -(-nlev[sd].max() // k)
                    ds, ls = d[stream == s].astype(np.int64), lev[stream == s].astype(np.int64)
                    key = (((ds - sd[0]) * C + ls) * 100000 + ls) * 4096 + ds
                    assert (np.diff(key) >= 0).all(), name
            exact = np.array_equal(got, ref)
            print(f"[priority {priority:#x}] {name} chunks {len(d)} sweep rel {rel_max(got, ref):.2e} "
                  f"bitexact {exact}", flush=True)
            assert exact, name
            phi = dev(np.zeros(p.n_cells))
            psi = dev(np.zeros((p.n_dirs, p.n_cells)))
            J.solve(g, dev(p.sigma_t), dev(p.sigma_s), dev(p.q), phi, psi, mode=J.JSWEEP_FP64, tol=0.0, max_iter=6,
                    allow_not_converged=True)
            e1, e2 = rel_max(host(phi), phi_ref), rel_max(host(psi), psi_ref)
            assert e1 <= 1e-12 and e2 <= 1e-12, name
        finally:
            g.close()


def test_priority_through_params_and_back(cases):
    """A priority requested in the solve's parameters reorders the work list
    on first use; the FP32-refined solve and the return to BFS stay exact."""
    name, p, ref, psi_ref, phi_ref = cases[0]
    g = J.build_graph(p.mesh, p.omega, p.weight)
    try:
        out = {}
        for pr in (J.JSWEEP_PRIORITY_SLBD, J.JSWEEP_PRIORITY_LDCP | J.JSWEEP_PRIORITY_ANGLE_MAJOR,
                   J.JSWEEP_PRIORITY_BFS):
            phi = dev(np.zeros(p.n_cells))
            psi = dev(np.zeros((p.n_dirs, p.n_cells)))
            J.solve(g, dev(p.sigma_t), dev(p.sigma_s), dev(p.q), phi, psi, mode=J.JSWEEP_FP64, tol=0.0, max_iter=6,
                    params=J.Params(priority=pr), allow_not_converged=True)
            assert rel_max(host(phi), phi_ref) <= 1e-12 and rel_max(host(psi), psi_ref) <= 1e-12
            phi32 = dev(np.zeros(p.n_cells))
            st = J.solve(g, dev(p.sigma_t), dev(p.sigma_s), dev(p.q), phi32, mode=J.JSWEEP_FP32_REFINED, tol=1e-10,
                         max_iter=500, params=J.Params(priority=pr))
            out[pr] = host(phi32)
            print(f"[priority params {pr:#x}] refined sweeps {st['sweeps']} rho {st['residual']:.2e}", flush=True)
        base = out[J.JSWEEP_PRIORITY_BFS]
        for pr, v in out.items():
            assert rel_max(v, base) <= 1e-9, pr
        J.set_params(g, J.Params(priority=J.JSWEEP_PRIORITY_SLBD))
        psi = dev(np.zeros((p.n_dirs, p.n_cells)))
        J.sweep(g, dev(p.sigma_t), dev(p.q), psi)
        assert np.array_equal(host(psi), ref)
        with pytest.raises(J.JsweepError):
            J.set_params(g, J.Params(priority=7))
        with pytest.raises(J.JsweepError):
            J.set_params(g, J.Params(priority=J.JSWEEP_PRIORITY_BFS | J.JSWEEP_PRIORITY_ANGLE_MAJOR |
                                     J.JSWEEP_PRIORITY_ANGLE_WEIGHT(2)))
    finally:
        g.close()
