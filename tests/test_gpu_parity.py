"""GPU parity: the HIP path through the C ABI against the oracle.

* graph construction (in-degrees, levels, level pointers, level-ordered
  cells, lagged edges): bit-exact;
* one FP64 sweep and 20 FP64 source iterations: max relative difference
  <= 1e-12 in psi and phi;
* FP32-refined solve converged to rho <= 1e-11 against the oracle at
  rho <= 1e-13: <= 1e-8 normwise relative in phi."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import J, dev, gpu_graph, host, need_gpu, rel_max, torch

pytestmark = pytest.mark.gpu


def _small_cases():
    return [
        ("delaunay_s4", W.config(1)),
        ("hex12_s8_lagged", W.config(2, "small")),
        ("tetcheck16_s8", W.config(3, "small")),
        ("tetlogn8_s16", W.config(5, "small")),
        ("hex3_cyclic", W.Problem("hex3cyc", W.hex_lattice(3, 0.3, 1), *W.quadrature(8, 3),
                                  np.full(27, 1.3), np.full(27, 0.9), np.ones(27))),
    ]


@pytest.fixture(scope="module")
def cases(oracle_mod):
    need_gpu()
    out = []
    for name, p in _small_cases():
        print(f"[case] {name} cells={p.n_cells} dirs={p.n_dirs}", flush=True)
        out.append((name, p, oracle_mod.graph_for(p), gpu_graph(p)))
    return out


def test_graph_bit_exact(cases):
    for name, p, og, gg in cases:
        info = J.graph_info(gg)
        assert info["n_lagged"] == og.n_lagged, name
        assert info["max_levels"] == og.max_levels, name
        for m in range(p.n_dirs):
            a = og.direction(m)
            b = J.graph_export(gg, m)
            for x, y in zip(a, b):
                assert np.array_equal(x, y), (name, m)
        if og.n_lagged:
            for x, y in zip(og.lagged(), J.graph_lagged(gg)):
                assert np.array_equal(x, y), name


def test_fp64_sweep(cases):
    for name, p, og, gg in cases:
        rng = np.random.default_rng(7)
        src = rng.uniform(0.0, 2.0, p.n_cells)
        prev = rng.uniform(0.0, 1.0, (p.n_dirs, p.n_cells))
        ref = og.sweep(p.sigma_t, src, 0.25, prev)
        psi = dev(prev)
        phi = dev(np.zeros(p.n_cells))
        J.sweep(gg, dev(p.sigma_t), dev(src), psi, phi, psi_boundary=0.25)
        got = host(psi)
        err = rel_max(got, ref)
        print(f"[sweep64] {name} rel {err:.3e} bitexact {np.array_equal(got, ref)}", flush=True)
        assert err <= 1e-12, name
        assert rel_max(host(phi), og.phi(p.weight, ref)) <= 1e-12


def test_fp64_sweep_deterministic(cases):
    name, p, og, gg = cases[2]
    src = dev(np.linspace(0.1, 1.0, p.n_cells))
    a = dev(np.zeros((p.n_dirs, p.n_cells)))
    b = dev(np.zeros((p.n_dirs, p.n_cells)))
    J.sweep(gg, dev(p.sigma_t), src, a)
    J.sweep(gg, dev(p.sigma_t), src, b)
    assert torch.equal(a, b)


def test_patch_program_and_sweep(cases):
    """PATCH strategy: its program applies to every case (bands where a
    direction's patch graph has a cycle), and one FP64 sweep with boundary
    inflow and a lagged previous iterate matches the oracle."""
    for name, p, og, gg in cases:
        info = J.patch_info(gg)
        print(f"[patch] {name} {info}", flush=True)
        assert info["available"], name
        assert info["tasks"] >= p.n_dirs and info["rounds"] >= info["tasks"]
        J.set_params(gg, J.Params(strategy=J.JSWEEP_STRATEGY_PATCH))
        try:
            rng = np.random.default_rng(7)
            src = rng.uniform(0.0, 2.0, p.n_cells)
            prev = rng.uniform(0.0, 1.0, (p.n_dirs, p.n_cells))
            ref = og.sweep(p.sigma_t, src, 0.25, prev)
            for rep in range(2):
                psi = dev(prev)
                J.sweep(gg, dev(p.sigma_t), dev(src), psi, psi_boundary=0.25)
                got = host(psi)
                err = rel_max(got, ref)
                print(f"[patch sweep64] {name} rep {rep} rel {err:.3e} bitexact {np.array_equal(got, ref)}", flush=True)
                assert err <= 1e-12, name
        finally:
            J.set_params(gg, None)


def test_set_params_validation_and_reset(cases):
    """jsweep_set_params: bad parameters are refused, pinned parameters
    apply to jsweep_sweep, None returns to the defaults (same fluxes)."""
    name, p, og, gg = cases[0]
    with pytest.raises(J.JsweepError):
        J.set_params(gg, J.Params(strategy=9))
    with pytest.raises(J.JsweepError):
        J.set_params(gg, J.Params(waves_per_block=-1))
    ref = og.sweep(p.sigma_t, p.q)
    for prm in (J.Params(strategy=J.JSWEEP_STRATEGY_DIRECTION), None):
        J.set_params(gg, prm)
        psi = dev(np.zeros((p.n_dirs, p.n_cells)))
        J.sweep(gg, dev(p.sigma_t), dev(p.q), psi)
        assert rel_max(host(psi), ref) <= 1e-12, prm


@pytest.mark.parametrize("strategy", [J.JSWEEP_STRATEGY_DATA_DRIVEN, J.JSWEEP_STRATEGY_PATCH])
def test_sweep_trace_respects_dependencies(cases, strategy):
    """Trace of one sweep (work-list chunks, or PATCH tasks): every unit
    became ready only after each of its upstream units had become ready and
    published, stamps are ordered taken <= ready <= done, and the units
    cover every (cell, direction) once."""
    for name, p, og, gg in cases[:3]:
        J.set_params(gg, J.Params(strategy=strategy))
        try:
            J.jsweep_trace(gg, True)
            psi = dev(np.zeros((p.n_dirs, p.n_cells)))
            J.sweep(gg, dev(p.sigma_t), dev(p.q), psi)
            tr = J.jsweep_trace_read(gg)
        finally:
            J.jsweep_trace(gg, False)
            J.set_params(gg, None)
        x0 = int(tr["take"].min())
        take, ready, done = ((tr[k] - x0) % (1 << 32) for k in ("take", "ready", "done"))
        n = len(take)
        ptr, deps = tr["deps_ptr"], tr["deps"]
        down = np.repeat(np.arange(n), np.diff(ptr))
        print(f"[trace s{strategy}] {name} units {n} deps {len(deps)} span {(done.max()) / 100:.1f} us", flush=True)
        assert (take <= ready).all() and (ready <= done).all(), name
        assert int(tr["count"].sum()) == p.n_cells * p.n_dirs, name
        assert len(deps) == 0 or (ready[deps] < ready[down]).all(), name


@pytest.mark.parametrize("strategy", [J.JSWEEP_STRATEGY_DATA_DRIVEN, J.JSWEEP_STRATEGY_DIRECTION,
                                      J.JSWEEP_STRATEGY_DIRECTION_LDS, J.JSWEEP_STRATEGY_PATCH])
def test_fp64_source_iteration_20(cases, strategy):
    for name, p, og, gg in cases:
        psi_ref, phi_ref, hist = og.source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, 20)
        phi = dev(np.zeros(p.n_cells))
        psi = dev(np.zeros((p.n_dirs, p.n_cells)))
        st = J.solve(gg, dev(p.sigma_t), dev(p.sigma_s), dev(p.q), phi, psi, mode=J.JSWEEP_FP64, tol=0.0,
                     max_iter=20, params=J.Params(strategy=strategy), allow_not_converged=True)
        assert st["sweeps"] == 20
        e1, e2 = rel_max(host(phi), phi_ref), rel_max(host(psi), psi_ref)
        print(f"[si64 s{strategy}] {name} phi {e1:.3e} psi {e2:.3e} rho {st['residual']:.3e} vs {hist[-1]:.3e}", flush=True)
        assert e1 <= 1e-12 and e2 <= 1e-12, name
        assert abs(st["residual"] - hist[-1]) <= 1e-6 * hist[-1] + 1e-15


@pytest.mark.parametrize("strategy", [J.JSWEEP_STRATEGY_DATA_DRIVEN, J.JSWEEP_STRATEGY_DIRECTION,
                                      J.JSWEEP_STRATEGY_DIRECTION_LDS, J.JSWEEP_STRATEGY_PATCH])
def test_fp32_refined_converges_to_oracle(cases, strategy):
    for name, p, og, gg in cases:
        if p.n_cells * p.n_dirs > 2_000_000:
            continue
        _, phi_ref, hist = og.source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, 20000, 1e-13)
        assert hist[-1] <= 1e-13
        phi = dev(np.zeros(p.n_cells))
        st = J.solve(gg, dev(p.sigma_t), dev(p.sigma_s), dev(p.q), phi, mode=J.JSWEEP_FP32_REFINED, tol=1e-11,
                     max_iter=20000, params=J.Params(strategy=strategy))
        got = host(phi)
        err = float(np.linalg.norm(got - phi_ref) / np.linalg.norm(phi_ref))
        print(f"[refined s{strategy}] {name} outer {st['outer_iters']} sweeps {st['sweeps']} (oracle {len(hist)}) "
              f"rho {st['residual']:.2e} phi rel {err:.3e}", flush=True)
        assert err <= 1e-8, name


def test_sweep_precision_switches_and_alternation(cases):
    """The work-list sweep's level-ordered flux arrays hold an empty marker
    of the running precision: FP64 sweeps alternating with FP32 correction
    sweeps (an FP32-refined solve) on one graph keep every FP64 sweep equal
    to the oracle's, twice in a row each time (both arrays)."""
    dd = J.Params(strategy=J.JSWEEP_STRATEGY_DATA_DRIVEN)
    for name, p, og, gg in cases[:4]:
        J.set_params(gg, dd)
        try:
            rng = np.random.default_rng(11)
            src = rng.uniform(0.0, 2.0, p.n_cells)
            ref = og.sweep(p.sigma_t, src)
            for rnd in range(2):
                for rep in range(2):
                    psi = dev(np.zeros((p.n_dirs, p.n_cells)))
                    J.sweep(gg, dev(p.sigma_t), dev(src), psi)
                    err = rel_max(host(psi), ref)
                    print(f"[switch] {name} round {rnd} rep {rep} rel {err:.3e}", flush=True)
                    assert err <= 1e-12, (name, rnd, rep)
                phi = dev(np.zeros(p.n_cells))
                J.solve(gg, dev(p.sigma_t), dev(p.sigma_s), dev(p.q), phi, mode=J.JSWEEP_FP32_REFINED, tol=0.0,
                        max_iter=3, params=dd, allow_not_converged=True)
        finally:
            J.set_params(gg, None)


@pytest.mark.parametrize("shape", [(1, 1, 1), (8, 4, 2), (16, 4, 4), (5, 9, 1)])
def test_launch_shapes(cases, shape):
    """Work-list sweep with other launch shapes (waves per workgroup,
    workgroups per CU -- capped at 4 -- and chunks per ticket): same fluxes."""
    wpb, bpc, grab = shape
    prm = J.Params(waves_per_block=wpb, blocks_per_cu=bpc, chunks_per_ticket=grab,
                   strategy=J.JSWEEP_STRATEGY_DATA_DRIVEN)
    for name, p, og, gg in cases[1:4]:
        ref = og.sweep(p.sigma_t, p.q)
        J.set_params(gg, prm)
        try:
            psi = dev(np.zeros((p.n_dirs, p.n_cells)))
            J.sweep(gg, dev(p.sigma_t), dev(p.q), psi)
        finally:
            J.set_params(gg, None)
        err = rel_max(host(psi), ref)
        print(f"[shape {shape}] {name} rel {err:.3e}", flush=True)
        assert err <= 1e-12, (name, shape)


def test_stalled_sweep_reports_and_recovers(oracle_mod, monkeypatch):
    """A stall, forced from the host with a one-tick watchdog (every wave
    that has polled eight times in vain gives up and ends), is reported as
    JSWEEP_E_STALLED; the next sweep on the same graph starts from freshly
    emptied flux arrays and matches the oracle."""
    need_gpu()
    p = W.config(2, "small")
    og = oracle_mod.graph_for(p)
    gg = gpu_graph(p)
    try:
        J.set_params(gg, J.Params(strategy=J.JSWEEP_STRATEGY_DATA_DRIVEN))
        ref = og.sweep(p.sigma_t, p.q)
        psi = dev(np.zeros((p.n_dirs, p.n_cells)))
        J.sweep(gg, dev(p.sigma_t), dev(p.q), psi)
        assert rel_max(host(psi), ref) <= 1e-12
        monkeypatch.setenv("JSWEEP_WATCHDOG_MS", "0.00001")
        with pytest.raises(J.JsweepError) as e:
            J.sweep(gg, dev(p.sigma_t), dev(p.q), dev(np.zeros((p.n_dirs, p.n_cells))))
        assert e.value.code == J.JSWEEP_E_STALLED
        monkeypatch.delenv("JSWEEP_WATCHDOG_MS")
        for rep in range(2):
            psi = dev(np.zeros((p.n_dirs, p.n_cells)))
            J.sweep(gg, dev(p.sigma_t), dev(p.q), psi)
            err = rel_max(host(psi), ref)
            print(f"[stall] recovered sweep {rep} rel {err:.3e}", flush=True)
            assert err <= 1e-12
    finally:
        gg.close()


def test_compact_and_full_programs(oracle_mod, cases):
    """Meshes with more than 3 inflow slots: the jittered 12^3 hexahedra get
    the compact FP64 program (3 slots in the arrays, the rest in the chunk
    blocks); an 8^3 lattice jittered by 0.3 has chunks with too many further
    slots and keeps the full program.  Both sweep and iterate like the
    oracle."""
    need_gpu()
    name, p, og, gg = cases[1]
    info = J.program_info(gg)
    print(f"[program] {name} {info}", flush=True)
    assert info["slots"] > 3 and info["block_slots"] == info["slots"] - 3
    om, w = W.quadrature(8, 3)
    n = 8
    q = W.Problem("hex8_j30", W.hex_lattice(n, 0.3, 2), om, w, np.full(n ** 3, 1.1), np.full(n ** 3, 0.6),
                  np.ones(n ** 3))
    og2 = oracle_mod.graph_for(q)
    gg2 = gpu_graph(q)
    try:
        info = J.program_info(gg2)
        print(f"[program] {q.name} {info}", flush=True)
        assert info["slots"] > 3 and info["block_slots"] == 0
        for g_, o_, pr in ((gg, og, p), (gg2, og2, q)):
            J.set_params(g_, J.Params(strategy=J.JSWEEP_STRATEGY_DATA_DRIVEN))
            try:
                ref = o_.sweep(pr.sigma_t, pr.q)
                psi = dev(np.zeros((pr.n_dirs, pr.n_cells)))
                J.sweep(g_, dev(pr.sigma_t), dev(pr.q), psi)
                assert rel_max(host(psi), ref) <= 1e-12, pr.name
                psi_ref, phi_ref, _ = o_.source_iteration(pr.sigma_t, pr.sigma_s, pr.q, pr.weight, 5)
                phi = dev(np.zeros(pr.n_cells))
                psi = dev(np.zeros((pr.n_dirs, pr.n_cells)))
                J.solve(g_, dev(pr.sigma_t), dev(pr.sigma_s), dev(pr.q), phi, psi, mode=J.JSWEEP_FP64, tol=0.0,
                        max_iter=5, params=J.Params(strategy=J.JSWEEP_STRATEGY_DATA_DRIVEN), allow_not_converged=True)
                e1, e2 = rel_max(host(phi), phi_ref), rel_max(host(psi), psi_ref)
                print(f"[program] {pr.name} SI5 phi {e1:.2e} psi {e2:.2e}", flush=True)
                assert e1 <= 1e-12 and e2 <= 1e-12, pr.name
            finally:
                J.set_params(g_, None)
    finally:
        gg2.close()


def _tiny_problems():
    """The smallest meshes of each kind: one hexahedron, the 6 Kuhn
    tetrahedra of one cube, the triangles of a 2x2 point set; a pure
    absorber (c = 0) and a strong scatterer with boundary inflow."""
    om3, w3 = W.quadrature(8, 3)
    om2, w2 = W.quadrature(4, 2)
    out = []
    for name, mesh, om, w in (("hex1", W.hex_lattice(1), om3, w3), ("kuhn1", W.kuhn_tets(1), om3, w3),
                              ("tri2x2", W.delaunay_2d(2, 2, 0.0, 0), om2, w2)):
        n = mesh.n_cells
        out.append((name + "_absorber", W.Problem(name, mesh, om, w, np.full(n, 2.0), np.zeros(n), np.ones(n)), 0.0))
        out.append((name + "_scatter", W.Problem(name, mesh, om, w, np.full(n, 1.0), np.full(n, 0.99), np.ones(n)),
                    0.5))
    return out


@pytest.mark.parametrize("strategy", [J.JSWEEP_STRATEGY_DATA_DRIVEN, J.JSWEEP_STRATEGY_DIRECTION,
                                      J.JSWEEP_STRATEGY_DIRECTION_LDS, J.JSWEEP_STRATEGY_PATCH])
def test_tiny_meshes(oracle_mod, strategy):
    """Degenerate sizes: every chunk holds one or a few vertices, every
    vertex is a boundary vertex.  One FP64 sweep (with boundary inflow) and
    10 FP64 source iterations match the oracle."""
    need_gpu()
    for name, p, psi_b in _tiny_problems():
        og = oracle_mod.graph_for(p)
        gg = gpu_graph(p)
        try:
            J.set_params(gg, J.Params(strategy=strategy))
            ref = og.sweep(p.sigma_t, p.q, psi_b)
            psi = dev(np.zeros((p.n_dirs, p.n_cells)))
            J.sweep(gg, dev(p.sigma_t), dev(p.q), psi, psi_boundary=psi_b)
            err = rel_max(host(psi), ref)
            psi_ref, phi_ref, _ = og.source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, 10, psi_b=psi_b)
            phi = dev(np.zeros(p.n_cells))
            psi2 = dev(np.zeros((p.n_dirs, p.n_cells)))
            J.solve(gg, dev(p.sigma_t), dev(p.sigma_s), dev(p.q), phi, psi2, psi_boundary=psi_b, mode=J.JSWEEP_FP64,
                    tol=0.0, max_iter=10, params=J.Params(strategy=strategy), allow_not_converged=True)
            e1, e2 = rel_max(host(phi), phi_ref), rel_max(host(psi2), psi_ref)
            print(f"[tiny s{strategy}] {name} cells {p.n_cells} sweep {err:.2e} SI phi {e1:.2e} psi {e2:.2e}",
                  flush=True)
            assert err <= 1e-12 and e1 <= 1e-12 and e2 <= 1e-12, name
        finally:
            gg.close()


@pytest.mark.parametrize("strategy", [J.JSWEEP_STRATEGY_DATA_DRIVEN, J.JSWEEP_STRATEGY_DIRECTION])
def test_directions_parallel_to_faces(oracle_mod, strategy):
    """Omega . S == 0: on an undeformed 5^3 lattice, directions along the
    axes and in the coordinate planes are parallel to whole families of
    faces, which then carry no edge and no flux (neither inflow nor
    outflow).  Sweep and 10 source iterations match the oracle."""
    need_gpu()
    om = np.array([[1.0, 0.0, 0.0], [0.0, -1.0, 0.0], [0.0, 0.0, 1.0], [0.6, 0.8, 0.0], [0.0, -0.6, -0.8],
                   [-1.0, 0.0, 0.0], [0.48, 0.6, 0.64]])
    om = om / np.linalg.norm(om, axis=1, keepdims=True)
    w = np.full(len(om), 1.0 / len(om))
    n = 5
    mesh = W.hex_lattice(n)
    p = W.Problem("hex5_parallel", mesh, om, w, np.full(n ** 3, 1.5), np.full(n ** 3, 0.7), np.ones(n ** 3))
    og = oracle_mod.graph_for(p)
    gg = gpu_graph(p)
    try:
        J.set_params(gg, J.Params(strategy=strategy))
        for m in range(p.n_dirs):
            for x, y in zip(og.direction(m), J.graph_export(gg, m)):
                assert np.array_equal(x, y), m
        ref = og.sweep(p.sigma_t, p.q, 0.3)
        psi = dev(np.zeros((p.n_dirs, p.n_cells)))
        J.sweep(gg, dev(p.sigma_t), dev(p.q), psi, psi_boundary=0.3)
        err = rel_max(host(psi), ref)
        psi_ref, phi_ref, _ = og.source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, 10, psi_b=0.3)
        phi = dev(np.zeros(p.n_cells))
        psi2 = dev(np.zeros((p.n_dirs, p.n_cells)))
        J.solve(gg, dev(p.sigma_t), dev(p.sigma_s), dev(p.q), phi, psi2, psi_boundary=0.3, mode=J.JSWEEP_FP64, tol=0.0,
                max_iter=10, params=J.Params(strategy=strategy), allow_not_converged=True)
        e1, e2 = rel_max(host(phi), phi_ref), rel_max(host(psi2), psi_ref)
        print(f"[parallel s{strategy}] sweep {err:.2e} SI phi {e1:.2e} psi {e2:.2e}", flush=True)
        assert err <= 1e-12 and e1 <= 1e-12 and e2 <= 1e-12
    finally:
        gg.close()


@pytest.mark.parametrize("strategy", [J.JSWEEP_STRATEGY_DATA_DRIVEN, J.JSWEEP_STRATEGY_DIRECTION_LDS,
                                      J.JSWEEP_STRATEGY_PATCH])
def test_many_directions(oracle_mod, strategy):
    """2,000 seeded random directions (beyond the PATCH program's 1,023,
    which then falls back to the work list) on 48 jittered Kuhn tetrahedra:
    sampled graph arrays bit-exact, sweep and 5 source iterations match the
    oracle."""
    need_gpu()
    rng = np.random.default_rng(17)
    om = rng.normal(size=(2000, 3))
    om = om / np.linalg.norm(om, axis=1, keepdims=True)
    w = np.full(len(om), 1.0 / len(om))
    mesh = W.kuhn_tets(2, 0.15, 3)
    n = mesh.n_cells
    p = W.Problem("kuhn2_2000dirs", mesh, om, w, np.full(n, 1.2), np.full(n, 0.8), np.ones(n))
    og = oracle_mod.graph_for(p)
    gg = gpu_graph(p)
    try:
        for m in (0, 999, 1023, 1999):
            for x, y in zip(og.direction(m), J.graph_export(gg, m)):
                assert np.array_equal(x, y), m
        J.set_params(gg, J.Params(strategy=strategy))
        ref = og.sweep(p.sigma_t, p.q)
        psi = dev(np.zeros((p.n_dirs, p.n_cells)))
        J.sweep(gg, dev(p.sigma_t), dev(p.q), psi)
        err = rel_max(host(psi), ref)
        psi_ref, phi_ref, _ = og.source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, 5)
        phi = dev(np.zeros(p.n_cells))
        psi2 = dev(np.zeros((p.n_dirs, p.n_cells)))
        J.solve(gg, dev(p.sigma_t), dev(p.sigma_s), dev(p.q), phi, psi2, mode=J.JSWEEP_FP64, tol=0.0, max_iter=5,
                params=J.Params(strategy=strategy), allow_not_converged=True)
        e1, e2 = rel_max(host(phi), phi_ref), rel_max(host(psi2), psi_ref)
        print(f"[many dirs s{strategy}] sweep {err:.2e} SI phi {e1:.2e} psi {e2:.2e}", flush=True)
        assert err <= 1e-12 and e1 <= 1e-12 and e2 <= 1e-12
    finally:
        gg.close()
