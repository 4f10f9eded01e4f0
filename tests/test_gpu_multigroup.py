"""GPU: multigroup source iteration (every (direction, group) swept in one
launch, Jacobi over groups) through the C ABI against the oracle's
multigroup iteration: fluxes after a fixed number of iterations within
1e-12 (bit-exact in practice), the residual history, convergence to the
oracle's fixed point, one group equal to the single-group solve, and group
counts that leave part of the kernel's group slots empty; sign-tagged and marker
solves alternating on one graph."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import J, dev, gpu_graph, host, need_gpu, rel_max

pytestmark = pytest.mark.gpu


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
        out.append((name, p, oracle_mod.graph_for(p), gpu_graph(p)))
    return out


def _run(gg, mp, iters, tol=0.0, psi_b=0.0, history=0):
    G, nc, nd = mp.n_groups, mp.n_cells, mp.n_dirs
    phi = dev(np.zeros((G, nc)))
    psi = dev(np.zeros((G, nd, nc)))
    st = J.solve_groups(gg, dev(mp.sigma_t), dev(mp.sigma_s), dev(mp.q), phi, psi, psi_boundary=psi_b, tol=tol,
                        max_iter=iters, history=history, allow_not_converged=True)
    return host(phi), host(psi), st


@pytest.mark.parametrize("groups", [1, 2, 3, 4, 6, 8])
def test_groups_fixed_iterations(cases, groups):
    """Six iterations against the oracle (graphs with and without lagged
    edges; group counts odd and even, one, and the kernel's largest), then a
    single-group sweep of the same graph: the multigroup sweep keeps a
    position's groups adjacent in the level-position arrays, and must leave
    the next sweep's array empty for any group count."""
    for name, p, og, gg in cases:
        mp = W.multigroup(p, groups, seed=groups)
        psi_ref, phi_ref, hist = og.mg_source_iteration(mp.sigma_t, mp.sigma_s, mp.q, mp.weight, 6, psi_b=0.2)
        phi, psi, st = _run(gg, mp, 6, psi_b=0.2, history=8)
        e1, e2 = rel_max(phi, phi_ref), rel_max(psi, psi_ref)
        print(f"[groups {groups}] {name} phi {e1:.2e} psi {e2:.2e} bitexact {np.array_equal(psi, psi_ref)} "
              f"rho {st['residual']:.3e} vs {hist[-1]:.3e}", flush=True)
        assert st["sweeps"] == 6
        assert e1 <= 1e-12 and e2 <= 1e-12, name
        assert np.allclose(st["history"], hist, rtol=1e-9, atol=0), name
        out = dev(np.zeros((p.n_dirs, p.n_cells)))
        J.sweep(gg, dev(p.sigma_t), dev(p.q), out)
        assert np.array_equal(host(out), og.sweep(p.sigma_t, p.q)), name


def test_groups_converge_to_oracle(cases):
    for name, p, og, gg in cases[:2]:
        mp = W.multigroup(p, 4, seed=11)
        _, phi_ref, hist = og.mg_source_iteration(mp.sigma_t, mp.sigma_s, mp.q, mp.weight, 5000, 1e-13)
        phi, _, st = _run(gg, mp, 5000, tol=1e-11)
        err = float(np.linalg.norm(phi - phi_ref) / np.linalg.norm(phi_ref))
        print(f"[groups conv] {name} iterations {st['sweeps']} (oracle {len(hist)}) rho {st['residual']:.2e} "
              f"phi rel {err:.2e}", flush=True)
        assert st["converged"] and st["residual"] <= 1e-11
        assert err <= 1e-9


def test_one_group_equals_single_group_solve(cases):
    name, p, og, gg = cases[0]
    mp = W.multigroup(p, 1, seed=3)
    phi, psi, _ = _run(gg, mp, 8)
    phi1 = dev(np.zeros(p.n_cells))
    psi1 = dev(np.zeros((p.n_dirs, p.n_cells)))
    J.solve(gg, dev(mp.sigma_t[0]), dev(mp.sigma_s[0, 0]), dev(mp.q[0]), phi1, psi1, mode=J.JSWEEP_FP64, tol=0.0,
            max_iter=8, allow_not_converged=True)
    assert rel_max(phi[0], host(phi1)) <= 1e-13 and rel_max(psi[0], host(psi1)) <= 1e-13
    # the single-group sweeps that follow still see empty level-position arrays
    ref = og.sweep(p.sigma_t, p.q)
    out = dev(np.zeros((p.n_dirs, p.n_cells)))
    J.sweep(gg, dev(p.sigma_t), dev(p.q), out)
    assert np.array_equal(host(out), ref)


def test_groups_bad_arguments(cases):
    name, p, og, gg = cases[2]
    mp = W.multigroup(p, 9, seed=1)
    with pytest.raises(J.JsweepError) as e:
        _run(gg, mp, 2)
    assert e.value.code == J.JSWEEP_E_INVALID_ARG


def test_groups_tagged_and_marker_solves_alternate(cases):
    """With every input non-negative the multigroup sweeps tag their fluxes
    by sign; a negative source or inflow makes them write markers.  On one
    graph (with and without lagged edges): solves that switch between the
    two, change the group count and use odd and even iteration counts, then
    a single-group sweep; every result against the oracle."""
    rng = np.random.default_rng(5)
    for name, p, og, gg in cases[:2]:
        m4 = W.multigroup(p, 4, seed=21)
        m3 = W.multigroup(p, 3, seed=22)
        q4neg = m4.q.copy()
        q4neg[1] -= 1.5 * rng.random(p.n_cells)      # a negative source in one group
        assert (q4neg < 0).any()
        # (groups' problem, source, inflow, iterations)
        steps = [(m4, m4.q, 0.2, 5), (m4, q4neg, 0.2, 4), (m3, m3.q, 0.0, 3), (m3, m3.q, 0.1, 2),
                 (m4, m4.q, -0.1, 3), (m4, m4.q, 0.0, 4)]
        for i, (mp, q, psi_b, iters) in enumerate(steps):
            psi_ref, phi_ref, _ = og.mg_source_iteration(mp.sigma_t, mp.sigma_s, q, mp.weight, iters, psi_b=psi_b)
            G = mp.n_groups
            phi = dev(np.zeros((G, p.n_cells)))
            psi = dev(np.zeros((G, p.n_dirs, p.n_cells)))
            J.solve_groups(gg, dev(mp.sigma_t), dev(mp.sigma_s), dev(q), phi, psi, psi_boundary=psi_b, tol=0.0,
                           max_iter=iters, allow_not_converged=True)
            e1, e2 = rel_max(host(phi), phi_ref), rel_max(host(psi), psi_ref)
            kind = "negative" if (q < 0).any() or psi_b < 0 else "non-negative"
            print(f"[groups tags] {name} step {i} ({G} groups, {kind} inputs, {iters} iterations): phi {e1:.2e} "
                  f"psi {e2:.2e} bitexact {np.array_equal(host(psi), psi_ref)}", flush=True)
            assert e1 <= 1e-12 and e2 <= 1e-12, (name, i)
        out = dev(np.zeros((p.n_dirs, p.n_cells)))
        J.sweep(gg, dev(p.sigma_t), dev(p.q), out)
        assert np.array_equal(host(out), og.sweep(p.sigma_t, p.q)), name
