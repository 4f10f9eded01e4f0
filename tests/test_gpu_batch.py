"""GPU: batched ensemble solves (one sweep launch for every instance),
autotuning and solver options, against the oracle."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import J, dev, gpu_graph, host, need_gpu, rel_max, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ensemble(oracle_mod):
    need_gpu()
    probs = W.ensemble(seed=4, count=6, min_cells=300, max_cells=2500)
    out = []
    for p in probs:
        print(f"[instance] {p.name} dim {p.mesh.dim} cells {p.n_cells} dirs {p.n_dirs} c {p.meta['c']:.3f}", flush=True)
        out.append((p, oracle_mod.graph_for(p), gpu_graph(p)))
    return out


def _problems(ens):
    return [{"sigma_t": dev(p.sigma_t), "sigma_s": dev(p.sigma_s), "q": dev(p.q),
             "phi": dev(np.zeros(p.n_cells)), "psi": dev(np.zeros((p.n_dirs, p.n_cells)))} for p, _, _ in ens]


def test_batch_fp64_matches_oracle_after_20_iterations(ensemble):
    probs = _problems(ensemble)
    stats = J.solve_batch([g for _, _, g in ensemble], probs, mode=J.JSWEEP_FP64, tol=0.0, max_iter=20,
                          allow_not_converged=True)
    for (p, og, _), pr, st in zip(ensemble, probs, stats):
        psi_ref, phi_ref, hist = og.source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, 20)
        e1, e2 = rel_max(host(pr["phi"]), phi_ref), rel_max(host(pr["psi"]), psi_ref)
        print(f"[batch64] {p.name} phi {e1:.2e} psi {e2:.2e} sweeps {st['sweeps']} rho {st['residual']:.2e}", flush=True)
        assert st["sweeps"] == 20
        assert e1 <= 1e-12 and e2 <= 1e-12


@pytest.mark.parametrize("strategy", [J.JSWEEP_STRATEGY_DIRECTION, J.JSWEEP_STRATEGY_DIRECTION_LDS,
                                      J.JSWEEP_STRATEGY_DATA_DRIVEN])
def test_batch_fp64_each_sweep_kernel(ensemble, strategy):
    """The batched direction kernels (plain and LDS-window) and the union of
    the instances' work lists in one data-driven launch."""
    probs = _problems(ensemble)
    stats = J.solve_batch([g for _, _, g in ensemble], probs, mode=J.JSWEEP_FP64, tol=0.0, max_iter=5,
                          params=J.Params(strategy=strategy), allow_not_converged=True)
    for (p, og, _), pr, st in zip(ensemble, probs, stats):
        psi_ref, phi_ref, _ = og.source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, 5)
        e1, e2 = rel_max(host(pr["phi"]), phi_ref), rel_max(host(pr["psi"]), psi_ref)
        print(f"[batch64 s{strategy}] {p.name} phi {e1:.2e} psi {e2:.2e}", flush=True)
        assert st["sweeps"] == 5
        assert e1 <= 1e-12 and e2 <= 1e-12


@pytest.mark.parametrize("strategy", [J.JSWEEP_STRATEGY_DATA_DRIVEN, J.JSWEEP_STRATEGY_AUTO])
def test_batch_data_driven_partial_convergence_and_boundary(ensemble, strategy):
    """Union sweep with instances converging at different iterations and
    boundary inflow per instance: each instance's result equals its own
    solve.  DATA_DRIVEN keeps every instance in the list (the chunks of a
    converged instance only empty their entries); AUTO compacts the list to
    the instances still iterating once they hold less than half of its
    work (here after the tenth sweep, when two of the six still iterate)."""
    probs = _problems(ensemble)
    for k, pr in enumerate(probs):
        pr["psi_boundary"] = 0.1 * k
    stats = J.solve_batch([g for _, _, g in ensemble], probs, mode=J.JSWEEP_FP64, tol=1e-9, max_iter=2000,
                          params=J.Params(strategy=strategy))
    sweeps = [st["sweeps"] for st in stats]
    print(f"[batch64 union tol s{strategy}] sweeps {sweeps}", flush=True)
    assert len(set(sweeps)) > 1
    for k, ((p, og, g), pr, st) in enumerate(zip(ensemble, probs, stats)):
        psi_ref, phi_ref, hist = og.source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, st["sweeps"], psi_b=0.1 * k)
        assert rel_max(host(pr["phi"]), phi_ref) <= 1e-12, p.name
        # the angular fluxes of the iterate the instance stopped at, though
        # the batch went on sweeping the others
        assert rel_max(host(pr["psi"]), psi_ref) <= 1e-12, p.name
        assert st["residual"] <= 1e-9 and abs(st["residual"] - hist[-1]) <= 1e-6 * hist[-1]


def test_batch_refined_converges_to_oracle(ensemble):
    probs = _problems(ensemble)
    stats = J.solve_batch([g for _, _, g in ensemble], probs, mode=J.JSWEEP_FP32_REFINED, tol=1e-11, max_iter=20000)
    for (p, og, _), pr, st in zip(ensemble, probs, stats):
        _, phi_ref, hist = og.source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, 20000, 1e-13)
        got = host(pr["phi"])
        err = float(np.linalg.norm(got - phi_ref) / np.linalg.norm(phi_ref))
        print(f"[batch32] {p.name} outer {st['outer_iters']} sweeps {st['sweeps']} (oracle {len(hist)}) "
              f"rho {st['residual']:.2e} phi rel {err:.2e}", flush=True)
        assert st["residual"] <= 1e-11
        assert err <= 1e-8


def test_autotune_and_tuned_solve(ensemble):
    p, og, g = ensemble[1]
    prm = J.autotune([g], J.JSWEEP_FP64)
    d = prm.as_dict()
    assert d["strategy"] in (J.JSWEEP_STRATEGY_DATA_DRIVEN, J.JSWEEP_STRATEGY_DIRECTION,
                             J.JSWEEP_STRATEGY_DIRECTION_LDS, J.JSWEEP_STRATEGY_PATCH)
    assert d["strategy"] == J.JSWEEP_STRATEGY_DIRECTION_LDS or d["waves_per_block"] >= 1
    phi = dev(np.zeros(p.n_cells))
    J.solve(g, dev(p.sigma_t), dev(p.sigma_s), dev(p.q), phi, mode=J.JSWEEP_FP64, tol=0.0, max_iter=5,
            params=prm, allow_not_converged=True)
    _, phi_ref, _ = og.source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, 5)
    assert rel_max(host(phi), phi_ref) <= 1e-12
    prm_b = J.autotune([g for _, _, g in ensemble], J.JSWEEP_FP32_REFINED)
    # batches: the direction kernels, or the default hybrid (AUTO: the union
    # launch while most of the batch iterates)
    assert prm_b.as_dict()["strategy"] in (J.JSWEEP_STRATEGY_DIRECTION, J.JSWEEP_STRATEGY_DIRECTION_LDS,
                                           J.JSWEEP_STRATEGY_AUTO)


def test_warm_start_boundary_and_not_converged(ensemble):
    p, og, g = ensemble[0]
    st_, ss, q = dev(p.sigma_t), dev(p.sigma_s), dev(p.q)
    # 10 + 10 iterations with a warm start equal 20 from zero
    psi = dev(np.zeros((p.n_dirs, p.n_cells)))
    phi = dev(np.zeros(p.n_cells))
    r = J.solve(g, st_, ss, q, phi, psi, psi_boundary=0.4, mode=J.JSWEEP_FP64, tol=0.0, max_iter=10,
                allow_not_converged=True)
    assert not r["converged"]
    J.solve(g, st_, ss, q, phi, psi, psi_boundary=0.4, mode=J.JSWEEP_FP64 | J.JSWEEP_WARM_START, tol=0.0,
            max_iter=10, allow_not_converged=True)
    psi_ref, phi_ref, _ = og.source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, 20, psi_b=0.4)
    assert rel_max(host(phi), phi_ref) <= 1e-12 and rel_max(host(psi), psi_ref) <= 1e-12
    with pytest.raises(J.JsweepError) as e:
        J.solve(g, st_, ss, q, phi, mode=J.JSWEEP_FP64, tol=1e-30, max_iter=3)
    assert e.value.code == J.JSWEEP_E_NOT_CONVERGED


def test_residual_history(ensemble):
    p, og, g = ensemble[2]
    phi = dev(np.zeros(p.n_cells))
    r = J.solve(g, dev(p.sigma_t), dev(p.sigma_s), dev(p.q), phi, mode=J.JSWEEP_FP64, tol=0.0, max_iter=8,
                history=16, allow_not_converged=True)
    _, _, hist = og.source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, 8)
    assert len(r["history"]) == 8
    assert np.allclose(r["history"], hist, rtol=1e-9, atol=1e-300)


ENSEMBLE_GOLDEN = (49, 86, 95, 216)   # smallest / largest tetrahedron and triangle meshes of the ensemble


def test_full_ensemble_256():
    """The whole 256-instance ensemble (500 - 50,000 cells, S4 - S8) in one
    batch: 20 FP64 source iterations against the oracle's sampled fluxes of
    its smallest and largest triangle and tetrahedron instances
    (tests/golden/fullsize_ens<i>.txt, oracle-only), then FP32-refined and
    FP64 batch solves to rho <= 1e-11, with the autotuned parameters and
    with the plain direction kernel, against the oracle's converged fluxes
    of those instances and against each other for every instance."""
    need_gpu()
    import os
    import sys
    sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden"))
    from make_fullsize_golden import load
    ps = W.ensemble(seed=4, count=256, min_cells=500, max_cells=50000)
    print(f"[ensemble] {len(ps)} instances, {sum(p.n_cells for p in ps)} cells", flush=True)
    gs = [gpu_graph(p) for p in ps]
    try:
        tuned = J.autotune(gs, J.JSWEEP_FP32_REFINED)
        print(f"[ensemble] autotuned {tuned.as_dict()}", flush=True)

        def problems():
            return [{"sigma_t": dev(p.sigma_t), "sigma_s": dev(p.sigma_s), "q": dev(p.q),
                     "phi": dev(np.zeros(p.n_cells)), "psi": dev(np.zeros((p.n_dirs, p.n_cells)))} for p in ps]

        pr = problems()
        J.solve_batch(gs, pr, mode=J.JSWEEP_FP64, tol=0.0, max_iter=20, params=tuned, allow_not_converged=True)
        gold = {i: load(f"ens{i}") for i in ENSEMBLE_GOLDEN}
        for i, gd in gold.items():
            ph = host(pr[i]["phi"])
            psi = host(pr[i]["psi"])
            e1 = rel_max(ph[gd["cells"]], gd["phi_fixed"])
            e2 = rel_max(psi[gd["psi_m"], gd["psi_k"]], gd["psi"])
            print(f"[ensemble] instance {i} ({ps[i].n_cells} cells, {ps[i].n_dirs} dirs) 20 SI: phi {e1:.2e} "
                  f"psi {e2:.2e}", flush=True)
            assert e1 <= 1e-12 and e2 <= 1e-12, i
        sols = {}
        for label, mode, prm in (("fp64", J.JSWEEP_FP64, tuned), ("refined", J.JSWEEP_FP32_REFINED, tuned),
                                 ("refined_plain", J.JSWEEP_FP32_REFINED,
                                  J.Params(strategy=J.JSWEEP_STRATEGY_DIRECTION)),
                                 ("refined_union", J.JSWEEP_FP32_REFINED,
                                  J.Params(strategy=J.JSWEEP_STRATEGY_DATA_DRIVEN))):
            pr = problems()
            st = J.solve_batch(gs, pr, mode=mode, tol=1e-11, max_iter=20000, params=prm)
            sols[label] = [host(x["phi"]) for x in pr]
            assert max(x["residual"] for x in st) <= 1e-11, label
            for i, gd in gold.items():
                ref = gd["phi_converged"]
                got = sols[label][i][gd["cells"]]
                err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
                print(f"[ensemble] {label} instance {i}: sweeps {st[i]['sweeps']} rho {st[i]['residual']:.2e} "
                      f"phi vs oracle {err:.2e}", flush=True)
                assert err <= 1e-8, (label, i)
        for label in ("refined", "refined_plain", "refined_union"):
            worst = max(float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(sols[label], sols["fp64"]))
            print(f"[ensemble] {label} vs fp64: worst instance phi rel {worst:.2e}", flush=True)
            assert worst <= 1e-8
    finally:
        for g in gs:
            g.close()


@pytest.mark.parametrize("strategy", [J.JSWEEP_STRATEGY_DATA_DRIVEN, J.JSWEEP_STRATEGY_AUTO,
                                      J.JSWEEP_STRATEGY_DIRECTION])
def test_batch_with_lagged_edges(oracle_mod, strategy):
    """Instances whose graphs have cycles (lagged edges: the deformed hex
    lattices) batched with a lag-free one: the union keeps its FP64 fluxes
    in level order, so the lagged values and their residual terms are read
    at the level positions; after a fixed number of iterations, and to a
    tolerance where the instances stop at different sweeps (psi from the
    iterate each stopped at), every instance against the oracle."""
    need_gpu()
    ps = [W.config(2, "small"),
          W.Problem("hex3cyc", W.hex_lattice(3, 0.3, 1), *W.quadrature(8, 3), np.full(27, 1.3), np.full(27, 0.9),
                    np.ones(27)),
          W.config(3, "small")]
    ogs = [oracle_mod.graph_for(p) for p in ps]
    assert ogs[0].n_lagged > 0 and ogs[1].n_lagged > 0 and ogs[2].n_lagged == 0
    gs = [gpu_graph(p) for p in ps]
    try:
        for tol, iters in ((0.0, 7), (1e-9, 2000)):
            pr = [{"sigma_t": dev(p.sigma_t), "sigma_s": dev(p.sigma_s), "q": dev(p.q), "phi": dev(np.zeros(p.n_cells)),
                   "psi": dev(np.zeros((p.n_dirs, p.n_cells))), "psi_boundary": 0.1 * k} for k, p in enumerate(ps)]
            st = J.solve_batch(gs, pr, mode=J.JSWEEP_FP64, tol=tol, max_iter=iters,
                               params=J.Params(strategy=strategy), allow_not_converged=tol == 0.0)
            for k, (p, og) in enumerate(zip(ps, ogs)):
                psi_ref, phi_ref, _ = og.source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, st[k]["sweeps"],
                                                          psi_b=0.1 * k)
                e1, e2 = rel_max(host(pr[k]["phi"]), phi_ref), rel_max(host(pr[k]["psi"]), psi_ref)
                print(f"[batch lagged s{strategy} tol {tol}] {p.name}: sweeps {st[k]['sweeps']} phi {e1:.2e} "
                      f"psi {e2:.2e}", flush=True)
                assert e1 <= 1e-12 and e2 <= 1e-12, (p.name, tol)
    finally:
        for g in gs:
            g.close()
