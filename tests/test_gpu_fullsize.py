"""GPU parity at the benchmark sizes, with the default launch configuration.

* jittered 64^3 hexahedra, S8 (262,144 cells x 80 directions, 236 lagged
  edges): graph arrays and lagged edges bit-exact for every direction, the
  compact FP64 program in use, one FP64 sweep and three FP64 source
  iterations against the oracle, and the FP32-refined solve to 1e-8 against
  the FP64 one;
* Kuhn tetrahedra of a 96^3 lattice, S8 (5.3M cells x 80 directions) and
  of a 60^3 lattice, S16 (1.3M cells x 288 directions): the oracle is built
  for four sampled directions only (directions are independent), and the
  GPU graph arrays and FP64 sweep of those directions are compared;
* against the sampled oracle fluxes of tests/golden/fullsize_<name>.txt
  (written by the oracle-only script there): 20 FP64 source iterations of
  the hexahedral workload and 2 of each tetrahedral one over every
  direction (scalar flux at 2,048 cells, angular flux at 1,024 (direction,
  cell) pairs, within 1e-12), and the FP64 and FP32-refined solves to
  rho <= 1e-11 against the oracle's solution at rho <= 1e-13 (within 1e-8)
  and against each other."""
import os
import sys

import numpy as np
import pytest

import workloads as W
from tests.gpu_common import J, dev, gpu_graph, host, need_gpu, rel_max, torch

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    sys.path.insert(0, GOLDEN)
    from make_fullsize_golden import load
    return load(name)


@pytest.mark.parametrize("k,name", [(2, "hex64_s8"), (3, "tetcheck96_s8"), (5, "tetlogn60_s16")])
def test_full_source_iterations_vs_oracle_samples(k, name):
    need_gpu()
    gold = golden(name)
    n_it = gold["fixed_iterations"]
    p = W.config(k)
    print(f"[case] {name} cells={p.n_cells} dirs={p.n_dirs} iterations={n_it}", flush=True)
    gg = gpu_graph(p)
    try:
        phi = dev(np.zeros(p.n_cells))
        psi = torch.zeros(p.n_dirs * p.n_cells, dtype=torch.float64, device="cuda")
        st = J.solve(gg, dev(p.sigma_t), dev(p.sigma_s), dev(p.q), phi, psi, mode=J.JSWEEP_FP64, tol=0.0,
                     max_iter=n_it, allow_not_converged=True)
        assert st["sweeps"] == n_it
        ph = host(phi)
        got_phi = ph[gold["cells"]]
        got_psi = psi.view(p.n_dirs, p.n_cells)[torch.as_tensor(gold["psi_m"]), torch.as_tensor(gold["psi_k"])]
        got_psi = host(got_psi)
        e1, e2 = rel_max(got_phi, gold["phi_fixed"]), rel_max(got_psi, gold["psi"])
        big, val = gold["fixed_max_cell"]
        print(f"[{name}] {n_it} SI: phi {e1:.2e} psi {e2:.2e} bitexact {np.array_equal(got_phi, gold['phi_fixed'])} "
              f"max cell {int(np.argmax(ph))} vs {big}", flush=True)
        assert e1 <= 1e-12 and e2 <= 1e-12
        assert abs(ph[big] - val) <= 1e-12 * abs(val)
    finally:
        gg.close()


@pytest.mark.parametrize("k,name", [(3, "tetcheck96_s8"), (5, "tetlogn60_s16")])
def test_full_refined_vs_fp64_and_oracle(k, name):
    need_gpu()
    gold = golden(name)
    p = W.config(k)
    print(f"[case] {name} refined and FP64 to 1e-11", flush=True)
    gg = gpu_graph(p)
    try:
        sol = {}
        for mode in (J.JSWEEP_FP64, J.JSWEEP_FP32_REFINED):
            phi = dev(np.zeros(p.n_cells))
            st = J.solve(gg, dev(p.sigma_t), dev(p.sigma_s), dev(p.q), phi, mode=mode, tol=1e-11, max_iter=5000)
            ph = host(phi)
            sol[mode] = ph
            ref = gold["phi_converged"]
            got = ph[gold["cells"]]
            err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
            print(f"[{name}] mode {mode}: sweeps {st['sweeps']} outer {st['outer_iters']} rho {st['residual']:.2e} "
                  f"phi vs oracle (sampled) {err:.2e}", flush=True)
            assert st["residual"] <= 1e-11
            assert err <= 1e-8
        err = float(np.linalg.norm(sol[J.JSWEEP_FP32_REFINED] - sol[J.JSWEEP_FP64]) /
                    np.linalg.norm(sol[J.JSWEEP_FP64]))
        print(f"[{name}] refined vs FP64 phi rel {err:.2e}", flush=True)
        assert err <= 1e-8
    finally:
        gg.close()


def test_hex64_s8_full(oracle_mod):
    need_gpu()
    p = W.config(2)
    print(f"[case] {p.name} cells={p.n_cells} dirs={p.n_dirs}", flush=True)
    og = oracle_mod.graph_for(p)
    gg = gpu_graph(p)
    info = J.graph_info(gg)
    assert info["n_lagged"] == og.n_lagged > 0 and info["max_levels"] == og.max_levels
    prog = J.program_info(gg)
    print(f"[hex64] program {prog}", flush=True)
    assert prog["slots"] == 5 and prog["block_slots"] == 2   # the compact FP64 program
    for m in range(p.n_dirs):
        for x, y in zip(og.direction(m), J.graph_export(gg, m)):
            assert np.array_equal(x, y), m
    for x, y in zip(og.lagged(), J.graph_lagged(gg)):
        assert np.array_equal(x, y)
    ref = og.sweep(p.sigma_t, p.q)
    psi = dev(np.zeros((p.n_dirs, p.n_cells)))
    J.sweep(gg, dev(p.sigma_t), dev(p.q), psi)
    got = psi.cpu().numpy()
    print(f"[hex64] sweep rel {rel_max(got, ref):.2e} bitexact {np.array_equal(got, ref)}", flush=True)
    assert rel_max(got, ref) <= 1e-12
    info = J.patch_info(gg)
    print(f"[hex64] patch program {info}", flush=True)
    assert info["available"]
    psi_ref, phi_ref, _ = og.source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, 3)
    for strategy in (J.JSWEEP_STRATEGY_AUTO, J.JSWEEP_STRATEGY_DATA_DRIVEN, J.JSWEEP_STRATEGY_DIRECTION_LDS,
                     J.JSWEEP_STRATEGY_PATCH):
        phi = dev(np.zeros(p.n_cells))
        psi = dev(np.zeros((p.n_dirs, p.n_cells)))
        J.solve(gg, dev(p.sigma_t), dev(p.sigma_s), dev(p.q), phi, psi, mode=J.JSWEEP_FP64, tol=0.0, max_iter=3,
                params=J.Params(strategy=strategy), allow_not_converged=True)
        e1, e2 = rel_max(phi.cpu().numpy(), phi_ref), rel_max(psi.cpu().numpy(), psi_ref)
        print(f"[hex64] 3 SI strategy {strategy}: phi {e1:.2e} psi {e2:.2e}", flush=True)
        assert e1 <= 1e-12 and e2 <= 1e-12
    # FP32-refined solve to 1e-8 against the FP64 one (pinned to the oracle
    # above): the same flux within the refined tolerance, and no more outer
    # iterations or sweeps than a correct correction source needs (a
    # misplaced per-direction residual would leave the corrections poor)
    sol = {}
    for mode in (J.JSWEEP_FP64, J.JSWEEP_FP32_REFINED):
        phi = dev(np.zeros(p.n_cells))
        st = J.solve(gg, dev(p.sigma_t), dev(p.sigma_s), dev(p.q), phi, mode=mode, tol=1e-8, max_iter=200)
        sol[mode] = (phi.cpu().numpy(), st)
        print(f"[hex64] to 1e-8 mode {mode}: sweeps {st['sweeps']} outer {st['outer_iters']} "
              f"rho {st['residual']:.2e}", flush=True)
        assert st["residual"] <= 1e-8
    (phi64, st64), (phi32, st32) = sol[J.JSWEEP_FP64], sol[J.JSWEEP_FP32_REFINED]
    err = float(np.linalg.norm(phi32 - phi64) / np.linalg.norm(phi64))
    print(f"[hex64] refined vs FP64 phi rel {err:.2e}", flush=True)
    assert err <= 1e-8
    assert st32["outer_iters"] <= 4 and st32["sweeps"] <= st64["sweeps"] + 4


@pytest.mark.parametrize("k,sample", [(3, [0, 17, 45, 79]), (5, [0, 100, 200, 287])])
def test_tet_full_sampled_directions(oracle_mod, k, sample):
    need_gpu()
    p = W.config(k)
    print(f"[case] {p.name} cells={p.n_cells} dirs={p.n_dirs} sample={sample}", flush=True)
    gg = gpu_graph(p)
    prog = J.program_info(gg)
    assert prog["slots"] <= 3 and prog["block_slots"] == 0   # a tet has at most 3 inflow faces
    og = oracle_mod.Graph(p.mesh, p.omega[sample])
    for i, m in enumerate(sample):
        for x, y in zip(og.direction(i), J.graph_export(gg, m)):
            assert np.array_equal(x, y), m
    psi = torch.zeros(p.n_dirs * p.n_cells, dtype=torch.float64, device="cuda")
    J.sweep(gg, dev(p.sigma_t), dev(p.q), psi)
    ref = og.sweep(p.sigma_t, p.q)
    got = psi.view(p.n_dirs, p.n_cells)[sample].cpu().numpy()
    err = rel_max(got, ref)
    print(f"[{p.name}] sampled sweep rel {err:.2e} bitexact {np.array_equal(got, ref)}", flush=True)
    assert err <= 1e-12
