"""GPU: jsweep_sweep_noalloc (the sweep entry point that allocates no device
memory, staging V s in the library's fixed device array) against
jsweep_sweep, through the C ABI: bit-identical angular and scalar fluxes on
two calls in a row, the second on a smaller graph, and again after a
regular sweep on the first graph."""
import numpy as np
import pytest

import workloads as W
from tests.gpu_common import J, dev, gpu_graph, host, need_gpu

pytestmark = pytest.mark.gpu


def _sweep(fn, g, p, psi_b, prev):
    psi = dev(prev)
    phi = dev(np.zeros(p.n_cells))
    fn(g, dev(p.sigma_t), dev(p.q), psi, phi, psi_boundary=psi_b)
    return host(psi), host(phi)


def test_noalloc_sweep_matches_sweep():
    need_gpu()
    big, small = W.config(3, "small"), W.config(2, "small")      # 24,576 tets S8; 1,728 hexes S8 (lagged edges)
    assert small.n_cells < big.n_cells
    graphs = {}
    try:
        for p in (big, small):
            graphs[p.name] = gpu_graph(p)
        rng = np.random.default_rng(5)
        for p, psi_b in ((big, 0.0), (small, 0.35), (big, 0.1)):
            g = graphs[p.name]
            prev = rng.uniform(0.0, 1.0, (p.n_dirs, p.n_cells))   # read on lagged edges
            print(f"[noalloc] {p.name} cells {p.n_cells} psi_b {psi_b}", flush=True)
            a_psi, a_phi = _sweep(J.sweep_noalloc, g, p, psi_b, prev)
            b_psi, b_phi = _sweep(J.sweep, g, p, psi_b, prev)
            assert np.array_equal(a_psi, b_psi) and np.array_equal(a_phi, b_phi), p.name
            assert np.isfinite(a_psi).all() and a_psi.max() > 0.0
    finally:
        for g in graphs.values():
            g.close()


def test_noalloc_rejects_other_strategies():
    need_gpu()
    p = W.config(2, "small")
    g = gpu_graph(p)
    try:
        J.set_params(g, J.Params(strategy=J.JSWEEP_STRATEGY_DIRECTION))
        with pytest.raises(J.JsweepError) as e:
            _sweep(J.sweep_noalloc, g, p, 0.0, np.zeros((p.n_dirs, p.n_cells)))
        assert e.value.code == J.JSWEEP_E_INVALID_ARG
    finally:
        g.close()
