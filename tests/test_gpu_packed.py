"""GPU: the work-list sweep's packed upwind positions (three 21-bit
distances back from the vertex's own level position per 8-byte word; the
codes that do not fit are entries of the chunk block).

The largest packed distance is lowered through JSWEEP_PACK_MAX_DELTA when
the graph is built, so that many codes escape.  From the oracle's level
order the test predicts, chunk by chunk, how many (vertex, inflow face)
codes escape; the graph must use packed codes exactly when no chunk has
more than 12 of them, and every sweep and source iteration must stay
bit-identical to the oracle either way."""
import os

import numpy as np
import pytest

import workloads as W
from tests.gpu_common import J, dev, host, need_gpu, rel_max

pytestmark = pytest.mark.gpu

KEY = "JSWEEP_PACK_MAX_DELTA"
ESC_MAX = 12


def _escapes(og, omega, max_delta):
    """Largest number of escaped codes in any chunk (64 consecutive level
    positions of one (direction, level)), and the total."""
    S, fcell, _, _ = og.geometry()
    inner = fcell[:, 1] >= 0
    a, b, Si = fcell[inner, 0], fcell[inner, 1], S[inner]
    worst, total = 0, 0
    for m in range(og.n_dirs):
        _, level, lp, lc = og.direction(m)
        om = omega[m]
        d = om[0] * Si[:, 0] + om[1] * Si[:, 1]
        if Si.shape[1] > 2:
            d = d + om[2] * Si[:, 2]
        e = d != 0.0
        ea, eb = a[e], b[e]
        up = np.where(level[ea] < level[eb], ea, eb)
        dn = np.where(level[ea] < level[eb], eb, ea)
        pos = np.empty(og.n_cells, np.int64)
        pos[lc] = np.arange(og.n_cells)
        far = pos[dn] - pos[up] > max_delta
        if not far.any():
            continue
        L = level[dn[far]]
        chunk = L.astype(np.int64) * (og.n_cells + 1) + (pos[dn[far]] - lp[L]) // 64
        _, counts = np.unique(chunk, return_counts=True)
        worst = max(worst, int(counts.max()))
        total += int(far.sum())
    return worst, total


def _graph(p, max_delta=None):
    old = os.environ.get(KEY)
    try:
        if max_delta is None:
            os.environ.pop(KEY, None)
        else:
            os.environ[KEY] = str(max_delta)
        return J.build_graph(p.mesh, p.omega, p.weight)
    finally:
        if old is None:
            os.environ.pop(KEY, None)
        else:
            os.environ[KEY] = old


# distances tried per mesh: the default, then lowered ones (on the 16^3 tet
# mesh 12,000 and 8,000 leave 4 and 10 escaped codes in the worst chunk,
# 4,000 leaves 20; on the triangles 400 and 150 leave 4 and 7, 60 leaves 17)
@pytest.mark.parametrize("name,k,dists", [("tetcheck16_s8", 3, (None, 12000, 8000, 4000)),
                                          ("delaunay40x50_s4", 1, (None, 400, 150, 60))])
def test_packed_codes_with_escapes(oracle_mod, name, k, dists):
    need_gpu()
    p = W.config(k, "small") if k == 3 else W.config(k)
    print(f"[case] {name} cells={p.n_cells} dirs={p.n_dirs}", flush=True)
    og = oracle_mod.graph_for(p)
    ref = og.sweep(p.sigma_t, p.q)
    psi_ref, phi_ref, _ = og.source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, 4)
    seen_escaping_packed = False
    for md in dists:
        worst, total = _escapes(og, p.omega, md if md is not None else (1 << 21) - 4)
        want_packed = worst <= ESC_MAX
        g = _graph(p, md)
        try:
            info = J.program_info(g)
            print(f"[packed {name}] max distance {md}: escaped codes {total}, at most {worst} per chunk, "
                  f"packed {info['packed']} (expected {want_packed})", flush=True)
            assert info["packed"] == want_packed
            seen_escaping_packed |= info["packed"] and total > 0
            psi = dev(np.zeros((p.n_dirs, p.n_cells)))
            J.sweep(g, dev(p.sigma_t), dev(p.q), psi)
            assert np.array_equal(host(psi), ref), md
            for mode in (J.JSWEEP_FP64, J.JSWEEP_FP32_REFINED):
                phi = dev(np.zeros(p.n_cells))
                psi = dev(np.zeros((p.n_dirs, p.n_cells)))
                if mode == J.JSWEEP_FP64:
                    J.solve(g, dev(p.sigma_t), dev(p.sigma_s), dev(p.q), phi, psi, mode=mode, tol=0.0, max_iter=4,
                            allow_not_converged=True)
                    assert rel_max(host(phi), phi_ref) <= 1e-12 and rel_max(host(psi), psi_ref) <= 1e-12
                else:
                    st = J.solve(g, dev(p.sigma_t), dev(p.sigma_s), dev(p.q), phi, mode=mode, tol=1e-10,
                                 max_iter=500)
                    assert st["residual"] <= 1e-10
        finally:
            g.close()
    assert seen_escaping_packed, "no tried distance left escaped codes in a packed program"


def test_hex_program_not_packed():
    need_gpu()
    p = W.config(2, "small")
    g = J.build_graph(p.mesh, p.omega, p.weight)
    try:
        info = J.program_info(g)
        assert info["slots"] > 3 and not info["packed"]
    finally:
        g.close()


def test_batch_union_packed_with_escapes(oracle_mod):
    """The batched union builds packed codes of its merged program (the
    instances' lagged indices rebased, escapes like any other): with the
    largest distance lowered to 800, four small instances keep packed
    programs while 842 codes escape; 10 FP64 iterations of the union sweep
    against the oracle, and an FP32-refined batch solve."""
    need_gpu()
    import torch
    ps = W.ensemble(seed=9, count=4, min_cells=600, max_cells=4000)
    md = 800
    refs, total = [], 0
    for p in ps:
        og = oracle_mod.graph_for(p)
        worst, n = _escapes(og, p.omega, md)
        assert worst <= ESC_MAX
        total += n
        refs.append(og.source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, 10))
    assert total > 0
    old = os.environ.get(KEY)
    os.environ[KEY] = str(md)
    try:
        gs = [J.build_graph(p.mesh, p.omega, p.weight) for p in ps]
        try:
            assert all(J.program_info(g)["packed"] for g in gs)
            pr = [{"sigma_t": dev(p.sigma_t), "sigma_s": dev(p.sigma_s), "q": dev(p.q),
                   "phi": dev(np.zeros(p.n_cells)), "psi": dev(np.zeros((p.n_dirs, p.n_cells)))} for p in ps]
            J.solve_batch(gs, pr, mode=J.JSWEEP_FP64, tol=0.0, max_iter=10,
                          params=J.Params(strategy=J.JSWEEP_STRATEGY_DATA_DRIVEN), allow_not_converged=True)
            for i, (p, (psi_ref, phi_ref, _)) in enumerate(zip(ps, refs)):
                e1, e2 = rel_max(host(pr[i]["phi"]), phi_ref), rel_max(host(pr[i]["psi"]), psi_ref)
                print(f"[packed union] instance {i} ({p.n_cells} cells, {p.n_dirs} dirs): phi {e1:.2e} psi {e2:.2e}",
                      flush=True)
                assert e1 <= 1e-12 and e2 <= 1e-12
            pr = [{"sigma_t": dev(p.sigma_t), "sigma_s": dev(p.sigma_s), "q": dev(p.q),
                   "phi": dev(np.zeros(p.n_cells))} for p in ps]
            st = J.solve_batch(gs, pr, mode=J.JSWEEP_FP32_REFINED, tol=1e-10, max_iter=2000,
                               params=J.Params(strategy=J.JSWEEP_STRATEGY_DATA_DRIVEN))
            assert all(x["residual"] <= 1e-10 for x in st)
            torch.cuda.synchronize()
        finally:
            for g in gs:
                g.close()
    finally:
        if old is None:
            os.environ.pop(KEY, None)
        else:
            os.environ[KEY] = old
