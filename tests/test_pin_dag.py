"""Pins for the oracle's dependency graph, lag rule and levels.

* undeformed hex lattice: level = i' + j' + k' and in-degree
  [i'>0] + [j'>0] + [k'>0] with indices counted from each direction's
  inflow corner (closed form of the longest path on a Cartesian grid);
* tiny meshes: edges from the face signs, strongly connected components by
  exhaustive reachability, the lag rule (inside a cycle keep edges from
  lower to higher cell id), longest-path levels by depth-first search and
  in-degrees, all compared with the oracle;
* Delaunay triangulations are acyclic in every direction (no lagged edge);
* the level-ordered cell list is sorted by (level, id) and its pointer array
  matches the level histogram;
* with lagging refused, a cyclic mesh is reported as an error."""
import numpy as np
import pytest

import workloads as W
from tests.brute import edges_for_direction, lag_rule_bruteforce, longest_path_levels


def test_cartesian_levels_closed_form(oracle_mod):
    n = 5
    om, _ = W.quadrature(8, 3)
    g = oracle_mod.Graph(W.hex_lattice(n), om)
    assert g.n_lagged == 0
    idx = np.arange(n)
    I, J, K = (a.ravel() for a in np.meshgrid(idx, idx, idx, indexing="ij"))
    for m in range(g.n_dirs):
        o = om[m]
        ip = I if o[0] > 0 else n - 1 - I
        jp = J if o[1] > 0 else n - 1 - J
        kp = K if o[2] > 0 else n - 1 - K
        indeg, level, lvl_ptr, lvl_cells = g.direction(m)
        assert (level == ip + jp + kp).all()
        assert (indeg == (ip > 0).astype(int) + (jp > 0) + (kp > 0)).all()
        assert len(lvl_ptr) == 3 * (n - 1) + 2


def _tiny():
    return [
        ("tri", W.delaunay_2d(6, 7, 0.3, 2), 4),
        ("tet", W.kuhn_tets(2, 0.15, 3), 8),
        ("hex_cyclic8", W.hex_lattice(3, 0.3, 1), 8),
        ("hex_cyclic16", W.hex_lattice(3, 0.3, 0), 16),
        ("hex4_cyclic", W.hex_lattice(4, 0.35, 23), 8),
    ]


@pytest.mark.parametrize("name,mesh,sn", _tiny())
def test_dag_bruteforce(oracle_mod, name, mesh, sn):
    om, _ = W.quadrature(sn, mesh.dim)
    g = oracle_mod.Graph(mesh, om)
    S, fcell, cface, vol = g.geometry()
    n = g.n_cells
    lm, lu, lv, lf = g.lagged()
    got_lag = {}
    for a, b, c in zip(lm, lu, lv):
        got_lag.setdefault(int(a), set()).add((int(b), int(c)))
    total = 0
    for m in range(g.n_dirs):
        edges = edges_for_direction(S, fcell, om[m], mesh.dim)
        lag = lag_rule_bruteforce(n, edges)
        total += len(lag)
        assert lag == got_lag.get(m, set()), m
        kept = [e for e in edges if e not in lag]
        lev = longest_path_levels(n, kept)
        indeg = np.zeros(n, dtype=int)
        for _, v in kept:
            indeg[v] += 1
        oi, ol, optr, ocells = g.direction(m)
        assert (ol == lev).all() and (oi == indeg).all()
        order = sorted(range(n), key=lambda c: (lev[c], c))
        assert (ocells == np.array(order)).all()
        hist = np.bincount(lev, minlength=lev.max() + 1)
        assert (np.diff(optr) == hist).all() and optr[0] == 0
    assert total == g.n_lagged
    if name.startswith("hex") and "cyclic" in name:
        assert g.n_lagged > 0


def test_delaunay_is_acyclic(oracle_mod):
    p = W.config(1)
    g = oracle_mod.graph_for(p)
    assert g.n_lagged == 0


def test_refuse_cycles(oracle_mod):
    om, _ = W.quadrature(8, 3)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.Graph(W.hex_lattice(3, 0.3, 1), om, refuse_cycles=True)
    oracle_mod.Graph(W.kuhn_tets(2, 0.15, 3), om, refuse_cycles=True)
