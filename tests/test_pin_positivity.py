"""Positivity of the step scheme, the property the FP64 work-list sweep uses
when it tags each flux by its sign bit instead of writing empty markers.

Each cell's balance is psi_K = (V_K s_K + sum_in a_f psi_up) / (sigma_t,K V_K
+ sum_out a_f) with a_f = |Omega . S_f| > 0.  With sigma_t > 0 and sigma_s,
q and the boundary inflow >= 0 every term is >= 0, so every flux of every
source iteration is >= 0, and its zeros are +0.0 (sign bit clear): checked
on the oracle for triangles, tetrahedra, hexahedra and a lattice whose
cycles lag edges, with exact zeros among the inputs.  A -0.0 source,
scattering cross section and inflow, on the other hand, make every flux
-0.0, which is why the sweep treats -0.0 inputs as negative."""
import numpy as np
import pytest

import workloads as W


def _cases():
    return [
        ("tri", W.delaunay_2d(7, 8, 0.3, 51), 6),
        ("tet", W.kuhn_tets(3, 0.15, 52), 8),
        ("hex", W.hex_lattice(3, 0.15, 53), 8),
        ("hex_cyclic", W.hex_lattice(3, 0.3, 1), 8),
    ]


@pytest.mark.parametrize("name,mesh,sn", _cases())
@pytest.mark.parametrize("psi_b", [0.0, 0.45])
def test_nonnegative_inputs_give_sign_clear_fluxes(oracle_mod, name, mesh, sn, psi_b):
    om, w = W.quadrature(sn, mesh.dim)
    g = oracle_mod.Graph(mesh, om)
    n = g.n_cells
    rng = np.random.default_rng(61)
    st = rng.uniform(0.3, 2.5, n)
    ss = rng.uniform(0.0, 0.95, n) * st
    ss[rng.random(n) < 0.25] = 0.0
    q = rng.uniform(0.0, 2.0, n)
    q[rng.random(n) < 0.35] = 0.0
    psi, phi, _ = g.source_iteration(st, ss, q, w, 4, psi_b=psi_b)
    assert (psi >= 0.0).all() and not np.signbit(psi).any(), name
    assert not np.signbit(phi).any(), name
    if name == "hex_cyclic":
        assert g.n_lagged > 0
    # no source and no inflow: every flux is exactly +0.0
    psi0, phi0, _ = g.source_iteration(st, ss, np.zeros(n), w, 3, psi_b=0.0)
    assert (psi0 == 0.0).all() and not np.signbit(psi0).any() and not np.signbit(phi0).any()


@pytest.mark.parametrize("name,mesh,sn", _cases()[:3])
def test_negative_zero_inputs_give_negative_zero_fluxes(oracle_mod, name, mesh, sn):
    om, w = W.quadrature(sn, mesh.dim)
    g = oracle_mod.Graph(mesh, om)
    n = g.n_cells
    st = np.random.default_rng(62).uniform(0.3, 2.5, n)
    psi, _, _ = g.source_iteration(st, np.full(n, -0.0), np.full(n, -0.0), w, 3, psi_b=-0.0)
    assert (psi == 0.0).all() and np.signbit(psi).all(), name
    # a +0.0 inflow alone clears the sign of every flux fed by a boundary
    psi_p, _, _ = g.source_iteration(st, np.full(n, -0.0), np.full(n, -0.0), w, 3, psi_b=0.0)
    assert (psi_p == 0.0).all() and not np.signbit(psi_p).all(), name


@pytest.mark.parametrize("name,mesh,sn", [_cases()[1], _cases()[3]])
def test_multigroup_nonnegative_inputs_give_sign_clear_fluxes(oracle_mod, name, mesh, sn):
    """The multigroup iteration: a group's source sums the non-negative
    scattering from every group, so its fluxes stay sign-clear too."""
    om, w = W.quadrature(sn, mesh.dim)
    g = oracle_mod.Graph(mesh, om)
    n, G = g.n_cells, 3
    rng = np.random.default_rng(63)
    st = rng.uniform(0.3, 2.5, (G, n))
    ss = rng.uniform(0.0, 0.3, (G, G, n)) * st[None, :, :]
    ss[rng.random((G, G, n)) < 0.3] = 0.0
    q = rng.uniform(0.0, 1.0, (G, n))
    q[1] = 0.0                      # a group fed by scattering only
    psi, phi, _ = g.mg_source_iteration(st, ss, q, w, 4, psi_b=0.2)
    assert (psi >= 0.0).all() and not np.signbit(psi).any(), name
    assert not np.signbit(phi).any() and (phi[1] > 0.0).any(), name
