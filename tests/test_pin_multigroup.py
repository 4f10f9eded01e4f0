"""Pins for the oracle's multigroup source iteration (appendix form of the
transport equation with a flux per ordinate and energy group; appendix
algorithm "Source iterative Sn solver": step 2.1 updates the scattering
source and the coupling terms, step 2.2 sweeps every angle and energy,
step 2.3 reduces the error).

* dense linear solve of the whole multigroup system (un-lagged streaming,
  group-to-group isotropic scattering with up- and downscatter), on
  triangle, tetrahedron and hexahedron meshes, one of them with lagged
  edges: the converged source iteration matches it;
* one group reduces to the single-group source iteration, bit for bit;
* groups without coupling reduce to independent single-group iterations
  with each group's own cross sections and source, bit for bit;
* the multigroup residual and its norm match the dense operator applied to
  a random non-solution."""
import numpy as np
import pytest

import workloads as W
from tests.brute import dense_direction_operator, dense_mg_solution


def _mg(mesh, sn, groups, seed, c=0.8):
    om, w = W.quadrature(sn, mesh.dim)
    rng = np.random.default_rng(seed)
    n = mesh.n_cells
    st = rng.uniform(0.5, 2.0, n)
    base = W.Problem("pin", mesh, om, w, st, c * st, rng.uniform(0.2, 1.5, n))
    return W.multigroup(base, groups, seed + 1)


def _cases():
    return [
        ("tri", W.delaunay_2d(6, 7, 0.3, 51), 4, 3),
        ("tet", W.kuhn_tets(2, 0.15, 52), 4, 3),
        ("hex", W.hex_lattice(3, 0.15, 53), 4, 3),
        ("hex_cyclic", W.hex_lattice(3, 0.3, 1), 8, 2),
    ]


@pytest.mark.parametrize("name,mesh,sn,groups", _cases())
def test_mg_fixed_point_dense(oracle_mod, name, mesh, sn, groups):
    p = _mg(mesh, sn, groups, 61)
    g = oracle_mod.Graph(mesh, p.omega)
    S, fcell, cface, vol = g.geometry()
    psi, phi, hist = g.mg_source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, 3000, 1e-14)
    assert hist[-1] <= 1e-14
    ref = dense_mg_solution(S, fcell, cface, vol, p.sigma_t, p.sigma_s, p.q, p.omega, p.weight, mesh.dim)
    phi_ref = np.einsum("gmk,m->gk", ref, p.weight)
    assert np.abs(phi - phi_ref).max() <= 1e-12 * np.abs(phi_ref).max()
    assert np.abs(psi - ref).max() <= 1e-12 * np.abs(ref).max()
    assert g.mg_residual(p.sigma_t, p.sigma_s, p.q, p.weight, ref, phi_ref) < 1e-13
    if name == "hex_cyclic":
        assert g.n_lagged > 0


@pytest.mark.parametrize("name,mesh,sn,groups", _cases()[:3])
def test_mg_one_group_is_single_group(oracle_mod, name, mesh, sn, groups):
    p = _mg(mesh, sn, 1, 71)
    g = oracle_mod.Graph(mesh, p.omega)
    psi, phi, hist = g.mg_source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, 12, psi_b=0.3)
    psi1, phi1, hist1 = g.source_iteration(p.sigma_t[0], p.sigma_s[0, 0], p.q[0], p.weight, 12, psi_b=0.3)
    assert np.array_equal(psi[0], psi1) and np.array_equal(phi[0], phi1)
    assert np.allclose(hist, hist1, rtol=1e-12, atol=0)


@pytest.mark.parametrize("name,mesh,sn,groups", _cases())
def test_mg_decoupled_groups(oracle_mod, name, mesh, sn, groups):
    p = _mg(mesh, sn, groups, 81)
    ss = np.zeros_like(p.sigma_s)
    for k in range(groups):
        ss[k, k] = p.sigma_s[k, k]
    g = oracle_mod.Graph(mesh, p.omega)
    psi, phi, _ = g.mg_source_iteration(p.sigma_t, ss, p.q, p.weight, 10)
    for k in range(groups):
        psi1, phi1, _ = g.source_iteration(p.sigma_t[k], ss[k, k], p.q[k], p.weight, 10)
        assert np.array_equal(psi[k], psi1) and np.array_equal(phi[k], phi1), k


@pytest.mark.parametrize("name,mesh,sn,groups", _cases())
def test_mg_residual_dense(oracle_mod, name, mesh, sn, groups):
    p = _mg(mesh, sn, groups, 91)
    g = oracle_mod.Graph(mesh, p.omega)
    S, fcell, cface, vol = g.geometry()
    rng = np.random.default_rng(92)
    G, nd, n = groups, g.n_dirs, g.n_cells
    psi = rng.uniform(0.0, 2.0, (G, nd, n))
    phi = rng.uniform(0.0, 2.0, (G, n))
    psi_b = 0.25
    rho = g.mg_residual(p.sigma_t, p.sigma_s, p.q, p.weight, psi, phi, psi_b=psi_b)
    rr = 0.0
    for k in range(G):
        src = p.q[k] + np.einsum("gk,gk->k", p.sigma_s[:, k, :], phi)
        for m in range(nd):
            L, bnd, _ = dense_direction_operator(S, fcell, cface, vol, p.sigma_t[k], p.omega[m], mesh.dim)
            r = src - (L @ psi[k, m] - bnd * psi_b) / vol
            rr += p.weight[m] * np.sum(vol * r * r)
    rho_ref = np.sqrt(rr) / np.sqrt(np.sum(vol * p.q * p.q))
    assert abs(rho - rho_ref) <= 1e-13 * rho_ref
    assert rho > 1e-2
