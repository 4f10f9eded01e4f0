"""Pins for the oracle's residual and its norm (appendix algorithm "Source
iterative Sn solver", step 2.3: the error reduction that stops the
iteration).

The residual of the discrete transport equation is
    r_{K,m} = q_K + sigma_s,K phi_K - (L_m psi_m - b_m)_K / V_K
with L_m the full (un-lagged) step-scheme operator of direction m and b_m
the boundary inflow, and the stopping quantity is
    rho = sqrt(sum_K V_K sum_m w_m r_{K,m}^2) / sqrt(sum_K V_K q_K^2).

Two independent checks, both sensitive to the volume weight, the direction
weights and the scaling by ||q||:
* the dense operator, assembled in numpy from the mesh geometry, applied to
  a random angular flux that is not a solution (boundary inflow on, meshes
  with lagged edges included: the residual must use every edge);
* the sweep identity: after one source-iteration sweep from zero on a
  lag-free mesh the balance of every (cell, direction) holds exactly with
  source q, so r_{K,m} = sigma_s,K phi_K for every direction m and
  rho = ||sigma_s phi|| / ||q|| with the plain volume-weighted cell norm
  (the direction weights sum to one)."""
import numpy as np
import pytest

import workloads as W
from tests.brute import dense_direction_operator


def _cases():
    return [
        ("tri", W.delaunay_2d(7, 8, 0.3, 31), 6),
        ("tet", W.kuhn_tets(3, 0.15, 32), 8),
        ("hex", W.hex_lattice(3, 0.15, 33), 8),
        ("hex_cyclic", W.hex_lattice(3, 0.3, 1), 8),
    ]


def _dense_residual(S, fcell, cface, vol, st, ss, q, om, w, dim, psi, phi, psi_b):
    nd, n = psi.shape
    r = np.zeros((nd, n))
    for m in range(nd):
        L, bnd, lag_terms = dense_direction_operator(S, fcell, cface, vol, st, om[m], dim)
        assert not lag_terms            # no lag set given: the full operator
        r[m] = q + ss * phi - (L @ psi[m] - bnd * psi_b) / vol
    num = np.sqrt(np.sum(vol * (w @ (r * r))))
    den = np.sqrt(np.sum(vol * q * q))
    return r, num / den


@pytest.mark.parametrize("name,mesh,sn", _cases())
@pytest.mark.parametrize("psi_b", [0.0, 0.45])
def test_residual_matches_dense_operator(oracle_mod, name, mesh, sn, psi_b):
    om, w = W.quadrature(sn, mesh.dim)
    g = oracle_mod.Graph(mesh, om)
    S, fcell, cface, vol = g.geometry()
    rng = np.random.default_rng(41)
    n = g.n_cells
    st = rng.uniform(0.3, 2.5, n)
    ss = rng.uniform(0.1, 0.9, n) * st
    q = rng.uniform(0.2, 1.8, n)
    psi = rng.uniform(0.0, 2.0, (g.n_dirs, n))      # not a solution
    phi = rng.uniform(0.0, 2.0, n)                   # independent of psi: the sigma_s phi term on its own
    rho, r = g.residual(st, ss, q, w, psi, phi, psi_b=psi_b, want_r=True)
    r_ref, rho_ref = _dense_residual(S, fcell, cface, vol, st, ss, q, om, w, mesh.dim, psi, phi, psi_b)
    scale = np.abs(r_ref).max()
    assert np.abs(r - r_ref).max() <= 1e-13 * scale
    assert abs(rho - rho_ref) <= 1e-13 * rho_ref
    assert rho > 1e-2                                # a genuinely non-zero residual
    if name == "hex_cyclic":
        assert g.n_lagged > 0


@pytest.mark.parametrize("name,mesh,sn", _cases()[:3])
def test_residual_norm_weights(oracle_mod, name, mesh, sn):
    """A wrong weighting changes rho: the dense reference with the volumes,
    the direction weights or the ||q|| scale left out differs from the
    oracle's value (so the match above is not a coincidence of uniform
    data)."""
    om, w = W.quadrature(sn, mesh.dim)
    g = oracle_mod.Graph(mesh, om)
    S, fcell, cface, vol = g.geometry()
    rng = np.random.default_rng(43)
    n = g.n_cells
    st = rng.uniform(0.3, 2.5, n)
    ss = 0.5 * st
    q = rng.uniform(0.2, 1.8, n)
    psi = rng.uniform(0.0, 2.0, (g.n_dirs, n))
    phi = psi.T @ w
    rho = g.residual(st, ss, q, w, psi, phi)
    r, rho_ref = _dense_residual(S, fcell, cface, vol, st, ss, q, om, w, mesh.dim, psi, phi, 0.0)
    assert abs(rho - rho_ref) <= 1e-13 * rho_ref
    no_vol = np.sqrt(np.sum(w @ (r * r))) / np.sqrt(np.sum(q * q))
    uniform_w = np.sqrt(np.sum(vol * np.mean(r * r, axis=0))) / np.sqrt(np.sum(vol * q * q))
    unscaled = np.sqrt(np.sum(vol * (w @ (r * r))))
    for wrong in (no_vol, unscaled):
        assert abs(wrong - rho) > 1e-6 * rho
    if np.ptp(w) > 0:
        assert abs(uniform_w - rho) > 1e-6 * rho


@pytest.mark.parametrize("name,mesh,sn", _cases()[:3])
@pytest.mark.parametrize("psi_b", [0.0, 0.3])
def test_residual_after_first_sweep_is_scattering(oracle_mod, name, mesh, sn, psi_b):
    om, w = W.quadrature(sn, mesh.dim)
    g = oracle_mod.Graph(mesh, om)
    assert g.n_lagged == 0
    _, _, _, vol = g.geometry()
    rng = np.random.default_rng(47)
    n = g.n_cells
    st = rng.uniform(0.3, 2.5, n)
    ss = rng.uniform(0.1, 0.95, n) * st
    q = rng.uniform(0.2, 1.8, n)
    psi = g.sweep(st, q, psi_b=psi_b)                # first iteration: source q
    phi = g.phi(w, psi)
    rho, r = g.residual(st, ss, q, w, psi, phi, psi_b=psi_b, want_r=True)
    expect = np.broadcast_to(ss * phi, r.shape)
    assert np.abs(r - expect).max() <= 1e-12 * np.abs(expect).max()
    rho_ref = np.sqrt(np.sum(vol * (ss * phi) ** 2)) / np.sqrt(np.sum(vol * q * q))
    assert abs(rho - rho_ref) <= 1e-12 * rho_ref
