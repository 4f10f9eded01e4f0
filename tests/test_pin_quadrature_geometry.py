"""Pins for the inputs (quadrature) and for the oracle's geometry step.

Quadrature: the direction counts of LQ_N, unit directions, weights summing
to one, octant and axis-permutation symmetry, and exact integration of the
even angular moments (S4-S8 exact; S16 to the least-squares level).

Geometry (oracle): per-cell closure sum_f S_f^out = 0, total volume of the
unit square / cube, exact values on an undeformed lattice, face counts from
the mesh topology, face orientation (lower cell -> higher cell, outward on
the boundary) checked against vertex centroids, and triangle / tetrahedron
measures recomputed with determinants."""
import itertools

import numpy as np
import pytest

import workloads as W
from tests.brute import cell_face_terms


@pytest.mark.parametrize("N,n3", [(2, 8), (4, 24), (6, 48), (8, 80), (16, 288)])
def test_quadrature_counts_norms_weights(N, n3):
    om, w = W.quadrature(N, 3)
    assert om.shape == (n3, 3)
    assert np.abs(np.linalg.norm(om, axis=1) - 1.0).max() < 1e-15
    assert abs(w.sum() - 1.0) < 1e-14 and (w > 0).all()
    om2, w2 = W.quadrature(N, 2)
    assert om2.shape == (n3 // 2, 3) and (om2[:, 2] > 0).all()
    assert abs(w2.sum() - 1.0) < 1e-14


@pytest.mark.parametrize("N", [4, 6, 8, 16])
def test_quadrature_symmetry(N):
    om, w = W.quadrature(N, 3)
    key = {tuple(np.round(v, 14)): wt for v, wt in zip(om, w)}
    for signs in itertools.product([1, -1], repeat=3):
        for perm in itertools.permutations(range(3)):
            for v, wt in zip(om, w):
                t = tuple(np.round(np.array(signs) * v[list(perm)], 14))
                assert t in key and abs(key[t] - wt) < 1e-15


@pytest.mark.parametrize("N,tol", [(4, 1e-13), (6, 1e-13), (8, 1e-13), (16, 1e-8)])
def test_quadrature_even_moments(N, tol):
    om, w = W.quadrature(N, 3)
    for a in range(0, N + 1):
        for b in range(0, N + 1 - a):
            for c in range(0, N + 1 - a - b):
                got = float(np.sum(w * om[:, 0] ** a * om[:, 1] ** b * om[:, 2] ** c))
                assert abs(got - W.sphere_moment(a, b, c)) < tol, (a, b, c)


def _meshes():
    return [
        ("tri", W.delaunay_2d(9, 11, 0.3, 7)),
        ("tet", W.kuhn_tets(3, 0.15, 8)),
        ("hex", W.hex_lattice(3, 0.15, 9)),
        ("hex_cyclic", W.hex_lattice(3, 0.3, 1)),
    ]


@pytest.mark.parametrize("name,mesh", _meshes())
def test_geometry_closure_and_total_volume(oracle_mod, name, mesh):
    om, _ = W.quadrature(4, mesh.dim)
    g = oracle_mod.Graph(mesh, om)
    S, fcell, cface, vol = g.geometry()
    scale = np.abs(S).sum(axis=1).max()
    for K in range(g.n_cells):
        tot = np.zeros(3)
        for j in range(g.faces_per_cell):
            s, _ = cell_face_terms(S, fcell, cface, K, j)
            tot += s
        assert np.abs(tot).max() <= 1e-14 * scale
    assert abs(vol.sum() - 1.0) < 1e-13
    assert (vol > 0).all()


def test_face_counts(oracle_mod):
    n = 3
    om, _ = W.quadrature(4, 3)
    g = oracle_mod.Graph(W.kuhn_tets(n, 0.1, 1), om)
    assert g.n_faces == 12 * n ** 3 + 6 * n ** 2
    g = oracle_mod.Graph(W.hex_lattice(n, 0.1, 1), om)
    assert g.n_faces == 3 * n ** 3 + 3 * n ** 2
    m = W.delaunay_2d(7, 8, 0.3, 3)
    g = oracle_mod.Graph(m, W.quadrature(4, 2)[0])
    assert g.n_faces == m.n_vertices + m.n_cells - 1          # Euler, triangulated disk


@pytest.mark.parametrize("name,mesh", _meshes())
def test_face_orientation(oracle_mod, name, mesh):
    om, _ = W.quadrature(4, mesh.dim)
    g = oracle_mod.Graph(mesh, om)
    S, fcell, cface, vol = g.geometry()
    cen = mesh.coords[mesh.cells].mean(axis=1)
    d = mesh.dim
    for f in range(g.n_faces):
        K, L = fcell[f]
        assert L == -1 or K < L
        if L >= 0:
            assert np.dot(S[f, :d], cen[L] - cen[K]) > 0
        else:
            j = int(np.nonzero(cface[K] == f)[0][0])
            others = [v for v in mesh.cells[K] if v not in set(_face_vertices(mesh, K, j))]
            assert np.dot(S[f, :d], mesh.coords[_face_vertices(mesh, K, j)].mean(axis=0) -
                          mesh.coords[others].mean(axis=0)) > 0


def _face_vertices(mesh, K, j):
    c = mesh.cells[K]
    if mesh.cell_type == W.TRI:
        return [c[(j + 1) % 3], c[(j + 2) % 3]]
    if mesh.cell_type == W.TET:
        return [c[i] for i in range(4) if i != j]
    hexf = [[0, 1, 3, 2], [4, 5, 7, 6], [0, 1, 5, 4], [2, 3, 7, 6], [0, 2, 6, 4], [1, 3, 7, 5]]
    return [c[i] for i in hexf[j]]


def test_measures_by_determinant(oracle_mod):
    m = W.delaunay_2d(9, 11, 0.3, 7)
    g = oracle_mod.Graph(m, W.quadrature(4, 2)[0])
    _, _, _, vol = g.geometry()
    x = m.coords[m.cells]
    ref = 0.5 * np.abs(np.linalg.det(np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0]], axis=1)))
    assert np.abs(vol - ref).max() <= 1e-14 * ref.max()
    m = W.kuhn_tets(3, 0.15, 8)
    g = oracle_mod.Graph(m, W.quadrature(4, 3)[0])
    _, _, _, vol = g.geometry()
    x = m.coords[m.cells]
    ref = np.abs(np.linalg.det(np.stack([x[:, 1] - x[:, 0], x[:, 2] - x[:, 0], x[:, 3] - x[:, 0]], axis=1))) / 6
    assert np.abs(vol - ref).max() <= 1e-14 * ref.max()


def test_undeformed_lattice_exact(oracle_mod):
    n = 4
    h = 1.0 / n
    om, _ = W.quadrature(4, 3)
    g = oracle_mod.Graph(W.hex_lattice(n), om)
    S, fcell, cface, vol = g.geometry()
    assert (vol == h ** 3).all()
    for f in range(g.n_faces):
        nz = np.nonzero(S[f])[0]
        assert len(nz) == 1 and abs(S[f, nz[0]]) == h * h
    g = oracle_mod.Graph(W.kuhn_tets(n), om)
    _, _, _, vol = g.geometry()
    assert (vol == h ** 3 / 6).all()
