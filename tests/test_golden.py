"""Oracle against the stored fixtures in tests/golden (see make_golden.py)."""
import os

import numpy as np

import workloads as W

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_closed_form_fixture(oracle_mod):
    data = np.loadtxt(os.path.join(HERE, "closed_form_hex4.txt"))
    om, _ = W.quadrature(8, 3)
    g = oracle_mod.Graph(W.hex_lattice(4), om)
    psi = g.sweep(np.full(64, 1.3), np.full(64, 2.5))
    for row in data:
        m = int(row[0])
        assert np.allclose(row[1:4], om[m], rtol=0, atol=1e-15)
        assert np.abs(psi[m] - row[4:]).max() <= 1e-14 * row[4:].max()


def test_oracle_regression_fixture(oracle_mod):
    ref = np.loadtxt(os.path.join(HERE, "oracle_delaunay_phi20.txt"))
    p = W.config(1)
    g = oracle_mod.graph_for(p)
    _, phi, _ = g.source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, 20)
    assert np.array_equal(phi, ref)
