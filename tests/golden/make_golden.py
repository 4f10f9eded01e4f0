"""Writes the stored expected values under tests/golden/.

* ``closed_form_hex4.txt``: pure-absorber angular flux on an undeformed 4^3
  hexahedral lattice (sigma_t = 1.3, q = 2.5, vacuum) for three S8
  directions, from the closed form of the step recursion (lattice-path sum
  evaluated in mpmath with 50 digits).  The paper prints no worked numerical
  example (its worked examples live in figures that are not part of its
  text), so closed forms stand in.
* ``oracle_delaunay_phi20.txt``: scalar flux of the 2D Delaunay workload
  (2,000 jittered points, S4, 20 source iterations) computed by the oracle;
  a regression fixture for the oracle itself.

Run from the repository root:  python tests/golden/make_golden.py
Only workloads/, oracle/ and tests/brute.py are used."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402
from tests.brute import closed_form_absorber  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    om, _ = W.quadrature(8, 3)
    rows = []
    for m in (0, 41, 79):
        psi = closed_form_absorber(4, 0.25, 1.3, 2.5, om[m]).ravel()
        rows.append(np.concatenate([[m], om[m], psi]))
    np.savetxt(os.path.join(HERE, "closed_form_hex4.txt"), np.array(rows), fmt="%.17g",
               header="m omega_x omega_y omega_z psi[cell 0..63] (lattice cube order); sigma_t=1.3 q=2.5 h=0.25")
    p = W.config(1)
    g = oracle.graph_for(p)
    _, phi, hist = g.source_iteration(p.sigma_t, p.sigma_s, p.q, p.weight, 20)
    np.savetxt(os.path.join(HERE, "oracle_delaunay_phi20.txt"), phi, fmt="%.17g",
               header=f"oracle phi after 20 source iterations, {p.name}, rho={hist[-1]:.6e}")


if __name__ == "__main__":
    main()
