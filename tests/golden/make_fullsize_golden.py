"""Writes the sampled oracle values the full-size GPU parity tests and the
benchmark's error report compare against.  Calls only ``oracle/`` (and the
seeded input generators of ``workloads/``); nothing here comes from the HIP
path.

The full-size workloads are too large to compare whole in a GPU test: the
oracle needs minutes per configuration.  Directions of one sweep are
independent (paper Sec. V-B), so this script runs the oracle's own
per-direction sweep on disjoint direction ranges in parallel threads (the
oracle releases the interpreter lock inside its C code); the scalar flux is
still the oracle's ascending-direction sum and the residual the oracle's
explicit un-lagged operator (appendix algorithm "Source iterative Sn
solver", steps 2.1-2.3).  The iterate sequence is exactly the serial
oracle's.

For each workload it stores, at a seeded sample of cells (plus the cell of
the largest flux), the scalar flux after a fixed number of source
iterations from zero and, where asked, at convergence (rho <= 1e-13), and
at a seeded sample of (direction, cell) pairs the angular flux after the
fixed iterations.

Usage: python tests/golden/make_fullsize_golden.py [hex64_s8] [tetcheck96_s8] [tetlogn60_s16]
       (default: all three; files tests/golden/fullsize_<name>.txt)"""
from __future__ import annotations

import os
import sys
import threading
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

N_CELL_SAMPLES = 2048
N_PSI_SAMPLES = 1024
TOL_CONVERGED = 1e-13

# workload -> (config number, fixed iteration count, converge?); "ens<i>"
# is instance i of the 256-instance ensemble (seed 4, 500 - 50,000 cells):
# its smallest and largest triangle and tetrahedron meshes
PLAN = {
    "hex64_s8": (2, 20, True),
    "tetcheck96_s8": (3, 2, True),
    "tetlogn60_s16": (5, 2, True),
    "ens49": (None, 20, True),
    "ens86": (None, 20, True),
    "ens95": (None, 20, True),
    "ens216": (None, 20, True),
}

_ENSEMBLE = None


def problem(name):
    global _ENSEMBLE
    k = PLAN[name][0]
    if k is not None:
        return W.config(k)
    if _ENSEMBLE is None:
        _ENSEMBLE = W.ensemble(seed=4, count=256, min_cells=500, max_cells=50000)
    return _ENSEMBLE[int(name[3:])]


def log(msg):
    print(f"[golden] {msg}", flush=True)


def threaded_sweep(g, sigma_t, src, psi_prev, psi, threads):
    nd = g.n_dirs
    bounds = np.linspace(0, nd, threads + 1).astype(int)
    ths = [threading.Thread(target=g.sweep_dirs, args=(int(a), int(b), sigma_t, src),
                            kwargs={"psi_prev": psi_prev, "psi": psi})
           for a, b in zip(bounds[:-1], bounds[1:]) if b > a]
    for t in ths:
        t.start()
    for t in ths:
        t.join()


def samples(p, seed=12345):
    rng = np.random.default_rng(seed)
    cells = np.sort(rng.choice(p.n_cells, size=min(N_CELL_SAMPLES, p.n_cells), replace=False))
    pm = rng.integers(0, p.n_dirs, size=N_PSI_SAMPLES)
    pk = rng.integers(0, p.n_cells, size=N_PSI_SAMPLES)
    return cells, pm, pk


def run(name, threads):
    _, n_fixed, converge = PLAN[name]
    p = problem(name)
    t0 = time.time()
    g = oracle.graph_for(p)
    log(f"{name}: oracle graph built in {time.time() - t0:.0f} s ({g.n_lagged} lagged edges)")
    cells, pm, pk = samples(p)
    nd, nc = p.n_dirs, p.n_cells
    psi = np.zeros((nd, nc))
    phi = np.zeros(nc)
    prev = np.zeros((nd, nc)) if g.n_lagged else None
    fixed_phi = fixed_psi = None
    conv_phi, conv_it, conv_rho = None, None, None
    it = 0
    max_it = 5000 if converge else n_fixed
    rho = 1.0
    while it < max_it:
        src = p.q + p.sigma_s * phi
        if prev is not None:
            prev[...] = psi
        threaded_sweep(g, p.sigma_t, src, prev, psi, threads)
        phi = g.phi(p.weight, psi)
        it += 1
        if it == n_fixed:
            fixed_phi = phi[cells].copy()
            fixed_psi = psi[pm, pk].copy()
            big = int(np.argmax(phi))
            fixed_big = (big, float(phi[big]))
            log(f"{name}: {n_fixed} iterations stored")
            if not converge:
                break
        if it >= n_fixed and (it % 4 == 0 or rho < 1e3 * TOL_CONVERGED):
            rho = g.residual(p.sigma_t, p.sigma_s, p.q, p.weight, psi, phi)
            log(f"{name}: iteration {it} rho {rho:.3e} ({time.time() - t0:.0f} s)")
            if rho <= TOL_CONVERGED:
                conv_phi, conv_it, conv_rho = phi.copy(), it, rho
                break
    path = os.path.join(HERE, f"fullsize_{name}.txt")
    with open(path, "w") as f:
        f.write(f"# Oracle values for {name} ({nc} cells x {nd} directions), written by make_fullsize_golden.py\n")
        f.write("# (oracle/ only: per-direction sweeps of the appendix source-iteration algorithm, steps 2.1-2.3,\n")
        f.write("# ascending-direction scalar flux, explicit un-lagged residual).  Samples: numpy default_rng(12345).\n")
        f.write(f"fixed_iterations {n_fixed}\n")
        f.write(f"fixed_max_cell {fixed_big[0]} {fixed_big[1]!r}\n")
        if conv_phi is not None:
            big = int(np.argmax(conv_phi))
            f.write(f"converged_iterations {conv_it} rho {conv_rho!r} tol {TOL_CONVERGED!r}\n")
            f.write(f"converged_max_cell {big} {float(conv_phi[big])!r}\n")
            f.write(f"converged_phi_norm2 {float(np.linalg.norm(conv_phi))!r}\n")
        f.write(f"cells {len(cells)}  # cell, phi after fixed iterations" +
                (", phi at convergence" if conv_phi is not None else "") + "\n")
        for i, K in enumerate(cells):
            line = f"{K} {float(fixed_phi[i])!r}"
            if conv_phi is not None:
                line += f" {float(conv_phi[K])!r}"
            f.write(line + "\n")
        f.write(f"psi {len(pm)}  # direction, cell, psi after fixed iterations\n")
        for m, K, v in zip(pm, pk, fixed_psi):
            f.write(f"{m} {K} {float(v)!r}\n")
    log(f"{name}: wrote {path} ({time.time() - t0:.0f} s)")


def load(name):
    """Parse a fixture: dict with fixed_iterations, cells, phi_fixed,
    phi_converged (or None), psi (m, K, value arrays) and the header values."""
    path = os.path.join(HERE, f"fullsize_{name}.txt")
    out = {"phi_converged": None}
    with open(path) as f:
        lines = [ln.split("#")[0].split() for ln in f if not ln.startswith("#")]
    i = 0
    while i < len(lines):
        w = lines[i]
        if not w:
            i += 1
            continue
        if w[0] == "fixed_iterations":
            out["fixed_iterations"] = int(w[1])
        elif w[0] == "fixed_max_cell":
            out["fixed_max_cell"] = (int(w[1]), float(w[2]))
        elif w[0] == "converged_iterations":
            out["converged_iterations"], out["converged_rho"] = int(w[1]), float(w[3])
        elif w[0] == "converged_max_cell":
            out["converged_max_cell"] = (int(w[1]), float(w[2]))
        elif w[0] == "converged_phi_norm2":
            out["converged_phi_norm2"] = float(w[1])
        elif w[0] == "cells":
            n = int(w[1])
            rows = lines[i + 1:i + 1 + n]
            out["cells"] = np.array([int(r[0]) for r in rows])
            out["phi_fixed"] = np.array([float(r[1]) for r in rows])
            if len(rows[0]) > 2:
                out["phi_converged"] = np.array([float(r[2]) for r in rows])
            i += n
        elif w[0] == "psi":
            n = int(w[1])
            rows = lines[i + 1:i + 1 + n]
            out["psi_m"] = np.array([int(r[0]) for r in rows])
            out["psi_k"] = np.array([int(r[1]) for r in rows])
            out["psi"] = np.array([float(r[2]) for r in rows])
            i += n
        i += 1
    return out


if __name__ == "__main__":
    names = sys.argv[1:] or list(PLAN)
    threads = int(os.environ.get("ORACLE_THREADS", os.cpu_count() or 1))
    for n in names:
        run(n, threads)
