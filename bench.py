"""Benchmark of the data-driven transport sweep on one MI355X.

Workload: the jittered 64^3 hexahedral mesh (262,144 cells, interior
vertices moved by up to 0.15 h), level-symmetric S8 (80 directions),
sigma_t = exp(N(0, 0.5^2)) per cell, scattering ratio 0.9, q = 1 in the
central eighth, vacuum boundaries; FP64.

A step is one FP64 source iteration through the C ABI: scattering source,
data-driven sweep of all 80 directions over the per-direction dependency
graph, scalar flux and FP64 residual.  The graph is built once before the
timed region (preprocessing).  value = cell-angle updates per second over
the timed steps.

Also reported:
  roofline      the sweep kernel's algorithmic bytes per launch (each
                angular flux written once and read once per downwind
                neighbour, 8 B each) over its average launch time, from HIP
                events around every sweep launch in the timed region;
                traffic from the committed rocprofv3 counter summary when it
                was taken on the current kernel source, else null;
  cpu_baseline  the oracle (serial FP64 CPU code) timed on a bounded sample
                of the same workload on this host;
  time_to_tol   wall time of jsweep_solve to rho <= 1e-8, plain FP64 and
                FP32-refined, with the error of each result against the FP64
                GPU fixed point (and the sample sweep's error vs the oracle).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def _source_hash() -> str:
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1803_09876_amd", "csrc", "sweep.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def _traffic(kernel_key: str, launches_bytes_alg: float):
    """HBM bytes per launch from the committed counter summary, or None if
    it was measured on a different sweep kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    rec = data.get(kernel_key)
    if not rec or rec.get("source_hash") != _source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def algorithmic_bytes(J, g, n_cells, n_dirs, word):
    """(1 + n_in) * word summed over all vertices: one write per vertex and
    one read per interior upwind edge (lagged edges included)."""
    edges = 0
    for m in range(n_dirs):
        indeg, _, _, _ = J.graph_export(g, m)
        edges += int(indeg.sum())
    edges += J.graph_info(g)["n_lagged"]
    return (n_cells * n_dirs + edges) * word, edges


def cpu_baseline(problem, psi_gpu_sample):
    import oracle
    t = time.time()
    og = oracle.graph_for(problem)
    t_build = time.time() - t
    t = time.time()
    ref = og.sweep(problem.sigma_t, problem.q)
    dt = time.time() - t
    upd = problem.n_cells * problem.n_dirs
    err = None
    if psi_gpu_sample is not None:
        err = float(np.abs(psi_gpu_sample - ref).max() / np.abs(ref).max())
    return {
        "value": upd / dt,
        "unit": "cell-angle updates/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"one FP64 sweep of all {problem.n_dirs} directions of {problem.name} "
                  f"({upd} cell-angle updates) after a {t_build:.1f} s graph build, serial",
    }, err


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the sweep path of this "
              f"build is a single-device kernel).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1803_09876_amd as J
    import workloads as W

    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    J.load_library()
    p = W.config(2)
    nc, nd = p.n_cells, p.n_dirs
    t = time.time()
    g = J.build_graph(p.mesh, p.omega, p.weight)
    torch.cuda.synchronize()
    t_build = time.time() - t
    info = J.graph_info(g)
    st, ss, q = (torch.tensor(a, device="cuda") for a in (p.sigma_t, p.sigma_s, p.q))
    phi = torch.zeros(nc, dtype=torch.float64, device="cuda")
    psi = torch.zeros(nd * nc, dtype=torch.float64, device="cuda")

    # warmup, then the timed steps (K source iterations, no early stop)
    J.solve(g, st, ss, q, phi, psi, mode=J.JSWEEP_FP64, tol=0.0, max_iter=max(1, args.warmup),
            allow_not_converged=True)
    J.jsweep_profile(g, True)
    J.jsweep_profile_read(g, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J.solve(g, st, ss, q, phi, psi, mode=J.JSWEEP_FP64, tol=0.0, max_iter=args.steps, allow_not_converged=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    launches, kernel_ms = J.jsweep_profile_read(g, reset=True)
    J.jsweep_profile(g, False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = nc * nd * args.steps / (t1 - t0)

    bytes_alg, edges = algorithmic_bytes(J, g, nc, nd, 8)
    avg_kernel_s = kernel_ms / max(1, launches) * 1e-3
    achieved = bytes_alg / avg_kernel_s / 1e9
    kernel_key = "k_sweep<double,6,3> hex64_s8"
    traffic = _traffic(kernel_key, bytes_alg)

    # one sweep on fixed inputs for the comparison with the oracle
    psi_s = torch.zeros(nd * nc, dtype=torch.float64, device="cuda")
    J.sweep(g, st, q, psi_s)
    psi_sample = psi_s.view(nd, nc).cpu().numpy()

    # time to rho <= 1e-8: plain FP64 vs FP32-refined
    ttt = {}
    phi64 = torch.zeros_like(phi)
    for name, mode in (("fp64", J.JSWEEP_FP64), ("fp32_refined", J.JSWEEP_FP32_REFINED)):
        out = torch.zeros_like(phi)
        torch.cuda.synchronize()
        a = time.perf_counter()
        s = J.solve(g, st, ss, q, out, mode=mode, tol=1e-8, max_iter=5000)
        torch.cuda.synchronize()
        ttt[name] = {"seconds": time.perf_counter() - a, "sweeps": s["sweeps"], "outer": s["outer_iters"],
                     "residual": s["residual"]}
        if name == "fp64":
            phi64 = out
        else:
            ttt[name]["phi_rel_err_vs_fp64"] = float(torch.linalg.norm(out - phi64) / torch.linalg.norm(phi64))
    ttt["speedup_fp32_refined"] = ttt["fp64"]["seconds"] / ttt["fp32_refined"]["seconds"]

    cpu, err = (None, None) if args.no_cpu else cpu_baseline(p, psi_sample)

    line = {
        "metric": "cell-angle updates/s per sweep; time-to-1e-8 residual, FP32-refined vs FP64",
        "value": value,
        "unit": "cell-angle updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "hex64_s8: jittered 64^3 hexahedra (262,144 cells), S8 (80 directions), "
                               "scattering ratio 0.9, FP64 source iteration step",
                   "cells": nc, "dirs": nd, "lagged_edges": info["n_lagged"], "max_levels": info["max_levels"],
                   "graph_build_s": t_build},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "kernel": kernel_key, "algorithmic_bytes_per_launch": bytes_alg,
                     "interior_edges": edges, "avg_kernel_ms": avg_kernel_s * 1e3, "launches": launches},
        "cpu_baseline": cpu,
        "sweep_updates_per_s_kernel": nc * nd / avg_kernel_s,
        "time_to_tol": ttt,
        "sweep_rel_err_vs_oracle": err,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
