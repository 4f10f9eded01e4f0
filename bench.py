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
                FP32-refined, on this workload and on the S16 tetrahedral one
                (60^3 lattice, 6 tets per cube, 288 directions), each the
                fastest of three solves after an untimed warm-up of the mode,
                with the error of each result against the FP64 GPU fixed point
                (and the sample sweep's error vs the oracle);
  ensemble      256 independent meshes (500-50,000 cells, half triangles,
                half tets, S4-S8) solved together by jsweep_solve_batch (one
                sweep launch for every instance and direction): FP64 step
                throughput and time-to-1e-8, FP64 vs FP32-refined (each the
                fastest of three after a warm-up), with the autotuned launch
                parameters.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-s16]
                       [--no-ensemble] [--copy-probe] [--steps-only]
  --copy-probe  first copies 512 MiB device to device (the calibration
                dispatch for HBM byte counters taken on this run)
  --steps-only  only the timed steps and the roofline (for profiler runs)
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


def _traffic(kernel_key: str):
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


TTT_REPEATS = 3


def time_to_tol(J, torch, g, p, tol=1e-8):
    """jsweep_solve to rho <= tol, plain FP64 then FP32-refined, from zero;
    each the fastest of TTT_REPEATS solves after an untimed warm-up."""
    st, ss, q = (torch.tensor(a, device="cuda") for a in (p.sigma_t, p.sigma_s, p.q))
    out, ref = {}, None
    for name, mode in (("fp64", J.JSWEEP_FP64), ("fp32_refined", J.JSWEEP_FP32_REFINED)):
        # untimed warm-up of the mode's kernels (one outer iteration)
        J.solve(g, st, ss, q, torch.zeros(p.n_cells, dtype=torch.float64, device="cuda"), mode=mode, tol=0.0,
                max_iter=1, allow_not_converged=True)
        best = None
        for _ in range(TTT_REPEATS):
            phi = torch.zeros(p.n_cells, dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            a = time.perf_counter()
            s = J.solve(g, st, ss, q, phi, mode=mode, tol=tol, max_iter=20000)
            torch.cuda.synchronize()
            sec = time.perf_counter() - a
            best = sec if best is None else min(best, sec)
        out[name] = {"seconds": best, "sweeps": s["sweeps"], "outer": s["outer_iters"], "residual": s["residual"]}
        if ref is None:
            ref = phi
        else:
            out[name]["phi_rel_err_vs_fp64"] = float(torch.linalg.norm(phi - ref) / torch.linalg.norm(ref))
    out["speedup_fp32_refined"] = out["fp64"]["seconds"] / out["fp32_refined"]["seconds"]
    return out


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


def ensemble_bench(J, W, torch, steps=5):
    ps = W.ensemble(seed=4, count=256, min_cells=500, max_cells=50000)
    gs = [J.build_graph(p.mesh, p.omega, p.weight) for p in ps]
    upd = sum(p.n_cells * p.n_dirs for p in ps)
    tuned = J.autotune(gs, mode=J.JSWEEP_FP32_REFINED)

    def problems():
        return [{"sigma_t": torch.tensor(p.sigma_t, device="cuda"), "sigma_s": torch.tensor(p.sigma_s, device="cuda"),
                 "q": torch.tensor(p.q, device="cuda"), "phi": torch.zeros(p.n_cells, dtype=torch.float64, device="cuda")}
                for p in ps]

    out = {"instances": len(ps), "cells": sum(p.n_cells for p in ps), "cell_angle_updates_per_sweep": upd,
           "autotuned": tuned.as_dict()}
    pr = problems()
    J.solve_batch(gs, pr, mode=J.JSWEEP_FP64, tol=0.0, max_iter=2, params=tuned, allow_not_converged=True)
    torch.cuda.synchronize()
    a = time.perf_counter()
    J.solve_batch(gs, pr, mode=J.JSWEEP_FP64, tol=0.0, max_iter=steps, params=tuned, allow_not_converged=True)
    torch.cuda.synchronize()
    step = (time.perf_counter() - a) / steps
    out["fp64_step_ms"] = step * 1e3
    out["fp64_updates_per_s"] = upd / step
    ttt, ref = {}, None
    for name, mode in (("fp64", J.JSWEEP_FP64), ("fp32_refined", J.JSWEEP_FP32_REFINED)):
        # untimed warm-up of the mode (its first use builds the FP32 records
        # and coefficients of every instance), then the fastest of
        # TTT_REPEATS solves from zero
        J.solve_batch(gs, problems(), mode=mode, tol=0.0, max_iter=2, params=tuned, allow_not_converged=True)
        best = None
        for _ in range(TTT_REPEATS):
            pr = problems()
            torch.cuda.synchronize()
            a = time.perf_counter()
            st = J.solve_batch(gs, pr, mode=mode, tol=1e-8, max_iter=20000, params=tuned)
            torch.cuda.synchronize()
            sec = time.perf_counter() - a
            best = sec if best is None else min(best, sec)
        ttt[name] = {"seconds": best, "max_sweeps": max(x["sweeps"] for x in st),
                     "max_residual": max(x["residual"] for x in st)}
        phis = torch.cat([x["phi"] for x in pr])
        if ref is None:
            ref = phis
        else:
            ttt[name]["phi_rel_err_vs_fp64"] = float(torch.linalg.norm(phis - ref) / torch.linalg.norm(ref))
    ttt["speedup_fp32_refined"] = ttt["fp64"]["seconds"] / ttt["fp32_refined"]["seconds"]
    out["time_to_tol"] = ttt
    for g in gs:
        g.close()
    return out


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def extras(args, J, W, torch, g, p, st, ss, q, phi):
    """FP32 sweep kernel time, the oracle comparison, time-to-1e-8 and the CPU baseline."""
    nc, nd = p.n_cells, p.n_dirs
    # FP32 sweep kernel time on the same graph (correction sweeps)
    J.jsweep_profile(g, True)
    J.solve(g, st, ss, q, torch.zeros_like(phi), mode=J.JSWEEP_FP32_REFINED, tol=0.0, max_iter=1 + args.warmup,
            allow_not_converged=True)
    J.jsweep_profile_read(g, reset=True)
    J.solve(g, st, ss, q, torch.zeros_like(phi), mode=J.JSWEEP_FP32_REFINED, tol=0.0, max_iter=10,
            allow_not_converged=True)
    n32, ms32 = J.jsweep_profile_read(g, reset=True)
    J.jsweep_profile(g, False)
    avg32_s = ms32 / max(1, n32) * 1e-3
    log(f"FP32 sweep kernel {avg32_s * 1e3:.3f} ms")
    # one sweep on fixed inputs for the comparison with the oracle
    psi_s = torch.zeros(nd * nc, dtype=torch.float64, device="cuda")
    J.sweep(g, st, q, psi_s)
    psi_sample = psi_s.view(nd, nc).cpu().numpy()
    # time to rho <= 1e-8: plain FP64 vs FP32-refined
    ttt = {p.name: time_to_tol(J, torch, g, p)}
    log(f"time to 1e-8 on {p.name}: {json.dumps(ttt[p.name])}")
    if not args.no_s16:
        p5 = W.config(5)
        g5 = J.build_graph(p5.mesh, p5.omega, p5.weight)
        ttt[p5.name] = time_to_tol(J, torch, g5, p5)
        g5.close()
        log(f"time to 1e-8 on {p5.name}: {json.dumps(ttt[p5.name])}")
    ens = None
    if not args.no_ensemble:
        ens = ensemble_bench(J, W, torch)
        log(f"ensemble: {json.dumps(ens)}")
    cpu, err = (None, None) if args.no_cpu else cpu_baseline(p, psi_sample)
    return avg32_s, ttt, ens, cpu, err


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-s16", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--steps-only", action="store_true")
    ap.add_argument("--ttt-only", action="store_true",
                    help="only the time-to-1e-8 solves (FP64 and FP32-refined) on hex64_s8 and, unless --no-s16, "
                         "tetlogn60_s16; prints one JSON line")
    ap.add_argument("--ensemble-only", action="store_true",
                    help="only the 256-instance batched solve (for profiling the batch kernels)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the sweep path of this "
              f"library is a single-device kernel).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1803_09876_amd as J
    import workloads as W

    if not torch.cuda.is_available():
        print("no GPU available", file=sys.stderr)
        sys.exit(1)
    J.load_library()
    if args.copy_probe:
        x = torch.ones(64 << 20, dtype=torch.float64, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    if args.ensemble_only:
        ens = ensemble_bench(J, W, torch, steps=max(1, args.steps))
        print(json.dumps({"ensemble": ens}))
        return
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
    log(f"{p.name}: graph built in {t_build:.2f} s")
    if args.ttt_only:
        ttt = {p.name: time_to_tol(J, torch, g, p)}
        if not args.no_s16:
            p5 = W.config(5)
            g5 = J.build_graph(p5.mesh, p5.omega, p5.weight)
            ttt[p5.name] = time_to_tol(J, torch, g5, p5)
            g5.close()
        print(json.dumps({"time_to_tol": ttt}))
        return

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
    kernel_key = "k_sweep<double> hex64_s8"
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, sweep kernel {avg_kernel_s * 1e3:.3f} ms")

    avg32_s, ttt, ens, cpu, err = None, None, None, None, None
    if not args.steps_only:
        avg32_s, ttt, ens, cpu, err = extras(args, J, W, torch, g, p, st, ss, q, phi)

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
                     "frac": achieved / PEAK_HBM_GBS, "traffic": _traffic(kernel_key),
                     "kernel": kernel_key, "algorithmic_bytes_per_launch": bytes_alg,
                     "interior_edges": edges, "avg_kernel_ms": avg_kernel_s * 1e3, "launches": launches},
        "cpu_baseline": cpu,
        "sweep_kernel_ms": {"fp64": avg_kernel_s * 1e3, "fp32": avg32_s * 1e3 if avg32_s else None},
        "sweep_updates_per_s_kernel": {"fp64": nc * nd / avg_kernel_s,
                                       "fp32": nc * nd / avg32_s if avg32_s else None},
        "time_to_tol": ttt,
        "ensemble": ens,
        "sweep_rel_err_vs_oracle": err,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
