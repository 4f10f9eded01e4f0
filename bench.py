"""Benchmark of the data-driven transport sweep on one MI355X.

Headline workload (the largest single-GPU configuration): Kuhn tetrahedra
of a jittered 96^3 lattice (6 tets per cube, 5,308,416 cells, interior
vertices moved by up to 0.15 h), level-symmetric S8 (80 directions), a
checkerboard of 8^3 material blocks (sigma_t 1 / 10, scattering ratio
0.5 / 0.99), q = 1, vacuum boundaries.

A step is one FP64 source iteration through the C ABI: scattering source,
data-driven sweep of all 80 directions over the per-direction dependency
graph, scalar flux and FP64 residual.  The graph is built once before the
timed region (preprocessing).  value = cell-angle updates per second over
the timed steps, inputs resident in HBM.

Also reported:
  roofline      the FP64 sweep kernel's algorithmic bytes per launch (each
                angular flux written once and read once per downwind
                neighbour, 8 B each) over its average launch time, from HIP
                events around every sweep launch in the timed region;
                traffic from the committed rocprofv3 counter summary when it
                was taken on the current kernel source, else null;
  fp32_correction_sweep  the same for the FP32 correction sweep of the
                refined solve (4 B per flux plus the 4 B per-(cell,
                direction) correction source);
  cpu_baseline  the oracle (plain FP64 CPU code) timed on this host: one
                sweep of all 80 directions of the 64^3 hexahedral workload
                serially and with its directions spread over threads, and
                its source iteration to rho <= 1e-8 with threaded sweeps;
  time_to_tol   wall time of jsweep_solve to rho <= 1e-8, plain FP64 and
                FP32-refined, on this workload, on the 64^3 hexahedral S8
                one and on the S16 tetrahedral one (60^3 lattice, 288
                directions), each the fastest of three solves after an
                untimed warm-up of the mode, with the error of each result
                against the oracle's converged scalar flux at the sampled
                cells of tests/golden/fullsize_<name>.txt;
  ensemble      256 independent meshes (500-50,000 cells, half triangles,
                half tets, S4-S8) solved together by jsweep_solve_batch:
                FP64 step throughput and time-to-1e-8, FP64 vs
                FP32-refined (each the fastest of three after a warm-up),
                with the autotuned launch parameters;
  flux_pass     the rest of a step (step time minus the sweep kernel's):
                the flux pass's algorithmic bytes (12 B per cell-angle pair
                and 56 B per cell) and the rate they imply;
  hbm_copy_probe  the best of five 2 GiB device-to-device copies (HIP
                events): the bandwidth this GPU sustains on a plain stream,
                the FP64 sweep's algorithmic rate as a fraction of it, and
                the sweep's counted HBM rate (counter summary over launch
                time) beside it.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-ttt]
                       [--no-ensemble] [--copy-probe] [--steps-only]
                       [--workload tetcheck96_s8|hex64_s8|tetlogn60_s16] [--fp32-steps]
                       [--groups-only]
  --copy-probe  first copies 512 MiB device to device (the calibration
                dispatch for HBM byte counters taken on this run)
  --steps-only  only the timed steps and the roofline (for profiler runs)
  --fp32-steps  with --steps-only: time FP32 correction sweeps instead
  --groups-only only the 4-group source iterations (for profiler runs)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
WORKLOADS = {"delaunay40x50_s4": 1, "hex64_s8": 2, "tetcheck96_s8": 3, "tetlogn60_s16": 5}
DESCR = {
    "tetcheck96_s8": "Kuhn tetrahedra of a jittered 96^3 lattice (5,308,416 cells), S8 (80 directions), "
                     "8^3-block checkerboard (sigma_t 1/10, c 0.5/0.99), FP64 source iteration step",
    "hex64_s8": "jittered 64^3 hexahedra (262,144 cells), S8 (80 directions), scattering ratio 0.9, "
                "FP64 source iteration step",
    "tetlogn60_s16": "Kuhn tetrahedra of a jittered 60^3 lattice (1,296,000 cells), S16 (288 directions), "
                     "lognormal sigma_t, c 0.95, FP64 source iteration step",
    "delaunay40x50_s4": "2D Delaunay of 2,000 jittered points (3,822 triangles), S4 (12 directions), "
                        "FP64 source iteration step",
}


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


def _golden(name):
    """Sampled oracle values of a full-size workload (or None)."""
    path = os.path.join(ROOT, "tests", "golden", f"fullsize_{name}.txt")
    if not os.path.exists(path):
        return None
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    from make_fullsize_golden import load
    return load(name)


def err_vs_oracle(phi, gold):
    """max and normwise relative error of phi against the oracle's converged
    scalar flux at the sampled cells."""
    if gold is None or gold.get("phi_converged") is None:
        return None
    ref = gold["phi_converged"]
    got = phi[gold["cells"]]
    return {"max_rel": float(np.abs(got - ref).max() / np.abs(ref).max()),
            "norm_rel": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
            "sampled_cells": int(len(ref)), "oracle_rho": gold.get("converged_rho")}


TTT_REPEATS = 3


def time_to_tol(J, torch, g, p, tol=1e-8):
    """jsweep_solve to rho <= tol, plain FP64 then FP32-refined, from zero;
    each the fastest of TTT_REPEATS solves after an untimed warm-up."""
    st, ss, q = (torch.tensor(a, device="cuda") for a in (p.sigma_t, p.sigma_s, p.q))
    gold = _golden(p.name)
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
        phi_h = phi.cpu().numpy()
        out[name]["phi_err_vs_oracle"] = err_vs_oracle(phi_h, gold)
        if ref is None:
            ref = phi
        else:
            out[name]["phi_rel_err_vs_fp64"] = float(torch.linalg.norm(phi - ref) / torch.linalg.norm(ref))
    out["speedup_fp32_refined"] = out["fp64"]["seconds"] / out["fp32_refined"]["seconds"]
    return out


def multigroup_bench(J, W, torch, g, p, edges, single_sweep_ms, groups=4, iters=4, warmup=1):
    """FP64 multigroup source iterations (Jacobi over groups, every
    (direction, group) in one sweep launch) on the workload's graph: time
    per iteration, the multigroup sweep kernel's time and roofline, and the
    single-group sweep time for comparison."""
    mp = W.multigroup(p, groups)
    st, ss, q = (torch.tensor(a, device="cuda") for a in (mp.sigma_t, mp.sigma_s, mp.q))
    phi = torch.zeros((groups, p.n_cells), dtype=torch.float64, device="cuda")
    J.solve_groups(g, st, ss, q, phi, tol=0.0, max_iter=warmup, allow_not_converged=True)

    def timed(k):
        torch.cuda.synchronize()
        a = time.perf_counter()
        J.solve_groups(g, st, ss, q, phi, tol=0.0, max_iter=k, allow_not_converged=True)
        torch.cuda.synchronize()
        return time.perf_counter() - a

    # a solve's set-up (its per-group denominators) apart from its
    # iterations: the difference of a short and a longer solve
    t_short = timed(2)
    J.jsweep_profile(g, True)
    J.jsweep_profile_read(g, reset=True)
    t_long = timed(2 + iters)
    n, ms = J.jsweep_profile_read(g, reset=True)
    J.jsweep_profile(g, False)
    sec = (t_long - t_short) / iters
    setup = t_short - 2 * sec
    upd = p.n_cells * p.n_dirs * groups
    kms = ms / max(1, n)
    del st, ss, q, phi
    return {"groups": groups, "iteration_ms": sec * 1e3, "updates_per_s": upd / sec, "solve_setup_ms": setup * 1e3,
            "sweep_kernel_ms": kms, "sweep_updates_per_s_kernel": upd / (kms * 1e-3),
            "single_group_sweep_ms": single_sweep_ms,
            "groups_x_single_group_sweep_ms": None if single_sweep_ms is None else groups * single_sweep_ms,
            "roofline": roofline((p.n_cells * p.n_dirs + edges) * 8 * groups, kms,
                                 f"k_sweep<double> {groups} groups {p.name}", n, edges)}


def interior_edges(J, g, n_dirs):
    """Interior upwind edges summed over directions (lagged ones included):
    the in-degrees of every direction plus the lagged edges."""
    edges = 0
    for m in range(n_dirs):
        indeg, _, _, _ = J.graph_export(g, m, want=("indeg",))
        edges += int(indeg.sum())
    return edges + J.graph_info(g)["n_lagged"]


def host_cpu():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return model, avail


def cpu_baseline(W):
    """The oracle timed on this host (hexahedral 64^3 S8 workload): one
    serial sweep of all directions, the same sweep with directions spread
    over threads, and its source iteration to rho <= 1e-8 with threaded
    sweeps (the residual is the oracle's serial operator form)."""
    import oracle
    p = W.config(2)
    model, avail = host_cpu()
    threads = max(1, min(16, avail))
    t = time.time()
    og = oracle.graph_for(p)
    t_build = time.time() - t
    upd = p.n_cells * p.n_dirs
    t = time.time()
    og.sweep(p.sigma_t, p.q)
    serial = time.time() - t

    def threaded(src, prev, psi):
        b = np.linspace(0, p.n_dirs, threads + 1).astype(int)
        ths = [threading.Thread(target=og.sweep_dirs, args=(int(x), int(y), p.sigma_t, src),
                                kwargs={"psi_prev": prev, "psi": psi}) for x, y in zip(b[:-1], b[1:]) if y > x]
        for th in ths:
            th.start()
        for th in ths:
            th.join()

    psi = np.zeros((p.n_dirs, p.n_cells))
    t = time.time()
    threaded(p.q, None, psi)
    par = time.time() - t
    # source iteration to 1e-8 (threaded sweeps)
    psi = np.zeros((p.n_dirs, p.n_cells))
    prev = np.zeros_like(psi)
    phi = np.zeros(p.n_cells)
    t = time.time()
    it, rho = 0, 1.0
    while rho > 1e-8 and it < 200:
        prev[...] = psi
        threaded(p.q + p.sigma_s * phi, prev, psi)
        phi = og.phi(p.weight, psi)
        rho = og.residual(p.sigma_t, p.sigma_s, p.q, p.weight, psi, phi)
        it += 1
    solve_s = time.time() - t
    return {
        "value": upd / par,
        "unit": "cell-angle updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"one FP64 sweep of all {p.n_dirs} directions of {p.name} ({upd} cell-angle updates), "
                  f"directions spread over {threads} threads (graph build {t_build:.1f} s, untimed)",
        "serial_value": upd / serial,
        "serial_cores": 1,
        "cpu_model": model,
        "host_cpus_available": avail,
        "solve_to_1e-8": {"seconds": solve_s, "sweeps": it, "residual": rho, "threads": threads,
                          "workload": p.name},
    }


def ensemble_bench(J, W, torch, steps=5, ttt_solves=True):
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
    J.jsweep_profile(gs[0], True)      # the batch's data-driven launches are recorded on its first graph
    J.jsweep_profile_read(gs[0], reset=True)
    a = time.perf_counter()
    J.solve_batch(gs, pr, mode=J.JSWEEP_FP64, tol=0.0, max_iter=steps, params=tuned, allow_not_converged=True)
    torch.cuda.synchronize()
    step = (time.perf_counter() - a) / steps
    launches, kms = J.jsweep_profile_read(gs[0], reset=True)
    J.jsweep_profile(gs[0], False)
    out["fp64_step_ms"] = step * 1e3
    out["fp64_updates_per_s"] = upd / step
    if launches:
        edges = sum(interior_edges(J, g, p.n_dirs) for g, p in zip(gs, ps))
        out["roofline"] = roofline((upd + edges) * 8, kms / launches,
                                   "k_sweep<double> union of the 256-instance ensemble", launches, edges)
    if not ttt_solves:
        for g in gs:
            g.close()
        return out
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


def fp32_sweep_ms(J, torch, g, st, ss, q, nc, warmup, n=10):
    """Average FP32 correction-sweep kernel time (HIP events) over the inner
    sweeps of an FP32-refined solve."""
    J.jsweep_profile(g, True)
    J.solve(g, st, ss, q, torch.zeros(nc, dtype=torch.float64, device="cuda"), mode=J.JSWEEP_FP32_REFINED,
            tol=0.0, max_iter=1 + warmup, allow_not_converged=True)
    J.jsweep_profile_read(g, reset=True)
    J.solve(g, st, ss, q, torch.zeros(nc, dtype=torch.float64, device="cuda"), mode=J.JSWEEP_FP32_REFINED,
            tol=0.0, max_iter=n, allow_not_converged=True)
    n32, ms32 = J.jsweep_profile_read(g, reset=True)
    J.jsweep_profile(g, False)
    return ms32 / max(1, n32), n32


def copy_probe(torch, mib=2048, reps=5):
    """Achievable HBM bandwidth on this GPU: the best of `reps` device-to-
    device copies of `mib` MiB (each moves 2 x mib MiB: read and write),
    timed with HIP events on the current stream."""
    n = (mib << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    best = None
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        y.copy_(x)
        e1.record()
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        best = ms if best is None else min(best, ms)
    del x, y
    return {"bytes_moved": 2 * (mib << 20), "ms": best, "gbs": 2 * (mib << 20) / (best * 1e-3) / 1e9}


def roofline(bytes_alg, avg_ms, kernel_key, launches, edges):
    achieved = bytes_alg / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": achieved / PEAK_HBM_GBS, "traffic": _traffic(kernel_key), "kernel": kernel_key,
            "algorithmic_bytes_per_launch": bytes_alg, "interior_edges": edges, "avg_kernel_ms": avg_ms,
            "launches": launches}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="tetcheck96_s8", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ttt", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-groups", action="store_true")
    ap.add_argument("--copy-probe", action="store_true")
    ap.add_argument("--steps-only", action="store_true")
    ap.add_argument("--fp32-steps", action="store_true")
    ap.add_argument("--groups-only", action="store_true",
                    help="only the 4-group source iterations of the workload (for profiling the multigroup sweep)")
    ap.add_argument("--ttt-only", action="store_true",
                    help="only the time-to-1e-8 solves (FP64 and FP32-refined) of the workload; one JSON line")
    ap.add_argument("--ensemble-steps-only", action="store_true",
                    help="only the batched ensemble's FP64 steps (every instance iterating)")
    ap.add_argument("--ensemble-only", action="store_true",
                    help="only the 256-instance batched solve (for profiling the batch kernels)")
    ap.add_argument("--priority-list", default="", help="with --priorities: comma-separated names to time")
    ap.add_argument("--priorities", action="store_true",
                    help="only the FP64 sweep kernel time of the workload under every work-list priority "
                         "(BFS, LDCP, SLBD, each also angle-major); one JSON line")
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
    if args.ensemble_only or args.ensemble_steps_only:
        ens = ensemble_bench(J, W, torch, steps=max(1, args.steps), ttt_solves=not args.ensemble_steps_only)
        print(json.dumps({"ensemble": ens}))
        return
    p = W.config(WORKLOADS[args.workload])
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
        print(json.dumps({"time_to_tol": {p.name: time_to_tol(J, torch, g, p)}}))
        return
    if args.priorities:
        res = {}
        names = {J.JSWEEP_PRIORITY_BFS: "BFS", J.JSWEEP_PRIORITY_LDCP: "LDCP", J.JSWEEP_PRIORITY_SLBD: "SLBD",
                 J.JSWEEP_PRIORITY_PACED: "PACED"}
        plist = [(names[b] + ("+angle-major" if am else ""), b | am)
                 for am in (0, J.JSWEEP_PRIORITY_ANGLE_MAJOR) for b in names]
        plist += [(f"BFS+C=L/{k}", J.JSWEEP_PRIORITY_BFS | J.JSWEEP_PRIORITY_ANGLE_WEIGHT(k)) for k in range(1, 8)]
        plist += [(f"LDCP+C=L/{k}", J.JSWEEP_PRIORITY_LDCP | J.JSWEEP_PRIORITY_ANGLE_WEIGHT(k)) for k in (2, 3)]
        plist += [(f"PACED+C=L/{k}", J.JSWEEP_PRIORITY_PACED | J.JSWEEP_PRIORITY_ANGLE_WEIGHT(k)) for k in (5, 7)]
        if args.priority_list:
            keep = set(args.priority_list.split(","))
            plist = [x for x in plist if x[0] in keep]
        for key, pr in plist:
            t = time.time()
            J.set_params(g, J.Params(priority=pr))
            t_order = time.time() - t
            J.solve(g, st, ss, q, phi, psi, mode=J.JSWEEP_FP64, tol=0.0, max_iter=max(1, args.warmup),
                    allow_not_converged=True)
            J.jsweep_profile(g, True)
            J.jsweep_profile_read(g, reset=True)
            J.solve(g, st, ss, q, phi, psi, mode=J.JSWEEP_FP64, tol=0.0, max_iter=args.steps,
                    allow_not_converged=True)
            n, ms = J.jsweep_profile_read(g, reset=True)
            J.jsweep_profile(g, False)
            ms32, _ = fp32_sweep_ms(J, torch, g, st, ss, q, nc, args.warmup, args.steps)
            res[key] = {"priority": pr, "fp64_sweep_ms": ms / max(1, n), "fp32_sweep_ms": ms32,
                        "reorder_s": t_order}
            log(f"priority {key}: {res[key]}")
        J.set_params(g, None)
        print(json.dumps({"workload": p.name, "priorities": res}))
        return
    if args.groups_only:
        mg = multigroup_bench(J, W, torch, g, p, interior_edges(J, g, nd), None, iters=max(1, args.steps))
        log(f"multigroup: {json.dumps(mg)}")
        print(json.dumps({"workload": p.name, "multigroup": mg}))
        return
    if args.steps_only and args.fp32_steps:
        ms, n = fp32_sweep_ms(J, torch, g, st, ss, q, nc, args.warmup, args.steps)
        log(f"FP32 correction sweep {ms:.3f} ms over {n} launches")
        print(json.dumps({"workload": p.name, "fp32_sweep_ms": ms, "launches": n}))
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
    edges = interior_edges(J, g, nd)
    avg64 = kernel_ms / max(1, launches)
    roof = roofline((nc * nd + edges) * 8, avg64, f"k_sweep<double> {p.name}", launches, edges)
    log(f"timed {args.steps} steps: {ms_per_step:.3f} ms/step, sweep kernel {avg64:.3f} ms, "
        f"roofline frac {roof['frac']:.3f}")
    # the rest of a step is the flux pass (one kernel: scalar flux gathered
    # through the level positions, identity residual, next source and V s):
    # 8 B of flux and 4 B of position per (direction, cell), 7 per-cell
    # doubles (phi, sigma_s, q, V read; phi, source, V s written)
    rest_ms = ms_per_step - avg64
    flux_bytes = nc * nd * 12 + nc * 8 * 7
    flux_pass = {"ms_step_minus_sweep": rest_ms, "algorithmic_bytes": flux_bytes,
                 "gbs": flux_bytes / (rest_ms * 1e-3) / 1e9 if rest_ms > 0 else None,
                 "note": "lagged-edge terms not counted" if info["n_lagged"] else None}

    line_extra = {}
    if not args.steps_only:
        ms32, n32 = fp32_sweep_ms(J, torch, g, st, ss, q, nc, args.warmup)
        roof32 = roofline((nc * nd + edges) * 4 + nc * nd * 4, ms32, f"k_sweep<float> {p.name}", n32, edges)
        log(f"FP32 correction sweep {ms32:.3f} ms, roofline frac {roof32['frac']:.3f}")
        line_extra["fp32_correction_sweep"] = {"updates_per_s": nc * nd / (ms32 * 1e-3), "roofline": roof32}
        if not args.no_groups:
            mg = multigroup_bench(J, W, torch, g, p, edges, avg64)
            log(f"multigroup: {json.dumps(mg)}")
            line_extra["multigroup"] = mg
        # one sweep on fixed inputs, compared with the oracle's sampled angular flux is in the GPU tests
        ttt = None
        if not args.no_ttt:
            ttt = {p.name: time_to_tol(J, torch, g, p)}
            log(f"time to 1e-8 on {p.name}: {json.dumps(ttt[p.name])}")
        g.close()
        if not args.no_ttt:
            for k in (2, 5):
                if WORKLOADS[args.workload] == k:
                    continue
                pk = W.config(k)
                gk = J.build_graph(pk.mesh, pk.omega, pk.weight)
                ttt[pk.name] = time_to_tol(J, torch, gk, pk)
                gk.close()
                log(f"time to 1e-8 on {pk.name}: {json.dumps(ttt[pk.name])}")
        line_extra["time_to_tol"] = ttt
        ens = None
        if not args.no_ensemble:
            ens = ensemble_bench(J, W, torch)
            log(f"ensemble: {json.dumps(ens)}")
        line_extra["ensemble"] = ens
        cpu = None
        if not args.no_cpu:
            cpu = cpu_baseline(W)
            log(f"cpu baseline: {json.dumps(cpu)}")
        line_extra["cpu_baseline"] = cpu
        probe = copy_probe(torch)
        probe["sweep_frac_of_copy"] = roof["achieved"] / probe["gbs"]
        if roof["traffic"]:
            probe["sweep_counted_gbs"] = roof["traffic"] / (avg64 * 1e-3) / 1e9
        log(f"copy probe: {json.dumps(probe)}")
        line_extra["hbm_copy_probe"] = probe

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
        "config": {"workload": f"{p.name}: {DESCR[p.name]}",
                   "cells": nc, "dirs": nd, "lagged_edges": info["n_lagged"], "max_levels": info["max_levels"],
                   "graph_build_s": t_build},
        "roofline": roof,
        "cpu_baseline": line_extra.pop("cpu_baseline", None),
        "sweep_kernel_ms": {"fp64": avg64},
        "sweep_updates_per_s_kernel": {"fp64": nc * nd / (avg64 * 1e-3)},
        "flux_pass": flux_pass,
    }
    line.update(line_extra)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
