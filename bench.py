"""Benchmark: DOF-iterations/s of J-FFT PCG on a 256^3 periodic cell (one MI355X).

One step = one pass of the whole hot path on one synthetic input resident in
HBM: set the material (copy E, Algorithm 2 diagonal, J^1/2), assemble the
right-hand side, run PCG with the Green-Jacobi preconditioner to a true
relative residual of 1e-8, remove the mean and evaluate the homogenised
stress.  The headline path is the mixed-precision solver (FP32 stencil, FFT,
preconditioner and vectors; FP64 dots, alpha/beta, iterate and an FP64
iterative-refinement residual); the plain FP64 solver is timed on the same
input and reported beside it.

value = DOF x PCG iterations (all inner iterations) / wall time of the timed
steps, with DOF = 3 n^3.  The same line carries the served-stream figures
("serving": capacity, Poisson-arrival throughput, p50/p99 latency of
homogenisation requests, mixed and FP64), the roofline of the dominant
kernel and the CPU oracle baseline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 256]
                       [--contrast 1e4] [--no-cpu] [--no-fp64] [--no-serve]
       python bench.py --workload simp2d [--cells 512]   (batched 2D SIMP cells)
       python bench.py --workload powerlaw [--pl-n 200]  (nonlinear Newton example)
       python bench.py --workload tri [--tri-cells 32]   (2D linear triangles)
       python bench.py --workload topopt [--topo-iters 30] (phase-field topology optimisation)
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
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X, FP64 vector (no MFMA)
# FP32 vector peak without packed FP32 instructions (this build does not use
# them): 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz.  The 157.3
# TFLOP/s of the data sheet counts packed (two-wide) FP32 FMAs.
FP32_VECTOR_PEAK_TFLOPS = 78.6
# Algorithmic flops of one element of the power-law tangent operator
# (Sec. 2.2, Sec. 4) in the factorised Gauss-point form, counted from the
# method's operations (a*x + b*y = 3 flops, FMA = 2): gradients of the
# iterate and of p at the 8 Gauss points (2 fields x 3 components x 3
# directions x [4 differences + 4 two-point interpolations x 6 + 4 scalings]
# = 576); per Gauss point the two Mandel strains (12), the macro strain (6),
# the tangent (matrix 64: trace, deviator, e.e, e.d, g and h for the integer
# exponent, the 6 stress components; inclusion 17), the weight (6), the
# element energy p.Kp (12), the shear factors (3) and the family sums (9);
# the corner forces (3 components x 3 directions x [4 interpolations x 6 +
# 4 scalings + 8 additions] = 324).  Matrix element 1796, inclusion 1420.
TANGENT_FLOPS_MATRIX = 576 + 8 * (12 + 6 + 64 + 6 + 12 + 3 + 9) + 324
TANGENT_FLOPS_INCLUSION = 576 + 8 * (12 + 6 + 17 + 6 + 12 + 3 + 9) + 324


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--contrast", type=float, default=1e4)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates HBM byte counters)")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-stream measurement")
    ap.add_argument("--fused-control", type=int, default=-1,
                    help="topopt: run the CG scalar steps in the last block of their producer "
                         "kernels (1) or as their own launches (0); -1: the library default")
    ap.add_argument("--serve-mode", choices=("slots", "handles", "both"), default="both",
                    help="serving runs: continuous batching over group slots, whole handles "
                         "per worker, or both")
    ap.add_argument("--graph", type=int, default=8,
                    help="PCG iterations per captured HIP graph in the timed steps (0: direct launches)")
    ap.add_argument("--serve-requests", type=int, default=400)
    ap.add_argument("--pl-n", type=int, default=200, help="powerlaw: nodes per axis")
    ap.add_argument("--tri-cells", type=int, default=32, help="tri: 512^2 cells in the group")
    ap.add_argument("--topo-iters", type=int, default=30, help="topopt: L-BFGS steps")
    ap.add_argument("--topo-n", type=int, default=256, help="topopt: nodes per axis")
    ap.add_argument("--workload", default="grf256",
                    choices=["grf256", "simp2d", "contrast", "powerlaw", "tri", "topopt",
                             "sweeps"],
                    help="grf256: the headline 256^3 cell (+ served stream); simp2d: 512 "
                         "batched 2D SIMP cells of uneven sizes")
    ap.add_argument("--cells", type=int, default=512, help="simp2d: number of cells")
    return ap.parse_args()


def copy_probe():
    """A plain device-to-device copy of exactly 2^30 bytes, five times: the
    reference against which rocprofv3 FETCH_SIZE / WRITE_SIZE are scaled."""
    import torch

    x = torch.ones(2 ** 27, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(5):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": 2 ** 30, "copy_probe_bytes_written": 2 ** 30,
                      "launches": 5}), flush=True)


def spectrum_ratio(n):
    m = n // 2
    return (m + 1) / (2.0 * m)


def algorithmic_bytes(kernel, dim, N, n_x, real_bytes):
    """Bytes a kernel must move per launch in the fused design (each array
    read or written once): fields of d components, half spectrum of d
    components, element moduli."""
    field = dim * N * real_bytes
    spec = dim * N * spectrum_ratio(n_x) * 2 * real_bytes
    scalar = N * real_bytes
    table = {
        # z, p_old, u read; u, p_new, q written; E read
        "stiffness_cg": 6 * field + scalar,
        "stiffness_apply": 2 * field + scalar,
        # r, q, J^1/2 read; r written; spectrum written
        "fft_x_forward": 4 * field + spec,
        "fft_y_forward": 2 * spec,
        "fft_green_axis": 2 * spec,
        "fft_y_inverse": 2 * spec,
        # spectrum, J^1/2 read; z written (r.z is formed in the Green pass)
        "fft_x_inverse": spec + 2 * field,
        # power-law tangent: the CG stiffness traffic plus the Newton iterate
        "stiffness_cg_tangent": 7 * field + scalar,
        "diag_precond": 5 * field,
    }
    return table.get(kernel)


# precision of each kernel name in the mixed path
MIXED_KERNEL_BYTES = {"stiffness_apply": 8}


def source_hash():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2508_02613_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(workload_key, kernel):
    """HBM traffic per launch from committed rocprofv3 counter summaries,
    only if they were taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except Exception:
        return None
    ent = data.get(workload_key, {}).get(kernel)
    if not ent or ent.get("source_sha") != source_hash():
        return None
    return ent.get("bytes_per_launch")


def run_restarted(args, E, nu, macro, tol, maxit):
    """One mixed-precision solve with the FP32 CG restarted at every
    refinement sweep (the alternative to the default continued CG), for the
    iteration and time-to-solution comparison in the bench line."""
    import torch

    import paper_2508_02613_amd as pkg

    stream = torch.cuda.Stream()
    cell = pkg.Cell(E.shape, precision=pkg.MIXED, pc=pkg.PC_GREEN_JACOBI, stream=stream)
    if args.graph:
        cell.set_graph_iterations(args.graph)
    cell.set_mixed_params(continue_cg=False)
    Ed = torch.from_numpy(E).to("cuda")
    reps = []
    for _ in range(2):  # the first solve warms up the graph
        cell.set_material(Ed, nu=nu)
        _, _, rep, _ = cell.solve(macro, tol=tol, maxit=maxit)
        reps.append(rep)
    cell.close()
    rep = reps[-1]
    return {"iters": rep.iters, "outer_sweeps": rep.outer, "loop_ms": rep.loop_ms,
            "rel_res_true": rep.rel_res_true}


def run_gpu(args, precision_name, E, nu, macro, tol, maxit):
    """Timed steps as a production caller runs them (own stream, PCG
    iterations replayed from captured HIP graphs, no per-kernel events), then
    the same number of steps again with HIP events around every launch on the
    cell's stream for the per-kernel durations (events keep graph replay off,
    which is why they are not in the timed steps)."""
    import torch

    import paper_2508_02613_amd as pkg

    prec = pkg.MIXED if precision_name == "mixed" else pkg.FP64
    shape = E.shape
    stream = torch.cuda.Stream()
    cell = pkg.Cell(shape, precision=prec, pc=pkg.PC_GREEN_JACOBI, stream=stream)
    if args.graph:
        cell.set_graph_iterations(args.graph)
    Ed = torch.from_numpy(E).to("cuda")
    u = torch.empty((3,) + shape, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()

    def step():
        cell.set_material(Ed, nu=nu)
        return cell.solve(macro, tol=tol, maxit=maxit, out=u)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for _ in range(args.steps):
        _, sbar, rep, _ = step()
        reps.append(rep)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-kernel durations over the same number of steps
    cell.reset_timing()
    cell.enable_timing(True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    stats = cell.kernel_stats()
    cell.enable_timing(False)
    cell.close()
    wall = t1 - t0
    iters = sum(r.iters for r in reps)
    return {"wall_s": wall, "iters": iters, "reps": reps, "stats": stats, "sigma_bar": sbar,
            "events_wall_s": t3 - t2}


def cpu_baseline(E, macro, nu):
    """The oracle, timed on one PCG iteration's operators (K p and the
    Green-Jacobi preconditioner with its naive DFT) on the full 256^3 input.
    Its one-off set-up (Algorithm 1 DFTs of 9 fields, Algorithm 2 with 24
    element-loop stiffness applications) is not part of the sample; the
    per-iteration cost does not depend on the values of G^ and diag, so the
    sample passes placeholders of the right shape for them."""
    import oracle

    lam, mu = oracle.lame_from_nu(nu)
    shape = E.shape
    dim = len(shape)
    rng = np.random.default_rng(0)
    p = rng.standard_normal((dim,) + shape)
    G = np.zeros((dim, dim) + shape, dtype=complex)
    G[0, 0] = 1.0
    diag = np.ones((dim,) + shape)
    t0 = time.perf_counter()
    q = oracle.stiffness(E, p, lam, mu)
    t1 = time.perf_counter()
    z, _ = oracle.precond(oracle.PC_GREEN_JACOBI, q, diag=diag, G=G)
    t2 = time.perf_counter()
    # dots and updates of one iteration (numpy, same order of work)
    a = float((p * q).sum())
    p += a * z
    t3 = time.perf_counter()
    per_iter = t3 - t0
    dofs = dim * E.size
    return {
        "value": dofs / per_iter,
        "unit": "DOF·it/s",
        "cores": oracle.num_threads(), "cpu": host_cpu(),
        "kind": "oracle",
        "sample": (f"one PCG iteration of the FP64 C oracle (element-loop K·p {t1 - t0:.1f} s, "
                   f"Green-Jacobi M^-1 with naive separable DFT {t2 - t1:.1f} s, dots/axpys "
                   f"{t3 - t2:.1f} s) on the same {shape[0]}^3 input; set-up excluded"),
        "seconds_per_iteration": per_iter,
    }


def host_cpu():
    """Model name of the host CPU (from /proc/cpuinfo) and its logical CPUs."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def serve_field_pool(count, seed):
    """The served-stream materials: 3D cells with side uniform from {32, 48,
    64, 96, 128}, smooth GRF (correlation length 0.1) with contrast
    log-uniform in [1e2, 1e4].  A pool of distinct fields that the request
    streams draw from (generating one field per request would take longer on
    the host than serving it)."""
    import jfft_inputs as ji

    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice((32, 48, 64, 96, 128)))
        c = float(10 ** rng.uniform(2.0, 4.0))
        out.append(ji.grf_field((n, n, n), c, seed=seed * 100003 + i, ell=0.1))
    return out


def serve_requests(pool, count, seed):
    """`count` requests (C_eff of 6 load cases each), fields drawn from the pool."""
    from paper_2508_02613_amd.serve import Request

    rng = np.random.default_rng(seed)
    return [Request(i, pool[int(rng.integers(len(pool)))]) for i in range(count)]


LOAD_FRACTIONS = (0.5, 0.8, 0.95)




def run_serving(args):
    """Saturated capacity (all requests at t = 0), then Poisson arrivals at
    0.5, 0.8 and 0.95 x that capacity, for the mixed and the FP64 solver at
    equal final accuracy (true relative residual <= 1e-8 for every load
    case).  p99 is reported only for runs of at least 200 requests (at least
    two samples above it)."""
    import paper_2508_02613_amd as pkg
    from paper_2508_02613_amd.serve import Server, SlotServer

    nreq = args.serve_requests
    pool = serve_field_pool(80, 7)
    out = {"workload": (f"{nreq} requests per run, 3D side uniform from {{32,48,64,96,128}}, GRF "
                        "contrast log-uniform 1e2-1e4 (drawn from 80 distinct fields), 6 load "
                        "cases -> C_eff each, 64 GiB admission budget, 8 PCG iterations per "
                        "graph; Poisson arrivals at 0.5, 0.8 and 0.95 x the measured capacity. "
                        "mixed, fp64: 4 workers with whole handles, merge <= 4 waiting requests "
                        "of side <= 64; slots_mixed: continuous batching over group slots (one "
                        "group of 2 requests = 12 slots per shape; the library runs 4-iteration "
                        "chunks until a load case finishes or 2 ms pass, then the driver "
                        "harvests and admits)"),
           "unit": "requests/s (6 solves each); latency ms"}
    runs = []
    if args.serve_mode in ("handles", "both"):
        runs += [("mixed", pkg.MIXED, False), ("fp64", pkg.FP64, False)]
    if args.serve_mode in ("slots", "both"):
        runs += [("slots_mixed", pkg.MIXED, True)]
    for name, prec, slots in runs:
        print(f"[serving] {name}: warm-up, capacity, then Poisson loads {LOAD_FRACTIONS}",
              file=sys.stderr, flush=True)
        if slots:
            srv = SlotServer(budget_bytes=64 << 30, precision=prec, graph_iterations=4,
                             slots_per_group=2)
        else:
            srv = Server(workers=4, budget_bytes=64 << 30, precision=prec, graph_iterations=8)
        srv.run(serve_requests(pool, 8, 99), rate=None)  # warm-up: handles, graphs, kernels
        sat = srv.run(serve_requests(pool, nreq, 1), rate=None)
        row = {"capacity_requests_per_s": sat["requests_per_s"],
               "capacity_solves_per_s": sat["solves_per_s"], "loads": {}}
        ok = sat["all_ok"]
        worst = sat["max_rel_res_true"]
        for frac in LOAD_FRACTIONS:
            lam = frac * sat["requests_per_s"]
            print(f"[serving] {name}: capacity {sat['requests_per_s']:.1f} req/s; load {frac}",
                  file=sys.stderr, flush=True)
            po = srv.run(serve_requests(pool, nreq, 2), rate=lam, seed=3)
            row["loads"][str(frac)] = {
                "poisson_rate": lam, "requests": po["requests"],
                "requests_per_s": po["requests_per_s"], "solves_per_s": po["solves_per_s"],
                "p50_latency_ms": po["p50_latency_ms"], "p95_latency_ms": po["p95_latency_ms"],
                "p99_latency_ms": po["p99_latency_ms"] if po["requests"] >= 200 else None}
            if slots:
                row["loads"][str(frac)]["mean_busy_slots_per_wakeup"] = po["mean_busy_slots_per_wakeup"]
            else:
                row["loads"][str(frac)]["mean_merged"] = po["mean_merged"]
            ok = ok and po["all_ok"]
            worst = max(worst, po["max_rel_res_true"])
        srv.close()
        row["all_ok"] = ok
        row["max_rel_res_true"] = worst
        out[name] = row
    return out


def run_simp2d(args):
    """Batch of 2D plane-strain SIMP cells of uneven sizes: sides uniform from
    {64, 128, 256, 512}, E = rho^3 with rho in [1e-3, 1] from blurred noise
    (4 px), nu 0.3, macro strain cycling e11, e22, e12; groups per size on
    their own streams, mixed precision, launch parameters and graph depth per
    size from the autotuner (tuned during the warm-up step).
    Baseline: the same cells one at a time with the FP64 solver."""
    import torch

    import jfft_inputs as ji
    import paper_2508_02613_amd as pkg
    from paper_2508_02613_amd.groups import solve_cells

    rng = np.random.default_rng(args.seed)
    sizes = rng.choice((64, 128, 256, 512), size=args.cells)
    fields = [ji.simp_field(int(n), seed=args.seed * 7919 + i) for i, n in enumerate(sizes)]
    macros = [ji.unit_macro_strain(2, i % 3) for i in range(args.cells)]
    dofs = np.array([2 * int(n) ** 2 for n in sizes])
    # launch parameters per size from the autotuner (measured during warm-up)
    for _ in range(max(1, args.warmup)):
        solve_cells(fields, macros, tol=1e-8, precision=pkg.MIXED, want_u=False, autotune=True)
    walls, its = [], None
    for _ in range(args.steps):
        res, wall = solve_cells(fields, macros, tol=1e-8, precision=pkg.MIXED, want_u=False,
                                autotune=True)
        walls.append(wall)
        its = np.array([r["report"].iters for r in res])
        ok = all(r["report"].status == "ok" for r in res)
        worst = max(r["report"].rel_res_true for r in res)
    wall = float(np.mean(walls))
    # roofline of the dominant kernel: the group of the largest cells alone,
    # event-timed (its launch parameters from the autotuner's cache), so no
    # other group's kernels overlap the timed launches
    from paper_2508_02613_amd import tune

    n_big = int(sizes.max())
    idx = [i for i, n in enumerate(sizes) if n == n_big]
    grp = pkg.Cell((n_big, n_big), precision=pkg.MIXED, batch=len(idx),
                   stream=torch.cuda.Stream())
    tune.apply(grp, tune.autotune((n_big, n_big), batch=len(idx), precision=pkg.MIXED))
    grp.set_material(np.stack([fields[i] for i in idx]), nu=0.3)
    mac = np.stack([macros[i] for i in idx])
    grp.solve_batch(mac, tol=1e-8, maxit=20000)
    grp.reset_timing()
    grp.enable_timing(True)
    _, _, reps_ev, _ = grp.solve_batch(mac, tol=1e-8, maxit=20000)
    torch.cuda.synchronize()
    stats = grp.kernel_stats()
    tun = grp.tunables()
    grp.close()
    ev_iters = sum(r.iters for r in reps_ev)
    launches, tot_ms = stats["stiffness_cg"]
    N_big = n_big * n_big
    cell_bytes = algorithmic_bytes("stiffness_cg", 2, N_big, n_big, 4)
    achieved = cell_bytes * ev_iters / (tot_ms * 1e-3) / 1e9
    # one at a time, FP64, same cells and tolerance
    t0 = time.perf_counter()
    its64 = []
    for E, m in zip(fields, macros):
        cell = pkg.Cell(E.shape, precision=pkg.FP64)
        cell.set_material(E, nu=0.3)
        _, _, rep, _ = cell.solve(m, tol=1e-8, maxit=20000)
        its64.append(rep.iters)
        cell.close()
    torch.cuda.synchronize()
    wall64 = time.perf_counter() - t0
    value = float((dofs * its).sum() / wall)
    return {
        "metric": "DOF·iterations/s (batched 2D SIMP cells, mixed precision)",
        "value": value, "unit": "DOF·it/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": (f"{args.cells} 2D plane-strain cells, sides uniform from "
                                "{64,128,256,512}, SIMP E = rho^3, rho in [1e-3, 1] (blurred "
                                "noise, 4 px), nu 0.3, one macro strain each, Green-Jacobi "
                                "PCG to 1e-8, groups per size on concurrent streams, "
                                "autotuned launch parameters and graph depth per size"),
                   "cells": args.cells, "total_dofs": int(dofs.sum())},
        "cells_per_s": args.cells / wall,
        "all_ok": ok, "max_rel_res_true": worst,
        "iterations": {"mean": float(its.mean()), "max": int(its.max())},
        "one_at_a_time_fp64": {"wall_s": wall64, "cells_per_s": args.cells / wall64,
                               "value": float((dofs * np.array(its64)).sum() / wall64),
                               "iterations_mean": float(np.mean(its64))},
        "speedup_vs_one_at_a_time_fp64": wall64 / wall,
        "roofline": {"bound": "hbm", "kernel": f"stiffness_cg (2D Q1, FP32, {n_big}^2 group)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": load_traffic(f"simp2d_mixed_{n_big}x{len(idx)}", "stiffness_cg"),
                     "avg_ms": tot_ms / launches, "launches": launches,
                     "cell_iterations": ev_iters,
                     "algorithmic_bytes_per_cell_iteration": cell_bytes,
                     "algorithmic_bytes_per_launch": cell_bytes * len(idx),
                     "tunables": tun,
                     "measured": (f"HIP events on the group's stream around every launch: the "
                                  f"{len(idx)} cells of side {n_big} as one group alone, one "
                                  "further solve with direct launches")},
        "kernels_ms_largest_group": {k: v[1] for k, v in sorted(stats.items())},
    }


def run_contrast_sweep(args):
    """256^3 GRF cells at contrasts 1e3, 1e4, 1e5: mixed vs FP64 solver on
    e11 (iterations, DOF-iterations/s, relative difference of the mean-free
    fluctuation), and the 6 x 6 C_eff of both solvers (six load cases as one
    group) with their relative difference."""
    import torch

    import jfft_inputs as ji
    import paper_2508_02613_amd as pkg

    n = args.n
    shape = (n, n, n)
    macro = ji.unit_macro_strain(3, 0)
    rows = []
    for contrast in (1e3, 1e4, 1e5):
        E = ji.grf_field(shape, contrast, seed=args.seed, ell=0.1)
        Ed = torch.from_numpy(E).cuda()
        row = {"contrast": contrast}
        us = {}
        for name, prec in (("mixed", pkg.MIXED), ("fp64", pkg.FP64)):
            cell = pkg.Cell(shape, precision=prec, stream=torch.cuda.Stream())
            if args.graph:
                cell.set_graph_iterations(args.graph)
            cell.set_material(Ed, nu=0.3)
            cell.solve(macro, tol=1e-8, maxit=20000)  # warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u, sbar, rep, _ = cell.solve(macro, tol=1e-8, maxit=20000)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            us[name] = u.clone()
            cell.close()
            row[name] = {"iters": rep.iters, "outer": rep.outer, "wall_ms": wall * 1e3,
                         "loop_ms": rep.loop_ms, "rel_res_true": rep.rel_res_true,
                         "dof_it_per_s": 3 * E.size * rep.iters / wall}
        d = torch.linalg.vector_norm(us["mixed"] - us["fp64"]) / torch.linalg.vector_norm(us["fp64"])
        row["u_rel_diff_mixed_vs_fp64"] = float(d)
        del us
        Cm, rm = pkg.effective_stiffness(Ed, nu=0.3, tol=1e-8, precision=pkg.MIXED,
                                         stream=torch.cuda.Stream(), graph_iterations=args.graph)
        C64, r64 = pkg.effective_stiffness(Ed, nu=0.3, tol=1e-8, precision=pkg.FP64,
                                           stream=torch.cuda.Stream(), graph_iterations=args.graph)
        row["ceff_rel_diff_mixed_vs_fp64"] = float(np.abs(Cm - C64).max() / np.abs(C64).max())
        row["ceff_iters_mixed"] = [r.iters for r in rm]
        row["ceff_iters_fp64"] = [r.iters for r in r64]
        row["ceff_fp64_diag"] = [float(C64[i, i]) for i in range(6)]
        rows.append(row)
        torch.cuda.empty_cache()
    return {"metric": "contrast sweep, 256^3 GRF cell (mixed vs FP64 J-FFT PCG)",
            "config": {"workload": (f"{n}^3 GRF cells (ell 0.1, seed {args.seed}), contrasts "
                                    "1e3/1e4/1e5, nu 0.3, tol 1e-8; e11 timed after one warm-up "
                                    "solve; C_eff from six load cases as one group")},
            "rows": rows}


def run_sweeps(args):
    """The paper's grid-refinement sweeps (Sec. 4.1 laminate with total
    contrast 10 and 1e4, Sec. 4.2 cosine geometry with contrast 1e4 and
    infinity): the geometry G_p refined onto T_n for n = 16 ... 512 and
    p = 4 ... n (powers of two), linear triangles, C = rho C0 (lambda0 = 2/3,
    mu0 = 1/2), macro gradient (1, 1, 1), u0 = 0, ||r||^2 <= 1e-10, at most
    999 iterations (the cap of the paper's figures), with the Green, Jacobi
    and Green-Jacobi preconditioners.  The paper's own grids reach n = 1024;
    the library's FFT lengths stop at 512.  The counts stand beside the
    trends the paper states in words (its figures are not in the text)."""
    import torch

    import jfft_inputs as ji
    import paper_2508_02613_amd as pkg

    lam0, mu0 = 2.0 / 3.0, 0.5
    macro = np.array([1.0, 1.0, 1.0])
    kinds = {"laminate_chi1e1": lambda p: ji.laminate_field((p, p), 10.0),
             "laminate_chi1e4": lambda p: ji.laminate_field((p, p), 1e4),
             "cosine_chi_inf": lambda p: ji.cosine_void_field(p, None),
             "cosine_chi1e4": lambda p: ji.cosine_void_field(p, 1e4)}
    pcs = {"green": pkg.PC_GREEN, "jacobi": pkg.PC_JACOBI, "green_jacobi": pkg.PC_GREEN_JACOBI}
    ns = [16, 32, 64, 128, 256, 512]
    stream = torch.cuda.Stream()
    tables = {k: {name: {} for name in pcs} for k in kinds}
    total_it, total_dofit = 0, 0.0
    t0 = time.perf_counter()
    for n in ns:
        for name, pc in pcs.items():
            cell = pkg.Cell((n, n), pc=pc, element="tri", stream=stream)
            cell.set_stop_rule(absolute=True)
            if args.graph:
                cell.set_graph_iterations(args.graph)
            for kind, geo in kinds.items():
                row = {}
                p = 4
                while p <= n:
                    E = ji.refine_geometry(geo(p), n)
                    cell.set_material(E, lame=(lam0, mu0))
                    _, _, rep, _ = cell.solve(macro, tol=1e-10, maxit=999)
                    row[str(p)] = rep.iters if rep.status == "ok" else f">={rep.iters}"
                    total_it += rep.iters
                    total_dofit += 2.0 * n * n * rep.iters
                    p *= 2
                tables[kind][name][str(n)] = row
            cell.close()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"metric": "PCG iterations on the paper's grid-refinement sweeps (Sec. 4.1 laminate, "
                      "Sec. 4.2 cosine with voids)",
            "unit": "iterations", "data": "synthetic (the paper's density formulas)",
            "config": {"workload": "2D periodic cell, linear triangles, C = rho C0 (lambda0 2/3, "
                                   "mu0 1/2), macro (1, 1, 1), u0 = 0, ||r||^2 <= 1e-10, cap 999; "
                                   "geometry G_p refined onto T_n", "n": ns, "p": "4 .. n"},
            "tables": tables, "solves_wall_s": wall, "total_iterations": total_it,
            "dof_it_per_s": total_dofit / wall,
            "note": "iteration tables: tables[geometry][preconditioner][n][p]; '>=999' marks "
                    "the cap"}


def run_powerlaw(args):
    """Nonlinear example of Sec. 4: n^3 nodes (voxels of unit edge), 8
    spherical linear inclusions (radius 0.15 of the cell, seeded centres; the
    paper does not give its geometry) in the power-law matrix (K = 2, sigma0 =
    0.5, eps0 = 0.1, n = 5; inclusions K = 2, mu = 1/2), macro shear
    e6 = 0.05 sqrt2 in one load step, Newton to ||f|| < 1e-5 with PCG to
    ||r||^2 <= 1e-10 (the rules of Sec. 4).  One step = one whole Newton
    solve (set the material, every Newton step with its Algorithm 2 diagonal
    and PCG solve, sigma_bar).  Headline: Green-Jacobi in mixed precision
    (FP32 tangent solves refined against the FP64 tangent residual); FP64
    Green-Jacobi and FP64 Green beside it (PCG iterations per Newton step,
    the figure of Sec. 4)."""
    import torch

    import jfft_inputs as ji
    import paper_2508_02613_amd as pkg

    n = args.pl_n
    shape = (n, n, n)
    phase = 1.0 - ji.spherical_inclusions(shape, 8, 0.15, seed=args.seed)
    macro = np.array([0, 0, 0, 0, 0, 0.05 * np.sqrt(2)])
    L = (float(n),) * 3
    N = phase.size
    dofs = 3 * N
    ph = torch.from_numpy(phase).to("cuda")
    stream = torch.cuda.Stream()
    runs = {}
    for name, pc, prec in (("green_jacobi", pkg.PC_GREEN_JACOBI, pkg.FP64),
                           ("green", pkg.PC_GREEN, pkg.FP64),
                           ("mixed_green_jacobi", pkg.PC_GREEN_JACOBI, pkg.MIXED)):
        cell = pkg.Cell(shape, precision=prec, pc=pc, lengths=L, stream=stream)
        if args.graph:
            cell.set_graph_iterations(args.graph)
        cell.set_stop_rule(absolute=True)
        u = torch.empty((3,) + shape, dtype=torch.float64, device="cuda")

        def step():
            cell.set_material_powerlaw(ph)
            return cell.solve_newton(macro, newton_tol=1e-5, pcg_tol=1e-10, max_newton=20,
                                     maxit=20000, out=u)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = []
        for _ in range(args.steps):
            _, sbar, rep = step()
            reps.append(rep)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        stats = None
        if name != "green":
            cell.reset_timing()
            cell.enable_timing(True)
            step()
            torch.cuda.synchronize()
            stats = cell.kernel_stats()
            cell.enable_timing(False)
        cell.close()
        runs[name] = {"wall_s": wall, "reps": reps, "sigma_bar": sbar, "stats": stats}
    M = runs["mixed_green_jacobi"]  # headline: mixed precision, as the linear headline
    F = runs["green_jacobi"]
    G = runs["green"]

    def iters(run):
        return sum(sum(r.pcg_iters) for r in run["reps"])

    n_matrix = int(np.count_nonzero(phase > 0.5))  # elements of the power-law matrix

    def roofline(run, prec):
        # tangent CG stiffness kernel: FP32 in the mixed path's inner solves
        launches, tot_ms = run["stats"]["stiffness_cg"]
        rb = 4 if prec == "f32" else 8
        bytes_launch = algorithmic_bytes("stiffness_cg_tangent", 3, N, n, rb)
        flops_launch = TANGENT_FLOPS_MATRIX * n_matrix + TANGENT_FLOPS_INCLUSION * (N - n_matrix)
        avg_ms = tot_ms / launches
        gbs = bytes_launch / (avg_ms * 1e-3) / 1e9
        tf = flops_launch / (avg_ms * 1e-3) / 1e12
        peak = FP32_VECTOR_PEAK_TFLOPS if prec == "f32" else FP64_VECTOR_PEAK_TFLOPS
        return {"bound": "alu", "kernel": f"stiffness_cg (power-law tangent, {prec.upper()})",
                "achieved": tf, "peak": peak, "unit": "TFLOP/s", "frac": tf / peak,
                "traffic": load_traffic(f"powerlaw_{n}", f"stiffness_cg_{prec}"),
                "algorithmic_flops_per_launch": flops_launch,
                "flops_per_element": {"matrix": TANGENT_FLOPS_MATRIX,
                                      "inclusion": TANGENT_FLOPS_INCLUSION},
                "peak_basis": ("FP32 vector without packed math" if prec == "f32"
                               else "FP64 vector"),
                "hbm_achieved_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
                "avg_ms": avg_ms, "launches": launches,
                "algorithmic_bytes_per_launch": bytes_launch,
                "measured": "HIP events on the cell's stream around every launch, one "
                            "further Newton solve with direct launches"}

    def newton(run):
        r = run["reps"][-1]
        return {"steps": r.steps, "pcg_iters": r.pcg_iters, "res": r.res,
                "ms_per_solve": 1e3 * run["wall_s"] / args.steps,
                "value": dofs * iters(run) / run["wall_s"]}

    line = {
        "metric": "DOF·iterations/s (power-law Newton, J-FFT PCG on the tangent)",
        "value": dofs * iters(M) / M["wall_s"], "unit": "DOF·it/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * M["wall_s"] / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": (f"nonlinear example {n}^3 nodes, voxels of unit edge, 8 "
                                f"spherical linear inclusions (radius 0.15, seed {args.seed}) in a "
                                "power-law matrix (K 2, sigma0 0.5, eps0 0.1, n 5), macro shear "
                                "e6 0.05 sqrt2, Newton to ||f|| < 1e-5, Green-Jacobi PCG to "
                                "||r||^2 <= 1e-10; mixed precision: FP32 tangent solves refined "
                                "against the FP64 tangent residual"),
                   "n": n, "dofs": dofs, "inclusion_fraction": float(1.0 - phase.mean()),
                   "graph_iterations": args.graph},
        "newton": {"mixed_green_jacobi": newton(M),
                   "green_jacobi": newton(F),
                   "green": dict(newton(G), sigma_bar_rel_diff_vs_gj=float(
                       np.abs(G["sigma_bar"] - F["sigma_bar"]).max()
                       / np.abs(F["sigma_bar"]).max()))},
        "sigma_bar": [float(v) for v in M["sigma_bar"]],
        "sigma_bar_rel_diff_mixed_vs_fp64": float(
            np.abs(M["sigma_bar"] - F["sigma_bar"]).max() / np.abs(F["sigma_bar"]).max()),
        "roofline": roofline(M, "f32"),
        "fp64": {"value": dofs * iters(F) / F["wall_s"],
                 "ms_per_step": 1e3 * F["wall_s"] / args.steps,
                 "roofline": roofline(F, "f64"),
                 "kernels_ms_per_solve": {k: v[1] for k, v in sorted(F["stats"].items())}},
        "kernels_ms_per_solve": {k: v[1] for k, v in sorted(M["stats"].items())},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline_powerlaw(args.seed)
    return line


def run_tri(args):
    """2D linear triangles (two per pixel, the paper's own 2D element).
    Throughput: a group of B plane-strain cells of 512^2 nodes (the largest
    FFT length of the library) with smooth GRF moduli (ell 0.1, contrast
    1e4, seeds 0..B-1), nu 0.3, macro e11, Green-Jacobi PCG to relative
    residual 1e-8, mixed precision as the headline (FP64 beside it); one step
    = set the materials and solve the group.  Trend: the motivating example
    of Sec. 1 at 256^2 (soft disc 1e-4, radius 0.25, i filter passes) with
    the absolute rule ||r||^2 <= 1e-10, Green vs Green-Jacobi iterations."""
    import torch

    import jfft_inputs as ji
    import paper_2508_02613_amd as pkg

    n, B = 512, args.tri_cells
    shape = (n, n)
    N = n * n
    Es = np.stack([ji.grf_field(shape, 1e4, seed=s, ell=0.1) for s in range(B)])
    macros = np.tile(np.array([1.0, 0.0, 0.0]), (B, 1))
    Ed = torch.from_numpy(Es).to("cuda")
    stream = torch.cuda.Stream()
    runs = {}
    for name, prec in (("mixed", pkg.MIXED), ("fp64", pkg.FP64)):
        grp = pkg.Cell(shape, precision=prec, pc=pkg.PC_GREEN_JACOBI, stream=stream, batch=B,
                       element="tri")
        if args.graph:
            grp.set_graph_iterations(args.graph)
        u = torch.empty((B, 2) + shape, dtype=torch.float64, device="cuda")

        def step():
            grp.set_material(Ed, nu=0.3)
            return grp.solve_batch(macros, tol=1e-8, maxit=20000, out=u)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = 0
        for _ in range(args.steps):
            _, sbar, reps, _ = step()
            its += sum(r.iters for r in reps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        grp.reset_timing()
        grp.enable_timing(True)
        _, _, reps_ev, _ = step()
        torch.cuda.synchronize()
        stats = grp.kernel_stats()
        grp.enable_timing(False)
        grp.close()
        runs[name] = {"wall_s": wall, "iters": its, "reps": reps, "stats": stats, "sbar": sbar,
                      "ev_iters": sum(r.iters for r in reps_ev)}
    R = runs["mixed"]
    dofs = 2 * N * B
    value = 2 * N * R["iters"] / R["wall_s"]
    # stiffness roofline: algorithmic bytes of one cell-iteration times the
    # cell-iterations of the event-timed step, over the kernel's event time
    launches, tot_ms = R["stats"]["stiffness_cg"]
    cell_bytes = algorithmic_bytes("stiffness_cg", 2, N, n, 4)
    achieved = cell_bytes * R["ev_iters"] / (tot_ms * 1e-3) / 1e9
    # the motivating example's trend
    trend = []
    for filters in (0, 1, 2, 4, 8, 16, 32):
        E = ji.filtered_inclusion_field(256, filters)
        row = {"filters": filters}
        for pname, pc in (("green", pkg.PC_GREEN), ("green_jacobi", pkg.PC_GREEN_JACOBI)):
            cell = pkg.Cell((256, 256), pc=pc, element="tri", stream=stream)
            cell.set_stop_rule(absolute=True)
            cell.set_material(E, nu=0.3)
            _, _, rep, _ = cell.solve(np.array([1.0, 0.0, 0.0]), tol=1e-10, maxit=20000)
            cell.close()
            row[pname] = rep.iters
            row[pname + "_loop_ms"] = rep.loop_ms
        trend.append(row)
    F = runs["fp64"]
    line = {
        "metric": "DOF·iterations/s (2D linear triangles, J-FFT PCG, group of 512² cells)",
        "value": value, "unit": "DOF·it/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * R["wall_s"] / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": (f"{B} 2D plane-strain cells of 512^2 nodes, two linear "
                                "triangles per pixel, GRF E (ell 0.1, contrast 1e4, seeds "
                                f"0..{B - 1}), nu 0.3, macro e11, Green-Jacobi PCG to relative "
                                "residual 1e-8, mixed precision, one group on one stream"),
                   "cells": B, "n": n, "dofs": dofs, "graph_iterations": args.graph},
        "iters_per_cell": R["iters"] / (args.steps * B),
        "max_rel_res_true": max(r.rel_res_true for r in R["reps"]),
        "fp64": {"value": 2 * N * F["iters"] / F["wall_s"],
                 "ms_per_step": 1e3 * F["wall_s"] / args.steps,
                 "iters_per_cell": F["iters"] / (args.steps * B),
                 "sigma_bar_rel_diff_vs_mixed": float(np.abs(F["sbar"] - R["sbar"]).max()
                                                      / np.abs(F["sbar"]).max())},
        "roofline": {"bound": "hbm", "kernel": "stiffness_cg (2D triangles, FP32)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": load_traffic(f"tri_mixed_{n}x{B}", "stiffness_cg"),
                     "avg_ms": tot_ms / launches, "launches": launches,
                     "cell_iterations": R["ev_iters"],
                     "algorithmic_bytes_per_cell_iteration": cell_bytes,
                     # a launch with every cell active (what `traffic` measures)
                     "algorithmic_bytes_per_launch": cell_bytes * B,
                     "measured": "HIP events on the group's stream around every launch, one "
                                 "further step with direct launches"},
        "kernels_ms_per_step": {k: v[1] for k, v in sorted(R["stats"].items())},
        "trend_motivating_example_256": trend,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline_tri(reps=100)
    return line


def run_topopt(args):
    """Phase-field topology optimisation of Sec. 4 (eq. aim_fun): n^2 nodes,
    two linear triangles per pixel, C = rho C0 (lambda0 2/3, mu0 1/2), three
    unit load cases, targets K 0.025 and mu 0.15, eta 0.01, rho_0 uniform in
    [0, 1] (seed), projected L-BFGS (memory 10) with every solve from u = 0
    by Green-Jacobi PCG to relative residual 1e-8, FP64.  One step = the
    whole run of --topo-iters L-BFGS steps.  Beside it: the PCG iterations
    of Green, Jacobi and Green-Jacobi on the start density and on the last
    accepted one (the comparison of the paper's figure)."""
    import torch

    import paper_2508_02613_amd as pkg

    n, K = args.topo_n, args.topo_iters
    shape = (n, n)
    lam0, mu0 = 2.0 / 3.0, 0.5
    Kt, mut = 0.025, 0.15
    lt = Kt - 2.0 * mut / 3.0
    T = np.array([[lt + 2 * mut, lt, 0.0], [lt, lt + 2 * mut, 0.0], [0.0, 0.0, 2 * mut]])
    rho0 = np.random.default_rng(args.seed).uniform(0.0, 1.0, shape)
    stream = torch.cuda.Stream()
    grp = pkg.Cell(shape, precision=pkg.FP64, pc=pkg.PC_GREEN_JACOBI, stream=stream, batch=3,
                   element="tri")
    if args.graph:
        grp.set_graph_iterations(args.graph)
    if args.fused_control >= 0:
        grp.set_tunables(fused_control=args.fused_control)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rho, out = grp.topopt_lbfgs(rho0, T, K, eta=0.01, tol=1e-8, maxit=200000)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    grp.close()
    cmp = {}
    for label, r in (("rho_0", rho0), (f"rho_{out['steps']}", rho)):
        row = {}
        for pname, pc in (("green", pkg.PC_GREEN), ("jacobi", pkg.PC_JACOBI),
                          ("green_jacobi", pkg.PC_GREEN_JACOBI)):
            g = pkg.Cell(shape, precision=pkg.FP64, pc=pc, stream=stream, batch=3, element="tri")
            if args.graph:
                g.set_graph_iterations(args.graph)
            f, _, its = g.topopt_eval(r, T, eta=0.01, tol=1e-8, maxit=200000)
            g.close()
            row[pname] = its
        rr = r.cpu().numpy() if hasattr(r, "cpu") else r
        row["contrast"] = float(rr.max() / rr.min()) if rr.min() > 0 else None
        cmp[label] = row
    # roofline: one further evaluation at the start density with HIP events
    # around every launch (direct launches); the dominant kernel by time
    g = pkg.Cell(shape, precision=pkg.FP64, pc=pkg.PC_GREEN_JACOBI, stream=stream, batch=3,
                 element="tri")
    g.enable_timing(True)
    _, _, ev_its = g.topopt_eval(rho0, T, eta=0.01, tol=1e-8, maxit=200000)
    torch.cuda.synchronize()
    stats = g.kernel_stats()
    g.enable_timing(False)
    g.close()
    dom = max((k for k in stats if algorithmic_bytes(k, 2, n * n, n, 8)), key=lambda k: stats[k][1])
    launches, tot_ms = stats[dom]
    cell_bytes = algorithmic_bytes(dom, 2, n * n, n, 8)
    achieved = cell_bytes * sum(ev_its) / (tot_ms * 1e-3) / 1e9
    dofs = 2 * n * n
    per_step = [max(i) for i in out["iters"]]
    line = {
        "metric": "DOF·iterations/s (phase-field topology optimisation, J-FFT PCG solves)",
        "value": dofs * out["pcg_total"] / wall, "unit": "DOF·it/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": 1e3 * wall, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": (f"{n}^2 nodes, two linear triangles per pixel, C = rho C0 "
                                "(lambda0 2/3, mu0 1/2), 3 unit load cases, targets K 0.025 mu "
                                f"0.15, eta 0.01, rho_0 ~ U(0,1) seed {args.seed}, projected "
                                f"L-BFGS (m 10) for {K} steps, Green-Jacobi PCG to 1e-8 from u = 0, "
                                "FP64"),
                   "n": n, "lbfgs_steps": K, "graph_iterations": args.graph,
                   "fused_control": args.fused_control},
        "lbfgs": {"steps": out["steps"], "evals": out["evals"], "pcg_total": out["pcg_total"],
                  "f": out["f"], "gnorm": out["gnorm"],
                  "pcg_iters_per_step_max_over_load_cases": per_step,
                  "ms_per_step": 1e3 * wall / max(out["steps"], 1)},
        "pcg_iters_by_preconditioner": cmp,
        "roofline": {"bound": "hbm", "kernel": f"{dom} (2D triangles, FP64, three load cases)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "avg_ms": tot_ms / launches, "launches": launches,
                     "cell_iterations": sum(ev_its),
                     "algorithmic_bytes_per_cell_iteration": cell_bytes,
                     "algorithmic_bytes_per_launch": 3 * cell_bytes,
                     "measured": "HIP events on the group's stream around every launch of one "
                                 "further evaluation at rho_0 (direct launches)",
                     "kernels_ms": {k: v[1] for k, v in sorted(stats.items())}},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline_tri(n=n, E=rho0, lame=(lam0, mu0), cells=3, reps=200)
    return line


def cpu_baseline_tri(n=512, E=None, lame=None, cells=1, reps=1):
    """The triangle oracle timed on one PCG iteration's operators (element
    loop K p, Green-Jacobi preconditioner with the naive separable DFT, dots
    and updates), reps times per cell: by default once on one 512^2 GRF cell
    of the group; the topology workload passes its density (C = rho C0) and
    its three load cases."""
    import jfft_inputs as ji
    import oracle
    from oracle import triangles as tri

    if E is None:
        E = ji.grf_field((n, n), 1e4, seed=0, ell=0.1)
    lam, mu = oracle.lame_from_nu(0.3) if lame is None else lame
    rng = np.random.default_rng(0)
    G = np.zeros((2, 2, n, n), dtype=complex)
    G[0, 0] = 1.0
    diag = np.ones((2, n, n))
    tk = tm = tv = 0.0
    for _ in range(cells * reps):
        p = rng.standard_normal((2, n, n))
        t0 = time.perf_counter()
        q = tri.stiffness(E, p, lam, mu)
        t1 = time.perf_counter()
        z, _ = oracle.precond(oracle.PC_GREEN_JACOBI, q, diag=diag, G=G)
        t2 = time.perf_counter()
        a = float((p * q).sum())
        p += a * z
        t3 = time.perf_counter()
        tk, tm, tv = tk + t1 - t0, tm + t2 - t1, tv + t3 - t2
    per_iter = (tk + tm + tv) / (cells * reps)
    what = "cell" if cells == 1 else f"load case, each of {cells}"
    count = "one PCG iteration" if reps == 1 else f"{reps} PCG iterations"
    return {"value": 2 * n * n / per_iter, "unit": "DOF·it/s", "cores": oracle.num_threads(), "cpu": host_cpu(),
            "kind": "oracle",
            "sample": (f"{count} of the triangle oracle per {n}^2 {what} (element loop "
                       f"{tk:.2f} s, Green-Jacobi M^-1 with naive DFT {tm:.2f} s, "
                       f"dots/axpys {tv:.2f} s in total); set-up excluded"),
            "seconds_per_iteration": per_iter}


def cpu_baseline_powerlaw(seed):
    """The power-law oracle timed on one PCG iteration's operators (tangent
    K(u) p by its vectorised element loop, Green-Jacobi preconditioner with
    the naive separable DFT, dots and updates) on the bench's 200^3 cell
    (about 20 s with 16 threads)."""
    import jfft_inputs as ji
    import oracle
    from oracle import powerlaw as pl

    n = 200
    shape = (n, n, n)
    phase = 1.0 - ji.spherical_inclusions(shape, 8, 0.15, seed=seed)
    rng = np.random.default_rng(0)
    u = 0.01 * rng.standard_normal((3,) + shape)
    p = rng.standard_normal((3,) + shape)
    macro = np.array([0, 0, 0, 0, 0, 0.05 * np.sqrt(2)])
    G = np.zeros((3, 3) + shape, dtype=complex)
    G[0, 0] = 1.0
    diag = np.ones((3,) + shape)
    L = (float(n),) * 3
    t0 = time.perf_counter()
    q = pl.tangent_op(u, p, macro, phase, pl.PowerLaw(), L)
    t1 = time.perf_counter()
    z, _ = oracle.precond(oracle.PC_GREEN_JACOBI, q, diag=diag, G=G)
    t2 = time.perf_counter()
    a = float((p * q).sum())
    p += a * z
    t3 = time.perf_counter()
    per_iter = t3 - t0
    return {"value": 3 * phase.size / per_iter, "unit": "DOF·it/s",
            "cores": oracle.num_threads(), "cpu": host_cpu(), "kind": "oracle",
            "sample": (f"one PCG iteration of the power-law oracle at {n}^3 (tangent element "
                       f"loop {t1 - t0:.1f} s, Green-Jacobi M^-1 with naive DFT {t2 - t1:.1f} s, "
                       f"dots/axpys {t3 - t2:.1f} s); Newton set-up excluded"),
            "seconds_per_iteration": per_iter}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU: --gpus {args.gpus} is not supported (the "
              "solver runs each cell or cell group on one MI355X; there is no multi-GPU path)",
              file=sys.stderr)
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe:
        copy_probe()
        return
    if args.workload == "simp2d":
        print(json.dumps(run_simp2d(args)), flush=True)
        return
    if args.workload == "contrast":
        print(json.dumps(run_contrast_sweep(args)), flush=True)
        return
    if args.workload == "powerlaw":
        print(json.dumps(run_powerlaw(args)), flush=True)
        return
    if args.workload == "tri":
        print(json.dumps(run_tri(args)), flush=True)
        return
    if args.workload == "topopt":
        print(json.dumps(run_topopt(args)), flush=True)
        return
    if args.workload == "sweeps":
        print(json.dumps(run_sweeps(args)), flush=True)
        return
    import jfft_inputs as ji

    n = args.n
    shape = (n, n, n)
    E = ji.grf_field(shape, args.contrast, seed=args.seed, ell=0.1)
    nu = 0.3
    macro = ji.unit_macro_strain(3, 0)
    tol, maxit = 1e-8, 20000
    N = E.size
    dofs = 3 * N
    workload = (f"3D periodic cell {n}^3 nodes, trilinear hex Q1 with 8 Gauss points, "
                f"smooth Gaussian-random-field E (ell 0.1, contrast {args.contrast:g}, seed "
                f"{args.seed}), nu 0.3, macro strain e11, Green-Jacobi (J-FFT) PCG to "
                f"relative residual 1e-8")
    results = {}
    if not args.no_mixed:
        results["mixed"] = run_gpu(args, "mixed", E, nu, macro, tol, maxit)
    if not args.no_fp64:
        results["fp64"] = run_gpu(args, "fp64", E, nu, macro, tol, maxit)
    head = "mixed" if "mixed" in results else "fp64"
    R = results[head]
    value = dofs * R["iters"] / R["wall_s"]
    ms_per_step = 1e3 * R["wall_s"] / args.steps

    # roofline of the dominant kernel (largest total event time in the timed steps)
    stats = R["stats"]
    dom = max((k for k in stats if algorithmic_bytes(k, 3, N, n, 4) is not None),
              key=lambda k: stats[k][1])
    launches, tot_ms = stats[dom]
    # launches that did work: the stiffness kernel runs once per PCG iteration
    executed = R["iters"] if dom == "stiffness_cg" else None
    rb = 4 if head == "mixed" else 8
    if head == "mixed":
        rb = MIXED_KERNEL_BYTES.get(dom, 4)
    bytes_launch = algorithmic_bytes(dom, 3, N, n, rb)
    avg_ms = tot_ms / launches
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    wkey = f"{head}_{n}"
    traffic = load_traffic(wkey, dom)
    line = {
        "metric": "DOF·iterations/s (J-FFT PCG, 256³); served solves/s + p99 latency",
        "value": value,
        "unit": "DOF·it/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": workload, "n": n, "dofs": dofs, "precision": head,
                   "preconditioner": "green_jacobi", "contrast": args.contrast, "tol": tol,
                   "graph_iterations": args.graph},
        "iters_per_step": R["iters"] / args.steps,
        "outer_sweeps": R["reps"][-1].outer,
        "rel_res_true": R["reps"][-1].rel_res_true,
        "loop_ms": R["reps"][-1].loop_ms,
        "time_to_solution_ms": R["reps"][-1].loop_ms,
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "avg_ms": avg_ms, "launches": launches,
                     "launches_with_work": executed,
                     "algorithmic_bytes_per_launch": bytes_launch,
                     "measured": (f"HIP events on the cell's stream around every launch, over "
                                  f"{args.steps} further steps of the same workload "
                                  f"({1e3 * R['events_wall_s'] / args.steps:.1f} ms/step with "
                                  f"the events, direct launches)")},
        "kernels_ms_per_step": {k: v[1] / args.steps for k, v in sorted(stats.items())},
    }
    if "fp64" in results and head != "fp64":
        F = results["fp64"]
        line["fp64"] = {"value": dofs * F["iters"] / F["wall_s"],
                        "ms_per_step": 1e3 * F["wall_s"] / args.steps,
                        "iters_per_step": F["iters"] / args.steps,
                        "rel_res_true": F["reps"][-1].rel_res_true,
                        "loop_ms": F["reps"][-1].loop_ms,
                        "time_to_solution_ms": F["reps"][-1].loop_ms,
                        "sigma_bar_rel_diff_vs_mixed": float(
                            np.abs(F["sigma_bar"] - R["sigma_bar"]).max()
                            / np.abs(F["sigma_bar"]).max()),
                        "kernels_ms_per_step": {k: v[1] / args.steps
                                                for k, v in sorted(F["stats"].items())}}
        line["time_to_solution_speedup_vs_fp64"] = F["reps"][-1].loop_ms / R["reps"][-1].loop_ms
    if head == "mixed":
        line["mixed_restarted"] = run_restarted(args, E, nu, macro, tol, maxit)
    if not args.no_serve:
        line["serving"] = run_serving(args)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(E, macro, nu)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
