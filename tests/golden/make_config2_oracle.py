"""Write tests/golden/config2_oracle.json: the oracle's results on the 64^3
effective-stiffness workload (periodic Gaussian-random-field cell, contrast
1e4, correlation length 0.1, nu = 0.3, the six unit macro strains, GRF seeds
0-2, Green-Jacobi PCG, FP64), which are too slow to recompute inside a GPU
test run.

Calls only the oracle (and the seeded input generators).  For every case:

* the tight solve (relative residual 1e-12, close to the exact discrete
  solution u*): iteration count, sigma_bar, u* at sampled nodes and its
  projections on seeded Gaussian sketch vectors;
* thirteen solves at the configuration's tolerance 1e-8, the rounding
  variants of tests/oracle_spread.py: the C loop five times with serial
  inner products and five with Dot2 (on the input, on inputs changed by one
  ulp, with the one-ulp noise model), and its Python loop with numpy's FFT
  as the transform step three times.  For each:
  iteration count, sigma_bar, true residual and the exact relative distance
  ||u - u*|| / ||u*||.  The spread of these counts is how far rounding moves
  the oracle's own stopping iteration; the unperturbed solve's sketch
  projections are stored too.

Usage: python tests/golden/make_config2_oracle.py [--seeds 0 1 2] [--cases 0 1 2 3 4 5]
The file is rewritten after every case, so an interrupted run keeps what it
finished; on the next run a case missing some of the variants gets them
added (after its tight solve is repeated for u*).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import jfft_inputs as ji  # noqa: E402
import oracle  # noqa: E402
from oracle_spread import c_oracle, perturbed_inputs  # noqa: E402

OUT = os.path.join(HERE, "config2_oracle.json")
N = 64
CONTRAST = 1e4
ELL = 0.1
NU = 0.3
TOL = 1e-8
TOL_TIGHT = 1e-12
MAXIT = 5000
N_SKETCH = 24
SKETCH_SEED = 20250802
N_SAMPLES = 128
SAMPLE_SEED = 2613


def sketch(u, shape):
    return [float(np.dot(w.ravel(), u.ravel()))
            for w in ji.sketch_vectors(shape, N_SKETCH, SKETCH_SEED)]


def run_case(seed, g, case=None):
    """Compute a case, or (case given) add the variants it lacks."""
    lam, mu = oracle.lame_from_nu(NU)
    shape = (N, N, N)
    E = ji.grf_field(shape, CONTRAST, seed=seed, ell=ELL)
    macro = ji.unit_macro_strain(3, g)
    f = oracle.rhs(E, macro, lam, mu)
    t0 = time.time()
    tight = oracle.solve(E, macro, lam, mu, pc=oracle.PC_GREEN_JACOBI, tol=TOL_TIGHT, maxit=MAXIT)
    ustar = tight.u
    if case is not None:
        assert tight.iters == case["tight"]["iters"]  # the oracle is deterministic
        have = {r["input"] for r in case["runs"]}
        solve = c_oracle(macro, lam, mu, pc=oracle.PC_GREEN_JACOBI, tol=TOL, maxit=MAXIT)
        nrm = case["tight"]["u_norm"]
        for name, Ev, fv, ns, dm, tr in perturbed_inputs(E, f):
            if name in have:
                continue
            r = solve(Ev, fv, ns, dm, tr)
            case["runs"].append({"input": name, "iters": r.iters, "status": r.status,
                                 "relres_true": r.relres_true, "sigma_bar": r.sigma_bar.tolist(),
                                 "err_vs_tight": float(np.linalg.norm(r.u - ustar) / nrm)})
            print(f"  seed {seed} case {g} {name}: iters {r.iters} (added)", flush=True)
        case["seconds"] = case.get("seconds", 0.0) + time.time() - t0
        return case
    nrm = float(np.linalg.norm(ustar))
    nodes = ji.sample_nodes(N ** 3, N_SAMPLES, SAMPLE_SEED)
    ud = ustar.reshape(3, -1)
    case = {
        "seed": seed, "load_case": g,
        "tight": {
            "tol": TOL_TIGHT, "iters": tight.iters, "status": tight.status,
            "relres_true": tight.relres_true, "sigma_bar": tight.sigma_bar.tolist(),
            "u_norm": nrm, "nodes": nodes.tolist(),
            "u_nodes": [ud[c, nodes].tolist() for c in range(3)],
            "sketch": sketch(ustar, ustar.shape),
        },
        "runs": [],
    }
    solve = c_oracle(macro, lam, mu, pc=oracle.PC_GREEN_JACOBI, tol=TOL, maxit=MAXIT)
    for name, Ev, fv, ns, dm, tr in perturbed_inputs(E, f):
        r = solve(Ev, fv, ns, dm, tr)
        run = {"input": name, "iters": r.iters, "status": r.status,
               "relres_true": r.relres_true, "sigma_bar": r.sigma_bar.tolist(),
               "err_vs_tight": float(np.linalg.norm(r.u - ustar) / nrm)}
        if name == "unperturbed":
            run["sketch"] = sketch(r.u, r.u.shape)
        case["runs"].append(run)
        print(f"  seed {seed} case {g} {name}: iters {r.iters} err_vs_tight "
              f"{run['err_vs_tight']:.2e}", flush=True)
    case["seconds"] = time.time() - t0
    return case


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seeds", type=int, nargs="*", default=[0, 1, 2])
    ap.add_argument("--cases", type=int, nargs="*", default=list(range(6)))
    args = ap.parse_args()
    data = {"workload": {"n": N, "contrast": CONTRAST, "ell": ELL, "nu": NU, "tol": TOL,
                         "tol_tight": TOL_TIGHT, "maxit": MAXIT, "preconditioner": "green_jacobi",
                         "n_sketch": N_SKETCH, "sketch_seed": SKETCH_SEED,
                         "n_samples": N_SAMPLES, "sample_seed": SAMPLE_SEED},
            "cases": []}
    if os.path.exists(OUT):
        with open(OUT) as fh:
            data = json.load(fh)
    nvar = len(perturbed_inputs(np.ones(1), np.ones(1)))
    for seed in args.seeds:
        for g in args.cases:
            old = [c for c in data["cases"] if (c["seed"], c["load_case"]) == (seed, g)]
            if old and len(old[0]["runs"]) >= nvar:
                continue
            print(f"seed {seed} load case {g}", flush=True)
            if old:
                run_case(seed, g, old[0])
            else:
                data["cases"].append(run_case(seed, g))
            data["cases"].sort(key=lambda c: (c["seed"], c["load_case"]))
            with open(OUT + ".tmp", "w") as fh:
                json.dump(data, fh, indent=0)
            os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main()
