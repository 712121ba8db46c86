"""Write tests/golden/config2_oracle.json: the oracle's results on the 64^3
effective-stiffness workload (periodic Gaussian-random-field cell, contrast
1e4, correlation length 0.1, nu = 0.3, the six unit macro strains, GRF seeds
0-2, Green-Jacobi PCG, FP64), which are too slow to recompute inside a GPU
test run.

Calls only the oracle (and the seeded input generators).  For every case:

* the tight solve (relative residual 1e-12, close to the exact discrete
  solution u*): iteration count, sigma_bar, u* at sampled nodes and its
  projections on seeded Gaussian sketch vectors;
* ten solves at the configuration's tolerance 1e-8 (tests/oracle_spread.py):
  five with the oracle's serial inner products and five with Dot2, on the
  input, on inputs changed by one ulp (f scaled by 1 +- 2^-52, E moved by one
  ulp per element) and with the rounding-difference model (each K p and
  M^-1 r entry moved by one ulp, seeded).  For each:
  iteration count, sigma_bar, true residual and the exact relative distance
  ||u - u*|| / ||u*||.  The spread of these counts is how far rounding moves
  the oracle's own stopping iteration; the unperturbed solve's sketch
  projections are stored too.

Usage: python tests/golden/make_config2_oracle.py [--seeds 0 1 2] [--cases 0 1 2 3 4 5]
The file is rewritten after every case, so an interrupted run keeps what it
finished (finished cases are skipped on the next run).
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
from oracle_spread import perturbed_inputs  # noqa: E402

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


def run_case(seed, g):
    lam, mu = oracle.lame_from_nu(NU)
    shape = (N, N, N)
    E = ji.grf_field(shape, CONTRAST, seed=seed, ell=ELL)
    macro = ji.unit_macro_strain(3, g)
    f = oracle.rhs(E, macro, lam, mu)
    t0 = time.time()
    tight = oracle.solve(E, macro, lam, mu, pc=oracle.PC_GREEN_JACOBI, tol=TOL_TIGHT, maxit=MAXIT)
    ustar = tight.u
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
    for name, Ev, fv, ns, dm in perturbed_inputs(E, f):
        r = oracle.solve(Ev, macro, lam, mu, pc=oracle.PC_GREEN_JACOBI, tol=TOL, maxit=MAXIT, f=fv,
                         noise_seed=ns, dot_mode=dm)
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
    done = {(c["seed"], c["load_case"]) for c in data["cases"]}
    for seed in args.seeds:
        for g in args.cases:
            if (seed, g) in done:
                continue
            print(f"seed {seed} load case {g}", flush=True)
            data["cases"].append(run_case(seed, g))
            data["cases"].sort(key=lambda c: (c["seed"], c["load_case"]))
            with open(OUT + ".tmp", "w") as fh:
                json.dump(data, fh, indent=0)
            os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main()
