"""How far rounding moves the oracle's own stopping iteration: the window a
GPU iteration count is held to.

Two FP64 PCG programs of the same method (different summation orders, an FFT
against a naive DFT, a closed form against Algorithm 2's probing for diag(K))
round every operator application and every inner product differently.  CG
amplifies such differences, and the accuracy of the arithmetic shifts the
stop systematically: more accurate programs stop earlier at tight
tolerances (the oracle's serial sums in index order and its naive DFT carry
errors that grow with the number of terms, a tree reduction, Dot2 or an FFT
much smaller ones), and on spectra with few distinct eigenvalues (a
laminate of a few layers) an accurate program reaches CG's finite
termination where a less accurate one needs several more iterations.
Instead of a heuristic slack, the oracle is run thirteen times:

* its C loop, five times with its plain serial inner products and five with
  Dot2 (inner products as if in twice the working precision): on the input;
  on inputs changed by one unit in the last place (f scaled by 1 + 2^-52 or
  1 - 2^-52; E moved by one ulp per element); and with its
  rounding-difference model on (every entry of each K p and M^-1 r result
  moved by one ulp in a seeded direction);
* the same loop in Python over the same operators with numpy's FFT as the
  preconditioner's transform step (oracle.solve_py), three times: pairwise
  and correctly rounded (math.fsum) inner products, and the latter with the
  noise model on.

The GPU count must lie in [min - 1, max + 1] of those thirteen counts.
"""
from __future__ import annotations

import jfft_inputs as ji
import oracle

ULP = 2.0 ** -52


def perturbed_inputs(E, f):
    """(name, E', f', noise_seed, dot_mode, transform) of the thirteen oracle
    runs (f' None: assemble from E'; dot_mode 0 the loop's plain sums, 1
    Dot2 / math.fsum; transform "dft" the naive DFT, "fft" numpy's FFT)."""
    return [("unperturbed", E, None, 0, 0, "dft"),
            ("f*(1+2^-52)", E, f * (1 + ULP), 0, 0, "dft"),
            ("E ulp seed 1", ji.ulp_perturbed(E, 1), None, 0, 0, "dft"),
            ("operator ulp noise seed 1", E, None, 1, 0, "dft"),
            ("operator ulp noise seed 2", E, None, 2, 0, "dft"),
            ("Dot2", E, None, 0, 1, "dft"),
            ("Dot2, f*(1-2^-52)", E, f * (1 - ULP), 0, 1, "dft"),
            ("Dot2, E ulp seed 2", ji.ulp_perturbed(E, 2), None, 0, 1, "dft"),
            ("Dot2, operator ulp noise seed 3", E, None, 3, 1, "dft"),
            ("Dot2, operator ulp noise seed 4", E, None, 4, 1, "dft"),
            ("FFT transform", E, None, 0, 0, "fft"),
            ("FFT transform, fsum", E, None, 0, 1, "fft"),
            ("FFT transform, fsum, operator ulp noise seed 5", E, None, 5, 1, "fft")]


def c_oracle(macro, lam, mu, **kw):
    """Solve callable for iteration_window over the C oracle (oracle.solve;
    its transform is the naive DFT) and its Python loop (oracle.solve_py)
    for the FFT variants.  kw: pc, tol, maxit, stop_mode, u0, hist_len, ..."""
    def run(Ev, fv, ns, dm, tr):
        if tr == "dft":
            return oracle.solve(Ev, macro, lam, mu, f=fv, noise_seed=ns, dot_mode=dm, **kw)
        return oracle.solve_py(Ev, macro, lam, mu, f=fv, noise_seed=ns, dot_mode=dm,
                               transform=tr, **kw)
    return run


def iteration_window(solve, E, f):
    """Run `solve(E', f', noise_seed, dot_mode, transform)` on the thirteen
    variants; it returns an object with `.iters` (or an int).  Returns (lo,
    hi, counts, results) with [lo, hi] = [min - 1, max + 1] of the counts;
    results[0] is the unperturbed run of the C loop with plain arithmetic."""
    results = [solve(Ev, fv, ns, dm, tr) for _, Ev, fv, ns, dm, tr in perturbed_inputs(E, f)]
    counts = [int(getattr(r, "iters", r)) for r in results]
    return min(counts) - 1, max(counts) + 1, counts, results
