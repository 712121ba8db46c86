"""How far rounding moves the oracle's own stopping iteration: the window a
GPU iteration count is held to.

Two FP64 PCG programs of the same method (different summation orders, an FFT
against a naive DFT, a closed form against Algorithm 2's probing for diag(K))
round every operator application and every inner product differently.  CG
amplifies such differences, and the accuracy of the inner products shifts
the stop systematically: the oracle's serial sums in index order carry an
error that grows with the number of terms, a tree reduction (as on the GPU)
or Dot2 much less, and the more accurate runs stop earlier at tight
tolerances.  Instead of a heuristic slack, the oracle is run ten times, five
with its plain serial inner products and five with Dot2 (inner products as
if in twice the working precision): on the input; on inputs changed by one
unit in the last place (f scaled by 1 + 2^-52 or 1 - 2^-52; E moved by one
ulp per element); and with its rounding-difference model on (every entry of
each K p and M^-1 r result moved by one ulp in a seeded direction).  The GPU
count must lie in [min - 1, max + 1] of those ten counts.
"""
from __future__ import annotations

import jfft_inputs as ji

ULP = 2.0 ** -52


def perturbed_inputs(E, f):
    """(name, E', f', noise_seed, dot_mode) of the ten oracle runs (f' None:
    assemble from E'; dot_mode 0 serial sums, 1 Dot2)."""
    return [("unperturbed", E, None, 0, 0),
            ("f*(1+2^-52)", E, f * (1 + ULP), 0, 0),
            ("E ulp seed 1", ji.ulp_perturbed(E, 1), None, 0, 0),
            ("operator ulp noise seed 1", E, None, 1, 0),
            ("operator ulp noise seed 2", E, None, 2, 0),
            ("Dot2", E, None, 0, 1),
            ("Dot2, f*(1-2^-52)", E, f * (1 - ULP), 0, 1),
            ("Dot2, E ulp seed 2", ji.ulp_perturbed(E, 2), None, 0, 1),
            ("Dot2, operator ulp noise seed 3", E, None, 3, 1),
            ("Dot2, operator ulp noise seed 4", E, None, 4, 1)]


def iteration_window(solve, E, f):
    """Run `solve(E', f', noise_seed, dot_mode)` on the ten variants; it
    returns an object with `.iters` (or an int).  Returns (lo, hi, counts,
    results) with [lo, hi] = [min - 1, max + 1] of the counts; results[0] is
    the unperturbed run with plain arithmetic."""
    results = [solve(Ev, fv, ns, dm) for _, Ev, fv, ns, dm in perturbed_inputs(E, f)]
    counts = [int(getattr(r, "iters", r)) for r in results]
    return min(counts) - 1, max(counts) + 1, counts, results
