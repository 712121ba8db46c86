"""GPU parity on the paper's two grid-refinement sweeps (Sec. 4.1 laminate,
Sec. 4.2 cosine geometry with voids): the geometry G_p (p pixels per axis)
refined onto the discretisation T_n (n nodes per axis, n >= p), the paper's
element (two linear triangles per pixel), its reference law C0 (lambda0 =
2/3, mu0 = 1/2) scaled by the density, macro gradient (1, 1, 1), u0 = 0, the
absolute stopping rule ||r||^2 <= 1e-10 and the cap of 999 iterations of its
figures.  Every GPU iteration count (Green, Jacobi, Green-Jacobi) must lie in
the oracle's window (tests/oracle_spread.py); a case the oracle ends at the
cap must end there on the GPU too.  The full sweeps up to n = 512 run in
bench.py --workload sweeps.
"""
import numpy as np
import pytest

import jfft_inputs as ji
from oracle import triangles as tri
from oracle_spread import iteration_window

pytestmark = pytest.mark.gpu

LAM0, MU0 = 2.0 / 3.0, 0.5
MACRO = np.array([1.0, 1.0, 1.0])
TOL, CAP = 1e-10, 999


def _pkg():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    import paper_2508_02613_amd as pkg

    pkg.load_library()
    return pkg


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def geometry(kind, p):
    """The density on G_p: laminate (Sec. 4.1) with total contrast 10 or 1e4,
    cosine (Sec. 4.2) with contrast 1e4 or infinity (exact voids)."""
    if kind == "laminate-1e1":
        return ji.laminate_field((p, p), 10.0)
    if kind == "laminate-1e4":
        return ji.laminate_field((p, p), 1e4)
    if kind == "cosine-inf":
        return ji.cosine_void_field(p, None)
    if kind == "cosine-1e4":
        return ji.cosine_void_field(p, 1e4)
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["laminate-1e1", "laminate-1e4", "cosine-inf", "cosine-1e4"])
def test_sweep_counts_match_oracle(kind):
    pkg = _pkg()
    for n in (16, 32, 64):
        cells = {pc: pkg.Cell((n, n), pc=pc, element="tri")
                 for pc in (pkg.PC_GREEN, pkg.PC_JACOBI, pkg.PC_GREEN_JACOBI)}
        for c in cells.values():
            c.set_stop_rule(absolute=True)
        for p in sorted({4, 16, n}):
            E = ji.refine_geometry(geometry(kind, p), n)
            f = tri.rhs(E, MACRO, LAM0, MU0)
            row = []
            for pc, cell in cells.items():
                cell.set_material(E, lame=(LAM0, MU0))
                _, _, rep, _ = cell.solve(MACRO, tol=TOL, maxit=CAP)
                lo, hi, counts, runs = iteration_window(
                    lambda Ev, fv, ns, dm, tr: tri.solve(Ev, MACRO, LAM0, MU0, pc=pc, tol=TOL,
                                                         maxit=CAP, stop_absolute=True, f=fv,
                                                         noise_seed=ns, dot_mode=dm,
                                                         transform=tr), E, f)
                capped = any(r.status == "not_converged" for r in runs)
                row.append(f"pc{pc} gpu={rep.iters} oracle={min(counts)}..{max(counts)}")
                assert lo <= rep.iters <= hi, (kind, n, p, pc, rep.iters, counts)
                assert rep.status == "ok" or (capped and rep.status == "not_converged"), \
                    (kind, n, p, pc, rep.status, [r.status for r in runs])
            say(f"{kind} n={n} p={p}: " + "; ".join(row))
        for c in cells.values():
            c.close()
