"""jfft_solve_static (the entry point for callers that cannot allocate device
memory) against jfft_solve on the same inputs, through the C ABI: two calls
in a row on one GPU's static workspace, the second with a smaller cell, in
FP64 and in mixed precision.  The kernels and their launch configuration are
the same as jfft_solve's with direct launches, so the results must be
bitwise equal.  A cell whose workspace exceeds the static array is refused
before any device work."""
import numpy as np
import pytest

import jfft_inputs as ji

pytestmark = pytest.mark.gpu


def _pkg():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    import paper_2508_02613_amd as pkg

    pkg.load_library()
    return pkg


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _regular(pkg, E, precision, macro, tol):
    cell = pkg.Cell(E.shape, precision=precision, pc=pkg.PC_GREEN_JACOBI)
    cell.set_material(E, nu=0.3)
    u, sbar, rep, sig = cell.solve(macro, tol=tol, maxit=5000, want_sigma=True)
    out = (u.cpu().numpy(), sbar, rep, sig.cpu().numpy())
    cell.close()
    return out


def _static(pkg, E, precision, macro, tol):
    torch = pkg._torch()
    cell = pkg.Cell(E.shape, precision=precision, pc=pkg.PC_GREEN_JACOBI, workspace=False)
    dim = E.ndim
    sig = torch.empty((dim * (dim + 1) // 2, 2 ** dim) + E.shape, dtype=torch.float64,
                      device="cuda")
    u, sbar, rep, sig = cell.solve_static(E, 0.3, macro, tol=tol, maxit=5000, sigma=sig)
    torch.cuda.synchronize()
    out = (u.cpu().numpy(), sbar, rep, sig.cpu().numpy())
    cell.close()
    return out


@pytest.mark.parametrize("precision,shapes", [(0, [(64, 64, 64), (24, 20, 16)]),
                                              (1, [(256, 256), (48, 64)])],
                         ids=["fp64-3d", "mixed-2d"])
def test_static_workspace_equals_solve(precision, shapes):
    pkg = _pkg()
    for shape in shapes:  # two calls in a row, the second on a smaller cell
        dim = len(shape)
        E = ji.grf_field(shape, 1e4, seed=len(shape) + shape[0], ell=0.15)
        macro = ji.unit_macro_strain(dim, 0) + 0.5 * ji.unit_macro_strain(dim, dim)
        say(f"static workspace: {shape} precision={precision}")
        us, ss, rs, gs = _static(pkg, E, precision, macro, 1e-8)
        ur, sr, rr, gr = _regular(pkg, E, precision, macro, 1e-8)
        say(f"  iters static={rs.iters} solve={rr.iters} status {rs.status}/{rr.status} "
            f"max|du|={np.abs(us - ur).max():.1e}")
        assert rs.status == "ok" and rr.status == "ok"
        assert rs.iters == rr.iters and rs.outer == rr.outer
        assert np.array_equal(us, ur)
        assert np.array_equal(ss, sr)
        assert np.array_equal(gs, gr)
        assert rs.rel_res_true == rr.rel_res_true


def test_static_workspace_refuses_large_cells():
    pkg = _pkg()
    say("static workspace: too large a cell is refused")
    torch = pkg._torch()
    shape = (96, 96, 96)
    cell = pkg.Cell(shape, precision=pkg.FP64, workspace=False)
    assert cell.workspace_bytes > 128 << 20
    E = torch.ones(shape, dtype=torch.float64, device="cuda")
    with pytest.raises(pkg.JfftError, match="static workspace"):
        cell.solve_static(E, 0.3, ji.unit_macro_strain(3, 0))
    cell.close()
