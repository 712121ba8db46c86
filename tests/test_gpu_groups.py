"""GPU tests of many cells of uneven sizes (2D SIMP densities, the batched
topology-optimisation workload): groups per grid shape on concurrent streams,
graph-replayed PCG, mixed precision.  Each cell's result must be bitwise the
result of the same cell solved alone with direct launches; one member is
checked against the oracle.
"""
import numpy as np
import pytest

import jfft_inputs as ji
import oracle

pytestmark = pytest.mark.gpu

LAM, MU = oracle.lame_from_nu(0.3)


def _pkg():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    import paper_2508_02613_amd as pkg

    pkg.load_library()
    return pkg


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _cells(sizes, seed0):
    fields = [ji.simp_field(n, seed=seed0 + i) for i, n in enumerate(sizes)]
    macros = [ji.unit_macro_strain(2, i % 3) for i in range(len(sizes))]
    return fields, macros


@pytest.mark.parametrize("precision", [0, 1])
def test_uneven_groups_equal_single_cells(precision):
    pkg = _pkg()
    from paper_2508_02613_amd.groups import solve_cells

    sizes = [64, 128, 64, 32, 128, 64, 32, 64]
    say(f"uneven SIMP groups {sizes} precision={precision}")
    fields, macros = _cells(sizes, 100)
    res, wall = solve_cells(fields, macros, tol=1e-8, precision=precision, graph_iterations=8)
    for i, (E, m) in enumerate(zip(fields, macros)):
        cell = pkg.Cell(E.shape, precision=precision)
        cell.set_material(E, nu=0.3)
        u, sbar, rep, _ = cell.solve(m, tol=1e-8, maxit=20000)
        r = res[i]
        assert r["report"].status == "ok" and rep.status == "ok"
        assert r["report"].iters == rep.iters, (i, r["report"].iters, rep.iters)
        assert np.array_equal(r["u"].cpu().numpy(), u.cpu().numpy()), f"cell {i}"
        assert np.array_equal(r["sigma_bar"], sbar)
        assert 0 < r["report"].rel_res_true <= 1.5e-8
        cell.close()
    say(f"  iterations {[r['report'].iters for r in res]} wall {wall * 1e3:.1f} ms")


def test_simp_member_matches_oracle():
    """Group members against the oracle: iteration counts within +-1 plus the
    flat stretch of the oracle's convergence curve around the threshold (at
    tol 1e-8 and 1e-12); fields near the exact discrete solution at tol 1e-12
    (1e-10)."""
    pkg = _pkg()
    from paper_2508_02613_amd.groups import solve_cells

    fields, macros = _cells([64, 64, 64], 7)
    for tol in (1e-8, 1e-12):
        say(f"SIMP 64^2 group members vs oracle (FP64, tol {tol:g})")
        res, _ = solve_cells(fields, macros, tol=tol, graph_iterations=4)
        for i in range(3):
            ref = oracle.solve(fields[i], macros[i], LAM, MU, pc=3, tol=tol, maxit=20000,
                               hist_len=20000)
            u = res[i]["u"].cpu().numpy()
            it = res[i]["report"].iters
            err = np.linalg.norm(u - ref.u) / np.linalg.norm(ref.u)
            say(f"  cell {i}: iters gpu={it} oracle={ref.iters} err(u)={err:.2e}")
            # +-1, plus the iterations over which the oracle's residual lies
            # within a factor 10 of the threshold: where the convergence curve
            # is that flat, rounding differences (amplified by the 1e9
            # contrast) move the crossing by a few iterations
            fn = np.linalg.norm(oracle.rhs(fields[i], macros[i], LAM, MU))
            rel = ref.res[:ref.iters] / fn
            slack = 1 + int(np.count_nonzero((rel >= tol / 10) & (rel <= 10 * tol)))
            say(f"    slack {slack}")
            assert abs(it - ref.iters) <= slack
            if tol == 1e-8:
                assert err <= 1e-6
            else:
                assert err <= 1e-10
                np.testing.assert_allclose(res[i]["sigma_bar"], ref.sigma_bar, rtol=1e-10,
                                           atol=1e-12 * np.abs(ref.sigma_bar).max())


def test_green_jacobi_beats_green_on_simp():
    """The paper's claim on smooth high-contrast data, on the GPU path: the
    Green-Jacobi preconditioner needs far fewer iterations than Green."""
    pkg = _pkg()
    say("SIMP 128^2: Green vs Green-Jacobi iterations")
    E = ji.simp_field(128, seed=0)
    its = {}
    for pc in (pkg.PC_GREEN, pkg.PC_GREEN_JACOBI):
        cell = pkg.Cell(E.shape, pc=pc)
        cell.set_material(E, nu=0.3)
        _, _, rep, _ = cell.solve(ji.unit_macro_strain(2, 0), tol=1e-8, maxit=20000)
        assert rep.status == "ok"
        its[pc] = rep.iters
        cell.close()
    ref_g = oracle.solve(E, ji.unit_macro_strain(2, 0), LAM, MU, pc=1, tol=1e-8, maxit=20000)
    ref_gj = oracle.solve(E, ji.unit_macro_strain(2, 0), LAM, MU, pc=3, tol=1e-8, maxit=20000)
    say(f"  gpu Green {its[pkg.PC_GREEN]} GJ {its[pkg.PC_GREEN_JACOBI]}; oracle Green {ref_g.iters} "
        f"GJ {ref_gj.iters}")
    # counts to 5% (contrast 1e9 makes the stopping iteration rounding-sensitive;
    # exact parity is checked in test_simp_member_matches_oracle)
    assert abs(its[pkg.PC_GREEN_JACOBI] - ref_gj.iters) <= 0.05 * ref_gj.iters
    assert abs(its[pkg.PC_GREEN] - ref_g.iters) <= 0.05 * ref_g.iters
    assert its[pkg.PC_GREEN_JACOBI] * 10 < its[pkg.PC_GREEN]
