"""GPU parity of the 2D linear-triangle discretisation (two triangles per
pixel, the paper's own 2D element) against the FP64 oracle
oracle/triangles.py (pinned in test_oracle_triangles.py): the operators K p,
f, Algorithm 2's diagonal and M^-1 element by element on grids of several
tiles with ragged tails and non-square pixels; solves with the four
preconditioners (iterations, u, sigma_bar, the stress field); the mixed
path's final residual; the paper's trend on its motivating example under its
absolute stopping rule; element switching and argument checks.
"""
import numpy as np
import pytest

import jfft_inputs as ji
import oracle
from oracle import triangles as tri
from oracle_spread import iteration_window

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


def _window(E, macro, pc, tol, lengths=None, stop_absolute=False):
    """The oracle's iteration window (oracle_spread): (lo, hi, counts, the
    unperturbed oracle result)."""
    f = tri.rhs(E, macro, LAM, MU, lengths)
    lo, hi, counts, runs = iteration_window(
        lambda Ev, fv, ns, dm, tr: tri.solve(Ev, macro, LAM, MU, pc=pc, tol=tol, maxit=20000,
                                             lengths=lengths, stop_absolute=stop_absolute, f=fv,
                                             noise_seed=ns, dot_mode=dm, transform=tr), E, f)
    return lo, hi, counts, runs[0]


CASES = [((32, 32), None), ((24, 20), (1.0, 0.6)), ((40, 36), (0.7, 1.3))]


@pytest.mark.parametrize("shape,lengths", CASES)
def test_operators_match_oracle(shape, lengths):
    pkg = _pkg()
    say(f"triangle operators {shape} lengths={lengths}")
    E = ji.uniform_random_field(shape, 1.0, 1e3, seed=3)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2,) + shape)
    macro = np.array([0.3, -0.2, 0.5])
    out = {}
    for pc in (pkg.PC_GREEN, pkg.PC_GREEN_JACOBI):
        cell = pkg.Cell(shape, pc=pc, lengths=lengths, element="tri")
        cell.set_material(E, nu=0.3)
        out[pc] = cell.apply_precond(x).cpu().numpy()
        if pc == pkg.PC_GREEN:
            Kx = cell.apply_stiffness(x).cpu().numpy()
            f = cell.assemble_rhs(macro).cpu().numpy()
            d = cell.jacobi_diag().cpu().numpy()
        cell.close()
    Kx_ref = tri.stiffness(E, x, LAM, MU, lengths)
    f_ref = tri.rhs(E, macro, LAM, MU, lengths)
    d_ref = tri.jacobi_diag(E, LAM, MU, lengths)
    assert np.abs(Kx - Kx_ref).max() <= 1e-12 * np.abs(Kx_ref).max()
    assert np.abs(f - f_ref).max() <= 1e-12 * np.abs(f_ref).max()
    assert np.abs(d - d_ref).max() <= 1e-12 * np.abs(d_ref).max()
    G = tri.green(shape, LAM, MU, lengths)
    zG, _ = oracle.precond(oracle.PC_GREEN, x, G=G, lengths=lengths)
    zGJ, _ = oracle.precond(oracle.PC_GREEN_JACOBI, x, diag=d_ref, G=G, lengths=lengths)
    assert np.abs(out[pkg.PC_GREEN] - zG).max() <= 1e-11 * np.abs(zG).max()
    assert np.abs(out[pkg.PC_GREEN_JACOBI] - zGJ).max() <= 1e-11 * np.abs(zGJ).max()


@pytest.mark.parametrize("pc", [1, 3, 2, 0])
@pytest.mark.parametrize("case", ["sine32", "rand24x20"])
def test_solve_matches_oracle(case, pc):
    pkg = _pkg()
    if case == "sine32":
        E, lengths, tol = ji.sine_contrast_field(32), None, 1e-8
    else:
        E, lengths, tol = ji.uniform_random_field((24, 20), 1.0, 1e2, seed=7), (1.0, 0.6), 1e-10
    macro = np.array([1.0, 0.0, 0.0]) if case == "sine32" else np.array([0.2, -0.1, 0.4])
    say(f"triangle solve {case} pc={pc}")
    lo, hi, counts, ref = _window(E, macro, pc, tol, lengths)
    cell = pkg.Cell(E.shape, pc=pc, lengths=lengths, element="tri")
    cell.set_material(E, nu=0.3)
    u, sbar, rep, sig = cell.solve(macro, tol=tol, maxit=20000, want_sigma=True)
    ug, sg = u.cpu().numpy(), sig.cpu().numpy()
    cell.close()
    say(f"  iters gpu={rep.iters} oracle={counts} window [{lo}, {hi}]")
    assert rep.status == "ok" and ref.status == "ok"
    assert lo <= rep.iters <= hi
    assert rep.rel_res_true <= 2 * tol
    if pc in (1, 3):  # the FFT-based preconditioners reach the solution closely
        # same iterates up to rounding: their difference is a small fraction
        # of the error left at the stopping tolerance
        rel = 1e-6 if case == "sine32" else 1e-8
        assert np.abs(ug - ref.u).max() <= rel * np.abs(ref.u).max()
        sig_ref, sbar_ref = tri.stress(E, macro, ug, LAM, MU, lengths)
        assert np.abs(sg - sig_ref).max() <= 1e-12 * np.abs(sig_ref).max()
        assert np.abs(sbar - sbar_ref).max() <= 1e-12 * np.abs(sbar_ref).max()
        assert np.abs(sbar - ref.sigma_bar).max() <= 1e-6 * np.abs(ref.sigma_bar).max()


def test_tight_solve_u_parity():
    """At tol 1e-12 the GPU and oracle solutions agree to 1e-10."""
    pkg = _pkg()
    E = ji.sine_contrast_field(32)
    macro = np.array([1.0, 0.0, 0.0])
    say("triangle tight solve 32^2 GJ")
    lo, hi, counts, ref = _window(E, macro, 3, 1e-12)
    cell = pkg.Cell(E.shape, pc=pkg.PC_GREEN_JACOBI, element="tri")
    cell.set_material(E, nu=0.3)
    u, sbar, rep, _ = cell.solve(macro, tol=1e-12, maxit=20000)
    ug = u.cpu().numpy()
    cell.close()
    say(f"  iters gpu={rep.iters} oracle={counts} window [{lo}, {hi}]")
    assert lo <= rep.iters <= hi
    assert np.abs(ug - ref.u).max() <= 1e-10 * np.abs(ref.u).max()
    assert np.abs(sbar - ref.sigma_bar).max() <= 1e-11 * np.abs(ref.sigma_bar).max()


def test_mixed_precision_reaches_fp64_solution():
    pkg = _pkg()
    E = ji.grf_field((128, 128), 1e4, seed=2, ell=0.1)
    macro = np.array([0.0, 0.0, 1.0])
    say("triangle mixed vs FP64 128^2")
    res = {}
    for prec in (pkg.FP64, pkg.MIXED):
        cell = pkg.Cell(E.shape, precision=prec, element="tri")
        cell.set_material(E, nu=0.3)
        u, sbar, rep, _ = cell.solve(macro, tol=1e-8, maxit=20000)
        res[prec] = (u.cpu().numpy(), sbar, rep)
        cell.close()
    (u64, s64, r64), (u32, s32, r32) = res[pkg.FP64], res[pkg.MIXED]
    assert r64.status == "ok" and r32.status == "ok"
    assert r32.rel_res_true <= 1e-8 and r64.rel_res_true <= 1e-8
    assert np.abs(u32 - u64).max() <= 1e-6 * np.abs(u64).max()
    assert np.abs(s32 - s64).max() <= 1e-7 * np.abs(s64).max()


def test_motivating_example_trend_with_triangles():
    """The paper's motivating example on its own element: a soft disc in a
    stiff matrix, smoothed by repeated filtering, absolute rule ||r||^2 <=
    1e-10.  Iteration counts lie in the oracle's window (oracle_spread);
    Green wins on the sharp disc, Green-Jacobi on the smoothed one."""
    pkg = _pkg()
    tol = 1e-10
    macro = np.array([1.0, 0.0, 0.0])
    its = {}
    for filters in (0, 8):
        E = ji.filtered_inclusion_field(64, filters)
        fn2 = float((tri.rhs(E, macro, LAM, MU) ** 2).sum())
        for pc in (pkg.PC_GREEN, pkg.PC_GREEN_JACOBI):
            lo, hi, counts, ref = _window(E, macro, pc, tol, stop_absolute=True)
            cell = pkg.Cell(E.shape, pc=pc, element="tri")
            cell.set_stop_rule(absolute=True)
            cell.set_material(E, nu=0.3)
            _, _, rep, _ = cell.solve(macro, tol=tol, maxit=20000)
            cell.close()
            say(f"  filters={filters} pc={pc}: gpu={rep.iters} oracle={counts} "
                f"window [{lo}, {hi}]")
            assert rep.status == "ok" and ref.status == "ok"
            assert lo <= rep.iters <= hi
            assert (rep.rel_res ** 2) * fn2 <= tol * 1.0001
            its[(filters, pc)] = rep.iters
    assert its[(0, pkg.PC_GREEN)] < its[(0, pkg.PC_GREEN_JACOBI)]
    assert its[(8, pkg.PC_GREEN_JACOBI)] < its[(8, pkg.PC_GREEN)]


def test_element_switch_and_errors():
    pkg = _pkg()
    say("triangle element switch and errors")
    with pytest.raises(pkg.JfftError):
        pkg.Cell((8, 8, 8), element="tri")
    with pytest.raises(ValueError):
        pkg.Cell((8, 8), element="hex")
    E = ji.uniform_random_field((16, 16), 1.0, 10.0, seed=1)
    cell = pkg.Cell((16, 16))
    cell.set_material(E, nu=0.3)
    _, s_quad, _, _ = cell.solve(np.array([1.0, 0, 0]), tol=1e-10)
    assert cell._lib.jfft_set_element(cell._h, 7) != 0
    assert cell._lib.jfft_set_element(cell._h, 1) == 0
    cell.element = "tri"
    with pytest.raises(pkg.JfftError) as e:  # the element change cleared the material
        cell.solve(np.array([1.0, 0, 0]), tol=1e-10)
    assert e.value.name == "no_material"
    cell.set_material(E, nu=0.3)
    _, s_tri, rep, _ = cell.solve(np.array([1.0, 0, 0]), tol=1e-10)
    ref = tri.solve(E, np.array([1.0, 0, 0]), LAM, MU, tol=1e-10)
    cell.close()
    assert np.abs(s_tri - ref.sigma_bar).max() <= 1e-8 * np.abs(ref.sigma_bar).max()
    assert np.abs(s_tri - s_quad).max() > 1e-6 * np.abs(s_quad).max()  # a different element


def test_full_size_operators_and_group():
    """The bench configuration (512^2 nodes, GRF contrast 1e4): K p, f,
    Algorithm 2's diagonal and the Green-Jacobi M^-1 against the oracle on
    the whole field, and a group of four 512^2 cells giving bitwise the
    single-cell solve."""
    pkg = _pkg()
    n = 512
    shape = (n, n)
    say(f"triangle operators full size {shape}")
    E = ji.grf_field(shape, 1e4, seed=0, ell=0.1)
    x = np.random.default_rng(4).standard_normal((2,) + shape)
    macro = np.array([1.0, 0.0, 0.0])
    cell = pkg.Cell(shape, pc=pkg.PC_GREEN_JACOBI, element="tri")
    cell.set_material(E, nu=0.3)
    Kx = cell.apply_stiffness(x).cpu().numpy()
    f = cell.assemble_rhs(macro).cpu().numpy()
    d = cell.jacobi_diag().cpu().numpy()
    z = cell.apply_precond(x).cpu().numpy()
    u1, s1, r1, _ = cell.solve(macro, tol=1e-8, maxit=20000)
    u1 = u1.cpu().numpy()
    cell.close()
    assert np.abs(Kx - tri.stiffness(E, x, LAM, MU)).max() <= 1e-12 * np.abs(Kx).max()
    assert np.abs(f - tri.rhs(E, macro, LAM, MU)).max() <= 1e-12 * np.abs(f).max()
    d_ref = tri.jacobi_diag(E, LAM, MU)
    assert np.abs(d - d_ref).max() <= 1e-12 * np.abs(d_ref).max()
    zr, _ = oracle.precond(oracle.PC_GREEN_JACOBI, x, diag=d_ref, G=tri.green(shape, LAM, MU))
    assert np.abs(z - zr).max() <= 1e-11 * np.abs(zr).max()
    say("  group of four 512^2 cells")
    Es = np.stack([E] + [ji.grf_field(shape, 1e4, seed=s, ell=0.1) for s in (1, 2, 3)])
    grp = pkg.Cell(shape, pc=pkg.PC_GREEN_JACOBI, batch=4, element="tri")
    grp.set_material(Es, nu=0.3)
    ug, sg, rg, _ = grp.solve_batch(np.tile(macro, (4, 1)), tol=1e-8, maxit=20000)
    ug = ug.cpu().numpy()
    grp.close()
    assert rg[0].iters == r1.iters and all(r.status == "ok" for r in rg)
    assert np.array_equal(ug[0], u1) and np.array_equal(sg[0], s1)
