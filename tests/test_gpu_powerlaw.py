"""GPU parity of the power-law Newton solve (nonlinear example, Sec. 4;
Newton linearisation, Sec. 2.2, eq. lin_system) against the FP64 oracle
oracle/powerlaw.py (itself pinned in test_oracle_powerlaw.py):

* the operators of one Newton step at a random iterate: the force
  f = -B^T W sigma(E + B u), the tangent action K(u) p and Algorithm 2 on
  K(u), element by element, on grids of several stiffness tiles with ragged
  tails, cubic and non-cubic elements;
* whole Newton solves with the three preconditioners: step count, PCG
  iterations per step, ||f|| per step, u (mean removed) and sigma_bar;
* the linear limit (n = 1, proportional inclusion moduli) against the
  library's own linear solve, graph replay against direct launches, and the
  argument and state checks of the entry points.
"""
import numpy as np
import pytest

import jfft_inputs as ji
import oracle
from oracle import powerlaw as pl

pytestmark = pytest.mark.gpu

PRM = pl.PowerLaw()
SHEAR = np.array([0.01, 0.0, -0.01, 0.0, 0.0, 0.05 * np.sqrt(2)])


def _pkg():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    import paper_2508_02613_amd as pkg

    pkg.load_library()
    return pkg


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _cell(pkg, shape, pc, lengths=None):
    return pkg.Cell(shape, pc=pc, lengths=lengths)


def _set(cell, phase, prm=PRM):
    cell.set_material_powerlaw(phase, K=prm.K, sigma0=prm.sigma0, eps0=prm.eps0, n=prm.n,
                               K_incl=prm.K_incl, mu_incl=prm.mu_incl)


OP_CASES = [((12, 16, 18), None), ((16, 16, 16), None), ((10, 30, 20), (1.0, 1.5, 0.5))]


@pytest.mark.parametrize("tiles3d", [1, 2])
@pytest.mark.parametrize("shape,lengths", OP_CASES)
def test_operators_match_oracle(shape, lengths, tiles3d):
    """Both 3D block shapes of the tangent kernel (16 x 14 and 32 x 6 nodes)."""
    pkg = _pkg()
    say(f"power-law operators {shape} lengths={lengths} tiles3d={tiles3d}")
    rng = np.random.default_rng(11)
    phase = 1.0 - ji.spherical_inclusions(shape, 3, 0.22, seed=2)
    u = 0.02 * rng.standard_normal((3,) + shape)
    p = rng.standard_normal((3,) + shape)
    macro = rng.uniform(-0.05, 0.05, 6)
    cell = _cell(pkg, shape, pkg.PC_GREEN_JACOBI, lengths)
    cell.set_tunables(tiles3d=tiles3d)
    _set(cell, phase)
    f = cell.powerlaw_force(macro, u).cpu().numpy()
    Kp = cell.powerlaw_tangent(macro, u, p).cpu().numpy()
    d = cell.powerlaw_jacobi_diag(macro, u).cpu().numpy()
    cell.set_diag_method("probing")
    d_probe = cell.powerlaw_jacobi_diag(macro, u).cpu().numpy()
    cell.close()
    f_ref = pl.force(u, macro, phase, PRM, lengths)
    Kp_ref = pl.tangent_op(u, p, macro, phase, PRM, lengths)
    d_ref = pl.jacobi_diag(u, macro, phase, PRM, lengths)
    assert np.abs(f - f_ref).max() <= 1e-12 * np.abs(f_ref).max()
    assert np.abs(Kp - Kp_ref).max() <= 1e-12 * np.abs(Kp_ref).max()
    # closed form (formed with the force) and Algorithm 2's probing
    assert np.abs(d - d_ref).max() <= 1e-12 * np.abs(d_ref).max()
    assert np.abs(d_probe - d_ref).max() <= 1e-12 * np.abs(d_ref).max()
    assert d.min() > 0


def test_operators_at_zero_iterate_and_matrix_only():
    """u = 0 in a homogeneous matrix: f = 0 for any macro strain (every
    element has the same stress, whose divergence vanishes), and the tangent
    is the same for every element."""
    pkg = _pkg()
    shape = (8, 8, 8)
    say(f"power-law operators at u = 0 {shape}")
    phase = np.ones(shape)
    u = np.zeros((3,) + shape)
    p = np.random.default_rng(3).standard_normal((3,) + shape)
    cell = _cell(pkg, shape, pkg.PC_GREEN)
    _set(cell, phase)
    f = cell.powerlaw_force(SHEAR, u).cpu().numpy()
    Kp = cell.powerlaw_tangent(SHEAR, u, p).cpu().numpy()
    cell.close()
    Kp_ref = pl.tangent_op(u, p, SHEAR, phase, PRM)
    assert np.abs(f).max() <= 1e-15
    assert np.abs(Kp - Kp_ref).max() <= 1e-12 * np.abs(Kp_ref).max()


def _newton_windows(phase, pc, kw, macro=SHEAR):
    """The oracle's Newton solve and the per-step PCG iteration windows: min - 1
    .. max + 1 of the step counts over the plain run and four runs with the
    oracle's rounding-difference model on (every K p and M^-1 r entry moved
    by one ulp in a seeded direction; see tests/oracle_spread.py).  Runs that
    take a different number of Newton steps than the plain one are reported
    and left out of the windows."""
    ref = pl.newton(phase, macro, PRM, pc=pc, **kw)
    runs = [ref] + [pl.newton(phase, macro, PRM, pc=pc, noise_seed=s, **kw) for s in (1, 2, 3, 4)]
    steps = [r.pcg_iters for r in runs]
    same = [s for s in steps if len(s) == len(ref.pcg_iters)]
    lo = [min(s[i] for s in same) - 1 for i in range(len(ref.pcg_iters))]
    hi = [max(s[i] for s in same) + 1 for i in range(len(ref.pcg_iters))]
    return ref, steps, lo, hi


def _in_windows(iters, lo, hi):
    return len(iters) == len(lo) and all(a <= k <= b for k, a, b in zip(iters, lo, hi))


@pytest.mark.parametrize("pc", ["GJ", "G", "J"])
def test_newton_matches_oracle(pc):
    pkg = _pkg()
    shape = (12, 16, 18)
    say(f"power-law Newton {shape} pc={pc}")
    codes = {"GJ": (pkg.PC_GREEN_JACOBI, oracle.PC_GREEN_JACOBI),
             "G": (pkg.PC_GREEN, oracle.PC_GREEN), "J": (pkg.PC_JACOBI, oracle.PC_JACOBI)}
    gpc, opc = codes[pc]
    phase = 1.0 - ji.spherical_inclusions(shape, 3, 0.2, seed=5)
    kw = dict(newton_tol=1e-10, pcg_tol=1e-10, max_newton=20, maxit=5000)
    ref, steps, lo, hi = _newton_windows(phase, opc, kw)
    cell = _cell(pkg, shape, gpc)
    _set(cell, phase)
    u, sbar, rep = cell.solve_newton(SHEAR, **kw)
    ug = u.cpu().numpy()
    cell.close()
    say(f"  gpu {rep}  oracle runs {steps} windows {list(zip(lo, hi))}")
    assert rep.converged and ref.converged
    assert rep.steps == len(ref.pcg_iters)
    assert all(a <= k <= b for k, a, b in zip(rep.pcg_iters, lo, hi)), (rep.pcg_iters, lo, hi)
    assert abs(rep.res[0] - ref.res[0]) <= 1e-12 * ref.res[0]
    for i in range(1, len(ref.res)):
        if rep.pcg_iters[:i] == ref.pcg_iters[:i]:
            # two PCG runs that differ only in rounding stop at the same
            # iteration with residuals a small fraction of the stopping
            # threshold apart; that difference carries into ||f|| of the
            # next Newton step
            lin = max(kw["pcg_tol"] * ref.res[i - 1], 0.1 * kw["newton_tol"])
            assert abs(rep.res[i] - ref.res[i]) <= 1e-6 * ref.res[i] + 0.05 * lin, \
                (i, rep.res, ref.res)
    assert rep.res[-1] < kw["newton_tol"]
    uo = ref.u - ref.u.reshape(3, -1).mean(axis=1).reshape(3, 1, 1, 1)
    assert np.abs(ug.reshape(3, -1).mean(axis=1)).max() <= 1e-15 * np.abs(uo).max() * ug[0].size
    # the oracle's own solutions with the three preconditioners differ by up
    # to 6e-9 in u and 5e-11 in sigma_bar (relative to the largest entry):
    # the room a converged Newton solve leaves
    assert np.abs(ug - uo).max() <= 2e-8 * np.abs(uo).max()
    assert np.abs(sbar - ref.sigma_bar).max() <= 2e-10 * np.abs(ref.sigma_bar).max()


def test_newton_unit_voxels_absolute_rule():
    """Voxels of unit edge (cell side n) with the stopping rules of Sec. 4:
    ||f|| < 1e-5 for Newton and ||r||^2 <= 1e-10 for each PCG solve."""
    pkg = _pkg()
    n = 16
    shape = (n, n, n)
    say(f"power-law Newton unit voxels, absolute rule {shape}")
    phase = 1.0 - ji.spherical_inclusions(shape, 8, 0.15, seed=5)
    macro = np.array([0, 0, 0, 0, 0, 0.05 * np.sqrt(2)])
    L = (float(n),) * 3
    ref, steps, lo, hi = _newton_windows(
        phase, oracle.PC_GREEN_JACOBI,
        dict(newton_tol=1e-5, pcg_tol=1e-10, lengths=L, pcg_absolute=True), macro)
    cell = _cell(pkg, shape, pkg.PC_GREEN_JACOBI, L)
    cell.set_stop_rule(absolute=True)
    _set(cell, phase)
    u, s, r = cell.solve_newton(macro, newton_tol=1e-5, pcg_tol=1e-10)
    cell.close()
    say(f"  gpu {r}  oracle runs {steps} windows {list(zip(lo, hi))}")
    assert r.converged and ref.converged and r.steps == len(ref.pcg_iters) >= 3
    assert _in_windows(r.pcg_iters, lo, hi), (r.pcg_iters, lo, hi)
    assert abs(r.res[0] - ref.res[0]) <= 1e-12 * ref.res[0]
    same = r.pcg_iters == ref.pcg_iters
    assert np.abs(s - ref.sigma_bar).max() <= (1e-10 if same else 1e-6) * np.abs(ref.sigma_bar).max()


@pytest.mark.parametrize("rule", ["relative", "absolute"])
def test_newton_mixed_precision_matches_fp64(rule):
    """FP32 tangent solves refined against the FP64 tangent residual reach
    the FP64 Newton solution: the same steps and ||f|| history to the
    accuracy the inner tolerances leave, u and sigma_bar close."""
    pkg = _pkg()
    n = 16
    shape = (n, n, n)
    say(f"power-law Newton mixed vs FP64 {shape} {rule} rule")
    phase = 1.0 - ji.spherical_inclusions(shape, 8, 0.15, seed=5)
    macro = np.array([0, 0, 0, 0, 0, 0.05 * np.sqrt(2)])
    if rule == "absolute":
        L, kw = (float(n),) * 3, dict(newton_tol=1e-5, pcg_tol=1e-10)
    else:
        L, kw = None, dict(newton_tol=1e-10, pcg_tol=1e-10)
    out = {}
    for prec in (pkg.FP64, pkg.MIXED):
        cell = pkg.Cell(shape, precision=prec, pc=pkg.PC_GREEN_JACOBI, lengths=L)
        cell.set_stop_rule(absolute=rule == "absolute")
        _set(cell, phase)
        u, s, r = cell.solve_newton(macro, **kw)
        out[prec] = (u.cpu().numpy(), s, r)
        cell.close()
    (u64, s64, r64), (u32, s32, r32) = out[pkg.FP64], out[pkg.MIXED]
    say(f"  fp64 {r64}\n  mixed {r32}")
    assert r64.converged and r32.converged
    assert abs(r32.res[0] - r64.res[0]) <= 1e-12 * r64.res[0]
    for a, b in zip(r32.res[1:-1], r64.res[1:-1]):
        assert abs(a - b) <= 1e-3 * b
    if rule == "relative":
        assert r32.steps == r64.steps
        assert np.abs(u32 - u64).max() <= 1e-5 * np.abs(u64).max()
        assert np.abs(s32 - s64).max() <= 1e-7 * np.abs(s64).max()
    else:
        # Sec. 4's rules put the inner tolerance (||r|| <= 1e-5) at the Newton
        # tolerance (||f|| < 1e-5): the last step's residual sits at the
        # threshold.  The mixed inner solves stop on the true FP64 residual,
        # the FP64 ones on the recursive residual, one iteration apart; that
        # can decide one Newton step either way; both meet ||f|| < 1e-5
        assert abs(r32.steps - r64.steps) <= 1
        assert np.abs(u32 - u64).max() <= 1e-4 * np.abs(u64).max()
        assert np.abs(s32 - s64).max() <= 1e-5 * np.abs(s64).max()


def test_newton_probing_diagonal_equals_closed_form():
    pkg = _pkg()
    shape = (12, 16, 18)
    say(f"power-law Newton, probing vs closed-form tangent diagonal {shape}")
    phase = 1.0 - ji.spherical_inclusions(shape, 3, 0.2, seed=5)
    out = []
    for method in ("closed_form", "probing"):
        cell = _cell(pkg, shape, pkg.PC_GREEN_JACOBI)
        cell.set_diag_method(method)
        _set(cell, phase)
        u, s, r = cell.solve_newton(SHEAR, newton_tol=1e-10, pcg_tol=1e-10)
        out.append((u.cpu().numpy(), s, r))
        cell.close()
    (u0, s0, r0), (u1, s1, r1) = out
    _, steps, lo, hi = _newton_windows(phase, oracle.PC_GREEN_JACOBI,
                                       dict(newton_tol=1e-10, pcg_tol=1e-10))
    say(f"  closed form {r0.pcg_iters} probing {r1.pcg_iters} oracle windows {list(zip(lo, hi))}")
    assert r0.converged and r1.converged and r0.steps == r1.steps
    assert _in_windows(r0.pcg_iters, lo, hi) and _in_windows(r1.pcg_iters, lo, hi)
    assert np.abs(u0 - u1).max() <= 2e-8 * np.abs(u1).max()
    assert np.abs(s0 - s1).max() <= 2e-10 * np.abs(s1).max()


def test_newton_step_cap_and_paper_tolerance():
    """max_newton = 1 stops after one step with JFFT_E_NOT_CONVERGED and
    every output written; the paper's tolerance (||f|| < 1e-5) on the same
    cell converges in the oracle's number of steps."""
    pkg = _pkg()
    shape = (12, 12, 12)
    say(f"power-law Newton step cap {shape}")
    phase = 1.0 - ji.spherical_inclusions(shape, 3, 0.2, seed=5)
    cell = _cell(pkg, shape, pkg.PC_GREEN_JACOBI)
    _set(cell, phase)
    u1, s1, r1 = cell.solve_newton(SHEAR, newton_tol=1e-10, max_newton=1)
    ref1, _, lo1, hi1 = _newton_windows(phase, oracle.PC_GREEN_JACOBI,
                                        dict(newton_tol=1e-10, max_newton=1))
    assert not r1.converged and r1.steps == 1 and len(r1.res) == 2
    assert _in_windows(r1.pcg_iters, lo1, hi1), (r1.pcg_iters, lo1, hi1)
    if r1.pcg_iters == ref1.pcg_iters:
        assert abs(r1.res[1] - ref1.res[1]) <= 1e-6 * ref1.res[1]
    assert np.abs(s1 - ref1.sigma_bar).max() <= 1e-6 * np.abs(ref1.sigma_bar).max()
    u, s, r = cell.solve_newton(SHEAR)
    ref, _, lo, hi = _newton_windows(phase, oracle.PC_GREEN_JACOBI, {})
    cell.close()
    assert r.converged and r.steps == len(ref.pcg_iters)
    assert _in_windows(r.pcg_iters, lo, hi), (r.pcg_iters, lo, hi)
    same = r.pcg_iters == ref.pcg_iters
    assert np.abs(s - ref.sigma_bar).max() <= (1e-10 if same else 1e-6) * np.abs(ref.sigma_bar).max()


def test_newton_homogeneous_matrix_zero_steps():
    pkg = _pkg()
    shape = (8, 8, 8)
    say(f"power-law Newton homogeneous {shape}")
    cell = _cell(pkg, shape, pkg.PC_GREEN_JACOBI)
    _set(cell, np.ones(shape))
    u, s, r = cell.solve_newton(SHEAR)
    ug = u.cpu().numpy()
    cell.close()
    assert r.converged and r.steps == 0 and r.pcg_iters == [] and r.res[0] <= 1e-15
    assert np.abs(ug).max() == 0.0
    np.testing.assert_allclose(s, pl.stress(SHEAR, np.array(1.0), PRM), rtol=1e-13, atol=1e-16)


def test_linear_limit_equals_linear_solve():
    """n = 1 and inclusion moduli t times the matrix's: a linear problem, one
    Newton step; the result equals the library's linear solve with E = 1 in
    the matrix and t in the inclusions."""
    pkg = _pkg()
    shape = (16, 16, 16)
    say(f"power-law linear limit {shape}")
    mu = PRM.sigma0 / (3.0 * PRM.eps0)
    t = 10.0
    prm1 = pl.PowerLaw(K=PRM.K, sigma0=PRM.sigma0, eps0=PRM.eps0, n=1.0, K_incl=t * PRM.K,
                       mu_incl=t * mu)
    incl = ji.spherical_inclusions(shape, 2, 0.2, seed=1)
    phase = 1.0 - incl
    cell = _cell(pkg, shape, pkg.PC_GREEN_JACOBI)
    _set(cell, phase, prm1)
    u, s, r = cell.solve_newton(SHEAR, newton_tol=1e-13, pcg_tol=1e-12)
    un = u.cpu().numpy()
    assert r.converged and r.steps == 1, r
    lam = PRM.K - 2 * mu / 3
    cell.set_material(1.0 + (t - 1.0) * incl, lame=(lam, mu))
    ul, sl, rl, _ = cell.solve(SHEAR, tol=1e-12, maxit=5000)
    ulin = ul.cpu().numpy()
    cell.close()
    assert np.abs(un - ulin).max() <= 1e-9 * np.abs(ulin).max()
    np.testing.assert_allclose(s, sl, rtol=1e-10, atol=1e-14)


def test_graph_replay_equals_direct_launches():
    pkg = _pkg()
    shape = (12, 16, 18)
    say(f"power-law Newton graph replay {shape}")
    phase = 1.0 - ji.spherical_inclusions(shape, 3, 0.2, seed=5)
    import torch

    out = []
    st = torch.cuda.Stream()  # graphs are captured on a stream of the caller's
    for G in (0, 8, 8):
        cell = pkg.Cell(shape, pc=pkg.PC_GREEN_JACOBI, stream=st)
        cell.set_graph_iterations(G)
        _set(cell, phase)
        u, s, r = cell.solve_newton(SHEAR, newton_tol=1e-10, pcg_tol=1e-10)
        # a second solve on the same handle replays the captured graph again
        u2, s2, r2 = cell.solve_newton(SHEAR, newton_tol=1e-10, pcg_tol=1e-10)
        st.synchronize()
        out.append((u.cpu().numpy(), s, r.pcg_iters, u2.cpu().numpy(), s2, r2.pcg_iters))
        cell.close()
    for o in out[1:]:
        assert o[2] == out[0][2] and o[5] == out[0][2]
        assert np.array_equal(o[0], out[0][0]) and np.array_equal(o[3], out[0][0])
        assert np.array_equal(o[1], out[0][1]) and np.array_equal(o[4], out[0][1])


def test_argument_and_state_checks():
    pkg = _pkg()
    say("power-law argument checks")
    shape = (8, 8, 8)
    phase = np.ones(shape)
    c2 = pkg.Cell((16, 16), pc=pkg.PC_GREEN)
    with pytest.raises(pkg.JfftError):
        c2.set_material_powerlaw(np.ones((16, 16)))
    c2.close()
    cb = pkg.Cell(shape, pc=pkg.PC_GREEN, batch=2)
    with pytest.raises(pkg.JfftError):
        cb.set_material_powerlaw(np.ones(shape))
    cb.close()
    cell = _cell(pkg, shape, pkg.PC_GREEN_JACOBI)
    with pytest.raises(pkg.JfftError) as e:
        cell.solve_newton(SHEAR)
    assert e.value.name == "no_material"
    for bad in (dict(n=0.5), dict(K=-1.0), dict(mu_incl=0.0), dict(eps0=float("nan"))):
        args = dict(K=2.0, sigma0=0.5, eps0=0.1, n=5.0, K_incl=2.0, mu_incl=0.5)
        args.update(bad)
        with pytest.raises(pkg.JfftError):
            cell.set_material_powerlaw(phase, **args)
    bad_phase = phase.copy()
    bad_phase[1, 2, 3] = -1.0
    with pytest.raises(pkg.JfftError):
        _set(cell, bad_phase)
    _set(cell, phase)
    with pytest.raises(pkg.JfftError):
        cell.solve_newton(SHEAR, newton_tol=0.0)
    with pytest.raises(pkg.JfftError):
        cell.solve_newton(SHEAR, pcg_tol=1.5)
    with pytest.raises(pkg.JfftError):
        cell.solve_newton(np.array([0, 0, 0, 0, 0, np.inf]))
    # the linear entry points refuse the power-law material, and a linear
    # material set afterwards works again
    with pytest.raises(pkg.JfftError) as e:
        cell.solve(np.zeros(6))
    assert e.value.name == "no_material"
    lam, mu = oracle.lame_from_nu(0.3)
    E = ji.uniform_random_field(shape, 1.0, 10.0, seed=2)
    cell.set_material(E, nu=0.3)
    u, sbar, rep, _ = cell.solve(np.array([1.0, 0, 0, 0, 0, 0]), tol=1e-10, maxit=500)
    ref = oracle.solve(E, np.array([1.0, 0, 0, 0, 0, 0]), lam, mu, pc=oracle.PC_GREEN_JACOBI,
                       tol=1e-10, maxit=500)
    cell.close()
    assert abs(rep.iters - ref.iters) <= 1
    assert np.abs(u.cpu().numpy() - ref.u).max() <= 1e-9 * np.abs(ref.u).max()


def test_operators_full_size_sampled():
    """The bench configuration (200^3 nodes, voxels of unit edge, 8 spherical
    inclusions): force, tangent action and the closed-form diagonal at 3000
    seeded nodes against the oracle's evaluation at those nodes."""
    pkg = _pkg()
    n = 200
    shape = (n, n, n)
    say(f"power-law operators full size {shape}, sampled")
    phase = 1.0 - ji.spherical_inclusions(shape, 8, 0.15, seed=0)
    rng = np.random.default_rng(21)
    u = 0.01 * rng.standard_normal((3,) + shape)
    p = rng.standard_normal((3,) + shape)
    macro = np.array([0, 0, 0, 0, 0, 0.05 * np.sqrt(2)])
    L = (float(n),) * 3
    cell = _cell(pkg, shape, pkg.PC_GREEN_JACOBI, L)
    _set(cell, phase)
    f = cell.powerlaw_force(macro, u).cpu().numpy().reshape(3, -1)
    Kp = cell.powerlaw_tangent(macro, u, p).cpu().numpy().reshape(3, -1)
    d = cell.powerlaw_jacobi_diag(macro, u).cpu().numpy().reshape(3, -1)
    cell.close()
    nodes = rng.choice(n ** 3, 3000, replace=False)
    fr, kr, dr = pl.at_nodes(u, p, macro, phase, PRM, nodes, L)
    assert np.abs(f[:, nodes] - fr).max() <= 1e-12 * np.abs(fr).max()
    assert np.abs(Kp[:, nodes] - kr).max() <= 1e-12 * np.abs(kr).max()
    assert np.abs(d[:, nodes] - dr).max() <= 1e-12 * np.abs(dr).max()
