"""GPU parity of the phase-field topology optimisation (Sec. 4, eq. aim_fun)
against the FP64 oracle oracle/topopt.py (pinned in test_oracle_topopt.py):
the objective, its parts and its gradient on grids with ragged tiles,
non-square pixels and voids; the projected L-BFGS trajectory (objective
history, steps, evaluations, PCG iterations, final density); the mixed
path; argument checks.
"""
import numpy as np
import pytest

import oracle
from oracle import topopt as to

pytestmark = pytest.mark.gpu

T = to.target_stresses()


def _pkg():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    import paper_2508_02613_amd as pkg

    pkg.load_library()
    return pkg


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _group(pkg, shape, lengths=None, precision=0):
    return pkg.Cell(shape, precision=precision, pc=pkg.PC_GREEN_JACOBI, lengths=lengths, batch=3,
                    element="tri")


@pytest.mark.parametrize("shape,lengths,voids", [((16, 16), None, False),
                                                 ((24, 20), (1.0, 0.6), False),
                                                 ((20, 20), None, True)])
def test_objective_and_gradient_match_oracle(shape, lengths, voids):
    pkg = _pkg()
    say(f"topopt eval {shape} lengths={lengths} voids={voids}")
    rng = np.random.default_rng(2)
    rho = rng.uniform(0.2, 0.9, shape)
    if voids:
        rho[3:7, 4:9] = 0.0
    eta = 0.02
    ref = to.evaluate(rho, eta=eta, tol=1e-12, lengths=lengths)
    grp = _group(pkg, shape, lengths)
    f, grad, its = grp.topopt_eval(rho, T, eta=eta, tol=1e-12)
    g = grad.cpu().numpy()
    grp.close()
    say(f"  f gpu={f} oracle=({ref.f}, {ref.f_sigma}, {ref.f_pf}) iters gpu={its} oracle={ref.iters}")
    assert f[2] == pytest.approx(ref.f_pf, rel=1e-12)
    assert f[1] == pytest.approx(ref.f_sigma, rel=1e-9)
    assert f[0] == pytest.approx(ref.f, rel=1e-9)
    assert np.abs(g - ref.g).max() <= 1e-8 * np.abs(ref.g).max()
    assert all(abs(a - b) <= max(2, round(0.05 * b)) for a, b in zip(its, ref.iters))


# one full block of 256 nodes; ragged tails of the L-BFGS vector kernels on
# non-square pixels; several blocks with a tail
@pytest.mark.parametrize("shape,lengths,seed,K", [((16, 16), None, 0, 8),
                                                  ((24, 20), (1.0, 0.6), 1, 6),
                                                  ((40, 36), None, 1, 6)])
def test_lbfgs_trajectory_matches_oracle(shape, lengths, seed, K):
    pkg = _pkg()
    say(f"topopt L-BFGS {shape} lengths={lengths} seed={seed} steps={K}")
    rho0 = np.random.default_rng(seed).uniform(0.0, 1.0, shape)
    ref = to.lbfgs(lambda r: to.evaluate(r, eta=0.01, tol=1e-12, lengths=lengths), rho0, K)
    grp = _group(pkg, shape, lengths)
    rho, out = grp.topopt_lbfgs(rho0, T, K, eta=0.01, tol=1e-12)
    r = rho.cpu().numpy()
    grp.close()
    say(f"  gpu steps={out['steps']} evals={out['evals']} f={out['f']}")
    say(f"  oracle steps={len(ref.f) - 1} evals={ref.evals} f={ref.f}")
    assert out["steps"] == len(ref.f) - 1 and out["evals"] == ref.evals
    np.testing.assert_allclose(out["f"], ref.f, rtol=1e-8)
    np.testing.assert_allclose(out["gnorm"], ref.gnorm, rtol=1e-6)
    for a, b in zip(out["iters"], ref.iters):
        assert all(abs(x - y) <= max(2, round(0.05 * y)) for x, y in zip(a, b))
    assert np.abs(r - ref.rho).max() <= 1e-6
    assert all(b <= a for a, b in zip(out["f"], out["f"][1:]))


def test_mixed_precision_objective():
    pkg = _pkg()
    shape = (32, 32)
    say(f"topopt eval mixed vs FP64 {shape}")
    rho = np.random.default_rng(5).uniform(0.1, 1.0, shape)
    out = {}
    for prec in (pkg.FP64, pkg.MIXED):
        grp = _group(pkg, shape, precision=prec)
        f, grad, its = grp.topopt_eval(rho, T, eta=0.01, tol=1e-10)
        out[prec] = (f, grad.cpu().numpy())
        grp.close()
    (f64, g64), (f32, g32) = out[pkg.FP64], out[pkg.MIXED]
    assert f32[0] == pytest.approx(f64[0], rel=1e-8)
    assert np.abs(g32 - g64).max() <= 1e-6 * np.abs(g64).max()


def test_argument_checks():
    pkg = _pkg()
    say("topopt argument checks")
    rho = np.full((16, 16), 0.5)
    for kw in (dict(batch=3), dict(batch=2, element="tri")):
        grp = pkg.Cell((16, 16), pc=pkg.PC_GREEN_JACOBI, **kw)
        with pytest.raises(pkg.JfftError):
            grp.topopt_eval(rho, T)
        grp.close()
    grp = _group(pkg, (16, 16))
    with pytest.raises(pkg.JfftError):
        grp.topopt_eval(rho, T, eta=0.0)
    with pytest.raises(pkg.JfftError):
        grp.topopt_lbfgs(rho, T, 2, m=0)
    grp.close()


def test_full_size_phase_field_part():
    """The bench size (256^2): the phase-field part of the objective against
    the oracle (the mechanical part's solves are checked on small grids)."""
    pkg = _pkg()
    n = 256
    say(f"topopt phase field full size {n}^2")
    rho = np.random.default_rng(0).uniform(0.0, 1.0, (n, n))
    grp = _group(pkg, (n, n))
    f, grad, its = grp.topopt_eval(rho, T, eta=0.01, tol=1e-8, maxit=200000)
    grp.close()
    fpf, _ = to.phase_field(rho, 0.01)
    assert f[2] == pytest.approx(fpf, rel=1e-12)
    assert f[0] == pytest.approx(f[1] + f[2], rel=1e-15)


def test_full_size_lbfgs_properties():
    """The bench size (256^2), two L-BFGS steps: properties that hold at any
    size -- f decreases, the density stays in [0, 1], and the reported f and
    ||g||_inf are those of a fresh evaluation at the final density."""
    pkg = _pkg()
    n = 256
    say(f"topopt L-BFGS properties full size {n}^2")
    rho0 = np.random.default_rng(0).uniform(0.0, 1.0, (n, n))
    grp = _group(pkg, (n, n))
    rho, out = grp.topopt_lbfgs(rho0, T, 2, eta=0.01, tol=1e-8, maxit=200000)
    r = rho.cpu().numpy()
    f, grad, its = grp.topopt_eval(r, T, eta=0.01, tol=1e-8, maxit=200000)
    g = grad.cpu().numpy()
    grp.close()
    say(f"  steps={out['steps']} evals={out['evals']} f={out['f']} eval f={f[0]}")
    assert out["steps"] == 2
    assert out["f"][2] < out["f"][1] < out["f"][0]
    assert r.min() >= 0.0 and r.max() <= 1.0
    assert f[0] == pytest.approx(out["f"][-1], rel=1e-12)
    assert np.abs(g).max() == pytest.approx(out["gnorm"][-1], rel=1e-12)
    assert its == out["iters"][-1]
    fpf, _ = to.phase_field(r, 0.01)
    assert f[2] == pytest.approx(fpf, rel=1e-12)
