"""Pins of the power-law (nonlinear example) oracle, against facts fixed by
the law and the discretisation, not by the oracle itself:

* the law's linear limit (n = 1) and closed forms of sigma for pure shear;
* the tangent is the derivative of the law (central differences), symmetric,
  positive definite;
* with n = 1 and equal phases, the nonlinear force and tangent operator equal
  the C oracle's linear operators (independent code: its own element loop,
  B matrices and Gauss rule);
* the tangent operator is the derivative of the force (central differences);
* Algorithm 2 on the tangent operator equals the diagonal of the dense
  tangent matrix; the dense matrix is symmetric;
* Newton: one step in the linear limit, matching the C oracle's linear solve;
  zero steps on a homogeneous matrix, with sigma_bar = sigma(E); quadratic
  convergence on the power-law problem.
"""
import numpy as np
import pytest

import jfft_inputs as ji
import oracle
from oracle import powerlaw as pl

PRM = pl.PowerLaw()


def _linear_prm():
    # n = 1: g = sigma0 (2/3) / eps0 = 2 mu; the inclusion given the same moduli
    mu = PRM.sigma0 / (3.0 * PRM.eps0)
    return pl.PowerLaw(K=PRM.K, sigma0=PRM.sigma0, eps0=PRM.eps0, n=1.0, K_incl=PRM.K,
                       mu_incl=mu), mu


def test_law_linear_limit_and_pure_shear():
    prm1, mu = _linear_prm()
    rng = np.random.default_rng(0)
    eps = rng.standard_normal((6, 5))
    s = pl.stress(eps, np.ones(5), prm1)
    tr = eps[:3].sum(axis=0)
    lin = prm1.K * tr * pl.IM[:, None] + 2 * mu * (eps - pl.IM[:, None] * tr / 3)
    assert np.allclose(s, lin, rtol=1e-14, atol=1e-14)
    # pure shear eps_12 = gamma/2: Mandel entry 6 = sqrt2 gamma/2, e.e = gamma^2/2,
    # eps_eq = gamma / sqrt3; sigma_6 = g(eps_eq) sqrt2 gamma / 2
    for gamma in (0.01, 0.1, 0.3):
        eps = np.zeros(6)
        eps[5] = np.sqrt(2) * gamma / 2
        seq = gamma / np.sqrt(3)
        g = PRM.sigma0 * (2 / 3) * seq ** (PRM.n - 1) / PRM.eps0 ** PRM.n
        s = pl.stress(eps, np.array(1.0), PRM)
        assert np.allclose(s, [0, 0, 0, 0, 0, g * eps[5]], rtol=1e-14, atol=1e-16)
    # hydrostatic strain: sigma = K tr I, no deviatoric stress
    eps = np.array([0.01, 0.01, 0.01, 0, 0, 0])
    assert np.allclose(pl.stress(eps, np.array(1.0), PRM), PRM.K * 0.03 * pl.IM, rtol=1e-14)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_tangent_is_derivative_symmetric_positive(seed):
    rng = np.random.default_rng(seed)
    eps = 0.05 * rng.standard_normal(6)
    C = pl.tangent_matrix(eps, 1.0, PRM)
    h = 1e-6
    for j in range(6):
        d = np.zeros(6)
        d[j] = h
        fd = (pl.stress(eps + d, np.array(1.0), PRM) - pl.stress(eps - d, np.array(1.0), PRM)) / (2 * h)
        assert np.allclose(C[:, j], fd, rtol=1e-6, atol=1e-9 * np.abs(C).max())
    assert np.allclose(C, C.T, atol=1e-13 * np.abs(C).max())
    assert np.linalg.eigvalsh(C).min() > 0
    Ci = pl.tangent_matrix(eps, 0.0, PRM)  # inclusion: K I(x)I + 2 mu P_dev
    assert np.allclose(Ci, PRM.K_incl * np.outer(pl.IM, pl.IM) + 2 * PRM.mu_incl * pl.PDEV,
                       atol=1e-14)


@pytest.mark.parametrize("shape", [(4, 4, 4), (6, 4, 8)])
def test_linear_limit_equals_c_oracle(shape):
    prm1, mu = _linear_prm()
    lam = prm1.K - 2 * mu / 3
    rng = np.random.default_rng(4)
    u = rng.standard_normal((3,) + shape)
    p = rng.standard_normal((3,) + shape)
    macro = rng.uniform(-0.1, 0.1, 6)
    phase = (rng.random(shape) > 0.5).astype(float)  # both phases carry the same law
    E1 = np.ones(shape)
    f = pl.force(u, macro, phase, prm1)
    ref = oracle.rhs(E1, macro, lam, mu) - oracle.stiffness(E1, u, lam, mu)
    assert np.abs(f - ref).max() <= 1e-12 * np.abs(ref).max()
    Kp = pl.tangent_op(u, p, macro, phase, prm1)
    assert np.abs(Kp - oracle.stiffness(E1, p, lam, mu)).max() <= 1e-12 * np.abs(Kp).max()


def test_tangent_operator_is_derivative_of_force():
    shape = (4, 4, 4)
    rng = np.random.default_rng(5)
    phase = (rng.random(shape) > 0.3).astype(float)
    macro = np.array([0, 0, 0, 0, 0, 0.05 * np.sqrt(2)])
    u = 0.02 * rng.standard_normal((3,) + shape)
    p = rng.standard_normal((3,) + shape)
    h = 1e-6
    fd = -(pl.force(u + h * p, macro, phase, PRM) - pl.force(u - h * p, macro, phase, PRM)) / (2 * h)
    Kp = pl.tangent_op(u, p, macro, phase, PRM)
    assert np.abs(Kp - fd).max() <= 1e-6 * np.abs(Kp).max()


def test_alg2_on_tangent_equals_dense_diagonal():
    shape = (4, 4, 4)
    rng = np.random.default_rng(6)
    phase = (rng.random(shape) > 0.4).astype(float)
    macro = np.array([0.01, -0.02, 0, 0, 0.03, 0.05])
    u = 0.02 * rng.standard_normal((3,) + shape)
    n = 3 * np.prod(shape)
    K = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        K[:, j] = pl.tangent_op(u, e.reshape((3,) + shape), macro, phase, PRM).ravel()
    assert np.abs(K - K.T).max() <= 1e-12 * np.abs(K).max()
    d = pl.jacobi_diag(u, macro, phase, PRM)
    assert np.abs(d.ravel() - np.diag(K)).max() <= 1e-13 * np.abs(K).max()


def test_newton_linear_limit_one_step_matches_c_oracle():
    """n = 1 with an inclusion of proportional moduli (t times the matrix's):
    a heterogeneous linear problem, which the C oracle solves with E = 1 in the
    matrix and t in the inclusions; Newton takes one step."""
    prm1, mu = _linear_prm()
    t = 10.0
    prm1.K_incl, prm1.mu_incl = t * prm1.K, t * mu
    lam = prm1.K - 2 * mu / 3
    shape = (8, 8, 8)
    incl = ji.spherical_inclusions(shape, 2, 0.2, seed=1)
    phase = 1.0 - incl
    macro = np.array([0, 0, 0, 0, 0, 0.05 * np.sqrt(2)])
    res = pl.newton(phase, macro, prm1, newton_tol=1e-13, pcg_tol=1e-12)
    assert res.converged and len(res.pcg_iters) == 1, (res.res, res.pcg_iters)
    E = 1.0 + (t - 1.0) * incl
    ref = oracle.solve(E, macro, lam, mu, pc=oracle.PC_GREEN_JACOBI, tol=1e-12, maxit=5000)
    u = res.u - res.u.reshape(3, -1).mean(axis=1).reshape(3, 1, 1, 1)
    assert np.abs(u - ref.u).max() <= 1e-9 * np.abs(ref.u).max()
    np.testing.assert_allclose(res.sigma_bar, ref.sigma_bar, rtol=1e-10, atol=1e-14)


def test_newton_homogeneous_matrix_zero_steps():
    shape = (6, 6, 6)
    phase = np.ones(shape)
    macro = np.array([0.01, 0, -0.01, 0, 0, 0.05 * np.sqrt(2)])
    res = pl.newton(phase, macro, PRM)
    assert res.converged and res.pcg_iters == [] and res.res[0] < 1e-12
    np.testing.assert_allclose(res.sigma_bar, pl.stress(macro, np.array(1.0), PRM), rtol=1e-13)


def test_newton_power_law_converges_quadratically():
    shape = (8, 8, 8)
    phase = 1.0 - ji.spherical_inclusions(shape, 2, 0.2, seed=3)
    macro = np.array([0, 0, 0, 0, 0, 0.05 * np.sqrt(2)])
    res = pl.newton(phase, macro, PRM, newton_tol=1e-11, pcg_tol=1e-12)
    r = np.array(res.res)
    assert res.converged and len(res.pcg_iters) >= 3
    assert np.all(np.diff(r) < 0)
    # quadratic phase: ||f_{i+1}|| / ||f_i||^2 stays bounded while ||f|| falls
    # by orders of magnitude
    q = r[2:] / r[1:-1] ** 2
    assert r[-1] < 1e-6 * r[1] and q.max() < 1e3 * max(q.min(), 1e-3) + 1e6
    assert r[-1] / r[-2] < 1e-2


def test_newton_absolute_inner_rule_equals_relative_rule_at_same_threshold():
    """The absolute inner rule ||r||^2 <= t stops where the relative rule
    ||r|| <= (sqrt(t) / ||f||) ||f|| does: one linear-limit step, same PCG
    iterations and result for t = (1e-9 ||f_0||)^2."""
    prm1, mu = _linear_prm()
    prm1.K_incl, prm1.mu_incl = 10 * prm1.K, 10 * mu
    shape = (8, 8, 8)
    phase = 1.0 - ji.spherical_inclusions(shape, 2, 0.2, seed=1)
    macro = np.array([0, 0, 0, 0, 0, 0.05 * np.sqrt(2)])
    f0 = np.linalg.norm(pl.force(np.zeros((3,) + shape), macro, phase, prm1))
    rel = pl.newton(phase, macro, prm1, newton_tol=1e-30, pcg_tol=1e-9, max_newton=1)
    ab = pl.newton(phase, macro, prm1, newton_tol=1e-30, pcg_tol=(1e-9 * f0) ** 2, max_newton=1,
                   pcg_absolute=True)
    assert rel.pcg_iters == ab.pcg_iters and rel.pcg_iters[0] > 3
    assert np.abs(rel.u - ab.u).max() <= 1e-12 * np.abs(rel.u).max()


def test_at_nodes_equals_whole_field_functions():
    """The sampled-node evaluation (for large grids) equals the whole-field
    force, tangent action and Algorithm 2 diagonal at every node."""
    shape = (4, 6, 4)
    rng = np.random.default_rng(9)
    phase = (rng.random(shape) > 0.4).astype(float)
    macro = rng.uniform(-0.05, 0.05, 6)
    u = 0.02 * rng.standard_normal((3,) + shape)
    p = rng.standard_normal((3,) + shape)
    L = (1.0, 1.3, 0.8)
    nodes = np.arange(int(np.prod(shape)))
    f, kp, dg = pl.at_nodes(u, p, macro, phase, PRM, nodes, L)
    ff = pl.force(u, macro, phase, PRM, L).reshape(3, -1)
    kk = pl.tangent_op(u, p, macro, phase, PRM, L).reshape(3, -1)
    dd = pl.jacobi_diag(u, macro, phase, PRM, L).reshape(3, -1)
    assert np.abs(f - ff).max() <= 1e-13 * np.abs(ff).max()
    assert np.abs(kp - kk).max() <= 1e-13 * np.abs(kk).max()
    assert np.abs(dg - dd).max() <= 1e-13 * np.abs(dd).max()
