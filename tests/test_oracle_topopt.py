"""Pins of the topology-optimisation oracle (oracle/topopt.py) against facts
fixed by the mathematics, not by the oracle itself:

* phase field: zero for rho = 0 or 1; the double well's closed form for a
  constant field; the gradient term against the exact integral of a
  sampled sinusoid (P1 interpolation, O(h^2)); gradient = central
  differences of the energy;
* objective: sigma_bar_g . e_a symmetric in (g, a) (the homogenised
  stiffness is symmetric); a homogeneous density gives sigma_bar_g =
  rho C0 e_g and the gradient in closed form; the full gradient (mutual
  energy identity plus phase field) against central differences at tight
  solver tolerance;
* projected L-BFGS: the minimiser of an SPD quadratic inside the box, the
  clipped minimiser of a separable quadratic whose minimiser lies outside,
  and Rosenbrock's minimum (1, 1) on the box corner.
"""
import numpy as np
import pytest

import oracle
from oracle import topopt as to
from oracle import triangles as tri


def test_phase_field_closed_forms():
    eta = 0.01
    n = 16
    for c in (0.0, 1.0):
        f, g = to.phase_field(np.full((n, n), c), eta)
        assert f == 0.0 and np.abs(g).max() == 0.0
    c = 0.3
    f, g = to.phase_field(np.full((n, n), c), eta)
    cell = 1.0 / (n * n)
    assert f == pytest.approx(n * n * cell / eta * c * c * (1 - c) ** 2, rel=1e-14)
    assert np.allclose(g, cell / eta * 2 * c * (1 - c) * (1 - 2 * c), rtol=1e-14)
    # gradient term of rho = 0.5 + a sin(2 pi x): exact integral a^2 (2 pi)^2 / 2
    # (unit cell); the double well is removed by comparing two amplitudes
    for n in (32, 64):
        x = np.arange(n) / n
        res = []
        for a in (0.05, 0.1):
            rho = np.tile(0.5 + a * np.sin(2 * np.pi * x), (n, 1))
            f, _ = to.phase_field(rho, eta)
            fw = (1.0 / (n * n)) / eta * float((rho * rho * (1 - rho) ** 2).sum())
            res.append((f - fw) / eta)
        exact = [a * a * (2 * np.pi) ** 2 / 2 for a in (0.05, 0.1)]
        assert abs(res[1] - exact[1]) <= 2.0 * (2 * np.pi / n) ** 2 * exact[1]


def test_phase_field_gradient_is_derivative():
    rng = np.random.default_rng(0)
    rho = rng.uniform(0.1, 0.9, (6, 8))
    eta = 0.05
    f, g = to.phase_field(rho, eta, lengths=(1.0, 0.7))
    h = 1e-6
    for (i, j) in [(0, 0), (2, 5), (5, 7), (3, 1)]:
        rp, rm = rho.copy(), rho.copy()
        rp[i, j] += h
        rm[i, j] -= h
        fd = (to.phase_field(rp, eta, (1.0, 0.7))[0] - to.phase_field(rm, eta, (1.0, 0.7))[0]) / (2 * h)
        assert fd == pytest.approx(g[i, j], rel=1e-6, abs=1e-9 * abs(g).max())


def test_objective_homogeneous_closed_form():
    n = 8
    c = 0.6
    rho = np.full((n, n), c)
    ev = to.evaluate(rho, eta=0.01, tol=1e-12)
    C0 = tri.material(to.LAM0, to.MU0)
    assert np.allclose(ev.sigma_bar, c * C0, rtol=1e-12, atol=1e-14)
    assert ev.iters == [0, 0, 0]
    # f_sigma gradient: every pixel alike, d sigma_bar_g,a / d rho_e = C0_ga / N
    d = c * C0 - to.target_stresses()
    want = float((2 * d * C0).sum()) / (n * n)
    _, gpf = to.phase_field(rho, 0.01)
    assert np.allclose(ev.g - gpf, want, rtol=1e-12)


def test_homogenised_stiffness_symmetric_and_gradient_matches_differences():
    rng = np.random.default_rng(3)
    n = 8
    rho = rng.uniform(0.2, 0.95, (n, n))
    ev = to.evaluate(rho, eta=0.02, tol=1e-13)
    sb = ev.sigma_bar
    assert np.abs(sb - sb.T).max() <= 1e-10 * np.abs(sb).max()
    h = 1e-6
    for (i, j) in [(0, 0), (3, 4), (7, 2)]:
        rp, rm = rho.copy(), rho.copy()
        rp[i, j] += h
        rm[i, j] -= h
        fd = (to.evaluate(rp, eta=0.02, tol=1e-13).f - to.evaluate(rm, eta=0.02, tol=1e-13).f) / (2 * h)
        assert fd == pytest.approx(ev.g[i, j], rel=2e-5, abs=1e-8 * np.abs(ev.g).max())


def _quadratic(Q, b):
    def fun(x):
        g = Q @ x.ravel() - b
        return to.Eval(f=0.5 * float(x.ravel() @ Q @ x.ravel()) - float(b @ x.ravel()),
                       g=g.reshape(x.shape), f_sigma=0.0, f_pf=0.0, sigma_bar=None, iters=[])
    return fun


def test_lbfgs_quadratic_inside_and_outside_the_box():
    rng = np.random.default_rng(1)
    n = 12
    M = rng.standard_normal((n, n))
    Q = M @ M.T + n * np.eye(n)
    xs = rng.uniform(0.2, 0.8, n)
    res = to.lbfgs(_quadratic(Q, Q @ xs), np.full(n, 0.5), 60)
    assert np.abs(res.rho - xs).max() <= 1e-7
    # separable, minimiser partly outside [0, 1]: the clipped minimiser
    q = rng.uniform(1.0, 5.0, n)
    xs = rng.uniform(-0.5, 1.5, n)
    res = to.lbfgs(_quadratic(np.diag(q), q * xs), np.full(n, 0.5), 60)
    assert np.abs(res.rho - np.clip(xs, 0, 1)).max() <= 1e-7
    assert all(b <= a + 1e-15 for a, b in zip(res.f, res.f[1:]))  # monotone


def test_lbfgs_rosenbrock_corner():
    def fun(x):
        a, b = x
        f = (1 - a) ** 2 + 100 * (b - a * a) ** 2
        g = np.array([-2 * (1 - a) - 400 * a * (b - a * a), 200 * (b - a * a)])
        return to.Eval(f=f, g=g, f_sigma=f, f_pf=0.0, sigma_bar=None, iters=[])
    res = to.lbfgs(fun, np.array([0.2, 0.3]), 200)
    assert np.abs(res.rho - 1.0).max() <= 1e-6
