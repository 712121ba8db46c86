"""Pins of the linear-triangle oracle (oracle/triangles.py) against facts
fixed by the discretisation and the mathematics, not by the oracle itself:

* element: symmetric, positive semi-definite, null space = the three rigid
  modes; constant strain = sym(G) for an affine displacement G x (patch test);
* homogeneous material: f = 0, zero iterations, sigma_bar = C macro;
* laminate: the layered closed form, which P1 reproduces exactly (the exact
  displacement is piecewise linear with kinks on element edges);
* Algorithm 1: K^(k) equals the action of the assembled K on Fourier modes,
  G^ K^ = I for k != 0; real symmetric (the split is symmetric under the
  point reflection x -> -x) but its coupling block is not odd in ky alone,
  unlike the quadrilateral's (no symmetry under the reflection of one axis);
* Algorithm 2 equals the diagonal of the dense assembled K;
* PCG equals a dense bordered (zero-mean) direct solve on small grids.
"""
import numpy as np
import pytest

import jfft_inputs as ji
import oracle
from oracle import triangles as tri

LAM, MU = oracle.lame_from_nu(0.3)


def _dense(E, lengths=None):
    n = 2 * E.size
    K = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        K[:, j] = tri.stiffness(E, e.reshape((2,) + E.shape), LAM, MU, lengths).ravel()
    return K


@pytest.mark.parametrize("h", [(1.0, 1.0), (0.5, 1.3)])
def test_element_symmetric_psd_rigid_null_space_patch(h):
    Ke = tri.element_matrix(h, LAM, MU)
    assert np.abs(Ke - Ke.T).max() <= 1e-14 * np.abs(Ke).max()
    w = np.linalg.eigvalsh(Ke)
    assert w.min() > -1e-13 * w.max()
    assert (w > 1e-10 * w.max()).sum() == 5  # 8 dofs - 3 rigid modes
    xs = np.array([c[0] * h[0] for c in tri.CORNERS])
    ys = np.array([c[1] * h[1] for c in tri.CORNERS])
    rigid = [np.r_[np.ones(4), np.zeros(4)], np.r_[np.zeros(4), np.ones(4)], np.r_[-ys, xs]]
    for v in rigid:
        assert np.abs(Ke @ v).max() <= 1e-13 * np.abs(Ke).max()
    # patch test: u = G x gives the strain sym(G) in both triangles
    rng = np.random.default_rng(0)
    G = rng.standard_normal((2, 2))
    ue = np.r_[G[0, 0] * xs + G[0, 1] * ys, G[1, 0] * xs + G[1, 1] * ys]
    Bs, A = tri.triangle_B(h)
    want = np.array([G[0, 0], G[1, 1], np.sqrt(2) * 0.5 * (G[0, 1] + G[1, 0])])
    for B in Bs:
        assert np.allclose(B @ ue, want, rtol=1e-14, atol=1e-14)
    assert A == pytest.approx(0.5 * h[0] * h[1], rel=1e-15)


def test_homogeneous_material():
    E = np.full((8, 12), 3.0)
    macro = np.array([0.3, -0.2, 0.5])
    f, fa = tri.rhs(E, macro, LAM, MU, with_abs=True)
    assert np.abs(f).max() <= 1e-14 * np.abs(fa).max()
    res = tri.solve(E, macro, LAM, MU)
    assert res.iters == 0 and np.abs(res.u).max() == 0.0
    np.testing.assert_allclose(res.sigma_bar, 3.0 * tri.material(LAM, MU) @ macro, rtol=1e-14)


@pytest.mark.parametrize("axis", [0, 1])
def test_laminate_closed_form(axis):
    """Layers of E normal to x (axis 0) or y (axis 1): traction continuity
    and compatibility give sigma_bar in closed form (plane strain)."""
    n = 16
    rng = np.random.default_rng(3)
    layers = rng.uniform(1.0, 50.0, n)
    E = np.tile(layers, (n, 1)) if axis == 0 else np.tile(layers[:, None], (1, n))
    macro = np.array([0.01, -0.02, 0.03])
    res = tri.solve(E, macro, LAM, MU, pc=oracle.PC_GREEN_JACOBI, tol=1e-13)
    # layer-normal direction nn, in-plane direction tt
    nn, tt = (0, 1) if axis == 0 else (1, 0)
    en, et, g = macro[nn], macro[tt], macro[2] * np.sqrt(2)
    lam, mu = LAM * layers, MU * layers
    l2m = lam + 2 * mu
    snn = (en + np.mean(lam / l2m) * et) / np.mean(1.0 / l2m)
    enl = (snn - lam * et) / l2m  # normal strain of each layer
    stt = np.mean(lam * enl + l2m * et)
    s12 = g / np.mean(1.0 / mu)
    want = np.zeros(3)
    want[nn], want[tt], want[2] = snn, stt, np.sqrt(2) * s12
    np.testing.assert_allclose(res.sigma_bar, want, rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("lengths", [None, (1.0, 0.6)])
def test_algorithm1_symbol_is_fourier_action(lengths):
    shape = (6, 10)
    ny, nx = shape
    G = tri.green(shape, LAM, MU, lengths)
    ones = np.ones(shape)
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    for ky, kx in [(0, 1), (1, 0), (1, 1), (2, 3), (5, 7), (3, 5)]:
        ph = np.exp(2j * np.pi * (kx * xx / nx + ky * yy / ny))
        Kh = np.empty((2, 2), dtype=complex)
        for a in range(2):
            v = np.zeros((2,) + shape, dtype=complex)
            v[a] = ph
            Kv = (tri.stiffness(ones, v.real, LAM, MU, lengths)
                  + 1j * tri.stiffness(ones, v.imag, LAM, MU, lengths))
            Kh[:, a] = (Kv / ph).mean(axis=(1, 2))
            assert np.abs(Kv - Kh[:, a].reshape(2, 1, 1) * ph).max() <= 1e-12 * np.abs(Kv).max()
        Gk = G[:, :, ky, kx]
        assert np.abs(Gk @ Kh - np.eye(2)).max() <= 1e-12
        assert np.abs(Gk - Gk.T).max() <= 1e-12 * np.abs(Gk).max()
        assert np.abs(Gk.imag).max() <= 1e-12 * np.abs(Gk).max()
    assert np.abs(G[:, :, 0, 0]).max() == 0.0
    # coupling block at (kx, ky) and (kx, -ky): opposite for quadrilaterals
    # (odd in each wavenumber), not for the triangles
    Kp = np.linalg.inv(G[:, :, 1, 2].real)
    Km = np.linalg.inv(G[:, :, ny - 1, 2].real)
    assert abs(Kp[0, 1] + Km[0, 1]) > 1e-2 * abs(Kp[0, 1])


def test_algorithm2_equals_dense_diagonal():
    E = ji.uniform_random_field((6, 8), 1.0, 100.0, seed=4)
    d = tri.jacobi_diag(E, LAM, MU)
    K = _dense(E)
    assert np.abs(K - K.T).max() <= 1e-13 * np.abs(K).max()
    assert np.abs(d.ravel() - np.diag(K)).max() <= 1e-14 * np.abs(K).max()


@pytest.mark.parametrize("pc", [oracle.PC_GREEN, oracle.PC_GREEN_JACOBI, oracle.PC_JACOBI,
                                oracle.PC_NONE])
def test_pcg_equals_dense_bordered_solve(pc):
    shape = (4, 6)
    E = ji.uniform_random_field(shape, 1.0, 30.0, seed=5)
    macro = np.array([0.2, -0.1, 0.4])
    K = _dense(E)
    f = tri.rhs(E, macro, LAM, MU).ravel()
    n = f.size
    # zero mean per component as the bordering constraint
    Cm = np.zeros((2, n))
    Cm[0, : n // 2] = 1.0
    Cm[1, n // 2:] = 1.0
    Kb = np.block([[K, Cm.T], [Cm, np.zeros((2, 2))]])
    ub = np.linalg.solve(Kb, np.r_[f, 0.0, 0.0])[:n]
    res = tri.solve(E, macro, LAM, MU, pc=pc, tol=1e-13)
    assert res.status == "ok"
    assert np.abs(res.u.ravel() - ub).max() <= 1e-10 * np.abs(ub).max()
    assert res.relres_true <= 1e-12
