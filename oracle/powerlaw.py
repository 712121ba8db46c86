"""Plain FP64 numpy oracle of the nonlinear (power-law) example of Sec. 4:
Newton linearisation (Sec. 2.2, eq. lin_system) of a periodic 3D cell with
linear elastic inclusions in a power-law matrix, each linear system solved by
PCG with the same preconditioners as the linear problem.

TEST INFRASTRUCTURE ONLY: imported by tests/ and the benchmark's CPU
baseline.  The product library never imports it, and it imports nothing from
the product library.  The preconditioner application and the Green symbol are
the C oracle's (oracle.precond, oracle.green: Algorithm 1); everything else is
written out here, element by element (vectorised over elements), from the
definitions:

* trilinear hexahedra, 2 x 2 x 2 Gauss points, element e indexed by its lowest
  node, periodic (as for the linear problem);
* Mandel vectors (11, 22, 33, 23, 13, 12), shear entries sqrt2 eps_ij;
* matrix (phase 1): sigma = K tr(eps) I_M + g(eps_eq) e, e = dev(eps),
  eps_eq = sqrt(2/3 e.e), g(s) = sigma0 (2/3) s^(n-1) / eps0^n (the law of
  the nonlinear example, Sec. 4);
* inclusion (phase 0): sigma = K_i tr(eps) I_M + 2 mu_i e;
* tangent, derived from the law: C = K I_M (x) I_M + g P_dev
  + g (n - 1) e (x) e / (e.e)  (dg/ds = g (n-1)/s and d eps_eq = (2/3) e.d eps
  / eps_eq);
* Newton: f(u) = -B^T W sigma(E + B u); stop when ||f|| < eta; solve
  K(u) du = f(u) with PCG to max(pcg_tol ||f||, eta / 10) (no inner solve
  below the Newton tolerance), or to ||r||^2 <= pcg_tol (the absolute rule of
  Sec. 4); u += du.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

import oracle

SQ2 = np.sqrt(2.0)
IM = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])
PDEV = np.eye(6) - np.outer(IM, IM) / 3.0


@dataclass
class PowerLaw:
    K: float = 2.0        # bulk modulus of the matrix
    sigma0: float = 0.5   # reference shear stress
    eps0: float = 0.1     # reference strain
    n: float = 5.0        # exponent
    K_incl: float = 2.0   # inclusion bulk modulus
    mu_incl: float = 0.5  # inclusion shear modulus


# ----------------------------------------------------------- material law --
def _g(s, prm: PowerLaw):
    """g(s) = sigma0 (2/3) s^(n-1) / eps0^n, with g(0) = 0 for n > 1."""
    s = np.asarray(s, dtype=np.float64)
    if prm.n == 1.0:
        return np.full_like(s, prm.sigma0 * (2.0 / 3.0) / prm.eps0)
    with np.errstate(divide="ignore", invalid="ignore"):
        out = prm.sigma0 * (2.0 / 3.0) * np.power(s, prm.n - 1.0) / prm.eps0 ** prm.n
    return np.where(s > 0, out, 0.0)


def _split(eps):
    """trace, deviator (Mandel), equivalent strain; eps has Mandel axis first."""
    tr = eps[0] + eps[1] + eps[2]
    e = eps - IM.reshape((6,) + (1,) * (eps.ndim - 1)) * tr / 3.0
    ee = (e * e).sum(axis=0)
    return tr, e, ee, np.sqrt(2.0 / 3.0 * ee)


def stress(eps, phase, prm: PowerLaw):
    """sigma(eps) per point; eps (6, ...), phase (...) in {0, 1}."""
    tr, e, ee, seq = _split(eps)
    Im = IM.reshape((6,) + (1,) * (eps.ndim - 1))
    s_m = prm.K * tr * Im + _g(seq, prm) * e
    s_i = prm.K_incl * tr * Im + 2.0 * prm.mu_incl * e
    return np.where(phase > 0.5, s_m, s_i)


def tangent_apply(eps, deps, phase, prm: PowerLaw):
    """C(eps) deps per point."""
    tr, e, ee, seq = _split(eps)
    dtr, de, _, _ = _split(deps)
    Im = IM.reshape((6,) + (1,) * (eps.ndim - 1))
    g = _g(seq, prm)
    with np.errstate(divide="ignore", invalid="ignore"):
        h = np.where(ee > 0, g * (prm.n - 1.0) / ee, 0.0)
    edot = (e * deps).sum(axis=0)
    s_m = prm.K * dtr * Im + g * de + h * edot * e
    s_i = prm.K_incl * dtr * Im + 2.0 * prm.mu_incl * de
    return np.where(phase > 0.5, s_m, s_i)


def tangent_matrix(eps, phase, prm: PowerLaw):
    """6 x 6 tangent at one point (eps (6,), phase scalar)."""
    eps = np.asarray(eps, dtype=np.float64)
    return np.stack([tangent_apply(eps, np.eye(6)[j], np.asarray(phase), prm) for j in range(6)],
                    axis=1)


# -------------------------------------------------------- discretisation --
def gauss_B(h):
    """B_q (6 x 24, dofs ordered [component][corner], corner c = cx + 2 cy + 4 cz)
    at the 8 Gauss points q = gx + 2 gy + 4 gz, and the Gauss weight vol/8."""
    hx, hy, hz = h
    xi = [0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)]
    Bs = []
    for q in range(8):
        gq = (q & 1, (q >> 1) & 1, q >> 2)
        p = [xi[gq[0]], xi[gq[1]], xi[gq[2]]]
        dN = np.zeros((3, 8))  # dN_c / dx_a
        for c in range(8):
            cc = (c & 1, (c >> 1) & 1, c >> 2)
            val = [p[a] if cc[a] else 1.0 - p[a] for a in range(3)]
            for a in range(3):
                sgn = 1.0 if cc[a] else -1.0
                other = np.prod([val[b] for b in range(3) if b != a])
                dN[a, c] = sgn * other / (hx, hy, hz)[a]
        B = np.zeros((6, 24))
        X, Y, Z = 0, 8, 16  # offsets of u_x, u_y, u_z
        B[0, X:X + 8] = dN[0]
        B[1, Y:Y + 8] = dN[1]
        B[2, Z:Z + 8] = dN[2]
        B[3, Y:Y + 8] = dN[2] / SQ2
        B[3, Z:Z + 8] = dN[1] / SQ2
        B[4, X:X + 8] = dN[2] / SQ2
        B[4, Z:Z + 8] = dN[0] / SQ2
        B[5, X:X + 8] = dN[1] / SQ2
        B[5, Y:Y + 8] = dN[0] / SQ2
        Bs.append(B)
    return np.array(Bs), hx * hy * hz / 8.0


def _gather(u):
    """(3, nz, ny, nx) nodal field -> (24, nz, ny, nx) corner values per element."""
    out = []
    for i in range(3):
        for c in range(8):
            cx, cy, cz = c & 1, (c >> 1) & 1, c >> 2
            out.append(np.roll(u[i], shift=(-cz, -cy, -cx), axis=(0, 1, 2)))
    return np.array(out)


def _scatter(ye):
    """(24, nz, ny, nx) element corner forces -> (3, nz, ny, nx) nodal sums."""
    shape = ye.shape[1:]
    f = np.zeros((3,) + shape)
    for i in range(3):
        for c in range(8):
            cx, cy, cz = c & 1, (c >> 1) & 1, c >> 2
            f[i] += np.roll(ye[8 * i + c], shift=(cz, cy, cx), axis=(0, 1, 2))
    return f


def _h(shape, lengths):
    nz, ny, nx = shape
    L = (1.0, 1.0, 1.0) if lengths is None else lengths
    return (L[0] / nx, L[1] / ny, L[2] / nz)


def strains(u, macro, lengths=None):
    """eps at the Gauss points: (8, 6, nz, ny, nx) = macro + B_q u_e."""
    B, _ = gauss_B(_h(u.shape[1:], lengths))
    ue = _gather(u)
    eps = np.einsum("qij,j...->qi...", B, ue)
    return eps + np.asarray(macro, dtype=np.float64).reshape((1, 6) + (1,) * 3)


def force(u, macro, phase, prm: PowerLaw, lengths=None):
    """Newton right-hand side f(u) = -B^T W sigma(E + B u) (eq. lin_system)."""
    B, w = gauss_B(_h(u.shape[1:], lengths))
    eps = strains(u, macro, lengths)
    ye = np.zeros((24,) + u.shape[1:])
    for q in range(8):
        ye += np.einsum("ij,i...->j...", B[q], stress(eps[q], phase, prm))
    return -w * _scatter(ye)


def tangent_op(u, p, macro, phase, prm: PowerLaw, lengths=None):
    """K(u) p = B^T W C(E + B u) B p."""
    B, w = gauss_B(_h(u.shape[1:], lengths))
    eps = strains(u, macro, lengths)
    pe = _gather(p)
    ye = np.zeros((24,) + u.shape[1:])
    for q in range(8):
        dq = np.einsum("ij,j...->i...", B[q], pe)
        ye += np.einsum("ij,i...->j...", B[q], tangent_apply(eps[q], dq, phase, prm))
    return w * _scatter(ye)


def at_nodes(u, p, macro, phase, prm: PowerLaw, nodes, lengths=None):
    """Force f, tangent action K(u) p and diag(K(u)) at the listed nodes only
    (flat indices into (nz, ny, nx)), from the 8 elements around each: node I
    is corner o of element I - o; the element's force, tangent action and
    diagonal entries at that corner are summed over o.  For checks on grids
    too large for the whole-field functions above."""
    shape = u.shape[1:]
    nz, ny, nx = shape
    nodes = np.asarray(nodes)
    z, rem = np.divmod(nodes, nx * ny)
    y, x = np.divmod(rem, nx)
    Bq, w = gauss_B(_h(shape, lengths))
    mac = np.asarray(macro, dtype=float).reshape(6, 1)
    S = nodes.size
    f = np.zeros((3, S))
    kp = np.zeros((3, S))
    dg = np.zeros((3, S))
    for o in range(8):
        ox, oy, oz = o & 1, (o >> 1) & 1, o >> 2
        ex, ey, ez = (x - ox) % nx, (y - oy) % ny, (z - oz) % nz
        ue = np.empty((24, S))
        pe = np.empty((24, S))
        for i in range(3):
            for c in range(8):
                cx, cy, cz = c & 1, (c >> 1) & 1, c >> 2
                idx = (((ez + cz) % nz), ((ey + cy) % ny), ((ex + cx) % nx))
                ue[8 * i + c] = u[i][idx]
                pe[8 * i + c] = p[i][idx]
        ph = phase[ez, ey, ex]
        for q in range(8):
            B = Bq[q]
            eps = B @ ue + mac
            sig = stress(eps, ph, prm)
            tp = tangent_apply(eps, B @ pe, ph, prm)
            for i in range(3):
                col = B[:, 8 * i + o]
                f[i] -= w * (col @ sig)
                kp[i] += w * (col @ tp)
                cd = tangent_apply(eps, np.repeat(col[:, None], S, axis=1), ph, prm)
                dg[i] += w * (col @ cd)
    return f, kp, dg


def stress_average(u, macro, phase, prm: PowerLaw, lengths=None):
    """sigma_bar = sum_e sum_q w sigma_q / |Y|."""
    eps = strains(u, macro, lengths)
    s = np.zeros(6)
    for q in range(8):
        s += stress(eps[q], phase, prm).reshape(6, -1).sum(axis=1)
    return s / (8.0 * phase.size)


def jacobi_diag(u, macro, phase, prm: PowerLaw, lengths=None):
    """Algorithm 2 on K(u): d 2^d applications to unit combs."""
    shape = u.shape[1:]
    nz, ny, nx = shape
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    diag = np.zeros((3,) + shape)
    for a in range(3):
        for o in range(8):
            ox, oy, oz = o & 1, (o >> 1) & 1, o >> 2
            mask = ((xx & 1) == ox) & ((yy & 1) == oy) & ((zz & 1) == oz)
            comb = np.zeros((3,) + shape)
            comb[a][mask] = 1.0
            Kc = tangent_op(u, comb, macro, phase, prm, lengths)
            diag[a][mask] = Kc[a][mask]
    return diag


# ------------------------------------------------------------- solvers ----
def _ulp_noise(rng):
    """One-ulp moves of every nonzero entry in seeded random directions (the
    C oracle's rounding-difference model for parity windows); identity when
    rng is None."""
    def noisy(x):
        if rng is None:
            return x
        up = rng.random(x.shape) < 0.5
        moved = np.where(up, np.nextafter(x, np.inf), np.nextafter(x, -np.inf))
        return np.where(x == 0.0, 0.0, moved)
    return noisy


def pcg(Kop, f, pc, diag=None, G=None, tol=1e-8, maxit=5000, noise=None):
    """Textbook PCG on K du = f from du = 0, stop at ||r|| <= tol ||f||
    (recursive residual); the preconditioner is oracle.precond.  noise: a
    function applied to every K p and M^-1 r result (rounding-difference
    model), or None."""
    if noise is None:
        noise = _ulp_noise(None)
    x = np.zeros_like(f)
    r = f.copy()
    fn = np.linalg.norm(f)
    if fn == 0.0:
        return x, 0
    z = noise(oracle.precond(pc, r, diag=diag, G=G)[0])
    p = z.copy()
    rz = float((r * z).sum())
    for k in range(maxit):
        q = noise(Kop(p))
        pq = float((p * q).sum())
        if not pq > 0.0:  # breakdown (nothing left that the preconditioner sees)
            return x, k
        alpha = rz / pq
        x += alpha * p
        r -= alpha * q
        if np.linalg.norm(r) <= tol * fn:
            return x, k + 1
        z = noise(oracle.precond(pc, r, diag=diag, G=G)[0])
        rz_new = float((r * z).sum())
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, maxit


@dataclass
class NewtonResult:
    u: np.ndarray
    sigma_bar: np.ndarray
    res: list = field(default_factory=list)      # ||f(u^(i))||, i = 0, 1, ...
    pcg_iters: list = field(default_factory=list)
    converged: bool = False


def newton(phase, macro, prm: PowerLaw, pc=oracle.PC_GREEN_JACOBI, newton_tol=1e-5,
           pcg_tol=1e-8, max_newton=20, maxit=5000, lam_ref=None, mu_ref=None, lengths=None,
           pcg_absolute=False, noise_seed=0):
    """Newton with PCG inner solves from u^(0) = 0 (Sec. 2.2); the Green
    reference material defaults to the inclusion's.  pcg_absolute: the inner
    solve stops at ||r||^2 <= pcg_tol (the stopping rule of Sec. 4) instead
    of the relative rule with the inexact-Newton floor.  noise_seed != 0
    turns on the rounding-difference model in every PCG solve."""
    noise = _ulp_noise(np.random.default_rng(noise_seed) if noise_seed else None)
    shape = phase.shape
    if lam_ref is None:
        lam_ref, mu_ref = prm.K_incl - 2.0 * prm.mu_incl / 3.0, prm.mu_incl
    G = oracle.green(shape, lam_ref, mu_ref, lengths) if pc in (oracle.PC_GREEN,
                                                                oracle.PC_GREEN_JACOBI) else None
    u = np.zeros((3,) + shape)
    out = NewtonResult(u=u, sigma_bar=np.zeros(6))
    for _ in range(max_newton + 1):
        f = force(u, macro, phase, prm, lengths)
        fn = float(np.linalg.norm(f))
        out.res.append(fn)
        if fn < newton_tol:
            out.converged = True
            break
        if len(out.pcg_iters) == max_newton:
            break
        diag = None
        if pc in (oracle.PC_JACOBI, oracle.PC_GREEN_JACOBI):
            diag = jacobi_diag(u, macro, phase, prm, lengths)
        if pcg_absolute:
            rtol = np.sqrt(pcg_tol) / fn
        else:
            # inexact Newton: no inner solve below a tenth of the Newton tolerance
            rtol = max(pcg_tol, 0.1 * newton_tol / fn)
        du, k = pcg(lambda p: tangent_op(u, p, macro, phase, prm, lengths), f, pc, diag, G,
                    rtol, maxit, noise)
        out.pcg_iters.append(k)
        u = u + du
    out.u = u
    out.sigma_bar = stress_average(u, macro, phase, prm, lengths)
    return out
