"""Plain FP64 numpy oracle of the phase-field topology optimisation of Sec. 4
(the workload of eq. aim_fun and eq. lin_system_topopt), on the paper's 2D
element (two linear triangles per pixel, oracle/triangles.py).

TEST INFRASTRUCTURE ONLY: imported by tests/.  The product library never
imports it, and it imports nothing from the product library.

What is computed, written out from the definitions:

* material C(rho) = rho C0 (Sec. 4: lambda0 = 2/3, mu0 = 1/2), rho sampled at
  the nodes and assigned to the pixel whose lowest node it is;
* three load cases macro_g = e_g (Mandel unit vectors), each solved from
  u = 0 by PCG (the triangle oracle's solver);
* f_sigma(rho) = sum_g || sigma_bar_g(rho) - t_g ||^2, t_g = C_target e_g,
  C_target isotropic with K = 0.025, mu = 0.15 (lambda = K - 2 mu / 3);
* its gradient by the classical mutual-energy identity: with the local
  strains eps_g = e_g + B u_g of the exact solutions, sigma_bar_g . e_a =
  (1/|Y|) sum_e sum_t A eps_a^T C(rho_e) eps_g, and the derivative in rho_e
  is that element's term with C0 (no extra solve: the adjoint of load case
  a is load case a itself);
* the phase-field term f_pf = eta int |grad rho|^2 + (1/eta) int rho^2
  (1 - rho)^2 with rho interpolated linearly on the triangles for the
  gradient term and the double well integrated by nodal quadrature (each
  node carries one pixel's area) -- the paper does not give its
  discretisation;
* L-BFGS (two-loop recursion, memory m) projected on the box [0, 1]: the
  variables held at a bound by their gradient (rho = 0 with g > 0, rho = 1
  with g < 0) are frozen for the step (their gradient entries are zeroed
  before the recursion and their direction entries after it); the trial
  point clip(rho + alpha d) with alpha halved from 1 until the Armijo
  condition f(trial) <= f + c1 g . (trial - rho) holds; a pair (s, y) is
  kept when y . s > 1e-12 ||s|| ||y||; the first direction is -g scaled to a
  largest entry of 0.1, later ones use H0 = s.y / y.y of the newest pair;
  the iteration stops early when no halving gives a decrease.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

import oracle
from oracle import triangles as tri

LAM0, MU0 = 2.0 / 3.0, 0.5
K_TARGET, MU_TARGET = 0.025, 0.15


def target_stresses(K=K_TARGET, mu=MU_TARGET):
    """t_g = C_target e_g (rows), plane-strain Mandel C of (lambda, mu)."""
    return tri.material(K - 2.0 * mu / 3.0, mu)


def _grad_tri(shape, lengths):
    """Corner gradients of the two triangles of a pixel (as in triangles.py)."""
    hx, hy = tri._h(shape, lengths)
    Bs, A = tri.triangle_B((hx, hy))
    # scalar gradient rows: the x and y derivative of each corner's shape function
    G = []
    for B in Bs:
        gx = B[0, 0:4]
        gy = B[1, 4:8]
        G.append(np.stack([gx, gy]))  # [2, 4]
    return G, A, hx * hy


def _gather1(r):
    return np.stack([np.roll(r, shift=(-cy, -cx), axis=(0, 1)) for (cx, cy) in tri.CORNERS])


def _scatter1(ye):
    out = np.zeros(ye.shape[1:])
    for c, (cx, cy) in enumerate(tri.CORNERS):
        out += np.roll(ye[c], shift=(cy, cx), axis=(0, 1))
    return out


def phase_field(rho, eta, lengths=None):
    """f_pf and its gradient in the nodal values."""
    G, A, cell = _grad_tri(rho.shape, lengths)
    re = _gather1(rho)  # [4, ny, nx]
    f = 0.0
    ge = np.zeros_like(re)
    for Gt in G:
        grad = np.einsum("dc,c...->d...", Gt, re)  # [2, ny, nx]
        f += eta * A * float((grad * grad).sum())
        ge += 2.0 * eta * A * np.einsum("dc,d...->c...", Gt, grad)
    g = _scatter1(ge)
    w = rho * rho * (1.0 - rho) ** 2
    f += cell / eta * float(w.sum())
    g += cell / eta * 2.0 * rho * (1.0 - rho) * (1.0 - 2.0 * rho)
    return f, g


@dataclass
class Eval:
    f: float
    g: np.ndarray
    f_sigma: float
    f_pf: float
    sigma_bar: np.ndarray  # [3 load cases, 3]
    iters: list


def evaluate(rho, eta=0.01, pc=oracle.PC_GREEN_JACOBI, tol=1e-10, maxit=20000, lengths=None,
             targets=None):
    """f(rho) = f_sigma + f_pf and its gradient (three PCG solves)."""
    t = target_stresses() if targets is None else targets
    E = np.asarray(rho, dtype=float)
    Bs, A = tri.triangle_B(tri._h(E.shape, lengths))
    C0 = tri.material(LAM0, MU0)
    vol = E.size * 2 * A
    sb = np.zeros((3, 3))
    eps = []  # per load case: [2 triangles][3, ny, nx]
    iters = []
    for gm in range(3):
        macro = np.eye(3)[gm]
        res = tri.solve(E, macro, LAM0, MU0, pc=pc, tol=tol, maxit=maxit, lengths=lengths)
        iters.append(res.iters)
        sb[gm] = res.sigma_bar
        ue = tri._gather(res.u)
        eps.append([np.einsum("ij,j...->i...", B, ue) + macro.reshape(3, 1, 1) for B in Bs])
    d = sb - t
    f_sigma = float((d * d).sum())
    g = np.zeros(E.shape)
    for gm in range(3):
        for a in range(3):
            wga = 2.0 * d[gm, a] / vol
            for tt in range(2):
                g += wga * A * np.einsum("i...,ij,j...->...", eps[a][tt], C0, eps[gm][tt])
    f_pf, g_pf = phase_field(E, eta, lengths)
    return Eval(f=f_sigma + f_pf, g=g + g_pf, f_sigma=f_sigma, f_pf=f_pf, sigma_bar=sb,
                iters=iters)


@dataclass
class LbfgsResult:
    rho: np.ndarray
    f: list = field(default_factory=list)       # f(rho_k), k = 0, 1, ...
    gnorm: list = field(default_factory=list)   # ||g_k||_inf
    iters: list = field(default_factory=list)   # PCG iterations of the accepted evaluations
    evals: int = 0


def lbfgs(fun, x0, n_iter, m=10, c1=1e-4, max_halvings=30):
    """Projected L-BFGS on [0, 1] (see the module docstring); fun(x) -> Eval."""
    x = np.clip(np.asarray(x0, dtype=float), 0.0, 1.0)
    ev = fun(x)
    out = LbfgsResult(rho=x, evals=1)
    out.f.append(ev.f)
    out.gnorm.append(float(np.abs(ev.g).max()))
    out.iters.append(ev.iters)
    S, Y = [], []
    for _ in range(n_iter):
        g = ev.g
        free = ~(((x <= 0.0) & (g > 0.0)) | ((x >= 1.0) & (g < 0.0)))
        # two-loop recursion on the free variables' gradient
        q = np.where(free, g, 0.0)
        al = []
        for s, y in reversed(list(zip(S, Y))):
            r = 1.0 / float((y * s).sum())
            a = r * float((s * q).sum())
            al.append((a, r))
            q -= a * y
        if S:
            h0 = float((S[-1] * Y[-1]).sum()) / float((Y[-1] * Y[-1]).sum())
        else:
            h0 = 0.1 / max(float(np.abs(q).max()), 1e-300)
        z = h0 * q
        for (s, y), (a, r) in zip(zip(S, Y), reversed(al)):
            b = r * float((y * z).sum())
            z += (a - b) * s
        d = np.where(free, -z, 0.0)
        alpha = 1.0
        accepted = False
        for _ in range(max_halvings):
            xt = np.clip(x + alpha * d, 0.0, 1.0)
            st = xt - x
            gs = float((g * st).sum())
            if gs < 0.0:
                evt = fun(xt)
                out.evals += 1
                if evt.f <= ev.f + c1 * gs:
                    accepted = True
                    break
            alpha *= 0.5
        if not accepted:
            break
        yv = evt.g - g
        sy = float((st * yv).sum())
        if sy > 1e-12 * np.linalg.norm(st) * np.linalg.norm(yv):
            S.append(st)
            Y.append(yv)
            if len(S) > m:
                S.pop(0)
                Y.pop(0)
        x, ev = xt, evt
        out.f.append(ev.f)
        out.gnorm.append(float(np.abs(ev.g).max()))
        out.iters.append(ev.iters)
    out.rho = x
    return out
