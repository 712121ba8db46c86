"""Plain FP64 numpy oracle of the 2D linear-triangle discretisation (the
paper's own 2D element: continuous piecewise-linear finite elements on a
regular grid, Sec. 2 and Sec. 4; plane strain).

TEST INFRASTRUCTURE ONLY: imported by tests/ and the benchmark's CPU
baseline.  The product library never imports it, and it imports nothing from
the product library.  The preconditioner application is the C oracle's
(oracle.precond); everything else is written out here from the definitions:

* every pixel (element e, indexed by its lowest node, periodic) is split into
  two linear triangles along its anti-diagonal: T0 = corners (0, 1, 2) and
  T1 = corners (3, 2, 1), corner c = cx + 2 cy at (cx hx, cy hy) (the paper
  does not say which diagonal);
* one quadrature point per triangle (exact: the strain is constant), weight
  the triangle's area hx hy / 2;
* Mandel vectors (11, 22, 12) with the shear entry sqrt2 eps_12; isotropic
  plane-strain C(E) = E C^(lam, mu), E constant per pixel;
* K u = sum_e sum_t A B_t^T C_e B_t u_e (eq. lin_system_exp), f = -sum_e sum_t
  A B_t^T C_e macro;
* Algorithm 1 (Green operator): responses of K_ref to a unit impulse of each
  component at node 0, their DFT, the 2 x 2 block inverted at every k != 0,
  G^(0) = 0 (the layout oracle.precond takes, complex; the blocks come out
  real symmetric, since the triangulation is symmetric under the point
  reflection x -> -x, but not of the separable quadrilateral form: it is
  not symmetric under the reflection of one axis);
* Algorithm 2 (Jacobi diagonal): K applied to the d 2^d unit combs;
* PCG as the C oracle runs it (start u = 0, recursive residual, stop at
  ||r|| <= tol ||f|| or ||r||^2 <= tol, homogeneous test ||f|| <= 1e-13
  ||f_abs||), then the mean of u removed and sigma_bar = sum A sigma / |Y|.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

import oracle

SQ2 = np.sqrt(2.0)
# corner offsets (cx, cy) and the corners of the two triangles
CORNERS = ((0, 0), (1, 0), (0, 1), (1, 1))
TRIANGLES = ((0, 1, 2), (3, 2, 1))


def _h(shape, lengths):
    ny, nx = shape
    L = (1.0, 1.0) if lengths is None else lengths
    return (L[0] / nx, L[1] / ny)


def triangle_B(h):
    """B_t (3 x 8) of both triangles, columns i * 4 + c (component i, corner
    c), from the gradients of the linear shape functions; and the area."""
    hx, hy = h
    out = []
    for tri in TRIANGLES:
        # N_c(x) = a_c + g_c . x on the triangle: solve for (a, gx, gy) from
        # N_c(x_k) = delta_ck at its three corners
        P = np.array([[1.0, CORNERS[k][0] * hx, CORNERS[k][1] * hy] for k in tri])
        coef = np.linalg.solve(P, np.eye(3))  # column j: (a, gx, gy) of corner tri[j]
        B = np.zeros((3, 8))
        for j, c in enumerate(tri):
            gx, gy = coef[1, j], coef[2, j]
            B[0, 0 * 4 + c] = gx
            B[1, 1 * 4 + c] = gy
            B[2, 0 * 4 + c] = gy / SQ2
            B[2, 1 * 4 + c] = gx / SQ2
        out.append(B)
    return out, 0.5 * hx * hy


def material(lam, mu):
    """Plane-strain isotropic C^ in Mandel form (3 x 3)."""
    return np.array([[lam + 2 * mu, lam, 0.0], [lam, lam + 2 * mu, 0.0], [0.0, 0.0, 2 * mu]])


def element_matrix(h, lam, mu):
    """8 x 8 stiffness of one pixel (both triangles), unit modulus."""
    Bs, A = triangle_B(h)
    C = material(lam, mu)
    return sum(A * B.T @ C @ B for B in Bs)


def _gather(u):
    """u [2, ny, nx] -> element vectors [8, ny, nx], index i * 4 + c."""
    out = np.empty((8,) + u.shape[1:])
    for i in range(2):
        for c, (cx, cy) in enumerate(CORNERS):
            out[i * 4 + c] = np.roll(u[i], shift=(-cy, -cx), axis=(0, 1))
    return out


def _scatter(ye):
    """element vectors [8, ny, nx] -> nodal sums [2, ny, nx]."""
    out = np.zeros((2,) + ye.shape[1:])
    for i in range(2):
        for c, (cx, cy) in enumerate(CORNERS):
            out[i] += np.roll(ye[i * 4 + c], shift=(cy, cx), axis=(0, 1))
    return out


def stiffness(E, u, lam, mu, lengths=None):
    """K u (eq. lin_system_exp) for the pixel-constant modulus E [ny, nx]."""
    Ke = element_matrix(_h(E.shape, lengths), lam, mu)
    return _scatter(np.einsum("ij,j...->i...", Ke, _gather(u)) * E)


def rhs(E, macro, lam, mu, lengths=None, with_abs=False):
    """f = -sum_e E_e sum_t A B_t^T C^ macro; with_abs also returns the sum
    of the absolute element contributions (scale of the homogeneous test)."""
    Bs, A = triangle_B(_h(E.shape, lengths))
    C = material(lam, mu)
    F = sum(A * B.T @ (C @ np.asarray(macro, dtype=float)) for B in Bs)  # [8]
    ye = -F.reshape(8, 1, 1) * E
    f = _scatter(ye)
    if with_abs:
        return f, _scatter(np.abs(ye))
    return f


def stress(E, macro, u, lam, mu, lengths=None):
    """sigma at the quadrature point of each triangle [3, 2, ny, nx] (Mandel)
    and sigma_bar = sum A sigma / |Y|."""
    Bs, A = triangle_B(_h(E.shape, lengths))
    C = material(lam, mu)
    ue = _gather(u)
    sig = np.empty((3, 2) + E.shape)
    for t, B in enumerate(Bs):
        eps = np.einsum("ij,j...->i...", B, ue) + np.asarray(macro, dtype=float).reshape(3, 1, 1)
        sig[:, t] = np.einsum("ij,j...->i...", C, eps) * E
    return sig, sig.reshape(3, -1).mean(axis=1)


def green(shape, lam_ref, mu_ref, lengths=None):
    """Algorithm 1: G^[b, a, ky, kx] (complex, full spectrum), the layout
    oracle.precond takes."""
    shape = tuple(int(s) for s in shape)
    ones = np.ones(shape)
    Kh = np.empty((2, 2) + shape, dtype=complex)
    for a in range(2):
        imp = np.zeros((2,) + shape)
        imp[a, 0, 0] = 1.0
        resp = stiffness(ones, imp, lam_ref, mu_ref, lengths)
        for b in range(2):
            Kh[b, a] = np.fft.fft2(resp[b])
    G = np.zeros_like(Kh)
    blocks = np.moveaxis(Kh, (0, 1), (-2, -1))  # [ny, nx, 2, 2]
    inv = np.zeros_like(blocks)
    mask = np.ones(shape, dtype=bool)
    mask[0, 0] = False
    inv[mask] = np.linalg.inv(blocks[mask])
    G[:] = np.moveaxis(inv, (-2, -1), (0, 1))
    return G


def jacobi_diag(E, lam, mu, lengths=None):
    """Algorithm 2: K applied to the unit combs e_a on the nodes of parity o."""
    ny, nx = E.shape
    yy, xx = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    diag = np.zeros((2,) + E.shape)
    for a in range(2):
        for o in range(4):
            mask = ((xx & 1) == (o & 1)) & ((yy & 1) == (o >> 1))
            comb = np.zeros((2,) + E.shape)
            comb[a][mask] = 1.0
            Kc = stiffness(E, comb, lam, mu, lengths)
            diag[a][mask] = Kc[a][mask]
    return diag


@dataclass
class SolveResult:
    u: np.ndarray
    sigma_bar: np.ndarray
    iters: int
    relres_true: float
    status: str
    res: np.ndarray  # recursive ||r_k||, k = 1..iters


def solve(E, macro, lam, mu, pc=oracle.PC_GREEN_JACOBI, lam_ref=None, mu_ref=None, tol=1e-8,
          maxit=5000, void_value=1.0, stop_absolute=False, lengths=None, f=None, noise_seed=0,
          dot_mode=0, transform="dft"):
    """PCG on K u = f from u = 0 (the C oracle's loop, with the triangle
    operators), then mean removal and sigma_bar.  f defaults to the assembled
    right-hand side; a given f replaces it (the cancellation test of the
    homogeneous case still uses the assembled |f|).  noise_seed != 0 moves
    every entry of each K p and M^-1 r result by one ulp in a seeded random
    direction, the C oracle's rounding-difference model for parity windows;
    dot_mode = 1 sums the products of every inner product and norm with
    math.fsum (correctly rounded) instead of numpy's pairwise sum;
    transform="fft" applies the preconditioner with numpy's FFT
    (oracle.precond_fft) instead of the naive DFT."""
    E = np.asarray(E, dtype=np.float64)
    if lam_ref is None:
        lam_ref, mu_ref = lam, mu
    f_asm, fa = rhs(E, macro, lam, mu, lengths, with_abs=True)
    f = f_asm if f is None else np.asarray(f, dtype=np.float64)
    fn, fan = np.linalg.norm(f), np.linalg.norm(fa)
    if dot_mode == 1:
        fn = math.sqrt(math.fsum((f * f).ravel()))
    diag = jacobi_diag(E, lam, mu, lengths) if pc in (oracle.PC_JACOBI,
                                                      oracle.PC_GREEN_JACOBI) else None
    G = green(E.shape, lam_ref, mu_ref, lengths) if pc in (oracle.PC_GREEN,
                                                           oracle.PC_GREEN_JACOBI) else None

    rng = np.random.default_rng(noise_seed) if noise_seed else None

    def noisy(x):
        if rng is None:
            return x
        up = rng.random(x.shape) < 0.5
        moved = np.where(up, np.nextafter(x, np.inf), np.nextafter(x, -np.inf))
        return np.where(x == 0.0, 0.0, moved)

    def M(r):
        if transform == "fft":
            return noisy(oracle.precond_fft(pc, r, diag=diag, G=G, void_value=void_value))
        return noisy(oracle.precond(pc, r, diag=diag, G=G, void_value=void_value,
                                    lengths=lengths)[0])

    def dot(a, b):
        return math.fsum((a * b).ravel()) if dot_mode == 1 else float((a * b).sum())

    def norm(a):
        return math.sqrt(dot(a, a)) if dot_mode == 1 else np.linalg.norm(a)

    def done(rn):
        return rn * rn <= tol if stop_absolute else rn <= tol * fn

    u = np.zeros((2,) + E.shape)
    r = f.copy()
    k = 0
    hist = []
    status = "ok"
    homog = fn <= 1e-13 * fan
    if not (homog or done(norm(r))):
        z = M(r)
        p = z.copy()
        rz = dot(r, z)
        while True:
            if k >= maxit:
                status = "not_converged"
                break
            q = noisy(stiffness(E, p, lam, mu, lengths))
            pq = dot(p, q)
            alpha = rz / pq
            if not (pq > 0.0) or not np.isfinite(alpha):
                status = "breakdown"
                break
            u += alpha * p
            r -= alpha * q
            k += 1
            hist.append(norm(r))
            if done(hist[-1]):
                break
            if k >= maxit:
                status = "not_converged"
                break
            z = M(r)
            rz_new = dot(r, z)
            p = z + (rz_new / rz) * p
            rz = rz_new
    u -= u.reshape(2, -1).mean(axis=1).reshape(2, 1, 1)
    rt = np.linalg.norm(f - stiffness(E, u, lam, mu, lengths))
    _, sbar = stress(E, macro, u, lam, mu, lengths)
    return SolveResult(u=u, sigma_bar=sbar, iters=k,
                       relres_true=(rt / fn if fn > 0 and not homog else 0.0), status=status,
                       res=np.array(hist))
