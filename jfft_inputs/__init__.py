"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This module only *generates* material fields, macro strains and start vectors.
It holds none of the solver's arithmetic (no stiffness, no Green operator, no
CG), so neither the oracle nor the HIP library depends on the other through it.

Array conventions (shared by both sides):
  * a scalar field (Young's-modulus field E) has shape (ny, nx) in 2D and
    (nz, ny, nx) in 3D, C order, x fastest; entry E[k, j, i] is the value of
    the element whose lowest-index corner is node (i, j, k);
  * a displacement-like field has shape (d, ny, nx) / (d, nz, ny, nx);
  * node (i, j, k) sits at x = (i*h_x, j*h_y, k*h_z) with h = l / n.

Workload recipes follow the paper's smooth high-contrast densities
(Sec. 1 motivating example, Sec. 4.1 laminate, Sec. 4.2 cosine geometry with
voids) and the synthetic stand-ins for fields the paper does not publish
(Gaussian random fields, smoothed SIMP densities).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "node_coords", "sine_contrast_field", "grf_field", "simp_field",
    "laminate_field", "cosine_void_field", "filtered_inclusion_field",
    "uniform_random_field", "random_start", "unit_macro_strain", "mandel_size",
    "spherical_inclusions", "ulp_perturbed", "sketch_vectors", "sample_nodes",
    "refine_geometry",
]


def mandel_size(dim: int) -> int:
    """Number of independent strain components d* = d(d+1)/2 (Sec. 2)."""
    return dim * (dim + 1) // 2


def node_coords(shape, lengths=None):
    """Nodal coordinates (x_1, ..., x_d) as broadcastable arrays, x fastest.

    `shape` is the array shape (.., ny, nx); the result is returned in axis
    order (x, y[, z]) with each array shaped like the field.
    """
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    if lengths is None:
        lengths = (1.0,) * dim
    n_xyz = shape[::-1]
    grids = np.meshgrid(*[np.arange(n) * (l / n) for n, l in zip(shape, lengths[::-1])],
                        indexing="ij")
    # grids[a] varies along array axis a; array axis a is spatial axis dim-1-a
    return tuple(grids[dim - 1 - a] for a in range(dim))


def sine_contrast_field(n: int = 32, amplitude: float = 2.0) -> np.ndarray:
    """2D smooth contrast field E = 10^(a sin(2 pi x) sin(2 pi y)) sampled at the
    lowest corner node of every pixel (material sampling rule of Sec. 4).
    With a = 2 the contrast max/min is 1e4 whenever n is a multiple of 4."""
    x, y = node_coords((n, n))
    return 10.0 ** (amplitude * np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y))


def _minimum_image_wavenumbers(n: int) -> np.ndarray:
    k = np.arange(n)
    return np.where(k <= n // 2, k, k - n).astype(np.float64)


def grf_field(shape, contrast: float, seed: int, ell: float = 0.1) -> np.ndarray:
    """Smooth log-normal field E = exp(s (g - min g)) with min E = 1 and
    max E = contrast exactly.

    g is a periodic Gaussian random field with squared-exponential covariance
    exp(-r^2 / (2 ell^2)) on the unit cell: white noise filtered in Fourier
    space by sqrt(S(k)), S(k) = exp(-2 pi^2 ell^2 |k|^2) with integer
    minimum-image wave vectors.  Stand-in for the paper's smooth densities,
    which are not published.
    """
    shape = tuple(int(s) for s in shape)
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape)
    ks = np.meshgrid(*[_minimum_image_wavenumbers(s) for s in shape], indexing="ij")
    k2 = sum(k * k for k in ks)
    filt = np.sqrt(np.exp(-2.0 * np.pi ** 2 * ell ** 2 * k2))
    g = np.real(np.fft.ifftn(filt * np.fft.fftn(w)))
    g = (g - g.min()) / (g.max() - g.min())
    return np.exp(np.log(contrast) * g)


def simp_field(n: int, seed: int, sigma_px: float = 4.0, rho_min: float = 1e-3,
               power: float = 3.0, e0: float = 1.0) -> np.ndarray:
    """2D SIMP stiffness field E = E0 rho^p with rho in [rho_min, 1].

    Uniform noise blurred by a periodic Gaussian of standard deviation
    `sigma_px` pixels, min-max normalised to [0, 1], then mapped affinely to
    [rho_min, 1] (so the contrast of E is exactly rho_min^-p)."""
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.0, 1.0, size=(n, n))
    k = _minimum_image_wavenumbers(n)
    k2 = k[:, None] ** 2 + k[None, :] ** 2
    filt = np.exp(-2.0 * np.pi ** 2 * (sigma_px / n) ** 2 * k2)
    s = np.real(np.fft.ifft2(filt * np.fft.fft2(w)))
    s = (s - s.min()) / (s.max() - s.min())
    rho = rho_min + (1.0 - rho_min) * s
    return e0 * rho ** power


def laminate_field(shape, chi: float) -> np.ndarray:
    """Laminate of Sec. 4.1: the density is linear in x_1,
    rho = chi + (1 - chi) x_1 / (1 - dx_1), sampled at the nodes, so the
    element columns run from chi (x_1 = 0) down to 1 (last column)."""
    shape = tuple(int(s) for s in shape)
    nx = shape[-1]
    dx = 1.0 / nx
    x1 = np.arange(nx) * dx
    col = chi + (1.0 - chi) * x1 / (1.0 - dx)
    return np.broadcast_to(col, shape).copy()


def cosine_void_field(n: int, chi: float | None) -> np.ndarray:
    """Cosine geometry of Sec. 4.2,
    rho = 0.5 + 0.25 (cos 2 pi (x1 - x2) + cos 2 pi (x1 + x2)) + 1/chi;
    chi = None means chi = infinity, which leaves exact zeros (voids)."""
    x, y = node_coords((n, n))
    rho = 0.5 + 0.25 * (np.cos(2 * np.pi * (x - y)) + np.cos(2 * np.pi * (x + y)))
    rho = np.where(np.abs(rho) < 1e-14, 0.0, rho)
    if chi is not None:
        rho = rho + 1.0 / chi
    return rho


def filtered_inclusion_field(n: int, filters: int, radius: float = 0.25,
                             soft: float = 1e-4, hard: float = 1.0) -> np.ndarray:
    """Motivating example of Sec. 1: a soft disc (density `soft`) in a stiff
    matrix, smoothed by `filters` periodic applications of the 3x3 kernel
    (1/16)[1 2 1]^T[1 2 1].  The radius is our choice (the paper does not give
    it)."""
    x, y = node_coords((n, n))
    rho = np.where((x - 0.5) ** 2 + (y - 0.5) ** 2 < radius ** 2, soft, hard)
    w = np.array([1.0, 2.0, 1.0]) / 4.0
    for _ in range(filters):
        rho = w[0] * np.roll(rho, 1, 0) + w[1] * rho + w[2] * np.roll(rho, -1, 0)
        rho = w[0] * np.roll(rho, 1, 1) + w[1] * rho + w[2] * np.roll(rho, -1, 1)
    return rho


def uniform_random_field(shape, lo: float, hi: float, seed: int) -> np.ndarray:
    """I.i.d. uniform element values in [lo, hi]."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=tuple(shape))


def random_start(shape, seed: int) -> np.ndarray:
    """Seeded CG start vector: i.i.d. N(0, 1) per degree of freedom, made
    mean-free per component.  `shape` is the scalar grid shape; the result has
    a leading component axis of length d = len(shape)."""
    shape = tuple(int(s) for s in shape)
    d = len(shape)
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((d,) + shape)
    axes = tuple(range(1, d + 1))
    return u - u.mean(axis=axes, keepdims=True)


def unit_macro_strain(dim: int, gamma: int) -> np.ndarray:
    """Unit macro strain e_gamma in Mandel notation (3D order 11,22,33,23,13,12;
    2D order 11,22,12)."""
    e = np.zeros(mandel_size(dim))
    e[gamma] = 1.0
    return e


def spherical_inclusions(shape, count: int, radius: float, seed: int) -> np.ndarray:
    """Indicator (1 inside, 0 outside) of `count` spheres of radius `radius`
    (fraction of the unit cell) at seeded random centres, periodic minimum-image
    distance, sampled at each element's lowest node: a stand-in for the
    inclusion geometry of the nonlinear example, which the paper does not give."""
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in shape)
    coords = [np.arange(n) / n for n in shape]  # (z, y, x), broadcast per axis
    out = np.zeros(shape)
    for _ in range(int(count)):
        c = rng.random(len(shape))
        d2 = np.zeros(shape)
        for ax, (a, ca) in enumerate(zip(coords, c)):
            d = np.abs(a - ca)
            d = np.minimum(d, 1.0 - d)
            sh = [1] * len(shape)
            sh[ax] = shape[ax]
            d2 = d2 + (d * d).reshape(sh)
        out[d2 <= radius * radius] = 1.0
    return out



def ulp_perturbed(a, seed: int) -> np.ndarray:
    """Copy of `a` with every entry moved by one unit in the last place, up or
    down with equal probability (seeded); exact zeros stay zero.  Used to
    measure how far rounding-level changes of the input move a solver's
    stopping iteration."""
    a = np.asarray(a, dtype=np.float64)
    up = np.random.default_rng(seed).random(a.shape) < 0.5
    out = np.where(up, np.nextafter(a, np.inf), np.nextafter(a, -np.inf))
    return np.where(a == 0.0, 0.0, out)


def sketch_vectors(shape, count: int, seed: int):
    """Yield `count` seeded i.i.d. N(0, 1) arrays of `shape`, one at a time.
    For any array x of that shape, E[(w . x)^2] = ||x||^2, so the mean square
    of the projections estimates a squared norm (a sketch of a field too large
    to store)."""
    rng = np.random.default_rng(seed)
    for _ in range(int(count)):
        yield rng.standard_normal(tuple(shape))


def sample_nodes(n_nodes: int, count: int, seed: int) -> np.ndarray:
    """Sorted seeded sample of `count` distinct flat node indices."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(int(n_nodes), size=int(count), replace=False))


def refine_geometry(rho_p, n: int) -> np.ndarray:
    """A geometry of p x p pixels (Sec. 4: G_p, the density sampled at the
    geometry's nodal points and assigned to the whole pixel) on the finer
    discretisation grid T_n, n a multiple of p: every geometry pixel covers
    (n / p)^2 elements of the same density."""
    rho_p = np.asarray(rho_p, dtype=np.float64)
    p = rho_p.shape[0]
    if rho_p.shape != (p, p) or n % p:
        raise ValueError("a square p x p geometry and n a multiple of p are needed")
    r = n // p
    return np.kron(rho_p, np.ones((r, r)))
