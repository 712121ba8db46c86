"""Python access to the plain FP64 CPU oracle (oracle/jfft_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline of the benchmark.  The product library never imports it, and it
imports nothing from the product library.

Every function marshals numpy arrays into the C oracle and back; all arithmetic
of the method lives in the C file.  Field conventions follow jfft_inputs:
E has shape (ny, nx) / (nz, ny, nx); vector fields (d, ...) with x fastest.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "libjfft_oracle.so")
_lib = None

PC_NONE, PC_GREEN, PC_JACOBI, PC_GREEN_JACOBI = 0, 1, 2, 3
STATUS = {0: "ok", 1: "invalid", 2: "odd_grid", 4: "not_converged", 5: "breakdown", 6: "oom"}

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIBPATH):
        from . import build as _b  # noqa: F401  (plain gcc build of the C oracle)
        _b.build()
    lib = C.CDLL(_LIBPATH)
    sig = {
        "or_stiffness": [C.c_int, _ip, _dp, C.c_double, C.c_double, _dp, _dp, _dp],
        "or_stiffness_at_node": [C.c_int, _ip, _dp, C.c_double, C.c_double, _dp, _dp, C.c_long, _dp],
        "or_rhs": [C.c_int, _ip, _dp, C.c_double, C.c_double, _dp, _dp, _dp, _dp],
        "or_stress": [C.c_int, _ip, _dp, C.c_double, C.c_double, _dp, _dp, _dp, _dp, _dp],
        "or_jacobi_diag": [C.c_int, _ip, _dp, C.c_double, C.c_double, _dp, _dp, _ip],
        "or_dft": [C.c_int, _ip, _dp, _dp, _dp, _dp, C.c_int],
        "or_green": [C.c_int, _ip, _dp, C.c_double, C.c_double, _dp, _dp],
        "or_precond": [C.c_int, _ip, _dp, C.c_int, _dp, C.c_double, _dp, _dp, _dp, _dp, _dp],
        "or_solve": [C.c_int, _ip, _dp, C.c_double, C.c_double, _dp, _dp, C.c_int, C.c_double,
                     C.c_double, C.c_double, C.c_double, C.c_int, C.c_int, _dp, _dp, _dp, _ip,
                     _dp, _dp, _dp, _dp, _dp, C.c_int, C.c_int, _dp, _dp, C.c_int,
                     C.c_ulonglong, C.c_int],
        "or_time_iterations": [C.c_int, _ip, _dp, C.c_double, C.c_double, _dp, _dp, C.c_int,
                               C.c_double, C.c_double, C.c_int, _dp],
        "or_num_threads": [],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.or_dot.argtypes = [C.c_int, C.c_long, _dp, _dp]
    lib.or_dot.restype = C.c_double
    _lib = lib
    return lib


def _d(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _grid(E, lengths):
    shape = E.shape
    dim = len(shape)
    n = (C.c_int * 3)(*([int(s) for s in shape[::-1]] + [1] * (3 - dim)))
    ln = (C.c_double * 3)(*(list(lengths) if lengths is not None else [1.0] * dim) + [1.0] * (3 - dim))
    return dim, n, ln


def _check(st, what):
    if st not in (0,):
        raise RuntimeError(f"oracle {what} failed: {STATUS.get(st, st)}")


def lame_from_nu(nu: float, young: float = 1.0):
    """Lame constants of the isotropic reference tensor C^(nu) with unit modulus."""
    lam = young * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = young / (2.0 * (1.0 + nu))
    return lam, mu


def num_threads() -> int:
    return int(_load().or_num_threads())


def stiffness(E, u, lam, mu, lengths=None):
    """K u (eq. lin_system_exp) by element loops."""
    lib = _load()
    E = np.ascontiguousarray(E, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    dim, n, ln = _grid(E, lengths)
    out = np.empty_like(u)
    _check(lib.or_stiffness(dim, n, ln, lam, mu, _d(E), _d(u), _d(out)), "stiffness")
    return out


def stiffness_at_node(E, u, lam, mu, node_index: int, lengths=None):
    """(K u) at one node (flat index, x fastest)."""
    lib = _load()
    E = np.ascontiguousarray(E, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    dim, n, ln = _grid(E, lengths)
    out = np.zeros(dim)
    _check(lib.or_stiffness_at_node(dim, n, ln, lam, mu, _d(E), _d(u), int(node_index), _d(out)),
           "stiffness_at_node")
    return out


def rhs(E, macro, lam, mu, lengths=None, with_abs=False):
    """f = -B^T W C(E) macro, without mean projection."""
    lib = _load()
    E = np.ascontiguousarray(E, dtype=np.float64)
    dim, n, ln = _grid(E, lengths)
    macro = np.ascontiguousarray(macro, dtype=np.float64)
    f = np.empty((dim,) + E.shape)
    fa = np.empty_like(f) if with_abs else None
    _check(lib.or_rhs(dim, n, ln, lam, mu, _d(E), _d(macro), _d(f), _d(fa)), "rhs")
    return (f, fa) if with_abs else f


def stress(E, macro, u, lam, mu, lengths=None, want_field=False):
    """Quadrature-point stresses (optional, shape (d*, 2^d, N)) and sigma_bar."""
    lib = _load()
    E = np.ascontiguousarray(E, dtype=np.float64)
    dim, n, ln = _grid(E, lengths)
    ds = dim * (dim + 1) // 2
    macro = np.ascontiguousarray(macro, dtype=np.float64)
    u = None if u is None else np.ascontiguousarray(u, dtype=np.float64)
    sq = np.empty((ds, 2 ** dim, E.size)) if want_field else None
    sbar = np.empty(ds)
    _check(lib.or_stress(dim, n, ln, lam, mu, _d(E), _d(macro), _d(u), _d(sq), _d(sbar)), "stress")
    return (sbar, sq) if want_field else sbar


def jacobi_diag(E, lam, mu, lengths=None):
    """Algorithm 2: diag(K) by d 2^d comb applications; returns (diag, napply)."""
    lib = _load()
    E = np.ascontiguousarray(E, dtype=np.float64)
    dim, n, ln = _grid(E, lengths)
    diag = np.empty((dim,) + E.shape)
    cnt = C.c_int(0)
    _check(lib.or_jacobi_diag(dim, n, ln, lam, mu, _d(E), _d(diag), C.byref(cnt)), "jacobi_diag")
    return diag, int(cnt.value)


def dft(x, sign=-1):
    """Naive separable DFT over all axes of a 2D/3D array (sign -1 forward,
    +1 inverse without normalisation)."""
    lib = _load()
    x = np.asarray(x)
    re = np.ascontiguousarray(x.real, dtype=np.float64)
    im = np.ascontiguousarray(x.imag if np.iscomplexobj(x) else np.zeros(x.shape), dtype=np.float64)
    dim = x.ndim
    n = (C.c_int * 3)(*([int(s) for s in x.shape[::-1]] + [1] * (3 - dim)))
    ore = np.empty(x.shape)
    oim = np.empty(x.shape)
    _check(lib.or_dft(dim, n, _d(re), _d(im), _d(ore), _d(oim), int(sign)), "dft")
    return ore + 1j * oim


def green(shape, lam_ref, mu_ref, lengths=None):
    """Algorithm 1: G^[beta, alpha, k...] as complex array (d, d, *shape)."""
    lib = _load()
    shape = tuple(int(s) for s in shape)
    dim = len(shape)
    E = np.ones(shape)
    _, n, ln = _grid(E, lengths)
    gr = np.empty((dim, dim) + shape)
    gi = np.empty_like(gr)
    _check(lib.or_green(dim, n, ln, lam_ref, mu_ref, _d(gr), _d(gi)), "green")
    return gr + 1j * gi


def precond(pc, r, diag=None, G=None, void_value=1.0, lengths=None):
    """z = M^-1 r; returns (z, max|Im|/max|Re| of the inverse transform)."""
    lib = _load()
    r = np.ascontiguousarray(r, dtype=np.float64)
    dim = r.shape[0]
    shape = r.shape[1:]
    _, n, ln = _grid(np.empty(shape), lengths)
    z = np.empty_like(r)
    ratio = C.c_double(0.0)
    gr = gi = None
    if G is not None:
        gr = np.ascontiguousarray(G.real)
        gi = np.ascontiguousarray(G.imag)
    dg = None if diag is None else np.ascontiguousarray(diag, dtype=np.float64)
    _check(lib.or_precond(dim, n, ln, int(pc), _d(dg), float(void_value), _d(gr), _d(gi), _d(r),
                          _d(z), C.byref(ratio)), "precond")
    return z, float(ratio.value)


@dataclass
class SolveResult:
    u: np.ndarray
    sigma_bar: np.ndarray
    iters: int
    relres: float
    relres_true: float
    status: str
    alpha: np.ndarray
    beta: np.ndarray
    res: np.ndarray
    timing: np.ndarray


def solve(E, macro, lam, mu, pc=PC_GREEN_JACOBI, lam_ref=None, mu_ref=None, tol=1e-8,
          maxit=1000, u0=None, void_value=1.0, stop_mode=0, hist_len=0, lengths=None,
          remove_mean=True, f=None, project_rhs=False, noise_seed=0, dot_mode=0) -> SolveResult:
    """Full PCG solve of K u = f; see or_solve.  f defaults to the assembled
    right-hand side, not projected to zero mean (project_rhs=True projects
    it).  noise_seed != 0 moves every entry of each K p and M^-1 r result by
    one ulp in a seeded direction, and dot_mode = 1 forms the inner products
    and norms as if in twice the working precision (Dot2) instead of the
    serial sum: rounding-difference models for parity windows (0, 0 = plain
    arithmetic)."""
    lib = _load()
    E = np.ascontiguousarray(E, dtype=np.float64)
    dim, n, ln = _grid(E, lengths)
    if lam_ref is None:
        lam_ref, mu_ref = lam, mu
    macro = np.ascontiguousarray(macro, dtype=np.float64)
    u = np.empty((dim,) + E.shape)
    u0 = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64)
    sbar = np.empty(dim * (dim + 1) // 2)
    it = C.c_int(0)
    rr = C.c_double(0.0)
    rt = C.c_double(0.0)
    h = max(int(hist_len), 0)
    ah = np.full(max(h, 1), np.nan)
    bh = np.full(max(h, 1), np.nan)
    rh = np.full(max(h, 1), np.nan)
    tm = np.zeros(3)
    f = None if f is None else np.ascontiguousarray(f, dtype=np.float64)
    st = lib.or_solve(dim, n, ln, lam, mu, _d(E), _d(macro), int(pc), lam_ref, mu_ref,
                      float(void_value), float(tol), int(stop_mode), int(maxit), _d(u0), _d(u),
                      _d(sbar), C.byref(it), C.byref(rr), C.byref(rt), _d(ah), _d(bh), _d(rh), h,
                      1 if remove_mean else 0, _d(tm), _d(f), 1 if project_rhs else 0,
                      int(noise_seed), int(dot_mode))
    if st not in (0, 4, 5):
        raise RuntimeError(f"oracle solve failed: {STATUS.get(st, st)}")
    k = int(it.value)
    return SolveResult(u=u, sigma_bar=sbar, iters=k, relres=float(rr.value),
                       relres_true=float(rt.value), status=STATUS[st],
                       alpha=ah[:min(k, h)], beta=bh[:min(max(k - 1, 0), h)],
                       res=rh[:min(k, h)], timing=tm)


def dot(a, b, mode=0):
    """The oracle's inner product: mode 0 serial sum in index order, 1 Dot2."""
    a = np.ascontiguousarray(a, dtype=np.float64).ravel()
    b = np.ascontiguousarray(b, dtype=np.float64).ravel()
    assert a.size == b.size
    return float(_load().or_dot(int(mode), a.size, _d(a), _d(b)))


def precond_fft(pc, r, diag=None, G=None, void_value=1.0):
    """z = M^-1 r as `precond` computes it (eq. prec_lin_systemJG_2 and its
    Green / Jacobi / identity special cases), with numpy's FFT as the
    transform step instead of the naive DFT: a second rounding of the same
    operator, used as a rounding variant for parity windows (an FFT's
    rounding grows like log n, the naive DFT's like n)."""
    r = np.asarray(r, dtype=np.float64)
    d = r.shape[0]
    axes = tuple(range(1, r.ndim))
    if pc == PC_NONE:
        return r.copy()
    dg = None
    if diag is not None:
        dg = np.where(np.asarray(diag) == 0.0, void_value, diag)
    if pc == PC_JACOBI:
        return r / dg
    jh = 1.0 / np.sqrt(dg) if pc == PC_GREEN_JACOBI else np.ones_like(r)
    S = np.fft.fftn(jh * r, axes=axes)
    Z = np.einsum("ba...,a...->b...", G, S)
    return jh * np.real(np.fft.ifftn(Z, axes=axes))


def solve_py(E, macro, lam, mu, pc=PC_GREEN_JACOBI, tol=1e-8, maxit=1000, u0=None,
             void_value=1.0, stop_mode=0, lengths=None, f=None, noise_seed=0, dot_mode=0,
             transform="fft", hist_len=0) -> SolveResult:
    """The PCG loop of or_solve written out in Python over the oracle's
    operators (K by element loops, f, Algorithm 2's diagonal, Algorithm 1's
    G^), for rounding variants that the C loop does not have: the transform
    step by numpy's FFT (transform="fft") or the naive DFT ("dft"), inner
    products by numpy's pairwise sum (dot_mode 0) or math.fsum (1,
    correctly rounded), and the one-ulp noise on every K p and M^-1 r result
    (noise_seed != 0).  Same stopping rules, breakdown test, iteration count
    and post-processing as or_solve."""
    import math

    E = np.ascontiguousarray(E, dtype=np.float64)
    dim = E.ndim
    f_asm, fa = rhs(E, macro, lam, mu, lengths, with_abs=True)
    f = f_asm if f is None else np.asarray(f, dtype=np.float64)
    diag = jacobi_diag(E, lam, mu, lengths)[0] if pc in (PC_JACOBI, PC_GREEN_JACOBI) else None
    G = green(E.shape, lam, mu, lengths) if pc in (PC_GREEN, PC_GREEN_JACOBI) else None
    rng = np.random.default_rng(noise_seed) if noise_seed else None

    def noisy(x):
        if rng is None:
            return x
        up = rng.random(x.shape) < 0.5
        moved = np.where(up, np.nextafter(x, np.inf), np.nextafter(x, -np.inf))
        return np.where(x == 0.0, 0.0, moved)

    def dot(a, b):
        return math.fsum((a * b).ravel()) if dot_mode == 1 else float((a * b).sum())

    def M(r):
        if transform == "fft":
            z = precond_fft(pc, r, diag=diag, G=G, void_value=void_value)
        else:
            z = precond(pc, r, diag=diag, G=G, void_value=void_value, lengths=lengths)[0]
        return noisy(z)

    def K(x):
        return stiffness(E, x, lam, mu, lengths)

    fnorm = math.sqrt(dot(f, f))
    fabsnorm = math.sqrt(dot(fa, fa))
    homog = fnorm <= 1e-13 * fabsnorm
    if u0 is not None:
        u = np.array(u0, dtype=np.float64)
        r = f - K(u)
    else:
        u = np.zeros_like(f)
        r = f.copy()
    rnorm = math.sqrt(dot(r, r))

    def done(rn):
        return rn <= tol * fnorm if stop_mode == 0 else rn * rn <= tol

    k, status = 0, "ok"
    alphas, betas, hist = [], [], []
    if homog:
        u[:] = 0.0
        rnorm = 0.0
    elif not done(rnorm):
        z = M(r)
        p = z.copy()
        rz = dot(r, z)
        while True:
            if k >= maxit:
                status = "not_converged"
                break
            q = noisy(K(p))
            pq = dot(p, q)
            alpha = rz / pq if pq != 0.0 else float("inf")
            if not (pq > 0.0) or not math.isfinite(alpha):
                status = "breakdown"
                break
            u += alpha * p
            r -= alpha * q
            k += 1
            rnorm = math.sqrt(dot(r, r))
            alphas.append(alpha)
            hist.append(rnorm)
            if done(rnorm):
                break
            if k >= maxit:
                status = "not_converged"
                break
            z = M(r)
            rz_new = dot(r, z)
            beta = rz_new / rz
            if not math.isfinite(beta):
                status = "breakdown"
                break
            betas.append(beta)
            rz = rz_new
            p = z + beta * p
    rt = math.sqrt(dot(f - K(u), f - K(u)))
    u -= u.reshape(dim, -1).mean(axis=1).reshape((dim,) + (1,) * dim)
    sbar = stress(E, macro, u, lam, mu, lengths)
    h = max(int(hist_len), 0)
    return SolveResult(u=u, sigma_bar=sbar, iters=k,
                       relres=(rnorm / fnorm if fnorm > 0 and not homog else 0.0),
                       relres_true=(rt / fnorm if fnorm > 0 and not homog else 0.0), status=status,
                       alpha=np.array(alphas[:h]), beta=np.array(betas[:h]),
                       res=np.array(hist[:h]), timing=np.zeros(3))


def time_iterations(E, macro, lam, mu, pc=PC_GREEN_JACOBI, iters=1, lengths=None):
    """Wall seconds (setup, `iters` PCG iterations, first preconditioner apply)."""
    lib = _load()
    E = np.ascontiguousarray(E, dtype=np.float64)
    dim, n, ln = _grid(E, lengths)
    macro = np.ascontiguousarray(macro, dtype=np.float64)
    tm = np.zeros(3)
    _check(lib.or_time_iterations(dim, n, ln, lam, mu, _d(E), _d(macro), int(pc), lam, mu,
                                  int(iters), _d(tm)), "time_iterations")
    return tm


def effective_stiffness(E, lam, mu, pc=PC_GREEN_JACOBI, tol=1e-10, maxit=5000, lengths=None):
    """Homogenised Mandel stiffness: column gamma is sigma_bar for macro = e_gamma."""
    dim = E.ndim
    ds = dim * (dim + 1) // 2
    Ceff = np.empty((ds, ds))
    its = []
    for g in range(ds):
        m = np.zeros(ds)
        m[g] = 1.0
        res = solve(E, m, lam, mu, pc=pc, tol=tol, maxit=maxit, lengths=lengths)
        Ceff[:, g] = res.sigma_bar
        its.append(res.iters)
    return Ceff, its
