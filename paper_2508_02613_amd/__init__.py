"""MI355X (gfx950) J-FFT solver: PCG with the Green-Jacobi preconditioner for
periodic linear-elastic cell problems (arXiv 2508.02613).

Thin Python binding over the C ABI in include/jfft.h (libjfft.so, built
in-tree by paper_2508_02613_amd/build.py).  The binding only marshals
arguments: every step of the solver runs in the library's HIP kernels.
PyTorch provides device memory and streams.

The library must be present: importing this package on a machine without the
built library, or calling it without a GPU, raises instead of falling back to
any CPU path.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

__all__ = ["load_library", "Cell", "Report", "PC_NONE", "PC_GREEN", "PC_JACOBI",
           "PC_GREEN_JACOBI", "FP64", "MIXED", "JfftError", "EXPORTED_SYMBOLS", "lame_from_nu",
           "effective_stiffness"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(_HERE, "libjfft.so")

PC_NONE, PC_GREEN, PC_JACOBI, PC_GREEN_JACOBI = 0, 1, 2, 3
FP64, MIXED = 0, 1
_STATUS = {0: "ok", 1: "invalid", 2: "odd_grid", 3: "no_material", 4: "not_converged",
           5: "breakdown", 6: "oom", 7: "hip"}

_vp = C.c_void_p
_dp = C.POINTER(C.c_double)


class _Tunables(C.Structure):
    _fields_ = [("tz", C.c_int), ("ygrid", C.c_int), ("tiles2d", C.c_int), ("xrows", C.c_int),
                ("fused_control", C.c_int), ("tiles3d", C.c_int)]


class _Report(C.Structure):
    _fields_ = [("iters", C.c_int), ("outer", C.c_int), ("status", C.c_int),
                ("rel_res", C.c_double), ("rel_res_true", C.c_double),
                ("setup_ms", C.c_double), ("loop_ms", C.c_double), ("post_ms", C.c_double)]


# name -> (restype, argtypes); every symbol declared in include/jfft.h
_SIGS = {
    "jfft_create_cell": (C.c_int, [C.c_int, C.POINTER(C.c_int), _dp, C.c_int, C.c_int, _vp,
                                   C.POINTER(_vp)]),
    "jfft_create_batch": (C.c_int, [C.c_int, C.POINTER(C.c_int), _dp, C.c_int, C.c_int, C.c_int,
                                    _vp, C.POINTER(_vp)]),
    "jfft_batch_size": (C.c_int, [_vp, C.POINTER(C.c_int)]),
    "jfft_workspace_bytes": (C.c_int, [_vp, C.POINTER(C.c_size_t)]),
    "jfft_bind_workspace": (C.c_int, [_vp, _vp, C.c_size_t]),
    "jfft_set_material": (C.c_int, [_vp, _vp, C.c_double]),
    "jfft_set_material_lame": (C.c_int, [_vp, _vp, C.c_double, C.c_double]),
    "jfft_solve": (C.c_int, [_vp, _dp, C.c_double, C.c_int, _vp, _vp, _vp, _dp,
                             C.POINTER(_Report)]),
    "jfft_solve_static": (C.c_int, [_vp, _vp, C.c_double, _dp, C.c_double, C.c_int, _vp, _vp,
                                    _vp, _dp, C.POINTER(_Report)]),
    "jfft_solve_batch": (C.c_int, [_vp, _dp, C.c_double, C.c_int, _vp, _vp, _vp, _dp,
                                   C.POINTER(_Report)]),
    "jfft_slot_admit": (C.c_int, [_vp, C.c_int, _vp, C.c_double, _dp, C.c_double, C.c_int]),
    "jfft_slots_step": (C.c_int, [_vp, C.c_int, C.POINTER(C.c_int)]),
    "jfft_slots_run": (C.c_int, [_vp, C.c_double, C.POINTER(C.c_int)]),
    "jfft_slot_harvest": (C.c_int, [_vp, C.c_int, _vp, _vp, _dp, C.POINTER(_Report)]),
    "jfft_set_graph_iterations": (C.c_int, [_vp, C.c_int]),
    "jfft_set_tunables": (C.c_int, [_vp, C.POINTER(_Tunables)]),
    "jfft_get_tunables": (C.c_int, [_vp, C.POINTER(_Tunables)]),
    "jfft_apply_stiffness": (C.c_int, [_vp, _vp, _vp]),
    "jfft_apply_precond": (C.c_int, [_vp, _vp, _vp]),
    "jfft_apply_precond_fp32": (C.c_int, [_vp, _vp, _vp]),
    "jfft_assemble_rhs": (C.c_int, [_vp, _dp, _vp]),
    "jfft_jacobi_diag": (C.c_int, [_vp, _vp]),
    "jfft_enable_history": (C.c_int, [_vp, C.c_int]),
    "jfft_get_history": (C.c_int, [_vp, _dp, _dp, _dp, C.c_int, C.POINTER(C.c_int)]),
    "jfft_get_batch_history": (C.c_int, [_vp, C.c_int, _dp, _dp, _dp, C.c_int,
                                         C.POINTER(C.c_int)]),
    "jfft_enable_timing": (C.c_int, [_vp, C.c_int]),
    "jfft_kernel_stats": (C.c_int, [_vp, C.c_int, C.POINTER(C.c_char_p), C.POINTER(C.c_long),
                                    _dp, C.POINTER(C.c_int)]),
    "jfft_reset_timing": (C.c_int, [_vp]),
    "jfft_set_void_value": (C.c_int, [_vp, C.c_double]),
    "jfft_set_mixed_params": (C.c_int, [_vp, C.c_double, C.c_int]),
    "jfft_set_mixed_inner_cap": (C.c_int, [_vp, C.c_int]),
    "jfft_set_mixed_continue": (C.c_int, [_vp, C.c_int, C.c_double]),
    "jfft_set_stop_rule": (C.c_int, [_vp, C.c_int]),
    "jfft_set_diag_method": (C.c_int, [_vp, C.c_int]),
    "jfft_set_element": (C.c_int, [_vp, C.c_int]),
    "jfft_set_material_powerlaw": (C.c_int, [_vp, _vp, C.c_double, C.c_double, C.c_double,
                                             C.c_double, C.c_double, C.c_double]),
    "jfft_solve_newton": (C.c_int, [_vp, _dp, C.c_double, C.c_double, C.c_int, C.c_int, _vp, _dp,
                                    C.POINTER(C.c_int), _dp, C.POINTER(C.c_int)]),
    "jfft_powerlaw_force": (C.c_int, [_vp, _dp, _vp, _vp]),
    "jfft_powerlaw_tangent": (C.c_int, [_vp, _dp, _vp, _vp, _vp]),
    "jfft_powerlaw_jacobi_diag": (C.c_int, [_vp, _dp, _vp, _vp]),
    "jfft_topopt_eval": (C.c_int, [_vp, _vp, C.c_double, C.c_double, _dp, C.c_double, C.c_double,
                                   C.c_int, _dp, _vp, C.POINTER(C.c_int)]),
    "jfft_topopt_lbfgs": (C.c_int, [_vp, _vp, C.c_double, C.c_double, _dp, C.c_double, C.c_double,
                                    C.c_int, C.c_int, C.c_int, _dp, _dp, C.POINTER(C.c_int),
                                    C.POINTER(C.c_int), C.POINTER(C.c_int),
                                    C.POINTER(C.c_longlong)]),
    "jfft_destroy_cell": (None, [_vp]),
    "jfft_last_error": (C.c_char_p, []),
    "jfft_version": (C.c_char_p, []),
}
EXPORTED_SYMBOLS = tuple(_SIGS)

_lib = None


class JfftError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"jfft {_STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = _STATUS.get(status, str(status))


def load_library(path: str | None = None):
    """Load libjfft.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIBPATH
    if not os.path.exists(p):
        raise ImportError(f"{p} not found: build it with `python paper_2508_02613_amd/build.py` "
                          "(the solver has no CPU fallback)")
    lib = C.CDLL(p)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def lame_from_nu(nu: float):
    return nu / ((1 + nu) * (1 - 2 * nu)), 1.0 / (2 * (1 + nu))


def _check(st):
    if st != 0:
        msg = _lib.jfft_last_error().decode(errors="replace")
        raise JfftError(st, msg)


@dataclass
class NewtonReport:
    """Outcome of solve_newton: Newton steps, convergence, PCG iterations per
    step and ||f|| before each step (and at the end)."""
    steps: int
    converged: bool
    pcg_iters: list
    res: list


@dataclass
class Report:
    iters: int
    outer: int
    status: str
    rel_res: float
    rel_res_true: float
    setup_ms: float
    loop_ms: float
    post_ms: float


def _report(rep):
    return Report(rep.iters, rep.outer, _STATUS.get(rep.status, str(rep.status)), rep.rel_res,
                  rep.rel_res_true, rep.setup_ms, rep.loop_ms, rep.post_ms)


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the J-FFT library needs a ROCm GPU (torch.cuda.is_available() is False)")
    return torch


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


class Cell:
    """One periodic cell, or a group of `batch` cells of one shape, on one GPU
    stream.

    shape: (ny, nx) or (nz, ny, nx) node counts (x fastest, as the E arrays);
    precision FP64 or MIXED; pc one of PC_*; stream a torch.cuda.Stream (None =
    current stream).  The workspace is a torch uint8 tensor bound to the cell.
    With batch > 1, material fields and results carry a leading cell index and
    solve_batch replaces solve.  element (2D): "quad" (bilinear, 2 x 2 Gauss
    points) or "tri" (two linear triangles per pixel, the paper's 2D element).
    """

    def __init__(self, shape, precision=FP64, pc=PC_GREEN_JACOBI, lengths=None, stream=None,
                 device=None, batch=1, element="quad", workspace=True):
        torch = _torch()
        lib = load_library()
        self.torch = torch
        self.shape = tuple(int(s) for s in shape)
        self.dim = len(self.shape)
        self.device = torch.device(device if device is not None else "cuda")
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        n = (C.c_int * 3)(*(list(self.shape[::-1]) + [1] * (3 - self.dim)))
        ln = None
        if lengths is not None:
            ln = (C.c_double * 3)(*(list(lengths) + [1.0] * (3 - self.dim)))
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.jfft_create_batch(self.dim, n, ln, int(precision), int(pc), int(batch),
                                         C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self.batch = int(batch)
        self._h = h
        if element not in ("quad", "tri"):
            raise ValueError(f"unknown element {element!r}")
        self.element = element
        if element == "tri":
            _check(lib.jfft_set_element(h, 1))
        self._lib = lib
        nb = C.c_size_t(0)
        _check(lib.jfft_workspace_bytes(h, C.byref(nb)))
        self.workspace_bytes = int(nb.value)
        self._ws = None
        if workspace:  # workspace=False: for solve_static only (no device memory here)
            with torch.cuda.stream(self.stream):
                self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8,
                                       device=self.device)
            base = self._ws.data_ptr()
            aligned = (base + 255) // 256 * 256
            _check(lib.jfft_bind_workspace(h, C.c_void_p(aligned), self.workspace_bytes))
        self.N = int(np.prod(self.shape))
        self.ds = self.dim * (self.dim + 1) // 2

    # ----------------------------------------------------------------- api
    def close(self):
        if getattr(self, "_h", None):
            self._lib.jfft_destroy_cell(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a, shape=None):
        torch = self.torch
        if isinstance(a, np.ndarray):
            a = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
        t = a.to(device=self.device, dtype=torch.float64).contiguous()
        if shape is not None:
            assert tuple(t.shape) == tuple(shape), (t.shape, shape)
        return t

    def _nq(self):
        # quadrature points per element: 2^d Gauss points, or one per triangle
        return 2 if self.element == "tri" else 2 ** self.dim

    def set_material(self, E, nu=None, lame=None):
        E = self._dev(E, self.shape if self.batch == 1 else (self.batch,) + self.shape)
        self._E = E
        if lame is not None:
            _check(self._lib.jfft_set_material_lame(self._h, _ptr(E), float(lame[0]), float(lame[1])))
        else:
            _check(self._lib.jfft_set_material(self._h, _ptr(E), float(nu)))

    def set_void_value(self, v):
        _check(self._lib.jfft_set_void_value(self._h, float(v)))

    def set_diag_method(self, method="closed_form"):
        """How diag(K) is formed for the Jacobi part (Sec. 3.2): "closed_form"
        (isotropic Q1, one pass over E) or "probing" (Algorithm 2 as stated).
        Takes effect at the next set_material."""
        codes = {"closed_form": 0, "probing": 1}
        if method not in codes:
            raise ValueError(f"unknown diagonal method {method!r}")
        _check(self._lib.jfft_set_diag_method(self._h, codes[method]))

    def set_stop_rule(self, absolute=False):
        """absolute=False: ||r|| <= tol ||f||; True: ||r||^2 <= tol (the paper's runs)."""
        _check(self._lib.jfft_set_stop_rule(self._h, 1 if absolute else 0))

    def set_mixed_params(self, inner_tol=1e-6, max_outer=30, inner_cap=None, continue_cg=None,
                         reduction=1e-2):
        """Mixed refinement: inner tolerance of a restarted sweep, sweep cap,
        FP32 iteration cap per sweep, and whether later sweeps continue the
        FP32 CG (reliable updates every `reduction` of the residual, the
        default) or restart it."""
        _check(self._lib.jfft_set_mixed_params(self._h, float(inner_tol), int(max_outer)))
        if inner_cap is not None:
            _check(self._lib.jfft_set_mixed_inner_cap(self._h, int(inner_cap)))
        if continue_cg is not None:
            _check(self._lib.jfft_set_mixed_continue(self._h, 1 if continue_cg else 0,
                                                     float(reduction)))

    def solve(self, macro, tol=1e-8, maxit=1000, u0=None, want_sigma=False, out=None):
        """Returns (u [d, ...] device tensor, sigma_bar numpy, Report, sigma or None)."""
        torch = self.torch
        vshape = (self.dim,) + self.shape
        u = out if out is not None else torch.empty(vshape, dtype=torch.float64, device=self.device)
        sig = None
        if want_sigma:
            sig = torch.empty((self.ds, self._nq()) + self.shape, dtype=torch.float64,
                              device=self.device)
        u0t = self._dev(u0, vshape) if u0 is not None else None
        m = (C.c_double * self.ds)(*[float(v) for v in np.asarray(macro, dtype=float)])
        sbar = (C.c_double * self.ds)()
        rep = _Report()
        st = self._lib.jfft_solve(self._h, m, float(tol), int(maxit), _ptr(u0t), _ptr(u),
                                  _ptr(sig), sbar, C.byref(rep))
        if st not in (0, 4, 5):
            _check(st)
        return u, np.array(sbar[:]), _report(rep), sig

    def solve_static(self, E, nu, macro, tol=1e-8, maxit=1000, u0=None, u=None, sigma=None):
        """jfft_solve_static: set the material and solve in the library's
        static workspace (no device allocation inside the call).  u (and sigma,
        if given) are caller-owned device tensors; allocated here when None.
        Returns (u, sigma_bar, Report, sigma)."""
        torch = self.torch
        vshape = (self.dim,) + self.shape
        E = self._dev(E, self.shape)
        self._E = E
        if u is None:
            u = torch.empty(vshape, dtype=torch.float64, device=self.device)
        u0t = self._dev(u0, vshape) if u0 is not None else None
        m = (C.c_double * self.ds)(*[float(v) for v in np.asarray(macro, dtype=float)])
        sbar = (C.c_double * self.ds)()
        rep = _Report()
        st = self._lib.jfft_solve_static(self._h, _ptr(E), float(nu), m, float(tol), int(maxit),
                                         _ptr(u0t), _ptr(u), _ptr(sigma), sbar, C.byref(rep))
        if st not in (0, 4, 5):
            _check(st)
        return u, np.array(sbar[:]), _report(rep), sigma

    def solve_batch(self, macros, tol=1e-8, maxit=1000, u0=None, want_sigma=False, out=None):
        """All cells of the group: macros [B, d*].  Returns (u [B, d, ...],
        sigma_bar [B, d*], [Report] * B, sigma [B, d*, 2^d, ...] or None)."""
        torch = self.torch
        B = self.batch
        vshape = (B, self.dim) + self.shape
        u = out if out is not None else torch.empty(vshape, dtype=torch.float64, device=self.device)
        sig = None
        if want_sigma:
            sig = torch.empty((B, self.ds, self._nq()) + self.shape, dtype=torch.float64,
                              device=self.device)
        u0t = self._dev(u0, vshape) if u0 is not None else None
        mac = np.ascontiguousarray(np.asarray(macros, dtype=np.float64).reshape(B, self.ds))
        sbar = np.zeros((B, self.ds))
        reps = (_Report * B)()
        st = self._lib.jfft_solve_batch(self._h, mac.ctypes.data_as(_dp), float(tol), int(maxit),
                                        _ptr(u0t), _ptr(u), _ptr(sig), sbar.ctypes.data_as(_dp),
                                        reps)
        if st not in (0, 4, 5):
            _check(st)
        return u, sbar, [_report(r) for r in reps], sig

    # ------------------------------------------- continuous batching (slots)
    SLOT_FREE, SLOT_RUNNING, SLOT_FINISHED = 0, 1, 2

    def slot_admit(self, slot, E, nu, macro, tol=1e-8, maxit=1000):
        """Start one cell's solve in slot `slot` of the group
        (jfft_slot_admit): E [shape], macro [d*]."""
        E = self._dev(E, self.shape)
        m = (C.c_double * self.ds)(*[float(v) for v in np.asarray(macro, dtype=float)])
        _check(self._lib.jfft_slot_admit(self._h, int(slot), _ptr(E), float(nu), m, float(tol),
                                         int(maxit)))

    def slots_step(self, iterations=8):
        """At least `iterations` PCG iterations of every running slot; returns
        the slot states (SLOT_FREE / SLOT_RUNNING / SLOT_FINISHED) as an array."""
        st = (C.c_int * self.batch)()
        _check(self._lib.jfft_slots_step(self._h, int(iterations), st))
        return np.array(st[:], dtype=np.int32)

    def slots_run(self, max_ms=2.0):
        """Chunks of PCG iterations until a slot finishes, none runs, or
        max_ms have passed (jfft_slots_run); returns the slot states."""
        st = (C.c_int * self.batch)()
        _check(self._lib.jfft_slots_run(self._h, float(max_ms), st))
        return np.array(st[:], dtype=np.int32)

    def slot_harvest(self, slot, want_u=True, want_sigma=False):
        """Results of a finished slot, which becomes free: (u [d, ...] or
        None, sigma_bar [d*], Report, sigma [d*, 2^d, ...] or None)."""
        torch = self.torch
        u = sig = None
        if want_u:
            u = torch.empty((self.dim,) + self.shape, dtype=torch.float64, device=self.device)
        if want_sigma:
            sig = torch.empty((self.ds, self._nq()) + self.shape, dtype=torch.float64,
                              device=self.device)
        sbar = (C.c_double * self.ds)()
        rep = _Report()
        st = self._lib.jfft_slot_harvest(self._h, int(slot), _ptr(u), _ptr(sig), sbar,
                                         C.byref(rep))
        if st not in (0, 4, 5):
            _check(st)
        return u, np.array(sbar[:]), _report(rep), sig

    def tunables(self):
        t = _Tunables()
        _check(self._lib.jfft_get_tunables(self._h, C.byref(t)))
        return {"tz": int(t.tz), "ygrid": int(t.ygrid), "tiles2d": int(t.tiles2d),
                "xrows": int(t.xrows), "fused_control": int(t.fused_control),
                "tiles3d": int(t.tiles3d)}

    def set_tunables(self, tz=None, ygrid=None, tiles2d=None, xrows=None, fused_control=None,
                     tiles3d=None):
        """Launch parameters (None keeps the current value; see jfft_tunables)."""
        cur = self.tunables()
        t = _Tunables(int(tz if tz is not None else cur["tz"]),
                      int(ygrid if ygrid is not None else cur["ygrid"]),
                      int(tiles2d if tiles2d is not None else cur["tiles2d"]),
                      int(xrows if xrows is not None else cur["xrows"]),
                      int(fused_control if fused_control is not None
                          else cur["fused_control"]),
                      int(tiles3d if tiles3d is not None else cur["tiles3d"]))
        _check(self._lib.jfft_set_tunables(self._h, C.byref(t)))

    def set_graph_iterations(self, iterations):
        """0: direct launches; even k in [2, 64]: replay k PCG iterations as one HIP graph."""
        _check(self._lib.jfft_set_graph_iterations(self._h, int(iterations)))

    def apply_stiffness(self, x):
        x = self._dev(x, (self.dim,) + self.shape)
        out = self.torch.empty_like(x)
        _check(self._lib.jfft_apply_stiffness(self._h, _ptr(x), _ptr(out)))
        self.stream.synchronize()
        return out

    def apply_precond(self, x, fp32=False):
        """M^-1 x in FP64, or (fp32=True, mixed cells) as the FP32 inner
        solves apply it (x rounded to FP32, the result widened to FP64)."""
        x = self._dev(x, (self.dim,) + self.shape)
        out = self.torch.empty_like(x)
        fn = self._lib.jfft_apply_precond_fp32 if fp32 else self._lib.jfft_apply_precond
        _check(fn(self._h, _ptr(x), _ptr(out)))
        self.stream.synchronize()
        return out

    def assemble_rhs(self, macro):
        out = self.torch.empty((self.dim,) + self.shape, dtype=self.torch.float64, device=self.device)
        m = (C.c_double * self.ds)(*[float(v) for v in np.asarray(macro, dtype=float)])
        _check(self._lib.jfft_assemble_rhs(self._h, m, _ptr(out)))
        self.stream.synchronize()
        return out

    def jacobi_diag(self):
        out = self.torch.empty((self.dim,) + self.shape, dtype=self.torch.float64, device=self.device)
        _check(self._lib.jfft_jacobi_diag(self._h, _ptr(out)))
        self.stream.synchronize()
        return out

    # ------------------------------------------- power-law Newton (Sec. 4)
    def set_material_powerlaw(self, phase, K=2.0, sigma0=0.5, eps0=0.1, n=5.0, K_incl=2.0,
                              mu_incl=0.5):
        """phase [nz, ny, nx]: 1 = power-law matrix, 0 = linear inclusion."""
        ph = self._dev(phase, self.shape)
        self._E = ph
        _check(self._lib.jfft_set_material_powerlaw(self._h, _ptr(ph), float(K), float(sigma0),
                                                    float(eps0), float(n), float(K_incl),
                                                    float(mu_incl)))

    def solve_newton(self, macro, newton_tol=1e-5, pcg_tol=1e-8, max_newton=20, maxit=5000,
                     out=None):
        """Newton from u = 0.  Returns (u [3, ...] device tensor (mean removed),
        sigma_bar numpy [6], NewtonReport)."""
        torch = self.torch
        u = out if out is not None else torch.empty((3,) + self.shape, dtype=torch.float64,
                                                    device=self.device)
        m = (C.c_double * 6)(*[float(v) for v in np.asarray(macro, dtype=float)])
        sbar = (C.c_double * 6)()
        its = (C.c_int * max(1, int(max_newton)))()
        res = (C.c_double * (int(max_newton) + 1))()
        steps = C.c_int(0)
        st = self._lib.jfft_solve_newton(self._h, m, float(newton_tol), float(pcg_tol),
                                         int(max_newton), int(maxit), _ptr(u), sbar, its, res,
                                         C.byref(steps))
        if st not in (0, 4):
            _check(st)
        k = int(steps.value)
        rep = NewtonReport(steps=k, converged=st == 0, pcg_iters=[int(v) for v in its[:k]],
                           res=[float(v) for v in res[:k + 1]])
        return u, np.array(sbar[:]), rep

    def _pl_args(self, macro, uk):
        m = (C.c_double * 6)(*[float(v) for v in np.asarray(macro, dtype=float)])
        return m, self._dev(uk, (3,) + self.shape)

    def powerlaw_force(self, macro, uk):
        """f = -B^T W sigma(E + B uk)."""
        m, ukt = self._pl_args(macro, uk)
        out = self.torch.empty_like(ukt)
        _check(self._lib.jfft_powerlaw_force(self._h, m, _ptr(ukt), _ptr(out)))
        return out

    def powerlaw_tangent(self, macro, uk, x):
        """K(uk) x."""
        m, ukt = self._pl_args(macro, uk)
        x = self._dev(x, (3,) + self.shape)
        out = self.torch.empty_like(x)
        _check(self._lib.jfft_powerlaw_tangent(self._h, m, _ptr(ukt), _ptr(x), _ptr(out)))
        return out

    def powerlaw_jacobi_diag(self, macro, uk):
        """diag(K(uk)) by Algorithm 2."""
        m, ukt = self._pl_args(macro, uk)
        out = self.torch.empty_like(ukt)
        _check(self._lib.jfft_powerlaw_jacobi_diag(self._h, m, _ptr(ukt), _ptr(out)))
        return out

    # ------------------------ phase-field topology optimisation (Sec. 4)
    def topopt_eval(self, rho, targets, eta=0.01, tol=1e-8, maxit=20000, lame0=(2 / 3, 0.5)):
        """Group of 3 triangle cells: f = (f, f_sigma, f_pf), gradient [ny, nx]
        (device tensor) and the three solves' iterations."""
        r = self._dev(rho, self.shape)
        grad = self.torch.empty_like(r)
        t = np.ascontiguousarray(np.asarray(targets, dtype=np.float64).reshape(9))
        f = (C.c_double * 3)()
        its = (C.c_int * 3)()
        _check(self._lib.jfft_topopt_eval(self._h, _ptr(r), float(lame0[0]), float(lame0[1]),
                                          t.ctypes.data_as(_dp), float(eta), float(tol),
                                          int(maxit), f, _ptr(grad), its))
        return np.array(f[:]), grad, list(its)

    def topopt_lbfgs(self, rho0, targets, n_iter, eta=0.01, tol=1e-8, maxit=20000, m=10,
                     lame0=(2 / 3, 0.5)):
        """Projected L-BFGS from rho0.  Returns (rho device tensor, dict with
        f, gnorm, iters per accepted iterate, steps, evals)."""
        r = self._dev(rho0, self.shape).clone()
        t = np.ascontiguousarray(np.asarray(targets, dtype=np.float64).reshape(9))
        fh = (C.c_double * (n_iter + 1))()
        gh = (C.c_double * (n_iter + 1))()
        ih = (C.c_int * (3 * (n_iter + 1)))()
        steps, evals, total = C.c_int(0), C.c_int(0), C.c_longlong(0)
        _check(self._lib.jfft_topopt_lbfgs(self._h, _ptr(r), float(lame0[0]), float(lame0[1]),
                                           t.ctypes.data_as(_dp), float(eta), float(tol),
                                           int(maxit), int(n_iter), int(m), fh, gh, ih,
                                           C.byref(steps), C.byref(evals), C.byref(total)))
        k = int(steps.value)
        return r, {"f": list(fh[:k + 1]), "gnorm": list(gh[:k + 1]),
                   "iters": [list(ih[3 * i:3 * i + 3]) for i in range(k + 1)], "steps": k,
                   "evals": int(evals.value), "pcg_total": int(total.value)}

    def enable_history(self, cap):
        _check(self._lib.jfft_enable_history(self._h, int(cap)))

    def history(self, cap, index=0):
        a = np.zeros(cap)
        b = np.zeros(cap)
        r = np.zeros(cap)
        cnt = C.c_int(0)
        _check(self._lib.jfft_get_batch_history(self._h, int(index), a.ctypes.data_as(_dp),
                                                b.ctypes.data_as(_dp), r.ctypes.data_as(_dp),
                                                int(cap), C.byref(cnt)))
        k = cnt.value
        return a[:k], b[:k], r[:k]

    def enable_timing(self, on=True):
        _check(self._lib.jfft_enable_timing(self._h, 1 if on else 0))

    def reset_timing(self):
        _check(self._lib.jfft_reset_timing(self._h))

    def kernel_stats(self):
        """{kernel name: (launches, total ms)} measured with HIP events on the cell's stream."""
        cnt = C.c_int(0)
        _check(self._lib.jfft_kernel_stats(self._h, -1, None, None, None, C.byref(cnt)))
        out = {}
        for i in range(cnt.value):
            nm = C.c_char_p()
            la = C.c_long(0)
            ms = C.c_double(0)
            _check(self._lib.jfft_kernel_stats(self._h, i, C.byref(nm), C.byref(la), C.byref(ms),
                                               None))
            if la.value:
                out[nm.value.decode()] = (int(la.value), float(ms.value))
        return out


def effective_stiffness(E, nu=0.3, lame=None, tol=1e-8, maxit=20000, precision=FP64,
                        pc=PC_GREEN_JACOBI, lengths=None, stream=None, graph_iterations=0):
    """Homogenised Mandel stiffness of one periodic cell (Sec. 5).

    The d* unit macro strains e_g are solved as one group of d* cells that
    share the material field E; column g of the result is sigma_bar for e_g.
    Returns (C [d*, d*] numpy array, [Report] per load case)."""
    torch = _torch()
    if isinstance(E, np.ndarray):
        E = torch.from_numpy(np.ascontiguousarray(E, dtype=np.float64))
    shape = tuple(E.shape)
    dim = len(shape)
    ds = dim * (dim + 1) // 2
    grp = Cell(shape, precision=precision, pc=pc, lengths=lengths, stream=stream, batch=ds)
    try:
        if graph_iterations:
            grp.set_graph_iterations(graph_iterations)
        Ed = E.to(device=grp.device, dtype=torch.float64)
        grp.set_material(Ed.unsqueeze(0).expand((ds,) + shape).contiguous(), nu=nu, lame=lame)
        _, sbar, reps, _ = grp.solve_batch(np.eye(ds), tol=tol, maxit=maxit)
    finally:
        grp.close()
    return np.ascontiguousarray(sbar.T), reps
