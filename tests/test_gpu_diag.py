"""GPU tests of the two ways the library forms diag(K) for the Jacobi part of
the preconditioner (Sec. 3.2): Algorithm 2 as stated (d 2^d applications of
K to unit combs) and its closed form for isotropic Q1 elements, diag = k_a
times the box sum of the moduli (the closed form itself is pinned against
the oracle's Algorithm 2 in test_oracle_pins.py::test_p6_alg2_diagonal).
The two must agree up to rounding, on cubic and non-cubic elements, with
voids, and give the same solves.
"""
import numpy as np
import pytest

import jfft_inputs as ji
import oracle

pytestmark = pytest.mark.gpu

LAM, MU = oracle.lame_from_nu(0.3)


def _pkg():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    import paper_2508_02613_amd as pkg

    pkg.load_library()
    return pkg


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


CASES = [((32, 32), None), ((24, 20), (1.0, 0.6)), ((16, 16, 16), None),
         ((12, 10, 18), (1.3, 0.7, 1.0)), ((8, 8, 8), (1.0, 1.0, 2.0))]


def _field(shape, voids, seed):
    E = ji.uniform_random_field(shape, 1.0, 1e3, seed=seed)
    if voids:
        # a void region: every element around some nodes is zero (diag = 0 there)
        sl = tuple(slice(2, 5) for _ in shape)
        E[sl] = 0.0
    return E


@pytest.mark.parametrize("shape,lengths", CASES)
@pytest.mark.parametrize("voids", [False, True])
def test_closed_form_equals_probing(shape, lengths, voids):
    pkg = _pkg()
    say(f"diag closed form vs probing {shape} lengths={lengths} voids={voids}")
    dim = len(shape)
    E = _field(shape, voids, 7)
    x = np.random.default_rng(1).standard_normal((dim,) + shape)
    out = {}
    for method in ("closed_form", "probing"):
        cell = pkg.Cell(shape, pc=pkg.PC_JACOBI, lengths=lengths)
        cell.set_void_value(2.5)
        cell.set_diag_method(method)
        cell.set_material(E, nu=0.3)
        out[method] = cell.apply_precond(x).cpu().numpy()  # diag^-1 x after the void rule
        probe = cell.jacobi_diag().cpu().numpy()           # Algorithm 2, zeros kept
        cell.close()
    a, b = out["closed_form"], out["probing"]
    rel = np.abs(a - b).max() / np.abs(b).max()
    say(f"  max |closed - probing| / max = {rel:.2e}")
    assert rel <= 1e-13
    # where Algorithm 2 gives an exact zero both apply the void value
    zero = probe == 0.0
    assert zero.any() == voids
    if voids:
        np.testing.assert_allclose(a[zero], x[zero] / 2.5, rtol=4e-15)
    # and the probing diagonal is the oracle's (Algorithm 2 on the CPU)
    ref, _ = oracle.jacobi_diag(E, LAM, MU, lengths=lengths)
    assert np.abs(probe - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("shape,lengths", CASES)
@pytest.mark.parametrize("voids", [False, True])
def test_green_jacobi_closed_form_equals_probing(shape, lengths, voids):
    """The Green-Jacobi preconditioner built on the closed-form diagonal equals
    the one built on Algorithm 2's probing, with voids and rectangular
    elements."""
    pkg = _pkg()
    say(f"GJ closed form vs probing {shape} lengths={lengths} voids={voids}")
    dim = len(shape)
    E = _field(shape, voids, 11)
    x = np.random.default_rng(2).standard_normal((dim,) + shape)
    out = {}
    for method in ("closed_form", "probing"):
        cell = pkg.Cell(shape, pc=pkg.PC_GREEN_JACOBI, lengths=lengths)
        cell.set_void_value(0.4)
        cell.set_diag_method(method)
        cell.set_material(E, nu=0.3)
        out[method] = cell.apply_precond(x).cpu().numpy()
        cell.close()
    a, b = out["closed_form"], out["probing"]
    rel = np.abs(a - b).max() / np.abs(b).max()
    say(f"  max |closed - probing| / max = {rel:.2e}")
    assert rel <= 1e-12


@pytest.mark.parametrize("shape,lengths,prec", [((12, 10, 18), (1.3, 0.7, 1.0), 0),
                                                ((16, 16, 16), None, 1),
                                                ((24, 20), (1.0, 0.6), 0)])
def test_solves_agree(shape, lengths, prec):
    pkg = _pkg()
    say(f"solve closed form vs probing {shape} prec={prec}")
    dim = len(shape)
    E = ji.grf_field(shape, 1e3, seed=3, ell=0.15)
    macro = ji.unit_macro_strain(dim, 0)
    res = {}
    for method in ("closed_form", "probing"):
        cell = pkg.Cell(shape, precision=prec, pc=pkg.PC_GREEN_JACOBI, lengths=lengths)
        cell.set_diag_method(method)
        cell.set_material(E, nu=0.3)
        u, sbar, rep, _ = cell.solve(macro, tol=1e-10, maxit=5000)
        res[method] = (u.cpu().numpy(), sbar, rep)
        cell.close()
    (ua, sa, ra), (ub, sb, rb) = res["closed_form"], res["probing"]
    say(f"  iters {ra.iters} vs {rb.iters}")
    assert ra.status == "ok" and rb.status == "ok"
    assert abs(ra.iters - rb.iters) <= 1
    assert np.linalg.norm(ua - ub) / np.linalg.norm(ub) <= 1e-8
    np.testing.assert_allclose(sa, sb, rtol=1e-9, atol=1e-12)
    # the default is the closed form
    cell = pkg.Cell(shape, precision=prec, pc=pkg.PC_GREEN_JACOBI, lengths=lengths)
    cell.set_material(E, nu=0.3)
    u, sbar, rep, _ = cell.solve(macro, tol=1e-10, maxit=5000)
    cell.close()
    assert rep.iters == ra.iters and np.array_equal(u.cpu().numpy(), ua)


def test_method_argument_errors():
    pkg = _pkg()
    cell = pkg.Cell((8, 8))
    with pytest.raises(ValueError):
        cell.set_diag_method("dense")
    cell.set_material(np.ones((8, 8)), nu=0.3)
    cell.set_diag_method("probing")  # clears the material: J^1/2 must be formed again
    with pytest.raises(pkg.JfftError) as e:
        cell.solve([0.1, 0, 0])
    assert e.value.name == "no_material"
    cell.close()
