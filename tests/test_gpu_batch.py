"""GPU tests of cell groups (jfft_create_batch / jfft_solve_batch) and of the
graph-replayed PCG loop.

Every reduction of the library has a layout fixed by the cell shape alone, so
a cell solved inside a group must give bitwise the results of the same cell
solved alone, whatever the other cells hold and whenever they stop; a loop
replayed from a captured HIP graph runs the same kernels with the same
arguments, so it must match direct launches bitwise too.  Parity of the
single-cell path with the oracle is covered in test_gpu_parity.py; one group
member is checked against the oracle here as well.
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


def _fields(shape, contrasts, seeds):
    return [ji.grf_field(shape, c, seed=s, ell=0.15) for c, s in zip(contrasts, seeds)]


def _macros(dim, B, seed):
    ds = dim * (dim + 1) // 2
    return np.random.default_rng(seed).uniform(-1.0, 1.0, (B, ds))


def _single(pkg, shape, E, macro, prec, pc, tol, maxit, hist=0):
    cell = pkg.Cell(shape, precision=prec, pc=pc)
    cell.set_material(E, nu=0.3)
    if hist:
        cell.enable_history(hist)
    u, sbar, rep, sig = cell.solve(macro, tol=tol, maxit=maxit, want_sigma=True)
    out = (u.cpu().numpy(), sbar, rep, sig.cpu().numpy())
    h = cell.history(hist) if hist else None
    cell.close()
    return out, h


@pytest.mark.parametrize("shape,prec,pc", [
    ((32, 32), 0, 3), ((24, 20), 0, 1), ((16, 16, 16), 0, 3), ((12, 10, 18), 1, 3),
    ((8, 8, 8), 0, 2), ((16, 16, 16), 1, 1)])
def test_group_equals_single(shape, prec, pc):
    pkg = _pkg()
    say(f"group vs single {shape} prec={prec} pc={pc}")
    dim = len(shape)
    B = 4
    # mixed difficulty: the cells stop at different iterations
    Es = _fields(shape, [10.0, 1e4, 1e2, 1e3], [11, 12, 13, 14])
    macros = _macros(dim, B, 5)
    tol, maxit = 1e-8, 5000
    grp = pkg.Cell(shape, precision=prec, pc=pc, batch=B)
    assert grp.batch == B
    grp.set_material(np.stack(Es), nu=0.3)
    hist = 64 if prec == 0 else 0
    if hist:
        grp.enable_history(hist)
    u, sbar, reps, sig = grp.solve_batch(macros, tol=tol, maxit=maxit, want_sigma=True)
    u = u.cpu().numpy()
    sig = sig.cpu().numpy()
    iters = []
    for i in range(B):
        (us, sbs, rs, sgs), hs = _single(pkg, shape, Es[i], macros[i], prec, pc, tol, maxit, hist)
        assert reps[i].status == "ok" and rs.status == "ok"
        assert reps[i].iters == rs.iters and reps[i].outer == rs.outer
        assert np.array_equal(u[i], us), f"cell {i}: u differs from the single-cell solve"
        assert np.array_equal(sbar[i], sbs)
        assert np.array_equal(sig[i], sgs)
        assert reps[i].rel_res_true == rs.rel_res_true
        if hist:
            hg = grp.history(hist, index=i)
            for a, b in zip(hg, hs):
                assert np.array_equal(a, b, equal_nan=True)
            k = min(hist, rs.iters)
            assert len(hg[1]) == k
            assert not np.isnan(hg[1][:min(k, rs.iters - 1)]).any()
            if rs.iters <= hist:
                assert np.isnan(hg[1][-1]), "the last iteration forms no beta"
        iters.append(rs.iters)
    assert len(set(iters)) > 1, "the cells should stop at different iterations"
    grp.close()


def test_group_member_matches_oracle():
    pkg = _pkg()
    say("group member vs oracle 32x32")
    shape = (32, 32)
    Es = _fields(shape, [1e3, 1e4, 10.0], [21, 22, 23])
    macros = _macros(2, 3, 9)
    grp = pkg.Cell(shape, pc=pkg.PC_GREEN_JACOBI, batch=3)
    grp.set_material(np.stack(Es), nu=0.3)
    u, sbar, reps, _ = grp.solve_batch(macros, tol=1e-12, maxit=5000)
    u = u.cpu().numpy()
    for i in range(3):
        ref = oracle.solve(Es[i], macros[i], LAM, MU, pc=3, tol=1e-12, maxit=5000, remove_mean=True)
        say(f"  cell {i}: iters gpu={reps[i].iters} oracle={ref.iters}")
        assert reps[i].status == "ok" and ref.status == "ok"
        assert abs(reps[i].iters - ref.iters) <= 0.03 * ref.iters  # rounding-sensitive at 1e-12
        err = np.linalg.norm(u[i] - ref.u) / np.linalg.norm(ref.u)
        assert err <= 1e-9, (i, err)
        np.testing.assert_allclose(sbar[i], ref.sigma_bar, rtol=1e-9, atol=1e-12)
    grp.close()


def test_group_homogeneous_and_zero_macro_members():
    """A homogeneous cell and a zero load stop at iteration 0 while the others run."""
    pkg = _pkg()
    say("group with trivial members 16^3")
    shape = (16, 16, 16)
    Es = [np.ones(shape), ji.grf_field(shape, 1e3, seed=4, ell=0.15), ji.grf_field(shape, 1e2, seed=5)]
    macros = _macros(3, 3, 2)
    macros[2] = 0.0
    grp = pkg.Cell(shape, pc=pkg.PC_GREEN_JACOBI, batch=3)
    grp.set_material(np.stack(Es), nu=0.3)
    u, sbar, reps, _ = grp.solve_batch(macros, tol=1e-8, maxit=2000)
    u = u.cpu().numpy()
    assert reps[0].iters == 0 and reps[2].iters == 0 and reps[1].iters > 5
    assert np.abs(u[0]).max() == 0.0 and np.abs(u[2]).max() == 0.0
    (us, sbs, rs, _), _ = _single(pkg, shape, Es[1], macros[1], 0, 3, 1e-8, 2000)
    assert np.array_equal(u[1], us) and rs.iters == reps[1].iters
    # homogeneous cell: sigma_bar = C^ macro (Mandel: lambda tr(eps) 1 + 2 mu eps)
    m = macros[0]
    expect = 2 * MU * m + LAM * m[:3].sum() * np.array([1, 1, 1, 0, 0, 0])
    np.testing.assert_allclose(sbar[0], expect, rtol=0, atol=1e-13)
    assert np.abs(sbar[2]).max() == 0.0
    grp.close()


def test_group_not_converged_member():
    pkg = _pkg()
    say("group with a member hitting maxit")
    shape = (24, 20)
    Es = [ji.grf_field(shape, 10.0, seed=1), ji.grf_field(shape, 1e4, seed=2, ell=0.1)]
    grp = pkg.Cell(shape, pc=pkg.PC_NONE, batch=2)
    grp.set_material(np.stack(Es), nu=0.3)
    u, sbar, reps, _ = grp.solve_batch(_macros(2, 2, 3), tol=1e-10, maxit=60)
    st = {r.status for r in reps}
    assert "not_converged" in st
    assert all(r.iters <= 60 for r in reps)
    grp.close()


@pytest.mark.parametrize("shape,prec,G", [((16, 16, 16), 0, 8), ((16, 16, 16), 1, 16),
                                          ((32, 32), 0, 2), ((12, 10, 18), 0, 64)])
def test_graph_replay_equals_direct(shape, prec, G):
    pkg = _pkg()
    import torch

    say(f"graph replay {shape} prec={prec} G={G}")
    s = torch.cuda.Stream()
    B = 3
    dim = len(shape)
    Es = _fields(shape, [1e3, 1e1, 1e4], [31, 32, 33])
    macros = _macros(dim, B, 7)
    res = []
    for g in (0, G):
        grp = pkg.Cell(shape, precision=prec, pc=pkg.PC_GREEN_JACOBI, batch=B, stream=s)
        grp.set_graph_iterations(g)
        grp.set_material(np.stack(Es), nu=0.3)
        # two solves: the second replays the graph captured by the first
        for rep_i in range(2):
            u, sbar, reps, _ = grp.solve_batch(macros * (1 + rep_i), tol=1e-8, maxit=3000)
            res.append((g, rep_i, u.cpu().numpy(), sbar.copy(), [r.iters for r in reps]))
        # a new material rebuilds the graph
        grp.set_material(np.stack(Es[::-1]), nu=0.3)
        u, sbar, reps, _ = grp.solve_batch(macros, tol=1e-8, maxit=3000)
        res.append((g, 2, u.cpu().numpy(), sbar.copy(), [r.iters for r in reps]))
        grp.close()
    direct = [r for r in res if r[0] == 0]
    graph = [r for r in res if r[0] == G]
    for a, b in zip(direct, graph):
        assert a[1] == b[1]
        assert a[4] == b[4], (a[4], b[4])
        assert np.array_equal(a[2], b[2])
        assert np.array_equal(a[3], b[3])
    # the doubled load doubles the solution (linearity, exact up to rounding)
    np.testing.assert_allclose(direct[1][2], 2 * direct[0][2], rtol=0, atol=1e-9 * np.abs(direct[0][2]).max())


def test_group_argument_errors():
    pkg = _pkg()
    import torch

    say("group argument errors")
    grp = pkg.Cell((8, 8), batch=2)
    grp.set_material(np.ones((2, 8, 8)), nu=0.3)
    with pytest.raises(pkg.JfftError) as e:
        grp.solve([0.1, 0, 0])
    assert e.value.name == "invalid"
    with pytest.raises(pkg.JfftError):
        grp.apply_stiffness(np.zeros((2, 8, 8)))
    with pytest.raises(pkg.JfftError):
        grp.set_graph_iterations(3)
    with pytest.raises(pkg.JfftError):
        grp.set_graph_iterations(66)
    with pytest.raises(pkg.JfftError):
        grp.history(8, index=2)
    bad = np.ones((2, 8, 8))
    bad[1, 3, 3] = -1.0
    with pytest.raises(pkg.JfftError) as e:
        grp.set_material(bad, nu=0.3)
    assert "cell 1" in str(e.value)
    grp.close()
    with pytest.raises(pkg.JfftError):
        pkg.Cell((8, 8), batch=0)
    # graph replay on the legacy default stream is refused
    if torch.cuda.current_stream().cuda_stream == 0:
        c = pkg.Cell((8, 8))
        with pytest.raises(pkg.JfftError):
            c.set_graph_iterations(4)
        c.close()
