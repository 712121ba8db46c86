"""GPU tests of the launch-parameter autotuner: valid, cached, and neutral
for results (a tuned group equals single cells run with the same tile
shapes), and every tile shape solves the same problem."""
import numpy as np
import pytest

import jfft_inputs as ji

pytestmark = pytest.mark.gpu


def _pkg():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a GPU")
    import paper_2508_02613_amd as pkg

    pkg.load_library()
    return pkg


def say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.mark.parametrize("shape,batch", [((16, 16, 16), 3), ((32, 32), 4)])
def test_autotune_cached_and_result_neutral(shape, batch, tmp_path, monkeypatch):
    pkg = _pkg()
    from paper_2508_02613_amd import tune

    monkeypatch.setenv("JFFT_TUNE_CACHE", str(tmp_path / "tunables.json"))
    say(f"autotune {shape} batch {batch}")
    p = tune.autotune(shape, batch=batch, precision=pkg.MIXED, iters=12)
    say(f"  {p}")
    assert p["ygrid"] >= 1 and p["graph_iterations"] in (0, 8, 16)
    if len(shape) == 3:
        assert 2 <= p["tz"] <= shape[0] and p["tiles3d"] in (1, 2)
    else:
        assert p["tiles2d"] in (1, 2, 3, 4)
    assert p["xrows"] >= 1 and p["xrows"] & (p["xrows"] - 1) == 0
    assert (tmp_path / "tunables.json").exists()
    assert tune.autotune(shape, batch=batch, precision=pkg.MIXED) == p  # from the cache
    # another group size reuses the shape's tile shapes
    p2 = tune.autotune(shape, batch=batch + 1, precision=pkg.MIXED, iters=12)
    assert all(p2[k] == p[k] for k in tune.SHAPE_KEYS)
    dim = len(shape)
    Es = [ji.grf_field(shape, 1e3, seed=s, ell=0.15) for s in range(batch)]
    macros = np.random.default_rng(1).uniform(-1, 1, (batch, dim * (dim + 1) // 2))
    grp = pkg.Cell(shape, precision=pkg.MIXED, batch=batch, stream=__import__("torch").cuda.Stream())
    tune.apply(grp, p)
    grp.set_material(np.stack(Es), nu=0.3)
    u, sbar, reps, _ = grp.solve_batch(macros, tol=1e-8)
    u = u.cpu().numpy()
    grp.close()
    for i in range(batch):
        c = pkg.Cell(shape, precision=pkg.MIXED)
        c.set_tunables(tz=p["tz"], tiles2d=p["tiles2d"], tiles3d=p["tiles3d"], xrows=p["xrows"],
                       fused_control=p["fused_control"])
        c.set_material(Es[i], nu=0.3)
        ui, si, ri, _ = c.solve(macros[i], tol=1e-8)
        c.close()
        assert reps[i].iters == ri.iters
        assert np.array_equal(u[i], ui.cpu().numpy())
        assert np.array_equal(sbar[i], si)


def test_tunables_validation():
    pkg = _pkg()
    c = pkg.Cell((16, 16, 16))
    t = c.tunables()
    assert 2 <= t["tz"] <= 16 and t["ygrid"] >= 1
    with pytest.raises(pkg.JfftError):
        c.set_tunables(tz=1)
    with pytest.raises(pkg.JfftError):
        c.set_tunables(tz=17)
    with pytest.raises(pkg.JfftError):
        c.set_tunables(ygrid=0)
    with pytest.raises(pkg.JfftError):
        c.set_tunables(xrows=3)
    with pytest.raises(pkg.JfftError):
        c.set_tunables(tiles2d=5)
    with pytest.raises(pkg.JfftError):
        c.set_tunables(tiles3d=3)
    with pytest.raises(pkg.JfftError):
        c.set_tunables(tiles3d=-1)
    tz_auto = t["tz"]
    c.set_tunables(tz=8, ygrid=300, xrows=2)
    assert c.tunables() == {"tz": 8, "ygrid": 300, "tiles2d": 0, "xrows": 2, "fused_control": 0,
                            "tiles3d": 1}
    c.set_tunables(tz=0)  # back to the automatic choice
    assert c.tunables()["tz"] == tz_auto
    c.set_tunables(tz=8)
    c.set_tunables(tiles3d=2)
    assert c.tunables()["tiles3d"] == 2
    c.set_tunables(tiles3d=0)
    assert c.tunables()["tiles3d"] == 1
    c.set_tunables(xrows=1 << 20)  # clamped to the most rows that fit
    assert 2 <= c.tunables()["xrows"] < 1 << 20
    c.close()
    c = pkg.Cell((64, 64), precision=pkg.FP64)
    assert c.tunables()["tiles2d"] == 1
    c.set_tunables(tiles2d=2)
    assert c.tunables()["tiles2d"] == 2
    c.set_tunables(tiles2d=0)
    assert c.tunables()["tiles2d"] == 1
    c.close()
    c = pkg.Cell((16, 16, 16), precision=pkg.MIXED)
    d3 = c.tunables()["tiles3d"]
    assert d3 == 2 and c.tunables()["tiles2d"] == 0
    for t3 in (1, 2):
        c.set_tunables(tiles3d=t3)
        assert c.tunables()["tiles3d"] == t3
    c.set_tunables(tiles3d=0)
    assert c.tunables()["tiles3d"] == d3
    c.close()


@pytest.mark.parametrize("shape,prec", [((90, 72), "FP64"), ((90, 72), "MIXED"),
                                        ((30, 20, 18), "FP64"), ((30, 20, 18), "MIXED"),
                                        ((18, 36, 40), "MIXED"), ((40, 40, 40), "MIXED")])
def test_tile_shapes_solve_the_same_problem(shape, prec):
    """Every tile shape (2D block shapes 16 or 32 nodes wide and high, 3D
    blocks of 16 x 14 or 32 x 6 nodes, x-pass rows per block, down
    to one row) gives the same solution up to the regrouping of partial sums:
    iteration counts within one, fields within the solver tolerance.  The
    grids leave ragged tiles and blocks in every direction (3D shapes are
    (nz, ny, nx): 18 nodes in x are less than one 32-wide block; the cube
    runs the cubic form of the 3D element kernel, the others the general
    one)."""
    pkg = _pkg()
    dim = len(shape)
    E = ji.grf_field(shape, 1e3, seed=3, ell=0.15)
    macro = np.random.default_rng(2).uniform(-1, 1, dim * (dim + 1) // 2)
    ref = None
    c = pkg.Cell(shape, precision=getattr(pkg, prec))
    c.set_material(E, nu=0.3)
    rb = c.tunables()["xrows"]
    codes = (1, 2, 3, 4) if dim == 2 else (1, 2)
    key = "tiles2d" if dim == 2 else "tiles3d"
    shapes = [(t, xr) for t in codes for xr in (rb, 4, 1)]
    for t, xr in shapes:
        c.set_tunables(xrows=xr, **{key: t})
        u, sbar, rep, _ = c.solve(macro, tol=1e-10, maxit=5000)
        u = u.cpu().numpy()
        say(f"{shape} {prec} {key} {t} xrows {xr}: iters {rep.iters} res {rep.rel_res_true:.1e}")
        assert rep.status == "ok" and rep.rel_res_true <= 1.5e-10
        if ref is None:
            ref = (u, sbar, rep.iters)
            continue
        assert abs(rep.iters - ref[2]) <= 1
        assert np.abs(u - ref[0]).max() <= 1e-7 * np.abs(ref[0]).max()
        assert np.abs(sbar - ref[1]).max() <= 1e-8 * np.abs(ref[1]).max()
    c.close()


@pytest.mark.parametrize("shape,prec,graph", [((48, 40), "FP64", 0), ((48, 40), "MIXED", 8),
                                              ((20, 16, 18), "FP64", 8),
                                              ((20, 16, 18), "MIXED", 0)])
def test_fused_control_matches_separate_launches(shape, prec, graph):
    """The CG scalar steps run in the last block of their producer kernels
    or as single-block kernels (default): the same solve up to the order of
    the partial sums (iteration counts within one, fields within the
    tolerance), for a group of three cells that stop at different
    iterations, with and without graph replay; the history (alpha, beta,
    residuals) agrees to rounding on the common prefix."""
    import torch

    pkg = _pkg()
    dim = len(shape)
    ds = dim * (dim + 1) // 2
    Es = np.stack([ji.grf_field(shape, 10.0 ** (2 + k), seed=60 + k, ell=0.15) for k in range(3)])
    macros = np.random.default_rng(5).uniform(-1, 1, (3, ds))
    out = {}
    for fused in (1, 0):
        g = pkg.Cell(shape, precision=getattr(pkg, prec), batch=3, stream=torch.cuda.Stream())
        g.set_tunables(fused_control=fused)
        assert g.tunables()["fused_control"] == fused
        if graph:
            g.set_graph_iterations(graph)
        if prec == "FP64":
            g.enable_history(200)
        g.set_material(Es, nu=0.3)
        u, sbar, reps, _ = g.solve_batch(macros, tol=1e-10, maxit=5000)
        hist = [g.history(200, i) for i in range(3)] if prec == "FP64" else None
        out[fused] = (u.cpu().numpy(), sbar, reps, hist)
        g.close()
    (u1, s1, r1, h1), (u0, s0, r0, h0) = out[1], out[0]
    for i in range(3):
        say(f"{shape} {prec} graph {graph} cell {i}: iters fused {r1[i].iters} separate "
            f"{r0[i].iters}")
        assert r1[i].status == "ok" and r0[i].status == "ok"
        assert abs(r1[i].iters - r0[i].iters) <= 1
        assert np.abs(u1[i] - u0[i]).max() <= 1e-7 * np.abs(u0[i]).max()
        assert np.abs(s1[i] - s0[i]).max() <= 1e-8 * np.abs(s0[i]).max()
        if h1 is not None:
            k = min(len(h1[i][0]), len(h0[i][0]), 15)
            assert k >= 10
            for a, b in zip(h1[i], h0[i]):
                np.testing.assert_allclose(a[:k - 1], b[:k - 1], rtol=1e-9)


def test_tz_follows_material_kind():
    """The automatic z march: 32 planes for the FP32 32 x 6 block on a 256^3
    cell, 16 for the 16 x 14 block (tz 0 re-makes the choice after a change
    of block shape) and for the power-law tangent (re-chosen when the
    material kind changes); a tz set explicitly stays."""
    pkg = _pkg()
    n = 256
    shape = (n, n, n)
    c = pkg.Cell(shape, precision=pkg.MIXED)
    t = c.tunables()
    say(f"256^3 mixed cell tunables {t}")
    assert t["tiles3d"] == 2 and t["tz"] == 32
    c.set_tunables(tiles3d=1)
    assert c.tunables()["tz"] == 32  # a shape change alone keeps tz
    c.set_tunables(tz=0)
    assert c.tunables()["tz"] == 16
    c.set_tunables(tiles3d=0, tz=0)
    assert c.tunables()["tz"] == 32
    phase = np.ones(shape)
    phase[:, :, : n // 4] = 0.0
    c.set_material_powerlaw(phase)
    assert c.tunables()["tiles3d"] == 1 and c.tunables()["tz"] == 16
    c.set_material(ji.grf_field((32, 32, 32), 10.0, seed=1, ell=0.2).repeat(8, 0).repeat(8, 1)
                   .repeat(8, 2), nu=0.3)
    assert c.tunables()["tiles3d"] == 2 and c.tunables()["tz"] == 32
    c.set_tunables(tz=24)
    c.set_material_powerlaw(phase)
    assert c.tunables()["tz"] == 24
    c.set_tunables(tz=0)
    assert c.tunables()["tz"] == 16
    c.close()
