"""GPU tests of the launch-parameter autotuner: valid, cached, and neutral
for results (a tuned group equals single cells run with the same tz)."""
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
        assert 2 <= p["tz"] <= shape[0]
    assert (tmp_path / "tunables.json").exists()
    assert tune.autotune(shape, batch=batch, precision=pkg.MIXED) == p  # from the cache
    # another group size reuses the shape's tz
    p2 = tune.autotune(shape, batch=batch + 1, precision=pkg.MIXED, iters=12)
    assert p2["tz"] == p["tz"]
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
        c.set_tunables(tz=p["tz"])
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
    c.set_tunables(tz=8, ygrid=300)
    assert c.tunables() == {"tz": 8, "ygrid": 300}
    c.close()
