"""GPU tests of continuous batching over the slots of a group
(jfft_slot_admit / jfft_slots_step / jfft_slot_harvest): solves admitted at
different times, between chunks of PCG iterations, into slots that others
have just left, give bitwise the results of the same cell solved alone, and
the group refuses whole-group calls while slots are in use."""
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


def _solo(pkg, shape, prec, E, macro, tun, tol, maxit):
    c = pkg.Cell(shape, precision=prec)
    c.set_tunables(tz=tun["tz"], tiles2d=tun["tiles2d"], tiles3d=tun["tiles3d"], xrows=tun["xrows"],
                   fused_control=tun["fused_control"])
    c.set_material(E, nu=0.3)
    u, sbar, rep, sig = c.solve(macro, tol=tol, maxit=maxit, want_sigma=True)
    out = (u.cpu().numpy(), sbar, rep, sig.cpu().numpy())
    c.close()
    return out


@pytest.mark.parametrize("shape,prec,graph,run", [((40, 48), "FP64", 8, False),
                                                  ((40, 48), "MIXED", 8, False),
                                                  ((16, 18, 20), "FP64", 0, False),
                                                  ((16, 18, 20), "MIXED", 16, False),
                                                  ((40, 48), "MIXED", 4, True),
                                                  ((16, 18, 20), "FP64", 0, True)])
def test_slots_match_solo_solves(shape, prec, graph, run):
    """Seven cells through a group of three slots: two admitted at once, one
    a chunk later, the rest as slots free up; each harvested result (u,
    sigma field, sigma_bar, iteration count) equals the solo solve bitwise.
    run: the library loops the chunks until a slot finishes (jfft_slots_run)
    instead of one call per chunk."""
    import torch

    pkg = _pkg()
    P = getattr(pkg, prec)
    dim = len(shape)
    ds = dim * (dim + 1) // 2
    ncell, B, tol, maxit = 7, 3, 1e-9, 5000
    Es = [ji.grf_field(shape, 10.0 ** (2 + k % 3), seed=40 + k, ell=0.15) for k in range(ncell)]
    macros = np.random.default_rng(7).uniform(-1, 1, (ncell, ds))
    grp = pkg.Cell(shape, precision=P, batch=B, stream=torch.cuda.Stream())
    if graph:
        grp.set_graph_iterations(graph)
    tun = grp.tunables()
    say(f"slots {shape} {prec} graph {graph} run {run}: {ncell} cells through {B} slots, "
        f"tunables {tun}")
    pending = list(range(ncell))
    owner = [None] * B
    results = {}
    grp.slot_admit(0, Es[0], 0.3, macros[0], tol=tol, maxit=maxit)
    grp.slot_admit(2, Es[1], 0.3, macros[1], tol=tol, maxit=maxit)
    owner[0], owner[2] = 0, 1
    pending = pending[2:]
    steps = 0
    while len(results) < ncell:
        states = grp.slots_run(5.0) if run else grp.slots_step(8)
        steps += 1
        assert steps < 2000
        for s in range(B):
            if states[s] == grp.SLOT_FINISHED:
                u, sbar, rep, sig = grp.slot_harvest(s, want_u=True, want_sigma=True)
                results[owner[s]] = (u.cpu().numpy(), sbar, rep, sig.cpu().numpy(), steps)
                owner[s] = None
        # admit into free slots (slot 1 stays empty for the first chunk)
        for s in range(B):
            if owner[s] is None and pending and (s != 1 or steps >= 1):
                k = pending.pop(0)
                grp.slot_admit(s, Es[k], 0.3, macros[k], tol=tol, maxit=maxit)
                owner[s] = k
    assert (grp.slots_step(2) == grp.SLOT_FREE).all()
    grp.close()
    for k in range(ncell):
        u, sbar, rep, sig, at = results[k]
        us, ss, rs, sgs = _solo(pkg, shape, P, Es[k], macros[k], tun, tol, maxit)
        say(f"  cell {k}: harvested after chunk {at}, iters {rep.iters} (solo {rs.iters}), "
            f"sweeps {rep.outer}, true res {rep.rel_res_true:.1e}")
        assert rep.status == "ok" and rs.status == "ok"
        assert rep.iters == rs.iters and rep.outer == rs.outer
        assert rep.rel_res_true == rs.rel_res_true
        assert np.array_equal(u, us)
        assert np.array_equal(sig, sgs)
        assert np.array_equal(sbar, ss)


def test_slot_states_and_errors():
    import torch

    pkg = _pkg()
    shape = (32, 32)
    grp = pkg.Cell(shape, precision=pkg.MIXED, batch=2, stream=torch.cuda.Stream())
    grp.set_graph_iterations(8)
    E = ji.grf_field(shape, 1e3, seed=1, ell=0.15)
    assert (grp.slots_step(1) == grp.SLOT_FREE).all()  # nothing admitted: no work
    grp.slot_admit(1, E, 0.3, [1.0, 0.0, 0.0], tol=1e-8)
    with pytest.raises(pkg.JfftError):
        grp.slot_admit(1, E, 0.3, [1.0, 0.0, 0.0])      # busy slot
    with pytest.raises(pkg.JfftError):
        grp.slot_admit(2, E, 0.3, [1.0, 0.0, 0.0])      # out of range
    with pytest.raises(pkg.JfftError):
        grp.slot_admit(0, E, 0.25, [1.0, 0.0, 0.0])     # other Lame constants while one runs
    with pytest.raises(pkg.JfftError):
        grp.slot_harvest(1)                              # still running
    grp.slot_admit(0, -E, 0.3, [1.0, 0.0, 0.0])          # negative moduli: checked on the device
    st = grp.slots_step(2)
    assert st[0] == grp.SLOT_FINISHED
    with pytest.raises(pkg.JfftError, match="negative or non-finite"):
        grp.slot_harvest(0)
    assert grp.slots_step(2)[0] == grp.SLOT_FREE
    with pytest.raises(pkg.JfftError):
        grp.solve_batch(np.zeros((2, 3)))                # whole-group call while busy
    with pytest.raises(pkg.JfftError):
        grp.set_material(np.stack([E, E]), nu=0.3)
    with pytest.raises(pkg.JfftError):
        grp.set_tunables(xrows=4)                        # would regroup a running slot's sums
    with pytest.raises(pkg.JfftError):
        grp.set_stop_rule(absolute=True)
    grp.set_graph_iterations(4)                          # changes no result: allowed
    # a homogeneous cell stops at once
    grp.slot_admit(0, np.ones(shape), 0.3, [0.0, 1.0, 0.0], tol=1e-8)
    for _ in range(500):
        st = grp.slots_step(8)
        if (st == grp.SLOT_FINISHED).all():
            break
    assert (st == grp.SLOT_FINISHED).all()
    u0, s0, r0, _ = grp.slot_harvest(0)
    assert r0.status == "ok" and r0.iters == 0 and np.abs(u0.cpu().numpy()).max() == 0.0
    u1, s1, r1, _ = grp.slot_harvest(1)
    assert r1.status == "ok" and r1.rel_res_true <= 1e-8
    # free again: whole-group solves work, and give the slot's result for that cell
    grp.set_material(np.stack([np.ones(shape), E]), nu=0.3)
    u, sbar, reps, _ = grp.solve_batch(np.array([[0.0, 1.0, 0.0], [1.0, 0.0, 0.0]]), tol=1e-8)
    assert np.array_equal(u[1].cpu().numpy(), u1.cpu().numpy())
    assert np.array_equal(sbar[1], s1) and reps[1].iters == r1.iters
    grp.close()


@pytest.mark.parametrize("shape,prec,pc,element,absolute", [
    ((36, 40), "FP64", "PC_GREEN", "tri", True),
    ((36, 40), "MIXED", "PC_JACOBI", "quad", False),
    ((12, 16, 18), "MIXED", "PC_GREEN", "quad", True)])
def test_slots_options_match_solo(shape, prec, pc, element, absolute):
    """The group's options apply to its slots as to a solo cell: other
    preconditioners (Green alone, Jacobi alone), the triangle element and
    the paper's absolute stopping rule; four cells through two slots, each
    bitwise equal to the solo solve with the same options."""
    import torch

    pkg = _pkg()
    P, PC = getattr(pkg, prec), getattr(pkg, pc)
    dim = len(shape)
    ds = dim * (dim + 1) // 2
    Es = [ji.grf_field(shape, 10.0 ** (1 + k % 2), seed=70 + k, ell=0.2) for k in range(4)]
    macros = np.random.default_rng(11).uniform(-1, 1, (4, ds))
    tol = 1e-10 if absolute else 1e-9

    def configure(c):
        c.set_stop_rule(absolute=absolute)

    grp = pkg.Cell(shape, precision=P, pc=PC, batch=2, stream=torch.cuda.Stream(),
                   element=element)
    grp.set_graph_iterations(8)
    configure(grp)
    tun = grp.tunables()
    owner, pending, results, steps = [None, None], list(range(4)), {}, 0
    while len(results) < 4:
        for s in range(2):
            if owner[s] is None and pending:
                k = pending.pop(0)
                grp.slot_admit(s, Es[k], 0.3, macros[k], tol=tol, maxit=20000)
                owner[s] = k
        st = grp.slots_run(5.0)
        steps += 1
        assert steps < 5000
        for s in range(2):
            if st[s] == grp.SLOT_FINISHED:
                u, sbar, rep, _ = grp.slot_harvest(s)
                results[owner[s]] = (u.cpu().numpy(), sbar, rep)
                owner[s] = None
    grp.close()
    for k in range(4):
        c = pkg.Cell(shape, precision=P, pc=PC, element=element)
        configure(c)
        c.set_tunables(tz=tun["tz"], tiles2d=tun["tiles2d"], tiles3d=tun["tiles3d"], xrows=tun["xrows"],
                       fused_control=tun["fused_control"])
        c.set_material(Es[k], nu=0.3)
        us, ss, rs, _ = c.solve(macros[k], tol=tol, maxit=20000)
        us = us.cpu().numpy()
        c.close()
        u, sbar, rep = results[k]
        say(f"{shape} {prec} {pc} {element} abs={absolute} cell {k}: iters {rep.iters} "
            f"(solo {rs.iters}) status {rep.status}")
        assert rep.status == rs.status == "ok"
        assert rep.iters == rs.iters
        assert np.array_equal(u, us) and np.array_equal(sbar, ss)
