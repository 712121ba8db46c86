"""GPU tests of the serving loop: continuous batching of homogenisation
requests (six load cases each) with memory-footprint admission.  Every
request's C_eff must be bitwise the C_eff of the same cell solved alone,
whether it was merged with other requests, ran beside them on other streams,
or waited for memory."""
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


def _requests(count, seed, sides):
    from paper_2508_02613_amd.serve import Request

    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        n = int(rng.choice(sides))
        c = float(10 ** rng.uniform(2, 4))
        out.append(Request(i, ji.grf_field((n, n, n), c, seed=1000 * seed + i, ell=0.1)))
    return out


@pytest.mark.parametrize("precision,budget_handles", [(0, 100), (1, 100), (1, 1.5)])
def test_served_results_equal_alone(precision, budget_handles):
    pkg = _pkg()
    from paper_2508_02613_amd.serve import Server, workspace_bytes

    reqs = _requests(10, 3, (32, 48))
    one = workspace_bytes((48, 48, 48), precision, pkg.PC_GREEN_JACOBI, 6)
    budget = int(budget_handles * one)
    say(f"serve 10 requests (32/48), precision={precision}, budget {budget / 2**20:.0f} MiB")
    srv = Server(workers=3, budget_bytes=budget, precision=precision, max_merge=3,
                 graph_iterations=8)
    stats = srv.run(reqs, rate=None)
    srv.close()
    say(f"  {stats}")
    assert stats["all_ok"] and 0 < stats["max_rel_res_true"] <= 1.5e-8
    assert all(r.rel_res_true > 0 for r in reqs)
    if budget_handles < 2:
        assert stats["handles_evicted"] > 0 or stats["handles_created"] <= 2
    for r in reqs:
        Ca, reps = pkg.effective_stiffness(r.E, nu=0.3, tol=1e-8, precision=precision)
        assert [x.iters for x in reps] == r.iters, (r.rid, r.iters)
        assert np.array_equal(Ca, r.C), f"request {r.rid}: C_eff differs alone vs served"
        assert r.latency > 0 and r.done >= r.start >= r.arrival - 1e-9


def test_poisson_arrivals_complete_in_order_of_capacity():
    pkg = _pkg()
    from paper_2508_02613_amd.serve import Server

    reqs = _requests(12, 4, (32, 48, 64))
    srv = Server(workers=4, budget_bytes=8 << 30, precision=pkg.MIXED, graph_iterations=8)
    stats = srv.run(reqs, rate=40.0, seed=1)
    srv.close()
    say(f"  Poisson 40/s: {stats}")
    assert stats["all_ok"]
    assert stats["p99_latency_ms"] >= stats["p50_latency_ms"] > 0
    arr = sorted(r.arrival for r in reqs)
    assert arr[-1] > 0.05  # arrivals are spread in time


@pytest.mark.parametrize("precision,budget_groups", [(0, 100), (1, 100), (1, 1.2)])
def test_slot_server_results_equal_alone(precision, budget_groups):
    """Continuous batching below handle granularity (SlotServer): requests of
    two shapes stream through groups of 2 x 6 slots at Poisson arrivals, so
    load cases of different requests enter and leave one group between
    chunks; each C_eff equals the cell solved alone, bitwise.  With a budget
    of about one group the two shapes take turns (eviction)."""
    pkg = _pkg()
    from paper_2508_02613_amd.serve import SlotServer, workspace_bytes

    reqs = _requests(9, 5, (32, 48))
    one = workspace_bytes((48, 48, 48), precision, pkg.PC_GREEN_JACOBI, 12)
    budget = int(budget_groups * one)
    say(f"slot server: 9 requests (32/48), precision={precision}, budget {budget / 2**20:.0f} MiB")
    srv = SlotServer(budget_bytes=budget, precision=precision, slots_per_group=2,
                     graph_iterations=8)
    stats = srv.run(reqs, rate=60.0, seed=2)
    srv.close()
    say(f"  {stats}")
    assert stats["all_ok"] and 0 < stats["max_rel_res_true"] <= 1.5e-8
    assert stats["driver_wakeups"] > 0 and stats["mean_busy_slots_per_wakeup"] > 0
    for r in reqs:
        Ca, reps = pkg.effective_stiffness(r.E, nu=0.3, tol=1e-8, precision=precision)
        assert [x.iters for x in reps] == r.iters, (r.rid, r.iters)
        assert np.array_equal(Ca, r.C), f"request {r.rid}: C_eff differs alone vs slot-served"
        assert r.latency > 0 and r.done >= r.start >= r.arrival - 1e-9
