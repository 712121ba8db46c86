"""Host logic of the serving loops, without a GPU: the scheduling of
SlotServer and Server and the memory admission of HandlePool, driven
through stand-in group handles that mimic the library's slot and group
calls (each solve "converges" after a number of iterations fixed by its
request and load case, and its sigma_bar encodes which request and load
case it belongs to).  What is checked: every request completes with its
six load cases in the right columns, slots are reused, a group never holds
more than its slots, memory admission evicts idle handles and makes
workers wait instead of exceeding the budget, and the timestamps are
ordered."""
import contextlib
import threading

import numpy as np
import pytest

import paper_2508_02613_amd.serve as serve


class FakeTorch:
    """torch on the CPU, with the stream calls the servers make as no-ops."""

    class cuda:
        @staticmethod
        def stream(s):
            return contextlib.nullcontext()

        class Stream:
            pass

    def __getattr__(self, name):
        import torch
        return getattr(torch, name)


FAKE_TORCH = FakeTorch()


def _first(E):
    return int(float(E.reshape(-1)[0]))


class FakeGroup:
    SLOT_FREE, SLOT_RUNNING, SLOT_FINISHED = 0, 1, 2
    live = 0
    lock = threading.Lock()

    def __init__(self, shape, precision=None, pc=None, stream=None, batch=1):
        self.shape, self.batch, self.stream, self.device = shape, batch, stream, "cpu"
        self.state = [0] * batch
        self.left = [0] * batch
        self.tag = [None] * batch
        self.its = [0] * batch
        with FakeGroup.lock:
            FakeGroup.live += 1

    def close(self):
        with FakeGroup.lock:
            FakeGroup.live -= 1

    def set_graph_iterations(self, k):
        pass

    # slot calls
    def slot_admit(self, slot, E, nu, macro, tol=1e-8, maxit=1000):
        assert self.state[slot] == self.SLOT_FREE
        g = int(np.argmax(macro))
        rid = _first(E)
        self.state[slot] = self.SLOT_RUNNING
        self.left[slot] = 5 + (rid * 7) % 23 + g
        self.tag[slot] = (rid, g)
        self.its[slot] = 0

    def slots_step(self, iterations=8):
        for s in range(self.batch):
            if self.state[s] == self.SLOT_RUNNING:
                k = min(iterations, self.left[s])
                self.left[s] -= k
                self.its[s] += k
                if self.left[s] == 0:
                    self.state[s] = self.SLOT_FINISHED
        return np.array(self.state)

    def slots_run(self, max_ms=2.0):
        for _ in range(8):  # a few chunks, or until a slot finishes
            st = self.slots_step(4)
            if (st == self.SLOT_FINISHED).any() or not (st == self.SLOT_RUNNING).any():
                break
        return np.array(self.state)

    def slot_harvest(self, slot, want_u=True, want_sigma=False):
        assert self.state[slot] == self.SLOT_FINISHED
        rid, g = self.tag[slot]
        self.state[slot] = self.SLOT_FREE
        rep = serve_report(self.its[slot])
        return None, np.full(6, 1000.0 * rid + g), rep, None

    # whole-group calls (Server)
    def set_material(self, Es, nu=0.3):
        self.Es = Es

    def solve_batch(self, macros, tol=1e-8, maxit=1000):
        k = len(macros) // 6
        sbar = np.zeros((len(macros), 6))
        reps = []
        for j in range(len(macros)):
            rid = _first(self.Es[j])
            g = j % 6
            sbar[j] = 1000.0 * rid + g
            reps.append(serve_report(5 + (rid * 7) % 23 + g))
        return None, sbar, reps, None


def serve_report(iters):
    class R:
        pass
    r = R()
    r.iters, r.status, r.rel_res_true = iters, "ok", 1e-9
    return r


@pytest.fixture
def fake(monkeypatch):
    monkeypatch.setattr(serve, "_torch", lambda: FAKE_TORCH)
    monkeypatch.setattr(serve, "Cell", FakeGroup)
    monkeypatch.setattr(serve, "workspace_bytes",
                        lambda shape, precision, pc, batch: int(np.prod(shape)) * batch)
    FakeGroup.live = 0
    yield


def _requests(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        side = int(rng.choice((4, 6, 8)))
        out.append(serve.Request(i, np.full((side, side, side), float(i))))
    return out


def _check(reqs):
    for r in reqs:
        assert r.status == "ok"
        want = 1000.0 * r.rid + np.arange(6)
        assert np.array_equal(r.C[0], want), (r.rid, r.C[0])  # column g from load case g
        assert r.done >= r.start >= r.arrival - 1e-9


@pytest.mark.parametrize("rate", [None, 400.0])
def test_slot_server_schedules_every_request(fake, rate):
    reqs = _requests(40, 1)
    srv = serve.SlotServer(budget_bytes=1 << 30, slots_per_group=2, graph_iterations=4)
    st = srv.run(reqs, rate=rate, seed=2)
    srv.close()
    _check(reqs)
    for r in reqs:
        assert r.iters == [5 + (r.rid * 7) % 23 + g for g in range(6)]
    assert st["requests"] == 40 and st["all_ok"]
    assert 0 < st["mean_busy_slots_per_wakeup"] <= 12
    assert st["handles_created"] == 3          # one group per shape, reused
    assert FakeGroup.live == 0


def test_slot_server_waits_for_memory(fake):
    """Budget for one group of the largest shape: the shapes take turns
    (evictions), and the bytes of the groups alive at once never exceed the
    budget."""
    reqs = _requests(24, 3)
    budget = 8 ** 3 * 12  # one group of the largest shape (2 requests x 6 slots)
    live, peak = [0], [0]
    lock = threading.Lock()
    orig_init, orig_close = FakeGroup.__init__, FakeGroup.close

    def init(self, shape, **k):
        orig_init(self, shape, **k)
        with lock:
            live[0] += int(np.prod(shape)) * self.batch
            peak[0] = max(peak[0], live[0])

    def close(self):
        orig_close(self)
        with lock:
            live[0] -= int(np.prod(self.shape)) * self.batch
    FakeGroup.__init__, FakeGroup.close = init, close
    try:
        srv = serve.SlotServer(budget_bytes=budget, slots_per_group=2, graph_iterations=4)
        st = srv.run(reqs, rate=None)
        srv.close()
    finally:
        FakeGroup.__init__, FakeGroup.close = orig_init, orig_close
    _check(reqs)
    assert 0 < peak[0] <= budget
    assert st["handles_evicted"] >= 1


def test_handle_server_merges_and_completes(fake):
    reqs = _requests(30, 4)
    srv = serve.Server(workers=3, budget_bytes=1 << 30, max_merge=3, graph_iterations=0)
    st = srv.run(reqs, rate=None)
    srv.close()
    _check(reqs)
    assert st["all_ok"] and st["mean_merged"] >= 1.0


def test_handle_pool_refuses_a_handle_above_the_budget(fake):
    pool = serve.HandlePool(100, 1, 3, 0, 0.3)
    with pytest.raises(MemoryError):
        pool.acquire(((8, 8, 8), 1))
