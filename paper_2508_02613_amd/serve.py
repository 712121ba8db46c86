"""Serving homogenisation requests on one GPU with continuous batching.

A request is one periodic 3D cell (material field E, Poisson ratio shared by
the server) and asks for its homogenised 6 x 6 Mandel stiffness C_eff, i.e.
six solves, one per unit macro strain (Sec. 5).  The server

* keeps a pool of warm group handles per (grid shape, requests merged):
  workspace, Fourier tables and the captured PCG graph stay on the device
  and are reused by later requests of the same shape;
* admits work by device-memory footprint: a handle is created only when the
  bytes the library reports for it (jfft_workspace_bytes, queried before any
  allocation) fit the budget next to the handles already allocated; idle
  handles of other shapes are evicted to make room; a worker waits otherwise;
* runs `workers` host threads, each driving its own handles (each handle has
  its own HIP stream), so requests that arrive while others are on the GPU
  start as soon as a worker and memory are free and their kernels overlap
  with the running ones;
* merges requests of one grid shape that are already waiting into one group
  launch (up to `max_merge` requests, 6 cells each);
* optionally (autotune) gives each new handle the launch parameters that
  tune.autotune() measured for its shape and size (tile shapes per shape only, so
  merging never changes a request's results).

Each cell's results are bitwise independent of what else is in its group or
on the device (reduction layouts depend on the cell shape only), so a request
gets the same C_eff alone and in the mix.  Only marshalling and scheduling
happen here: every step of a solve runs in the library's kernels.

SlotServer batches below handle granularity: one group handle per grid
shape whose cells are slots (jfft_slot_admit / jfft_slots_run /
jfft_slot_harvest).  A driver thread per active shape admits arrived
requests of its shape into free slots (six per request) between chunks of
PCG iterations, lets the library run chunks for every running slot until
one finishes (or a polling interval passes), and harvests the load cases
that stopped; a request is done when its six slots are.  A request
thus joins the running group at the next chunk boundary instead of waiting
for the group to drain, and leaves as soon as its own solves stop.
"""
from __future__ import annotations

import ctypes as C
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import MIXED, PC_GREEN_JACOBI, Cell, _check, _torch, load_library


@dataclass
class Request:
    rid: int
    E: np.ndarray                 # material field (nz, ny, nx), float64
    arrival: float = 0.0          # seconds after the start of the run
    C: np.ndarray | None = None   # result: homogenised Mandel stiffness
    iters: list = field(default_factory=list)
    rel_res_true: float = 0.0
    status: str = ""
    start: float = 0.0
    done: float = 0.0
    merged: int = 1               # requests in the group launch that served it

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def workspace_bytes(shape, precision, pc, batch) -> int:
    """Device bytes a group handle of `batch` cells needs (allocates nothing
    on the device)."""
    lib = load_library()
    dim = len(shape)
    n = (C.c_int * 3)(*(list(shape[::-1]) + [1] * (3 - dim)))
    h = C.c_void_p()
    _check(lib.jfft_create_batch(dim, n, None, int(precision), int(pc), int(batch), None,
                                 C.byref(h)))
    nb = C.c_size_t(0)
    try:
        _check(lib.jfft_workspace_bytes(h, C.byref(nb)))
    finally:
        lib.jfft_destroy_cell(h)
    return int(nb.value) + 256  # the binding aligns the workspace to 256 bytes


class HandlePool:
    """Warm group handles under a device-memory budget."""

    def __init__(self, budget_bytes, precision, pc, graph_iterations, nu, autotune=False):
        self.budget = int(budget_bytes)
        self.autotune = autotune
        self.precision, self.pc, self.graph_iterations, self.nu = precision, pc, graph_iterations, nu
        self.cv = threading.Condition()
        self.free = {}       # key -> [Cell]
        self.used = 0        # bytes of all allocated handles
        self.bytes = {}      # key -> bytes per handle
        self.created = 0
        self.evicted = 0

    def need(self, key):
        if key not in self.bytes:
            shape, k = key
            self.bytes[key] = workspace_bytes(shape, self.precision, self.pc, 6 * k)
        return self.bytes[key]

    def acquire(self, key):
        torch = _torch()
        with self.cv:
            need = self.need(key)
            if need > self.budget:
                raise MemoryError(f"one handle for {key} needs {need} B, above the budget")
            while True:
                lst = self.free.get(key)
                if lst:
                    return lst.pop()
                if self.used + need <= self.budget:
                    self.used += need
                    break
                victim = next(((k2, l2) for k2, l2 in self.free.items() if l2), None)
                if victim is not None:
                    k2, l2 = victim
                    l2.pop().close()
                    self.used -= self.bytes[k2]
                    self.evicted += 1
                    continue
                self.cv.wait()
        # allocate outside the lock; the bytes are already reserved
        shape, k = key
        cell = Cell(shape, precision=self.precision, pc=self.pc, stream=torch.cuda.Stream(),
                    batch=6 * k)
        if self.autotune:
            from . import tune

            tune.apply(cell, tune.autotune(shape, batch=6 * k, precision=self.precision,
                                           pc=self.pc))
        elif self.graph_iterations:
            cell.set_graph_iterations(self.graph_iterations)
        cell.key = key
        with self.cv:
            self.created += 1
        return cell

    def release(self, cell):
        with self.cv:
            self.free.setdefault(cell.key, []).append(cell)
            self.cv.notify_all()

    def close(self):
        with self.cv:
            for lst in self.free.values():
                for c in lst:
                    c.close()
            self.free.clear()
            self.used = 0


class Server:
    def __init__(self, workers=4, budget_bytes=64 << 30, precision=MIXED, pc=PC_GREEN_JACOBI,
                 tol=1e-8, maxit=20000, graph_iterations=8, nu=0.3, max_merge=4,
                 merge_max_side=64, autotune=False):
        self.workers = workers
        self.tol, self.maxit, self.nu = tol, maxit, nu
        self.max_merge, self.merge_max_side = max_merge, merge_max_side
        self.pool = HandlePool(budget_bytes, precision, pc, graph_iterations, nu, autotune)
        self.precision = precision

    def _solve(self, cell, reqs):
        """One group launch for `reqs` (same shape): 6 load cases each."""
        torch = _torch()
        k = len(reqs)
        shape = reqs[0].E.shape
        with torch.cuda.stream(cell.stream):
            Es = torch.empty((6 * k,) + shape, dtype=torch.float64, device=cell.device)
            for j, r in enumerate(reqs):
                Es[6 * j:6 * j + 6] = torch.from_numpy(r.E).to(cell.device, non_blocking=False)
        cell.set_material(Es, nu=self.nu)
        _, sbar, reps, _ = cell.solve_batch(np.tile(np.eye(6), (k, 1)), tol=self.tol,
                                            maxit=self.maxit)
        for j, r in enumerate(reqs):
            r.C = np.ascontiguousarray(sbar[6 * j:6 * j + 6].T)
            rr = reps[6 * j:6 * j + 6]
            r.iters = [x.iters for x in rr]
            r.rel_res_true = max(x.rel_res_true for x in rr)
            r.status = "ok" if all(x.status == "ok" for x in rr) else \
                ",".join(sorted({x.status for x in rr}))
            r.merged = k

    def run(self, requests, rate=None, seed=0):
        """Serve `requests`.  rate: Poisson arrival rate in requests/s (None:
        all arrive at t = 0, which measures the saturated capacity).  Returns
        a summary dict; the requests carry their results and timestamps."""
        rng = np.random.default_rng(seed)
        t = 0.0
        for r in requests:
            if rate:
                t += rng.exponential(1.0 / rate)
            r.arrival = t
        pending = sorted(requests, key=lambda r: r.arrival)
        lock = threading.Lock()
        errors = []
        t0 = time.perf_counter()

        def take():
            """Earliest request that has arrived (waits for it), plus waiting
            requests of the same shape to merge."""
            while True:
                with lock:
                    if not pending:
                        return None
                    now = time.perf_counter() - t0
                    head = pending[0]
                    if head.arrival <= now:
                        batch = [pending.pop(0)]
                        side = max(head.E.shape)
                        if side <= self.merge_max_side:
                            # merge only as many as one handle can hold in the budget
                            kmax = 1
                            while (kmax < self.max_merge and self.pool.need(
                                    (head.E.shape, kmax + 1)) <= self.pool.budget):
                                kmax += 1
                            i = 0
                            while i < len(pending) and len(batch) < kmax:
                                r = pending[i]
                                if r.arrival > now:
                                    break
                                if r.E.shape == head.E.shape:
                                    batch.append(pending.pop(i))
                                else:
                                    i += 1
                        return batch
                    wait = head.arrival - now
                time.sleep(min(wait, 0.002))

        def worker():
            try:
                while True:
                    batch = take()
                    if batch is None:
                        return
                    start = time.perf_counter() - t0
                    cell = self.pool.acquire((batch[0].E.shape, len(batch)))
                    try:
                        self._solve(cell, batch)
                    finally:
                        self.pool.release(cell)
                    done = time.perf_counter() - t0
                    for r in batch:
                        r.start, r.done = start, done
            except Exception as e:  # reported by run()
                errors.append(e)

        threads = [threading.Thread(target=worker) for _ in range(self.workers)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        makespan = time.perf_counter() - t0
        if errors:
            raise errors[0]
        lat = np.array([r.latency for r in requests])
        return {
            "requests": len(requests),
            "makespan_s": makespan,
            "requests_per_s": len(requests) / makespan,
            "solves_per_s": 6 * len(requests) / makespan,
            "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
            "p95_latency_ms": float(np.percentile(lat, 95) * 1e3),
            "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_latency_ms": float(lat.mean() * 1e3),
            "offered_rate": rate,
            "mean_merged": float(np.mean([r.merged for r in requests])),
            "handles_created": self.pool.created,
            "handles_evicted": self.pool.evicted,
            "all_ok": all(r.status == "ok" for r in requests),
            "max_rel_res_true": float(max(r.rel_res_true for r in requests)),
        }

    def close(self):
        self.pool.close()


class SlotServer:
    """Continuous batching over the slots of one group handle per grid shape.

    slots_per_group: requests a group holds at once (6 slots each), or a
    function of the grid shape that returns it; the group's device bytes
    count against budget_bytes like any handle, and a shape waits for memory
    like a worker does in Server.  A driver runs its group's iterations in
    the library (jfft_slots_run, chunks of the captured graph depth) until a
    load case finishes or poll_ms have passed, so it wakes only to harvest or
    to admit arrivals."""

    def __init__(self, budget_bytes=64 << 30, precision=MIXED, pc=PC_GREEN_JACOBI, tol=1e-8,
                 maxit=20000, graph_iterations=8, nu=0.3, slots_per_group=4, poll_ms=2.0,
                 autotune=False):
        self.tol, self.maxit, self.nu = tol, maxit, nu
        self.slots_per_group = slots_per_group
        self.poll_ms = poll_ms
        self.pool = HandlePool(budget_bytes, precision, pc, graph_iterations, nu, autotune)
        self.precision = precision

    def run(self, requests, rate=None, seed=0):
        """Serve `requests` (rate as in Server.run).  Returns a summary dict."""
        rng = np.random.default_rng(seed)
        t = 0.0
        for r in requests:
            if rate:
                t += rng.exponential(1.0 / rate)
            r.arrival = t
        arrivals = sorted(requests, key=lambda r: r.arrival)
        queues = {}          # shape -> [Request] arrived, not yet admitted
        drivers = {}         # shape -> Thread
        lock = threading.Lock()
        errors = []
        wakes = {"n": 0, "slots": 0}
        t0 = time.perf_counter()
        spg = self.slots_per_group

        def drive(shape):
            torch = _torch()
            k = int(spg(shape)) if callable(spg) else int(spg)
            cell = self.pool.acquire((shape, k))
            owner = [None] * (6 * k)    # slot -> (request, load case)
            left = {}                   # rid -> solves not yet harvested
            eye = np.eye(6)
            try:
                with torch.cuda.stream(cell.stream):
                    while True:
                        with lock:
                            q = queues[shape]
                            free = [s for s in range(6 * k) if owner[s] is None]
                            take = []
                            while q and len(free) >= 6 * (len(take) + 1):
                                take.append(q.pop(0))
                            if not take and all(o is None for o in owner):
                                # back to the pool before a new driver of this
                                # shape can look for a handle
                                self.pool.release(cell)
                                cell = None
                                del drivers[shape]
                                return
                        now = time.perf_counter() - t0
                        for r in take:
                            r.start = now
                            r.C = np.zeros((6, 6))
                            r.iters = [0] * 6
                            r._st = [""] * 6
                            r._res = [0.0] * 6
                            left[r.rid] = 6
                            E = torch.from_numpy(r.E).to(cell.device)
                            for g in range(6):
                                s = free.pop(0)
                                cell.slot_admit(s, E, self.nu, eye[g], tol=self.tol,
                                                maxit=self.maxit)
                                owner[s] = (r, g)
                        states = cell.slots_run(self.poll_ms)
                        with lock:
                            wakes["n"] += 1
                            wakes["slots"] += sum(o is not None for o in owner)
                        for s in np.nonzero(states == cell.SLOT_FINISHED)[0]:
                            r, g = owner[s]
                            _, sbar, rep, _ = cell.slot_harvest(int(s), want_u=False)
                            owner[s] = None
                            r.C[:, g] = sbar
                            r.iters[g] = rep.iters
                            r._st[g] = rep.status
                            r._res[g] = rep.rel_res_true
                            left[r.rid] -= 1
                            if left[r.rid] == 0:
                                r.done = time.perf_counter() - t0
                                r.rel_res_true = max(r._res)
                                r.status = ("ok" if all(x == "ok" for x in r._st)
                                            else ",".join(sorted(set(r._st))))
                                r.merged = 1
            except Exception as e:  # reported by run()
                errors.append(e)
                with lock:
                    drivers.pop(shape, None)
            finally:
                if cell is not None:
                    self.pool.release(cell)

        i = 0
        while i < len(arrivals) or drivers:
            if errors:
                break
            now = time.perf_counter() - t0
            with lock:
                while i < len(arrivals) and arrivals[i].arrival <= now:
                    r = arrivals[i]
                    queues.setdefault(r.E.shape, []).append(r)
                    i += 1
                for shape, q in queues.items():
                    if q and shape not in drivers:
                        th = threading.Thread(target=drive, args=(shape,))
                        drivers[shape] = th
                        th.start()
            time.sleep(0.0005)
        for th in list(drivers.values()):
            th.join()
        makespan = time.perf_counter() - t0
        if errors:
            raise errors[0]
        lat = np.array([r.latency for r in requests])
        return {
            "requests": len(requests),
            "makespan_s": makespan,
            "requests_per_s": len(requests) / makespan,
            "solves_per_s": 6 * len(requests) / makespan,
            "p50_latency_ms": float(np.percentile(lat, 50) * 1e3),
            "p95_latency_ms": float(np.percentile(lat, 95) * 1e3),
            "p99_latency_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_latency_ms": float(lat.mean() * 1e3),
            "offered_rate": rate,
            "driver_wakeups": wakes["n"],
            "mean_busy_slots_per_wakeup": wakes["slots"] / max(1, wakes["n"]),
            "handles_created": self.pool.created,
            "handles_evicted": self.pool.evicted,
            "all_ok": all(r.status == "ok" for r in requests),
            "max_rel_res_true": float(max(r.rel_res_true for r in requests)),
        }

    def close(self):
        self.pool.close()
