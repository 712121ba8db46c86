"""Many cells of uneven sizes: one group per grid shape, groups run side by
side on their own HIP streams.

Each group is one `Cell(batch=B)` handle, so one kernel launch serves all of
its cells; groups of different shapes overlap on the device because every
group has its own stream and its own host thread (the C calls release the
Python GIL while they wait).  Only marshalling happens here: every step of a
solve runs in the library's kernels.
"""
from __future__ import annotations

import threading
from collections import OrderedDict

import numpy as np

from . import FP64, PC_GREEN_JACOBI, Cell, _torch


def solve_cells(fields, macros, nu=0.3, tol=1e-8, maxit=20000, precision=FP64,
                pc=PC_GREEN_JACOBI, graph_iterations=0, want_u=True, autotune=False):
    """Solve cell i with material fields[i] (numpy or torch, any shape per cell)
    and macro strain macros[i].  With autotune, each group takes the launch
    parameters tune.autotune() measures (cached) for its shape and size.

    Returns a list of dicts {u (device tensor or None), sigma_bar, report} in
    input order, and the wall time of the solves (material set-up excluded).
    """
    import time

    torch = _torch()
    buckets = OrderedDict()
    for i, E in enumerate(fields):
        buckets.setdefault(tuple(E.shape), []).append(i)
    groups = []
    for shape, idx in buckets.items():
        stream = torch.cuda.Stream()
        grp = Cell(shape, precision=precision, pc=pc, stream=stream, batch=len(idx))
        if autotune:
            from . import tune

            tune.apply(grp, tune.autotune(shape, batch=len(idx), precision=precision, pc=pc))
        elif graph_iterations:
            grp.set_graph_iterations(graph_iterations)
        Es = torch.stack([torch.as_tensor(np.asarray(fields[i]), dtype=torch.float64)
                          for i in idx]).to(grp.device)
        grp.set_material(Es, nu=nu)
        mac = np.stack([np.asarray(macros[i], dtype=np.float64) for i in idx])
        groups.append((grp, idx, mac))
    torch.cuda.synchronize()
    out = [None] * len(fields)
    errors = []

    def run(grp, idx, mac):
        try:
            u, sbar, reps, _ = grp.solve_batch(mac, tol=tol, maxit=maxit)
            for k, i in enumerate(idx):
                out[i] = {"u": u[k] if want_u else None, "sigma_bar": sbar[k], "report": reps[k]}
        except Exception as e:  # re-raised in the caller's thread
            errors.append(e)

    t0 = time.perf_counter()
    threads = [threading.Thread(target=run, args=g) for g in groups]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for grp, _, _ in groups:
        grp.close()
    if errors:
        raise errors[0]
    return out, wall
