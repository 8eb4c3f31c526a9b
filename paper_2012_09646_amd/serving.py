"""Serving: request shapes recorded from workload programs, and runs of an
arrival trace through the native serving loop (dag_serve_*).

Buffer roles are derived from the program: a buffer no call modifies is
SHARED by all requests (e.g. the CSR graph, the pinned spot prices); a
modified buffer with initial contents is INIT (each request starts from a
pristine copy); any other modified buffer is PRIVATE.
"""

import ctypes as C

import numpy as np

from . import dagrt as D
from . import runner


def written_buffers(prog):
    w = set()
    for op in prog.ops:
        if op["kind"] == "kernel":
            w.update(b for b, m in op["args"] if m == "m")
        elif op["kind"] == "copy":
            w.add(op["dst"])
    return w


class ShapeTemplate:
    """One request shape: template buffers, pristine inputs, recorded region."""

    def __init__(self, ctx, prog, key, result=None, result_bytes=None):
        self.prog = prog
        self.key = key
        self.bound = runner.Bound(ctx, prog, read_bytes=0)
        w = written_buffers(prog)
        self.roles = []
        self.pristine = {}
        for name, b in prog.bufs.items():
            h = self.bound.h[name]
            if name not in w:
                self.roles.append((h, D.DAG_ROLE_SHARED, 0))
            elif b.init is not None:
                loc = D.DAG_PINNED_HOST if b.loc == "host" else D.DAG_DEVICE
                p = ctx.alloc(b.nbytes, loc)
                ctx.host_write(p, np.ascontiguousarray(b.init).view(np.uint8).ravel())
                self.pristine[name] = p
                self.roles.append((h, D.DAG_ROLE_INIT, p))
            else:
                self.roles.append((h, D.DAG_ROLE_PRIVATE, 0))
        self.result = result or prog.result or prog.outputs[-1]
        nb = prog.bufs[self.result].nbytes
        self.result_bytes = nb if result_bytes is None else min(nb, result_bytes)
        ctx.sync()
        self.bound.record(key)
        ctx.sync()


class Server:
    def __init__(self, ctx, budget_bytes, device_arena_bytes=None, host_arena_bytes=1 << 30,
                 lanes=8, bypass=32, copy_lanes=1, transfer_lanes=0):
        self.ctx = ctx
        cfg = D.dag_serve_config(int(budget_bytes), int(device_arena_bytes or budget_bytes),
                                 int(host_arena_bytes), lanes, bypass, int(copy_lanes), int(transfer_lanes))
        self.h = D.dag_serve_create(ctx.h, cfg)
        self.shapes = []

    def add(self, tmpl, sim_ns=0):
        sid = D.dag_serve_add_shape(self.ctx.h, self.h, tmpl.key, tmpl.roles, tmpl.bound.h[tmpl.result],
                                    tmpl.result_bytes, sim_ns)
        self.shapes.append(tmpl)
        return sid

    def footprint(self, sid):
        return D.dag_serve_shape_info(self.h, sid)

    def run(self, arrival_ns, shape, mode=D.DAG_SERVE_CONCURRENT, keep_results=False):
        n = len(arrival_ns)
        reqs = (D.dag_request * max(n, 1))()
        results = []
        for i in range(n):
            reqs[i].shape = int(shape[i])
            reqs[i].arrival_ns = int(arrival_ns[i])
            if keep_results:
                t = self.shapes[int(shape[i])]
                arr = np.zeros(t.result_bytes, dtype=np.uint8)
                results.append(arr)
                reqs[i].result = arr.ctypes.data if t.result_bytes else None
        done, stats = D.dag_serve_run(self.ctx.h, self.h, reqs, mode)
        out = {
            "admit_ns": np.array([done[i].admit_ns for i in range(n)], dtype=np.int64),
            "done_ns": np.array([done[i].done_ns for i in range(n)], dtype=np.int64),
            "lane": np.array([done[i].lane for i in range(n)], dtype=np.int32),
        }
        return out, stats, results

    def close(self):
        if self.h:
            D.dag_serve_destroy(self.h)
            self.h = None
