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

    def _result_array(self, sid):
        t = self.shapes[int(sid)]
        return np.zeros(t.result_bytes, dtype=np.uint8)

    def run(self, arrival_ns, shape, mode=D.DAG_SERVE_CONCURRENT, keep_results=False):
        """The whole trace as one session (dag_serve_run)."""
        n = len(arrival_ns)
        reqs = (D.dag_request * max(n, 1))()
        results = []
        for i in range(n):
            reqs[i].shape = int(shape[i])
            reqs[i].arrival_ns = int(arrival_ns[i])
            if keep_results:
                arr = self._result_array(shape[i])
                results.append(arr)
                reqs[i].result = arr.ctypes.data if arr.nbytes else None
        done, stats = D.dag_serve_run(self.ctx.h, self.h, reqs, mode)
        out = {
            "admit_ns": np.array([done[i].admit_ns for i in range(n)], dtype=np.int64),
            "done_ns": np.array([done[i].done_ns for i in range(n)], dtype=np.int64),
            "lane": np.array([done[i].lane for i in range(n)], dtype=np.int32),
        }
        return out, stats, results

    # online session: submissions (any thread) while one thread polls
    def start(self, mode=D.DAG_SERVE_CONCURRENT):
        D.dag_serve_start(self.ctx.h, self.h, mode)

    def submit(self, sid, arrival_ns=D.DAG_SERVE_NOW, result=None):
        return D.dag_serve_submit(self.h, sid, arrival_ns, result)

    def close_session(self):
        D.dag_serve_close(self.h)

    def poll(self, wait_us=0, cap=256):
        return D.dag_serve_poll(self.ctx.h, self.h, wait_us, cap)

    def stats(self):
        return D.dag_serve_stats(self.h)

    def run_online(self, arrival_ns, shape, mode=D.DAG_SERVE_CONCURRENT, keep_results=False, pace=True,
                   delays=None):
        """The same trace submitted by a producer thread while this thread
        polls: with pace, each request is submitted when its arrival time has
        come (arrival = the submission time); without, with its scheduled
        arrival, after sleeping delays[i] seconds (if given).  Returns
        (records (arrival, admit, done, shape, lane) by request index,
        summary, results)."""
        import threading
        import time

        n = len(arrival_ns)
        results = [self._result_array(shape[i]) if keep_results else None for i in range(n)]
        ids = [None] * n
        err = []
        self.start(mode)

        def producer():
            try:
                t0 = time.perf_counter_ns()
                for i in range(n):
                    if pace:
                        while time.perf_counter_ns() - t0 < int(arrival_ns[i]):
                            pass
                        ids[i] = self.submit(shape[i], D.DAG_SERVE_NOW, results[i])
                    else:
                        if delays is not None and delays[i] > 0:
                            time.sleep(float(delays[i]))
                        ids[i] = self.submit(shape[i], int(arrival_ns[i]), results[i])
            except Exception as e:  # reported by the polling thread
                err.append(e)
            finally:
                self.close_session()

        th = threading.Thread(target=producer)
        th.start()
        recs = {}
        try:
            while True:
                got, left = self.poll(wait_us=2000)
                for d in got:
                    recs[d.id] = (d.arrival_ns, d.admit_ns, d.done_ns, d.shape, d.lane)
                if not got and left == 0 and not th.is_alive():
                    got, left = self.poll(wait_us=0)
                    for d in got:
                        recs[d.id] = (d.arrival_ns, d.admit_ns, d.done_ns, d.shape, d.lane)
                    if not got and left == 0:
                        break
        finally:
            th.join()
        if err:
            raise err[0]
        by_index = [recs[ids[i]] for i in range(n)]
        return by_index, self.stats(), results

    def close(self):
        if self.h:
            D.dag_serve_destroy(self.h)
            self.h = None


# ---------------------------------------------------------------------------
# The serving mix of the benchmark: the four workloads at footprint scale 2^k
# ---------------------------------------------------------------------------
MIX_KINDS = ("vec", "bs", "img", "hits")
MIX_BUDGET = 64 << 30
MIX_HOST_ARENA = 8 << 30


def mix_templates(ctx, graphs=None, result_bytes=64, key0=1000, seed=4):
    """One ShapeTemplate per (workload, k), in the order the mix draws them."""
    from . import workloads as W
    tmpls = []
    key = key0
    for kind in MIX_KINDS:
        for k in W.SERVE_KS:
            prog = W.serve_program(kind, k, seed=seed, graphs=graphs)
            tmpls.append(ShapeTemplate(ctx, prog, key=key, result_bytes=result_bytes))
            key += 1
    return tmpls


def mix_server(ctx, tmpls, lanes=3, copy_lanes=1, transfer_lanes=1, bypass=32, budget=MIX_BUDGET,
               host_arena=MIX_HOST_ARENA):
    """The benchmark's server over the mix's shapes (3 lanes, one of them for
    the requests that copy between host and device, one copy stream per
    direction, a 64 GB admission budget)."""
    srv = Server(ctx, budget, host_arena_bytes=host_arena, lanes=lanes, bypass=bypass, copy_lanes=copy_lanes,
                 transfer_lanes=transfer_lanes)
    for t in tmpls:
        srv.add(t)
    return srv
