"""Submit a workload program (see ``workloads``) through the C ABI.

``Bound`` allocates the program's buffers in a context, uploads the initial
contents and turns the operation list into a ``dag_op`` batch once, so a run
is a single native call that the scheduler processes op by op, exactly as
the equivalent sequence of single calls.
"""

import ctypes as C

import numpy as np

from . import dagrt as D


class Bound:
    def __init__(self, ctx, prog, upload=True, read_bytes=None):
        """read_bytes: bytes copied back by each program host read (None =
        the whole buffer; 0 = wait only)."""
        self.ctx = ctx
        self.prog = prog
        self.h = {}
        self.name_of = {}
        for name, b in prog.bufs.items():
            loc = D.DAG_PINNED_HOST if b.loc == "host" else D.DAG_DEVICE
            self.h[name] = ctx.alloc(b.nbytes, loc)
            self.name_of[self.h[name]] = name
        if upload:
            self.upload()
        self.read_bytes = read_bytes
        self._keep = []
        self.read_bufs = {}
        self.ops = self._build_ops()

    def upload(self, names=None):
        for name, b in self.prog.bufs.items():
            if names is not None and name not in names:
                continue
            if b.init is None:
                data = np.zeros(b.nbytes, dtype=np.uint8)
            else:
                data = np.ascontiguousarray(b.init).view(np.uint8).ravel()
            self.ctx.host_write(self.h[name], data)

    def _build_ops(self):
        ops = (D.dag_op * len(self.prog.ops))()
        for i, op in enumerate(self.prog.ops):
            o = ops[i]
            kind = op["kind"]
            if kind == "kernel":
                kid = D.KERNEL_IDS[op["kernel"]]
                prm = D.make_params(op["kernel"], op.get("params", {}))
                args = D._args_array([(self.h[b], D.DAG_MUTABLE if m == "m" else D.DAG_CONST)
                                      for b, m in op["args"]])
                self._keep += [prm, args]
                o.kind = D.DAG_TASK_KERNEL
                o.kernel_id = kid
                o.params = C.cast(C.byref(prm), C.c_void_p)
                o.params_bytes = C.sizeof(prm)
                o.args = args
                o.nargs = len(op["args"])
            elif kind == "copy":
                o.kind = D.DAG_TASK_COPY
                o.dst = self.h[op["dst"]]
                o.src = self.h[op["src"]]
                o.dst_off = op.get("dst_off", 0)
                o.src_off = op.get("src_off", 0)
                o.bytes = op["bytes"]
            elif kind == "host_read":
                nb = self.prog.bufs[op["buf"]].nbytes
                if self.read_bytes is not None:
                    nb = min(nb, self.read_bytes)
                o.kind = D.DAG_TASK_HOST_READ
                o.dst = self.h[op["buf"]]
                o.bytes = nb
                if nb:
                    arr = np.zeros(nb, dtype=np.uint8)
                    self.read_bufs.setdefault(op["buf"], []).append(arr)
                    self._keep.append(arr)
                    o.host = arr.ctypes.data
            elif kind == "sync":
                o.kind = D.DAG_TASK_SYNC
            else:
                raise ValueError("unsupported op kind %r" % kind)
        return ops

    def run(self):
        """Submit the whole program; returns the task ids (program order)."""
        ids = D.dag_submit_batch(self.ctx.h, self.ops)
        self.ids = ids
        self.base = ids[0] - 1
        return ids

    def run_calls(self):
        """Same as run() but one C call per operation."""
        ids = []
        for i, op in enumerate(self.prog.ops):
            o = self.ops[i]
            if op["kind"] == "kernel":
                args = [(o.args[j].buf, o.args[j].mode) for j in range(o.nargs)]
                prm = D.make_params(op["kernel"], op.get("params", {}))
                ids.append(D.dag_submit_kernel(self.ctx.h, o.kernel_id, prm, args))
            elif op["kind"] == "copy":
                ids.append(D.dag_submit_copy(self.ctx.h, o.dst, o.dst_off, o.src, o.src_off, o.bytes))
            elif op["kind"] == "host_read":
                arr = self.read_bufs.get(op["buf"], [None])[0] if o.bytes else None
                ids.append(D.dag_host_read(self.ctx.h, o.dst, 0, arr, o.bytes))
            elif op["kind"] == "sync":
                D.dag_sync(self.ctx.h)
                ids.append(D.dag_get_stats(self.ctx.h).tasks)
        self.ids = ids
        self.base = ids[0] - 1
        return ids

    # ---- recurring shapes: record once, replay as one task -----------------------
    def _sub(self, idx):
        arr = (D.dag_op * len(idx))()
        for j, i in enumerate(idx):
            arr[j] = self.ops[i]
        return arr

    def record(self, key, lo=0, hi=None):
        """Record ops[lo:hi] (kernels and copies only) as region `key`; they
        also run once, eagerly."""
        hi = len(self.prog.ops) if hi is None else hi
        idx = [i for i in range(lo, hi) if self.prog.ops[i]["kind"] in ("kernel", "copy")]
        D.dag_region_begin(self.ctx.h, key)
        try:
            D.dag_submit_batch(self.ctx.h, self._sub(idx))
        finally:
            D.dag_region_end(self.ctx.h)

    def run_recurring(self, key, per, host_reads=True):
        """Run the program's kernel/copy calls in chunks of `per` (one
        iteration each), every chunk bracketed by dag_region_run_begin/end:
        the first chunk is recorded, identical later chunks replay it.
        Returns [(task id, replayed)] per chunk."""
        idx = [i for i, o in enumerate(self.prog.ops) if o["kind"] in ("kernel", "copy")]
        out = []
        for c0 in range(0, len(idx), per):
            D.dag_region_run_begin(self.ctx.h, key)
            D.dag_submit_batch(self.ctx.h, self._sub(idx[c0:c0 + per]))
            out.append(D.dag_region_run_end(self.ctx.h))
        if host_reads:
            hr = [i for i, o in enumerate(self.prog.ops) if o["kind"] == "host_read"]
            if hr:
                D.dag_submit_batch(self.ctx.h, self._sub(hr))
        return out

    def replay(self, key, times=1, host_reads=True):
        """Replay region `key` `times` times, then the program's host reads."""
        ids = [D.dag_region_launch(self.ctx.h, key) for _ in range(times)]
        if host_reads:
            idx = [i for i, o in enumerate(self.prog.ops) if o["kind"] == "host_read"]
            if idx:
                ids += D.dag_submit_batch(self.ctx.h, self._sub(idx))
        return ids

    # ---- results relative to the program (positions 1..n) ----------------------
    def edges(self):
        out = set()
        for s, d, b, k in self.ctx.edges():
            if s > self.base and d > self.base and d <= self.base + len(self.prog.ops):
                out.add((s - self.base, d - self.base, self.name_of[b], k))
        return out

    def streams(self):
        res = {}
        for pos in range(1, len(self.prog.ops) + 1):
            inf = self.ctx.info(self.base + pos)
            if inf.stream >= 0:
                res[pos] = inf.stream
        return res

    def waits(self):
        return {pos: [w - self.base for w in self.ctx.waits(self.base + pos)]
                for pos in range(1, len(self.prog.ops) + 1)}

    def read(self, name):
        b = self.prog.bufs[name]
        out = np.zeros(b.nbytes, dtype=np.uint8)
        self.ctx.host_read(self.h[name], out)
        return out

    def release(self):
        for h in self.h.values():
            self.ctx.release(h)
        self.h = {}
