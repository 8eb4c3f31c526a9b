"""Brute-force dependency DAG and stream-policy replay (test infrastructure).

Program model
-------------
A program is a list of operations in program order.  Operation ``j`` (1-based
position in the list) is a dict with a ``kind``:

``kernel`` / ``copy`` / ``macro``
    a computational element (CE) that runs on the GPU; ``args`` is a list of
    ``(buffer, mode)`` pairs (a copy reads ``src`` and modifies ``dst``), mode ``'c'`` (read-only / const annotation) or
    ``'m'`` (modifiable; an argument without annotation is modifiable).
    Paper Sec. IV-A (CEs, dependency sets) and Sec. IV-D (annotations).
``host_read`` / ``host_write``
    a host access to one buffer (``buf``), Sec. IV-A: it becomes a DAG vertex
    only if it conflicts with an active GPU computation, and then the host
    waits for that computation.
``sync``
    wait for everything; retires every active CE (not a vertex).

Dependency rule (Sec. IV-A and the read-only cases of its figure on
dependency computation with read-only arguments)
---------------------------------------------------------------------------
acc(t, b) is None, 'R' or 'W' ('W' = modifiable = read-write; an argument
listed twice takes the stronger mode).  For i < j:

* conflict(i, j, b): both access b and at least one writes it.
* shadow(k; i, j, b), i < k < j: k writes b, or k reads b while both i and j
  write b (a later writer depends on the readers in between, not on the
  earlier writer; a later reader depends on the writer, not on the readers).
* edge i -> j exists iff i is active when j arrives, i is a GPU CE (host
  accesses complete before the next call is issued, so they are never
  sources), and some b conflicts with no shadowing k.

Activity (Sec. IV-B): a CE stays active until the host requires its result or
the result of one of its descendants.  A host access that waits on tasks W
retires W and every ancestor of W in the DAG built so far; ``sync`` retires
all.  Retired CEs add no further edges.

Everything here is deliberately quadratic/cubic: it is only run on programs of
at most a few hundred operations.
"""

from collections import deque

RAW, WAR, WAW = 0, 1, 2
GPU_KINDS = ("kernel", "copy", "macro")
HOST_KINDS = ("host_read", "host_write")


def accesses(op):
    """Map buffer -> 'R' | 'W' for one operation (duplicates take 'W')."""
    kind = op["kind"]
    if kind == "copy":
        pairs = [(op["src"], "c"), (op["dst"], "m")]
    elif kind in GPU_KINDS:
        pairs = op["args"]
    elif kind == "host_read":
        pairs = [(op["buf"], "c")]
    elif kind == "host_write":
        pairs = [(op["buf"], "m")]
    elif kind == "sync":
        pairs = []
    else:
        raise ValueError("unknown op kind %r" % (kind,))
    acc = {}
    for buf, mode in pairs:
        if mode not in ("c", "m"):
            raise ValueError("mode must be 'c' or 'm'")
        a = "W" if mode == "m" else "R"
        if acc.get(buf) != "W":
            acc[buf] = a
    return acc


def _kind_of(a_src, a_dst):
    if a_src == "W" and a_dst == "R":
        return RAW
    if a_src == "R" and a_dst == "W":
        return WAR
    return WAW


class Dag:
    """Result of :func:`build_dag`.

    edges      set of (src, dst, buf, kind) with 1-based program positions
    parents    dict dst -> sorted list of distinct src
    vertex     dict position -> bool (host accesses without a conflict are
               not vertices)
    retired_by dict position -> position of the host access / sync that
               retired it (absent = still active at program end)
    waits_host dict host position -> sorted list of CEs the host waited on
    """

    def __init__(self, n):
        self.n = n
        self.edges = set()
        self.parents = {}
        self.vertex = {}
        self.retired_by = {}
        self.waits_host = {}

    def pair_edges(self):
        return sorted({(s, d) for (s, d, _, _) in self.edges})


def _ancestors(dag, roots):
    seen = set()
    stack = list(roots)
    while stack:
        t = stack.pop()
        if t in seen:
            continue
        seen.add(t)
        stack.extend(dag.parents.get(t, ()))
    return seen


def build_dag(ops):
    """Brute-force DAG of a program (pairwise conflict + shadow checks)."""
    n = len(ops)
    acc = [None] + [accesses(op) for op in ops]
    kinds = [None] + [op["kind"] for op in ops]
    dag = Dag(n)
    active = set()
    for j in range(1, n + 1):
        if kinds[j] == "sync":
            dag.vertex[j] = False
            for t in sorted(active):
                dag.retired_by[t] = j
            active.clear()
            continue
        found = []
        for i in range(1, j):
            if i not in active:
                continue
            for b, a_j in acc[j].items():
                a_i = acc[i].get(b)
                if a_i is None:
                    continue
                if a_i != "W" and a_j != "W":
                    continue
                shadowed = False
                for k in range(i + 1, j):
                    a_k = acc[k].get(b)
                    if a_k == "W" or (a_k == "R" and a_i == "W" and a_j == "W"):
                        shadowed = True
                        break
                if not shadowed:
                    found.append((i, j, b, _kind_of(a_i, a_j)))
        dag.edges.update(found)
        srcs = sorted({e[0] for e in found})
        dag.parents[j] = srcs
        if kinds[j] in GPU_KINDS:
            dag.vertex[j] = True
            active.add(j)
        else:
            dag.vertex[j] = bool(srcs)
            dag.waits_host[j] = srcs
            for t in sorted(_ancestors(dag, srcs) & active):
                dag.retired_by[t] = j
                active.discard(t)
    return dag


def replay_streams(ops, dag, max_streams):
    """Replay the stream-assignment policy and the event waits.

    Policy (Sec. IV-C): existing streams are reused in FIFO order and a new
    stream is created only when no stream is empty; the first child of a
    computation goes on its parent's stream and later children go elsewhere.
    Readings: the "first child" test is made on the active parents in
    submission order, taking the first one that is still the last task of its
    stream; streams that become empty at one host access enter the FIFO in
    creation order; with ``max_streams`` streams already alive and none
    empty, the stream whose last task is oldest is reused.

    Waits: a task waits only on active parents on other streams (Sec. IV-B:
    one event per computation, streams synchronise on events).  For each other
    stream only its latest parent there is a candidate, candidates are taken
    newest first, and one is skipped when it already happens-before the task
    through stream order and earlier waits.  The happens-before test here is a
    plain graph search over all recorded order edges.

    Returns (stream, waits): stream[pos] for GPU CEs, waits[pos] = sorted
    list of the parents actually waited on.
    """
    if max_streams < 1:
        raise ValueError("max_streams must be >= 1")
    stream = {}
    waits = {}
    tail = []            # stream index -> last task placed on it
    nactive = []         # stream index -> number of active tasks on it
    fifo = deque()
    in_fifo = []
    hb_pred = {}         # task -> list of tasks that happen-before it directly
    active = set()

    def hb_reaches(src, dst):
        """True if src happens-before-or-equals dst in the order graph."""
        if dst is None:
            return False
        seen = set()
        stack = [dst]
        while stack:
            t = stack.pop()
            if t == src:
                return True
            if t in seen:
                continue
            seen.add(t)
            stack.extend(hb_pred.get(t, ()))
        return False

    for j in range(1, len(ops) + 1):
        kind = ops[j - 1]["kind"]
        if kind not in GPU_KINDS:
            newly_empty = []
            for t in sorted(active):
                if dag.retired_by.get(t) == j:
                    active.discard(t)
                    s = stream[t]
                    nactive[s] -= 1
                    if nactive[s] == 0 and not in_fifo[s]:
                        newly_empty.append(s)
            for s in sorted(newly_empty):
                fifo.append(s)
                in_fifo[s] = True
            continue
        parents = [p for p in dag.parents.get(j, ()) if p in active]
        chosen = None
        for p in parents:
            if tail[stream[p]] == p:
                chosen = stream[p]
                break
        if chosen is None and fifo:
            chosen = fifo.popleft()
            in_fifo[chosen] = False
        if chosen is None and len(tail) < max_streams:
            tail.append(None)
            nactive.append(0)
            in_fifo.append(False)
            chosen = len(tail) - 1
        if chosen is None:
            chosen = min(range(len(tail)), key=lambda s: (tail[s], s))
        if in_fifo[chosen]:
            fifo.remove(chosen)
            in_fifo[chosen] = False
        prev = tail[chosen]
        latest = {}
        for p in parents:
            s = stream[p]
            if s != chosen and (s not in latest or p > latest[s]):
                latest[s] = p
        taken = []
        for p in sorted(latest.values(), reverse=True):
            if hb_reaches(p, prev) or any(hb_reaches(p, w) for w in taken):
                continue
            taken.append(p)
        preds = ([prev] if prev is not None else []) + taken
        hb_pred[j] = preds
        stream[j] = chosen
        waits[j] = sorted(taken)
        tail[chosen] = j
        nactive[chosen] += 1
        active.add(j)
    return stream, waits
