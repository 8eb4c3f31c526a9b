"""Parser of tests/golden/dag_cases.txt (program tokens -> oracle ops)."""

import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
KIND = {"RAW": 0, "WAR": 1, "WAW": 2}


def parse_ops(tokens):
    ops = []
    for tok in tokens:
        if tok == "SYNC":
            ops.append({"kind": "sync"})
            continue
        m = re.fullmatch(r"(K|HR|HW)\((.*)\)", tok)
        if not m:
            raise ValueError(tok)
        head, body = m.groups()
        if head == "K":
            args = [tuple(a.split(":")) for a in body.split(",")]
            ops.append({"kind": "kernel", "kernel": "spin", "params": {}, "args": args})
        elif head == "HR":
            ops.append({"kind": "host_read", "buf": body})
        else:
            ops.append({"kind": "host_write", "buf": body})
    return ops


def load_cases():
    cases = []
    cur = None
    with open(os.path.join(HERE, "golden", "dag_cases.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            if line.startswith("case "):
                parts = line.split()
                cur = {"name": parts[1], "max_streams": int(parts[2].split("=")[1])}
                cases.append(cur)
                continue
            key, val = line.split(":", 1)
            toks = val.split()
            if key == "ops":
                cur["ops"] = parse_ops(toks)
            elif key == "edges":
                edges = set()
                if toks != ["none"]:
                    for t in toks:
                        pair, buf, kind = t.split(":")
                        s, d = pair.split("-")
                        edges.add((int(s), int(d), buf, KIND[kind]))
                cur["edges"] = edges
            elif key == "streams":
                cur["streams"] = [None if t == "-" else int(t) for t in toks]
            elif key == "waits":
                cur["waits"] = [[] if t == "-" else [int(x) for x in t.split(",")] for t in toks]
    return cases


def random_program(rnd, n_ops, n_bufs, host=True):
    """Random program over n_bufs buffers: kernels with 1-4 args of random
    modes, interleaved host reads / writes and syncs."""
    bufs = ["b%d" % i for i in range(n_bufs)]
    ops = []
    for _ in range(n_ops):
        r = rnd.random()
        if host and r < 0.1:
            ops.append({"kind": "host_read", "buf": rnd.choice(bufs)})
        elif host and r < 0.15:
            ops.append({"kind": "host_write", "buf": rnd.choice(bufs)})
        elif host and r < 0.17:
            ops.append({"kind": "sync"})
        else:
            k = rnd.randint(1, 4)
            args = [(rnd.choice(bufs), rnd.choice("cm")) for _ in range(k)]
            ops.append({"kind": "kernel", "kernel": "spin", "params": {}, "args": args})
    return ops


def reach(preds, src, dst):
    stack, seen = [dst], set()
    while stack:
        t = stack.pop()
        if t == src:
            return True
        if t not in seen:
            seen.add(t)
            stack.extend(preds.get(t, ()))
    return False


def uncovered_edges(edges, streams, waits):
    """Edges between GPU tasks that stream order plus event waits do not
    order (brute-force search over the happens-before graph)."""
    preds, last = {}, {}
    for t in sorted(streams):
        s = streams[t]
        preds[t] = ([last[s]] if s in last else []) + list(waits.get(t, []))
        last[s] = t
    return [(s, d) for (s, d, *_rest) in edges if d in streams and s in streams and not reach(preds, s, d)]
