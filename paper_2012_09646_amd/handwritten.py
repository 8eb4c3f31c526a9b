"""Hand-written schedules of the benchmark DAGs, for comparison with the
scheduler (the paper measures its scheduler against hand-optimized
multi-stream code and CUDA Graphs built from it, Sec. V-D).

A schedule gives, for every kernel and copy call of a recorded region in
order, the stream it runs on and the earlier calls it waits for through
events, chosen the way a programmer would write multi-stream HIP code for
the workload.  ``dag_region_set_schedule`` installs it on the region after
checking that it orders every dependency the scheduler inferred; the region
then runs as a multi-stream replay (graph mode 1) or as a hipGraph (graph
mode 0), with no dependency analysis per call.
"""

from . import dagrt as D

HITS_CALLS_PER_ITERATION = 6


def schedule(prog):
    """Hand-written schedule of the region that ``bench.py`` records for
    `prog`: the whole DAG, or one iteration for HITS.  A list of
    (stream, [earlier call indices waited for])."""
    if prog.name == "vec":
        # x^2 and y^2 on two streams, the sum after both on the first
        return [(0, []), (1, []), (0, [1])]
    if prog.name == "bs":
        # the three-stage pipeline: copies in on stream 1, pricing on stream 0,
        # copies out on stream 2, each stage waiting for the stock's previous one
        n = sum(1 for o in prog.ops if o["kind"] in ("kernel", "copy"))
        out = []
        for i in range(0, n, 3):
            out += [(1, []), (0, [i]), (2, [i + 1])]
        return out
    if prog.name == "img":
        # branch k (blur, Sobel, min/max, normalise) on stream k; the combine on
        # stream 0 after the other two branches' normalisation
        return [(i % 3, []) for i in range(12)] + [(0, [10, 11])]
    if prog.name == "hits":
        # the authority chain on stream 0, the hub chain on stream 1; each
        # normalisation overwrites the vector the other chain's product reads
        # (the next iteration's ordering comes from the region launches)
        return [(0, []), (1, []), (0, []), (1, []), (0, [1]), (1, [0])]
    if prog.name == "ml":
        # naive Bayes and ridge on two streams, the ensemble after both
        return [(0, []), (1, []), (0, [1])]
    if prog.name == "dl":
        # image 1's layers on stream 0, image 2's on stream 1 (calls in the order
        # conv1 x2, conv2 x2, dense x2), the combination after both embeddings
        return [(0, []), (1, []), (0, []), (1, []), (0, []), (1, []), (0, [5])]
    raise ValueError("no hand-written schedule for %s" % prog.name)


def install(ctx, key, prog):
    D.dag_region_set_schedule(ctx.h, key, schedule(prog))
