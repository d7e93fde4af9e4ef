"""HIP-graph capture of a whole star-query step (four filtered builds plus the
fused kernel) and of a scalar query: every replay, with eager work in
between, equals the eager result and the oracle.  Also the autotuner's
graph-replay timing of a short query."""
import numpy as np
import pytest
import torch

from helpers import announce, star_oracle
from paper_2003_01178_amd import crystal as cx
from paper_2003_01178_amd import datagen, queries

pytestmark = pytest.mark.gpu


def test_graph_replays_star_step():
    announce("graph star")
    t = datagen.star_tables(n=2_000_000, workload=51)
    s = queries.StarSchema(t)
    plan = s.plan()
    stream = torch.cuda.Stream()
    out = torch.zeros(queries.STAR_GROUPS, dtype=torch.int64, device="cuda")
    st = cx.new_status()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        s.build(stream=stream)                        # eager first: caches device attributes
        plan.run(out=out, status=st, stream=stream)
    stream.synchronize()
    eager = out.cpu().numpy().copy()
    assert np.array_equal(eager, star_oracle(t)[0])
    with cx.Graph.capture(stream) as g:
        s.build(stream=stream)
        plan.run(out=out, status=st, stream=stream)
    other = queries.StarSchema(datagen.star_tables(n=300_000, workload=52))
    for rep in range(4):
        out.fill_(-1)                                 # the replay must clear and recompute
        torch.cuda.synchronize()
        g.launch(stream)
        stream.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager), rep
        other.build()                                 # unrelated eager work between replays
        other.plan().run()
        torch.cuda.synchronize()
    cx.check_status(st)
    g.close()


def test_graph_replays_scalar_query():
    announce("graph q11")
    f = datagen.q11_fact(1_000_000, workload=53)
    cols = [queries.to_dev(c) for c in (f.datekey, f.discount, f.quantity, f.price)]
    plan = queries.Q11Plan(*cols)
    stream = torch.cuda.Stream()
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = cx.new_status()                              # allocated before capture
    torch.cuda.synchronize()
    plan.run(out=out, status=st, stream=stream)
    stream.synchronize()
    eager = int(out.item())
    with cx.Graph.capture(stream) as g:
        plan.run(out=out, status=st, stream=stream)
    for rep in range(3):
        out.fill_(7)
        torch.cuda.synchronize()
        g.launch(stream)
        stream.synchronize()
        assert int(out.item()) == eager, rep
    g.close()


def test_autotuner_graph_timing_of_a_short_query():
    """The autotuner's graph-replay timing (a graph of ten launches of a
    6M-row Q1.1-shaped query, re-captured per call): a positive time per
    query well under a millisecond, the result of the replays equal to the
    eager one, and the same candidate timed twice within a factor of two."""
    from paper_2003_01178_amd import autotune
    announce("autotune graph timing")
    f = datagen.q11_fact(6_000_000, workload=54)
    plan = queries.Q11Plan(*[queries.to_dev(c) for c in (f.datekey, f.discount, f.quantity, f.price)])
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    st = cx.new_status()
    plan.run(out=out, status=st)
    torch.cuda.synchronize()
    eager = int(out.item())
    times = [autotune.time_graph_ms(lambda s: plan.run(out=out, status=st, stream=s), reps=5) for _ in range(2)]
    assert all(0.0 < t < 1.0 for t in times), times
    assert max(times) < 2 * min(times), times
    assert int(out.item()) == eager
    cx.check_status(st)
