"""crystal_run_star_query_noalloc (the star-query entry point that allocates
nothing, for callers that cannot allocate) against crystal_run_star_query on
the same plans: bit-exact int64 results, two calls in a row, the second on a
smaller input, for a scalar plan (SSB Q1.1 shape, whose partials go to the
library's fixed per-device array) and the grouped four-join plan."""
import numpy as np
import pytest
import torch

from helpers import announce, q11_oracle
from paper_2003_01178_amd import crystal as cx
from paper_2003_01178_amd import datagen, queries

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _reset_tuning():
    cx.tune_reset()
    yield
    cx.tune_reset()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_noalloc_q11_two_calls_second_smaller():
    out = torch.empty(1, dtype=torch.int64, device="cuda")
    st = cx.new_status("cuda")
    for n, seed in ((6_000_000, 901), (300_007, 902)):
        announce("noalloc q11", n)
        f = datagen.q11_fact(n, workload=seed)
        plan = queries.Q11Plan(dev(f.datekey), dev(f.discount), dev(f.quantity), dev(f.price))
        st.zero_()
        out.fill_(-1)  # stale contents must not leak into the result
        plan.query.run_noalloc(out, st)
        want, st2 = plan.run()
        torch.cuda.synchronize()
        cx.check_status(st)
        cx.check_status(st2)
        assert int(out.item()) == int(want.item()), n
        if n <= 300_007:
            assert int(out.item()) == q11_oracle(f)


def test_noalloc_q11_many_workgroups():
    """One workgroup per tile at a small tile: as many partials as the fixed
    array holds (8,192), then far fewer on the next call."""
    out = torch.empty(1, dtype=torch.int64, device="cuda")
    st = cx.new_status("cuda")
    for n, (block, ipt, gpc) in ((8192 * 256, (64, 4, 32)), (1000, (64, 4, 32))):
        announce("noalloc q11 grid", n, block, ipt, gpc)
        cx.tune_set(cx.K_STAR, block, ipt, gpc)
        f = datagen.q11_fact(n, workload=903 + n % 7)
        plan = queries.Q11Plan(dev(f.datekey), dev(f.discount), dev(f.quantity), dev(f.price))
        st.zero_()
        plan.query.run_noalloc(out, st)
        want, _ = plan.run()
        torch.cuda.synchronize()
        cx.check_status(st)
        assert int(out.item()) == int(want.item()), n


def test_noalloc_star_grouped_two_calls_second_smaller():
    out = torch.empty(queries.STAR_GROUPS, dtype=torch.int64, device="cuda")
    st = cx.new_status("cuda")
    for n, seed in ((2_000_003, 3), (100_001, 5)):
        announce("noalloc star", n)
        t = datagen.star_tables(n=n, workload=seed)
        s = queries.StarSchema(t)
        s.build()
        plan = s.plan()
        st.zero_()
        out.fill_(7)
        plan.run_noalloc(out, st)
        want, st2 = plan.run()
        torch.cuda.synchronize()
        cx.check_status(st)
        cx.check_status(st2)
        cx.check_status(s.status)
        assert torch.equal(out, want), n
