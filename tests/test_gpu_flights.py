"""More star-query shapes on the fused kernel (the SSB flights 1, 3 and 4
patterns on the synthetic star schema), each against the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle
from helpers import announce
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


@pytest.mark.parametrize("flight", [1, 2, 3])
@pytest.mark.parametrize("n", [4097, 1_000_003])
def test_q1x_matches_oracle(flight, n):
    announce("q1x", flight, n)
    f = datagen.q11_fact(n, workload=600 + flight)
    cols = [dev(c) for c in (f.datekey, f.discount, f.quantity, f.price)]
    for kw in (dict(year=1993, month=3, day=5), dict(year=1997, month=12, day=27)):
        q = queries.q1x_plan(cols, flight, **kw)
        out, st = q.run()
        cx.check_status(st)
        d, disc, qty = queries.q1x_consts(flight, **kw)
        want = oracle.star([f.datekey, f.discount, f.quantity, f.price], 1,
                           preds=[(0, *d), (1, *disc), (2, *qty)], agg=oracle.AGG_SUM_PRODUCT, agg_cols=(3, 1))
        assert int(out.item()) == int(want[0]), (flight, kw)


@pytest.fixture(scope="module")
def flights():
    t = datagen.star_tables(n=2_000_003, workload=77)
    s = queries.StarSchema(t)
    ft = queries.FlightTemplates(s)
    cx.check_status(ft.status)
    return t, ft


def _oracle_join(d, fk_col, filt=None, group=None, base=0, stride=0):
    jj = dict(fk_col=fk_col, key=d.key)
    if filt is not None:
        attr, lo, hi = filt
        jj.update(filter=attr, flo=lo, fhi=hi)
    if group is not None:
        jj.update(group=group, base=base, stride=stride)
    return jj


def test_q3_shape_matches_oracle(flights):
    t, ft = flights
    rng = np.random.default_rng(3)
    dims = t.dims
    for trial in range(3):
        c1, c3 = int(rng.integers(0, 25)), int(rng.integers(0, 21))
        years = (1992 + trial, 1996 + trial)
        announce("q3 shape", c1, c3, years)
        out, st = ft.q3(c1, c3, years).run()
        cx.check_status(st)
        joins = [_oracle_join(dims[1], 1, (dims[1].filter, c1, c1), dims[1].group % 8, 0, 1),
                 _oracle_join(dims[3], 3, (dims[3].filter, c3, c3 + 4)),
                 _oracle_join(dims[0], 0, (dims[0].year, *years), dims[0].year, 1992, 8000),
                 _oracle_join(dims[2], 2, None, dims[2].group, 0, 8)]
        want = oracle.star([*t.fk, t.m1, t.m2], 56_000, joins=joins, agg=oracle.AGG_SUM, agg_cols=(4, 0))
        assert want.any()
        assert np.array_equal(out.cpu().numpy(), want), (trial, c1, c3)


def test_q4_shape_matches_oracle(flights):
    t, ft = flights
    rng = np.random.default_rng(4)
    dims = t.dims
    for trial in range(3):
        c1, c2 = int(rng.integers(0, 23)), int(rng.integers(0, 25))
        years = [(1997, 1998), (1992, 1998), (1995, 1995)][trial]
        announce("q4 shape", c1, c2, years)
        out, st = ft.q4(c1, c2, years).run()
        cx.check_status(st)
        joins = [_oracle_join(dims[1], 1, (dims[1].filter, c1, c1 + 2), dims[1].group % 16, 0, 1),
                 _oracle_join(dims[0], 0, (dims[0].year, *years), dims[0].year, 1992, 16),
                 _oracle_join(dims[2], 2, (dims[2].filter, c2, c2)),
                 _oracle_join(dims[3], 3, (dims[3].filter, 0, 12))]
        want = oracle.star([*t.fk, t.m1, t.m2], 112, joins=joins, agg=oracle.AGG_SUM_DIFF, agg_cols=(4, 5))
        assert want.any()
        assert np.array_equal(out.cpu().numpy(), want), (trial, c1, c2)
