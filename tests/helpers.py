"""Test-side helpers: oracle arguments for the workload shapes, and printing
of the case a GPU step is about to run (flushed, so a fault names it)."""
import sys

import numpy as np

import oracle
from paper_2003_01178_amd import datagen

STAR_GROUPS = 7000


def announce(*what):
    print("CASE", *what, flush=True)
    sys.stdout.flush()


def star_oracle_joins(t, consts):
    """Oracle form of the star query: dim j keeps filter == consts[j]; group =
    (dim0.year - 1992) * 1000 + dim2.group; SUM(m1)."""
    joins = []
    for j, d in enumerate(t.dims):
        jj = dict(fk_col=j, key=d.key, filter=d.filter, flo=consts[j], fhi=consts[j])
        if j == 0:
            jj.update(group=d.year, base=1992, stride=1000)
        if j == 2:
            jj.update(group=d.group, base=0, stride=1)
        joins.append(jj)
    return joins


def star_oracle(t, consts=None):
    consts = t.consts if consts is None else consts
    return oracle.star([*t.fk, t.m1, t.m2], STAR_GROUPS, joins=star_oracle_joins(t, consts),
                       agg=oracle.AGG_SUM, agg_cols=(4, 0), return_survivors=True)


def q11_oracle(f, year=1994, disc=(1, 3), qty_max=24):
    lo, hi = datagen.q11_year_range(year)
    out = oracle.star([f.datekey, f.discount, f.quantity, f.price], 1,
                      preds=[(0, lo, hi), (1, disc[0], disc[1]), (2, -(2 ** 31), qty_max)],
                      agg=oracle.AGG_SUM_PRODUCT, agg_cols=(3, 1))
    return int(out[0])


def project_close(got, want, x1, x2, a, b):
    """|got - want| <= 1e-6 * (|a x1| + |b x2|): fp32 evaluation with two
    roundings is within 2^-23 (|a x1| + |b x2|) of the exact value and the
    oracle within 2^-24 of it, so 1e-6 holds with margin."""
    scale = np.abs(np.float64(a) * x1.astype(np.float64)) + np.abs(np.float64(b) * x2.astype(np.float64))
    err = np.abs(got.astype(np.float64) - want.astype(np.float64))
    return bool(np.all(err <= 1e-6 * scale + 1e-38))
