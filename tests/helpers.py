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


def oracle_star_rows(fact_cols, n_groups, threads=16, **kw):
    """oracle.star over contiguous row ranges on several threads (the
    oracle's C call releases the GIL); the partial group arrays are added
    modulo 2^64.  Every aggregate is a sum over rows, so this is the answer
    over the whole table, bit for bit."""
    from concurrent.futures import ThreadPoolExecutor
    oracle.load()
    n = len(fact_cols[0])
    threads = max(1, min(threads, n // 100_000 + 1))
    bounds = [n * i // threads for i in range(threads + 1)]

    def part(ab):
        a, b = ab
        return oracle.star([c[a:b] for c in fact_cols], n_groups, **kw)

    with ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(part, zip(bounds[:-1], bounds[1:])))
    total = np.zeros(int(n_groups), dtype=np.uint64)
    for p in parts:
        total += p.view(np.uint64)
    return total.view(np.int64)


def star_oracle_par(t, consts):
    """The star query (SUM(m1), dims filtered by consts, 7,000 groups) over
    all rows, on several threads."""
    return oracle_star_rows([*t.fk, t.m1, t.m2], STAR_GROUPS, joins=star_oracle_joins(t, consts),
                            agg=oracle.AGG_SUM, agg_cols=(4, 0))


def q11_oracle_par(datekey, discount, quantity, price, year, disc, qty_max):
    lo, hi = datagen.q11_year_range(year)
    out = oracle_star_rows([datekey, discount, quantity, price], 1,
                           preds=[(0, lo, hi), (1, disc[0], disc[1]), (2, -(2 ** 31), qty_max)],
                           agg=oracle.AGG_SUM_PRODUCT, agg_cols=(3, 1))
    return int(out[0])


def qmask_entries(qm):
    """A query-mask table read back from the device and decoded on the host
    with numpy, one int64 entry per key of its span, following the layout
    include/crystal.h states: a plain table is one 16-bit entry per key; a
    rank-compressed one is a directory of (presence bits of 32 keys, keys
    present before them) pairs, then one 16-bit entry per present key and a
    zero entry, so a key's entry is at the directory count plus the number of
    presence bits set below it."""
    span, ranked = int(qm.c.span), int(qm.c.ranked)
    raw = qm.mem.cpu().numpy().view(np.uint8)
    if not ranked:
        return raw[: 2 * span].view(np.uint16).astype(np.int64)
    n_dir = (span + 31) // 32 + 1
    dir_words = raw[: 8 * n_dir].view(np.uint32).reshape(-1, 2).astype(np.int64)
    ent = raw[8 * n_dir: 8 * n_dir + 2 * (ranked + 1)].view(np.uint16).astype(np.int64)
    k = np.arange(span, dtype=np.int64)
    bits, before = dir_words[k >> 5, 0], dir_words[k >> 5, 1]
    b = k & 31
    present = ((bits >> b) & 1) == 1
    below = np.bitwise_count((bits & ((np.int64(1) << b) - 1)).astype(np.uint64)).astype(np.int64)
    return np.where(present, ent[np.where(present, before + below, ranked)], ent[ranked])
