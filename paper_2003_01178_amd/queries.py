"""Host-side plans of the two query shapes the paper evaluates end to end.

* ``Q11Plan`` -- the fact-side selection of SSB Q1.1 (section 3.1, figure
  "Star Schema Benchmark Q1.1"): three range predicates on fact columns, then
  SUM(price * discount) into one int64.
* ``StarSchema`` / ``star_plan`` -- the pipelined multi-join of the section 5.3
  case study (SSB Q2.1 shape): four dimension tables are built (filtered at
  build time, perfect hashing over their dense keys), then one kernel probes
  them in plan order and adds SUM(m1) into a dense group array indexed by
  (year - 1992) * 1000 + dim3.group.

Only plan construction lives here; every step runs in the library's kernels.
"""
from __future__ import annotations

import torch

from . import crystal as cx
from . import datagen

N_YEARS = 7
GROUPS_PER_YEAR = 1000
STAR_GROUPS = N_YEARS * GROUPS_PER_YEAR
DEFAULT_JOIN_ORDER = (1, 0, 2, 3)   # smallest presence bitmap first


def to_dev(a, device="cuda"):
    return torch.from_numpy(a).to(device)


class Q11Plan:
    """SSB Q1.1 shape over resident columns (datekey, discount, quantity, price)."""

    def __init__(self, datekey, discount, quantity, price, year=1994, disc=(1, 3), qty_max=24):
        lo, hi = datagen.q11_year_range(year)
        self.query = cx.StarQuery(
            [datekey, discount, quantity, price], n_groups=1,
            preds=[(0, lo, hi), (1, disc[0], disc[1]), (2, cx.I32_MIN, qty_max)],
            agg=cx.AGG_SUM_PRODUCT, agg_cols=(3, 1))

    def run(self, out=None, status=None, stream=None):
        return self.query.run(out=out, status=status, stream=stream)


class StarSchema:
    """Star-schema tables resident in device memory, with their dimension tables."""

    def __init__(self, t: datagen.StarTables, device="cuda"):
        self.n = t.n
        self.fk = [to_dev(c, device) for c in t.fk]
        self.m1 = to_dev(t.m1, device)
        self.m2 = to_dev(t.m2, device)
        self.extra = {k: to_dev(v, device) for k, v in t.extra.items()}
        self.dims = []
        for d in t.dims:
            self.dims.append(dict(key=to_dev(d.key, device), filter=to_dev(d.filter, device),
                                  group=to_dev(d.group, device),
                                  year=to_dev(d.year, device) if d.year is not None else None,
                                  key_min=int(d.key.min()), key_max=int(d.key.max()), n=d.n))
        self.consts = list(t.consts)
        self.device = device
        # one perfect-hash table per dimension; payload: year (dim 0), group (dim 2)
        self.tables = []
        for j, d in enumerate(self.dims):
            self.tables.append(cx.HashTable(cx.HT_DIRECT, d["n"], d["key_min"], d["key_max"],
                                            has_payload=j in (0, 2), device=device))
        self.status = cx.new_status(device)

    @property
    def fact_cols(self):
        return [*self.fk, self.m1, self.m2]

    def build(self, consts=None, stream=None):
        """Filtered builds: dimension j keeps rows with filter == consts[j]."""
        consts = self.consts if consts is None else consts
        for j, d in enumerate(self.dims):
            payload = d["year"] if j == 0 else (d["group"] if j == 2 else None)
            self.tables[j].build(d["key"], payload=payload, filter_col=d["filter"],
                                 filter=(consts[j], consts[j]), status=self.status, stream=stream)
        return self.tables

    def plan(self, order=DEFAULT_JOIN_ORDER):
        joins = []
        for j in order:
            jj = dict(table=self.tables[j], fk_col=j)
            if j == 0:
                jj["group"] = (32, 0, datagen.FIRST_YEAR, GROUPS_PER_YEAR)
            if j == 2:
                jj["group"] = (32, 0, 0, 1)
            joins.append(jj)
        return cx.StarQuery(self.fact_cols, n_groups=STAR_GROUPS, joins=joins,
                            agg=cx.AGG_SUM, agg_cols=(4, 0))
