"""Host-side plans of the two query shapes the paper evaluates end to end.

* ``Q11Plan`` -- the fact-side selection of SSB Q1.1 (section 3.1, figure
  "Star Schema Benchmark Q1.1"): three range predicates on fact columns, then
  SUM(price * discount) into one int64.
* ``StarSchema`` / ``star_plan`` -- the pipelined multi-join of the section 5.3
  case study (SSB Q2.1 shape): four dimension tables are built (filtered at
  build time, perfect hashing over their dense keys), then one kernel probes
  them in plan order and adds SUM(m1) into a dense group array indexed by
  (year - 1992) * 1000 + dim3.group.

* ``ServingTemplates`` -- the shared-scan forms of both shapes over one fact
  table (the star schema plus the Q1.1 columns): unfiltered dimension tables
  that carry the group payloads, one query-mask table per dimension, and
  batches of up to 16 queries that differ only in their constants.

Only plan construction lives here; every step runs in the library's kernels.
"""
from __future__ import annotations

import numpy as np
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

    def run(self, out=None, status=None, stream=None, accumulate=False):
        return self.query.run(out=out, status=status, stream=stream, accumulate=accumulate)


def _value_range(col):
    col = np.asarray(col)
    return (int(col.min()), int(col.max())) if col.size else (0, -1)


class StarSchema:
    """Star-schema tables resident in device memory, with their dimension tables."""

    def __init__(self, t: datagen.StarTables, device="cuda"):
        self.n = t.n
        self.fk = [to_dev(c, device) for c in t.fk]
        self.m1 = to_dev(t.m1, device)
        self.m2 = to_dev(t.m2, device)
        self.extra = {k: to_dev(v, device) for k, v in t.extra.items()}
        # value range (min, max) of each fact column, recorded when the table
        # is loaded, as a catalog keeps column statistics: the served Q1.1
        # template sizes its value -> query-mask tables from them
        self.col_range = {"datekey": _value_range(t.fk[0]),
                          **{k: _value_range(v) for k, v in t.extra.items()}}
        self.dims = []
        for j, d in enumerate(t.dims):
            self.dims.append(dict(key=to_dev(d.key, device), filter=to_dev(d.filter, device),
                                  group=to_dev(d.group, device),
                                  year=to_dev(d.year, device) if d.year is not None else None,
                                  packed=to_dev(datagen.packed_payload(d, j), device),
                                  key_min=int(d.key.min()), key_max=int(d.key.max()), n=d.n))
        self.consts = list(t.consts)
        self.device = device
        self.tables = self.new_tables()
        self.status = cx.new_status(device)

    def new_tables(self):
        """One perfect-hash table per dimension; payload: year (dim 0), group (dim 2)."""
        return [cx.HashTable(cx.HT_DIRECT, d["n"], d["key_min"], d["key_max"], has_payload=j in (0, 2),
                             device=self.device) for j, d in enumerate(self.dims)]

    @property
    def fact_cols(self):
        return [*self.fk, self.m1, self.m2]

    def build_items(self, consts=None, tables=None):
        """Filtered builds: dimension j keeps rows with filter == consts[j]."""
        consts = self.consts if consts is None else consts
        tables = self.tables if tables is None else tables
        items = []
        for j, d in enumerate(self.dims):
            payload = d["year"] if j == 0 else (d["group"] if j == 2 else None)
            items.append((tables[j], d["key"], payload, d["filter"], (consts[j], consts[j])))
        return items

    def build(self, consts=None, stream=None, batched=True):
        """Filtered builds into self.tables.
        batched: all four tables in one clear and one build launch."""
        items = self.build_items(consts)
        if batched:
            cx.build_tables(items, status=self.status, stream=stream)
        else:
            for ht, keys, payload, filt, rng in items:
                ht.build(keys, payload=payload, filter_col=filt, filter=rng, status=self.status, stream=stream)
        return self.tables

    def plan(self, order=DEFAULT_JOIN_ORDER, tables=None):
        tables = self.tables if tables is None else tables
        joins = []
        for j in order:
            jj = dict(table=tables[j], fk_col=j)
            if j == 0:
                jj["group"] = (32, 0, datagen.FIRST_YEAR, GROUPS_PER_YEAR)
            if j == 2:
                jj["group"] = (32, 0, 0, 1)
            joins.append(jj)
        return cx.StarQuery(self.fact_cols, n_groups=STAR_GROUPS, joins=joins,
                            agg=cx.AGG_SUM, agg_cols=(4, 0))


# ------------------------------------------------------------ flight shapes --
def q1x_consts(flight, year=1994, month=1, day=6):
    """Fact-side predicates of the SSB flight-1 shapes (section 5.1 runs the
    SSB flights) on (datekey, discount, quantity): Q1.1 a year, discount 1..3,
    quantity < 25; Q1.2 a month, discount 4..6, quantity 26..35; Q1.3 seven
    consecutive days, discount 5..7, quantity 26..35."""
    if flight == 1:
        lo, hi = datagen.q11_year_range(year)
        return (lo, hi), (1, 3), (cx.I32_MIN, 24)
    if flight == 2:
        return (year * 10000 + month * 100 + 1, year * 10000 + month * 100 + 31), (4, 6), (26, 35)
    if flight == 3:
        return ((datagen.date_key(year, month, day), datagen.date_key(year, month, day, plus_days=6)),
                (5, 7), (26, 35))
    raise ValueError("flight 1 has queries 1, 2 and 3")


def q1x_plan(cols, flight, **kw):
    """SUM(price * discount) under the flight-1 predicates; cols = (datekey,
    discount, quantity, price)."""
    d, disc, qty = q1x_consts(flight, **kw)
    return cx.StarQuery(list(cols), n_groups=1, preds=[(0, *d), (1, *disc), (2, *qty)],
                        agg=cx.AGG_SUM_PRODUCT, agg_cols=(3, 1))


PACK_FILTER_SHIFT = datagen.PACK_FILTER_SHIFT


class FlightTemplates:
    """More star-query shapes over one star schema (the SSB flights 3 and 4
    pattern: joins filtered by ranges, several group attributes, SUM(m1) or
    SUM(m1 - m2)).  Dimension tables are built once, unfiltered, with packed
    payloads, so every template and constant set reads its filters and group
    fields from the payload at probe time (no per-query build)."""

    def __init__(self, schema: StarSchema):
        self.s = schema
        self.status = cx.new_status(schema.device)
        self.tables = []
        for d in schema.dims:
            # payload: the packed (filter, group) column drawn on the host
            ht = cx.HashTable(cx.HT_DIRECT, d["n"], d["key_min"], d["key_max"], has_payload=True,
                              device=schema.device)
            ht.build(d["key"], payload=d["packed"], status=self.status)
            self.tables.append(ht)

    def _join(self, j, filt=None, year=None, group=None):
        jj = dict(table=self.tables[j], fk_col=j)
        if filt is not None:
            jj["filter"] = (5, PACK_FILTER_SHIFT, filt[0], filt[1])
        if year is not None:                       # dim0: filter on the year field
            jj["filter"] = (10, 0, year[0] - datagen.FIRST_YEAR, year[1] - datagen.FIRST_YEAR)
        if group is not None:
            jj["group"] = group                    # (bits, shift, base, stride)
        return jj

    def q3(self, c1, c3, years=(1992, 1997)):
        """Flight-3 shape: three joins, dim1.filter = c1, dim3.filter in
        [c3, c3 + 4], year in `years`; group by (year, dim2.group, dim1.group
        mod 8); SUM(m1).  7 x 1000 x 8 = 56,000 groups."""
        joins = [self._join(1, filt=(c1, c1), group=(3, 0, 0, 1)),
                 self._join(3, filt=(c3, c3 + 4)),
                 self._join(0, year=years, group=(10, 0, 0, 8000)),
                 self._join(2, group=(10, 0, 0, 8))]
        return cx.StarQuery(self.s.fact_cols, n_groups=56_000, joins=joins, agg=cx.AGG_SUM, agg_cols=(4, 0))

    def q4(self, c1, c2, years=(1997, 1998)):
        """Flight-4 shape: four joins, year in `years`, dim1.filter in
        [c1, c1 + 2], dim2.filter = c2, dim3.filter <= 12; group by (year,
        dim1.group mod 16); SUM(m1 - m2).  7 x 16 = 112 groups."""
        joins = [self._join(1, filt=(c1, c1 + 2), group=(4, 0, 0, 1)),
                 self._join(0, year=years, group=(10, 0, 0, 16)),
                 self._join(2, filt=(c2, c2)),
                 self._join(3, filt=(0, 12))]
        return cx.StarQuery(self.s.fact_cols, n_groups=112, joins=joins, agg=cx.AGG_SUM_DIFF, agg_cols=(4, 5))


# ------------------------------------------------------------ serving forms --
Q11_COLS = ("discount", "quantity", "price")


class ServingTemplates:
    """Star-schema fact table with the Q1.1 columns, and the two query templates.

    Fact columns: 0-3 the foreign keys (0 = date key), 4-5 the measures,
    6 discount, 7 quantity, 8 price.
    """

    STAR, Q11 = 0, 1

    def __init__(self, schema: StarSchema):
        if not all(k in schema.extra for k in Q11_COLS):
            raise ValueError("the fact table needs the Q1.1 columns")
        self.s = schema
        dev = schema.device
        self.cols = [*schema.fk, schema.m1, schema.m2, *[schema.extra[k] for k in Q11_COLS]]
        # unfiltered dimension tables: presence plus the group payloads
        self.tables = []
        self.status = cx.new_status(dev)
        for j, d in enumerate(schema.dims):
            payload = d["year"] if j == 0 else (d["group"] if j == 2 else None)
            ht = cx.HashTable(cx.HT_DIRECT, d["n"], d["key_min"], d["key_max"], has_payload=payload is not None,
                              device=dev)
            ht.build(d["key"], payload=payload, status=self.status)
            self.tables.append(ht)
        # query-mask tables: rank-compressed where the dimension's keys fill
        # little of their span (the date keys), so that the date table fits
        # in LDS beside the first join's
        self.masks = [cx.QueryMask(d["key_min"], d["key_max"], device=dev, keys=d["key"], status=self.status)
                      for d in schema.dims]
        joins = []
        for j in DEFAULT_JOIN_ORDER:
            jj = dict(table=self.tables[j], fk_col=j)
            if j == 0:
                jj["group"] = (32, 0, datagen.FIRST_YEAR, GROUPS_PER_YEAR)
            if j == 2:
                jj["group"] = (32, 0, 0, 1)
            joins.append(jj)
        self.star_template = cx.StarQuery(self.cols, n_groups=STAR_GROUPS, joins=joins, agg=cx.AGG_SUM,
                                          agg_cols=(4, 0))
        self.star_scan = cx.SharedScan(self.star_template, [self.masks[j] for j in DEFAULT_JOIN_ORDER])
        # The Q1.1 template's three range predicates (datekey, discount,
        # quantity) run as lookups into per-batch value -> query-mask tables
        # over each column's value domain: a presence table over the domain
        # and a query mask per value, built like a dimension's.  A row passes
        # query q's range on a column iff its value's mask has bit q, which
        # is the range test itself for every value of the domain.
        # Each table covers every value between the column's minimum and
        # maximum (the table's statistics), so no row's value falls outside
        # it, whatever the data.
        # The date column's domain is its distinct values (2,556 dates over a
        # span of 61,130 yyyymmdd keys), so its mask table is rank-compressed
        # (20 KB instead of 122 KB) and the pass fits more workgroups per CU;
        # discount and quantity keep plain tables over their small ranges.
        self.q11_domains = [self._domain(*schema.col_range[name], fk_col, dev,
                                         values=torch.unique(self.cols[fk_col]) if fk_col == 0 else None)
                            for name, fk_col in (("datekey", 0), ("discount", 6), ("quantity", 7))]
        q11_joins = []
        for dm in self.q11_domains:
            ht = cx.HashTable(cx.HT_DIRECT, dm["n"], dm["key_min"], dm["key_max"], has_payload=False, device=dev)
            ht.build(dm["key"], status=self.status)
            dm["table"] = ht
            dm["mask"] = cx.QueryMask(dm["key_min"], dm["key_max"], device=dev, keys=dm["key"], status=self.status)
            q11_joins.append(dict(table=ht, fk_col=dm["fk_col"]))
        self.q11_template = cx.StarQuery(self.cols, n_groups=1, joins=q11_joins,
                                         agg=cx.AGG_SUM_PRODUCT, agg_cols=(8, 6))
        self.q11_scan = cx.SharedScan(self.q11_template, [dm["mask"] for dm in self.q11_domains])

    MAX_DOMAIN = 1 << 22

    @classmethod
    def _domain(cls, lo, hi, fk_col, dev, values=None):
        """Value domain of a fact column: every value from its minimum to its
        maximum, or `values` (its distinct values, device int32) when given."""
        if hi < lo:
            lo = hi = 0                                      # empty column: any one-value domain
            values = None
        if hi - lo + 1 > cls.MAX_DOMAIN:
            raise ValueError(f"fact column {fk_col} spans {hi - lo + 1} values; a value -> query-mask "
                             f"table covers at most {cls.MAX_DOMAIN}")
        keys = (torch.arange(lo, hi + 1, dtype=torch.int32, device=dev) if values is None
                else values.to(device=dev, dtype=torch.int32).contiguous())
        return dict(key=keys, filter=keys, n=keys.numel(), key_min=lo, key_max=hi, fk_col=fk_col)

    def server_templates(self):
        """Template descriptions for cx.Server: 0 the star query, 1 Q1.1."""
        d = self.s.dims
        star = dict(plan=self.star_template,
                    dims=[(d[j]["key"], d[j]["filter"], d[j]["n"], self.masks[j]) for j in DEFAULT_JOIN_ORDER])
        q11 = dict(plan=self.q11_template,
                   dims=[(dm["key"], dm["filter"], dm["n"], dm["mask"]) for dm in self.q11_domains])
        return [star, q11]

    @staticmethod
    def star_request(consts):
        """Keyword arguments of Server.submit for a star query (template 0)."""
        return dict(filters=[(consts[j], consts[j]) for j in DEFAULT_JOIN_ORDER])

    @classmethod
    def q11_request(cls, year, disc_lo, qty_max):
        """Keyword arguments of Server.submit for a Q1.1 query (template 1)."""
        return dict(filters=cls.q11_preds(year, disc_lo, qty_max))

    @property
    def n_rows(self):
        return self.s.n

    def build_star_masks(self, consts_per_query, stream=None):
        """Dimension j of query q keeps rows with filter == consts_per_query[q][j]."""
        cx.build_query_masks([(self.masks[j], d["key"], d["filter"], [(c[j], c[j]) for c in consts_per_query])
                              for j, d in enumerate(self.s.dims)], status=self.status, stream=stream)

    @staticmethod
    def q11_preds(year, disc_lo, qty_max):
        lo, hi = datagen.q11_year_range(year)
        return [(lo, hi), (disc_lo, disc_lo + 2), (cx.I32_MIN, qty_max)]

    def run_star_batch(self, outs, row_begin=0, row_end=None, status=None, stream=None):
        return self.star_scan.run([[] for _ in outs], outs, row_begin, row_end, status=status, stream=stream)

    def build_q11_masks(self, consts_per_query, stream=None):
        ranges = [self.q11_preds(*c) for c in consts_per_query]
        cx.build_query_masks([(dm["mask"], dm["key"], dm["filter"], [r[i] for r in ranges])
                              for i, dm in enumerate(self.q11_domains)], status=self.status, stream=stream)

    def run_q11_batch(self, consts, outs, row_begin=0, row_end=None, status=None, stream=None):
        self.build_q11_masks(consts, stream=stream)
        return self.q11_scan.run([[] for _ in outs], outs, row_begin, row_end, status=status, stream=stream)

    def single_star(self, consts):
        """The same star query as one plain launch (filtered builds)."""
        self.s.build(consts)
        return self.s.plan().run()[0]

    def single_q11(self, year, disc_lo, qty_max):
        preds = self.q11_preds(year, disc_lo, qty_max)
        q = cx.StarQuery(self.cols, n_groups=1, preds=[(0, *preds[0]), (6, *preds[1]), (7, *preds[2])],
                         agg=cx.AGG_SUM_PRODUCT, agg_cols=(8, 6))
        return q.run()[0]
