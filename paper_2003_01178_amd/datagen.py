"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers and lays them out as 4-byte columns; it
contains none of the query arithmetic.  Both the GPU path and the CPU oracle
are fed from the same host arrays it returns.

Seeds: base seed 200301178 plus the workload index; one numpy PCG64 stream per
column via ``SeedSequence.spawn``.  Workloads:

* ``q11_fact`` -- fact table with the columns of SSB Q1.1 (section 3.1):
  datekey (yyyymmdd of a uniform day over 7 years starting 1992-01-01),
  discount U{0..10}, quantity U{1..50}, extended price U{90000..10000000}.
* ``select_column`` -- int32 U{0..2^31-1} (section 4.2, Q3 micro-benchmark;
  the paper's column is 4-byte float, here int32 as the workload fixes).
* ``project_columns`` -- two fp32 columns U[0,1) (section 4.1, Q1/Q2).
* ``join_tables`` -- dimension keys a shuffled 0..D-1 with int32 payloads, probe
  keys uniform over 0..D-1 (section 4.3, Q4).
* ``star_tables`` -- a four-dimension star schema shaped like SSB at scale
  factor 20 (section 5.1): fact rows with four foreign keys and two measures,
  dimensions of 2,556 / 40,000 / 200,000 / 600,000 rows, each with a filter
  attribute U{0..24} and a group attribute U{0..999}; the date dimension also
  carries its year.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 200301178
N_DAYS = 2556                    # 7 years of days starting 1992-01-01
FIRST_YEAR = 1992
INT32_MIN = -(2 ** 31)
INT32_MAX = 2 ** 31 - 1


def streams(workload: int, n: int):
    """``n`` independent PCG64 generators for workload index ``workload``."""
    ss = np.random.SeedSequence(BASE_SEED + int(workload))
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(n)]


def day_keys(n_days: int = N_DAYS):
    """(yyyymmdd key, year) of consecutive days starting 1992-01-01."""
    d = np.datetime64("1992-01-01") + np.arange(n_days)
    year = d.astype("datetime64[Y]").astype(np.int64) + 1970
    month = d.astype("datetime64[M]").astype(np.int64) % 12 + 1
    mday = (d - d.astype("datetime64[M]")).astype(np.int64) + 1
    key = year * 10000 + month * 100 + mday
    return key.astype(np.int32), year.astype(np.int32)


def date_key(year: int, month: int, day: int, plus_days: int = 0) -> int:
    """yyyymmdd key of the calendar date `plus_days` days after year-month-day."""
    d = np.datetime64(f"{int(year):04d}-{int(month):02d}-{int(day):02d}") + int(plus_days)
    y = int(d.astype("datetime64[Y]").astype(np.int64)) + 1970
    m = int(d.astype("datetime64[M]").astype(np.int64)) % 12 + 1
    dd = int((d - d.astype("datetime64[M]")).astype(np.int64)) + 1
    return y * 10000 + m * 100 + dd


def day_codes(keys) -> np.ndarray:
    """Dictionary code of yyyymmdd date keys: the day's index from 1992-01-01
    (0..2555 over the seven years, 12 bits)."""
    all_keys, _ = day_keys()
    codes = np.searchsorted(all_keys, np.asarray(keys))
    if np.any(codes >= all_keys.size) or np.any(all_keys[np.minimum(codes, all_keys.size - 1)] != keys):
        raise ValueError("not a date key of the seven years")
    return codes.astype(np.int32)


# Packed dimension payload of the flight templates: bits 0..9 the group
# attribute (the date dimension: year - 1992), bits 16..20 the filter attribute.
PACK_FILTER_SHIFT = 16


def packed_payload(dim, j: int) -> np.ndarray:
    """Dimension j's packed payload column: (filter << 16) | group field."""
    grp = (dim.year - FIRST_YEAR) if j == 0 else dim.group
    return ((dim.filter.astype(np.int32) << PACK_FILTER_SHIFT) | grp.astype(np.int32)).astype(np.int32)


def _uniform(g, lo, hi, n):
    """Uniform int32 on the closed interval [lo, hi]."""
    return g.integers(lo, hi, size=int(n), dtype=np.int32, endpoint=True)


# ---------------------------------------------------------------- Q1.1 fact --
@dataclass
class Q11Fact:
    datekey: np.ndarray
    discount: np.ndarray
    quantity: np.ndarray
    price: np.ndarray

    @property
    def n(self):
        return self.datekey.size


def q11_fact(n: int = 6_000_000, workload: int = 0) -> Q11Fact:
    g = streams(workload, 4)
    keys, _ = day_keys()
    day = _uniform(g[0], 0, N_DAYS - 1, n)
    return Q11Fact(datekey=keys[day],
                   discount=_uniform(g[1], 0, 10, n),
                   quantity=_uniform(g[2], 1, 50, n),
                   price=_uniform(g[3], 90_000, 10_000_000, n))


def q11_year_range(year: int):
    """Inclusive datekey range of one calendar year."""
    return int(year) * 10000 + 101, int(year) * 10000 + 1231


# ------------------------------------------------------- operator workloads --
def select_column(n: int = 1 << 29, workload: int = 1) -> np.ndarray:
    (g,) = streams(workload, 1)
    return _uniform(g, 0, INT32_MAX, n)


def select_threshold_range(sigma: float):
    """Inclusive int32 range for ``y < v`` with v = round(sigma * 2^31).

    sigma = 1 keeps every value of U{0..2^31-1}; sigma = 0 keeps none."""
    v = int(round(float(sigma) * 2 ** 31))
    if v >= 2 ** 31:
        return INT32_MIN, INT32_MAX
    return INT32_MIN, v - 1


def project_columns(n: int = 1 << 29, workload: int = 11):
    g1, g2 = streams(workload, 2)
    return (g1.random(int(n), dtype=np.float32), g2.random(int(n), dtype=np.float32))


def radix_pairs(n: int = 1 << 28, workload: int = 12, key_bits: int = 32):
    """(keys, values) of the sort workload: uniform unsigned keys over
    [0, 2^key_bits) and uniform 32-bit values, both as int32 bit patterns."""
    gk, gv = streams(workload, 2)
    keys = gk.integers(0, 1 << int(key_bits), size=int(n), dtype=np.uint64).astype(np.uint32)
    vals = gv.integers(0, 1 << 32, size=int(n), dtype=np.uint64).astype(np.uint32)
    return keys.view(np.int32), vals.view(np.int32)


@dataclass
class JoinTables:
    dim_key: np.ndarray
    dim_val: np.ndarray
    fk: np.ndarray


def join_tables(d: int, n_probe: int = 1 << 28, workload: int = 2) -> JoinTables:
    g = streams(workload, 3)
    key = g[0].permutation(int(d)).astype(np.int32)
    val = _uniform(g[1], 0, INT32_MAX, d)
    fk = _uniform(g[2], 0, int(d) - 1, n_probe)
    return JoinTables(dim_key=key, dim_val=val, fk=fk)


# --------------------------------------------------------------- star schema --
DIM_ROWS = (N_DAYS, 40_000, 200_000, 600_000)


@dataclass
class Dim:
    key: np.ndarray
    filter: np.ndarray
    group: np.ndarray
    year: np.ndarray | None = None

    @property
    def n(self):
        return self.key.size


@dataclass
class StarTables:
    fk: list                 # four int32 fact columns, fk[0] = datekey
    m1: np.ndarray
    m2: np.ndarray
    dims: list               # four Dim
    consts: list             # seeded filter constants c_j in 0..24
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.m1.size


def star_dims(workload: int = 3, dim_rows=DIM_ROWS):
    g = streams(workload + 100, 4 * 3 + 1)
    dims = []
    for j, rows in enumerate(dim_rows):
        gk, gf, gg = g[3 * j], g[3 * j + 1], g[3 * j + 2]
        if j == 0:
            keys, years = day_keys(rows)
            perm = gk.permutation(rows)
            key, year = keys[perm], years[perm]
        else:
            key, year = gk.permutation(rows).astype(np.int32), None
        dims.append(Dim(key=key, filter=_uniform(gf, 0, 24, rows),
                        group=_uniform(gg, 0, 999, rows), year=year))
    consts = [int(c) for c in g[-1].integers(0, 25, size=4)]
    return dims, consts


def star_tables(n: int = 120_000_000, workload: int = 3, dim_rows=DIM_ROWS,
                with_q11_columns: bool = False) -> StarTables:
    """Fact table joined to four dimensions; fk[0] holds date keys."""
    dims, consts = star_dims(workload, dim_rows)
    g = streams(workload, 9)
    keys, _ = day_keys(dim_rows[0])
    day = _uniform(g[0], 0, dim_rows[0] - 1, n)
    fk = [keys[day]]
    for j in range(1, 4):
        fk.append(_uniform(g[j], 0, dim_rows[j] - 1, n))
    t = StarTables(fk=fk, m1=_uniform(g[4], 1, 1_000_000, n),
                   m2=_uniform(g[5], 1, 1_000_000, n), dims=dims, consts=consts)
    if with_q11_columns:
        t.extra["discount"] = _uniform(g[6], 0, 10, n)
        t.extra["quantity"] = _uniform(g[7], 1, 50, n)
        t.extra["price"] = _uniform(g[8], 90_000, 10_000_000, n)
    return t


def random_star_constants(rng: np.random.Generator):
    """Seeded predicate constants for the star-query template."""
    return [int(c) for c in rng.integers(0, 25, size=4)]


def random_q11_constants(rng: np.random.Generator):
    """Seeded constants for the Q1.1 template: (year, discount lo, quantity bound)."""
    year = FIRST_YEAR + int(rng.integers(0, 7))
    d = int(rng.integers(0, 9))
    q = int(rng.integers(2, 51))
    return year, d, q


# ------------------------------------------------ banded served fact table --
BAND_DENSE, BAND_SPARSE, BAND_PLAIN = 0, 1, 2


@dataclass
class BandedSpec:
    """Constants a banded table is drawn around: dense bands hold rows whose
    dimension-1 key has filter == c1, whose date key has filter == c0 and
    lies in `year`, and whose discount lies in [disc_lo, disc_lo + 2]."""
    c0: int
    c1: int
    year: int
    disc_lo: int


def banded_star_tables(n: int, band_rows: int = 1 << 19, workload: int = 51,
                       p_dense: float = 0.3, p_sparse: float = 0.5):
    """Served fact table (star schema plus the Q1.1 columns) in bands of
    ``band_rows`` rows of three kinds, drawn at random per band:

    * dense: every row passes the first two steps of the star template
      (dimension-1 and date joins, for queries with those two constants) and
      of the Q1.1 template (year and discount window);
    * sparse: about 1 row in 600 passes the two star joins and 1 in 400 the
      two Q1.1 tests (date keys outside ``year`` except for 5% of rows);
    * plain: drawn as ``star_tables``, except that 2% of discounts are
      U{11..15} and 2% of quantities are 0 or U{51..60} (values outside the
      generator's usual domains).

    Returns (StarTables, BandedSpec, band kinds)."""
    t = star_tables(n, workload=workload, with_q11_columns=True)
    g = streams(workload + 200, 8)
    d0, d1 = t.dims[0], t.dims[1]
    c1 = int(t.consts[1])
    keys1 = d1.key[d1.filter == c1]
    year = FIRST_YEAR + 2
    # a date filter constant that keeps some dates of `year`
    c0 = next(c for c in range(25) if np.any((d0.filter == c) & (d0.year == year)))
    dates_dense = d0.key[(d0.filter == c0) & (d0.year == year)]
    dates_other = d0.key[d0.year != year]
    disc_lo = 4
    n_bands = (n + band_rows - 1) // band_rows
    kinds = g[0].choice([BAND_DENSE, BAND_SPARSE, BAND_PLAIN], size=n_bands,
                        p=[p_dense, p_sparse, 1.0 - p_dense - p_sparse]).astype(np.int32)
    fk0, fk1, disc, qty = t.fk[0], t.fk[1], t.extra["discount"], t.extra["quantity"]
    for b, kind in enumerate(kinds):
        lo, hi = b * band_rows, min(n, (b + 1) * band_rows)
        m = hi - lo
        if kind == BAND_DENSE:
            fk1[lo:hi] = keys1[g[1].integers(0, keys1.size, m)]
            fk0[lo:hi] = dates_dense[g[2].integers(0, dates_dense.size, m)]
            disc[lo:hi] = _uniform(g[3], disc_lo, disc_lo + 2, m)
        elif kind == BAND_SPARSE:
            keep_year = g[4].random(m) < 0.05
            fk0[lo:hi] = np.where(keep_year, fk0[lo:hi], dates_other[g[2].integers(0, dates_other.size, m)])
        else:
            odd_d = g[5].random(m) < 0.02
            disc[lo:hi] = np.where(odd_d, _uniform(g[6], 11, 15, m), disc[lo:hi])
            odd_q = g[5].random(m) < 0.02
            wide = _uniform(g[7], 50, 60, m)
            qty[lo:hi] = np.where(odd_q, np.where(wide == 50, 0, wide), qty[lo:hi])
    return t, BandedSpec(c0=c0, c1=c1, year=year, disc_lo=disc_lo), kinds
