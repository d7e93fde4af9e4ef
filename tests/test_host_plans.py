"""Host-side plan and input helpers (no GPU): calendar date keys, the
flight-3 seven-day window across a month end, the packed flight payloads
and the served Q1.1 template's value domains."""
import numpy as np
import pytest

from paper_2003_01178_amd import datagen


def test_date_keys_follow_the_calendar():
    keys, years = datagen.day_keys()
    assert keys[0] == 19920101 and keys[59] == 19920229 and keys[60] == 19920301   # 1992 is a leap year
    assert keys[-1] == 19981230 and years[-1] == 1998
    for i in (0, 59, 365, 1000, 2555):
        y, m, d = keys[i] // 10000, keys[i] // 100 % 100, keys[i] % 100
        assert datagen.date_key(y, m, d) == keys[i]
        if i + 6 < keys.size:
            assert datagen.date_key(y, m, d, plus_days=6) == keys[i + 6]


def test_flight3_window_is_seven_days_across_a_month_end():
    queries = pytest.importorskip("paper_2003_01178_amd.queries")
    (lo, hi), _, _ = queries.q1x_consts(3, year=1997, month=12, day=27)
    assert (lo, hi) == (19971227, 19980102)
    keys, _ = datagen.day_keys()
    assert int(np.sum((keys >= lo) & (keys <= hi))) == 7


def test_packed_payload_fields():
    dims, _ = datagen.star_dims(workload=3)
    for j, d in enumerate(dims):
        p = datagen.packed_payload(d, j).astype(np.int64)
        assert np.array_equal(p >> datagen.PACK_FILTER_SHIFT, d.filter)
        want_group = d.year - datagen.FIRST_YEAR if j == 0 else d.group
        assert np.array_equal(p & 0x3FF, want_group)


def test_banded_table_bands():
    t, spec, kinds = datagen.banded_star_tables(8 * 4096 + 100, band_rows=4096, workload=5, p_dense=0.5,
                                                p_sparse=0.3)
    d0, d1 = t.dims[0], t.dims[1]
    f1 = dict(zip(d1.key.tolist(), d1.filter.tolist()))
    f0 = dict(zip(d0.key.tolist(), d0.filter.tolist()))
    y0 = dict(zip(d0.key.tolist(), d0.year.tolist()))
    for b, kind in enumerate(kinds):
        lo, hi = b * 4096, min(t.n, (b + 1) * 4096)
        if kind == datagen.BAND_DENSE:
            assert all(f1[k] == spec.c1 for k in t.fk[1][lo:hi].tolist())
            assert all(f0[k] == spec.c0 and y0[k] == spec.year for k in t.fk[0][lo:hi].tolist())
            disc = t.extra["discount"][lo:hi]
            assert disc.min() >= spec.disc_lo and disc.max() <= spec.disc_lo + 2
    assert t.extra["discount"].max() <= 15 and t.extra["quantity"].min() >= 0
