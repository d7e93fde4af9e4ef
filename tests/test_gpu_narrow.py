"""Compressed fact columns in the fused star kernel: narrow (frame-of-reference
uint8 / uint16) and bit-packed (1-16 bits per value, frame of reference)
columns, against the oracle on the same values as int32."""
import numpy as np
import pytest
import torch

import oracle
from helpers import STAR_GROUPS, announce, q11_oracle, star_oracle, star_oracle_joins
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


@pytest.mark.parametrize("width", [1, 2])
@pytest.mark.parametrize("n", [0, 1, 4097, 1_000_003])
def test_pack_column_round_trip(width, n):
    announce("pack", width, n)
    rng = np.random.default_rng(n + width)
    top = (1 << (8 * width)) - 1
    base = -1000
    x = (rng.integers(0, top + 1, size=n, dtype=np.int64) + base).astype(np.int32)
    col, st = cx.pack_column(dev(x), base, width)
    cx.check_status(st)
    got = col.data.cpu().numpy().view(np.uint8 if width == 1 else np.uint16).astype(np.int64)
    assert np.array_equal(got + base, x.astype(np.int64))


def test_pack_column_out_of_range():
    announce("pack erange")
    x = np.array([5, 6, 300, 7, 4], dtype=np.int32)       # 300 > 5 + 255, 4 < 5
    col, st = cx.pack_column(dev(x), 5, 1)
    assert int(st.item()) == cx.ERANGE
    got = col.data.cpu().numpy()
    assert got[0] == 0 and got[1] == 1 and got[3] == 2
    with pytest.raises(cx.CrystalError):
        cx.pack_column(dev(x), 0, 3)


@pytest.fixture(scope="module")
def star_small():
    t = datagen.star_tables(n=1_000_003, workload=3)
    return t, queries.StarSchema(t)


def narrow_star_cols(t, s):
    """fk0 (date keys) and fk1 (0..39999) as 16-bit offsets; the rest int32."""
    fk0, st0 = cx.pack_column(s.fk[0], int(t.dims[0].key.min()), 2)
    fk1, st1 = cx.pack_column(s.fk[1], 0, 2)
    cx.check_status(st0)
    cx.check_status(st1)
    return [fk0, fk1, s.fk[2], s.fk[3], s.m1, s.m2]


@pytest.mark.parametrize("order", [(1, 0, 2, 3), (0, 1, 2, 3), (2, 3, 1, 0), (3, 1, 2, 0)])
def test_star_with_narrow_keys_matches_oracle(star_small, order):
    """Narrow columns in the dense steps (first two joins) and in the sparse
    steps and group fields (later joins), per join order."""
    announce("narrow star", order)
    t, s = star_small
    s.status.zero_()
    s.build()
    cols = narrow_star_cols(t, s)
    plan = s.plan(order)
    q = cx.StarQuery(cols, n_groups=STAR_GROUPS, joins=plan.joins, agg=cx.AGG_SUM, agg_cols=(4, 0))
    out, st = q.run()
    cx.check_status(st)
    want, _ = star_oracle(t)
    assert np.array_equal(out.cpu().numpy(), want)


def test_narrow_measures_and_predicates(star_small):
    """A narrow measure (m1 mod 50,000 as uint16) and a narrow predicate column
    through every aggregate, grouped and scalar."""
    announce("narrow measures")
    t, s = star_small
    s.status.zero_()
    s.build()
    m1s = (t.m1 % 50_000).astype(np.int32)
    m2b = (t.m2 % 200 + 7).astype(np.int32)
    c_m1, st1 = cx.pack_column(dev(m1s), 0, 2)
    c_m2, st2 = cx.pack_column(dev(m2b), 7, 1)
    cx.check_status(st1)
    cx.check_status(st2)
    cols = narrow_star_cols(t, s)[:4] + [c_m1, c_m2]
    preds = [(5, 20, 150)]
    for agg in (cx.AGG_SUM, cx.AGG_SUM_PRODUCT, cx.AGG_SUM_DIFF, cx.AGG_COUNT):
        joins = [dict(table=s.tables[j], fk_col=j, group=(32, 0, 1992, 1000) if j == 0 else (32, 0, 0, 1))
                 for j in (0, 2)]
        q = cx.StarQuery(cols, n_groups=STAR_GROUPS, preds=preds, joins=joins, agg=agg, agg_cols=(4, 5))
        out, st = q.run()
        cx.check_status(st)
        oj = [jj for jj in star_oracle_joins(t, t.consts) if jj["fk_col"] in (0, 2)]
        want = oracle.star([*t.fk, m1s, m2b], STAR_GROUPS, preds=preds, joins=oj, agg=agg, agg_cols=(4, 5))
        assert np.array_equal(out.cpu().numpy(), want), agg
        qs = cx.StarQuery(cols, n_groups=1, preds=preds, joins=[dict(table=s.tables[2], fk_col=2)], agg=agg,
                          agg_cols=(4, 5))
        out, st = qs.run()
        cx.check_status(st)
        oj1 = [dict(jj, group=None) for jj in oj if jj["fk_col"] == 2]
        want1 = oracle.star([*t.fk, m1s, m2b], 1, preds=preds, joins=oj1, agg=agg, agg_cols=(4, 5))
        assert int(out.item()) == int(want1[0]), agg


@pytest.mark.parametrize("n", [4097, 3_000_001])
def test_q11_narrow_matches_oracle(n):
    """Q1.1 over datekey (uint16 from 1992-01-01), discount and quantity
    (uint8) and int32 price: 7 bytes per row instead of 16."""
    announce("narrow q11", n)
    f = datagen.q11_fact(n, workload=90 + n % 7)
    dk, s0 = cx.pack_column(dev(f.datekey), 19920101, 2)
    disc, s1 = cx.pack_column(dev(f.discount), 0, 1)
    qty, s2 = cx.pack_column(dev(f.quantity), 1, 1)
    for st in (s0, s1, s2):
        cx.check_status(st)
    for year, d, q in [(1994, 1, 24), (1992, 0, 50), (1998, 8, 2)]:
        plan = queries.Q11Plan(dk, disc, qty, dev(f.price), year=year, disc=(d, d + 2), qty_max=q)
        out, st = plan.run()
        cx.check_status(st)
        assert int(out.item()) == q11_oracle(f, year, (d, d + 2), q)


def test_shared_scan_rejects_narrow_columns(star_small):
    announce("narrow shared scan")
    t, s = star_small
    cols = narrow_star_cols(t, s)
    tmpl = cx.StarQuery(cols, n_groups=1, preds=[(4, 0, 10)], agg=cx.AGG_COUNT)
    scan = cx.SharedScan(tmpl, [])
    outs = [torch.zeros(1, dtype=torch.int64, device="cuda")]
    with pytest.raises(cx.CrystalError) as e:
        scan.run([[(0, 5)]], outs)
    assert e.value.code == cx.EINVAL


# ------------------------------------------------------------ bit-packed ---
def decode_bits(words, n, bits, base):
    """Host decoder of the documented layout: an LSB-first stream of 32-bit
    words, row i's field at stream bits [i * bits, (i + 1) * bits)."""
    w = words.astype(np.uint64) & np.uint64(0xFFFFFFFF)
    off = np.arange(n, dtype=np.uint64) * np.uint64(bits)
    q = (off >> np.uint64(5)).astype(np.int64)
    two = w[q] | (w[q + 1] << np.uint64(32))
    f = (two >> (off & np.uint64(31))) & np.uint64((1 << bits) - 1)
    return f.astype(np.int64) + base


@pytest.mark.parametrize("bits", [1, 2, 3, 5, 7, 8, 9, 11, 12, 13, 15, 16])
@pytest.mark.parametrize("n", [0, 1, 5, 4097, 1_000_003])
def test_pack_bits_round_trip(bits, n):
    announce("pack bits", bits, n)
    rng = np.random.default_rng(7 * n + bits)
    base = -123_456
    x = (rng.integers(0, 1 << bits, size=n, dtype=np.int64) + base).astype(np.int32)
    col, st = cx.pack_column_bits(dev(x), base, bits)
    cx.check_status(st)
    words = col.data.cpu().numpy().view(np.uint32)
    n_words = (n * bits + 31) // 32
    assert words.size == n_words + 4 and not np.any(words[n_words:])      # four zero words of padding
    assert np.array_equal(decode_bits(words, n, bits, base), x.astype(np.int64))


def test_pack_bits_out_of_range():
    announce("pack bits erange")
    x = np.array([10, 11, 10 + 63, 10 + 64, 9, 12], dtype=np.int32)       # 6 bits from 10: 74 and 9 are out
    col, st = cx.pack_column_bits(dev(x), 10, 6)
    assert int(st.item()) == cx.ERANGE
    got = decode_bits(col.data.cpu().numpy().view(np.uint32), 6, 6, 10)
    assert got[0] == 10 and got[1] == 11 and got[2] == 73 and got[5] == 12
    for bad in (0, 17):
        with pytest.raises(ValueError):
            cx.pack_column_bits(dev(x), 10, bad)


def bitpacked_star(t, s):
    """fk0 as 12-bit date codes (day index, with the date table keyed by code)
    and fk1 as 16-bit offsets; the rest int32.  Returns (cols, tables)."""
    codes, st0 = cx.pack_column_bits(dev(datagen.day_codes(t.fk[0])), 0, 12)
    fk1, st1 = cx.pack_column_bits(s.fk[1], 0, 16)
    cx.check_status(st0)
    cx.check_status(st1)
    d0 = s.dims[0]
    ht0 = cx.HashTable(cx.HT_DIRECT, d0["n"], 0, datagen.N_DAYS - 1, has_payload=True)
    ht0.build(dev(datagen.day_codes(t.dims[0].key)), payload=d0["year"], filter_col=d0["filter"],
              filter=(t.consts[0], t.consts[0]), status=s.status)
    tables = [ht0] + list(s.tables[1:])
    return [codes, fk1, s.fk[2], s.fk[3], s.m1, s.m2], tables


@pytest.mark.parametrize("order", [(1, 0, 2, 3), (0, 2, 1, 3), (2, 3, 1, 0), (3, 1, 0, 2)])
def test_star_with_bitpacked_keys_matches_oracle(star_small, order):
    """Both dense steps bit-packed (1, 0, ...), one bit-packed and one int32
    (0, 2, ...), and bit-packed keys in the sparse steps and group fields
    (2, 3, 1, 0), against the oracle on the original int32 date keys."""
    announce("bitpacked star", order)
    t, s = star_small
    s.status.zero_()
    s.build()
    cols, tables = bitpacked_star(t, s)
    joins = []
    for j in order:
        jj = dict(table=tables[j], fk_col=j)
        if j == 0:
            jj["group"] = (32, 0, datagen.FIRST_YEAR, queries.GROUPS_PER_YEAR)
        if j == 2:
            jj["group"] = (32, 0, 0, 1)
        joins.append(jj)
    for shape in [None, (256, 4, 0), (1024, 16, 2)]:
        cx.tune_reset()
        if shape:
            cx.tune_set(cx.K_STAR, *shape)
        q = cx.StarQuery(cols, n_groups=STAR_GROUPS, joins=joins, agg=cx.AGG_SUM, agg_cols=(4, 0))
        out, st = q.run()
        cx.check_status(st)
        cx.check_status(s.status)
        want, _ = star_oracle(t)
        assert np.array_equal(out.cpu().numpy(), want), (order, shape)


@pytest.mark.parametrize("n", [4097, 3_000_001])
def test_q11_bitpacked_matches_oracle(n):
    """Q1.1 over datekey (16 bits from 1992-01-01), discount (4 bits),
    quantity (6 bits from 1) and int32 price."""
    announce("bitpacked q11", n)
    f = datagen.q11_fact(n, workload=95 + n % 7)
    dk, s0 = cx.pack_column_bits(dev(f.datekey), 19920101, 16)
    disc, s1 = cx.pack_column_bits(dev(f.discount), 0, 4)
    qty, s2 = cx.pack_column_bits(dev(f.quantity), 1, 6)
    for st in (s0, s1, s2):
        cx.check_status(st)
    for year, d, q in [(1994, 1, 24), (1992, 0, 50), (1998, 8, 2)]:
        plan = queries.Q11Plan(dk, disc, qty, dev(f.price), year=year, disc=(d, d + 2), qty_max=q)
        out, st = plan.run()
        cx.check_status(st)
        assert int(out.item()) == q11_oracle(f, year, (d, d + 2), q)


@pytest.mark.parametrize("bits", list(range(1, 17)))
def test_bitpacked_predicates_every_width(bits):
    """Three range predicates over bit-packed columns of widths b, 17 - b and
    b (the first two are the dense steps, so every width runs through the
    four-row decode at every bit alignment; the third is read row by row),
    with bases that make the offsets span the whole width, then SUM(m):
    equal to the oracle on the int32 values."""
    announce("bitpacked predicates", bits)
    n = 100_003
    rng = np.random.default_rng(1000 + bits)
    widths = (bits, 17 - bits, bits)
    bases = [int(rng.integers(-(1 << 30), 1 << 30)) for _ in widths]
    cols = [(rng.integers(0, 1 << w, size=n, dtype=np.int64) + b).astype(np.int32) for w, b in zip(widths, bases)]
    m = rng.integers(-(1 << 20), 1 << 20, size=n, dtype=np.int64).astype(np.int32)
    packed = []
    for c, w, b in zip(cols, widths, bases):
        col, st = cx.pack_column_bits(dev(c), b, w)
        cx.check_status(st)
        packed.append(col)
    # each range keeps about three quarters of its column's values
    preds = []
    for k, (w, b) in enumerate(zip(widths, bases)):
        span = 1 << w
        lo = b + span // 8
        hi = b + span - 1 - span // 8
        preds.append((k, lo, hi))
    plan = cx.StarQuery([*packed, dev(m)], n_groups=1, preds=preds, agg=cx.AGG_SUM, agg_cols=(3, 0))
    out, st = plan.run()
    cx.check_status(st)
    want = oracle.star([*cols, m], 1, preds=preds, agg=oracle.AGG_SUM, agg_cols=(3, 0))
    assert int(out.item()) == int(want[0])
