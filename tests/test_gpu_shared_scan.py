"""GPU parity of shared-scan batches: every query of a batch equals the CPU
oracle and its own single-query launch, over the whole table and over row
segments accumulated launch by launch."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from helpers import STAR_GROUPS, announce, q11_oracle, qmask_entries, star_oracle, star_oracle_joins
from paper_2003_01178_amd import crystal as cx
from paper_2003_01178_amd import datagen, queries

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def serving():
    t = datagen.star_tables(n=1_000_003 + 1, workload=31, with_q11_columns=True)
    s = queries.StarSchema(t)
    return t, queries.ServingTemplates(s)


def q11_fact_of(t):
    return datagen.Q11Fact(datekey=t.fk[0], discount=t.extra["discount"], quantity=t.extra["quantity"],
                           price=t.extra["price"])


def zeros(n, k):
    return [torch.zeros(n, dtype=torch.int64, device="cuda") for _ in range(k)]


@pytest.mark.parametrize("nq", [1, 5, 16])
def test_star_batch_matches_oracle_and_single(serving, nq):
    announce("shared star", nq)
    t, sv = serving
    rng = np.random.default_rng(nq)
    consts = [datagen.random_star_constants(rng) for _ in range(nq)]
    sv.build_star_masks(consts)
    outs = zeros(STAR_GROUPS, nq)
    st = sv.run_star_batch(outs)
    cx.check_status(st)
    cx.check_status(sv.status)
    for q in range(nq):
        want, _ = star_oracle(t, consts[q])
        got = outs[q].cpu().numpy()
        assert np.array_equal(got, want), (q, consts[q])
    single = sv.single_star(consts[0]).cpu().numpy()
    assert np.array_equal(single, outs[0].cpu().numpy())


def test_star_batch_segments_accumulate(serving):
    announce("shared star segments")
    t, sv = serving
    rng = np.random.default_rng(99)
    consts = [datagen.random_star_constants(rng) for _ in range(16)]
    sv.build_star_masks(consts)
    outs = zeros(STAR_GROUPS, 16)
    n = sv.n_rows
    bounds = [0, 4 * 33_333, 4 * 150_001, n]
    for lo, hi in zip(bounds[:-1], bounds[1:]):
        cx.check_status(sv.run_star_batch(outs, lo, hi))
    for q in range(16):
        assert np.array_equal(outs[q].cpu().numpy(), star_oracle(t, consts[q])[0]), q


@pytest.mark.parametrize("nq", [1, 16])
def test_q11_batch_matches_oracle(serving, nq):
    announce("shared q11", nq)
    t, sv = serving
    f = q11_fact_of(t)
    rng = np.random.default_rng(1000 + nq)
    consts = [datagen.random_q11_constants(rng) for _ in range(nq)]
    outs = zeros(1, nq)
    for lo, hi in [(0, 4 * 100_000), (4 * 100_000, sv.n_rows)]:
        cx.check_status(sv.run_q11_batch(consts, outs, lo, hi))
    for q, (year, d, qm) in enumerate(consts):
        assert int(outs[q].item()) == q11_oracle(f, year, (d, d + 2), qm), (q, consts[q])
    y, d, qm = consts[0]
    assert int(sv.single_q11(y, d, qm).item()) == int(outs[0].item())


def test_qmask_table_bits(serving):
    """Entry k holds bit q exactly when the row with key k passes query q."""
    announce("qmask bits")
    t, sv = serving
    d = t.dims[1]
    ranges = [(0, 0), (3, 7), (24, 24), (0, 24), (5, 4)]
    st = sv.masks[1].build(sv.s.dims[1]["key"], sv.s.dims[1]["filter"], ranges)
    cx.check_status(st)
    raw = sv.masks[1].mem[: 2 * sv.masks[1].c.span].view(torch.int16).cpu().numpy().astype(np.uint16)
    want = np.zeros(sv.masks[1].c.span, dtype=np.uint16)
    for q, (lo, hi) in enumerate(ranges):
        keep = (d.filter >= lo) & (d.filter <= hi)
        want[d.key[keep] - d.key.min()] |= np.uint16(1 << q)
    assert np.array_equal(raw, want)


# ---------------------------------------------------- rank-compressed masks --
def test_date_mask_is_ranked_and_matches_plain(serving):
    """The date dimension's keys fill 2,556 of a 61,130-key span: its table is
    rank-compressed, and reads, key by key, like the plain table."""
    announce("qmask ranked dense")
    t, sv = serving
    d = sv.s.dims[0]
    assert sv.masks[0].ranked == d["n"]
    assert sv.masks[1].ranked == 0                       # dense key domain: plain table
    plain = cx.QueryMask(d["key_min"], d["key_max"], keys=d["key"], ranked=False)
    ranges = [(c, c) for c in range(16)]
    cx.check_status(sv.masks[0].build(d["key"], d["filter"], ranges))
    cx.check_status(plain.build(d["key"], d["filter"], ranges))
    got = qmask_entries(sv.masks[0])
    assert np.array_equal(got, qmask_entries(plain))
    dim = t.dims[0]
    want = np.zeros(plain.c.span, dtype=np.int64)
    for q, (lo, hi) in enumerate(ranges):
        keep = (dim.filter >= lo) & (dim.filter <= hi)
        want[dim.key[keep] - dim.key.min()] |= 1 << q
    assert np.array_equal(got, want)


def plain_scan(sv, template, dims):
    masks = [cx.QueryMask(d["key_min"], d["key_max"], keys=d["key"], ranked=False) for d in dims]
    return cx.SharedScan(template, masks), masks


@pytest.mark.parametrize("block,ipt", [(64, 4), (256, 8), (1024, 16)])
def test_ranked_and_plain_batches_agree(serving, block, ipt):
    """64-thread workgroups leave the ranked date table in global memory
    (staging it would cut below eight waves per CU); larger ones stage it."""
    announce("shared ranked vs plain", block, ipt)
    t, sv = serving
    cx.tune_set(cx.K_SHARED_SCAN, block, ipt, 0)
    try:
        rng = np.random.default_rng(block + ipt)
        consts = [datagen.random_star_constants(rng) for _ in range(16)]
        sv.build_star_masks(consts)
        outs = zeros(STAR_GROUPS, 16)
        cx.check_status(sv.run_star_batch(outs))
        dims = [sv.s.dims[j] for j in queries.DEFAULT_JOIN_ORDER]
        scan, masks = plain_scan(sv, sv.star_template, dims)
        for m, d, j in zip(masks, dims, queries.DEFAULT_JOIN_ORDER):
            cx.check_status(m.build(d["key"], d["filter"], [(c[j], c[j]) for c in consts]))
        ref = zeros(STAR_GROUPS, 16)
        cx.check_status(scan.run([[] for _ in ref], ref))
        for q in range(16):
            assert torch.equal(outs[q], ref[q]), q
        for q in (0, 15):
            assert np.array_equal(outs[q].cpu().numpy(), star_oracle(t, consts[q])[0]), q
        f = q11_fact_of(t)
        qc = [datagen.random_q11_constants(rng) for _ in range(16)]
        qo = zeros(1, 16)
        cx.check_status(sv.run_q11_batch(qc, qo))
        for q in (0, 7, 15):
            y, dl, qm = qc[q]
            assert int(qo[q].item()) == q11_oracle(f, y, (dl, dl + 2), qm), (q, qc[q])
    finally:
        cx.tune_reset()
    cx.check_status(sv.status)


def ranked_table(span, ranked, key_min=0):
    lib = cx.load()
    c = cx.QmaskTableC()
    c.span, c.key_min, c.ranked = span, key_min, ranked
    mem = torch.zeros(max(16, lib.crystal_qmask_ranked_bytes(span, ranked)), dtype=torch.uint8, device="cuda")
    c.mem = mem.data_ptr()
    return c, mem


def rank(c, keys):
    lib = cx.load()
    st = cx.new_status()
    k = torch.tensor(keys, dtype=torch.int32, device="cuda")
    assert lib.crystal_qmask_rank(ctypes.byref(c), cx._ptr(k), k.numel(), cx._ptr(st), cx._stream()) == cx.OK
    torch.cuda.synchronize()
    return int(st.item())


def test_qmask_rank_directory_and_errors():
    announce("qmask rank errors")
    lib = cx.load()
    c, mem = ranked_table(100, 8, key_min=1000)
    assert rank(c, [1000, 1031, 1032, 1099, 1031]) == cx.OK     # a duplicate counts once
    words = mem[:8 * 5].view(torch.int32).view(-1, 2).cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    assert list(words[:, 0]) == [1 | (1 << 31), 1, 0, 1 << 3, 0]     # presence bits per 32 keys
    assert list(words[:, 1]) == [0, 2, 3, 3, 4]                       # keys present before each entry
    # build: the entry of a key absent from the directory is an error
    st = cx.new_status()
    k = torch.tensor([1000, 1099, 1001], dtype=torch.int32, device="cuda")
    rs = (cx.Range * 1)(cx.Range(0, 0))
    assert lib.crystal_qmask_build(ctypes.byref(c), cx._ptr(k), None, 3, rs, 1, cx._ptr(st), cx._stream()) == cx.OK
    torch.cuda.synchronize()
    assert int(st.item()) == cx.ERANGE
    c2, _ = ranked_table(64, 2)
    assert rank(c2, [0, 5, 9]) == cx.EFULL                        # three keys, room for two
    c3, _ = ranked_table(64, 8)
    assert rank(c3, [0, 64]) == cx.ERANGE                          # 64 is past the span


def test_qmask_build_batch_matches_single_builds(serving):
    """One batched build of every join's table (a ranked date table among
    plain ones) leaves the same tables as one build per table."""
    announce("qmask build batch")
    t, sv = serving
    dims = sv.s.dims
    rng = np.random.default_rng(7)
    ranges = [[(int(a), int(a) + int(w)) for a, w in zip(rng.integers(0, 25, 16), rng.integers(0, 3, 16))]
              for _ in dims]
    single = [cx.QueryMask(d["key_min"], d["key_max"], keys=d["key"]) for d in dims]
    for m, d, r in zip(single, dims, ranges):
        cx.check_status(m.build(d["key"], d["filter"], r))
    batched = [cx.QueryMask(d["key_min"], d["key_max"], keys=d["key"]) for d in dims]
    # dirty the batched tables first: the batch clears before it builds
    for m, d in zip(batched, dims):
        cx.check_status(m.build(d["key"], None, [(0, 0)] * 16))
    cx.check_status(cx.build_query_masks([(m, d["key"], d["filter"], r) for m, d, r in zip(batched, dims, ranges)]))
    assert batched[0].ranked > 0 and batched[1].ranked == 0
    for j, (a, b) in enumerate(zip(single, batched)):
        assert np.array_equal(qmask_entries(a), qmask_entries(b)), j
    # a key outside a table's span is reported, as by the single build
    d = dims[1]
    bad_keys = d["key"].clone()
    bad_keys[5] = d["key_max"] + 1
    st = cx.build_query_masks([(batched[1], bad_keys, d["filter"], ranges[1])])
    torch.cuda.synchronize()
    assert int(st.item()) == cx.ERANGE


def test_ranked_table_wide_span():
    """A ranked table over a 2^24-key span (65,536 directory entries, ranked
    by one workgroup) reads like the plain table, key by key."""
    announce("qmask ranked wide span")
    rng = np.random.default_rng(11)
    span = 1 << 24
    keys = np.unique(rng.integers(0, span, 5000)).astype(np.int32) + 1000
    rng.shuffle(keys)
    filt = rng.integers(0, 10, keys.size).astype(np.int32)
    kd, fd = torch.from_numpy(keys).cuda(), torch.from_numpy(filt).cuda()
    ranges = [(q % 10, q % 10 + q // 10) for q in range(16)]
    ranked = cx.QueryMask(1000, 1000 + span - 1, keys=kd, ranked=True)
    plain = cx.QueryMask(1000, 1000 + span - 1, keys=kd, ranked=False)
    cx.check_status(ranked.status)
    assert ranked.ranked == keys.size
    cx.check_status(ranked.build(kd, fd, ranges))
    cx.check_status(plain.build(kd, fd, ranges))
    got = qmask_entries(ranked)
    assert np.array_equal(got, qmask_entries(plain))
    want = np.zeros(keys.size, dtype=np.int64)
    for q, (lo, hi) in enumerate(ranges):
        want |= ((filt >= lo) & (filt <= hi)).astype(np.int64) << q
    assert np.array_equal(got[keys.astype(np.int64) - 1000], want)


@pytest.mark.parametrize("nq", [3, 16])
def test_batch_with_fact_predicates(serving, nq):
    """A template with three fact predicates ahead of the four joins: the
    predicate steps run over whole tiles, and, with few queries, the third
    predicate and the joins also from the queue of sparse rows."""
    announce("shared preds", nq)
    t, sv = serving
    joins = []
    for j in queries.DEFAULT_JOIN_ORDER:
        jj = dict(table=sv.tables[j], fk_col=j)
        if j == 0:
            jj["group"] = (32, 0, datagen.FIRST_YEAR, queries.GROUPS_PER_YEAR)
        if j == 2:
            jj["group"] = (32, 0, 0, 1)
        joins.append(jj)
    # fact columns: 0-3 keys, 4-5 measures, 6 discount, 7 quantity, 8 price
    template = cx.StarQuery(sv.cols, n_groups=STAR_GROUPS, preds=[(6, 0, 0), (7, 0, 0), (5, 0, 0)],
                            joins=joins, agg=cx.AGG_SUM, agg_cols=(4, 0))
    scan = cx.SharedScan(template, [sv.masks[j] for j in queries.DEFAULT_JOIN_ORDER])
    rng = np.random.default_rng(300 + nq)
    consts = [datagen.random_star_constants(rng) for _ in range(nq)]
    # narrow discount and quantity ranges keep few rows alive for few queries
    preds = []
    for _ in range(nq):
        d = int(rng.integers(0, 11))
        qlo = int(rng.integers(1, 46))
        m2lo = int(rng.integers(1, 500_000))
        preds.append([(d, d), (qlo, qlo + 4), (m2lo, m2lo + 500_000)])
    sv.build_star_masks(consts)
    outs = zeros(STAR_GROUPS, nq)
    cx.check_status(scan.run(preds, outs))
    cols = [*t.fk, t.m1, t.m2, t.extra["discount"], t.extra["quantity"], t.extra["price"]]
    for q in range(nq):
        want = oracle.star(cols, STAR_GROUPS, preds=[(6, *preds[q][0]), (7, *preds[q][1]), (5, *preds[q][2])],
                           joins=star_oracle_joins(t, consts[q]), agg=oracle.AGG_SUM, agg_cols=(4, 0))
        assert np.array_equal(outs[q].cpu().numpy(), want), q


@pytest.mark.parametrize("block,ipt", [(64, 4), (1024, 16)])
def test_ranked_table_in_a_late_join(serving, block, ipt):
    """Join order (1, 2, 0, 3) puts the ranked date table third, where rows
    are sparse: it is read from the queue of sparse rows, in LDS (1024-thread
    workgroups stage it) or in global memory (64-thread ones do not)."""
    announce("shared late ranked join", block, ipt)
    t, sv = serving
    order = (1, 2, 0, 3)
    joins = []
    for j in order:
        jj = dict(table=sv.tables[j], fk_col=j)
        if j == 0:
            jj["group"] = (32, 0, datagen.FIRST_YEAR, queries.GROUPS_PER_YEAR)
        if j == 2:
            jj["group"] = (32, 0, 0, 1)
        joins.append(jj)
    template = cx.StarQuery(sv.cols, n_groups=STAR_GROUPS, joins=joins, agg=cx.AGG_SUM, agg_cols=(4, 0))
    assert sv.masks[0].ranked > 0
    scan = cx.SharedScan(template, [sv.masks[j] for j in order])
    cx.tune_set(cx.K_SHARED_SCAN, block, ipt, 0)
    try:
        rng = np.random.default_rng(block)
        consts = [datagen.random_star_constants(rng) for _ in range(8)]
        sv.build_star_masks(consts)
        outs = zeros(STAR_GROUPS, 8)
        cx.check_status(scan.run([[] for _ in outs], outs))
        for q in range(8):
            assert np.array_equal(outs[q].cpu().numpy(), star_oracle(t, consts[q])[0]), q
    finally:
        cx.tune_reset()
