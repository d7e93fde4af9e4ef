"""GPU parity of the operator calls (select, project, hash build/probe,
group-by) against the CPU oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import oracle
from helpers import announce, project_close
from paper_2003_01178_amd import crystal as cx
from paper_2003_01178_amd import datagen

pytestmark = pytest.mark.gpu
I32_MIN, I32_MAX = cx.I32_MIN, cx.I32_MAX
SIZES = [0, 1, 63, 64, 255, 4096, 4097, 3 * 4096 + 17, 100_003, 1_000_003]
SHAPES = [(64, 1), (128, 4), (256, 16), (1024, 16), (512, 2)]


@pytest.fixture(autouse=True)
def _reset_tuning():
    cx.tune_reset()
    yield
    cx.tune_reset()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


# ------------------------------------------------------------------ select --
def check_select(got_out, got_count, y, lo, hi, stable):
    want = oracle.select(y, lo, hi)
    c = int(got_count.item())
    assert c == want.size
    got = got_out[:c].cpu().numpy()
    if stable:
        assert np.array_equal(got, want)                 # input order, element by element
    else:
        # tiles land in reservation order: the multiset is unique, the order is not
        assert np.array_equal(np.sort(got), np.sort(want))


@pytest.mark.parametrize("stable", [False, True])
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("sigma", [0.0, 0.1, 0.5, 1.0])
def test_select_matches_oracle(n, sigma, stable):
    announce("select", n, sigma, stable)
    y = datagen.select_column(n, workload=1000 + n)
    lo, hi = datagen.select_threshold_range(sigma)
    out, cnt = cx.select(dev(y), lo, hi, stable=stable)
    check_select(out, cnt, y, lo, hi, stable)


@pytest.mark.parametrize("block,ipt", SHAPES)
def test_select_tile_shapes(block, ipt):
    announce("select shape", block, ipt)
    for stable in (False, True):
        cx.tune_set(cx.K_SELECT, block, ipt, 0)
        n = 3 * block * ipt + 5
        y = datagen.select_column(n, workload=7)
        out, cnt = cx.select(dev(y), 0, 2 ** 30, stable=stable)
        check_select(out, cnt, y, 0, 2 ** 30, stable)


@pytest.mark.parametrize("shape", [(512, 16, 1), (256, 8, 1)])
@pytest.mark.parametrize("sigma", [0.1, 0.5, 1.0])
def test_select_persistent_flushes(shape, sigma):
    """One workgroup per CU over 32M rows: each workgroup compacts many tiles
    (at least 16, asserted from the host) into its two-tile LDS buffer and
    reserves output space mid-loop whenever the buffer could not take
    another tile.  The output is compared with the oracle as a sorted
    multiset."""
    block, ipt, gpc = shape
    n = (1 << 25) + 12_345
    tiles = (n + block * ipt - 1) // (block * ipt)
    assert tiles / (gpc * torch.cuda.get_device_properties(0).multi_processor_count) >= 16
    announce("select persistent", shape, sigma)
    cx.tune_set(cx.K_SELECT, block, ipt, gpc)
    y = datagen.select_column(n, workload=2000)
    lo, hi = datagen.select_threshold_range(sigma)
    out, cnt = cx.select(dev(y), lo, hi)
    check_select(out, cnt, y, lo, hi, stable=False)


def test_select_unordered_keeps_tiles_contiguous():
    """Each tile's matches form one contiguous run: with every value
    matching, every aligned block of 1,024 outputs holds exactly one tile's
    values; within a tile the order is the documented slot-major one."""
    announce("select runs")
    cx.tune_set(cx.K_SELECT, 256, 4, 0)                  # 1024-item tiles
    n = 64 * 1024
    y = np.arange(n, dtype=np.int32)
    out, cnt = cx.select(dev(y), 0, n, stable=False)
    got = out[:int(cnt.item())].cpu().numpy()
    runs = got.reshape(-1, 1024)                         # every value matches: whole tiles
    srt = np.sort(runs, axis=1)
    assert np.all(np.diff(srt, axis=1) == 1) and np.all(srt[:, 0] % 1024 == 0)
    # within a tile: wave by wave, item slot by item slot, lane by lane (the
    # tile layout puts item (c, e) of thread t at offset (c * 256 + t) * 4 + e)
    want = np.array([(c * 256 + wv * 64 + ln) * 4 + e for wv in range(4) for c in range(1) for e in range(4)
                     for ln in range(64)])
    assert np.array_equal(runs[0] - runs[0].min(), want)
    assert np.array_equal(np.sort(got), y)


def test_select_tile_example_and_extremes():
    announce("select extremes")
    y = np.array([9, 2, 7, 8, 1, 3, 6, 12, 10, 0, 11, 4, 5, 14, 13, 15], dtype=np.int32)
    want = oracle.select(y, 6, I32_MAX).tolist()
    for stable in (False, True):
        out, cnt = cx.select(dev(y), 6, I32_MAX, stable=stable)
        assert int(cnt.item()) == 10
        got = out[:10].cpu().tolist()
        assert (got if stable else sorted(got)) == (want if stable else sorted(want))
    z = np.array([I32_MIN, -1, 0, 1, I32_MAX] * 1000, dtype=np.int32)
    for lo, hi in [(I32_MIN, I32_MAX), (I32_MIN, I32_MIN), (I32_MAX, I32_MAX), (0, 0), (5, 4)]:
        for stable in (False, True):
            out, cnt = cx.select(dev(z), lo, hi, stable=stable)
            check_select(out, cnt, z, lo, hi, stable)


def test_select_stable_is_deterministic():
    announce("select repeat")
    y = datagen.select_column(1 << 22, workload=5)
    x = dev(y)
    scratch = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    ref = None
    for _ in range(5):                       # the same scratch reused: the status words are cleared per call
        out, cnt = cx.select(x, I32_MIN, 2 ** 30, stable=True, scratch=scratch)
        s = out[:int(cnt.item())].cpu().numpy()
        ref = s if ref is None else ref
        assert np.array_equal(s, ref)
    assert np.array_equal(ref, oracle.select(y, I32_MIN, 2 ** 30))


# ----------------------------------------------------------------- project --
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("sigmoid", [False, True])
def test_project_matches_oracle(n, sigmoid):
    announce("project", n, sigmoid)
    x1, x2 = datagen.project_columns(n, workload=300 + n)
    got = cx.project(dev(x1), dev(x2), 2.0, 3.0, sigmoid=sigmoid).cpu().numpy()
    if sigmoid:
        want = oracle.project_sigmoid(x1, x2, 2.0, 3.0)
        assert np.all(np.abs(got.astype(np.float64) - want) <= 1e-6 * np.abs(want))
    else:
        want = oracle.project(x1, x2, 2.0, 3.0)
        assert project_close(got, want, x1, x2, 2.0, 3.0)


def test_project_exact_grid_and_signs():
    announce("project exact")
    rng = np.random.default_rng(1)
    i1, i2 = rng.integers(0, 2 ** 20, 100_000), rng.integers(0, 2 ** 20, 100_000)
    x1, x2 = (i1 / 2 ** 20).astype(np.float32), (i2 / 2 ** 20).astype(np.float32)
    got = cx.project(dev(x1), dev(x2), 2.0, 3.0).cpu().numpy()
    assert np.array_equal(got, oracle.project(x1, x2, 2.0, 3.0))      # exact in fp32
    for a, b in [(-1.5, 0.25), (3.0, -2.0), (0.0, 0.0)]:
        got = cx.project(dev(x1), dev(x2), a, b).cpu().numpy()
        assert project_close(got, oracle.project(x1, x2, a, b), x1, x2, a, b)


@pytest.mark.parametrize("block,ipt", [(64, 4), (128, 8), (1024, 16)])
def test_project_tile_shapes(block, ipt):
    announce("project shape", block, ipt)
    cx.tune_set(cx.K_PROJECT, block, ipt, 1)
    x1, x2 = datagen.project_columns(5 * block * ipt + 3, workload=4)
    got = cx.project(dev(x1), dev(x2), 2.0, 3.0).cpu().numpy()
    assert project_close(got, oracle.project(x1, x2, 2.0, 3.0), x1, x2, 2.0, 3.0)


# -------------------------------------------------------------- hash join --
@pytest.mark.parametrize("d", [1, 100, 1 << 13, 1 << 16, 1 << 20])
@pytest.mark.parametrize("kind", [cx.HT_LINEAR, cx.HT_DIRECT])
def test_join_matches_oracle(d, kind):
    announce("join", d, kind)
    t = datagen.join_tables(d, n_probe=1_000_003, workload=2000 + d)
    ht = cx.HashTable(kind, d, 0, d - 1)
    st = ht.build(dev(t.dim_key), payload=dev(t.dim_val))
    res = ht.probe(dev(t.fk)).cpu().tolist()
    cx.check_status(st)
    assert tuple(res) == oracle.join_sum(t.dim_key, t.dim_val, t.fk)
    assert res[1] == t.fk.size                                    # every probe key exists
    # Q4 form with a probe-side payload
    pv = np.arange(t.fk.size, dtype=np.int32) - 500_000
    res = ht.probe(dev(t.fk), dev(pv)).cpu().tolist()
    assert tuple(res) == oracle.join_sum(t.dim_key, t.dim_val, t.fk, pval=pv)


@pytest.mark.parametrize("kind", [cx.HT_LINEAR, cx.HT_DIRECT])
def test_join_filtered_build_misses_and_keys_only(kind):
    announce("join filtered", kind)
    rng = np.random.default_rng(4)
    d = 50_000
    key = (rng.permutation(d) * 3 - 70_000).astype(np.int32)      # sparse, negative keys
    val = rng.integers(I32_MIN, I32_MAX, size=d, dtype=np.int32, endpoint=True)
    filt = rng.integers(0, 25, size=d, dtype=np.int32)
    fk = rng.integers(-80_000, 90_000, size=333_333, dtype=np.int32)   # many misses
    ht = cx.HashTable(kind, d, int(key.min()), int(key.max()))
    st = ht.build(dev(key), dev(val), filter_col=dev(filt), filter=(3, 9))
    res = ht.probe(dev(fk)).cpu().tolist()
    cx.check_status(st)
    assert tuple(res) == oracle.join_sum(key, val, fk, bfilter=filt, flo=3, fhi=9)
    ko = cx.HashTable(kind, d, int(key.min()), int(key.max()), has_payload=False)
    st = ko.build(dev(key))
    res = ko.probe(dev(fk)).cpu().tolist()
    cx.check_status(st)
    assert tuple(res) == oracle.join_sum(key, None, fk)


def test_join_empty_inputs():
    announce("join empty")
    ht = cx.HashTable(cx.HT_LINEAR, 10)
    st = ht.build(dev(np.zeros(0, np.int32)), dev(np.zeros(0, np.int32)))
    assert ht.probe(dev(np.arange(100, dtype=np.int32))).cpu().tolist() == [0, 0]
    assert ht.probe(dev(np.zeros(0, np.int32))).cpu().tolist() == [0, 0]
    cx.check_status(st)


def test_join_device_errors():
    announce("join errors")
    ht = cx.HashTable(cx.HT_LINEAR, 8)
    st = ht.build(dev(np.array([1, 2, 3, 2], np.int32)), dev(np.arange(4, dtype=np.int32)))
    assert int(st.item()) == cx.EDUPKEY
    st = ht.build(dev(np.array([1, I32_MIN], np.int32)), dev(np.arange(2, dtype=np.int32)))
    assert int(st.item()) == cx.EINVAL
    full = cx.HashTable(cx.HT_LINEAR, 8)                           # 64 slots
    st = full.build(dev(np.arange(65, dtype=np.int32)), dev(np.arange(65, dtype=np.int32)))
    assert int(st.item()) == cx.EFULL
    dt = cx.HashTable(cx.HT_DIRECT, 0, 0, 99)
    st = dt.build(dev(np.array([5, 100], np.int32)), dev(np.arange(2, dtype=np.int32)))
    assert int(st.item()) == cx.ERANGE
    st = dt.build(dev(np.array([5, 6, 5], np.int32)), dev(np.arange(3, dtype=np.int32)))
    assert int(st.item()) == cx.EDUPKEY


# ---------------------------------------------------------------- group-by --
@pytest.mark.parametrize("groups", [1, 7, 7000, 100_000])
@pytest.mark.parametrize("n", [0, 1, 4097, 2_000_003])
def test_groupby_matches_oracle(groups, n):
    announce("groupby", groups, n)
    rng = np.random.default_rng(groups + n)
    g = rng.integers(0, groups, size=n, dtype=np.int32)
    v = rng.integers(I32_MIN, I32_MAX, size=n, dtype=np.int32, endpoint=True)
    sums, st = cx.groupby_agg(dev(g), dev(v), groups)
    got = sums.cpu().numpy()
    cx.check_status(st)
    assert np.array_equal(got, oracle.groupby(g, v, groups))


def test_groupby_lds_path_and_range_error():
    announce("groupby lds")
    n, groups = 40_000_000, 64                    # enough rows per group for LDS partials
    g = (np.arange(n) % groups).astype(np.int32)
    v = np.arange(n, dtype=np.int32)
    sums, st = cx.groupby_agg(dev(g), dev(v), groups)
    cx.check_status(st)
    assert np.array_equal(sums.cpu().numpy(), oracle.groupby(g, v, groups))
    g[123] = groups
    sums, st = cx.groupby_agg(dev(g), dev(v), groups)
    assert int(st.item()) == cx.ERANGE
    g[123] = 0
    want = oracle.groupby(g, v, groups)
    want[0] -= 123                                 # the skipped row (v = 123, group 0 in g)
    assert np.array_equal(sums.cpu().numpy(), want)


# ------------------------------------------------------------ batch build --
def test_build_batch_matches_single_builds():
    """crystal_ht_build_batch leaves every table byte-identical to its own
    crystal_ht_build (direct tables with and without payload and filter, and
    linear-probing tables), including a table with zero build rows."""
    announce("build batch")
    rng = np.random.default_rng(11)
    specs = []
    for kind, n, span, payload, filt in [(cx.HT_DIRECT, 2556, 5000, True, True),
                                         (cx.HT_DIRECT, 40_000, 40_000, False, True),
                                         (cx.HT_LINEAR, 200_000, 0, True, False),
                                         (cx.HT_LINEAR, 3_000, 0, False, True),
                                         (cx.HT_DIRECT, 0, 64, True, False)]:
        if kind == cx.HT_DIRECT:
            keys = rng.permutation(span)[:n].astype(np.int32) + 17
            lo, hi = 17, 17 + span - 1
        else:
            keys = rng.choice(2 ** 30, size=n, replace=False).astype(np.int32)
            lo, hi = 0, 0
        pay = rng.integers(-2 ** 31, 2 ** 31 - 1, size=n, dtype=np.int32) if payload else None
        flt = rng.integers(0, 25, size=n, dtype=np.int32) if filt else None
        specs.append((kind, keys, lo, hi, pay, flt))
    singles, batch_tables, items = [], [], []
    for kind, keys, lo, hi, pay, flt in specs:
        a = cx.HashTable(kind, max(len(keys), 1), lo, hi, has_payload=pay is not None)
        b = cx.HashTable(kind, max(len(keys), 1), lo, hi, has_payload=pay is not None)
        a.mem.fill_(0x5A)
        b.mem.fill_(0x5A)          # payload slots of absent keys are never written
        kd = dev(keys)
        pd = dev(pay) if pay is not None else None
        fd = dev(flt) if flt is not None else None
        rng_f = (3, 9) if flt is not None else (cx.I32_MIN, cx.I32_MAX)
        st = a.build(kd, payload=pd, filter_col=fd, filter=rng_f)
        cx.check_status(st)
        singles.append(a)
        batch_tables.append(b)
        items.append((b, kd, pd, fd, rng_f))
    st = cx.build_tables(items)
    cx.check_status(st)
    for a, b in zip(singles, batch_tables):
        n = a.nbytes
        if a.kind == cx.HT_DIRECT:
            assert torch.equal(a.mem[:n], b.mem[:n])     # bitmap and payloads: one place per key
        else:
            # linear probing places colliding keys in arrival order: compare the
            # set of occupied {key, payload} slots, which is unique
            sa, sb = (t.mem[:n].view(torch.int32).view(-1, 2).cpu().numpy() for t in (a, b))
            occ_a, occ_b = sa[sa[:, 0] != cx.I32_MIN], sb[sb[:, 0] != cx.I32_MIN]
            assert np.array_equal(occ_a[np.argsort(occ_a[:, 0])], occ_b[np.argsort(occ_b[:, 0])])
    with pytest.raises(cx.CrystalError):           # the same table twice
        cx.build_tables([items[0], items[0]])
