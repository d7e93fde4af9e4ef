"""GPU parity of radix histogram, radix partition and the radix sorts (least
and most significant digit first; section 4.4) against the CPU oracle,
through the C ABI.  The stable partition and both sorts have a unique
output, compared element by element; the unstable partition is compared
per partition as a multiset."""
import numpy as np
import pytest
import torch

import oracle
from helpers import announce
from paper_2003_01178_amd import crystal as cx
from paper_2003_01178_amd import datagen

pytestmark = pytest.mark.gpu
SIZES = [0, 1, 63, 64, 4096, 4097, 3 * 4096 + 17, 100_003, 1_000_003]
DIGITS = [(0, 8), (8, 8), (24, 8), (4, 4), (28, 4), (0, 1), (31, 1), (13, 7)]


@pytest.fixture(autouse=True)
def _reset_tuning():
    cx.tune_reset()
    yield
    cx.tune_reset()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def u32(t, n):
    return t[:n].cpu().numpy().view(np.uint32)


def pairs(n, workload, key_bits=32):
    k, v = datagen.radix_pairs(n, workload=workload, key_bits=key_bits)
    return k.view(np.uint32), v.view(np.uint32)


# --------------------------------------------------------------- histogram --
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("shift,bits", DIGITS)
def test_histogram_matches_oracle(n, shift, bits):
    announce("radix histogram", n, shift, bits)
    k, _ = pairs(n, 500 + n)
    got = cx.radix_histogram(dev(k.view(np.int32)), shift, bits).cpu().numpy().view(np.uint32)
    want = oracle.radix_histogram(k, shift, bits)
    assert np.array_equal(got.astype(np.int64), want)


# --------------------------------------------------------------- partition --
def check_partition(k, v, shift, bits, with_vals, key_dev=None):
    n = k.size
    kd = dev(k.view(np.int32)) if key_dev is None else key_dev
    vd = dev(v.view(np.int32)) if with_vals else None
    ok, ov, offs = cx.radix_partition(kd, shift, bits, vals=vd)
    wk, wv = oracle.radix_partition(k, v, shift, bits)
    assert np.array_equal(u32(ok, n), wk)
    if with_vals:
        assert np.array_equal(u32(ov, n), wv)
    h = oracle.radix_histogram(k, shift, bits)
    want_offs = np.concatenate([[0], np.cumsum(h)])
    assert np.array_equal(offs.cpu().numpy().astype(np.int64), want_offs)


@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("shift,bits", DIGITS)
def test_partition_matches_oracle(n, shift, bits):
    announce("radix partition", n, shift, bits)
    k, v = pairs(n, 600 + n)
    check_partition(k, v, shift, bits, with_vals=True)


@pytest.mark.parametrize("n", [4097, 1_000_003])
def test_partition_keys_only(n):
    announce("radix partition keys only", n)
    k, v = pairs(n, 700 + n)
    check_partition(k, v, 8, 8, with_vals=False)


@pytest.mark.parametrize("case", ["all_equal", "two_values", "narrow", "sorted", "reversed"])
def test_partition_skewed(case):
    """Degenerate digit distributions: one digit for every key (a whole wave
    of equal digits), two digits, keys from a small domain, presorted input."""
    announce("radix partition skewed", case)
    n = 300_007
    rng = np.random.default_rng(3)
    if case == "all_equal":
        k = np.full(n, 0xABCDEF12, dtype=np.uint32)
    elif case == "two_values":
        k = np.where(rng.random(n) < 0.5, 0x00000005, 0xFF000005).astype(np.uint32)
    elif case == "narrow":
        k = rng.integers(0, 5, size=n, dtype=np.uint64).astype(np.uint32) << np.uint32(8)
    elif case == "sorted":
        k = np.arange(n, dtype=np.uint32) * np.uint32(7919)
        k.sort()
    else:
        k = (np.arange(n, dtype=np.uint64)[::-1] * 12345).astype(np.uint32)
    v = np.arange(n, dtype=np.uint32)
    for shift in (0, 8, 24):
        check_partition(k, v, shift, 8, with_vals=True)


@pytest.mark.parametrize("block,ipt", [(256, 4), (256, 8), (512, 16), (1024, 4), (1024, 8), (1024, 16)])
@pytest.mark.parametrize("gpc", [0, 1, 3])
def test_partition_tile_shapes(block, ipt, gpc):
    announce("radix partition shape", block, ipt, gpc)
    cx.tune_set(cx.K_RADIX, block, ipt, gpc)
    for n in (block * ipt * 5 + 3, 777_777):
        k, v = pairs(n, 800 + n)
        check_partition(k, v, 0, 8, with_vals=True)


def test_partition_tuned_shape_several_tiles_per_workgroup():
    """The tuned 1024 x 16 tile with one workgroup per CU: every workgroup
    walks three or four tiles of its chunk, so each wave clears and reuses
    its digit counters, and ranks a tile while other waves may still write
    out the previous one.  Element by element against the oracle, for a
    uniform and a two-digit key distribution."""
    cx.tune_set(cx.K_RADIX, 1024, 16, 1)
    n = 3 * 256 * 1024 * 16 + 5
    k, v = pairs(n, 850)
    announce("radix partition several tiles per workgroup", n)
    check_partition(k, v, 8, 8, with_vals=True)
    k2 = np.where(np.random.default_rng(851).random(n) < 0.5, 0x00000500, 0x0000FA00).astype(np.uint32)
    check_partition(k2, v, 8, 8, with_vals=True)


def test_partition_errors():
    announce("radix partition errors")
    k = dev(np.arange(1000, dtype=np.int32))
    lib = cx.load()
    for shift, bits in [(0, 0), (0, 9), (25, 8), (-1, 4)]:
        with pytest.raises(cx.CrystalError) as e:
            cx.radix_partition(k, shift, bits)
        assert e.value.code == cx.EINVAL
    with pytest.raises(cx.CrystalError) as e:      # output overlapping the input
        cx.radix_partition(k, 0, 8, out_keys=k)
    assert e.value.code == cx.EINVAL
    out = torch.empty_like(k)
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    rc = lib.crystal_radix_partition(cx._ptr(k), None, 1000, 0, 8, cx._ptr(out), None, None, cx._ptr(small), 16,
                                     cx._stream())
    assert rc == cx.ESCRATCH
    rc = lib.crystal_sort_pairs(cx._ptr(k), None, 1000, cx._ptr(out), None, cx._ptr(small), 16, cx._stream())
    assert rc == cx.ESCRATCH
    torch.cuda.synchronize()


# -------------------------------------------------------------------- sort --
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("key_bits", [32, 12])
def test_sort_matches_oracle(n, key_bits):
    """12-bit keys make long runs of equal keys: stability decides the values."""
    announce("radix sort", n, key_bits)
    k, v = pairs(n, 900 + n, key_bits=key_bits)
    ok, ov = cx.sort_pairs(dev(k.view(np.int32)), dev(v.view(np.int32)))
    wk, wv = oracle.sort_pairs(k, v)
    assert np.array_equal(u32(ok, n), wk)
    assert np.array_equal(u32(ov, n), wv)


def test_sort_keys_only_and_tile_shape():
    announce("radix sort keys only")
    n = 1_000_003
    k, _ = pairs(n, 77)
    want = np.sort(k)
    ok, ov = cx.sort_pairs(dev(k.view(np.int32)))
    assert ov is None and np.array_equal(u32(ok, n), want)
    cx.tune_set(cx.K_RADIX, 1024, 8, 1)
    ok, _ = cx.sort_pairs(dev(k.view(np.int32)))
    assert np.array_equal(u32(ok, n), want)


def test_sort_repeated_calls_share_scratch():
    """Two sorts through one scratch buffer, the second smaller."""
    announce("radix sort scratch reuse")
    lib = cx.load()
    n1, n2 = 500_001, 4097
    scratch = torch.empty(lib.crystal_sort_pairs_scratch_bytes(n1, 1), dtype=torch.uint8, device="cuda")
    for n in (n1, n2):
        k, v = pairs(n, 1000 + n)
        ok, ov = cx.sort_pairs(dev(k.view(np.int32)), dev(v.view(np.int32)), scratch=scratch)
        wk, wv = oracle.sort_pairs(k, v)
        assert np.array_equal(u32(ok, n), wk) and np.array_equal(u32(ov, n), wv)


# --------------------------------------------------------------- MSB sort --
MSB_SIZES = [0, 1, 64, 8192, 8193, 3 * 8192 + 5, 200_003, 1_000_003, 3_000_017]


@pytest.mark.parametrize("n", MSB_SIZES)
@pytest.mark.parametrize("key_bits", [32, 20, 12])
def test_msb_sort_matches_oracle(n, key_bits):
    """Most significant digit first.  32-bit keys: two partition levels, then
    local sorts (200,003 pairs: the first level's segments are short and are
    grouped).  20- and 12-bit keys leave the top digits equal, so the input
    stays one segment for several levels, and 12-bit keys reach the last
    level with runs of equal keys that are copied.  Keys and values equal
    the oracle's stable sort."""
    announce("msb sort", n, key_bits)
    k, v = pairs(n, 1300 + n + key_bits, key_bits=key_bits)
    ok, ov = cx.sort_pairs(dev(k.view(np.int32)), dev(v.view(np.int32)), msb=True)
    wk, wv = oracle.sort_pairs(k, v)
    assert np.array_equal(u32(ok, n), wk)
    assert np.array_equal(u32(ov, n), wv)


@pytest.mark.parametrize("case", ["all_equal", "two_values", "top_byte_only", "sorted", "reversed", "one_big_rest_small"])
def test_msb_sort_degenerate_inputs(case):
    """Skewed digit distributions: every key equal (one segment down to the
    last level, then one copy), two values, keys that differ only in the top
    byte, presorted and reversed input, and one huge run of a key beside
    many short segments."""
    announce("msb sort degenerate", case)
    n = 300_007
    rng = np.random.default_rng(31)
    v = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    if case == "all_equal":
        k = np.full(n, 0x9E3779B9, dtype=np.uint32)
    elif case == "two_values":
        k = np.where(rng.random(n) < 0.5, 7, 0xFFFFFFF0).astype(np.uint32)
    elif case == "top_byte_only":
        k = (rng.integers(0, 256, size=n).astype(np.uint32) << np.uint32(24))
    elif case == "sorted":
        k = np.sort(rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32))
    elif case == "reversed":
        k = np.sort(rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32))[::-1].copy()
    else:
        k = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
        k[rng.random(n) < 0.6] = 0x12345678
    ok, ov = cx.sort_pairs(dev(k.view(np.int32)), dev(v.view(np.int32)), msb=True)
    wk, wv = oracle.sort_pairs(k, v)
    assert np.array_equal(u32(ok, n), wk)
    assert np.array_equal(u32(ov, n), wv)


def test_msb_sort_long_equal_runs_are_copied_in_pieces():
    """Three million pairs of two keys: both runs stay one segment down to the
    last digit and are then copied to the output in pieces, by many
    workgroups."""
    announce("msb sort equal runs")
    n = 3_000_017
    rng = np.random.default_rng(41)
    k = np.where(rng.random(n) < 0.3, 0x0A0B0C0D, 0xF0F0F0F0).astype(np.uint32)
    v = np.arange(n, dtype=np.uint32)
    ok, ov = cx.sort_pairs(dev(k.view(np.int32)), dev(v.view(np.int32)), msb=True)
    wk, wv = oracle.sort_pairs(k, v)
    assert np.array_equal(u32(ok, n), wk)
    assert np.array_equal(u32(ov, n), wv)


def test_msb_sort_keys_only_equals_lsb_sort():
    announce("msb sort keys only")
    n = 2_000_003
    k, _ = pairs(n, 1401)
    ok, ov = cx.sort_pairs(dev(k.view(np.int32)), msb=True)
    lk, _ = cx.sort_pairs(dev(k.view(np.int32)))
    assert ov is None
    assert np.array_equal(u32(ok, n), np.sort(k))
    assert np.array_equal(u32(ok, n), u32(lk, n))


def test_msb_sort_repeated_calls_share_scratch():
    """Two sorts through one scratch buffer, the second smaller (the work
    lists and counters of the first must not leak into the second)."""
    announce("msb sort scratch reuse")
    lib = cx.load()
    n1, n2 = 1_500_001, 40_961
    scratch = torch.empty(lib.crystal_sort_pairs_msb_scratch_bytes(n1, 1), dtype=torch.uint8, device="cuda")
    for n in (n1, n2):
        k, v = pairs(n, 1500 + n)
        ok, ov = cx.sort_pairs(dev(k.view(np.int32)), dev(v.view(np.int32)), scratch=scratch, msb=True)
        wk, wv = oracle.sort_pairs(k, v)
        assert np.array_equal(u32(ok, n), wk) and np.array_equal(u32(ov, n), wv)


def test_msb_sort_scratch_too_small():
    lib = cx.load()
    k = torch.zeros(100_000, dtype=torch.int32, device="cuda")
    out = torch.empty_like(k)
    small = torch.empty(1 << 16, dtype=torch.uint8, device="cuda")
    rc = lib.crystal_sort_pairs_msb(cx._ptr(k), None, k.numel(), cx._ptr(out), None, cx._ptr(small),
                                    small.numel(), cx._stream())
    assert rc == cx.ESCRATCH


# --------------------------------------------------------- unstable shuffle --
def check_unstable(k, v, shift, bits):
    """The unstable pass orders equal digits arbitrarily: partition bounds are
    exact, and each partition holds exactly the oracle's (key, value) pairs."""
    n = k.size
    ok, ov, offs = cx.radix_partition(dev(k.view(np.int32)), shift, bits, vals=dev(v.view(np.int32)), stable=False)
    wk, wv = oracle.radix_partition(k, v, shift, bits)
    h = oracle.radix_histogram(k, shift, bits)
    bounds = np.concatenate([[0], np.cumsum(h)])
    assert np.array_equal(offs.cpu().numpy().astype(np.int64), bounds)
    gk, gv = u32(ok, n), u32(ov, n)
    for d in range(1 << bits):
        a, b = bounds[d], bounds[d + 1]
        if a == b:
            continue
        got = np.sort(gk[a:b].astype(np.uint64) << np.uint64(32) | gv[a:b].astype(np.uint64))
        want = np.sort(wk[a:b].astype(np.uint64) << np.uint64(32) | wv[a:b].astype(np.uint64))
        assert np.array_equal(got, want), d


@pytest.mark.parametrize("n", [0, 1, 4097, 100_003, 1_000_003])
@pytest.mark.parametrize("shift,bits", [(0, 8), (24, 8), (4, 4), (31, 1)])
def test_unstable_partition_matches_oracle_per_partition(n, shift, bits):
    announce("radix unstable", n, shift, bits)
    k, v = pairs(n, 1100 + n)
    check_unstable(k, v, shift, bits)


@pytest.mark.parametrize("block,ipt", [(256, 16), (1024, 8), (1024, 16)])
def test_unstable_partition_skewed_and_shapes(block, ipt):
    announce("radix unstable skew", block, ipt)
    cx.tune_set(cx.K_RADIX, block, ipt, 0)
    n = 300_007
    rng = np.random.default_rng(5)
    for keys in (np.full(n, 0x01020304, dtype=np.uint32),
                 rng.integers(0, 3, size=n, dtype=np.uint64).astype(np.uint32),
                 rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)):
        check_unstable(keys, np.arange(n, dtype=np.uint32), 0, 8)
