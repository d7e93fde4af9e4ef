"""The C-ABI library loads and exports every symbol include/crystal.h declares;
host-only calls (descriptors, tuning table, struct layout) work without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "crystal.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(crystal_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def cx():
    from paper_2003_01178_amd import crystal
    crystal.load()
    return crystal


def test_every_declared_symbol_is_exported(cx):
    names = declared_functions()
    assert len(names) >= 15
    lib = ctypes.CDLL(cx.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_struct_layout_matches_binding(cx):
    lib = cx.load()
    assert lib.crystal_abi_version() == 10
    for which, ty in enumerate((cx.Range, cx.HT, cx.Pred, cx.Join, cx.StarQueryC, cx.QmaskTableC,
                                cx.BatchQueryC, cx.BatchC, cx.ServerTemplateC, cx.ServerConfigC,
                                cx.ServerStatsC, cx.BuildItemC, cx.ColFormatC, cx.QmaskBuildItemC)):
        assert lib.crystal_struct_size(which) == ctypes.sizeof(ty), ty.__name__
    assert lib.crystal_struct_size(99) == 0


def test_status_strings(cx):
    lib = cx.load()
    for code in range(8):
        assert lib.crystal_status_string(code).decode() not in ("", "unknown status")
    assert lib.crystal_status_string(1234).decode() == "unknown status"


def test_ht_descriptors(cx):
    lib = cx.load()
    ht = cx.HT()
    assert lib.crystal_ht_init(ctypes.byref(ht), cx.HT_LINEAR, 1 << 13, 0, 0, 1) == cx.OK
    assert ht.capacity == 1 << 14 and ht.log2_capacity == 14
    assert lib.crystal_ht_bytes(ctypes.byref(ht)) == (1 << 14) * 8          # 128 KiB at 50% fill
    assert lib.crystal_ht_init(ctypes.byref(ht), cx.HT_LINEAR, 3, 0, 0, 1) == cx.OK
    assert ht.capacity == 64                                                 # minimum capacity
    assert lib.crystal_ht_init(ctypes.byref(ht), cx.HT_LINEAR, 5, 0, 0, 1) == cx.OK
    assert ht.capacity == 64
    assert lib.crystal_ht_init(ctypes.byref(ht), cx.HT_LINEAR, 33, 0, 0, 1) == cx.OK
    assert ht.capacity == 128
    assert lib.crystal_ht_init(ctypes.byref(ht), cx.HT_DIRECT, 0, 10, 2009, 1) == cx.OK
    assert ht.capacity == 2000 and ht.key_min == 10
    words = ((2000 + 31) // 32 + 63) // 64 * 64
    assert lib.crystal_ht_bytes(ctypes.byref(ht)) == words * 4 + 2000 * 4
    assert lib.crystal_ht_init(ctypes.byref(ht), cx.HT_DIRECT, 0, 10, 2009, 0) == cx.OK
    assert lib.crystal_ht_bytes(ctypes.byref(ht)) == words * 4
    assert lib.crystal_ht_init(ctypes.byref(ht), cx.HT_DIRECT, 0, 5, 4, 0) == cx.EINVAL
    assert lib.crystal_ht_init(ctypes.byref(ht), 7, 10, 0, 0, 0) == cx.EINVAL
    assert lib.crystal_ht_init(ctypes.byref(ht), cx.HT_LINEAR, -1, 0, 0, 0) == cx.EINVAL


def test_host_argument_errors_return_without_launch(cx):
    lib = cx.load()
    vp16 = ctypes.c_void_p(16)
    assert lib.crystal_select(None, -1, cx.Range(0, 1), None, None, None) == cx.EINVAL
    assert lib.crystal_select(vp16, 10, cx.Range(0, 1), None, vp16, None) == cx.EINVAL
    assert lib.crystal_select(ctypes.c_void_p(20), 10, cx.Range(0, 1), ctypes.c_void_p(32),
                              vp16, None) == cx.EINVAL                         # misaligned column
    assert lib.crystal_select_stable(None, -1, cx.Range(0, 1), None, None, None, 0, None) == cx.EINVAL
    need = lib.crystal_select_stable_scratch_bytes(1 << 29)
    assert need >= (1 << 29) // (1024 * 16) * 8
    assert lib.crystal_select_stable(vp16, 1 << 29, cx.Range(0, 1), vp16, vp16, None, 0, None) == cx.ESCRATCH
    assert lib.crystal_select_stable(vp16, 1 << 29, cx.Range(0, 1), vp16, vp16, vp16, need - 8,
                                     None) == cx.ESCRATCH
    assert lib.crystal_project(None, None, 5, 1.0, 1.0, None, None) == cx.EINVAL
    assert lib.crystal_groupby_agg(None, None, 0, 0, ctypes.c_void_p(16), ctypes.c_void_p(16), None) == cx.EINVAL
    ht = cx.HT()
    assert lib.crystal_ht_build(ctypes.byref(ht), None, None, None, cx.Range(0, 0), 0,
                                ctypes.c_void_p(16), None) == cx.EINVAL           # no memory
    q = cx.StarQueryC()
    q.n_groups = 0
    vp16 = ctypes.c_void_p(16)
    assert lib.crystal_run_star_query(ctypes.byref(q), vp16, vp16, None, 0, None) == cx.EINVAL
    q.n_groups, q.n_joins = 1, 5
    assert lib.crystal_run_star_query(ctypes.byref(q), vp16, vp16, None, 0, None) == cx.EINVAL
    # a scalar plan needs scratch: missing or short scratch is reported before any launch
    q.n_joins, q.n_cols, q.n_rows, q.n_preds = 0, 1, 100, 1
    q.cols[0] = 4096
    q.preds[0] = cx.Pred(0, cx.Range(0, 5))
    q.agg = cx.AGG_COUNT
    need = lib.crystal_star_query_scratch_bytes(ctypes.byref(q))
    assert need >= 8 * 256
    assert lib.crystal_run_star_query(ctypes.byref(q), vp16, vp16, None, 0, None) == cx.ESCRATCH
    assert lib.crystal_run_star_query(ctypes.byref(q), vp16, vp16, ctypes.c_void_p(4096), need - 8, None) == cx.ESCRATCH
    q.n_groups = 10                     # grouped plan: no scratch needed
    assert lib.crystal_star_query_scratch_bytes(ctypes.byref(q)) == 0


def test_tuning_table(cx, tmp_path):
    cx.tune_reset()
    sel = cx.tune_variants(cx.K_SELECT)
    assert (128, 4) in sel and (256, 8) in sel and (64, 1) in sel and len(sel) == 25
    assert len(cx.tune_variants(cx.K_STAR)) == 15
    d = cx.tune_get(cx.K_STAR, 120_000_000)
    cx.tune_set(cx.K_STAR, 512, 8, 2, bucket_lo=20, bucket_hi=30)
    assert cx.tune_get(cx.K_STAR, 120_000_000) == (512, 8, 2)                # bucket 26
    assert cx.tune_get(cx.K_STAR, 1000) == d
    with pytest.raises(cx.CrystalError):
        cx.tune_set(cx.K_STAR, 512, 3, 0)                                    # not compiled
    p = tmp_path / "tune.txt"
    cx.tune_save(p)
    cx.tune_reset()
    assert cx.tune_get(cx.K_STAR, 120_000_000) == d
    cx.tune_load(p)
    assert cx.tune_get(cx.K_STAR, 120_000_000) == (512, 8, 2)
    cx.tune_reset()


def test_radix_host_errors(cx):
    """Argument errors of the radix calls are caught on the host, before any
    device work (the pointers below are never dereferenced)."""
    lib = cx.load()
    fake_a, fake_b = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 30)
    for shift, bits in [(0, 0), (0, 9), (25, 8), (-1, 4), (31, 2)]:
        assert lib.crystal_radix_partition(fake_a, None, 100, shift, bits, fake_b, None, None, None, 0,
                                           None) == cx.EINVAL
        assert lib.crystal_radix_histogram(fake_a, 100, shift, bits, fake_b, None) == cx.EINVAL
    # values without an output for them, overlapping output, n out of range
    assert lib.crystal_radix_partition(fake_a, fake_a, 100, 0, 8, fake_b, None, None, None, 0, None) == cx.EINVAL
    assert lib.crystal_radix_partition(fake_a, None, 100, 0, 8, ctypes.c_void_p((1 << 20) + 64), None, None,
                                       None, 0, None) == cx.EINVAL
    assert lib.crystal_sort_pairs(fake_a, None, -1, fake_b, None, None, 0, None) == cx.EINVAL
    assert lib.crystal_sort_pairs(fake_a, None, 1 << 32, fake_b, None, None, 0, None) == cx.EINVAL
    assert lib.crystal_sort_pairs(None, None, 0, None, None, None, 0, None) == cx.OK
    assert lib.crystal_sort_pairs_msb(fake_a, None, -1, fake_b, None, None, 0, None) == cx.EINVAL
    assert lib.crystal_sort_pairs_msb(fake_a, None, 1 << 32, fake_b, None, None, 0, None) == cx.EINVAL
    assert lib.crystal_sort_pairs_msb(fake_a, fake_a, 100, fake_b, None, None, 0, None) == cx.EINVAL
    assert lib.crystal_sort_pairs_msb(fake_a, None, 100, fake_b, None, None, 0, None) == cx.ESCRATCH
    assert lib.crystal_sort_pairs_msb(fake_a, None, 100, fake_b, None, ctypes.c_void_p((1 << 24) + 8), 1 << 20,
                                      None) == cx.EINVAL
    assert lib.crystal_sort_pairs_msb(None, None, 0, None, None, None, 0, None) == cx.OK
    assert lib.crystal_sort_pairs_msb_scratch_bytes(1 << 28, 1) > 2 * 4 * (1 << 28)
    assert lib.crystal_radix_histogram(fake_a, 100, 0, 8, None, None) == cx.EINVAL


def test_radix_tuning_variants(cx):
    lib = cx.load()
    n = cx.tune_variants(cx.K_RADIX)
    assert (256, 16) in n and all(b >= 256 for b, _ in n)
    assert lib.crystal_tune_set(cx.K_RADIX, -1, -1, 128, 16, 0) == cx.EINVAL
    assert lib.crystal_tune_set(cx.K_RADIX, -1, -1, 1024, 8, 2) == cx.OK
    cx.tune_reset()


def test_build_batch_and_pack_host_errors(cx):
    """Argument errors of the batched build and of crystal_pack_column are
    returned on the host before any device work."""
    lib = cx.load()
    st = ctypes.c_void_p(1 << 20)
    assert lib.crystal_ht_build_batch(None, 1, st, None) == cx.EINVAL
    items = (cx.BuildItemC * 9)()
    assert lib.crystal_ht_build_batch(items, 9, st, None) == cx.EINVAL          # more than 8 tables
    assert lib.crystal_ht_build_batch(items, -1, st, None) == cx.EINVAL
    assert lib.crystal_ht_build_batch(items, 1, st, None) == cx.EINVAL          # no table descriptor
    assert lib.crystal_ht_build_batch(items, 0, st, None) == cx.OK
    ht = cx.HT()
    assert lib.crystal_ht_init(ctypes.byref(ht), cx.HT_DIRECT, 10, 0, 9, 1) == cx.OK
    ht.mem = 1 << 20
    items[0].ht = ctypes.pointer(ht)
    items[0].keys = 1 << 21
    items[0].n = 10
    assert lib.crystal_ht_build_batch(items, 1, st, None) == cx.EINVAL          # payload table, no payload
    items[1] = items[0]
    items[0].payload = items[1].payload = 1 << 22
    assert lib.crystal_ht_build_batch(items, 2, st, None) == cx.EINVAL          # the same table twice
    fake = ctypes.c_void_p(1 << 20)
    out = ctypes.c_void_p(1 << 24)
    for width in (0, 3, 4):
        assert lib.crystal_pack_column(fake, 100, 0, width, out, st, None) == cx.EINVAL
    assert lib.crystal_pack_column(ctypes.c_void_p((1 << 20) + 4), 100, 0, 2, out, st, None) == cx.EINVAL
    assert lib.crystal_pack_column(fake, 100, 0, 2, out, None, None) == cx.EINVAL
    assert lib.crystal_pack_column(None, 0, 0, 1, None, st, None) == cx.OK


def test_build_batch_fused_host_errors(cx):
    """crystal_ht_build_batch_fused rejects bad counts, descriptors, zero
    ranges and any overlap between the memory it writes, before any device
    work."""
    lib = cx.load()
    st = ctypes.c_void_p(1 << 20)
    f = lib.crystal_ht_build_batch_fused
    none = (ctypes.POINTER(cx.HT) * 1)()
    items = (cx.BuildItemC * 9)()
    assert f(items, 9, none, 0, None, 0, st, None) == cx.EINVAL                  # more than 8 builds
    assert f(items, -1, none, 0, None, 0, st, None) == cx.EINVAL
    assert f(None, 1, none, 0, None, 0, st, None) == cx.EINVAL
    assert f(items, 0, none, 9, None, 0, st, None) == cx.EINVAL                  # more than 8 clears
    assert f(items, 0, None, 1, None, 0, st, None) == cx.EINVAL
    assert f(items, 0, none, 1, None, 0, st, None) == cx.EINVAL                  # no clear descriptor
    assert f(items, 0, none, 0, None, 0, None, None) == cx.EINVAL                # no status word
    assert f(items, 0, none, 0, None, -1, st, None) == cx.EINVAL
    assert f(items, 0, none, 0, None, 4, st, None) == cx.EINVAL                  # zero range without memory
    assert f(items, 0, none, 0, ctypes.c_void_p((1 << 24) + 4), 4, st, None) == cx.EINVAL  # misaligned
    assert f(items, 0, none, 0, None, 0, st, None) == cx.OK                      # nothing to do
    a, b = cx.HT(), cx.HT()
    for ht, mem in ((a, 1 << 20), (b, 1 << 21)):
        assert lib.crystal_ht_init(ctypes.byref(ht), cx.HT_DIRECT, 1000, 0, 999, 1) == cx.OK
        ht.mem = mem
    nbytes = lib.crystal_ht_bytes(ctypes.byref(a))
    items[0].ht = ctypes.pointer(a)
    items[0].keys = items[0].payload = 1 << 23
    items[0].n = 1000
    clear = (ctypes.POINTER(cx.HT) * 2)(ctypes.pointer(a), ctypes.pointer(b))
    clear_b = (ctypes.POINTER(cx.HT) * 1)(ctypes.pointer(b))
    assert f(items, 1, clear, 1, None, 0, st, None) == cx.EINVAL                 # builds into a cleared table
    # the zeroed range overlaps the built table's last bytes, then the cleared table's first
    assert f(items, 1, clear_b, 1, ctypes.c_void_p((1 << 20) + nbytes - 8),
             4, st, None) == cx.EINVAL
    assert f(items, 0, clear, 2, ctypes.c_void_p((1 << 21) - 16), 4, st, None) == cx.EINVAL
    items[1] = items[0]
    assert f(items, 2, none, 0, None, 0, st, None) == cx.EINVAL                  # the same table twice
    b.mem = (1 << 20) + nbytes - 16                                            # b starts inside a
    assert f(items, 1, clear_b, 1, None, 0, st, None) == cx.EINVAL


def test_star_query_format_validation(cx):
    """Column formats other than int32, uint16 and uint8 are rejected."""
    lib = cx.load()
    q = cx.StarQueryC()
    q.n_cols, q.n_rows, q.n_groups, q.agg = 1, 0, 1, cx.AGG_COUNT
    assert lib.crystal_star_query_scratch_bytes(ctypes.byref(q)) >= 0
    q.formats[0] = cx.ColFormatC(3, 0)
    st = ctypes.c_void_p(1 << 20)
    assert lib.crystal_run_star_query(ctypes.byref(q), ctypes.c_void_p(1 << 21), st, None, 0, None) == cx.EINVAL


def test_ranked_qmask_sizes_and_host_errors(cx):
    """Rank-compressed query-mask tables: ceil(span / 32) + 1 directory entries
    of 8 bytes, then ranked + 1 two-byte entries, rounded up to 16 bytes."""
    lib = cx.load()
    assert lib.crystal_qmask_ranked_bytes(61_130, 2556) == (8 * 1912 + 4 * 1279 + 15) // 16 * 16
    assert lib.crystal_qmask_ranked_bytes(1, 1) == 32        # two directory entries, one entry word
    for span, ranked in [(0, 4), (100, 0), (100, -1), ((1 << 26) + 1, 4)]:
        assert lib.crystal_qmask_ranked_bytes(span, ranked) == 0
    status = ctypes.c_int32()
    mem = ctypes.create_string_buffer(4096 + 16)
    addr = (ctypes.addressof(mem) + 15) // 16 * 16
    keys = ctypes.c_void_p(addr)
    bad = []
    for span, ranked, n in [(100, 0, 4), (100, -2, 4), ((1 << 26) + 1, 4, 4), (100, 4, -1), (0, 4, 4)]:
        t = cx.QmaskTableC(mem=addr, span=span, key_min=0, ranked=ranked)
        bad.append(lib.crystal_qmask_rank(ctypes.byref(t), keys, n, ctypes.byref(status), None))
    assert bad == [cx.EINVAL] * 5
    t = cx.QmaskTableC(mem=addr + 4, span=100, key_min=0, ranked=4)       # misaligned table
    assert lib.crystal_qmask_rank(ctypes.byref(t), keys, 4, ctypes.byref(status), None) == cx.EINVAL
    rs = (cx.Range * 1)(cx.Range(0, 0))
    t = cx.QmaskTableC(mem=addr, span=(1 << 26) + 1, key_min=0, ranked=4)
    assert lib.crystal_qmask_build(ctypes.byref(t), keys, None, 4, rs, 1, ctypes.byref(status), None) == cx.EINVAL


def test_qmask_build_batch_host_errors(cx):
    lib = cx.load()
    status = ctypes.c_int32()
    mem = ctypes.create_string_buffer(4096 + 16)
    addr = (ctypes.addressof(mem) + 15) // 16 * 16
    t1 = cx.QmaskTableC(mem=addr, span=100, key_min=0, ranked=0)
    t2 = cx.QmaskTableC(mem=addr + 1024, span=100, key_min=0, ranked=0)
    rs = (cx.Range * 2)(cx.Range(0, 1), cx.Range(2, 3))
    keys = ctypes.c_void_p(addr + 2048)

    def item(t, n=4, nq=2, k=keys, r=rs):
        return cx.QmaskBuildItemC(ctypes.pointer(t), k, None, n, ctypes.cast(r, ctypes.POINTER(cx.Range)), nq, 0)

    def call(items, n=None):
        arr = (cx.QmaskBuildItemC * max(1, len(items)))(*items)
        return lib.crystal_qmask_build_batch(arr, len(items) if n is None else n, ctypes.byref(status), None)

    assert call([item(t1), item(t1)]) == cx.EINVAL                  # one table twice
    assert call([item(t1)] * 1, n=5) == cx.EINVAL                   # more than CRYSTAL_MAX_JOINS
    assert call([item(t1), item(t2, n=-1)]) == cx.EINVAL
    assert call([item(t1, nq=17)]) == cx.EINVAL
    assert call([item(t1, k=None)]) == cx.EINVAL                    # rows without keys
    assert call([item(t1, r=None)]) == cx.EINVAL                    # queries without ranges
    bad = cx.QmaskTableC(mem=addr + 4, span=100, key_min=0, ranked=0)  # misaligned
    assert call([item(bad)]) == cx.EINVAL
    assert lib.crystal_qmask_build_batch(None, 1, ctypes.byref(status), None) == cx.EINVAL
    assert call([], n=0) == cx.OK


def test_shared_scan_tuning_classes(cx):
    """Grouped and scalar shared-scan templates are tuned separately; both
    classes take the 16-byte-vector tile shapes."""
    lib = cx.load()
    assert cx.K_SHARED_SCAN_SCALAR == 7 and lib.crystal_tune_variants(8, None, None, 0) == 0
    assert lib.crystal_tune_variants(cx.K_SHARED_SCAN_SCALAR, None, None, 0) == \
        lib.crystal_tune_variants(cx.K_SHARED_SCAN, None, None, 0) > 0
    try:
        assert lib.crystal_tune_set(cx.K_SHARED_SCAN_SCALAR, -1, -1, 1024, 8, 0) == cx.OK
        assert lib.crystal_tune_set(cx.K_SHARED_SCAN, -1, -1, 1024, 16, 0) == cx.OK
        assert cx.tune_get(cx.K_SHARED_SCAN_SCALAR, 1 << 26) == (1024, 8, 0)
        assert cx.tune_get(cx.K_SHARED_SCAN, 1 << 26) == (1024, 16, 0)
        assert lib.crystal_tune_set(cx.K_SHARED_SCAN_SCALAR, -1, -1, 1024, 3, 0) == cx.EINVAL
    finally:
        cx.tune_reset()


def test_star_noalloc_host_errors(cx):
    """The allocation-free star entry point checks its arguments and its fixed
    partials array's limit on the host, before anything is launched."""
    lib = cx.load()
    q = cx.StarQueryC()
    fake = ctypes.c_void_p(1 << 20)
    q.n_cols, q.n_groups, q.agg, q.agg_col0 = 1, 1, cx.AGG_SUM, 0
    q.cols[0] = 1 << 20
    st, out = ctypes.c_void_p(1 << 21), ctypes.c_void_p(1 << 22)
    # above CRYSTAL_STAR_NOALLOC_PARTIALS workgroups of 256 x 65535 rows: rejected
    q.n_rows = 8192 * 256 * 65535 + 1
    assert lib.crystal_run_star_query_noalloc(ctypes.byref(q), out, st, None) == cx.ESCRATCH
    # the ordinary entry point would need more than the fixed 64 KiB for it
    assert lib.crystal_star_query_scratch_bytes(ctypes.byref(q)) > 8192 * 8
    assert lib.crystal_run_star_query_noalloc(None, out, st, None) == cx.EINVAL
    assert lib.crystal_run_star_query_noalloc(ctypes.byref(q), None, st, None) == cx.EINVAL
    assert lib.crystal_run_star_query_noalloc(ctypes.byref(q), out, None, None) == cx.EINVAL
    q.cols[0] = (1 << 20) + 4                                                    # misaligned column
    q.n_rows = 100
    assert lib.crystal_run_star_query_noalloc(ctypes.byref(q), out, st, None) == cx.EINVAL
    del fake


def test_bitpacked_format_host_checks(cx):
    """Bit widths 1..16 only, and only with width 0; the packed size is the
    stream's words plus four words of padding."""
    lib = cx.load()
    assert lib.crystal_packed_column_bytes(10, 12) == (4 + 4) * 4      # 120 bits: 4 words, then padding
    assert lib.crystal_packed_column_bytes(0, 5) == 16
    assert lib.crystal_packed_column_bytes(10, 0) == 0 and lib.crystal_packed_column_bytes(10, 17) == 0
    st, fake = ctypes.c_void_p(1 << 21), ctypes.c_void_p(1 << 20)
    assert lib.crystal_pack_column_bits(fake, 10, 0, 17, fake, st, None) == cx.EINVAL
    assert lib.crystal_pack_column_bits(fake, 10, 0, 4, ctypes.c_void_p((1 << 20) + 4), st, None) == cx.EINVAL
    q = cx.StarQueryC()
    q.n_cols, q.n_rows, q.n_groups, q.agg = 1, 0, 1, cx.AGG_COUNT
    for width, bits in ((0, 17), (2, 4), (0, -1)):
        q.formats[0] = cx.ColFormatC(width, 0, bits, 0)
        assert lib.crystal_run_star_query(ctypes.byref(q), ctypes.c_void_p(1 << 21), st, None, 0, None) == cx.EINVAL
