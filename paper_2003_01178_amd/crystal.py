"""Thin ctypes binding over ``libcrystal.so`` (declared in ``include/crystal.h``).

Argument marshalling only: torch tensors supply device memory and
``torch.cuda`` streams, every computation runs in the library's HIP kernels.
The binding raises ``ImportError`` when the library is missing and cannot be
built, and never falls back to CPU code.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_LIB = os.path.join(_HERE, "libcrystal.so")
# CRYSTAL_LIB selects another build of the same library (e.g. a tuning experiment)
LIB_PATH = os.environ.get("CRYSTAL_LIB", DEFAULT_LIB)

OK, EINVAL, ESCRATCH, EFULL, EDUPKEY, EHIP, EBUSY, ERANGE, ETIMEDOUT = range(9)
HT_LINEAR, HT_DIRECT = 0, 1
AGG_SUM, AGG_SUM_PRODUCT, AGG_SUM_DIFF, AGG_COUNT = 0, 1, 2, 3
K_SELECT, K_PROJECT, K_HT_PROBE, K_GROUPBY, K_STAR, K_SHARED_SCAN, K_RADIX, K_SHARED_SCAN_SCALAR = range(8)
MAX_COLS, MAX_PREDS, MAX_JOINS = 16, 4, 4
I32_MIN, I32_MAX = -(2 ** 31), 2 ** 31 - 1

c_i32, c_i64, c_vp, c_f32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_float


class Range(ctypes.Structure):
    _fields_ = [("lo", c_i32), ("hi", c_i32)]


class HT(ctypes.Structure):
    _fields_ = [("mem", c_vp), ("capacity", c_i64), ("kind", c_i32), ("key_min", c_i32),
                ("has_payload", c_i32), ("log2_capacity", c_i32)]


class Pred(ctypes.Structure):
    _fields_ = [("col", c_i32), ("range", Range)]


class Join(ctypes.Structure):
    _fields_ = [("ht", HT), ("fk_col", c_i32), ("filter_bits", c_i32), ("filter_shift", c_i32),
                ("filter", Range), ("group_bits", c_i32), ("group_shift", c_i32),
                ("group_base", c_i32), ("reserved", c_i32), ("group_stride", c_i64)]


class BuildItemC(ctypes.Structure):
    _fields_ = [("ht", ctypes.POINTER(HT)), ("keys", c_vp), ("payload", c_vp), ("filter_col", c_vp),
                ("filter", Range), ("n", c_i64)]


MAX_BUILD_BATCH = 8


class ColFormatC(ctypes.Structure):
    _fields_ = [("width", c_i32), ("base", c_i32), ("bits", c_i32), ("reserved", c_i32)]


class StarQueryC(ctypes.Structure):
    _fields_ = [("cols", c_vp * MAX_COLS), ("n_rows", c_i64), ("n_cols", c_i32), ("n_preds", c_i32),
                ("preds", Pred * MAX_PREDS), ("n_joins", c_i32), ("agg", c_i32), ("agg_col0", c_i32),
                ("agg_col1", c_i32), ("n_groups", c_i64), ("joins", Join * MAX_JOINS),
                ("formats", ColFormatC * MAX_COLS)]


MAX_BATCH = 16


class QmaskTableC(ctypes.Structure):
    _fields_ = [("mem", c_vp), ("span", c_i64), ("key_min", c_i32), ("ranked", c_i32)]


class QmaskBuildItemC(ctypes.Structure):
    _fields_ = [("t", ctypes.POINTER(QmaskTableC)), ("keys", c_vp), ("filter_col", c_vp), ("n", c_i64),
                ("ranges", ctypes.POINTER(Range)), ("n_queries", c_i32), ("reserved", c_i32)]


class BatchQueryC(ctypes.Structure):
    _fields_ = [("preds", Range * MAX_PREDS), ("out", c_vp)]


class BatchC(ctypes.Structure):
    _fields_ = [("plan", StarQueryC), ("masks", QmaskTableC * MAX_JOINS), ("n_queries", c_i32),
                ("reserved", c_i32), ("queries", BatchQueryC * MAX_BATCH), ("row_begin", c_i64),
                ("row_end", c_i64)]


MAX_TEMPLATES = 4


class ServerTemplateC(ctypes.Structure):
    _fields_ = [("plan", StarQueryC), ("dim_keys", c_vp * MAX_JOINS), ("dim_filter", c_vp * MAX_JOINS),
                ("dim_rows", c_i64 * MAX_JOINS), ("masks", QmaskTableC * MAX_JOINS)]


class ServerConfigC(ctypes.Structure):
    _fields_ = [("n_templates", c_i32), ("slots_per_template", c_i32), ("segment_rows", c_i64),
                ("max_queue", c_i32), ("inflight_steps", c_i32), ("workspace", c_vp),
                ("workspace_bytes", ctypes.c_size_t), ("stream", c_vp), ("fake_executor", c_i32),
                ("reserved", c_i32), ("fake_step_ns", c_i64), ("templates", ServerTemplateC * MAX_TEMPLATES)]


class ServerStatsC(ctypes.Structure):
    _fields_ = [(k, c_i64) for k in ("admitted", "completed", "rejected", "queued", "steps", "busy_slot_steps",
                                      "n_segments", "cancelled", "timed_out")]


class CrystalError(RuntimeError):
    def __init__(self, code, what=""):
        super().__init__(f"{what}: {status_string(code)} ({code})" if what else status_string(code))
        self.code = code


_lib = None


def _declare(lib):
    P = ctypes.POINTER
    sig = {
        "crystal_status_string": (ctypes.c_char_p, [c_i32]),
        "crystal_abi_version": (c_i32, []),
        "crystal_struct_size": (ctypes.c_size_t, [c_i32]),
        "crystal_select": (c_i32, [c_vp, c_i64, Range, c_vp, c_vp, c_vp]),
        "crystal_select_stable_scratch_bytes": (ctypes.c_size_t, [c_i64]),
        "crystal_select_stable": (c_i32, [c_vp, c_i64, Range, c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp]),
        "crystal_project": (c_i32, [c_vp, c_vp, c_i64, c_f32, c_f32, c_vp, c_vp]),
        "crystal_project_sigmoid": (c_i32, [c_vp, c_vp, c_i64, c_f32, c_f32, c_vp, c_vp]),
        "crystal_ht_init": (c_i32, [P(HT), c_i32, c_i64, c_i32, c_i32, c_i32]),
        "crystal_ht_bytes": (ctypes.c_size_t, [P(HT)]),
        "crystal_ht_build": (c_i32, [P(HT), c_vp, c_vp, c_vp, Range, c_i64, c_vp, c_vp]),
        "crystal_ht_build_batch": (c_i32, [P(BuildItemC), c_i32, c_vp, c_vp]),
        "crystal_ht_build_batch_fused": (c_i32, [P(BuildItemC), c_i32, P(P(HT)), c_i32, c_vp, c_i64, c_vp, c_vp]),
        "crystal_ht_probe": (c_i32, [P(HT), c_vp, c_vp, c_i64, c_vp, c_vp, c_vp]),
        "crystal_groupby_agg": (c_i32, [c_vp, c_vp, c_i64, c_i64, c_vp, c_vp, c_vp]),
        "crystal_star_query_scratch_bytes": (ctypes.c_size_t, [P(StarQueryC)]),
        "crystal_run_star_query": (c_i32, [P(StarQueryC), c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp]),
        "crystal_run_star_query_accumulate": (c_i32, [P(StarQueryC), c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp]),
        "crystal_run_star_query_noalloc": (c_i32, [P(StarQueryC), c_vp, c_vp, c_vp]),
        "crystal_pack_column": (c_i32, [c_vp, c_i64, c_i32, c_i32, c_vp, c_vp, c_vp]),
        "crystal_packed_column_bytes": (ctypes.c_size_t, [c_i64, c_i32]),
        "crystal_pack_column_bits": (c_i32, [c_vp, c_i64, c_i32, c_i32, c_vp, c_vp, c_vp]),
        "crystal_qmask_bytes": (ctypes.c_size_t, [c_i64]),
        "crystal_qmask_ranked_bytes": (ctypes.c_size_t, [c_i64, c_i32]),
        "crystal_qmask_rank": (c_i32, [P(QmaskTableC), c_vp, c_i64, c_vp, c_vp]),
        "crystal_qmask_build_batch": (c_i32, [P(QmaskBuildItemC), c_i32, c_vp, c_vp]),
        "crystal_qmask_build": (c_i32, [P(QmaskTableC), c_vp, c_vp, c_i64, P(Range), c_i32, c_vp, c_vp]),
        "crystal_run_shared_scan": (c_i32, [P(BatchC), c_vp, c_vp]),
        "crystal_server_workspace_bytes": (ctypes.c_size_t, [P(ServerConfigC)]),
        "crystal_server_create": (c_i32, [P(ServerConfigC), P(c_vp)]),
        "crystal_server_submit": (c_i32, [c_vp, c_i32, P(Range), P(Range), c_i64, P(c_i64)]),
        "crystal_server_cancel": (c_i32, [c_vp, c_i64]),
        "crystal_server_poll": (c_i32, [c_vp, c_i64, c_vp, c_i64, P(c_i32), P(c_i64)]),
        "crystal_server_get_stats": (c_i32, [c_vp, P(ServerStatsC)]),
        "crystal_server_destroy": (c_i32, [c_vp]),
        "crystal_graph_begin": (c_i32, [c_vp]),
        "crystal_graph_end": (c_i32, [c_vp, P(c_vp)]),
        "crystal_graph_launch": (c_i32, [c_vp, c_vp]),
        "crystal_graph_destroy": (c_i32, [c_vp]),
        "crystal_radix_histogram": (c_i32, [c_vp, c_i64, c_i32, c_i32, c_vp, c_vp]),
        "crystal_radix_partition_scratch_bytes": (ctypes.c_size_t, [c_i64]),
        "crystal_radix_partition": (c_i32, [c_vp, c_vp, c_i64, c_i32, c_i32, c_vp, c_vp, c_vp, c_vp,
                                            ctypes.c_size_t, c_vp]),
        "crystal_radix_partition_unstable": (c_i32, [c_vp, c_vp, c_i64, c_i32, c_i32, c_vp, c_vp, c_vp, c_vp,
                                                     ctypes.c_size_t, c_vp]),
        "crystal_sort_pairs_scratch_bytes": (ctypes.c_size_t, [c_i64, c_i32]),
        "crystal_sort_pairs": (c_i32, [c_vp, c_vp, c_i64, c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp]),
        "crystal_sort_pairs_msb_scratch_bytes": (ctypes.c_size_t, [c_i64, c_i32]),
        "crystal_sort_pairs_msb": (c_i32, [c_vp, c_vp, c_i64, c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp]),
        "crystal_tune_variants": (c_i32, [c_i32, P(c_i32), P(c_i32), c_i32]),
        "crystal_tune_set": (c_i32, [c_i32, c_i32, c_i32, c_i32, c_i32, c_i32]),
        "crystal_tune_get": (c_i32, [c_i32, c_i64, P(c_i32), P(c_i32), P(c_i32)]),
        "crystal_tune_reset": (None, []),
        "crystal_tune_load": (c_i32, [ctypes.c_char_p]),
        "crystal_tune_save": (c_i32, [ctypes.c_char_p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def load(path: str = LIB_PATH):
    """Load the HIP library; build it only when no built library exists."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        if path != DEFAULT_LIB:
            raise ImportError(f"{path} does not exist")
        try:
            from . import build as _build
            _build.build()
        except Exception as e:  # pragma: no cover - depends on the toolchain
            raise ImportError(f"libcrystal.so is missing and could not be built: {e}") from e
    lib = _declare(ctypes.CDLL(path))
    for which, ty in enumerate((Range, HT, Pred, Join, StarQueryC, QmaskTableC, BatchQueryC, BatchC,
                                ServerTemplateC, ServerConfigC, ServerStatsC, BuildItemC, ColFormatC,
                                QmaskBuildItemC)):
        if lib.crystal_struct_size(which) != ctypes.sizeof(ty):
            raise ImportError(f"ABI layout mismatch for {ty.__name__}")
    _lib = lib
    tune_file = os.environ.get("CRYSTAL_TUNE_FILE", os.path.join(_HERE, "tune", "gfx950.txt"))
    if os.path.exists(tune_file):
        lib.crystal_tune_load(tune_file.encode())
    return lib


def status_string(code: int) -> str:
    return load().crystal_status_string(int(code)).decode()


def _check(rc, what):
    if rc != OK:
        raise CrystalError(rc, what)


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_vp(stream.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return c_vp(t.data_ptr())


def _col(t, dtype=torch.int32):
    if t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return _ptr(t)


def new_status(device="cuda"):
    return torch.zeros(1, dtype=torch.int32, device=device)


def check_status(status):
    """Raise if a device status word holds an error (synchronises)."""
    code = int(status.item())
    if code != OK:
        raise CrystalError(code, "device status")


# ------------------------------------------------------------------ calls --
def select(x, lo, hi, out=None, count=None, stable=False, scratch=None, stream=None):
    """Section 4.2 Q3: values of x with lo <= x <= hi -> (out, count tensor).

    stable=False: tiles land in the order of their atomic reservations;
    stable=True: the values in input order (decoupled look-back)."""
    lib = load()
    n = x.numel()
    out = torch.empty(max(n, 1), dtype=torch.int32, device=x.device) if out is None else out
    if out.numel() < n:
        raise ValueError("output buffer smaller than the input")
    count = torch.empty(1, dtype=torch.int64, device=x.device) if count is None else count
    if not stable:
        _check(lib.crystal_select(_col(x), n, Range(int(lo), int(hi)), _ptr(out), _ptr(count), _stream(stream)),
               "crystal_select")
        return out, count
    nbytes = lib.crystal_select_stable_scratch_bytes(n)
    if scratch is None or scratch.numel() < nbytes:
        scratch = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
    _check(lib.crystal_select_stable(_col(x), n, Range(int(lo), int(hi)), _ptr(out), _ptr(count), _ptr(scratch),
                                     scratch.numel(), _stream(stream)), "crystal_select_stable")
    return out, count


def project(x1, x2, a, b, out=None, sigmoid=False, stream=None):
    """Section 4.1 Q1 (or Q2 with sigmoid=True): a*x1 + b*x2 in fp32."""
    lib = load()
    n = x1.numel()
    if x2.numel() != n:
        raise ValueError("x1 and x2 differ in length")
    out = torch.empty_like(x1) if out is None else out
    fn = lib.crystal_project_sigmoid if sigmoid else lib.crystal_project
    _check(fn(_col(x1, torch.float32), _col(x2, torch.float32), n, float(a), float(b),
              _col(out, torch.float32), _stream(stream)), "crystal_project")
    return out


class HashTable:
    """A dimension hash table in caller-owned (torch) device memory."""

    def __init__(self, kind, n_keys=0, key_min=0, key_max=0, has_payload=True, device="cuda"):
        lib = load()
        self.desc = HT()
        _check(lib.crystal_ht_init(ctypes.byref(self.desc), int(kind), int(n_keys), int(key_min),
                                   int(key_max), 1 if has_payload else 0), "crystal_ht_init")
        nbytes = lib.crystal_ht_bytes(ctypes.byref(self.desc))
        self.mem = torch.empty(max(16, nbytes), dtype=torch.uint8, device=device)
        self.desc.mem = self.mem.data_ptr()
        self.nbytes = nbytes

    @property
    def kind(self):
        return self.desc.kind

    def build(self, keys, payload=None, filter_col=None, filter=(I32_MIN, I32_MAX), status=None,
              stream=None):
        lib = load()
        for extra in (payload, filter_col):
            if extra is not None and extra.numel() != keys.numel():
                raise ValueError("build columns differ in length")
        status = new_status(keys.device) if status is None else status
        _check(lib.crystal_ht_build(ctypes.byref(self.desc), _col(keys),
                                    _col(payload) if payload is not None else None,
                                    _col(filter_col) if filter_col is not None else None,
                                    Range(int(filter[0]), int(filter[1])), keys.numel(),
                                    _ptr(status), _stream(stream)), "crystal_ht_build")
        return status

    def probe(self, fk, probe_payload=None, out=None, stream=None):
        """Q4 probe: device int64[2] = (sum, matches)."""
        lib = load()
        if probe_payload is not None and probe_payload.numel() != fk.numel():
            raise ValueError("probe payload and keys differ in length")
        out = torch.empty(2, dtype=torch.int64, device=fk.device) if out is None else out
        base = out.data_ptr()
        _check(lib.crystal_ht_probe(ctypes.byref(self.desc), _col(fk),
                                    _col(probe_payload) if probe_payload is not None else None,
                                    fk.numel(), c_vp(base), c_vp(base + 8), _stream(stream)),
               "crystal_ht_probe")
        return out


def _build_items(items):
    if len(items) > MAX_BUILD_BATCH:
        raise ValueError("at most 8 tables per batch")
    arr = (BuildItemC * max(1, len(items)))()
    for i, (ht, keys, payload, filter_col, rng) in enumerate(items):
        for extra in (payload, filter_col):
            if extra is not None and extra.numel() != keys.numel():
                raise ValueError("build columns differ in length")
        arr[i].ht = ctypes.pointer(ht.desc)
        arr[i].keys = _col(keys)
        arr[i].payload = _col(payload) if payload is not None else None
        arr[i].filter_col = _col(filter_col) if filter_col is not None else None
        arr[i].filter = Range(int(rng[0]), int(rng[1]))
        arr[i].n = keys.numel()
    return arr


def build_tables(items, status=None, stream=None):
    """Build several tables with one clear launch and one build launch.

    items: (HashTable, keys, payload or None, filter_col or None, (lo, hi)) per table."""
    lib = load()
    if not items:
        return status
    arr = _build_items(items)
    dev = items[0][1].device
    status = new_status(dev) if status is None else status
    _check(lib.crystal_ht_build_batch(arr, len(items), _ptr(status), _stream(stream)), "crystal_ht_build_batch")
    return status


class BuildBatch:
    """The arguments of one fused build launch, marshalled once.

    items: (HashTable, keys, payload or None, filter_col or None, (lo, hi))
    per table to build, into tables that are already clear; clear: HashTables
    to clear in the same launch; zero: an int64 tensor to zero (or None).
    ``launch()`` repeats the call (crystal_ht_build_batch_fused) with these
    arguments, so a loop that runs the same builds every step spends no host
    time rebuilding them.  The tensors and tables are referenced, not copied."""

    def __init__(self, items, clear=(), zero=None, status=None):
        if len(clear) > MAX_BUILD_BATCH:
            raise ValueError("at most 8 tables to clear")
        if zero is not None and zero.dtype != torch.int64:
            raise ValueError("zero must be an int64 tensor")
        self.arr = _build_items(items)
        self.n_items = len(items)
        self.carr = (ctypes.POINTER(HT) * max(1, len(clear)))()
        for i, ht in enumerate(clear):
            self.carr[i] = ctypes.pointer(ht.desc)
        self.n_clear = len(clear)
        if status is None:
            dev = items[0][1].device if items else (zero.device if zero is not None else clear[0].mem.device)
            status = new_status(dev)
        self.status = status
        self.zero_ptr = _ptr(zero) if zero is not None else None
        self.zero_n = zero.numel() if zero is not None else 0
        self._keep = (list(items), list(clear), zero)

    def launch(self, stream=None):
        _check(load().crystal_ht_build_batch_fused(self.arr, self.n_items, self.carr, self.n_clear, self.zero_ptr,
                                                   self.zero_n, _ptr(self.status), _stream(stream)),
               "crystal_ht_build_batch_fused")
        return self.status


def build_tables_fused(items, clear=(), zero=None, status=None, stream=None):
    """One launch: build `items` into tables that are already clear, clear the
    HashTables in `clear`, and zero the int64 tensor `zero` (if given)."""
    return BuildBatch(items, clear=clear, zero=zero, status=status).launch(stream)


def groupby_agg(group, value, n_groups, out=None, status=None, stream=None):
    lib = load()
    if value.numel() != group.numel():
        raise ValueError("group and value columns differ in length")
    out = torch.empty(int(n_groups), dtype=torch.int64, device=group.device) if out is None else out
    status = new_status(group.device) if status is None else status
    _check(lib.crystal_groupby_agg(_col(group), _col(value), group.numel(), int(n_groups), _ptr(out),
                                   _ptr(status), _stream(stream)), "crystal_groupby_agg")
    return out, status


class Narrow:
    """A narrow fact column: stored uint8 or uint16 offsets (a uint8 or int16
    tensor holding the bits) from `base`, or, with `bits`, a bit-packed
    stream of `bits`-bit offsets (an int32 tensor of words) for n rows."""

    def __init__(self, data, base, bits=0, n=None):
        self.data, self.base, self.bits = data, int(base), int(bits)
        if self.bits:
            if data.dtype != torch.int32 or n is None:
                raise TypeError("bit-packed columns hold int32 words and a row count")
            self.width, self.n = 0, int(n)
        else:
            if data.dtype not in (torch.uint8, torch.int16):
                raise TypeError("narrow columns hold uint8 or 16-bit data")
            self.width, self.n = (1 if data.dtype == torch.uint8 else 2), data.numel()

    def numel(self):
        return self.n


def pack_column_bits(x, base, bits, status=None, stream=None):
    """Bit-packed copy of an int32 column: `bits`-bit offsets from `base`
    (1 <= bits <= 16).  Returns (Narrow, status); status is CRYSTAL_ERANGE if
    a value does not fit."""
    lib = load()
    n = x.numel()
    nbytes = lib.crystal_packed_column_bytes(n, int(bits))
    if nbytes == 0:
        raise ValueError("bits must be in 1..16")
    data = torch.empty(nbytes // 4, dtype=torch.int32, device=x.device)
    status = new_status(x.device) if status is None else status
    _check(lib.crystal_pack_column_bits(_col(x), n, int(base), int(bits), c_vp(data.data_ptr()), _ptr(status),
                                        _stream(stream)), "crystal_pack_column_bits")
    return Narrow(data, base, bits=bits, n=n), status


def pack_column(x, base, width, status=None, stream=None):
    """Narrow copy of an int32 column: offsets from `base` in `width` bytes.
    Returns (Narrow, status); status is CRYSTAL_ERANGE if a value does not fit."""
    lib = load()
    n = x.numel()
    data = torch.empty(max(n, 8), dtype=torch.uint8 if width == 1 else torch.int16, device=x.device)[:n]
    status = new_status(x.device) if status is None else status
    _check(lib.crystal_pack_column(_col(x), n, int(base), int(width), c_vp(data.data_ptr()), _ptr(status),
                                   _stream(stream)), "crystal_pack_column")
    return Narrow(data, base), status


class StarQuery:
    """Plan of a fused star query (marshalled once into the C struct).

    cols: list of fact columns: int32 device tensors, or Narrow columns.
    preds: list of (col, lo, hi).
    joins: list of dicts: ``table`` (HashTable), ``fk_col``, optional
        ``filter`` = (bits, shift, lo, hi), optional ``group`` = (bits, shift,
        base, stride).
    """

    def __init__(self, cols, n_groups=1, preds=(), joins=(), agg=AGG_SUM, agg_cols=(0, 0)):
        if len(cols) > MAX_COLS or len(preds) > MAX_PREDS or len(joins) > MAX_JOINS:
            raise ValueError("plan exceeds the ABI limits")
        n = cols[0].numel() if cols else 0
        for c in cols:
            t = c.data if isinstance(c, Narrow) else c
            if (not isinstance(c, Narrow) and t.dtype != torch.int32) or c.numel() != n or not t.is_cuda:
                raise ValueError("fact columns must be int32 device tensors (or Narrow columns) of equal length")
        self.cols, self.joins = list(cols), list(joins)   # keep the memory alive
        q = StarQueryC()
        for i, c in enumerate(cols):
            if isinstance(c, Narrow):
                q.cols[i] = c.data.data_ptr()
                q.formats[i] = ColFormatC(c.width, c.base, c.bits, 0)
            else:
                q.cols[i] = c.data_ptr()
        q.n_rows, q.n_cols, q.n_preds, q.n_joins = n, len(cols), len(preds), len(joins)
        for i, (col, lo, hi) in enumerate(preds):
            q.preds[i] = Pred(int(col), Range(int(lo), int(hi)))
        for i, j in enumerate(joins):
            cj = Join()
            cj.ht = j["table"].desc
            cj.fk_col = int(j["fk_col"])
            if j.get("filter") is not None:
                bits, shift, lo, hi = j["filter"]
                cj.filter_bits, cj.filter_shift, cj.filter = int(bits), int(shift), Range(int(lo), int(hi))
            if j.get("group") is not None:
                bits, shift, base, stride = j["group"]
                cj.group_bits, cj.group_shift = int(bits), int(shift)
                cj.group_base, cj.group_stride = int(base), int(stride)
            q.joins[i] = cj
        q.agg, q.agg_col0, q.agg_col1 = int(agg), int(agg_cols[0]), int(agg_cols[1])
        q.n_groups = int(n_groups)
        self.c = q
        self.n_groups = int(n_groups)
        self.n_rows = n
        dev = (cols[0].data if isinstance(cols[0], Narrow) else cols[0]).device if cols else "cuda"
        self.device = dev
        nbytes = load().crystal_star_query_scratch_bytes(ctypes.byref(q))
        self.scratch = torch.empty(max(16, nbytes), dtype=torch.uint8, device=dev) if nbytes else None
        self.scratch_bytes = nbytes

    def run(self, out=None, status=None, stream=None, accumulate=False):
        """Run the query into out (overwritten), or add into out with accumulate=True."""
        lib = load()
        dev = self.device
        if out is None:
            out = (torch.zeros if accumulate else torch.empty)(self.n_groups, dtype=torch.int64, device=dev)
        status = new_status(dev) if status is None else status
        fn = lib.crystal_run_star_query_accumulate if accumulate else lib.crystal_run_star_query
        _check(fn(ctypes.byref(self.c), _ptr(out), _ptr(status), _ptr(self.scratch), self.scratch_bytes,
                  _stream(stream)), "crystal_run_star_query")
        return out, status

    def run_noalloc(self, out, status, stream=None):
        """Run the query into out (overwritten) through the entry point that
        allocates nothing: a scalar result's partials go to the library's
        fixed per-device array instead of this plan's scratch.  out (int64,
        n_groups) and status (int32, 1) are the caller's device tensors."""
        if out.dtype != torch.int64 or out.numel() < self.n_groups or status.dtype != torch.int32:
            raise ValueError("out must hold n_groups int64 values and status one int32")
        _check(load().crystal_run_star_query_noalloc(ctypes.byref(self.c), _ptr(out), _ptr(status),
                                                     _stream(stream)), "crystal_run_star_query_noalloc")
        return out, status


# ----------------------------------------------------------- shared scan --
class QueryMask:
    """Query-mask table of one dimension for a shared-scan batch.

    With ``keys`` (the dimension's key column, device int32) and a sparse key
    domain the table is rank-compressed: a directory of the keys present,
    built here once, and one entry per present key.  ``ranked``: True forces
    that layout, False the plain one, None picks the ranked one when it takes
    at most half the plain table's bytes."""

    def __init__(self, key_min, key_max, device="cuda", keys=None, ranked=None, status=None, stream=None):
        lib = load()
        self.c = QmaskTableC()
        self.c.span = int(key_max) - int(key_min) + 1
        self.c.key_min = int(key_min)
        plain = lib.crystal_qmask_bytes(self.c.span)
        nbytes = plain
        if keys is not None and ranked is not False:
            rb = lib.crystal_qmask_ranked_bytes(self.c.span, keys.numel())
            if ranked or (rb and 2 * rb <= plain):
                if not rb:
                    raise ValueError("no ranked layout for this span and key count")
                self.c.ranked = keys.numel()
                nbytes = rb
        elif ranked:
            raise ValueError("a ranked table needs the dimension's key column")
        self.mem = torch.empty(max(16, nbytes), dtype=torch.uint8, device=device)
        self.c.mem = self.mem.data_ptr()
        self.status = None
        if self.c.ranked:
            self.status = new_status(keys.device) if status is None else status
            _check(lib.crystal_qmask_rank(ctypes.byref(self.c), _col(keys), keys.numel(), _ptr(self.status),
                                          _stream(stream)), "crystal_qmask_rank")

    @property
    def ranked(self):
        return int(self.c.ranked)

    def build(self, keys, filter_col, ranges, status=None, stream=None):
        """Bit q of key k: the dimension row with key k has filter_col in ranges[q]."""
        lib = load()
        if filter_col is not None and filter_col.numel() != keys.numel():
            raise ValueError("filter column and keys differ in length")
        status = new_status(keys.device) if status is None else status
        rs = (Range * max(1, len(ranges)))(*[Range(int(lo), int(hi)) for lo, hi in ranges])
        _check(lib.crystal_qmask_build(ctypes.byref(self.c), _col(keys),
                                       _col(filter_col) if filter_col is not None else None, keys.numel(),
                                       rs, len(ranges), _ptr(status), _stream(stream)), "crystal_qmask_build")
        return status


def build_query_masks(items, status=None, stream=None):
    """Build several joins' query-mask tables in one call (two launches):
    the same tables as QueryMask.build on each.  items: (QueryMask, keys,
    filter_col or None, ranges) per join, at most MAX_JOINS, distinct tables."""
    lib = load()
    if len(items) > MAX_JOINS:
        raise ValueError("at most MAX_JOINS tables per batch")
    arr = (QmaskBuildItemC * max(1, len(items)))()
    keep = []
    dev = items[0][1].device if items else "cuda"
    for i, (m, keys, filt, ranges) in enumerate(items):
        if filt is not None and filt.numel() != keys.numel():
            raise ValueError("filter column and keys differ in length")
        rs = (Range * max(1, len(ranges)))(*[Range(int(lo), int(hi)) for lo, hi in ranges])
        keep.append(rs)
        arr[i] = QmaskBuildItemC(ctypes.pointer(m.c), _col(keys), _col(filt) if filt is not None else None,
                                 keys.numel(), ctypes.cast(rs, ctypes.POINTER(Range)), len(ranges), 0)
    status = new_status(dev) if status is None else status
    _check(lib.crystal_qmask_build_batch(arr, len(items), _ptr(status), _stream(stream)),
           "crystal_qmask_build_batch")
    return status


class SharedScan:
    """A shared-scan batch over a template plan (a StarQuery)."""

    def __init__(self, template, masks):
        if len(masks) != template.c.n_joins:
            raise ValueError("one query-mask table per join")
        self.template, self.masks = template, list(masks)
        self.c = BatchC()
        self.c.plan = template.c
        for j, m in enumerate(masks):
            self.c.masks[j] = m.c

    def run(self, preds, outs, row_begin=0, row_end=None, status=None, stream=None):
        """preds[q]: the query's fact-predicate ranges; outs[q]: its int64
        output (accumulated into).  Rows [row_begin, row_end)."""
        lib = load()
        if len(preds) != len(outs) or len(outs) > MAX_BATCH:
            raise ValueError("one output per query, at most 16 queries")
        c = self.c
        c.n_queries = len(outs)
        for q, (pr, o) in enumerate(zip(preds, outs)):
            if o.dtype != torch.int64 or o.numel() < self.template.n_groups:
                raise ValueError("each output holds n_groups int64")
            bq = BatchQueryC()
            for i, (lo, hi) in enumerate(pr):
                bq.preds[i] = Range(int(lo), int(hi))
            bq.out = o.data_ptr()
            c.queries[q] = bq
        c.row_begin = int(row_begin)
        c.row_end = int(self.template.n_rows if row_end is None else row_end)
        dev = outs[0].device if outs else "cuda"
        status = new_status(dev) if status is None else status
        _check(lib.crystal_run_shared_scan(ctypes.byref(c), _ptr(status), _stream(stream)), "crystal_run_shared_scan")
        return status


# ----------------------------------------------------------------- graphs --
class Graph:
    """Capture the crystal calls made on a (non-default) stream, replay them.

    with Graph.capture(stream) as g: ...calls on `stream`...
    g.launch(stream)
    """

    def __init__(self):
        self.h = None

    @classmethod
    def capture(cls, stream):
        g = cls()
        g.stream = stream
        return g

    def __enter__(self):
        _check(load().crystal_graph_begin(c_vp(self.stream.cuda_stream)), "crystal_graph_begin")
        return self

    def __exit__(self, exc_type, exc, tb):
        h = c_vp()
        rc = load().crystal_graph_end(c_vp(self.stream.cuda_stream), ctypes.byref(h))
        if exc_type is None:
            _check(rc, "crystal_graph_end")
        self.h = h
        return False

    def launch(self, stream=None):
        _check(load().crystal_graph_launch(self.h, _stream(stream or self.stream)), "crystal_graph_launch")

    def close(self):
        if self.h:
            load().crystal_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- server --
class Server:
    """Continuous-batching server over shared-scan passes (crystal_server_*).

    templates: list of dicts with ``plan`` (a StarQuery or a raw StarQueryC)
    and, per join, ``dims``: (keys, filter, n_rows, QueryMask) -- device
    columns and the mask-table memory of that dimension.
    """

    def __init__(self, templates, slots=16, segment_rows=1 << 24, max_queue=1 << 16, inflight=2, stream=None,
                 fake_step_ns=0, device="cuda"):
        lib = load()
        cfg = ServerConfigC()
        cfg.n_templates = len(templates)
        cfg.slots_per_template = int(slots)
        cfg.segment_rows = int(segment_rows)
        cfg.max_queue = int(max_queue)
        cfg.inflight_steps = int(inflight)
        cfg.fake_executor = 1 if fake_step_ns else 0
        cfg.fake_step_ns = int(fake_step_ns)
        self.keep = []
        self.ticket_template = {}
        self.n_groups, self.n_preds, self.n_joins = [], [], []
        for t, tp in enumerate(templates):
            plan = tp["plan"]
            pc = plan.c if hasattr(plan, "c") else plan
            self.keep.append(plan)
            st = ServerTemplateC()
            st.plan = pc
            for j, (keys, filt, rows, qm) in enumerate(tp.get("dims", [])):
                st.dim_keys[j] = keys.data_ptr() if hasattr(keys, "data_ptr") else keys
                st.dim_filter[j] = filt.data_ptr() if hasattr(filt, "data_ptr") else filt
                st.dim_rows[j] = int(rows)
                st.masks[j] = qm.c if hasattr(qm, "c") else qm
                self.keep.append((keys, filt, qm))
            cfg.templates[t] = st
            self.n_groups.append(int(pc.n_groups))
            self.n_preds.append(int(pc.n_preds))
            self.n_joins.append(int(pc.n_joins))
        nbytes = lib.crystal_server_workspace_bytes(ctypes.byref(cfg))
        if not cfg.fake_executor:
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
            cfg.workspace = self.workspace.data_ptr()
            cfg.workspace_bytes = nbytes
            if stream is not None:
                cfg.stream = stream.cuda_stream
                self.stream = stream
        self.cfg = cfg
        h = c_vp()
        _check(lib.crystal_server_create(ctypes.byref(cfg), ctypes.byref(h)), "crystal_server_create")
        self.h = h

    def submit(self, template_id, preds=(), filters=(), deadline_ns=0):
        """Returns a ticket, or None when the template's queue is full.
        deadline_ns > 0: the query is dropped if not complete by then."""
        lib = load()
        pr = (Range * MAX_PREDS)(*[Range(int(a), int(b)) for a, b in preds])
        fr = (Range * MAX_JOINS)(*[Range(int(a), int(b)) for a, b in filters])
        tk = c_i64()
        rc = lib.crystal_server_submit(self.h, int(template_id), pr, fr, int(deadline_ns), ctypes.byref(tk))
        if rc == EBUSY:
            return None
        _check(rc, "crystal_server_submit")
        self.ticket_template[tk.value] = int(template_id)
        return tk.value

    def poll(self, ticket, template_id=None):
        """(done, result int64 array or None, latency_ns).  The result buffer
        is sized from the template the ticket was submitted to; a template_id
        given here only selects a size to pass (the library rejects one that
        is too small)."""
        import numpy as np
        lib = load()
        t = self.ticket_template.get(int(ticket), 0) if template_id is None else int(template_id)
        out = np.zeros(self.n_groups[t], dtype=np.int64)
        done, lat = c_i32(), c_i64()
        rc = lib.crystal_server_poll(self.h, int(ticket), out.ctypes.data_as(c_vp), out.size, ctypes.byref(done),
                                     ctypes.byref(lat))
        if rc == ETIMEDOUT:                       # dropped at its deadline: the ticket is released
            self.ticket_template.pop(int(ticket), None)
        _check(rc, "crystal_server_poll")
        if not done.value:
            return False, None, 0
        self.ticket_template.pop(int(ticket), None)
        return True, out, lat.value

    def cancel(self, ticket):
        """Withdraw a queued, running or finished query; its ticket is released."""
        _check(load().crystal_server_cancel(self.h, int(ticket)), "crystal_server_cancel")
        self.ticket_template.pop(int(ticket), None)

    def stats(self):
        st = ServerStatsC()
        _check(load().crystal_server_get_stats(self.h, ctypes.byref(st)), "crystal_server_get_stats")
        return {k: getattr(st, k) for k, _ in ServerStatsC._fields_}

    def close(self):
        if self.h:
            rc = load().crystal_server_destroy(self.h)
            self.h = None
            _check(rc, "crystal_server_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------- tuning --
def _words(t, n, what):
    """A device tensor of 32-bit words (int32 holding unsigned bits) with n items."""
    if t is None:
        return None
    if t.dtype != torch.int32:
        raise TypeError(f"{what}: expected int32 words, got {t.dtype}")
    if t.numel() < n:
        raise ValueError(f"{what}: {t.numel()} words, need {n}")
    return _ptr(t)


def _scratch(nbytes, scratch, device):
    if scratch is None or scratch.numel() < nbytes:
        scratch = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    return scratch


def radix_histogram(keys, shift, bits, hist=None, stream=None):
    """Section 4.4 histogram phase: counts of digit (key >> shift) & (2^bits - 1)."""
    lib = load()
    n = keys.numel()
    hist = torch.empty(1 << int(bits), dtype=torch.int32, device=keys.device) if hist is None else hist
    _check(lib.crystal_radix_histogram(_words(keys, n, "keys"), n, int(shift), int(bits),
                                       _words(hist, 1 << int(bits), "hist"), _stream(stream)),
           "crystal_radix_histogram")
    return hist


def radix_partition(keys, shift, bits, vals=None, out_keys=None, out_vals=None, part_offsets=None,
                    scratch=None, stream=None, stable=True):
    """Section 4.4 partition pass (histogram + shuffle) on one digit; stable=False
    takes the unstable shuffle (equal digits in any order within a partition).

    Returns (out_keys, out_vals or None, part_offsets[2^bits + 1])."""
    lib = load()
    n = keys.numel()
    dev = keys.device
    out_keys = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if out_keys is None else out_keys
    if vals is not None and out_vals is None:
        out_vals = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    nb = (1 << int(bits)) + 1
    part_offsets = torch.empty(nb, dtype=torch.int32, device=dev) if part_offsets is None else part_offsets
    scratch = _scratch(lib.crystal_radix_partition_scratch_bytes(n), scratch, dev)
    fn = lib.crystal_radix_partition if stable else lib.crystal_radix_partition_unstable
    _check(fn(_words(keys, n, "keys"), _words(vals, n, "vals"), n, int(shift), int(bits),
              _words(out_keys, n, "out_keys"), _words(out_vals, n, "out_vals"),
              _words(part_offsets, nb, "part_offsets"), _ptr(scratch), scratch.numel(), _stream(stream)),
           "crystal_radix_partition")
    return out_keys, out_vals, part_offsets


def sort_pairs(keys, vals=None, out_keys=None, out_vals=None, scratch=None, stream=None, msb=False):
    """Section 4.4 sort: stable sort of (key, value) pairs by unsigned 32-bit key.
    msb: most significant digit first (crystal_sort_pairs_msb), else four
    passes from the low byte up (crystal_sort_pairs); the results are equal."""
    lib = load()
    n = keys.numel()
    dev = keys.device
    out_keys = torch.empty(max(n, 1), dtype=torch.int32, device=dev) if out_keys is None else out_keys
    if vals is not None and out_vals is None:
        out_vals = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    name = "crystal_sort_pairs_msb" if msb else "crystal_sort_pairs"
    scratch = _scratch(getattr(lib, name + "_scratch_bytes")(n, int(vals is not None)), scratch, dev)
    _check(getattr(lib, name)(_words(keys, n, "keys"), _words(vals, n, "vals"), n,
                              _words(out_keys, n, "out_keys"), _words(out_vals, n, "out_vals"), _ptr(scratch),
                              scratch.numel(), _stream(stream)), name)
    return out_keys, out_vals


def tune_variants(kernel):
    lib = load()
    n = lib.crystal_tune_variants(int(kernel), None, None, 0)
    b, i = (c_i32 * n)(), (c_i32 * n)()
    lib.crystal_tune_variants(int(kernel), b, i, n)
    return list(zip(list(b), list(i)))


def tune_set(kernel, block, ipt, grid_per_cu=0, bucket_lo=-1, bucket_hi=-1):
    _check(load().crystal_tune_set(int(kernel), int(bucket_lo), int(bucket_hi), int(block), int(ipt),
                                   int(grid_per_cu)), "crystal_tune_set")


def tune_get(kernel, n):
    b, i, g = c_i32(), c_i32(), c_i32()
    _check(load().crystal_tune_get(int(kernel), int(n), ctypes.byref(b), ctypes.byref(i), ctypes.byref(g)),
           "crystal_tune_get")
    return b.value, i.value, g.value


def tune_reset():
    load().crystal_tune_reset()


def tune_load(path):
    _check(load().crystal_tune_load(str(path).encode()), "crystal_tune_load")


def tune_save(path):
    _check(load().crystal_tune_save(str(path).encode()), "crystal_tune_save")
