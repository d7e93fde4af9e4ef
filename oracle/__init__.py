"""Crystal CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain row-at-a-time CPU definitions of what the tile-based query path of
Shanbhag, Madden and Yu (SIGMOD 2020) computes: selection (section 4.2, Q3),
projection (section 4.1, Q1/Q2), hash join with sum (section 4.3, Q4), dense
group-by aggregation, and star queries (section 3.1 SSB Q1.1, section 5.3 SSB
Q2.1), and radix histogram / partition / sort of key-value pairs (section 4.4).  The arithmetic lives in ``crystal_oracle.c`` (plain C, compiled with
gcc, no SIMD intrinsics, FP contraction off); this module only marshals numpy
arrays into it.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path.

Parity pins: every function here is checked in ``tests/test_oracle_pins.py``
against closed forms, the paper's worked compaction example, exact special
cases and brute force on tiny inputs.  Only the sigmoid projection relies on
an error bound (against exponentials computed with ``decimal``) rather than
an exact value.

The C functions keep no global state, so several threads may call them at
once (ctypes releases the GIL during each call).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "crystal_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, EDUPKEY, ERANGE = 0, 1, 4, 7
AGG_SUM, AGG_SUM_PRODUCT, AGG_SUM_DIFF, AGG_COUNT = 0, 1, 2, 3


def build(src: str = _SRC, out: str = _LIB) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-o", out + ".tmp", src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


_lib = None


def _i32p():
    return ctypes.POINTER(ctypes.c_int32)


class _StarPlan(ctypes.Structure):
    _fields_ = [
        ("n_rows", ctypes.c_int64),
        ("n_cols", ctypes.c_int32),
        ("cols", ctypes.POINTER(ctypes.c_void_p)),
        ("n_preds", ctypes.c_int32),
        ("pred_col", ctypes.c_void_p),
        ("pred_lo", ctypes.c_void_p),
        ("pred_hi", ctypes.c_void_p),
        ("n_joins", ctypes.c_int32),
        ("join_fk_col", ctypes.c_void_p),
        ("dim_key", ctypes.POINTER(ctypes.c_void_p)),
        ("dim_rows", ctypes.c_void_p),
        ("dim_filter", ctypes.POINTER(ctypes.c_void_p)),
        ("dim_flo", ctypes.c_void_p),
        ("dim_fhi", ctypes.c_void_p),
        ("dim_group", ctypes.POINTER(ctypes.c_void_p)),
        ("group_base", ctypes.c_void_p),
        ("group_stride", ctypes.c_void_p),
        ("agg_kind", ctypes.c_int32),
        ("agg_col0", ctypes.c_int32),
        ("agg_col1", ctypes.c_int32),
        ("n_groups", ctypes.c_int64),
    ]


def load(path: str = _LIB):
    """Load the compiled oracle, building it first if no library exists."""
    global _lib
    if _lib is not None and path == _LIB:
        return _lib
    if not os.path.exists(path):
        build(out=path)
    lib = ctypes.CDLL(path)
    vp, i64, i32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.oracle_select.argtypes = [vp, i64, i32, i32, vp]
    lib.oracle_select.restype = i64
    lib.oracle_project.argtypes = [vp, vp, i64, f64, f64, vp]
    lib.oracle_project.restype = None
    lib.oracle_project_sigmoid.argtypes = [vp, vp, i64, f64, f64, vp]
    lib.oracle_project_sigmoid.restype = None
    lib.oracle_join_sum.argtypes = [vp, vp, vp, i32, i32, i64, vp, vp, i64,
                                    ctypes.POINTER(i64), ctypes.POINTER(i64)]
    lib.oracle_join_sum.restype = ctypes.c_int
    lib.oracle_groupby.argtypes = [vp, vp, i64, i64, vp]
    lib.oracle_groupby.restype = ctypes.c_int
    lib.oracle_star.argtypes = [ctypes.POINTER(_StarPlan), vp, ctypes.POINTER(i64)]
    lib.oracle_star.restype = ctypes.c_int
    lib.oracle_radix_histogram.argtypes = [vp, i64, i32, i32, vp]
    lib.oracle_radix_histogram.restype = ctypes.c_int
    lib.oracle_radix_partition.argtypes = [vp, vp, i64, i32, i32, vp, vp]
    lib.oracle_radix_partition.restype = ctypes.c_int
    lib.oracle_sort_pairs.argtypes = [vp, vp, i64, vp, vp]
    lib.oracle_sort_pairs.restype = ctypes.c_int
    if path == _LIB:
        _lib = lib
    return lib


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with code {code}")
        self.code = code


def select(y, lo: int, hi: int, lib=None):
    """Qualifying values of ``lo <= y <= hi`` in input order (section 4.2, Q3)."""
    lib = lib or load()
    y, yp = _c(y, np.int32)
    out = np.empty(y.size, dtype=np.int32)
    n = lib.oracle_select(yp, y.size, int(lo), int(hi), out.ctypes.data_as(ctypes.c_void_p))
    return out[:n].copy()


def project(x1, x2, a: float, b: float, lib=None):
    """a*x1 + b*x2, evaluated in double and rounded once to float (section 4.1, Q1)."""
    lib = lib or load()
    x1, p1 = _c(x1, np.float32)
    x2, p2 = _c(x2, np.float32)
    if x1.size != x2.size:
        raise ValueError("x1 and x2 differ in length")
    out = np.empty(x1.size, dtype=np.float32)
    lib.oracle_project(p1, p2, x1.size, float(a), float(b), out.ctypes.data_as(ctypes.c_void_p))
    return out


def project_sigmoid(x1, x2, a: float, b: float, lib=None):
    """sigmoid(a*x1 + b*x2) in double, rounded once to float (section 4.1, Q2)."""
    lib = lib or load()
    x1, p1 = _c(x1, np.float32)
    x2, p2 = _c(x2, np.float32)
    out = np.empty(x1.size, dtype=np.float32)
    lib.oracle_project_sigmoid(p1, p2, x1.size, float(a), float(b), out.ctypes.data_as(ctypes.c_void_p))
    return out


def join_sum(bkey, bval, pkey, pval=None, bfilter=None, flo=0, fhi=0, lib=None):
    """(SUM, match count) of the Q4 join (section 4.3); payloads may be None."""
    lib = lib or load()
    bkey, bkp = _c(bkey, np.int32)
    keep = []
    bvp = bfp = pvp = None
    if bval is not None:
        bval, bvp = _c(bval, np.int32)
        keep.append(bval)
    if bfilter is not None:
        bfilter, bfp = _c(bfilter, np.int32)
        keep.append(bfilter)
    pkey, pkp = _c(pkey, np.int32)
    if pval is not None:
        pval, pvp = _c(pval, np.int32)
        keep.append(pval)
    s, m = ctypes.c_int64(0), ctypes.c_int64(0)
    rc = lib.oracle_join_sum(bkp, bvp, bfp, int(flo), int(fhi), bkey.size, pkp, pvp,
                             pkey.size, ctypes.byref(s), ctypes.byref(m))
    if rc:
        raise OracleError(rc, "join_sum")
    return s.value, m.value


def groupby(g, v, n_groups: int, lib=None):
    """Dense int64 ``sums[g[i]] += v[i]``; raises on a group index out of range."""
    lib = lib or load()
    g, gp = _c(g, np.int32)
    v, vp = _c(v, np.int32)
    sums = np.zeros(int(n_groups), dtype=np.int64)
    rc = lib.oracle_groupby(gp, vp, g.size, int(n_groups), sums.ctypes.data_as(ctypes.c_void_p))
    if rc:
        raise OracleError(rc, "groupby")
    return sums


def star(fact_cols, n_groups, preds=(), joins=(), agg=AGG_SUM, agg_cols=(0, 0), lib=None,
         return_survivors=False):
    """Star query by its SQL definition (section 3.1 Q1.1, section 5.3 Q2.1).

    fact_cols: list of int32 arrays of equal length.
    preds: list of (col, lo, hi) inclusive fact predicates.
    joins: list of dicts with keys ``fk_col``, ``key`` (dimension key column),
        optional ``filter`` (dimension attribute) with ``flo``/``fhi``, optional
        ``group`` (dimension attribute) with ``base``/``stride``.
    Returns the dense int64 group array (and the survivor count if asked).
    """
    lib = lib or load()
    keep = []
    cols = [np.ascontiguousarray(c, dtype=np.int32) for c in fact_cols]
    keep += cols
    n_rows = cols[0].size if cols else 0
    for c in cols:
        if c.size != n_rows:
            raise ValueError("fact columns differ in length")
    col_ptrs = (ctypes.c_void_p * max(1, len(cols)))(*[c.ctypes.data for c in cols])
    nj = len(joins)

    def arr(vals, dt):
        a = np.ascontiguousarray(np.array(vals, dtype=dt).reshape(-1))
        if a.size == 0:
            a = np.zeros(1, dtype=dt)
        keep.append(a)
        return a.ctypes.data_as(ctypes.c_void_p)

    dim_key, dim_filter, dim_group = [], [], []
    for j in joins:
        k = np.ascontiguousarray(j["key"], dtype=np.int32)
        keep.append(k)
        dim_key.append(k.ctypes.data)
        if j.get("filter") is not None:
            f = np.ascontiguousarray(j["filter"], dtype=np.int32)
            keep.append(f)
            dim_filter.append(f.ctypes.data)
        else:
            dim_filter.append(None)
        if j.get("group") is not None:
            g = np.ascontiguousarray(j["group"], dtype=np.int32)
            keep.append(g)
            dim_group.append(g.ctypes.data)
        else:
            dim_group.append(None)
    VP = ctypes.c_void_p * max(1, nj)
    plan = _StarPlan(
        n_rows=n_rows, n_cols=len(cols), cols=col_ptrs,
        n_preds=len(preds),
        pred_col=arr([p[0] for p in preds], np.int32),
        pred_lo=arr([p[1] for p in preds], np.int32),
        pred_hi=arr([p[2] for p in preds], np.int32),
        n_joins=nj,
        join_fk_col=arr([j["fk_col"] for j in joins], np.int32),
        dim_key=VP(*dim_key),
        dim_rows=arr([np.asarray(j["key"]).size for j in joins], np.int64),
        dim_filter=VP(*dim_filter),
        dim_flo=arr([j.get("flo", 0) for j in joins], np.int32),
        dim_fhi=arr([j.get("fhi", 0) for j in joins], np.int32),
        dim_group=VP(*dim_group),
        group_base=arr([j.get("base", 0) for j in joins], np.int64),
        group_stride=arr([j.get("stride", 0) for j in joins], np.int64),
        agg_kind=int(agg), agg_col0=int(agg_cols[0]), agg_col1=int(agg_cols[1]),
        n_groups=int(n_groups))
    out = np.zeros(int(n_groups), dtype=np.int64)
    surv = ctypes.c_int64(0)
    rc = lib.oracle_star(ctypes.byref(plan), out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(surv))
    if rc:
        raise OracleError(rc, "star")
    return (out, surv.value) if return_survivors else out


def radix_histogram(keys, shift: int, bits: int, lib=None):
    """Counts of digit (key >> shift) & (2^bits - 1), keys as uint32 (section 4.4)."""
    lib = lib or load()
    k, kp = _c(keys, np.uint32)
    hist = np.zeros(1 << int(bits), dtype=np.int64)
    rc = lib.oracle_radix_histogram(kp, k.size, int(shift), int(bits), hist.ctypes.data_as(ctypes.c_void_p))
    if rc:
        raise OracleError(rc, "radix_histogram")
    return hist


def radix_partition(keys, vals, shift: int, bits: int, lib=None):
    """Stable partition of (key, value) pairs by digit (section 4.4)."""
    lib = lib or load()
    k, kp = _c(keys, np.uint32)
    v, vp = _c(vals, np.uint32)
    ok, ov = np.empty_like(k), np.empty_like(v)
    rc = lib.oracle_radix_partition(kp, vp, k.size, int(shift), int(bits), ok.ctypes.data_as(ctypes.c_void_p),
                                    ov.ctypes.data_as(ctypes.c_void_p))
    if rc:
        raise OracleError(rc, "radix_partition")
    return ok, ov


def sort_pairs(keys, vals, lib=None):
    """Stable sort of (key, value) pairs by unsigned 32-bit key (section 4.4)."""
    lib = lib or load()
    k, kp = _c(keys, np.uint32)
    v, vp = _c(vals, np.uint32)
    ok, ov = np.empty_like(k), np.empty_like(v)
    rc = lib.oracle_sort_pairs(kp, vp, k.size, ok.ctypes.data_as(ctypes.c_void_p), ov.ctypes.data_as(ctypes.c_void_p))
    if rc:
        raise OracleError(rc, "sort_pairs")
    return ok, ov
