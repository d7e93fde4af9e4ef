"""Tile-shape autotuner (section 3.3: the tile is BLOCK threads x IPT items).

For each kernel, every compiled (BLOCK, IPT) variant is timed at several
workgroups-per-CU settings on the workload it serves, with HIP events on the
launch stream (around replays of a graph of calls, for the calls shorter
than their own host-side set-up); variants whose result differs from the
first variant's are discarded.  The winner for each workload size is
written into the library's tuning table for the size buckets nearest to
that size, and the table is saved as a text cache (``tune/gfx950.txt``)
that ``crystal.load()`` reads.

Usage: ``python -m paper_2003_01178_amd.autotune [--kernels star,select,...]
[--out PATH] [--quick]``.  Prints a JSON report.  Entries of kernels that
were not swept in this run are kept from the existing table file.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import crystal as cx
from . import datagen, queries

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_OUT = os.path.join(HERE, "tune", "gfx950.txt")
GPCS = (0, 1, 2, 4, 8)


def time_ms(fn, reps=10, warmup=2):
    for _ in range(warmup):
        fn()
    ev = []
    for _ in range(reps):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        fn()
        e.record()
        ev.append((s, e))
    torch.cuda.synchronize()
    return float(np.median([s.elapsed_time(e) for s, e in ev]))


def time_graph_ms(launch, reps=10, per_graph=10):
    """Time of one `launch(stream)` call, from replays of a HIP graph of
    `per_graph` calls with events around each replay.  The host's work per
    call (argument marshalling, launch latency) stays outside the events,
    which matters when a call is shorter than that work.  The graph is
    captured afresh, so it holds the current tuning."""
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        launch(s)
        with cx.Graph.capture(s) as g:
            for _ in range(per_graph):
                launch(s)
        g.launch(s)
        s.synchronize()
        ev = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(s)
            g.launch(s)
            b.record(s)
            ev.append((a, b))
    torch.cuda.synchronize()
    g.close()
    return float(np.median([a.elapsed_time(b) for a, b in ev])) / per_graph


def bucket(n):
    return max(0, int(n).bit_length() - 1)


def sweep(kernel, n, call, result_of, candidates=None, gpcs=GPCS, reps=10, log=None, launch=None):
    """Time every (block, ipt, grid_per_cu); return sorted [(ms, b, i, g)].

    call() runs the workload once for the result check; with `launch`
    (launch(stream): the same work on the given stream, allocating nothing)
    the timing comes from graph replays, otherwise from events around
    single calls."""
    b0 = bucket(n)
    rows, ref = [], None
    for b, i in candidates or cx.tune_variants(kernel):
        for g in gpcs:
            cx.tune_set(kernel, b, i, g, bucket_lo=b0, bucket_hi=b0)
            call()
            torch.cuda.synchronize()
            r = result_of()
            if ref is None:
                ref = r
            elif not np.array_equal(r, ref):
                if log:
                    log(f"  discard {b}x{i} g{g}: result differs")
                continue
            ms = time_graph_ms(launch, reps=reps) if launch else time_ms(call, reps=reps)
            rows.append((ms, b, i, g))
            if log:
                log(f"  {kernel} n={n} {b}x{i} g{g}: {ms * 1e3:.1f} us")
    rows.sort()
    return rows


WINNERS = {}


def assign(kernel, results):
    """results: [(n, (b, i, g))]; cover all buckets, splitting between sizes."""
    WINNERS[kernel] = list(results)
    results = sorted(results)
    bks = [bucket(n) for n, _ in results]
    for k, (n, (b, i, g)) in enumerate(results):
        lo = 0 if k == 0 else (bks[k - 1] + bks[k]) // 2 + 1
        hi = 63 if k == len(results) - 1 else (bks[k] + bks[k + 1]) // 2
        cx.tune_set(kernel, b, i, g, bucket_lo=lo, bucket_hi=hi)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--kernels", default="star,q11,select,project,probe,groupby,shared,radix")
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--quick", action="store_true", help="fewer candidates and sizes")
    ap.add_argument("--reps", type=int, default=10)
    args = ap.parse_args(argv)
    log = lambda m: print(m, file=sys.stderr, flush=True)  # noqa: E731
    cx.load()
    cx.tune_reset()
    report = {}
    kernels = args.kernels.split(",")
    quick_vec = [(128, 8), (256, 8), (256, 16), (512, 8), (1024, 8), (256, 4)]
    star_results = []

    if "star" in kernels:
        n = 120_000_000
        t = datagen.star_tables(n=n, workload=3)
        s = queries.StarSchema(t)
        s.build()
        plan = s.plan()
        out = torch.empty(queries.STAR_GROUPS, dtype=torch.int64, device="cuda")
        st = cx.new_status()
        rows = sweep(cx.K_STAR, n, lambda: plan.run(out=out, status=st), lambda: out.cpu().numpy(),
                     candidates=quick_vec if args.quick else None, reps=args.reps, log=log,
                     launch=lambda strm: plan.run(out=out, status=st, stream=strm))
        star_results.append((n, rows[0][1:]))
        report["star_120M"] = rows[:8]
        del s, t
        torch.cuda.empty_cache()
    if "q11" in kernels:
        n = 6_000_000
        f = datagen.q11_fact(n)
        plan = queries.Q11Plan(*[queries.to_dev(c) for c in (f.datekey, f.discount, f.quantity, f.price)])
        out = torch.empty(1, dtype=torch.int64, device="cuda")
        st = cx.new_status()
        rows = sweep(cx.K_STAR, n, lambda: plan.run(out=out, status=st), lambda: out.cpu().numpy(),
                     candidates=quick_vec if args.quick else None, reps=args.reps, log=log,
                     launch=lambda strm: plan.run(out=out, status=st, stream=strm))
        star_results.append((n, rows[0][1:]))
        report["q11_6M"] = rows[:8]
    if star_results:
        assign(cx.K_STAR, star_results)

    if "select" in kernels:
        n = 1 << 29
        x = queries.to_dev(datagen.select_column(n))
        lo, hi = datagen.select_threshold_range(0.5)
        o = torch.empty(n, dtype=torch.int32, device="cuda")
        c = torch.empty(1, dtype=torch.int64, device="cuda")
        cands = [(128, 4), (256, 4), (256, 8), (256, 16), (512, 8), (512, 16), (1024, 8)] if args.quick else None
        # one workgroup per tile always (grid_per_cu does not apply to selection)
        rows = sweep(cx.K_SELECT, n, lambda: cx.select(x, lo, hi, out=o, count=c), lambda: c.cpu().numpy(),
                     candidates=cands, gpcs=(0,), reps=args.reps, log=log)
        assign(cx.K_SELECT, [(n, rows[0][1:])])
        report["select_2^29"] = rows[:8]
        del x, o
        torch.cuda.empty_cache()
    if "project" in kernels:
        n = 1 << 29
        x1h, x2h = datagen.project_columns(n)
        x1, x2 = queries.to_dev(x1h), queries.to_dev(x2h)
        o = torch.empty(n, dtype=torch.float32, device="cuda")
        rows = sweep(cx.K_PROJECT, n, lambda: cx.project(x1, x2, 2.0, 3.0, out=o),
                     lambda: o[:: 1 << 16].cpu().numpy(), candidates=quick_vec if args.quick else None,
                     gpcs=(0, 2, 4), reps=args.reps, log=log)
        assign(cx.K_PROJECT, [(n, rows[0][1:])])
        report["project_2^29"] = rows[:8]
        del x1, x2, o
        torch.cuda.empty_cache()
    if "probe" in kernels:
        n = 1 << 28
        jt = datagen.join_tables(1 << 20, n_probe=n)
        ht = cx.HashTable(cx.HT_LINEAR, 1 << 20)
        ht.build(queries.to_dev(jt.dim_key), queries.to_dev(jt.dim_val))
        fk = queries.to_dev(jt.fk)
        res = torch.empty(2, dtype=torch.int64, device="cuda")
        rows = sweep(cx.K_HT_PROBE, n, lambda: ht.probe(fk, out=res), lambda: res.cpu().numpy(),
                     candidates=quick_vec if args.quick else None, gpcs=(1, 2, 4, 8), reps=args.reps, log=log)
        assign(cx.K_HT_PROBE, [(n, rows[0][1:])])
        report["probe_D2^20"] = rows[:8]
        del fk
        torch.cuda.empty_cache()
    if "groupby" in kernels:
        n = 1 << 26
        rng = np.random.default_rng(0)
        g = queries.to_dev(rng.integers(0, 7000, size=n, dtype=np.int32))
        v = queries.to_dev(rng.integers(0, 1000, size=n, dtype=np.int32))
        o = torch.empty(7000, dtype=torch.int64, device="cuda")
        st = cx.new_status()
        rows = sweep(cx.K_GROUPBY, n, lambda: cx.groupby_agg(g, v, 7000, out=o, status=st),
                     lambda: o.cpu().numpy(), candidates=quick_vec if args.quick else None,
                     gpcs=(1, 2, 4), reps=args.reps, log=log)
        assign(cx.K_GROUPBY, [(n, rows[0][1:])])
        report["groupby_2^26_7000"] = rows[:8]

    if "shared" in kernels:
        # one 16-query pass per serving template over a 75M-row clock segment
        n = 75_000_000
        t = datagen.star_tables(n=n, workload=4, with_q11_columns=True)
        sv = queries.ServingTemplates(queries.StarSchema(t))
        del t
        rng = np.random.default_rng(7)
        sv.build_star_masks([datagen.random_star_constants(rng) for _ in range(16)])
        sv.build_q11_masks([datagen.random_q11_constants(rng) for _ in range(16)])
        outs_s = [torch.zeros(queries.STAR_GROUPS, dtype=torch.int64, device="cuda") for _ in range(16)]
        outs_q = [torch.zeros(1, dtype=torch.int64, device="cuda") for _ in range(16)]
        st_s, st_q = cx.new_status(), cx.new_status()

        # grouped templates (the star template) and scalar ones (Q1.1) are
        # tuned separately: their passes differ in registers and LDS
        def star_pass():
            for o in outs_s:
                o.zero_()
            sv.star_scan.run([[] for _ in outs_s], outs_s, 0, n)

        def q11_pass():
            for o in outs_q:
                o.zero_()
            sv.q11_scan.run([[] for _ in outs_q], outs_q, 0, n)

        # timed passes accumulate without the clears: each holds 16 queries' marshalling
        rows = sweep(cx.K_SHARED_SCAN, n, star_pass, lambda: np.concatenate([o.cpu().numpy() for o in outs_s]),
                     candidates=quick_vec if args.quick else None, gpcs=(0, 1, 2, 4), reps=args.reps, log=log,
                     launch=lambda strm: sv.star_scan.run([[] for _ in outs_s], outs_s, 0, n, status=st_s,
                                                          stream=strm))
        assign(cx.K_SHARED_SCAN, [(n, rows[0][1:])])
        report["shared_star_75M_16"] = rows[:8]
        rows = sweep(cx.K_SHARED_SCAN_SCALAR, n, q11_pass, lambda: np.concatenate([o.cpu().numpy() for o in outs_q]),
                     candidates=quick_vec if args.quick else None, gpcs=(0, 1, 2, 4), reps=args.reps, log=log,
                     launch=lambda strm: sv.q11_scan.run([[] for _ in outs_q], outs_q, 0, n, status=st_q,
                                                         stream=strm))
        assign(cx.K_SHARED_SCAN_SCALAR, [(n, rows[0][1:])])
        report["shared_q11_75M_16"] = rows[:8]
        del sv
        torch.cuda.empty_cache()
    if "radix" in kernels:
        n = 1 << 28
        kh, vh = datagen.radix_pairs(n)
        keys, vals = queries.to_dev(kh), queries.to_dev(vh)
        ok, ov = torch.empty_like(keys), torch.empty_like(vals)
        scratch = torch.empty(cx.load().crystal_radix_partition_scratch_bytes(n) * 4, dtype=torch.uint8,
                              device="cuda")
        rows = sweep(cx.K_RADIX, n, lambda: cx.radix_partition(keys, 0, 8, vals=vals, out_keys=ok, out_vals=ov,
                                                               scratch=scratch),
                     lambda: ok[:: 1 << 12].cpu().numpy(), gpcs=(0, 1, 2), reps=args.reps, log=log)
        assign(cx.K_RADIX, [(n, rows[0][1:])])
        report["radix_partition_2^28"] = rows[:8]
        del keys, vals, ok, ov
        torch.cuda.empty_cache()

    # the saved table holds only the winners, not every swept candidate; kernels
    # not swept in this run keep their entries from the existing file
    kept = []
    if os.path.exists(args.out):
        with open(args.out) as f:
            for line in f:
                parts = line.split()
                if len(parts) == 6 and not line.startswith("#") and int(parts[0]) not in WINNERS:
                    kept.append([int(x) for x in parts])
    cx.tune_reset()
    for k, lo, hi, b, i, g in kept:
        cx.tune_set(k, b, i, g, bucket_lo=lo, bucket_hi=hi)
    for kernel, results in WINNERS.items():
        assign(kernel, results)
    os.makedirs(os.path.dirname(os.path.abspath(args.out)), exist_ok=True)
    cx.tune_save(args.out)
    report["saved"] = args.out
    report["device"] = torch.cuda.get_device_name(0)
    report["when"] = time.strftime("%Y-%m-%d %H:%M:%S")
    print(json.dumps(report))


if __name__ == "__main__":
    main()
