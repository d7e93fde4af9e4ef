#!/usr/bin/env python3
"""Benchmark of the fused star query (and the operator micro-benchmarks).

Default workload: a 120,000,000-row fact table (four int32 foreign keys, two
int32 measures) joined to four dimensions of 2,556 / 40,000 / 200,000 /
600,000 rows, each filtered to about 1/25 of its rows, grouped by
(year, dim3.group) into 7,000 int64 sums.  One step = the four filtered
dimension builds plus the fused probe/aggregate kernel, on resident data.

Prints one JSON line.  ``roofline`` refers to the fused star kernel: its
algorithmic bytes (fact-column cache lines the selective loads must touch, at
the HBM fetch granularity) over its average duration measured with HIP events
on the launch stream.  ``cpu_baseline`` is the plain CPU oracle timed on the
host over full passes of the same workload, with the rows split over the
host threads (and on one thread beside it), next to the host's streaming
read bandwidth.  ``serving`` is the served mixed workload measured in the
same run: a 600M-row fact table, Poisson arrivals at 50..2,000 queries/s of
star-join and Q1.1-shaped queries answered by the continuous-batching
server, p50/p99 latency per rate, a burst, one launch per query beside it,
sampled answers checked against their single launches and the oracle, and
the roofline of one 16-query shared-scan pass per template.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
# HBM fetch granularity: a 128-byte line (rocprofv3 FETCH_SIZE of the star kernel, calibrated
# against a plain copy, equals the 128-byte live-line count)
FETCH_BYTES = int(os.environ.get("CRYSTAL_FETCH_BYTES", "128"))
LLC_BYTES = 256 * 2 ** 20   # MI355X last-level (Infinity) cache


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--workload", default="star", choices=["star", "q11", "select", "project", "join", "copy", "serve",
                                                              "pass", "partition", "sort", "groupby"])
    p.add_argument("--rows", type=int, default=0, help="override the fact/column length")
    p.add_argument("--sigma", type=float, default=0.5, help="select selectivity")
    p.add_argument("--sigma-sweep", action="store_true", help="select: also time sigma = 0, 0.1, ..., 1")
    p.add_argument("--dim", type=int, default=1 << 20, help="join build size D")
    p.add_argument("--kind", default="linear", choices=["linear", "direct"])
    p.add_argument("--bits", type=int, default=8, help="partition: radix bits")
    p.add_argument("--shift", type=int, default=0, help="partition: start bit")
    p.add_argument("--unstable", action="store_true", help="partition: the unstable shuffle")
    p.add_argument("--msb", action="store_true", help="sort: most significant digit first")
    p.add_argument("--order", default="1,0,2,3", help="star join order")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--graph", action="store_true",
                   help="star: replay the steps as HIP graphs (two steps per graph) instead of launching them")
    p.add_argument("--narrow", action="store_true",
                   help="star: bit-packed dense-phase foreign keys: date keys as 12-bit day codes, fk1 as 16 bits")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    p.add_argument("--tune", default="", help="kernel block,ipt,grid_per_cu override, e.g. 256,16,0")
    p.add_argument("--rates", default="50,200,500,1000,2000", help="serve: Poisson arrival rates (q/s)")
    p.add_argument("--seconds", type=float, default=0.0,
                   help="serve: arrival window per rate (0: 5,000 arrivals, between 5 and 10 s)")
    p.add_argument("--segments", type=int, default=8, help="serve: clock segments of the fact table")
    p.add_argument("--serve-rows", type=int, default=0, help="serve: fact rows (default 600M)")
    p.add_argument("--serve-pass-reps", type=int, default=20, help="serve: timed shared-scan passes per template")
    p.add_argument("--no-serve", action="store_true", help="star: skip the served-mix measurement")
    p.add_argument("--settle", type=float, default=0.25,
                   help="seconds of untimed steps before the warmup steps (0: none)")
    return p.parse_args()


def host_info():
    model = platform.processor()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def lines_touched(mask: np.ndarray, item_bytes: int = 4, line: int = FETCH_BYTES, bits: int = 0) -> int:
    """Number of `line`-byte lines of a column holding at least one live item
    (bits > 0: a bit-packed column; a field that straddles two lines touches
    both)."""
    if bits:
        idx = np.flatnonzero(mask).astype(np.int64)
        lb = 8 * line
        touched = np.zeros((mask.size * bits + lb - 1) // lb + 1, dtype=bool)
        touched[(idx * bits) // lb] = True
        touched[(idx * bits + bits - 1) // lb] = True
        return int(touched.sum())
    per = line // item_bytes
    n = mask.size
    pad = (-n) % per
    if pad:
        mask = np.concatenate([mask, np.zeros(pad, dtype=bool)])
    return int(mask.reshape(-1, per).any(axis=1).sum())


def star_algorithmic_bytes(t, order, line=FETCH_BYTES, bits=None):
    """Bytes the selective scan must fetch: column s is read at the lines that
    hold an item still alive before step s; the measure at the survivors.
    bits[j]: bits per stored value of foreign-key column j (default 32)."""
    alive = np.ones(t.n, dtype=bool)
    total = 0
    for j in order:
        d = t.dims[j]
        b = 32 if bits is None else bits[j]
        total += lines_touched(alive, line=line, bits=b if b != 32 else 0) * line
        kmin = int(d.key.min())
        keep = np.zeros(int(d.key.max()) - kmin + 1, dtype=bool)
        keep[d.key[d.filter == t.consts[j]] - kmin] = True
        fk = t.fk[j]
        ok = (fk >= kmin) & (fk - kmin < keep.size)
        hit = np.zeros(t.n, dtype=bool)
        hit[ok] = keep[fk[ok] - kmin]
        alive &= hit
    total += lines_touched(alive, line=line) * line          # m1 of the survivors
    return total, int(alive.sum())


def measured_traffic(order, n, packed=False):
    """HBM bytes per star-kernel launch from the committed rocprofv3 counter
    record (FETCH_SIZE and WRITE_SIZE scaled by a plain copy), or None when
    the record is missing, was taken on another workload, or the kernel
    sources changed since.  packed: the bit-packed layout's record."""
    from paper_2003_01178_amd import rocprof_summary
    name = "star_kernel_120M_bitpacked_traffic.json" if packed else "star_kernel_120M_traffic.json"
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", name)
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != rocprof_summary.source_hash():
        return None
    if rec.get("fact_rows", n) != n or rec.get("join_order", list(order)) != list(order):
        return None
    return rec.get("traffic_bytes")


def settle(fn, torch, seconds, chunk=50):
    """Call ``fn`` untimed, ``chunk`` calls between synchronizations, until ``seconds`` have passed.

    After idle the GPU's clocks take tens of milliseconds of work to reach their steady state, so a
    timed region of a few milliseconds right after start-up would measure that ramp and not the
    kernels.  Returns the number of calls made (0 when ``seconds`` is 0)."""
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(chunk):
            fn()
        torch.cuda.synchronize()
        n += chunk
    return n


def settle_record(n, seconds):
    return {"steps": n, "seconds": seconds,
            "note": "untimed steps before the warmup steps, so that the timed ones run at steady GPU clocks"}


class Timer:
    """HIP events around one call on the current stream, averaged."""

    def __init__(self, torch):
        self.torch = torch
        self.pairs = []

    def run(self, fn, stream=None):
        s = self.torch.cuda.Event(enable_timing=True)
        e = self.torch.cuda.Event(enable_timing=True)
        s.record(stream)
        r = fn()
        e.record(stream)
        self.pairs.append((s, e))
        return r

    def mean_ms(self):
        return float(np.mean([s.elapsed_time(e) for s, e in self.pairs])) if self.pairs else 0.0


def shared_pass_bytes(torch, mask_steps, agg_cols, reread_cols, n, line=FETCH_BYTES):
    """Algorithmic bytes of one shared-scan pass over rows [0, n): each join
    step reads its key column at the lines holding a row still alive for some
    query, the survivors' measure and group-key columns are read at their
    lines.  mask_steps: (key column, mask table as one entry per key, key_min) per step."""
    per = line // 4
    def lines(alive):
        pad = (-n) % per
        a = torch.nn.functional.pad(alive, (0, pad)) if pad else alive
        return int(a.view(-1, per).any(dim=1).sum().item())
    qm = torch.full((n,), -1, dtype=torch.int32, device="cuda")        # all queries alive
    total = 0
    for col, table, kmin in mask_steps:
        total += lines(qm != 0) * line
        off = col[:n].to(torch.int64) - kmin
        ok = (off >= 0) & (off < table.numel())
        m = torch.zeros(n, dtype=torch.int32, device="cuda")
        m[ok] = table[off[ok]].to(torch.int32) & 0xFFFF
        qm &= m
    surv = lines(qm != 0) * line
    return total + surv * (len(agg_cols) + len(reread_cols)), int((qm != 0).sum().item())


def shared_scan_roofline(torch, cx, datagen, queries, sv, seg, rng, reps):
    """Time one 16-query shared-scan pass per template over one clock
    segment with HIP events on its stream (around replays of a graph of
    passes), beside its algorithmic bytes."""
    star_c = [datagen.random_star_constants(rng) for _ in range(16)]
    q11_c = [datagen.random_q11_constants(rng) for _ in range(16)]
    sv.build_star_masks(star_c)
    sv.build_q11_masks(q11_c)
    torch.cuda.synchronize()
    d = sv.s.dims

    def mask_table(keys, filt, kmin, kmax, ranges):
        # per key of the span: bit q set when the row with that key passes query q (the
        # definition of a query-mask entry, computed here for the byte count only)
        table = torch.zeros(kmax - kmin + 1, dtype=torch.int32, device="cuda")
        m = torch.zeros_like(keys)
        for q, (lo, hi) in enumerate(ranges):
            m |= ((filt >= lo) & (filt <= hi)).to(torch.int32) << q
        table[(keys - kmin).long()] = m
        return table

    star_steps = [(sv.cols[j], mask_table(d[j]["key"], d[j]["filter"], d[j]["key_min"], d[j]["key_max"],
                                          [(c[j], c[j]) for c in star_c]), d[j]["key_min"])
                  for j in queries.DEFAULT_JOIN_ORDER]
    q11_ranges = [sv.q11_preds(*c) for c in q11_c]
    q11_steps = [(sv.cols[dm["fk_col"]], mask_table(dm["key"], dm["filter"], dm["key_min"], dm["key_max"],
                                                    [r[i] for r in q11_ranges]), dm["key_min"])
                 for i, dm in enumerate(sv.q11_domains)]
    b_star, s_star = shared_pass_bytes(torch, star_steps, [4], [0, 2], seg)
    # the Q1.1 measures: price, and discount, which its second step has read already
    b_q11, s_q11 = shared_pass_bytes(torch, q11_steps, [8], [], seg)
    # Each pass is timed inside a HIP graph of G passes, replayed with events around the
    # replays: the host marshals 16 queries' arguments per launch, which can take longer
    # than a pass, and events around single launches would then time the host.
    res = {}
    G = 10
    R = max(1, reps // G)
    gstream = torch.cuda.Stream()
    for name, scan, ng in (("star", sv.star_scan, queries.STAR_GROUPS), ("q11", sv.q11_scan, 1)):
        outs = [torch.zeros(ng, dtype=torch.int64, device="cuda") for _ in range(16)]
        st = cx.new_status()          # allocated before the capture: nothing is allocated inside it
        torch.cuda.synchronize()
        with torch.cuda.stream(gstream):
            for _ in range(2):
                scan.run([[] for _ in outs], outs, 0, seg, status=st, stream=gstream)
            with cx.Graph.capture(gstream) as graph:
                for _ in range(G):
                    scan.run([[] for _ in outs], outs, 0, seg, status=st, stream=gstream)
            graph.launch(gstream)
            gstream.synchronize()
            timer = Timer(torch)
            timer.run(lambda: [graph.launch(gstream) for _ in range(R)], gstream)
        torch.cuda.synchronize()
        cx.check_status(st)
        res[name] = timer.mean_ms() / (R * G)
    b = b_star + b_q11
    ms = res["star"] + res["q11"]
    return dict(kernel="crystal::shared_scan_kernel", achieved=b / (ms * 1e-3) / 1e9, algorithmic_bytes=b,
                kernel_ms=ms, passes={"rows": seg, "queries_per_pass": 16,
                                      "star": {"ms": res["star"], "bytes": b_star, "survivors": s_star},
                                      "q11": {"ms": res["q11"], "bytes": b_q11, "survivors": s_q11}})


def cpu_threads():
    """Host threads to use: the CPUs this process may run on, at most 16
    (one GPU's share of the host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def host_read_gbs(threads, nbytes=1 << 31, reps=3):
    """Streaming read bandwidth of the host: a max-reduction of a 2 GiB
    int32 array split over `threads` threads (numpy releases the GIL)."""
    from concurrent.futures import ThreadPoolExecutor
    x = np.ones(nbytes // 4, dtype=np.int32)
    bounds = [(x.size * i // threads, x.size * (i + 1) // threads) for i in range(threads)]
    best = 0.0
    with ThreadPoolExecutor(threads) as ex:
        for _ in range(reps):
            t0 = time.perf_counter()
            list(ex.map(lambda ab: x[ab[0]:ab[1]].max(), bounds))
            best = max(best, x.nbytes / (time.perf_counter() - t0) / 1e9)
    return best


def oracle_star_rows(oracle, cols, n_groups, threads, **kw):
    """The oracle's star query over contiguous row ranges on several threads
    (its C call releases the GIL), the partial group arrays added modulo
    2^64: the answer over all rows."""
    from concurrent.futures import ThreadPoolExecutor
    n = len(cols[0])
    bounds = [n * i // threads for i in range(threads + 1)]
    with ThreadPoolExecutor(threads) as ex:
        parts = list(ex.map(lambda ab: oracle.star([c[ab[0]:ab[1]] for c in cols], n_groups, **kw),
                            zip(bounds[:-1], bounds[1:])))
    total = np.zeros(int(n_groups), dtype=np.uint64)
    for q in parts:
        total += q.view(np.uint64)
    return total.view(np.int64)


def star_oracle_joins(t, consts, datagen, queries, order=(1, 2, 3, 0)):
    """Oracle join list of the star query (dimension j keeps filter ==
    consts[j]; group = (year - 1992) * 1000 + dim3.group), in `order`: the
    result does not depend on it, and the dense dimensions first make the
    oracle faster."""
    joins = []
    for j in order:
        d = t.dims[j]
        jj = dict(fk_col=j, key=d.key, filter=d.filter, flo=consts[j], fhi=consts[j])
        if j == 0:
            jj.update(group=d.year, base=datagen.FIRST_YEAR, stride=queries.GROUPS_PER_YEAR)
        if j == 2:
            jj.update(group=d.group, base=0, stride=1)
        joins.append(jj)
    return joins


def serve(args, torch, cx, datagen, queries):
    """Served mixed workload (600M fact rows, the star schema plus the Q1.1
    columns): Poisson arrivals of star-template and Q1.1-template queries
    with seeded constants, answered by the continuous-batching server over
    shared-scan passes, beside one launch per query.  Returns the `serving`
    object and the shared-scan pass roofline."""
    import oracle
    n = args.serve_rows or 600_000_000
    t0 = time.time()
    t = datagen.star_tables(n=n, workload=4, with_q11_columns=True)
    print(f"# serve: generated {n} fact rows x 9 columns in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    sv = queries.ServingTemplates(queries.StarSchema(t))
    torch.cuda.synchronize()
    rng = np.random.default_rng(2003)

    def draw(k):
        if k % 2 == 0:
            return 0, datagen.random_star_constants(rng)
        return 1, datagen.random_q11_constants(rng)

    def single(tp, c):
        return sv.single_star(c) if tp == 0 else sv.single_q11(*c)

    # one launch per query, back to back: each query's own latency (filtered
    # builds + fused kernel, or the Q1.1 kernel, to a synchronised result)
    for k in range(4):
        single(*draw(k))
    torch.cuda.synchronize()
    single_lat = []
    for k in range(64):
        tp, c = draw(k)
        q0 = time.perf_counter()
        single(tp, c)
        torch.cuda.synchronize()
        single_lat.append(time.perf_counter() - q0)
    single_lat = np.array(single_lat) * 1e3
    single_qps = len(single_lat) / (single_lat.sum() / 1e3)
    seg = (n // args.segments + 3) // 4 * 4
    srv = cx.Server(sv.server_templates(), slots=16, segment_rows=seg, max_queue=1 << 16, inflight=2)
    per_rate = []
    answers = []            # (template, constants, served answer), sampled for the checks
    try:
        for rate in [float(x) for x in args.rates.split(",")]:
            window = args.seconds if args.seconds > 0 else min(10.0, max(5.0, 5000.0 / rate))
            arrivals = np.cumsum(rng.exponential(1.0 / rate, size=int(rate * window * 1.3) + 16))
            arrivals = arrivals[arrivals < window]
            pending, lat, sampled = {}, [], 0
            st0 = srv.stats()
            start = time.perf_counter()
            i = 0
            while i < len(arrivals) or pending:
                now = time.perf_counter() - start
                while i < len(arrivals) and arrivals[i] <= now:
                    tp, c = draw(i)
                    tk = srv.submit(0, **sv.star_request(c)) if tp == 0 else srv.submit(1, **sv.q11_request(*c))
                    if tk is not None:
                        pending[tk] = (tp, c)
                    i += 1
                for tk in list(pending):
                    done, out, ns = srv.poll(tk)
                    if done:
                        lat.append(ns / 1e6)
                        tp, c = pending.pop(tk)
                        if sampled < 40 and len(lat) % 5 == 1:      # 40 answers per rate
                            answers.append((tp, c, out))
                            sampled += 1
                time.sleep(0.0002)
            wall = time.perf_counter() - start
            st1 = srv.stats()
            steps = st1["steps"] - st0["steps"]
            lat = np.array(lat)
            per_rate.append({"offered_qps": rate, "window_s": window, "queries": int(lat.size),
                             "served_qps": lat.size / wall,
                             "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                             "clock_steps": int(steps),
                             "mean_batch": (st1["busy_slot_steps"] - st0["busy_slot_steps"]) / max(1, steps)})
            print(f"# serve: rate {rate}: {per_rate[-1]}", file=sys.stderr, flush=True)
        # saturation: a burst of 256 queries submitted at once
        tks = {}
        start = time.perf_counter()
        for k in range(256):
            tp, c = draw(k)
            tk = srv.submit(0, **sv.star_request(c)) if tp == 0 else srv.submit(1, **sv.q11_request(*c))
            tks[tk] = (tp, c)
        burst_lat = []
        while tks:
            for tk in list(tks):
                done, out, ns = srv.poll(tk)
                if done:
                    burst_lat.append(ns / 1e6)
                    tks.pop(tk)
            time.sleep(0.0002)
        burst_qps = 256 / (time.perf_counter() - start)
    finally:
        srv.close()
    print(f"# serve: burst {burst_qps:.0f} q/s; checking answers", file=sys.stderr, flush=True)
    # every sampled served answer against its own single launch
    mism_single = 0
    for tp, c, out in answers:
        want = single(tp, c)
        mism_single += int(not np.array_equal(out, want.cpu().numpy().reshape(-1)))
    # twenty against the oracle (ten per template), over all 600M rows
    threads = cpu_threads()
    cols = [*t.fk, t.m1, t.m2]
    q11_cols = [t.fk[0], t.extra["discount"], t.extra["quantity"], t.extra["price"]]
    mism_oracle = n_oracle = 0
    o0 = time.perf_counter()
    for want_tp in (0, 1):
        for tp, c, out in [a for a in answers if a[0] == want_tp][:10]:
            if tp == 0:
                want = oracle_star_rows(oracle, cols, queries.STAR_GROUPS, threads, agg=oracle.AGG_SUM,
                                        agg_cols=(4, 0), joins=star_oracle_joins(t, c, datagen, queries))
            else:
                year, d, qm = c
                lo, hi = datagen.q11_year_range(year)
                want = oracle_star_rows(oracle, q11_cols, 1, threads, agg=oracle.AGG_SUM_PRODUCT, agg_cols=(3, 1),
                                        preds=[(0, lo, hi), (1, d, d + 2), (2, datagen.INT32_MIN, qm)])
            n_oracle += 1
            mism_oracle += int(not np.array_equal(out, want))
    print(f"# serve: {n_oracle} oracle checks in {time.perf_counter() - o0:.1f}s", file=sys.stderr, flush=True)
    pass_roof = shared_scan_roofline(torch, cx, datagen, queries, sv, seg, rng, args.serve_pass_reps)
    pass_roof["frac"] = pass_roof["achieved"] / HBM_PEAK_GBS
    del sv
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return {"workload": f"served mix: fact {n} rows x 9 int32 columns resident in HBM, 50/50 star-join / "
                        "Q1.1 templates with seeded constants, Poisson arrivals",
            "fact_rows": n, "segments": args.segments, "slots_per_template": 16,
            "rates": per_rate, "burst_256": {"qps": burst_qps, "p50_ms": float(np.percentile(burst_lat, 50)),
                                             "p99_ms": float(np.percentile(burst_lat, 99))},
            "single_launch": {"qps": single_qps, "p50_ms": float(np.percentile(single_lat, 50)),
                              "p99_ms": float(np.percentile(single_lat, 99)), "queries": int(single_lat.size),
                              "note": "one query at a time, back to back: its own latency, no queueing; "
                                      "offered rates above this q/s would queue without bound"},
            "checked_vs_single_launch": len(answers), "mismatches_vs_single_launch": mism_single,
            "checked_vs_oracle": n_oracle, "mismatches_vs_oracle": mism_oracle,
            "pass_roofline": pass_roof}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1 (the path would shard "
                                   "by fact row ranges, one share per GPU)",
                          "requested_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2003_01178_amd import crystal as cx
    from paper_2003_01178_amd import datagen, queries

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(3)
    cx.load()
    kernel_id = {"star": cx.K_STAR, "q11": cx.K_STAR, "select": cx.K_SELECT, "project": cx.K_PROJECT,
                 "join": cx.K_HT_PROBE, "copy": cx.K_SELECT, "serve": cx.K_SHARED_SCAN, "pass": cx.K_SHARED_SCAN,
                 "partition": cx.K_RADIX, "sort": cx.K_RADIX, "groupby": cx.K_GROUPBY}[args.workload]
    if args.tune:
        b, i, g = (int(x) for x in args.tune.split(","))
        cx.tune_set(kernel_id, b, i, g)
    model, ncpu = host_info()
    print(f"# host: {model}, {ncpu} logical CPUs; device: {torch.cuda.get_device_name(0)}",
          file=sys.stderr, flush=True)

    W, K = args.warmup, args.steps
    result = {"n_gpus": 1, "steps": K, "warmup": W, "higher_is_better": True, "scaling": "weak",
              "vs_baseline": None, "data": "synthetic"}
    roof = {"bound": "hbm", "peak": HBM_PEAK_GBS, "unit": "GB/s", "traffic": None,
            "fetch_bytes_model": FETCH_BYTES}
    cpu = None
    n_settle = None

    if args.workload == "star":
        n = args.rows or 120_000_000
        order = tuple(int(x) for x in args.order.split(","))
        t0 = time.time()
        t = datagen.star_tables(n=n, workload=3)
        print(f"# generated {n} fact rows in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
        s = queries.StarSchema(t)
        bits = None
        if args.narrow:
            # compressed layout (bit-packed): the date keys as 12-bit dictionary codes (the day's index
            # from 1992-01-01, with the date table keyed by that code) and fk1 (0..39,999) as 16 bits
            fk0, st0 = cx.pack_column_bits(queries.to_dev(datagen.day_codes(t.fk[0])), 0, 12)
            fk1, st1 = cx.pack_column_bits(s.fk[1], 0, 16)
            cx.check_status(st0)
            cx.check_status(st1)
            codes0 = queries.to_dev(datagen.day_codes(t.dims[0].key))
            bits = [12, 16, 32, 32]

        def table_set():
            """One set of the four dimension tables, their filtered build items and the plan over them."""
            tables = s.new_tables()
            items = s.build_items(tables=tables)
            plan = s.plan(order, tables=tables)
            if args.narrow:
                d0 = s.dims[0]
                tables[0] = cx.HashTable(cx.HT_DIRECT, d0["n"], 0, datagen.N_DAYS - 1, has_payload=True)
                items[0] = (tables[0], codes0, d0["year"], d0["filter"], (t.consts[0], t.consts[0]))
                joins = [dict(jj, table=tables[0]) if jj["fk_col"] == 0 else jj for jj in plan.joins]
                plan = cx.StarQuery([fk0, fk1, s.fk[2], s.fk[3], s.m1, s.m2], n_groups=queries.STAR_GROUPS,
                                    joins=joins, agg=cx.AGG_SUM, agg_cols=(4, 0))
            return tables, items, plan

        # Two table sets used in turn: a step's single build launch builds one set (cleared by the
        # previous step), clears the other set for the next step and zeroes the group array; the
        # fused kernel then adds into it.  A step is two launches instead of four.
        sets = [table_set(), table_set()]
        out = torch.empty(queries.STAR_GROUPS, dtype=torch.int64, device="cuda")
        status = cx.new_status()
        stream = torch.cuda.Stream()
        torch.cuda.synchronize()
        k_step = [0]

        # each set's build launch, its arguments marshalled once
        builds = [cx.BuildBatch(sets[p][1], clear=sets[1 - p][0], zero=out, status=s.status) for p in (0, 1)]

        def run_step(p):
            builds[p].launch(stream)
            sets[p][2].run(out=out, status=status, stream=stream, accumulate=True)

        with torch.cuda.stream(stream):
            cx.build_tables_fused([], clear=sets[0][0] + sets[1][0], status=s.status, stream=stream)
            run_step(0)                                 # eager first: caches device attributes
            run_step(1)
            # a step = the four filtered builds (with the other set's clear and the output's), then
            # the fused kernel.  By default both are launched on the stream one step after the other:
            # the host runs ahead of the GPU, which then starts each kernel as the previous one ends.
            # With --graph the steps are replayed as HIP graphs, one per period of the two sets (a
            # step on each, from either set), and one per set for an odd step; the GPU idles about
            # 8 us between graph replays, so this is about 2.5 us per step slower.
            use_graph = args.graph
            if use_graph:
                graphs, pairs = [], []
                for p in (0, 1):
                    with cx.Graph.capture(stream) as g:
                        run_step(p)
                    graphs.append(g)
                for p in (0, 1):
                    with cx.Graph.capture(stream) as g:
                        run_step(p)
                        run_step(1 - p)
                    pairs.append(g)

            def steps(m):
                """m steps, continuing the alternation of the table sets."""
                i = 0
                while i < m:
                    p = k_step[0] % 2
                    if use_graph and m - i >= 2:
                        pairs[p].launch(stream)
                        k_step[0] += 2
                        i += 2
                        continue
                    if use_graph:
                        graphs[p].launch(stream)
                    else:
                        run_step(p)
                    k_step[0] += 1
                    i += 1

            n_settle = 2 * settle(lambda: steps(2), torch, args.settle)
            steps(W)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            steps(K)
            torch.cuda.synchronize()
            elapsed = time.perf_counter() - t0
            # the kernel's own duration: HIP events on its stream around K back-to-back eager
            # launches of the fused kernel alone (the query accumulates into the group array,
            # so nothing else runs between the events), averaged per launch
            plan = sets[(k_step[0] - 1) % 2][2]                 # the set the last step built
            timer = Timer(torch)
            timer.run(lambda: [plan.run(out=out, status=status, stream=stream, accumulate=True)
                               for _ in range(K)], stream)
            torch.cuda.synchronize()
            plan.run(out=out, status=status, stream=stream)      # the result checked below
            torch.cuda.synchronize()
        cx.check_status(status)
        cx.check_status(s.status)
        kern_ms = timer.mean_ms() / K
        alg_bytes, survivors = star_algorithmic_bytes(t, order, bits=bits)
        alg_bytes_c64, _ = star_algorithmic_bytes(t, order, line=64, bits=bits)
        gpu_out = out.cpu().numpy()
        result.update(metric="fact rows/s & % HBM peak (fused star query); served queries/s + p99 latency",
                      value=n * K / elapsed, unit="rows/s", ms_per_step=elapsed / K * 1e3, dtype="int32",
                      config={"workload": "fused star query: fact 120M rows x (4 int32 FKs + 2 int32 "
                                          "measures), 4 dims (2556/40000/200000/600000 rows) filtered "
                                          "to ~1/25 each, group by (year, dim3.group) -> 7000 int64",
                              "fact_rows": n, "join_order": list(order), "survivors": survivors,
                              "tile": list(cx.tune_get(cx.K_STAR, n)),
                              "step": "4 filtered dimension builds (one launch, which also clears the other "
                                      "table set and the group array) + fused probe/aggregate kernel",
                              "launch": ("hip graphs: one per pair of steps (one on each table set), one "
                                         "for an odd step") if use_graph else
                                        "two launches per step on one stream, the host ahead of the GPU",
                              "columns": ("fk0 12-bit date codes, fk1 16-bit, bit-packed; others int32" if args.narrow
                                          else "int32")})
        result["settle"] = settle_record(n_settle, args.settle)
        roof.update(kernel="crystal::star_kernel", achieved=alg_bytes / (kern_ms * 1e-3) / 1e9,
                    algorithmic_bytes=alg_bytes, bytes_per_row=alg_bytes / n, kernel_ms=kern_ms,
                    kernel_rows_per_s=n / (kern_ms * 1e-3), algorithmic_bytes_c64=alg_bytes_c64,
                    frac_c64=alg_bytes_c64 / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS)
        roof["traffic"] = measured_traffic(order, n, packed=args.narrow)
        if not args.no_cpu_baseline:
            import oracle
            from_cols = [*t.fk, t.m1, t.m2]
            # the oracle runs the GPU plan's join order (any order gives the same result)
            joins = star_oracle_joins(t, t.consts, datagen, queries, order=order)
            budget = args.cpu_seconds / 2
            passes, c0 = 0, time.perf_counter()
            while True:
                want = oracle.star(from_cols, queries.STAR_GROUPS, joins=joins, agg=oracle.AGG_SUM, agg_cols=(4, 0))
                passes += 1
                if time.perf_counter() - c0 >= budget or passes >= 20:
                    break
            one = n * passes / (time.perf_counter() - c0)
            threads = cpu_threads()
            apasses, c0 = 0, time.perf_counter()
            while True:
                want_all = oracle_star_rows(oracle, from_cols, queries.STAR_GROUPS, threads, joins=joins,
                                            agg=oracle.AGG_SUM, agg_cols=(4, 0))
                apasses += 1
                if time.perf_counter() - c0 >= budget or apasses >= 50:
                    break
            allc = n * apasses / (time.perf_counter() - c0)
            read_gbs = host_read_gbs(threads)
            cpu = {"value": allc, "unit": "rows/s", "cores": threads, "kind": "oracle",
                   "sample": f"{apasses} full pass(es) over the {n}-row fact table, rows split over {threads} "
                             f"threads; single thread: {passes} pass(es)",
                   "single_thread_value": one, "host": model, "host_logical_cpus": ncpu,
                   "host_read_GBps": read_gbs,
                   "gpu_over_cpu_bandwidth": HBM_PEAK_GBS / read_gbs,
                   "paper_bandwidth_ratio": "16.2x (880 GB/s V100 over 54 GB/s i7-6900)"}
            result["exact_vs_oracle"] = bool(np.array_equal(gpu_out, want) and np.array_equal(gpu_out, want_all))
        result["paper_context"] = ("SSB q2.1 (3 joins, 120M rows) on V100: 3.86 ms = 3.1e10 rows/s; "
                                   "GPU/CPU 25x on SSB (different hardware and workload)")
        if not args.no_serve:
            del s, plan, t, sets
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            result["serving"] = serve(args, torch, cx, datagen, queries)

    elif args.workload == "q11":
        n = args.rows or 6_000_000
        f = datagen.q11_fact(n, workload=0)
        cols = [queries.to_dev(c) for c in (f.datekey, f.discount, f.quantity, f.price)]
        plan = queries.Q11Plan(*cols)
        out = torch.empty(1, dtype=torch.int64, device="cuda")
        status = cx.new_status()
        n_settle = settle(lambda: plan.run(out=out, status=status), torch, args.settle)
        for _ in range(W):
            plan.run(out=out, status=status)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(K):
            plan.run(out=out, status=status)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        # the kernels' own time per query (the fused kernel and its finalize): a HIP graph of G
        # back-to-back launches, replayed, with events around the replays on the graph's stream.
        # A step here is shorter than the host's launch call, so events around single launches
        # would measure the host's latency instead.
        G = 50
        reps = max(1, K // G)
        gstream = torch.cuda.Stream()
        with torch.cuda.stream(gstream):
            with cx.Graph.capture(gstream) as graph:
                for _ in range(G):
                    plan.run(out=out, status=status, stream=gstream)
            for _ in range(2):
                graph.launch(gstream)
            gstream.synchronize()
            timer = Timer(torch)
            timer.run(lambda: [graph.launch(gstream) for _ in range(reps)], gstream)
        torch.cuda.synchronize()
        cx.check_status(status)
        kern_ms = timer.mean_ms() / (reps * G)
        lo, hi = datagen.q11_year_range(1994)
        m = (f.datekey >= lo) & (f.datekey <= hi)
        b = lines_touched(np.ones(n, bool)) * FETCH_BYTES + lines_touched(m) * FETCH_BYTES
        m &= (f.discount >= 1) & (f.discount <= 3)
        b += lines_touched(m) * FETCH_BYTES
        m &= f.quantity <= 24
        b += lines_touched(m) * FETCH_BYTES * 2          # price and the discount re-read
        result.update(metric="fact rows/s (SSB Q1.1-shaped selection-scan-aggregate)", value=n * K / elapsed,
                      unit="rows/s", ms_per_step=elapsed / K * 1e3, dtype="int32",
                      config={"workload": "Q1.1 shape: 6M rows, 3 range predicates, SUM(price*disc)",
                              "fact_rows": n})
        result["settle"] = settle_record(n_settle, args.settle)
        roof.update(kernel="crystal::star_kernel", achieved=b / (kern_ms * 1e-3) / 1e9, algorithmic_bytes=b,
                    kernel_ms=kern_ms, kernel_ms_covers="the fused kernel and its scalar finalize kernel, "
                                                        "per query, from graph replays of 50 queries")

    elif args.workload == "select":
        n = args.rows or (1 << 29)
        y = datagen.select_column(n)
        x = queries.to_dev(y)
        lo, hi = datagen.select_threshold_range(args.sigma)
        outb = torch.empty(n, dtype=torch.int32, device="cuda")
        cnt = torch.empty(1, dtype=torch.int64, device="cuda")
        n_settle = settle(lambda: cx.select(x, lo, hi, out=outb, count=cnt), torch, args.settle)
        for _ in range(W):
            cx.select(x, lo, hi, out=outb, count=cnt)
        torch.cuda.synchronize()
        timer = Timer(torch)
        t0 = time.perf_counter()
        for _ in range(K):
            timer.run(lambda: cx.select(x, lo, hi, out=outb, count=cnt))
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        c = int(cnt.item())
        kern_ms = timer.mean_ms()
        b = 4 * n + 4 * c
        sweep = []
        if args.sigma_sweep:
            for k in range(11):
                slo, shi = datagen.select_threshold_range(k / 10)
                for _ in range(3):
                    cx.select(x, slo, shi, out=outb, count=cnt)
                st = Timer(torch)
                for _ in range(K):
                    st.run(lambda: cx.select(x, slo, shi, out=outb, count=cnt))
                torch.cuda.synchronize()
                sc = int(cnt.item())
                sms = st.mean_ms()
                sweep.append({"sigma": k / 10, "matches": sc, "kernel_ms": sms,
                              "GBps": (4 * n + 4 * sc) / (sms * 1e-3) / 1e9,
                              "frac": (4 * n + 4 * sc) / (sms * 1e-3) / 1e9 / HBM_PEAK_GBS})
                print(f"# sigma {k / 10}: {sweep[-1]}", file=sys.stderr, flush=True)
        result.update(metric="rows/s (selection, compacted output)", value=n * K / elapsed, unit="rows/s",
                      ms_per_step=elapsed / K * 1e3, dtype="int32",
                      config={"workload": f"select y < v on 2^29 int32, sigma={args.sigma}", "rows": n,
                              "matches": c, "tile": list(cx.tune_get(cx.K_SELECT, n))})
        result["settle"] = settle_record(n_settle, args.settle)
        if sweep:
            result["sigma_sweep"] = sweep
        roof.update(kernel="crystal::select_kernel", achieved=b / (kern_ms * 1e-3) / 1e9, algorithmic_bytes=b,
                    kernel_ms=kern_ms)

    elif args.workload == "project":
        n = args.rows or (1 << 29)
        x1h, x2h = datagen.project_columns(n)
        x1, x2 = queries.to_dev(x1h), queries.to_dev(x2h)
        outp = torch.empty(n, dtype=torch.float32, device="cuda")
        n_settle = settle(lambda: cx.project(x1, x2, 2.0, 3.0, out=outp), torch, args.settle)
        for _ in range(W):
            cx.project(x1, x2, 2.0, 3.0, out=outp)
        torch.cuda.synchronize()
        timer = Timer(torch)
        t0 = time.perf_counter()
        for _ in range(K):
            timer.run(lambda: cx.project(x1, x2, 2.0, 3.0, out=outp))
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        kern_ms = timer.mean_ms()
        b = 12 * n
        result.update(metric="rows/s (projection 2*x1 + 3*x2)", value=n * K / elapsed, unit="rows/s",
                      ms_per_step=elapsed / K * 1e3, dtype="f32",
                      config={"workload": "project 2*x1+3*x2 on 2^29 fp32", "rows": n,
                              "tile": list(cx.tune_get(cx.K_PROJECT, n))})
        roof.update(kernel="crystal::project_kernel", achieved=b / (kern_ms * 1e-3) / 1e9, algorithmic_bytes=b,
                    kernel_ms=kern_ms)

    elif args.workload == "join":
        n = args.rows or (1 << 28)
        d = args.dim
        jt = datagen.join_tables(d, n_probe=n)
        kind = cx.HT_LINEAR if args.kind == "linear" else cx.HT_DIRECT
        ht = cx.HashTable(kind, d, 0, d - 1)
        keys, vals, fk = queries.to_dev(jt.dim_key), queries.to_dev(jt.dim_val), queries.to_dev(jt.fk)
        st = ht.build(keys, vals)
        res = torch.empty(2, dtype=torch.int64, device="cuda")
        n_settle = settle(lambda: ht.probe(fk, out=res), torch, args.settle)
        for _ in range(W):
            ht.probe(fk, out=res)
        torch.cuda.synchronize()
        cx.check_status(st)
        timer = Timer(torch)
        t0 = time.perf_counter()
        for _ in range(K):
            timer.run(lambda: ht.probe(fk, out=res))
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        kern_ms = timer.mean_ms()
        # A table that fits in the 256 MB last-level cache (the Infinity Cache
        # in front of HBM) costs HBM nothing per probe after its first touch:
        # such probes are bound by the cache's random-access rate, and the
        # HBM bytes are the key stream alone.  A larger table costs one
        # 128-byte line per probe (section 4.3's model).
        llc_resident = ht.nbytes <= LLC_BYTES
        b = 4 * n + (0 if llc_resident else n * FETCH_BYTES)
        if llc_resident:
            roof["note"] = "table resident in the last-level cache: probes are bound by its random-access rate"
        result.update(metric="probes/s (hash join probe + sum)", value=n * K / elapsed, unit="probes/s",
                      ms_per_step=elapsed / K * 1e3, dtype="int32",
                      config={"workload": f"join probe: D={d} ({args.kind}, table {ht.nbytes} B), 2^28 probes",
                              "probes": n, "table_bytes": ht.nbytes, "tile": list(cx.tune_get(cx.K_HT_PROBE, n))})
        roof.update(kernel="crystal::ht_probe_kernel", achieved=b / (kern_ms * 1e-3) / 1e9, algorithmic_bytes=b,
                    kernel_ms=kern_ms)

    elif args.workload == "copy":
        # calibration: a plain device-to-device copy of known size (read n*4, write n*4 bytes)
        n = args.rows or (1 << 28)
        src = torch.arange(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(W):
            dst.copy_(src)
        torch.cuda.synchronize()
        timer = Timer(torch)
        t0 = time.perf_counter()
        for _ in range(K):
            timer.run(lambda: dst.copy_(src))
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        kern_ms = timer.mean_ms()
        b = 8 * n
        result.update(metric="bytes/s (plain copy, calibration)", value=b * K / elapsed, unit="B/s",
                      ms_per_step=elapsed / K * 1e3, dtype="int32",
                      config={"workload": f"device copy of {n} int32 ({4 * n} bytes read, {4 * n} written)",
                              "rows": n})
        roof.update(kernel="copy", achieved=b / (kern_ms * 1e-3) / 1e9, algorithmic_bytes=b, kernel_ms=kern_ms)

    elif args.workload == "pass":
        # one 16-query shared-scan pass per template over one clock segment of
        # the served table, timed alone (for kernel traces and counters)
        n = args.serve_rows or 600_000_000
        t = datagen.star_tables(n=n, workload=4, with_q11_columns=True)
        sv = queries.ServingTemplates(queries.StarSchema(t))
        del t
        seg = (n // args.segments + 3) // 4 * 4
        pr = shared_scan_roofline(torch, cx, datagen, queries, sv, seg, np.random.default_rng(2003), K)
        roof.update({k: pr[k] for k in ("kernel", "achieved", "algorithmic_bytes", "kernel_ms", "passes")})
        result.update(metric="rows/s per shared-scan pass pair (16 queries per template)",
                      value=seg / (pr["kernel_ms"] * 1e-3), unit="rows/s", ms_per_step=pr["kernel_ms"],
                      dtype="int32", config={"workload": f"one 16-query pass per template over {seg} of {n} "
                                                         "served fact rows", "rows": seg})

    elif args.workload == "serve":
        serving = serve(args, torch, cx, datagen, queries)
        pr = serving["pass_roofline"]
        roof.update({k: pr[k] for k in ("kernel", "achieved", "algorithmic_bytes", "kernel_ms", "passes")})
        b = serving["burst_256"]["qps"]
        result.update(metric="served queries/s + p99 latency (shared-scan continuous batching)", value=b,
                      unit="queries/s", ms_per_step=1e3 / b, dtype="int32",
                      config={"workload": serving["workload"], "segments": args.segments,
                              "slots_per_template": 16},
                      serving=serving)

    elif args.workload == "groupby":
        # dense group-by SUM(v) GROUP BY g: 2^28 rows into 7,000 groups (the star query's group array)
        n = args.rows or (1 << 28)
        rng = np.random.default_rng(datagen.BASE_SEED + 13)
        g = queries.to_dev(rng.integers(0, 7000, size=n, dtype=np.int32))
        v = queries.to_dev(rng.integers(1, 1_000_001, size=n, dtype=np.int32))
        o = torch.empty(7000, dtype=torch.int64, device="cuda")
        st = cx.new_status()
        n_settle = settle(lambda: cx.groupby_agg(g, v, 7000, out=o, status=st), torch, args.settle)
        for _ in range(W):
            cx.groupby_agg(g, v, 7000, out=o, status=st)
        torch.cuda.synchronize()
        timer = Timer(torch)
        t0 = time.perf_counter()
        for _ in range(K):
            timer.run(lambda: cx.groupby_agg(g, v, 7000, out=o, status=st))
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        cx.check_status(st)
        kern_ms = timer.mean_ms()
        b = 8 * n
        result.update(metric="rows/s (dense group-by, 7000 int64 groups)", value=n * K / elapsed, unit="rows/s",
                      ms_per_step=elapsed / K * 1e3, dtype="int32",
                      config={"workload": "SUM(v) GROUP BY g, 2^28 rows, g U{0..6999}", "rows": n,
                              "tile": list(cx.tune_get(cx.K_GROUPBY, n))})
        roof.update(kernel="crystal::groupby_kernel", achieved=b / (kern_ms * 1e-3) / 1e9, algorithmic_bytes=b,
                    kernel_ms=kern_ms)

    elif args.workload in ("partition", "sort"):
        # section 4.4: 2^28 pairs of 32-bit keys and 32-bit values
        n = args.rows or (1 << 28)
        kh, vh = datagen.radix_pairs(n)
        keys, vals = queries.to_dev(kh), queries.to_dev(vh)
        ok, ov = torch.empty_like(keys), torch.empty_like(vals)
        if args.workload == "partition":
            offs = torch.empty((1 << args.bits) + 1, dtype=torch.int32, device="cuda")
            scratch = torch.empty(cx.load().crystal_radix_partition_scratch_bytes(n), dtype=torch.uint8,
                                  device="cuda")
            call = lambda: cx.radix_partition(keys, args.shift, args.bits, vals=vals, out_keys=ok, out_vals=ov,
                                              part_offsets=offs, scratch=scratch, stable=not args.unstable)
            passes = 1
        elif args.msb:
            scratch = torch.empty(cx.load().crystal_sort_pairs_msb_scratch_bytes(n, 1), dtype=torch.uint8,
                                  device="cuda")
            call = lambda: cx.sort_pairs(keys, vals, out_keys=ok, out_vals=ov, scratch=scratch, msb=True)
            passes = 2   # uniform keys: two partition levels, then the local sort (counted below)
        else:
            scratch = torch.empty(cx.load().crystal_sort_pairs_scratch_bytes(n, 1), dtype=torch.uint8,
                                  device="cuda")
            call = lambda: cx.sort_pairs(keys, vals, out_keys=ok, out_vals=ov, scratch=scratch)
            passes = 4
        n_settle = settle(call, torch, args.settle, chunk=2)
        for _ in range(W):
            call()
        torch.cuda.synchronize()
        timer = Timer(torch)
        t0 = time.perf_counter()
        for _ in range(K):
            timer.run(call)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        kern_ms = timer.mean_ms()
        # per pass: the histogram reads the keys (4n), the shuffle reads keys and
        # values (8n) and writes them (8n); the MSB sort's local pass reads and
        # writes every pair once more (16n)
        b = passes * 20 * n + (16 * n if args.workload == "sort" and args.msb else 0)
        what = (f"radix partition ({'unstable' if args.unstable else 'stable'}) of 2^{n.bit_length() - 1} "
                f"key/value pairs on {args.bits} bits at bit {args.shift}"
                if args.workload == "partition" else
                f"radix sort ({'MSB first' if args.msb else 'LSB first'}) of {n} 32-bit key/value pairs")
        result.update(metric="pairs/s", value=n * K / elapsed, unit="pairs/s", ms_per_step=elapsed / K * 1e3,
                      dtype="u32", config={"workload": what, "pairs": n, "passes": passes,
                                           "tile": list(cx.tune_get(cx.K_RADIX, n))})
        roof.update(kernel="crystal radix pass (histogram + scan + shuffle)", achieved=b / (kern_ms * 1e-3) / 1e9,
                    algorithmic_bytes=b, kernel_ms=kern_ms)
        if not args.no_cpu_baseline and args.workload == "sort":
            import oracle
            m = 1 << 22
            t1 = time.perf_counter()
            reps = 0
            while time.perf_counter() - t1 < args.cpu_seconds or reps == 0:
                oracle.sort_pairs(kh[:m].view(np.uint32), vh[:m].view(np.uint32))
                reps += 1
            cpu_s = time.perf_counter() - t1
            cpu = {"value": m * reps / cpu_s, "unit": "pairs/s", "cores": 1, "kind": "oracle",
                   "sample": f"{reps} stable sorts of the first 2^22 pairs"}

    roof["frac"] = roof["achieved"] / roof["peak"]
    result["roofline"] = roof
    if n_settle is not None and "settle" not in result:
        result["settle"] = settle_record(n_settle, args.settle)
    if cpu is not None:
        result["cpu_baseline"] = cpu
    order = ["metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
             "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"]
    line = {k: result[k] for k in order if k in result}
    line.update({k: v for k, v in result.items() if k not in line})
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
