"""Shared-scan batches and the server at a size where every workgroup walks
many tiles, compared query by query with the oracle.

The fact table (2^25 + 1,236 rows, the served schema) is drawn in bands of
2^19 rows whose kind is random per band (``datagen.banded_star_tables``):
dense bands, where every row passes the first two steps of both templates
for the batch's constants, sparse bands, where about one row in 500 does,
and plain bands, which also hold discount and quantity values outside the
generator's usual domains.  With one workgroup per CU a workgroup's
consecutive tiles fall into different bands, so within one launch:

* the third step's column is loaded in full with the first two (a dense
  previous tile) and selectively (a sparse previous tile), switching both
  ways;
* rows alive after the dense steps are queued per wave in sparse bands and
  carried across tiles until 64 are queued, then drained at the end;
* the first step's column of each next tile is loaded while the current
  tile runs.

Tile shapes are forced so that tiles per workgroup is at least 8 (asserted
from the host); the served default shape runs too.
"""
import time

import numpy as np
import pytest
import torch

from helpers import STAR_GROUPS, announce, q11_oracle_par, star_oracle_par
from paper_2003_01178_amd import crystal as cx
from paper_2003_01178_amd import datagen, queries

pytestmark = pytest.mark.gpu

N = (1 << 25) + 1236
BAND = 1 << 19


@pytest.fixture(scope="module")
def banded():
    announce("banded table", N)
    t, spec, kinds = datagen.banded_star_tables(N, band_rows=BAND)
    sv = queries.ServingTemplates(queries.StarSchema(t))
    rng = np.random.default_rng(77)
    # star batch: the two dense-phase joins use the band constants, the two
    # late joins vary per query
    star_consts = [[spec.c0, spec.c1, int(rng.integers(0, 25)), int(rng.integers(0, 25))] for _ in range(16)]
    # Q1.1 batch: 13 queries on the dense bands' year and discount window,
    # three whose ranges reach the out-of-domain values (discount 11..15,
    # quantity 0 and 51..60)
    q11_consts = [(spec.year, spec.disc_lo, int(rng.integers(2, 61))) for _ in range(13)]
    q11_consts += [(spec.year, 9, 55), (spec.year, 12, 60), (spec.year + 1, 13, 0)]
    star_want = [star_oracle_par(t, c) for c in star_consts]
    f = (t.fk[0], t.extra["discount"], t.extra["quantity"], t.extra["price"])
    q11_want = [q11_oracle_par(*f, y, (d, d + 2), q) for y, d, q in q11_consts]
    torch.cuda.synchronize()
    return dict(t=t, sv=sv, kinds=kinds, star=(star_consts, star_want), q11=(q11_consts, q11_want))


def cu_count():
    return torch.cuda.get_device_properties(0).multi_processor_count


def band_transitions(kinds, block, ipt, grid):
    """(dense -> sparse, sparse -> dense) transitions between consecutive
    tiles of one workgroup, over all workgroups."""
    items = block * ipt
    n_tiles = (N + items - 1) // items
    ds = sd = 0
    for w in range(grid):
        tiles = np.arange(w, n_tiles, grid, dtype=np.int64)
        k = kinds[(tiles * items) // BAND]
        ds += int(np.sum((k[:-1] == datagen.BAND_DENSE) & (k[1:] == datagen.BAND_SPARSE)))
        sd += int(np.sum((k[:-1] == datagen.BAND_SPARSE) & (k[1:] == datagen.BAND_DENSE)))
    return ds, sd


SHAPES = [(256, 8, 1), (1024, 16, 1), (64, 4, 2), None]


def force_shape(shape, kinds):
    cx.tune_reset()
    if shape is None:
        return
    block, ipt, gpc = shape
    for k in (cx.K_SHARED_SCAN, cx.K_SHARED_SCAN_SCALAR):
        cx.tune_set(k, block, ipt, gpc)
    n_tiles = (N + block * ipt - 1) // (block * ipt)
    grid = gpc * cu_count()
    assert n_tiles / grid >= 8, (shape, n_tiles, grid)
    ds, sd = band_transitions(kinds, block, ipt, grid)
    assert ds > 0 and sd > 0, (shape, ds, sd)


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "default" if s is None else "x".join(map(str, s)))
def test_star_batch_full_size(banded, shape):
    announce("shared star full", shape)
    sv = banded["sv"]
    consts, want = banded["star"]
    try:
        force_shape(shape, banded["kinds"])
        sv.build_star_masks(consts)
        outs = [torch.zeros(STAR_GROUPS, dtype=torch.int64, device="cuda") for _ in consts]
        cx.check_status(sv.run_star_batch(outs))
        cx.check_status(sv.status)
        for q in range(16):
            assert np.array_equal(outs[q].cpu().numpy(), want[q]), (shape, q, consts[q])
    finally:
        cx.tune_reset()


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "default" if s is None else "x".join(map(str, s)))
def test_q11_batch_full_size(banded, shape):
    announce("shared q11 full", shape)
    sv = banded["sv"]
    consts, want = banded["q11"]
    try:
        force_shape(shape, banded["kinds"])
        outs = [torch.zeros(1, dtype=torch.int64, device="cuda") for _ in consts]
        cx.check_status(sv.run_q11_batch(consts, outs))
        cx.check_status(sv.status)
        for q in range(16):
            assert int(outs[q].item()) == want[q], (shape, q, consts[q])
    finally:
        cx.tune_reset()


def test_q11_domains_cover_the_columns(banded):
    """The value -> query-mask tables of the Q1.1 template span each
    column's own minimum to maximum (discount 0..15, quantity 0..60 here)."""
    sv = banded["sv"]
    t = banded["t"]
    for dm, col in zip(sv.q11_domains, (t.fk[0], t.extra["discount"], t.extra["quantity"])):
        assert dm["key_min"] == int(col.min()) and dm["key_max"] == int(col.max())
    assert sv.q11_domains[1]["key_max"] == 15 and sv.q11_domains[2]["key_min"] == 0
    # the date domain is the column's distinct values, in a rank-compressed table
    date = sv.q11_domains[0]
    assert np.array_equal(date["key"].cpu().numpy(), np.unique(t.fk[0]))
    assert date["mask"].ranked == len(np.unique(t.fk[0]))


def test_server_full_size_ragged_segments(banded):
    """The server over the whole table in segments of 3,000,004 rows (not a
    multiple of any tile), all 32 queries at once: every answer equals the
    oracle's."""
    announce("serve full size")
    sv = banded["sv"]
    s_consts, s_want = banded["star"]
    q_consts, q_want = banded["q11"]
    cx.tune_reset()
    srv = cx.Server(sv.server_templates(), slots=16, segment_rows=3_000_004, max_queue=64, inflight=2)
    try:
        tickets = [(srv.submit(0, **sv.star_request(c)), 0, i) for i, c in enumerate(s_consts)]
        tickets += [(srv.submit(1, **sv.q11_request(*c)), 1, i) for i, c in enumerate(q_consts)]
        res = {}
        t0 = time.time()
        while len(res) < len(tickets) and time.time() - t0 < 60:
            for tk, tp, i in tickets:
                if tk not in res:
                    done, out, _ = srv.poll(tk)
                    if done:
                        res[tk] = out
            time.sleep(0.001)
        assert len(res) == len(tickets), "served queries did not finish"
        assert srv.stats()["n_segments"] == (N + 3_000_003) // 3_000_004
    finally:
        srv.close()
    for tk, tp, i in tickets:
        if tp == 0:
            assert np.array_equal(res[tk], s_want[i]), ("star", i)
        else:
            assert int(res[tk][0]) == q_want[i], ("q11", i, q_consts[i])
