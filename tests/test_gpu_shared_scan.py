"""GPU parity of shared-scan batches: every query of a batch equals the CPU
oracle and its own single-query launch, over the whole table and over row
segments accumulated launch by launch."""
import numpy as np
import pytest
import torch

import oracle
from helpers import STAR_GROUPS, announce, q11_oracle, star_oracle
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
