"""GPU serving loop: queries submitted alone and in a mix, arriving while
others are on the GPU, each answer identical to its own single-query launch
and to the CPU oracle."""
import time

import numpy as np
import pytest
import torch

from helpers import announce, q11_oracle, star_oracle
from paper_2003_01178_amd import crystal as cx
from paper_2003_01178_amd import datagen, queries

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    t = datagen.star_tables(n=1_048_576, workload=41, with_q11_columns=True)
    sv = queries.ServingTemplates(queries.StarSchema(t))
    torch.cuda.synchronize()
    return t, sv


def make_server(sv, segment_rows=262_144, slots=16, inflight=2):
    return cx.Server(sv.server_templates(), slots=slots, segment_rows=segment_rows, max_queue=4096,
                     inflight=inflight)


def wait_all(srv, tickets, timeout=60):
    res = {}
    t0 = time.time()
    while len(res) < len(tickets) and time.time() - t0 < timeout:
        for tk, tp in tickets:
            if tk in res:
                continue
            done, out, ns = srv.poll(tk, tp)
            if done:
                res[tk] = (out, ns)
        time.sleep(0.001)
    assert len(res) == len(tickets), "served queries did not finish"
    return res


def q11_of(t):
    return datagen.Q11Fact(datekey=t.fk[0], discount=t.extra["discount"], quantity=t.extra["quantity"],
                           price=t.extra["price"])


def test_single_query_alone(setup):
    announce("serve alone")
    t, sv = setup
    srv = make_server(sv)
    try:
        consts = t.consts
        tk = srv.submit(0, filters=[(consts[j], consts[j]) for j in queries.DEFAULT_JOIN_ORDER])
        res = wait_all(srv, [(tk, 0)])
        out, ns = res[tk]
        assert np.array_equal(out, star_oracle(t, consts)[0])
        assert ns > 0
    finally:
        srv.close()


def test_mixed_queries_match_single_launch_and_oracle(setup):
    announce("serve mix")
    t, sv = setup
    f = q11_of(t)
    rng = np.random.default_rng(5)
    srv = make_server(sv)
    submitted = []
    try:
        for k in range(48):
            if k % 2 == 0:
                c = datagen.random_star_constants(rng)
                tk = srv.submit(0, filters=[(c[j], c[j]) for j in queries.DEFAULT_JOIN_ORDER])
                submitted.append((tk, 0, c))
            else:
                c = datagen.random_q11_constants(rng)
                tk = srv.submit(1, **sv.q11_request(*c))
                submitted.append((tk, 1, c))
            if k % 8 == 7:
                time.sleep(0.003)                # later requests arrive while earlier ones run
        res = wait_all(srv, [(tk, tp) for tk, tp, _ in submitted])
        st = srv.stats()
        assert st["completed"] == 48
    finally:
        srv.close()
    for i, (tk, tp, c) in enumerate(submitted):
        got = res[tk][0]
        if tp == 0:
            single = sv.single_star(c).cpu().numpy()
            assert np.array_equal(got, single), (i, c)
            if i < 8:
                assert np.array_equal(got, star_oracle(t, c)[0])
        else:
            single = int(sv.single_q11(*c).item())
            assert int(got[0]) == single, (i, c)
            if i < 8:
                year, d, q = c
                assert single == q11_oracle(f, year, (d, d + 2), q)


def test_segment_sizes_do_not_change_results(setup):
    announce("serve segments")
    t, sv = setup
    rng = np.random.default_rng(6)
    consts = [datagen.random_star_constants(rng) for _ in range(6)]
    answers = []
    for seg in (1_048_576, 131_072):
        srv = make_server(sv, segment_rows=seg, slots=4, inflight=3)
        try:
            tks = [(srv.submit(0, filters=[(c[j], c[j]) for j in queries.DEFAULT_JOIN_ORDER]), 0) for c in consts]
            res = wait_all(srv, tks)
            answers.append([res[tk][0] for tk, _ in tks])
        finally:
            srv.close()
    for a, b, c in zip(answers[0], answers[1], consts):
        assert np.array_equal(a, b)
        assert np.array_equal(a, star_oracle(t, c)[0])


def test_device_error_is_reported_not_served(setup):
    """A dimension key outside its query-mask table's span makes the mask
    build set CRYSTAL_ERANGE in the server's device status word: poll and
    stats report that code instead of releasing a wrong answer."""
    announce("serve device error")
    t, sv = setup
    star = dict(sv.server_templates()[0])
    dims = list(star["dims"])
    keys, filt, n, qm = dims[0]
    bad = keys.clone()
    bad[3] = int(keys.max().item()) + 1                  # one key past the table's span
    dims[0] = (bad, filt, n, qm)
    star["dims"] = dims
    srv = cx.Server([star], slots=4, segment_rows=262_144, max_queue=16, inflight=2)
    c = t.consts
    tk = srv.submit(0, filters=[(c[j], c[j]) for j in queries.DEFAULT_JOIN_ORDER])
    with pytest.raises(cx.CrystalError) as e:
        t0 = time.time()
        while time.time() - t0 < 30:
            done, _, _ = srv.poll(tk)
            assert not done, "an answer was released despite the device error"
            time.sleep(0.001)
    assert e.value.code == cx.ERANGE
    with pytest.raises(cx.CrystalError) as e:
        srv.stats()
    assert e.value.code == cx.ERANGE
    with pytest.raises(cx.CrystalError) as e:
        srv.close()
    assert e.value.code == cx.ERANGE
