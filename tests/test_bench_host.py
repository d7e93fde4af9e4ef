"""Host logic of bench.py, on the CPU: the one-GPU refusal, the settle phase
before the warmup steps, and the counting of touched cache lines behind the
algorithmic bytes of every roofline figure (int32 columns and bit-packed
fields that straddle two lines)."""
import importlib.util
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


class _FakeTorch:
    class cuda:
        @staticmethod
        def synchronize():
            pass


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    assert rec["requested_gpus"] == 2
    assert "one GPU" in rec["error"]


def test_settle_of_zero_seconds_calls_nothing():
    calls = []
    assert _bench().settle(lambda: calls.append(1), _FakeTorch, 0.0) == 0
    assert not calls


def test_settle_runs_whole_chunks_until_the_time_has_passed():
    calls = []
    n = _bench().settle(lambda: calls.append(1), _FakeTorch, 0.01, chunk=7)
    assert n == len(calls)
    assert n >= 7 and n % 7 == 0


def test_lines_touched_int32_columns():
    b = _bench()
    m = np.zeros(100, dtype=bool)      # 32 int32 per 128-byte line: four lines, the last one partial
    assert b.lines_touched(m, line=128) == 0
    m[[0, 31]] = True
    assert b.lines_touched(m, line=128) == 1
    m[32] = True
    assert b.lines_touched(m, line=128) == 2
    m[99] = True                       # the partial last line counts
    assert b.lines_touched(m, line=128) == 3
    assert b.lines_touched(np.ones(100, dtype=bool), line=128) == 4
    assert b.lines_touched(np.ones(100, dtype=bool), line=64) == 7


def test_lines_touched_bit_packed_fields():
    b = _bench()
    m = np.zeros(200, dtype=bool)      # 12-bit fields: a 128-byte line holds 1,024 bits
    m[85] = True                       # bits 1,020..1,031 cross the first line boundary
    assert b.lines_touched(m, line=128, bits=12) == 2
    m[:] = False
    m[84] = True                       # bits 1,008..1,019
    assert b.lines_touched(m, line=128, bits=12) == 1
    assert b.lines_touched(np.ones(200, dtype=bool), line=128, bits=12) == -(-200 * 12 // 1024)
