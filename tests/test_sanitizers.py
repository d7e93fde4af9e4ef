"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle, built with gcc's sanitizers, runs every pin.
* The HIP library's host code (argument checks, plan translation, tuning
  table, the serving loop's scheduler) is built with clang's sanitizers
  (``build.build_sanitized``) and runs the C-ABI host tests and the
  fake-executor server tests.

Each run is a subprocess with the sanitizer runtime preloaded; any report
aborts it, so a clean exit means no report.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:verify_asan_link_order=0:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _run(cmd, env_extra, timeout=600):
    env = dict(os.environ)
    env.update(SAN_ENV)
    env.update(env_extra)
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    tail = (r.stdout[-3000:] + "\n" + r.stderr[-3000:])
    assert r.returncode == 0, tail
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, tail
    return r


def test_oracle_pins_under_gcc_sanitizers(tmp_path):
    lib = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    "-o", str(lib), os.path.join(ROOT, "oracle", "crystal_oracle.c"), "-lm"], check=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    script = (
        "import sys; sys.path[:0] = ['tests', '.']\n"
        "import oracle\n"
        f"lib = oracle.load({str(lib)!r})\n"
        "from oracle_pins import ALL_PINS\n"
        "for p in ALL_PINS:\n"
        "    p(lib)\n"
        "print('pins', len(ALL_PINS))\n")
    r = _run([sys.executable, "-c", script], {"LD_PRELOAD": f"{asan}:{ubsan}"})
    assert "pins" in r.stdout


def test_library_host_code_under_clang_sanitizers(tmp_path):
    from paper_2003_01178_amd import build
    try:
        lib = build.build_sanitized(str(tmp_path / "san"))
        runtime = build.sanitizer_runtime()
    except (RuntimeError, FileNotFoundError) as e:  # pragma: no cover - depends on the toolchain
        pytest.skip(f"no sanitizer toolchain: {e}")
    r = _run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
              "tests/test_server_fake.py", "tests/test_capi_abi.py", "tests/test_sanitized_lib_loaded.py"],
             {"LD_PRELOAD": runtime, "CRYSTAL_LIB": lib, "CRYSTAL_EXPECT_LIB": lib})
    assert " passed" in r.stdout and "failed" not in r.stdout
