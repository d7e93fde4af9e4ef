"""When the sanitizer test runs the host tests against the sanitized library,
this checks that the binding really loaded that library (and not the
regular build).  In an ordinary run it only checks the default path."""
import os

from paper_2003_01178_amd import crystal as cx


def test_binding_loads_the_requested_library():
    cx.load()
    want = os.environ.get("CRYSTAL_EXPECT_LIB", cx.DEFAULT_LIB)
    assert os.path.realpath(cx.LIB_PATH) == os.path.realpath(want)
    maps = open("/proc/self/maps").read()
    assert os.path.realpath(want) in maps
