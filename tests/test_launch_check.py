"""The host-side launch-configuration check every kernel launch of the library
passes through (csrc/launch_check.hpp), compiled for the CPU with g++ and
called through a two-line shim."""
import ctypes as C
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1101_1427_amd", "csrc")

SHIM = r"""
#include "launch_check.hpp"
extern "C" const char *check(unsigned long long g, unsigned long long b, unsigned long long l) {
    return smc::launch_config_error(g, b, l);
}
"""


@pytest.fixture(scope="module")
def check(tmp_path_factory):
    d = tmp_path_factory.mktemp("launch_check")
    src = d / "shim.cpp"
    src.write_text(SHIM)
    so = d / "shim.so"
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-I", CSRC, str(src), "-o", str(so)],
                   check=True, capture_output=True)
    lib = C.CDLL(str(so))
    lib.check.restype = C.c_char_p
    lib.check.argtypes = [C.c_ulonglong] * 3
    return lambda g, b, l=0: (lib.check(g, b, l) or b"").decode()


def test_ordinary_configurations_pass(check):
    for g, b, l in [(1, 1, 0), (1, 1024, 0), (65536, 256, 0), (1024, 640, 160 * 1024), ((1 << 22) - 1, 1024, 0),
                    (0x7FFFFFFF, 1, 0)]:
        assert check(g, b, l) == "", (g, b, l)


def test_each_limit(check):
    assert "empty grid" in check(0, 256)
    assert "2^31-1" in check(1 << 31, 1)
    assert "workgroup size" in check(1, 0)
    assert "workgroup size" in check(1, 1025)
    assert "LDS" in check(1, 256, 160 * 1024 + 1)
    assert "2^32" in check(1 << 22, 1024)            # exactly 2^32 work-items
    assert "2^32" in check((1 << 23) + 1, 512)
