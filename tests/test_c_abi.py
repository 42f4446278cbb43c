"""The C ABI from a plain C program (CPU): tests/c/vgicp_example.c, built by
the package build with gcc against include/vgicp.h and libvgicp.so, runs its
checks that need no device (version, factor validation, NULL arguments, a
context on a device that does not exist)."""

import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXAMPLE = os.path.join(ROOT, "tests", "c", "vgicp_example")


def test_plain_c_client_without_a_device():
    assert os.path.exists(EXAMPLE), "tests/c/vgicp_example is not built: run the package build"
    r = subprocess.run([EXAMPLE], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    assert "no-device checks ok" in r.stdout


def test_plain_c_client_usage_error():
    r = subprocess.run([EXAMPLE, "only-one-argument"], capture_output=True, text=True,
                       timeout=60)
    assert r.returncode == 2 and "usage" in r.stderr
