"""The internal velocity order (slots) of the stage kernels, checked on the
host: a permutation of the velocity grid that inverts exactly, lexicographic
without octants, and sign-uniform over 64-slot waves on the symmetric 16^3,
24^3 and 32^3 grids. The check program includes the kernels' own header and
is built with hipcc for the host only."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


def test_slot_order_is_a_sign_grouped_permutation():
    hipcc = _hipcc()
    if hipcc is None:
        pytest.skip("hipcc not found")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "slot_order_check")
        subprocess.run([hipcc, "-std=c++17", "-O1", "--offload-host-only", "-Wno-unused-function",
                        "-I", os.path.join(ROOT, "include"),
                        os.path.join(HERE, "slot_order_check.cpp"), "-o", exe],
                       check=True, capture_output=True, timeout=300)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout
