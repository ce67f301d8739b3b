"""Planted mistakes in a scratch copy of the oracle fail its pins (CPU only).

Each case copies oracle/bgk_oracle.c into a temporary directory, plants one
plausible mistake by a textual substitution, builds the copy with the
oracle's own flags, and runs the pin that has to catch it in a child process
whose BGK_ORACLE_LIB names the mutated build: the child must fail. The
unmodified oracle passes the same pins (tests/test_oracle_pins_multid.py).

  per-axis scale   the transport takes 2/h_x on every axis: the
                   multi-dimensional free-streaming pin (exact shifted
                   solution on an anisotropic mesh) fails;
  limiter          beta halved, so every contracted slice is over-contracted:
                   the limiter-optimality pin (minimum exactly zero) fails;
  specular walls   the mirror always flips u_x: the y-wall mirror-image pin
                   fails.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "bgk_oracle.c")

MUTATIONS = {
    "per_axis_scale": ("    double sk = 2.0 / op->h[k];", "    double sk = 2.0 / op->h[0];",
                       "tests/test_oracle_pins_multid.py::test_free_streaming_multid_exact_order[2-1]"),
    "limiter_beta": ("    double beta = fabs(mean / (mean - fmin));",
                     "    double beta = 0.5 * fabs(mean / (mean - fmin));",
                     "tests/test_oracle_pins_multid.py::test_limiter_contracts_exactly_to_zero_minimum[2-3]"),
    "mirror_axis": ("  b[k] = op->nv1[k] - 1 - b[k];", "  b[0] = op->nv1[0] - 1 - b[0]; (void)k;",
                    "tests/test_oracle_pins_multid.py::test_specular_wall_equals_mirror_image[2-1-2]"),
}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name", list(MUTATIONS))
def test_planted_mistake_fails_its_pin(tmp_path, name):
    old, new, pin = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"the line to mutate is not unique in the oracle: {old!r}"
    mut = tmp_path / "bgk_oracle_mut.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "liborc_mut.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fopenmp", "-fPIC", "-shared",
                           "-fno-fast-math", "-ffp-contract=off", str(mut), "-o", str(lib), "-lm"])
    env = dict(os.environ, BGK_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", pin],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1, f"{name}: the pin did not fail (exit {r.returncode})\n{r.stdout[-2000:]}"
    assert "1 failed" in r.stdout
