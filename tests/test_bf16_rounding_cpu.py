"""Why BF16 storage keeps f^n in FP32 and stores only the stage increments.

Emulated with the oracle's FP64 residual (no GPU): SSP-RK3 steps of a shock
tube where (a) every stage value f^(s) is rounded to BF16 ("naive"), or (b)
only the stage increments D_s = f^(s) - f^n are rounded to BF16 (the library's
BGK_BF16). BF16 keeps 8 significant bits, so rounding f itself costs up to
2^-9 |f| per stage, while one step changes f by only ~dt |L| -- the per-step
change is below BF16's resolution and the naive trajectory is swamped.
Rounding the increments costs only ~2^-9 of the change itself.
"""
import numpy as np

from oracle import oracle as orc
from paper_2308_06196_amd import workloads as wl
from tests.helpers import initial_state, oracle_problem

A_RK = (0.0, 0.75, 1.0 / 3.0)
B_RK = (1.0, 0.25, 2.0 / 3.0)


def bf16(x):
    """Round FP64 values to BF16 (nearest, ties to even) through FP32."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def steps(pr, f, dt, n, mode):
    for _ in range(n):
        fn, g = f, f
        for s, (a, b) in enumerate(zip(A_RK, B_RK)):
            L, _ = orc.residual(pr, g)
            o = a * fn + b * (g + dt * L)
            if mode == "naive":
                g = bf16(o)
            elif mode == "increments" and s < 2:
                g = fn + bf16(o - fn)
            else:
                g = o
        f = g if mode == "fp64" else np.asarray(g, dtype=np.float32).astype(np.float64)
    return f


def test_naive_bf16_is_swamped_and_increments_are_not():
    pb = wl.sod1d(nelem=8, order=2, nv1=12)
    pr = oracle_problem(pb)
    f0 = initial_state(pb, "sod1d")
    dt = orc.stable_dt(pr, f0, 0.1)
    n = 10
    ref = steps(pr, f0, dt, n, "fp64")
    change = np.abs(ref - f0).max()
    e_naive = np.abs(steps(pr, f0, dt, n, "naive") - ref).max()
    e_inc = np.abs(steps(pr, f0, dt, n, "increments") - ref).max()
    print(f"change over {n} steps {change:.3e}; naive BF16 error {e_naive:.3e}; "
          f"BF16 increments error {e_inc:.3e}")
    # naive rounding errs by at least BF16's resolution of f itself
    assert e_naive > 2.0 ** -9 * np.abs(ref).max()
    # increments: within 2^-8 of the change (plus FP32 rounding of the state)
    assert e_inc < 2.0 ** -8 * change + 1e-6 * np.abs(ref).max()
    assert e_inc < 0.05 * e_naive
