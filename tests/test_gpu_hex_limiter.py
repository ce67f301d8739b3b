"""Positivity limiter on hexahedra (Sec. 2.1, Zhang-Shu) against the oracle.

A Sod-type jump across a periodic 3-D box ((rho, theta) = (1, 1) for x < 1/2,
(0.125, 0.8) beyond; two jumps with the periodic wrap) makes the FR transport
undershoot below zero in many (element, velocity) slices within the first
stage, at every order p = 1, 2, 3. Three SSP-RK3 steps run on every stage
kernel that handles hexahedra: the FP64 plane-split kernel (limiter mean and
minimum reduced over the lanes of a velocity group), the FP32
one-lane-per-velocity kernel and the BF16-increment plane-split kernel.

Tolerances: FP64 states within 1e-12 max|f| with the same number of
contracted slices as the oracle; FP32 within 1e-5 max|f| (the sign of a
slice minimum within FP32 rounding of zero may differ from the oracle's, so
only a positive count of contractions is required); BF16 increments within the
per-step bound of the increment rounding (tests/test_gpu_parity.py)."""
import sys

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2308_06196_amd import workloads as wl
from tests.helpers import oracle_problem, rel_max

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _jump_box(order, nelem=(4, 2, 2), nv1=8):
    return wl.problem(3, order, list(nelem), [0.0] * 3, [1.0] * 3, [nv1] * 3, [-6.0] * 3,
                      [6.0] * 3, 1e-3)


def _prim_jump(x):
    left = x[:, 0] < 0.5
    prim = np.zeros((len(x), 5))
    prim[:, 0] = np.where(left, 1.0, 0.125)
    prim[:, 4] = np.where(left, 1.0, 0.8)
    return prim


def _bf16_bound(pr, f0, dt, n):
    traj, inc = [f0], 0.0
    for _ in range(n):
        L, _ = orc.residual(pr, traj[-1])
        inc = max(inc, dt * float(np.abs(L).max()))
        traj.append(orc.rk3_step(pr, traj[-1], dt, 1)[0])
    return traj[-1], 1e-5 * float(np.abs(traj[-1]).max()) + 2.0 * n * 2.0 ** -8 * inc


@pytest.mark.parametrize("order", [1, 2, 3])
def test_hexahedral_limiter_matches_oracle(order):
    import torch
    from paper_2308_06196_amd import bgk
    pb = _jump_box(order)
    _say("hex limiter", order, pb["nelem"], pb["nvel"])
    pr = oracle_problem(pb)
    f0 = orc.maxwellian(pr, _prim_jump(orc.node_coords(pr)))
    dt = orc.stable_dt(pr, f0, 0.1)
    steps = 3
    f_orc, d_orc = orc.rk3_step(pr, f0, dt, steps)
    assert d_orc["limiter_hits"] > 1000
    f_b16, bound = _bf16_bound(pr, f0, dt, steps)
    for prec in (bgk.FP64, bgk.FP32, bgk.BF16):
        _say("hex limiter", order, bgk.PRECISION_NAME[prec])
        s = bgk.Solver(pb, precision=prec)
        s.set_state(torch.from_numpy(f0).to("cuda:0"))
        s.rk3_step(dt, steps)
        f = s.get_state().cpu().numpy()
        d = s.diagnostics()
        print(f"  p={order} {bgk.PRECISION_NAME[prec]}: gpu hits {d['limiter_hits']} "
              f"oracle {d_orc['limiter_hits']}", flush=True)
        if prec == bgk.FP64:
            assert rel_max(f, f_orc) < 1e-12
            assert d["limiter_hits"] == d_orc["limiter_hits"]
            assert d["limiter_bad"] == d_orc["limiter_bad"]
        elif prec == bgk.FP32:
            assert rel_max(f, f_orc) < 1e-5
            assert d["limiter_hits"] > 1000
        else:
            err = float(np.abs(f - f_b16).max())
            print(f"  bf16 error {err:.3e} bound {bound:.3e}", flush=True)
            assert err < bound
            assert d["limiter_hits"] > 1000
            assert d["positivity_violations"] == 0
        s.close()
