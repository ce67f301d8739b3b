"""Column-sweep stage kernels (RK stages run as sweeps along the last axis).

A work-group walks a segment of a column of elements in the upwind direction
of its velocity chunk and hands each element's outflow traces on the last
axis to the next element. The solver picks the segment length when it is
created; BGK_SWEEP_SEG forces it (0: per-element kernels). Here it is forced
on every kernel family, whether or not the solver would pick it:

  * against the FP64 oracle after two RK3 steps (FP64 1e-12, FP32 1e-5, BF16
    increments within the bound of the parity tests);
  * where the kernel forms the exterior traces on the VALU (quadrilaterals in
    every precision, one-lane hexahedra at p <= 2), bit for bit against the
    per-element kernel: the carried trace is the same sum in the same order.

The velocity grids are ragged (N_1d = 7 and 5), so some velocity chunks hold
both signs of the last velocity component (those lanes read their neighbour
as without the sweep); segments of 2 and 4 elements put entry elements
inside the columns; specular walls on the last axis cover the mirrored entry
traces.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2308_06196_amd import workloads as wl
from tests.helpers import initial_state, oracle_problem, rel_max

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a visible GPU"
    return t


def _problem(dim, order, walls):
    if dim == 2:
        pb, kind = wl.box2d(n=4, order=order, nv1=7), "box2d"
    else:
        pb, kind = wl.tgv3d(n=4, order=order, nv1=5), "tgv3d"
    if walls:
        bc = list(pb["bc"])
        bc[dim - 1] = (1, 1)
        pb["bc"] = bc
    return pb, kind


def _run(torch, monkeypatch, pb, f0, dt, precision, seg, steps=2):
    from paper_2308_06196_amd import bgk
    monkeypatch.setenv("BGK_SWEEP_SEG", str(seg))
    s = bgk.Solver(pb, precision=precision)
    monkeypatch.delenv("BGK_SWEEP_SEG")
    s.set_state(torch.from_numpy(np.ascontiguousarray(f0)).to("cuda:0"))
    s.rk3_step(dt, steps)
    f = s.get_state().cpu().numpy()
    d = s.diagnostics()
    assert d["newton_fail"] == 0 and d["stages"] == 3 * steps
    return f, d


def _bf16_bound(pr, f0, dt, n):
    # as in test_gpu_parity: 1e-5 max|f| + 2 n 2^-8 max_k dt |L(f^k)|
    traj, inc = [f0], 0.0
    for _ in range(n):
        L, _ = orc.residual(pr, traj[-1])
        inc = max(inc, dt * float(np.abs(L).max()))
        traj.append(orc.rk3_step(pr, traj[-1], dt, 1)[0])
    return traj[-1], 1e-5 * float(np.abs(traj[-1]).max()) + 2.0 * n * 2.0 ** -8 * inc


def _valu_traces(dim, order, precision):
    """The exterior traces are VALU sums in the sweep and per-element kernels."""
    if dim == 2:
        return True
    return order <= 2  # one lane per velocity; p = 3 runs matrix-core or plane-split paths


CASES = [(dim, order, prec, seg, walls)
         for dim in (2, 3) for order in (1, 2, 3) for prec in (0, 1, 2) for seg in (2, 4)
         for walls in (False, True) if not (walls and seg == 4)]


@pytest.mark.parametrize("dim,order,prec,seg,walls", CASES)
def test_sweep_matches_oracle(torch, monkeypatch, dim, order, prec, seg, walls):
    pb, kind = _problem(dim, order, walls)
    _say("sweep", f"d{dim}p{order}", ["fp64", "fp32", "bf16"][prec], f"seg={seg}",
         "walls" if walls else "periodic", pb["nelem"], pb["nvel"])
    pr = oracle_problem(pb)
    f0 = initial_state(pb, kind, seed=11, amp=0.2)
    dt = orc.stable_dt(pr, f0, 0.1)
    f_sw, d_sw = _run(torch, monkeypatch, pb, f0, dt, prec, seg)
    if prec == 2:
        f_orc, bound = _bf16_bound(pr, f0, dt, 2)
        err = float(np.abs(f_sw - f_orc).max())
        assert err < bound, (err, bound)
    else:
        f_orc, _ = orc.rk3_step(pr, f0, dt, 2)
        assert rel_max(f_sw, f_orc) < (1e-12 if prec == 0 else 1e-5)
    if _valu_traces(dim, order, prec):
        f_el, d_el = _run(torch, monkeypatch, pb, f0, dt, prec, 0)
        assert np.array_equal(f_sw, f_el)
        assert d_sw["limiter_hits"] == d_el["limiter_hits"]

