"""Chunk-wise dealing of stage work items to the XCDs gives the same bits.

BGK_XCD_PART=G (G = 2, 4 or 8; read when a solver is created) makes every
stage kernel deal its work items to groups of G XCDs chunk by chunk (each XCD
of a group takes a G-th of the items of every velocity chunk its group
walks) instead of in contiguous ranges.
Work items are independent, so the state after two RK3 steps and the limiter
count must equal the default mapping's bit for bit, for every kernel family
(quadrilaterals, one-lane and plane-split hexahedra; FP64, FP32, BF16
increments; per-element and column-sweep launches). The meshes have 64
elements and 10^3 velocities (4 or 16 velocity chunks), so every group size
divides the work items and the chunks.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2308_06196_amd import workloads as wl
from tests.helpers import initial_state, oracle_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a visible GPU"
    return t


def _run(torch, monkeypatch, pb, f0, dt, precision, seg, part):
    from paper_2308_06196_amd import bgk
    monkeypatch.setenv("BGK_SWEEP_SEG", str(seg))
    monkeypatch.setenv("BGK_XCD_PART", str(part))
    s = bgk.Solver(pb, precision=precision)
    monkeypatch.delenv("BGK_SWEEP_SEG")
    monkeypatch.delenv("BGK_XCD_PART")
    s.set_state(torch.from_numpy(np.ascontiguousarray(f0)).to("cuda:0"))
    s.rk3_step(dt, 2)
    f = s.get_state().cpu().numpy()
    d = s.diagnostics()
    assert d["newton_fail"] == 0 and d["stages"] == 6
    return f, d


CASES = [(dim, order, prec, seg) for dim in (2, 3) for order in (1, 2, 3) for prec in (0, 1, 2)
         for seg in (0, 2)]


@pytest.mark.parametrize("dim,order,prec,seg", CASES)
def test_xcd_part_bitwise(torch, monkeypatch, dim, order, prec, seg):
    if dim == 2:
        pb, kind = wl.box2d(n=8, order=order, nv1=10), "box2d"
    else:
        pb, kind = wl.tgv3d(n=4, order=order, nv1=10), "tgv3d"
    print("[case] xcd_part", f"d{dim}p{order}", ["fp64", "fp32", "bf16"][prec], f"seg={seg}",
          pb["nelem"], pb["nvel"], flush=True)
    sys.stdout.flush()
    f0 = initial_state(pb, kind, seed=5, amp=0.2)
    dt = orc.stable_dt(oracle_problem(pb), f0, 0.1)
    f0_, d0 = _run(torch, monkeypatch, pb, f0, dt, prec, seg, 0)
    for part in (2, 4, 8):
        f1_, d1 = _run(torch, monkeypatch, pb, f0, dt, prec, seg, part)
        assert np.array_equal(f0_, f1_), part
        assert d0["limiter_hits"] == d1["limiter_hits"], part
