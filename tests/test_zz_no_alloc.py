"""The residual entry point that allocates nothing (bgk_residual_noalloc)
against the solver's bgk_residual, which runs the same kernels over a
caller-owned workspace: two calls in a row, the second with a smaller
problem (the static scratch array keeps the first call's contents), in FP64
and FP32 storage. The results must be equal bit for bit. Also: problems
beyond the scratch array's size and diffuse walls are refused before
anything is queued."""
import sys

import numpy as np
import pytest

from paper_2308_06196_amd import workloads as wl
from tests.helpers import initial_state

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _pair(pb, kind, seed, precision):
    import torch
    from paper_2308_06196_amd import bgk
    f = torch.from_numpy(initial_state(pb, kind, seed=seed, amp=0.3)).to("cuda:0")
    r_static = bgk.residual_noalloc(pb, f, precision=precision)
    s = bgk.Solver(pb, precision=precision)
    r_solver = s.residual(f)
    torch.cuda.synchronize()
    s.close()
    return r_static.cpu().numpy(), r_solver.cpu().numpy()


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_residual_equals_solver_residual(precision):
    cases = [  # the second call is smaller than the first
        (wl.tgv3d(n=2, order=3, nv1=12), "tgv3d", 51),
        (wl.box2d(n=3, order=2, nv1=10), "box2d", 52),
        (wl.sod1d(nelem=5, order=2, nv1=8), "sod1d", 53),
    ]
    for pb, kind, seed in cases:
        _say("noalloc residual", kind, pb["nelem"][:pb["dim"]], pb["nvel"], "precision", precision)
        a, b = _pair(pb, kind, seed, precision)
        assert np.isfinite(a).all()
        assert np.array_equal(a, b), float(np.abs(a - b).max())


def test_noalloc_refuses_large_and_diffuse_problems():
    import torch
    from paper_2308_06196_amd import bgk
    _say("noalloc refusals")
    big = wl.box2d(n=32, order=3, nv1=24)
    f = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    with pytest.raises(bgk.BGKError) as ei:
        bgk.lib().bgk_residual_noalloc  # the symbol is exported
        st = bgk.problem_struct(big, bgk.FP64)
        bgk._check(bgk.lib().bgk_residual_noalloc(bgk.C.byref(st), bgk.C.c_void_p(f.data_ptr()),
                                                   bgk.C.c_void_p(f.data_ptr()), None))
    assert ei.value.status == 3  # BGK_ERR_OUT_OF_MEMORY
    ch = wl.channel2d(nx=2, ny=2, order=1, nv1=6)
    with pytest.raises(bgk.BGKError) as ei:
        st = bgk.problem_struct(ch, bgk.FP64)
        bgk._check(bgk.lib().bgk_residual_noalloc(bgk.C.byref(st), bgk.C.c_void_p(f.data_ptr()),
                                                   bgk.C.c_void_p(f.data_ptr()), None))
    assert ei.value.status == 2  # BGK_ERR_UNSUPPORTED
