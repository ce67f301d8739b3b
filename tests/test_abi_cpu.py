"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol declared in include/bgk.h, validates problems and reports errors, and
its host-side geometry (Golub-Welsch Gauss rule, velocity grid) agrees with
the oracle's independent construction. No device memory is touched."""
import ctypes as C

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2308_06196_amd import bgk
from paper_2308_06196_amd import workloads as wl
from tests.helpers import oracle_problem


def test_library_exports_every_declared_symbol():
    names = bgk.exported_names()
    assert len(names) >= 15
    L = bgk.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing


def test_status_strings():
    L = bgk.lib()
    for code, name in bgk.STATUS.items():
        assert L.bgk_status_str(code).decode() == name


@pytest.mark.parametrize("mutate,status", [
    (lambda p: p.update(dim=4), 1),
    (lambda p: p.update(order=5), 2),
    (lambda p: p["nvel"].__setitem__(0, 1), 1),
    (lambda p: p["nelem"].__setitem__(0, 0), 1),
    (lambda p: p.update(bc=[(1, 0), (0, 0), (0, 0)]), 1),
    (lambda p: p.update(vlo=[-5.0, -6.0, -6.0]), 1),   # specular needs symmetric grid
    (lambda p: p.update(limiter=3), 1),
    (lambda p: p.update(equilibrium=2), 1),
    (lambda p: p.update(sutherland=-1.0), 1),
    (lambda p: p.update(bc=[(2, 2), (0, 0), (0, 0)], wall_theta=[(0.0, 1.0)] * 3), 1),
])
def test_footprint_validation(mutate, status):
    pb = wl.sod1d()
    pb = {k: (list(v) if isinstance(v, list) else v) for k, v in pb.items()}
    mutate(pb)
    with pytest.raises(bgk.BGKError) as ei:
        bgk.footprint(pb)
    assert ei.value.status == status
    assert bgk.lib().bgk_last_error().decode()


def test_footprint_scales_with_precision():
    pb = wl.box2d()
    b64, nx, nv = bgk.footprint(pb, bgk.FP64)
    b32, _, _ = bgk.footprint(pb, bgk.FP32)
    b16, _, _ = bgk.footprint(pb, bgk.BF16)
    assert nx == 1024 * 16 and nv == 24 ** 3
    assert b64 >= 3 * nx * nv * 8 and b32 >= 3 * nx * nv * 4 and b32 < b64
    # BF16: two FP32 state buffers and one BF16 increment buffer
    assert b16 >= nx * nv * 10 and b16 < b32


def test_bf16_precision_limits():
    """BF16 storage (FP32 state, BF16 stage increments) is accepted; an unknown
    precision is an argument error and diffuse walls are not built for it."""
    bgk.footprint(wl.box2d(n=2), bgk.BF16)
    with pytest.raises(bgk.BGKError) as ei:
        bgk.footprint(wl.box2d(n=2), 3)
    assert ei.value.status == 1
    with pytest.raises(bgk.BGKError) as ei:
        bgk.footprint(wl.channel2d(nx=2, ny=2), bgk.BF16)
    assert ei.value.status == 2
    bgk.footprint(wl.channel2d(nx=2, ny=2), bgk.FP32)


def _host_only_solver(pb, precision=bgk.FP64):
    """Solver over a placeholder workspace address; only host-side entry points
    (coordinates, velocity grid, destroy) are called on it."""
    nbytes, nx, nv = bgk.footprint(pb, precision)
    st = bgk.problem_struct(pb, precision)
    s = C.c_void_p()
    rc = bgk.lib().bgk_create(C.byref(st), C.c_void_p(1 << 20), nbytes, None, C.byref(s))
    assert rc == 0
    return s, nx, nv


def test_create_rejects_small_or_misaligned_workspace():
    pb = wl.sod1d(nelem=4)
    nbytes, _, _ = bgk.footprint(pb)
    st = bgk.problem_struct(pb)
    s = C.c_void_p()
    assert bgk.lib().bgk_create(C.byref(st), C.c_void_p(1 << 20), nbytes - 1, None,
                                C.byref(s)) == 3
    assert bgk.lib().bgk_create(C.byref(st), C.c_void_p((1 << 20) + 8), nbytes, None,
                                C.byref(s)) == 1
    assert bgk.lib().bgk_create(C.byref(st), None, nbytes, None, C.byref(s)) == 1


@pytest.mark.parametrize("pb", [wl.sod1d(nelem=5, order=1), wl.box2d(n=3, order=3, nv1=6),
                                wl.tgv3d(n=2, order=2, nv1=4)])
def test_host_geometry_matches_oracle(pb):
    s, nx, nv = _host_only_solver(pb)
    try:
        x = np.zeros((nx, pb["dim"]))
        assert bgk.lib().bgk_node_coords(s, x.ctypes.data_as(C.POINTER(C.c_double))) == 0
        u, w = np.zeros((nv, 3)), np.zeros(nv)
        assert bgk.lib().bgk_velocity_grid(s, u.ctypes.data_as(C.POINTER(C.c_double)),
                                           w.ctypes.data_as(C.POINTER(C.c_double))) == 0
    finally:
        bgk.lib().bgk_destroy(s)
    pr = oracle_problem(pb)
    assert np.abs(x - orc.node_coords(pr)).max() < 1e-14
    uo, wo = orc.velocity_grid(pr)
    assert np.array_equal(u, uo) and np.array_equal(w, wo)


@pytest.mark.parametrize("pb", [wl.sod1d(nelem=5, order=2), wl.box2d(n=3, order=3),
                                wl.tgv3d(n=2, order=1)])
def test_ablation_node_weights_integrate_exactly(pb):
    """The study's quadrature weights, in the library's node order, integrate
    low-degree polynomials over the box exactly (checked at the oracle's nodes)."""
    from oracle import oracle as orc
    from paper_2308_06196_amd import ablation
    from tests.helpers import oracle_problem
    x = orc.node_coords(oracle_problem(pb))
    W = ablation.node_weights(pb)
    d = pb["dim"]
    vol = 1.0
    for k in range(d):
        vol *= pb["xhi"][k] - pb["xlo"][k]
    assert abs(W.sum() - vol) < 1e-12 * vol
    for k in range(d):
        lo, hi = pb["xlo"][k], pb["xhi"][k]
        exact = vol / (hi - lo) * (hi ** 3 - lo ** 3) / 3.0
        assert abs(W @ x[:, k] ** 2 - exact) < 1e-12 * abs(exact)


def test_diffuse_walls_rejected_on_hexahedra():
    pb = wl.tgv3d(n=2, order=1, nv1=4)
    pb["bc"] = [(0, 0), (0, 0), (2, 2)]
    with pytest.raises(bgk.BGKError) as ei:
        bgk.footprint(pb)
    assert ei.value.status == 2
