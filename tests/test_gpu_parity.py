"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle.

Tolerances (FP64 storage):
  * states (set, after RK3 steps): max |f_gpu - f_orc| <= 1e-12 max |f_orc|;
  * residual L = -T + C: max |L_gpu - L_orc| <= 1e-12 (max|T_orc| + max|C_orc|),
    i.e. relative to the size of the two terms whose difference L is (the
    collision term alone is amplified by 1/tau, so a bare relative error of L
    would measure cancellation, not the kernel);
  * moments: <= 1e-13 relative to rho (mass, momentum) and E (energy).
Every case prints its name, shape and seed before touching the GPU.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2308_06196_amd import workloads as wl
from tests.helpers import field_errors, initial_state, oracle_problem, rel_max

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a visible GPU"
    return t


def solver(pb, precision=0):
    from paper_2308_06196_amd import bgk
    return bgk.Solver(pb, precision=precision)


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


# Small cases covering every (d, p), periodic and specular, ragged velocity
# counts (N_v below, between and above multiples of the 256-wide chunk).
CASES = {
    "d1p1_sod_spec": (wl.sod1d(nelem=6, order=1, nv1=8), "sod1d"),
    "d1p2_sod_spec": (wl.sod1d(nelem=5, order=2, nv1=10), "sod1d"),
    "d1p3_sod_spec": (wl.sod1d(nelem=4, order=3, nv1=6), "sod1d"),
    "d2p1_box": (wl.box2d(n=3, order=1, nv1=7), "box2d"),
    "d2p2_box": (wl.box2d(n=3, order=2, nv1=8), "box2d"),
    "d2p3_box": (wl.box2d(n=2, order=3, nv1=9), "box2d"),
    "d3p1_tgv": (wl.tgv3d(n=2, order=1, nv1=6), "tgv3d"),
    "d3p2_tgv": (wl.tgv3d(n=2, order=2, nv1=5), "tgv3d"),
    "d3p3_tgv": (wl.tgv3d(n=2, order=3, nv1=4), "tgv3d"),
}


@pytest.mark.parametrize("name", list(CASES))
def test_maxwellian_and_state_roundtrip(torch, name):
    pb, kind = CASES[name]
    _say("maxwellian", name, pb["nelem"], pb["order"], pb["nvel"])
    pr = oracle_problem(pb)
    s = solver(pb)
    x = s.node_coords()
    prim = wl.PRIM[kind](x)
    s.set_maxwellian(prim)
    f_gpu = s.get_state().cpu().numpy()
    f_orc = orc.maxwellian(pr, wl.PRIM[kind](orc.node_coords(pr)))
    assert rel_max(f_gpu, f_orc) < 1e-13
    # exact round trip of an arbitrary FP64 state, host and device paths
    g = initial_state(pb, kind, seed=1, amp=0.3)
    s.set_state(dev(torch, g))
    assert np.array_equal(s.get_state().cpu().numpy(), g)
    s.set_state(g)
    out = np.zeros_like(g)
    s.get_state(out)
    assert np.array_equal(out, g)


@pytest.mark.parametrize("name", list(CASES))
def test_moments_match_oracle(torch, name):
    pb, kind = CASES[name]
    _say("moments", name)
    f = initial_state(pb, kind, seed=2, amp=0.3)
    s = solver(pb)
    s.set_state(dev(torch, f))
    Q = s.moments().cpu().numpy()
    Qo = orc.moments(oracle_problem(pb), f)
    scale = np.column_stack([Qo[:, 0]] * 4 + [Qo[:, 4]])
    assert np.abs(Q - Qo).max() / 1.0 < 1e-13 * scale.max()
    assert (np.abs(Q - Qo) / scale).max() < 1e-13


def _residual_case(torch, pb, kind, seed, precision=0):
    pr = oracle_problem(pb)
    f = initial_state(pb, kind, seed=seed, amp=0.3)
    s = solver(pb, precision)
    r = s.residual(dev(torch, f)).cpu().numpy()
    T = orc.transport(pr, f)
    Cc, dg = orc.collision(pr, f)
    L, _ = orc.residual(pr, f)
    scale = np.abs(T).max() + np.abs(Cc).max()
    return float(np.abs(r - L).max() / scale), s


@pytest.mark.parametrize("name", list(CASES))
def test_residual_matches_oracle(torch, name):
    pb, kind = CASES[name]
    _say("residual", name)
    err, s = _residual_case(torch, pb, kind, seed=3)
    assert err < 1e-12, err
    s.diagnostics()


@pytest.mark.parametrize("name", ["d1p2_sod_spec", "d2p3_box", "d3p2_tgv"])
def test_residual_anisotropic_velocity_grid(torch, name):
    pb, kind = CASES[name]
    pb = dict(pb)
    n = pb["nvel"][0]
    pb["nvel"] = [n, n + 3, n + 1]
    pb["vlo"] = [-6.0, -5.0, -7.0] if pb["dim"] == 1 else [-6.0, -5.5, -7.0]
    pb["vhi"] = [6.0, 5.0, 7.0] if pb["dim"] == 1 else [6.5, 5.0, 7.0]
    if pb["dim"] > 1:
        pb["bc"] = [(0, 0)] * 3
    _say("residual-aniso", name, pb["nvel"])
    err, _ = _residual_case(torch, pb, kind, seed=4)
    assert err < 1e-12, err


def test_residual_collisionless_and_installed_state(torch):
    pb, kind = CASES["d2p2_box"]
    pb = dict(pb, mu_ref=0.0)
    _say("residual-nocoll")
    f = initial_state(pb, kind, seed=5, amp=0.2)
    s = solver(pb)
    s.set_state(dev(torch, f))
    r = s.residual().cpu().numpy()  # of the installed state
    T = orc.transport(oracle_problem(pb), f)
    assert rel_max(r, -T) < 1e-12


def test_residual_host_buffers(torch):
    pb, kind = CASES["d1p2_sod_spec"]
    _say("residual-host")
    f = initial_state(pb, kind, seed=6, amp=0.3)
    pr = oracle_problem(pb)
    L, _ = orc.residual(pr, f)
    scale = np.abs(orc.transport(pr, f)).max() + np.abs(orc.collision(pr, f)[0]).max()
    for prec, tol in ((0, 1e-12), (1, 1e-5)):
        s = solver(pb, prec)
        out = np.zeros_like(f)
        s.residual(f, out)
        assert np.abs(out - L).max() / scale < tol


@pytest.mark.parametrize("name", list(CASES))
def test_rk3_steps_match_oracle(torch, name):
    pb, kind = CASES[name]
    _say("rk3", name)
    pr = oracle_problem(pb)
    f0 = initial_state(pb, kind, seed=7, amp=0.2)
    dt = orc.stable_dt(pr, f0, 0.1)
    s = solver(pb)
    s.set_state(dev(torch, f0))
    assert abs(s.stable_dt(0.1) - dt) <= 1e-14 * dt
    s.rk3_step(dt, 3)
    f_gpu = s.get_state().cpu().numpy()
    f_orc, dg = orc.rk3_step(pr, f0, dt, 3)
    assert rel_max(f_gpu, f_orc) < 1e-12
    d = s.diagnostics()
    assert d["newton_fail"] == 0 and d["stages"] == 9


def test_sod_full_run_fp64(torch):
    """Shock tube, 32 elements p=2, 16^3 on [-6,6]^3, Kn=1e-2, specular walls,
    CFL 0.1, 100 SSP-RK3 steps, FP64, limiter on."""
    pb = wl.sod1d()
    _say("sod-full", pb["nelem"], pb["nvel"])
    pr = oracle_problem(pb)
    f0 = initial_state(pb, "sod1d")
    dt = orc.stable_dt(pr, f0, 0.1)
    s = solver(pb)
    s.set_state(dev(torch, f0))
    s.rk3_step(dt, 100)
    f_gpu = s.get_state().cpu().numpy()
    f_orc, dg = orc.rk3_step(pr, f0, dt, 100)
    assert rel_max(f_gpu, f_orc) < 1e-12
    errs = field_errors(pb, s.moments().cpu().numpy(), orc.moments(pr, f_orc))
    assert max(errs.values()) < 1e-12, errs
    d = s.diagnostics()
    assert d["limiter_hits"] == dg["limiter_hits"]


def test_box2d_reduced_fp64_and_conservation(torch):
    """2-D periodic box (C2's IC and velocity grid) on 4x4 elements, p=3, 20 steps."""
    pb = wl.box2d(n=4)
    _say("box2d-reduced", pb["nelem"], pb["nvel"])
    pr = oracle_problem(pb)
    f0 = initial_state(pb, "box2d")
    dt = orc.stable_dt(pr, f0, 0.1)
    s = solver(pb)
    s.set_state(dev(torch, f0))
    W = _node_weights(pb)
    tot0 = W @ s.moments().cpu().numpy()
    s.rk3_step(dt, 20)
    tot1 = W @ s.moments().cpu().numpy()
    f_gpu = s.get_state().cpu().numpy()
    f_orc, _ = orc.rk3_step(pr, f0, dt, 20)
    assert rel_max(f_gpu, f_orc) < 1e-12
    scale = np.array([tot0[0]] * 4 + [tot0[4]])
    assert (np.abs(tot1 - tot0) / scale).max() < 1e-13 * 20


def _node_weights(pb):
    _, wq = orc.gauss_legendre(pb["order"] + 1)
    W = wq
    for _ in range(pb["dim"] - 1):
        W = np.outer(W, wq).ravel()
    ne = int(np.prod(pb["nelem"][: pb["dim"]]))
    return np.tile(W, ne)


def test_fp32_bulk_fields_within_tolerance(torch):
    """FP32 storage and transport, FP64 moments/Newton: per-field error after 20 steps."""
    pb = wl.box2d(n=4)
    _say("box2d-fp32", pb["nelem"])
    pr = oracle_problem(pb)
    f0 = initial_state(pb, "box2d")
    dt = orc.stable_dt(pr, f0, 0.1)
    s = solver(pb, precision=1)
    s.set_state(dev(torch, f0))
    s.rk3_step(dt, 20)
    f_orc, _ = orc.rk3_step(pr, f0, dt, 20)
    errs = field_errors(pb, s.moments().cpu().numpy(), orc.moments(pr, f_orc))
    print("fp32 field errors", errs)
    assert max(errs.values()) < 1e-5, errs
    assert rel_max(s.get_state().cpu().numpy(), f_orc) < 1e-5


def test_numerical_failure_is_reported(torch):
    from paper_2308_06196_amd import bgk
    pb, kind = CASES["d1p1_sod_spec"]
    _say("failure-path")
    s = solver(pb)
    with pytest.raises(bgk.BGKError) as ei:
        s.set_maxwellian(np.tile([-1.0, 0, 0, 0, 1.0], (s.nx, 1)))
    assert ei.value.status == 1
    f = initial_state(pb, kind)
    f[0, 0, :] *= -1.0  # one node with negative density: not realizable
    s.set_state(dev(torch, f))
    s.rk3_step(1e-4, 1)
    with pytest.raises(bgk.BGKError) as ei:
        s.synchronize()
    assert ei.value.status == 5
    with pytest.raises(bgk.BGKError) as ei:
        s.rk3_step(1e-4, 1)
    assert ei.value.status == 7
    s.set_state(dev(torch, initial_state(pb, kind)))  # recovers
    s.rk3_step(1e-4, 1)
    s.synchronize()


@pytest.mark.parametrize("name", ["d1p2_sod_spec", "d2p2_box", "d3p1_tgv", "d3p2_tgv",
                                  "d3p3_tgv"])
def test_fp32_rk3_matches_oracle(torch, name):
    """FP32 storage / FP64 moments and Newton: 3 steps within 1e-5 of the FP64 oracle."""
    pb, kind = CASES[name]
    _say("rk3-fp32", name)
    pr = oracle_problem(pb)
    f0 = initial_state(pb, kind, seed=8, amp=0.2)
    dt = orc.stable_dt(pr, f0, 0.1)
    s = solver(pb, precision=1)
    s.set_state(dev(torch, f0))
    s.rk3_step(dt, 3)
    f_orc, _ = orc.rk3_step(pr, f0, dt, 3)
    assert rel_max(s.get_state().cpu().numpy(), f_orc) < 1e-5
    s.diagnostics()


def test_mach2_reduced_fp32_and_fp64(torch):
    """Mach-2 box (3-D, p=2, 20^3 velocities on [-8,8]^3) on 3^3 elements, 2 steps."""
    pb = wl.mach2(n=3)
    _say("mach2-reduced", pb["nelem"])
    pr = oracle_problem(pb)
    f0 = initial_state(pb, "mach2")
    dt = orc.stable_dt(pr, f0, 0.1)
    f_orc, _ = orc.rk3_step(pr, f0, dt, 2)
    for prec, tol in ((0, 1e-12), (1, 1e-5)):
        s = solver(pb, precision=prec)
        s.set_state(dev(torch, f0))
        s.rk3_step(dt, 2)
        assert rel_max(s.get_state().cpu().numpy(), f_orc) < tol, prec
        s.diagnostics()


def test_large_mesh_one_step(torch):
    """A 16^3-element hexahedral mesh (262,144 nodes: the large-mesh Newton teams and
    the brick traversal) with a small velocity grid, one step vs the oracle."""
    pb = wl.tgv3d(n=16, order=3, nv1=4)
    _say("large-mesh", pb["nelem"], pb["nvel"])
    pr = oracle_problem(pb)
    f0 = initial_state(pb, "tgv3d", seed=9, amp=0.1)
    dt = orc.stable_dt(pr, f0, 0.1)
    s = solver(pb)
    s.set_state(dev(torch, f0))
    s.rk3_step(dt, 1)
    f_orc, _ = orc.rk3_step(pr, f0, dt, 1)
    assert rel_max(s.get_state().cpu().numpy(), f_orc) < 1e-12


CONTINUOUS_CASES = {
    "d1p2_sod_spec": CASES["d1p2_sod_spec"],
    "d2p3_box": CASES["d2p3_box"],
    # 8^3 velocities: on the 5^3 grid of d3p2_tgv the continuous Maxwellian's
    # quadrature error is so large that both sides lose realizability
    "d3p2_tgv8": (wl.tgv3d(n=2, order=2, nv1=8), "tgv3d"),
}


@pytest.mark.parametrize("name", list(CONTINUOUS_CASES))
def test_continuous_equilibrium_matches_oracle(torch, name):
    """Non-conservative model (continuous Maxwellian, no Newton): residual and three
    RK3 steps against the oracle at the FP64 tolerances."""
    pb, kind = CONTINUOUS_CASES[name]
    pb = dict(pb, equilibrium=1)
    _say("continuous-eq", name)
    err, s = _residual_case(torch, pb, kind, seed=12)
    assert err < 1e-12, err
    pr = oracle_problem(pb)
    f0 = initial_state(pb, kind, seed=13, amp=0.2)
    dt = orc.stable_dt(pr, f0, 0.1)
    s = solver(pb)
    s.set_state(dev(torch, f0))
    s.rk3_step(dt, 3)
    f_orc, _ = orc.rk3_step(pr, f0, dt, 3)
    assert rel_max(s.get_state().cpu().numpy(), f_orc) < 1e-12
    d = s.diagnostics()
    assert d["newton_it_max"] == 0 and d["newton_fail"] == 0


def _sod_diffuse():
    pb = wl.sod1d(nelem=5, order=2, nv1=10)
    pb["bc"] = [(2, 2), (0, 0), (0, 0)]
    pb["wall_theta"] = [(1.3, 0.7), (1.0, 1.0), (1.0, 1.0)]
    pb["wall_vel"] = [((0.0, 0.2, 0.0), (0.0, -0.1, 0.0)), ((0.0,) * 3,) * 2, ((0.0,) * 3,) * 2]
    return pb


DIFFUSE_CASES = {
    "d1p2_diffuse": (_sod_diffuse(), "sod1d"),
    "d2p1_channel": (wl.channel2d(nx=3, ny=4, order=1, nv1=7, theta_w=1.2, uw=0.3), "channel2d"),
    "d2p2_channel": (wl.channel2d(nx=3, ny=3, order=2, nv1=8, theta_w=0.9, uw=0.2), "channel2d"),
    "d2p3_channel": (wl.channel2d(nx=2, ny=3, order=3, nv1=9, theta_w=1.1, uw=0.25), "channel2d"),
}


@pytest.mark.parametrize("name", list(DIFFUSE_CASES))
def test_diffuse_walls_match_oracle(torch, name):
    """Diffuse (Maxwell) walls: residual, three RK3 steps (FP64) and the FP32 path
    against the oracle; total mass conserved on the GPU."""
    pb, kind = DIFFUSE_CASES[name]
    _say("diffuse", name, pb["nelem"], pb["order"], pb["nvel"])
    err, _ = _residual_case(torch, pb, kind, seed=21)
    assert err < 1e-12, err
    pr = oracle_problem(pb)
    f0 = initial_state(pb, kind, seed=22, amp=0.2)
    dt = orc.stable_dt(pr, f0, 0.1)
    f_orc, _ = orc.rk3_step(pr, f0, dt, 3)
    s = solver(pb)
    s.set_state(dev(torch, f0))
    s.rk3_step(dt, 3)
    assert rel_max(s.get_state().cpu().numpy(), f_orc) < 1e-12
    W = _node_weights(pb)
    m0 = W @ orc.moments(pr, f0)[:, 0]
    m1 = W @ s.moments().cpu().numpy()[:, 0]
    assert abs(m1 - m0) / m0 < 1e-13
    s32 = solver(pb, 1)
    s32.set_state(dev(torch, f0))
    s32.rk3_step(dt, 3)
    assert rel_max(s32.get_state().cpu().numpy(), f_orc) < 1e-5


@pytest.mark.parametrize("law", [{"omega": 0.81, "theta_ref": 0.8},
                                 {"sutherland": 0.4, "theta_ref": 0.8}])
@pytest.mark.parametrize("name", ["d1p2_sod_spec", "d2p2_box"])
def test_viscosity_laws_match_oracle(torch, name, law):
    """Power law with omega != 0 and Sutherland's law: residual and RK3 steps."""
    pb, kind = CASES[name]
    pb = dict(pb, **law)
    _say("viscosity", name, law)
    err, _ = _residual_case(torch, pb, kind, seed=31)
    assert err < 1e-12, err
    pr = oracle_problem(pb)
    f0 = initial_state(pb, kind, seed=32, amp=0.2)
    dt = orc.stable_dt(pr, f0, 0.1)
    s = solver(pb)
    s.set_state(dev(torch, f0))
    assert abs(s.stable_dt(0.1) - dt) <= 1e-14 * dt
    s.rk3_step(dt, 3)
    f_orc, _ = orc.rk3_step(pr, f0, dt, 3)
    assert rel_max(s.get_state().cpu().numpy(), f_orc) < 1e-12


def _bf16_bound(pr, f0, dt, n):
    """Oracle trajectory of n steps and the error bound of the BF16-increment path.

    A BF16 value is rounded to nearest with relative error <= 2^-8. The stored
    increments of a step are D1 = dt L(f^n) and D2 ~ (D1 + dt L(f1)) / 4, and
    the rounding of D1 reaches D2 and f^(n+1) through stable stages, so each
    step carries at most ~(4/3) 2^-8 max|dt L(f^n)| into the state. The bound
    doubles that per step and adds the FP32 arithmetic (1e-5 max|f|)."""
    traj, inc = [f0], 0.0
    for _ in range(n):
        L, _ = orc.residual(pr, traj[-1])
        inc = max(inc, dt * float(np.abs(L).max()))
        traj.append(orc.rk3_step(pr, traj[-1], dt, 1)[0])
    return traj, 1e-5 * float(np.abs(traj[-1]).max()) + 2.0 * n * 2.0 ** -8 * inc


@pytest.mark.parametrize("name", ["d1p2_sod_spec", "d2p2_box", "d2p3_box", "d3p1_tgv",
                                  "d3p2_tgv", "d3p3_tgv"])
def test_bf16_increments_rk3_matches_oracle(torch, name):
    """BF16 storage (FP32 f^n, BF16 stage increments): 3 steps against the FP64
    oracle within the bound of _bf16_bound; the same steps in FP32 storage stay
    within 1e-5, so the difference is the increment rounding."""
    pb, kind = CASES[name]
    _say("rk3-bf16", name)
    pr = oracle_problem(pb)
    f0 = initial_state(pb, kind, seed=8, amp=0.2)
    dt = orc.stable_dt(pr, f0, 0.1)
    traj, bound = _bf16_bound(pr, f0, dt, 3)
    s = solver(pb, precision=2)
    s.set_state(dev(torch, f0))
    s.rk3_step(dt, 3)
    err = float(np.abs(s.get_state().cpu().numpy() - traj[-1]).max())
    print(f"bf16 {name}: err {err:.3e} bound {bound:.3e} (max f {np.abs(traj[-1]).max():.3e})")
    assert err < bound
    s.diagnostics()


def test_bf16_fields_and_state_buffers(torch):
    """BF16 increments over 20 steps of the 2-D box: per-field errors against the
    oracle, the state exchange after an odd and an even number of steps (the
    state alternates between two FP32 buffers), the residual entry point, and
    batches refusing a BF16 solver."""
    from paper_2308_06196_amd import bgk
    pb = wl.box2d(n=4)
    _say("box2d-bf16", pb["nelem"])
    pr = oracle_problem(pb)
    f0 = initial_state(pb, "box2d")
    dt = orc.stable_dt(pr, f0, 0.1)
    traj, bound = _bf16_bound(pr, f0, dt, 20)
    s = solver(pb, precision=2)
    s.set_state(dev(torch, f0))
    s.rk3_step(dt, 19)
    assert rel_max(s.get_state().cpu().numpy(), traj[19], scale=1.0) < bound
    s.rk3_step(dt, 1)
    f20 = s.get_state().cpu().numpy()
    assert rel_max(f20, traj[20], scale=1.0) < bound
    errs = field_errors(pb, s.moments().cpu().numpy(), orc.moments(pr, traj[20]))
    print("bf16 field errors", errs, "state bound", bound)
    assert max(errs.values()) < 1e-4, errs
    # the residual of the installed state runs the FP32 kernel on the FP32
    # state: the same result as an FP32 solver holding the same values
    L = s.residual().cpu().numpy()
    s32 = solver(pb, precision=1)
    s32.set_state(dev(torch, f20))
    L32 = s32.residual().cpu().numpy()
    assert np.abs(L - L32).max() <= 1e-12 * np.abs(L32).max()
    s32.close()
    s.synchronize()
    st = torch.cuda.Stream()
    sb = bgk.Solver(pb, precision=2, stream=st)
    sb.set_state(dev(torch, f0))
    b = bgk.Batch(st, max_members=2)
    with pytest.raises(bgk.BGKError) as ei:
        b.add(sb, dt, 1)
    assert ei.value.status == 2
    b.close()
    sb.close()


@pytest.mark.parametrize("name", list(CASES))
def test_fp32_residual_matches_oracle(torch, name):
    """FP32 storage and arithmetic (hexahedra on the one-lane-per-velocity
    kernel): the residual of a state away from equilibrium (amplitude 0.3, so
    that the collision term is not a difference of nearly equal values) within
    1e-5 of max|T| + max|C|."""
    pb, kind = CASES[name]
    _say("residual-fp32", name)
    f = initial_state(pb, kind, seed=5, amp=0.3)
    pr = oracle_problem(pb)
    s = solver(pb, precision=1)
    r = s.residual(dev(torch, f)).cpu().numpy()
    L, _ = orc.residual(pr, f)
    scale = np.abs(orc.transport(pr, f)).max() + np.abs(orc.collision(pr, f)[0]).max()
    err = float(np.abs(r - L).max() / scale)
    print(f"fp32 residual {name}: {err:.2e}")
    assert err < 1e-5, err


@pytest.mark.parametrize("order", [1, 2, 3])
def test_hexahedra_specular_walls(torch, order):
    """A closed 3-D box (specular walls on all six faces: the exterior trace is
    the own trace at the mirrored velocity): residual and three RK3 steps
    against the oracle, FP64 (plane-split kernel) and FP32 (one lane per
    velocity)."""
    pb = dict(wl.tgv3d(n=2, order=order, nv1=6), bc=[(1, 1)] * 3)
    _say("hex-specular", order)
    pr = oracle_problem(pb)
    f0 = initial_state(pb, "tgv3d", seed=11, amp=0.2)
    dt = orc.stable_dt(pr, f0, 0.1)
    L, _ = orc.residual(pr, f0)
    scale = np.abs(orc.transport(pr, f0)).max() + np.abs(orc.collision(pr, f0)[0]).max()
    f_orc, _ = orc.rk3_step(pr, f0, dt, 3)
    for prec, tol in ((0, 1e-12), (1, 1e-5)):
        s = solver(pb, precision=prec)
        r = s.residual(dev(torch, f0)).cpu().numpy()
        assert np.abs(r - L).max() / scale < tol, prec
        s.set_state(dev(torch, f0))
        s.rk3_step(dt, 3)
        assert rel_max(s.get_state().cpu().numpy(), f_orc) < tol, prec
        s.diagnostics()


DEGENERATE = {
    # one element per axis: every neighbour is the element itself (periodic wrap)
    "d1_one_element": (dict(wl.sod1d(nelem=1, order=3, nv1=6), bc=[(0, 0)] * 3), "sod1d"),
    "d2_one_element": (wl.box2d(n=1, order=2, nv1=5), "box2d"),
    "d3_one_element": (wl.tgv3d(n=1, order=3, nv1=4), "tgv3d"),
    # one element between specular walls
    "d1_one_element_walls": (wl.sod1d(nelem=1, order=2, nv1=7), "sod1d"),
    # the smallest velocity grid, two nodes per component (8 velocities), in free
    # transport: there |u|^2 is the same at every velocity, so the energy moment
    # is a multiple of the mass and the conservative equilibrium is not defined
    # (covered by test_two_velocity_nodes_report_newton_failure)
    "d2_two_velocity_nodes": (dict(wl.box2d(n=3, order=1, nv1=2, vmax=1.5), mu_ref=0.0), "box2d"),
    "d3_two_velocity_nodes": (dict(wl.tgv3d(n=2, order=2, nv1=2, vmax=1.5), mu_ref=0.0), "tgv3d"),
}


def _fp32_collision_rounding(pb, pr, f):
    """Size of FP32 rounding in the collision term (g - f)/tau: a few FP32 ulps
    of max|f| times max 1/tau, with 1/tau = P / mu (omega = 0 here)."""
    if not pb["mu_ref"] > 0.0:
        return 0.0
    Q = orc.moments(pr, f)
    rho, E = Q[:, 0], Q[:, 4]
    gamma = pb["gamma"] or 5.0 / 3.0  # 0 selects (m + 2) / m
    P = (gamma - 1.0) * (E - 0.5 * (Q[:, 1:4] ** 2).sum(1) / rho)
    return 8.0 * 2.0 ** -24 * np.abs(f).max() * P.max() / pb["mu_ref"]


@pytest.mark.parametrize("name", list(DEGENERATE))
def test_degenerate_sizes_match_oracle(torch, name):
    """Degenerate meshes and velocity grids: residual and two RK3 steps against
    the oracle, FP64 (1e-12) and FP32 (1e-5; the FP32 residual also allows the
    rounding of its collision term, which coarse grids at Kn = 1e-3 expose)."""
    pb, kind = DEGENERATE[name]
    _say("degenerate", name, pb["nelem"], pb["nvel"])
    pr = oracle_problem(pb)
    f0 = initial_state(pb, kind, seed=13, amp=0.2)
    L, _ = orc.residual(pr, f0)
    scale = np.abs(orc.transport(pr, f0)).max() + np.abs(orc.collision(pr, f0)[0]).max()
    dt = orc.stable_dt(pr, f0, 0.1)
    f_orc, _ = orc.rk3_step(pr, f0, dt, 2)
    for prec, tol in ((0, 1e-12), (1, 1e-5)):
        s = solver(pb, precision=prec)
        r = s.residual(dev(torch, f0)).cpu().numpy()
        bound = tol * scale + (_fp32_collision_rounding(pb, pr, f0) if prec else 0.0)
        assert np.abs(r - L).max() < bound, (prec, "residual")
        s.set_state(dev(torch, f0))
        s.rk3_step(dt, 2)
        assert rel_max(s.get_state().cpu().numpy(), f_orc) < tol, (prec, "rk3")
        s.diagnostics()


@pytest.mark.parametrize("dim", [2, 3])
def test_two_velocity_nodes_report_newton_failure(torch, dim):
    """With two velocity nodes per component the energy row of the Newton
    Jacobian is a multiple of the mass row (|u|^2 = 3 vmax^2 everywhere), so the
    discretely conservative equilibrium of Sec. 2.1 has no solution for a
    general state. The oracle reports a failed solve at every node; the GPU path
    must report failures too, and diagnostics() must raise rather than let the
    result pass as valid."""
    from paper_2308_06196_amd import bgk
    pb = wl.box2d(n=3, order=1, nv1=2, vmax=1.5) if dim == 2 else wl.tgv3d(n=2, order=2, nv1=2, vmax=1.5)
    kind = "box2d" if dim == 2 else "tgv3d"
    _say("two velocity nodes, collision on", dim, pb["nelem"], pb["nvel"])
    pr = oracle_problem(pb)
    f0 = initial_state(pb, kind, seed=13, amp=0.2)
    _, d_orc = orc.residual(pr, f0)
    assert d_orc["newton_fail"] == pr.nx
    for prec in (0, 1):
        s = solver(pb, precision=prec)
        s.residual(dev(torch, f0))
        d = s.diagnostics(raise_on_failure=False)
        print("[case] prec", prec, "oracle", d_orc, "gpu", d, flush=True)
        assert d["newton_fail"] == pr.nx
        with pytest.raises(bgk.BGKError):
            s.diagnostics()
