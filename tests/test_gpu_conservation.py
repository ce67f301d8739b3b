"""Discrete conservation of the collision term on the GPU, every storage precision.

The discretely conservative equilibrium (Sec. 2.1, velocity discretization)
is built so that the discrete moments of the BGK term vanish:
M . [(g - f)/tau (x) psi] = 0 for psi = (1, u, |u|^2/2). bgk_collision_moments
forms the collision term exactly as the stage kernels do (FP64 equilibrium
rows, the stored values of f, FP64 arithmetic) and returns its moments per
node. Target: <= 1e-13 relative, scaled per node by (rho, rho, rho, rho, E)/tau,
for FP64 storage, FP32 storage and BF16 increments alike.

Negative control: the non-conservative model (the continuous Maxwellian
sampled at the nodes, which the paper contrasts with the DVM equilibrium) on
a coarse 8^3 grid must show moments of the quadrature error's size (> 1e-5),
so the measurement does see a collision term that does not conserve.
"""
import sys

import numpy as np
import pytest

from paper_2308_06196_amd import workloads as wl
from tests.helpers import initial_state

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _relative(pb, Q, Cm):
    gamma = pb["gamma"] or 5.0 / 3.0
    rho, E = Q[:, 0], Q[:, 4]
    P = (gamma - 1.0) * (E - 0.5 * (Q[:, 1:4] ** 2).sum(1) / rho)
    tau = pb["mu_ref"] / P  # omega = 0
    scale = np.column_stack([rho] * 4 + [E]) / tau[:, None]
    return float((np.abs(Cm) / scale).max())


CASES = {
    "sod1d": (wl.sod1d(nelem=6, order=2, nv1=12), "sod1d"),
    "box2d": (wl.box2d(n=3, order=3, nv1=16), "box2d"),
    "tgv3d_p3": (wl.tgv3d(n=2, order=3, nv1=12), "tgv3d"),
    "mach2_p2": (wl.mach2(n=2, order=2, nv1=16), "mach2"),
}


@pytest.mark.parametrize("name", list(CASES))
def test_collision_term_conserves_in_every_precision(name):
    import torch
    from paper_2308_06196_amd import bgk
    pb, kind = CASES[name]
    f0 = initial_state(pb, kind, seed=41, amp=0.3)
    for prec in (bgk.FP64, bgk.FP32, bgk.BF16):
        _say("collision moments", name, bgk.PRECISION_NAME[prec])
        s = bgk.Solver(pb, precision=prec)
        s.set_state(torch.from_numpy(f0).to("cuda:0"))
        Q = s.moments().cpu().numpy()
        Cm = s.collision_moments().cpu().numpy()
        r0 = _relative(pb, Q, Cm)
        # and after a few steps (stored FP32 state / BF16 increments)
        dt = s.stable_dt(0.1)
        s.rk3_step(dt, 3)
        Q = s.moments().cpu().numpy()
        Cm = s.collision_moments().cpu().numpy()
        r1 = _relative(pb, Q, Cm)
        print(f"  {name} {bgk.PRECISION_NAME[prec]}: collision moments {r0:.2e} "
              f"(after 3 steps {r1:.2e})", flush=True)
        assert r0 <= 1e-13 and r1 <= 1e-13
        # the stage kernels keep stepping from where the measurement left off
        s.rk3_step(dt, 1)
        s.diagnostics()
        s.close()


def test_collision_moments_see_the_non_conservative_model():
    import torch
    from paper_2308_06196_amd import bgk
    pb = dict(wl.sod1d(nelem=4, order=2, nv1=8, vmax=4.0), equilibrium=1)
    _say("collision moments, continuous Maxwellian on 8^3")
    f0 = initial_state(pb, "sod1d", seed=42, amp=0.3)
    s = bgk.Solver(pb, precision=bgk.FP64)
    s.set_state(torch.from_numpy(f0).to("cuda:0"))
    r = _relative(pb, s.moments().cpu().numpy(), s.collision_moments().cpu().numpy())
    print(f"  continuous model: {r:.2e}", flush=True)
    assert r > 1e-5
    s.close()


def test_collision_moments_zero_without_collisions_and_host_buffers():
    import torch
    from paper_2308_06196_amd import bgk
    pb, kind = CASES["box2d"]
    f0 = initial_state(pb, kind, seed=43, amp=0.2)
    _say("collision moments, host buffer and collisionless")
    s = bgk.Solver(pb, precision=bgk.FP32)
    s.set_state(torch.from_numpy(f0).to("cuda:0"))
    out = np.zeros((s.nx, 5))
    s.collision_moments(out)
    dev = s.collision_moments().cpu().numpy()
    assert np.array_equal(out, dev)
    s.close()
    s = bgk.Solver(dict(pb, mu_ref=0.0), precision=bgk.FP64)
    s.set_state(torch.from_numpy(f0).to("cuda:0"))
    assert np.abs(s.collision_moments().cpu().numpy()).max() == 0.0
    s.close()
