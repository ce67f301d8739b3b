"""Seeded synthetic workloads shaped like the paper's flows.

This module only states problems and initial primitive fields
(rho, U, theta) as functions of the node coordinates. It holds none of the
method's arithmetic (no quadrature, Maxwellian, moments or operators): the
HIP path and the oracle each turn these fields into a distribution function
with their own code. Both the product (benchmark, serving generator) and the
test-suite use it.

Nondimensionalisation: rho_ref = theta_ref = L_ref = 1, velocities in units of
sqrt(R T_ref); the viscosity law is mu = Kn (theta/theta_ref)^omega, so that
tau = mu / P (Sec. 2, BGK relaxation time).

Workloads (Cartesian boxes, 3-D velocity grids; the paper's own cases use
meshes and reference data that are not available, these stand in for them):
  sod1d   1-D shock tube on [0,1], specular walls, p=2, 32 elements, 16^3 on
          [-6,6]^3, left (1,0,1), right (0.125,0,0.8), Kn=1e-2.
  box2d   2-D periodic box [0,1]^2, 32x32 elements, p=3, 24^3 on [-6,6]^3,
          rho = 1 + 0.1 sin(2 pi x) sin(2 pi y), U = (0.1 cos 2 pi y,
          0.1 sin 2 pi x, 0), theta = 1, Kn=1e-3.
  tgv3d   3-D periodic Taylor-Green box [0,2 pi]^3, 16^3 elements, p=3,
          16^3 on [-5,5]^3, Mach 0.1, isothermal, Kn=1e-3.
  mach2   3-D periodic box [0,1]^3, 32^3 elements, p=2, 20^3 on [-8,8]^3,
          Mach-2 stream plus 5 % random-phase density/temperature modes.
  channel2d  Couette channel [0,1]^2, periodic in x, diffuse walls at y = 0, 1
          moving with -/+ 0.2 along x at unit temperature; gas initially at
          rest (8x8 elements, p=2, 12^3 on [-6,6]^3, Kn=1e-2 by default).
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = 5.0 / 3.0


def problem(dim, order, nelem, xlo, xhi, nvel, vlo, vhi, kn, bc=None, limiter=1):
    """Plain dict describing one problem; both sides build their own struct."""
    bc = bc if bc is not None else [(0, 0)] * dim
    pad = lambda t, v: list(t) + [v] * (3 - len(t))
    return {
        "dim": dim, "order": order,
        "nelem": pad(nelem, 1), "xlo": pad(xlo, 0.0), "xhi": pad(xhi, 1.0),
        "bc": [tuple(b) for b in bc] + [(0, 0)] * (3 - len(bc)),
        "nvel": list(nvel), "vlo": list(vlo), "vhi": list(vhi),
        "mu_ref": float(kn), "theta_ref": 1.0, "omega": 0.0, "gamma": 0.0,
        "limiter": limiter, "newton_maxit": 20, "newton_tol": 1e-14,
        "equilibrium": 0, "sutherland": 0.0,
        "wall_theta": [(1.0, 1.0)] * 3, "wall_vel": [((0.0,) * 3,) * 2] * 3,
    }


def dof(pb) -> int:
    ne = int(np.prod(pb["nelem"][: pb["dim"]]))
    return ne * (pb["order"] + 1) ** pb["dim"] * int(np.prod(pb["nvel"]))


# --------------------------------------------------------------------------
# Problems
# --------------------------------------------------------------------------

def sod1d(nelem=32, order=2, nv1=16, vmax=6.0, kn=1e-2):
    return problem(1, order, [nelem], [0.0], [1.0], [nv1] * 3, [-vmax] * 3, [vmax] * 3, kn,
                   bc=[(1, 1)])


def box2d(n=32, order=3, nv1=24, vmax=6.0, kn=1e-3):
    return problem(2, order, [n, n], [0.0, 0.0], [1.0, 1.0], [nv1] * 3, [-vmax] * 3,
                   [vmax] * 3, kn)


def tgv3d(n=16, order=3, nv1=16, vmax=5.0, kn=1e-3):
    L = 2.0 * math.pi
    return problem(3, order, [n] * 3, [0.0] * 3, [L] * 3, [nv1] * 3, [-vmax] * 3, [vmax] * 3, kn)


def mach2(n=32, order=2, nv1=20, vmax=8.0, kn=1e-2):
    return problem(3, order, [n] * 3, [0.0] * 3, [1.0] * 3, [nv1] * 3, [-vmax] * 3, [vmax] * 3, kn)


def channel2d(nx=8, ny=8, order=2, nv1=12, vmax=6.0, kn=1e-2, uw=0.2, theta_w=1.0):
    """Couette channel: periodic in x, diffuse (Maxwell) walls at y = 0 and
    y = 1 moving with -uw and +uw along x at temperature theta_w."""
    pb = problem(2, order, [nx, ny], [0.0, 0.0], [1.0, 1.0], [nv1] * 3, [-vmax] * 3,
                 [vmax] * 3, kn, bc=[(0, 0), (2, 2)])
    pb["wall_theta"] = [(1.0, 1.0), (theta_w, theta_w), (1.0, 1.0)]
    pb["wall_vel"] = [((0.0,) * 3,) * 2, ((-uw, 0.0, 0.0), (uw, 0.0, 0.0)), ((0.0,) * 3,) * 2]
    return pb


# --------------------------------------------------------------------------
# Initial primitive fields: x [nx, dim] -> prim [nx, 5] = (rho, Ux, Uy, Uz, theta)
# --------------------------------------------------------------------------

def prim_sod(x, amp=0.0, k=1, phase=0.0):
    """Left (1, 0, 1) for x < 0.5, right (0.125, 0, 0.8); optional seeded
    perturbation rho *= 1 + amp sin(2 pi k x + phase) (serving mix)."""
    xx = x[:, 0]
    left = xx < 0.5
    prim = np.zeros((len(xx), 5))
    prim[:, 0] = np.where(left, 1.0, 0.125)
    prim[:, 4] = np.where(left, 1.0, 0.8)
    if amp:
        prim[:, 0] *= 1.0 + amp * np.sin(2 * math.pi * k * xx + phase)
    return prim


def prim_box2d(x, amp=0.1):
    X, Y = x[:, 0], x[:, 1]
    prim = np.zeros((len(X), 5))
    prim[:, 0] = 1.0 + amp * np.sin(2 * math.pi * X) * np.sin(2 * math.pi * Y)
    prim[:, 1] = amp * np.cos(2 * math.pi * Y)
    prim[:, 2] = amp * np.sin(2 * math.pi * X)
    prim[:, 4] = 1.0
    return prim


def prim_tgv3d(x, mach=0.1):
    """Isothermal compressible Taylor-Green vortex: theta = 1, rho = p."""
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    U0 = mach * math.sqrt(GAMMA)
    prim = np.zeros((len(X), 5))
    prim[:, 1] = U0 * np.sin(X) * np.cos(Y) * np.cos(Z)
    prim[:, 2] = -U0 * np.cos(X) * np.sin(Y) * np.cos(Z)
    p = 1.0 + (U0 ** 2 / 16.0) * (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0)
    prim[:, 0] = p
    prim[:, 4] = 1.0
    return prim


def prim_mach2(x, seed=0):
    """Mach-2 stream along x with 5 % random-phase sinusoidal modes in rho and theta."""
    rng = np.random.default_rng(seed)

    def modes():
        m = np.zeros(len(x))
        for _ in range(4):
            k = rng.integers(1, 4, size=3)
            ph = rng.uniform(0.0, 2 * math.pi)
            m += np.sin(2 * math.pi * (x @ k) + ph)
        return 0.25 * m

    prim = np.zeros((len(x), 5))
    prim[:, 0] = 1.0 + 0.05 * modes()
    prim[:, 4] = 1.0 + 0.05 * modes()
    prim[:, 1] = 2.0 * math.sqrt(GAMMA)
    return prim


def prim_channel(x, amp=0.0, k=1, phase=0.0):
    """Gas at rest at unit temperature; optional seeded density modulation along
    the channel, rho = 1 + amp sin(2 pi k x + phase)."""
    prim = np.zeros((len(x), 5))
    prim[:, 0] = 1.0 + amp * np.sin(2 * math.pi * k * x[:, 0] + phase)
    prim[:, 4] = 1.0
    return prim


PRIM = {"sod1d": prim_sod, "box2d": prim_box2d, "tgv3d": prim_tgv3d, "mach2": prim_mach2,
        "channel2d": prim_channel}


def perturbation(seed: int, shape, amp: float = 0.3) -> np.ndarray:
    """Seeded multiplicative factor 1 + amp U[-1, 1] (keeps a positive f positive)."""
    rng = np.random.default_rng(seed)
    return 1.0 + amp * rng.uniform(-1.0, 1.0, size=shape)


# --------------------------------------------------------------------------
# Serving mix: Poisson arrivals of shock-tube and periodic-box requests
# --------------------------------------------------------------------------

def serving_requests(n=256, seed=0, rate=None, nv_choices=(8, 16, 24, 32), steps=100,
                     kinds=("sod1d", "box2d")):
    """Request descriptors drawn uniformly from `kinds`: 1-D shock tube with
    32..512 elements, 2-D periodic box with 16^2..64^2 elements, and (when
    listed) 2-D Couette channel with 16^2..64^2 elements, wall speed in
    [0.05, 0.3] and wall temperature in [0.8, 1.2]; p in {1,2,3}; N_1d from
    nv_choices; Kn log-uniform in [1e-4, 1]; perturbation amplitude in
    [0.01, 0.2]. Arrival times are Poisson with the given rate (all at 0 when
    rate is None)."""
    rng = np.random.default_rng(seed)
    # arrivals from a stream of their own: the requests do not depend on the rate
    rng_t = np.random.default_rng([seed, 7919])
    out = []
    t = 0.0
    for r in range(n):
        kind = kinds[int(rng.integers(0, len(kinds)))]
        order = int(rng.integers(1, 4))
        nv1 = int(rng.choice(nv_choices))
        kn = float(10.0 ** rng.uniform(-4.0, 0.0))
        amp = float(rng.uniform(0.01, 0.2))
        if kind == "sod1d":
            ne = int(rng.integers(32, 513))
            pb = sod1d(nelem=ne, order=order, nv1=nv1, kn=kn)
            prim_args = {"amp": amp, "k": int(rng.integers(1, 5)),
                         "phase": float(rng.uniform(0, 2 * math.pi))}
        elif kind == "box2d":
            ne1 = int(rng.integers(16, 65))
            pb = box2d(n=ne1, order=order, nv1=nv1, kn=kn)
            prim_args = {"amp": amp}
        elif kind == "channel2d":
            ne1 = int(rng.integers(16, 65))
            pb = channel2d(nx=ne1, ny=ne1, order=order, nv1=nv1, kn=kn,
                           uw=float(rng.uniform(0.05, 0.3)),
                           theta_w=float(rng.uniform(0.8, 1.2)))
            prim_args = {"amp": amp, "k": int(rng.integers(1, 5)),
                         "phase": float(rng.uniform(0, 2 * math.pi))}
        else:
            raise ValueError(kind)
        if rate:
            t += float(rng_t.exponential(1.0 / rate))
        out.append({"id": r, "kind": kind, "problem": pb, "prim_args": prim_args,
                    "arrival": t if rate else 0.0, "steps": steps})
    return out
