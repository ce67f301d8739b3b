"""Continuum-limit pin: the oracle's shock tube approaches the exact Euler Riemann
solution as Kn decreases (BGK recovers the hydrodynamic equations in the continuum
limit, Dzanic & Martinelli Sec. 1-2). The exact solver is itself pinned to Toro's
printed star state."""
import math
import os

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2308_06196_amd import workloads as wl
from tests import riemann

GOLD = os.path.join(os.path.dirname(__file__), "golden", "toro_sod_gamma14.txt")


def test_exact_riemann_solver_matches_toro():
    vals = {}
    for line in open(GOLD):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    p, u, rL, rR = riemann.star_state((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4)
    assert abs(p - vals["p_star"]) < 6e-6
    assert abs(u - vals["u_star"]) < 6e-6
    assert abs(rL - vals["rho_star_L"]) < 6e-6
    assert abs(rR - vals["rho_star_R"]) < 6e-6


def _sod_l1(kn, ne=64, t_end=0.1):
    pb = wl.sod1d(nelem=ne, order=2, kn=kn)
    pb["nvel"] = [24, 8, 8]
    keys = ["dim", "order", "nelem", "xlo", "xhi", "nvel", "vlo", "vhi", "bc", "mu_ref",
            "theta_ref", "omega", "gamma", "limiter", "newton_maxit", "newton_tol"]
    pr = orc.Problem(**{k: pb[k] for k in keys})
    x = orc.node_coords(pr)[:, 0]
    f = orc.maxwellian(pr, wl.prim_sod(orc.node_coords(pr)))
    dt0 = orc.stable_dt(pr, f, 0.1)
    n = int(math.ceil(t_end / dt0))
    f, d = orc.rk3_step(pr, f, t_end / n, n)
    assert d["newton_fail"] == 0
    rho = orc.moments(pr, f)[:, 0]
    ex = riemann.sample((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 5.0 / 3.0, (x - 0.5) / t_end)[:, 0]
    _, wq = orc.gauss_legendre(3)
    W = np.tile(wq, pr.ne) * (0.5 / ne)
    return float(np.sum(W * np.abs(rho - ex)))


def test_sod_approaches_euler_as_kn_decreases():
    errs = [_sod_l1(kn) for kn in (1e-2, 3e-3, 1e-3)]
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] < 0.02, errs
