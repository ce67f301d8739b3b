"""Taylor-Green diagnostics (kinetic energy, enstrophy) against the closed forms
of the incompressible Taylor-Green field at unit density: with
U = U0 (sin x cos y cos z, -cos x sin y cos z, 0) on [0, 2 pi]^3,
int |U|^2 / 2 = U0^2 pi^3 and int |curl U|^2 / 2 = 3 U0^2 pi^3. The element-local
derivative converges at order p + 1."""
import math

import numpy as np

from oracle import oracle as orc
from paper_2308_06196_amd import diagnostics as dg
from paper_2308_06196_amd import workloads as wl
from tests.helpers import oracle_problem


def _tgv_moments(pb):
    x = orc.node_coords(oracle_problem(pb))
    U0 = 0.1 * math.sqrt(5.0 / 3.0)
    U = np.stack([U0 * np.sin(x[:, 0]) * np.cos(x[:, 1]) * np.cos(x[:, 2]),
                  -U0 * np.cos(x[:, 0]) * np.sin(x[:, 1]) * np.cos(x[:, 2]),
                  np.zeros(len(x))], 1)
    Q = np.zeros((len(x), 5))
    Q[:, 0] = 1.0
    Q[:, 1:4] = U
    Q[:, 4] = 0.5 * (U * U).sum(1) + 1.5
    return Q, U0


def test_tgv_integrals_closed_form_and_order():
    errs = []
    for n in (4, 8, 16):
        pb = wl.tgv3d(n=n, order=3, nv1=4)
        Q, U0 = _tgv_moments(pb)
        r = dg.integrals(pb, Q)
        assert abs(r["mass"] / (2 * math.pi) ** 3 - 1) < 1e-13
        assert abs(r["kinetic_energy"] / (U0 ** 2 * math.pi ** 3) - 1) < 1e-12
        assert abs(r["mean_pressure"] / (2 * math.pi) ** 3 - 1) < 1e-13  # P = (2/3)(3/2)
        errs.append(abs(r["enstrophy"] / (3 * U0 ** 2 * math.pi ** 3) - 1))
    assert errs[1] < 5e-4
    assert errs[0] / errs[1] > 12 and errs[1] / errs[2] > 12  # order p + 1 = 4
