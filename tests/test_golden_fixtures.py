"""The stored long-run fixtures (tests/golden/make_golden.py, FP64 oracle)
still describe the current workloads, and hold what conservation fixes for
them: the per-node moments Q = (rho, rho U, E) after the run have positive
density and energy, zero total momentum (the 2-D and Taylor-Green velocity
fields integrate to zero over the periodic box and the scheme conserves
momentum; the Mach-2 stream has none across it), and total mass 1 for the
2-D and Mach-2 boxes (their density modes integrate to zero; the sampled
Maxwellians' trapezoid moments differ from the continuous ones only in the
far tails of the velocity range), with the Mach-2 stream's momentum
2 sqrt(gamma) per unit mass."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2308_06196_amd import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")
CASES = {"box2d": (wl.box2d(), 200, "box2d"), "tgv3d_n8": (wl.tgv3d(n=8), 100, "tgv3d"),
         "mach2_n8": (wl.mach2(n=8), 50, "mach2")}


def _weights(pb):
    _, wq = orc.gauss_legendre(pb["order"] + 1)
    W = wq
    for _ in range(pb["dim"] - 1):
        W = np.outer(W, wq).ravel()
    ne = int(np.prod(pb["nelem"][: pb["dim"]]))
    jac = np.prod([(pb["xhi"][k] - pb["xlo"][k]) / pb["nelem"][k] / 2.0 for k in range(pb["dim"])])
    return np.tile(W, ne) * jac


@pytest.mark.parametrize("name", list(CASES))
def test_fixture_matches_workload_and_conservation(name):
    meta = json.load(open(os.path.join(GOLD, f"{name}.json")))
    Q = np.load(os.path.join(GOLD, f"{name}_q.npy"))
    pb, steps, kind = CASES[name]
    assert meta["steps"] == steps and meta["kind"] == kind
    for k, v in pb.items():
        assert np.array_equal(np.asarray(meta["problem"][k]), np.asarray(v)), k
    ne = int(np.prod(pb["nelem"][: pb["dim"]]))
    assert Q.shape == (ne * (pb["order"] + 1) ** pb["dim"], 5)
    assert np.isfinite(Q).all() and (Q[:, 0] > 0).all() and (Q[:, 4] > 0).all()
    assert meta["oracle_diag"]["newton_fail"] == 0
    W = _weights(pb)
    vol = np.prod([pb["xhi"][k] - pb["xlo"][k] for k in range(pb["dim"])])
    mass = float(W @ Q[:, 0])
    mom = W @ Q[:, 1:4]
    if kind == "mach2":
        assert np.abs(mom[1:]).max() < 1e-12 * mass
        u = 2.0 * np.sqrt(5.0 / 3.0)
        assert abs(mom[0] / mass - u) < 1e-6 * u
        assert abs(mass / vol - 1.0) < 1e-6
    else:
        assert np.abs(mom).max() < 1e-12 * mass
    if name == "box2d":
        assert abs(mass / vol - 1.0) < 1e-7
