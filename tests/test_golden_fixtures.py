"""The stored long-run fixtures (tests/golden/make_golden.py, FP64 oracle)
still describe the current workloads, and hold what conservation fixes for
them: the per-node moments Q = (rho, rho U, E) after the run have positive
density and energy, zero total momentum (both initial velocity fields
integrate to zero over the periodic box and the scheme conserves momentum),
and, for the 2-D box, total mass 1 (its density perturbation integrates to
zero; the sampled Maxwellians' trapezoid moments differ from the continuous
ones only in the far tails of the [-6, 6] velocity range)."""
import json
import os

import numpy as np
import pytest

from oracle import oracle as orc
from paper_2308_06196_amd import workloads as wl

GOLD = os.path.join(os.path.dirname(__file__), "golden")
CASES = {"box2d": (wl.box2d(), 200), "tgv3d_n8": (wl.tgv3d(n=8), 100)}


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
    pb, steps = CASES[name]
    assert meta["steps"] == steps and meta["kind"] == ("box2d" if name == "box2d" else "tgv3d")
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
    assert np.abs(mom).max() < 1e-12 * mass
    if name == "box2d":
        assert abs(mass / vol - 1.0) < 1e-7
