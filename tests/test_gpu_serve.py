"""Batched serving on the GPU: members advanced by graph replay give bitwise
the same states as the same requests run alone; completions are reported per
member; a failing member does not disturb the others; the request loop
completes a small Poisson mix."""
import sys

import numpy as np
import pytest

from paper_2308_06196_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


MIX = [
    (wl.sod1d(nelem=40, order=2, nv1=8, kn=1e-2), "sod1d", {"amp": 0.1, "k": 2, "phase": 0.3}, 7),
    (wl.box2d(n=6, order=3, nv1=8, kn=1e-2), "box2d", {"amp": 0.05}, 5),
    (wl.sod1d(nelem=33, order=1, nv1=16, kn=1e-3), "sod1d", {"amp": 0.02, "k": 1, "phase": 1.0}, 9),
    (wl.box2d(n=5, order=2, nv1=12, kn=3e-3), "box2d", {"amp": 0.15}, 4),
]


def _solver(torch, pb, kind, args, stream, precision=0):
    from paper_2308_06196_amd import bgk
    s = bgk.Solver(pb, precision=precision, stream=stream)
    s.set_maxwellian(wl.PRIM[kind](s.node_coords(), **args))
    return s, s.stable_dt(0.1)


def test_batch_members_match_solo_runs_bitwise(torch):
    from paper_2308_06196_amd import bgk
    _say("batch-vs-solo", len(MIX))
    stream = torch.cuda.Stream()
    solo = []
    for pb, kind, args, n in MIX:
        s, dt = _solver(torch, pb, kind, args, stream)
        s.rk3_step(dt, n)
        solo.append(s.get_state().cpu().numpy())
        s.close()
    batch = bgk.Batch(stream, 8)
    members = []
    for pb, kind, args, n in MIX:
        s, dt = _solver(torch, pb, kind, args, stream)
        batch.add(s, dt, n)
        members.append(s)
    got = {}
    for _ in range(20):
        batch.step(2)
        for s, err in batch.poll():
            assert err is None
            got[members.index(s)] = s.get_state().cpu().numpy()
    assert len(got) == len(MIX) and batch.size() == 0
    for i in range(len(MIX)):
        assert np.array_equal(got[i], solo[i]), i
    batch.close()


def test_batch_failure_is_isolated(torch):
    from paper_2308_06196_amd import bgk
    _say("batch-failure")
    stream = torch.cuda.Stream()
    batch = bgk.Batch(stream, 4)
    good, dt = _solver(torch, *MIX[0][:3], stream)
    bad = bgk.Solver(MIX[1][0], stream=stream)
    f = np.ascontiguousarray(np.broadcast_to(1e-3, bad.shape))
    f = f.copy()
    f[0, 0, :] = -1.0  # a node with negative density: the equilibrium fails there
    bad.set_state(f)
    batch.add(good, dt, 3)
    batch.add(bad, 1e-4, 3)
    batch.step(5)
    res = {id(s): err for s, err in batch.poll()}
    assert res[id(good)] is None
    assert res[id(bad)] == "BGK_ERR_NEWTON"
    batch.close()


def test_request_loop_completes_mix(torch):
    """Shock tubes, periodic boxes and Couette channels (diffuse walls) arriving
    as a Poisson stream all complete."""
    from paper_2308_06196_amd import serve
    _say("serve-mix")
    descs = wl.serving_requests(n=15, seed=1, rate=200.0, nv_choices=(8, 16), steps=10,
                                kinds=("sod1d", "box2d", "channel2d"))
    assert {d["kind"] for d in descs} == {"sod1d", "box2d", "channel2d"}
    for d in descs:  # keep the test small
        pb = d["problem"]
        if pb["dim"] == 2:
            n = min(pb["nelem"][0], 12)
            pb["nelem"] = [n, n, 1]
    reqs = serve.make_requests(descs)
    ex = serve.BatchExecutor(max_members=8)
    m = serve.Server(ex, capacity_bytes=8 << 30, max_members=8, quantum=4).run(reqs)
    ex.close()
    print(m)
    assert m["completed"] == len(reqs) and m["failed"] == 0
    assert m["p99_s"] >= m["p50_s"] > 0
