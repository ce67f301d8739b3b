"""Batched serving on the GPU: members advanced by batched launches give bitwise
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


def test_batch_large_member_solo_launches_match_solo_runs_bitwise(torch):
    """Members of 8192 stage work items or more (filling the device alone) run
    their RK stages with their solo launches inside the batch (the column
    sweep where their solver sweeps); beside per-element family members, and
    finishing at different steps, every state is bitwise its solo run's."""
    from paper_2308_06196_amd import bgk
    mix = [
        (wl.box2d(n=32, order=1, nv1=16, kn=1e-2), "box2d", {"amp": 0.1}, 5, 0),   # 16384 items
        (wl.box2d(n=24, order=3, nv1=16, kn=3e-3), "box2d", {"amp": 0.05}, 3, 0),  # 9216 items
        (wl.box2d(n=24, order=2, nv1=16, kn=1e-3), "box2d", {"amp": 0.15}, 2, 0),  # 9216 items
        (wl.box2d(n=32, order=1, nv1=16, kn=1e-2), "box2d", {"amp": 0.1}, 4, 1),   # FP32
        # diffuse walls: wall densities from the batched launches
        (wl.channel2d(nx=32, ny=32, order=1, nv1=16, kn=1e-2, uw=0.2, theta_w=1.1), "channel2d",
         {"amp": 0.05, "k": 1, "phase": 0.0}, 3, 0),
        (wl.box2d(n=6, order=3, nv1=8, kn=1e-2), "box2d", {"amp": 0.1}, 6, 0),
        (wl.sod1d(nelem=40, order=2, nv1=8, kn=1e-2), "sod1d", {"amp": 0.1, "k": 2, "phase": 0.3}, 4, 0),
    ]
    _say("batch-large-solo-vs-solo", len(mix))
    stream = torch.cuda.Stream()
    solo = []
    for pb, kind, args, n, prec in mix:
        s, dt = _solver(torch, pb, kind, args, stream, precision=prec)
        s.rk3_step(dt, n)
        solo.append(s.get_state().cpu().numpy())
        s.close()
    batch = bgk.Batch(stream, 8)
    members = []
    for pb, kind, args, n, prec in mix:
        s, dt = _solver(torch, pb, kind, args, stream, precision=prec)
        batch.add(s, dt, n)
        members.append(s)
    got = {}
    for _ in range(20):
        batch.step(1)
        for s, err in batch.poll():
            assert err is None
            got[members.index(s)] = s.get_state().cpu().numpy()
    assert len(got) == len(mix) and batch.size() == 0
    for i in range(len(mix)):
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


def test_request_loop_with_workspace_arena(torch):
    """The same kind of mix with every workspace cut from one device arena
    (the serving benchmark's set-up), in the batched and the plain server:
    all requests complete and every range is back in the arena at the end."""
    from paper_2308_06196_amd import serve
    _say("serve-arena")
    descs = wl.serving_requests(n=12, seed=3, rate=200.0, nv_choices=(8, 16), steps=10)
    for d in descs:
        pb = d["problem"]
        if pb["dim"] == 2:
            n = min(pb["nelem"][0], 12)
            pb["nelem"] = [n, n, 1]
    cap = 2 << 30
    ex = serve.BatchExecutor(max_members=8, arena_bytes=cap)
    m = serve.Server(ex, capacity_bytes=cap, max_members=8, quantum=4).run(
        serve.make_requests(descs))
    assert ex.arena.in_use() == 0
    ex.close()
    assert m["completed"] == len(descs) and m["failed"] == 0
    q = serve.run_sequential(serve.make_requests(descs), cap, arena=True)
    assert q["completed"] == len(descs) and q["failed"] == 0


def test_batch_admission_mid_run_matches_solo(torch):
    """Continuous batching: a member admitted after the others have stepped, and a
    member that completes while the others go on, each end bitwise equal to the
    same request run alone (members never exchange data; the descriptor tables
    are rewritten around them)."""
    from paper_2308_06196_amd import bgk
    _say("batch mid-run admission")
    stream = torch.cuda.Stream()
    steps = [9, 3, 6]  # MIX[0] long, MIX[1] finishes early, MIX[3] joins late
    idx = [0, 1, 3]
    solo = []
    for i, n in zip(idx, steps):
        pb, kind, args, _ = MIX[i]
        s, dt = _solver(torch, pb, kind, args, stream)
        s.rk3_step(dt, n)
        solo.append(s.get_state().cpu().numpy())
        s.close()
    batch = bgk.Batch(stream, 4)
    members = []
    for i, n in zip(idx[:2], steps[:2]):
        pb, kind, args, _ = MIX[i]
        s, dt = _solver(torch, pb, kind, args, stream)
        batch.add(s, dt, n)
        members.append(s)
    got = {}
    batch.step(2)  # both members have stepped before the third arrives
    pb, kind, args, _ = MIX[idx[2]]
    s, dt = _solver(torch, pb, kind, args, stream)
    batch.add(s, dt, steps[2])
    members.append(s)
    for _ in range(30):
        batch.step(1)
        for m, err in batch.poll():
            assert err is None
            got[members.index(m)] = m.get_state().cpu().numpy()
        if batch.size() == 0:
            break
    assert len(got) == 3
    for k in range(3):
        assert np.array_equal(got[k], solo[k]), k
    batch.close()


def test_batch_table_churn_between_polls(torch):
    """Twenty membership changes without a poll: every change rewrites the
    descriptor tables through the two pinned staging buffers in turn (the
    host waits for the copy out of a buffer before refilling it); every member
    still ends bitwise equal to its solo run."""
    from paper_2308_06196_amd import bgk
    _say("batch table churn")
    stream = torch.cuda.Stream()
    pb_long, kind_long, args_long, _ = MIX[1]
    pb_short, kind_short, args_short, _ = MIX[0]
    s, dt_long = _solver(torch, pb_long, kind_long, args_long, stream)
    s.rk3_step(dt_long, 24)
    ref_long = s.get_state().cpu().numpy()
    s.close()
    s, dt_short = _solver(torch, pb_short, kind_short, args_short, stream)
    s.rk3_step(dt_short, 1)
    ref_short = s.get_state().cpu().numpy()
    s.close()
    batch = bgk.Batch(stream, 32)
    long_m, _ = _solver(torch, pb_long, kind_long, args_long, stream)
    batch.add(long_m, dt_long, 24)
    shorts = []
    for _ in range(20):  # every cycle: one admission and one completion
        m, _ = _solver(torch, pb_short, kind_short, args_short, stream)
        batch.add(m, dt_short, 1)
        shorts.append(m)
        batch.step(1)
    batch.step(10)
    done = dict((id(m), err) for m, err in batch.poll())
    assert len(done) == 21 and all(e is None for e in done.values())
    assert np.array_equal(long_m.get_state().cpu().numpy(), ref_long)
    for m in shorts:
        assert np.array_equal(m.get_state().cpu().numpy(), ref_short)
    batch.close()


def test_batch_families_walls_and_fp32_match_solo_bitwise(torch):
    """Several members of one kernel family in one launch (work-unit lists
    with several ranges), a diffuse-wall channel (wall flux and density
    launches) and FP32 storage next to FP64: every member bitwise equal to its
    solo run. Hexahedra and BF16 increments are refused with
    BGK_ERR_UNSUPPORTED."""
    from paper_2308_06196_amd import bgk
    _say("batch families, walls, fp32")
    cases = [
        (wl.box2d(n=6, order=3, nv1=8, kn=1e-2), "box2d", {"amp": 0.05}, 6, bgk.FP64),
        (wl.box2d(n=9, order=3, nv1=8, kn=3e-2), "box2d", {"amp": 0.1}, 5, bgk.FP64),
        (wl.box2d(n=4, order=3, nv1=12, kn=1e-3), "box2d", {"amp": 0.02}, 7, bgk.FP64),
        (wl.channel2d(nx=6, ny=6, order=2, nv1=12, kn=1e-2, uw=0.2, theta_w=1.1), "channel2d",
         {"amp": 0.05, "k": 1, "phase": 0.2}, 6, bgk.FP64),
        (wl.channel2d(nx=5, ny=5, order=2, nv1=8, kn=3e-2, uw=0.1, theta_w=0.9), "channel2d",
         {"amp": 0.02, "k": 2, "phase": 1.2}, 4, bgk.FP64),
        (wl.box2d(n=6, order=3, nv1=8, kn=1e-2), "box2d", {"amp": 0.05}, 6, bgk.FP32),
        (wl.sod1d(nelem=40, order=2, nv1=8, kn=1e-2), "sod1d",
         {"amp": 0.1, "k": 2, "phase": 0.3}, 9, bgk.FP32),
    ]
    stream = torch.cuda.Stream()
    solo = []
    for pb, kind, args, n, prec in cases:
        s, dt = _solver(torch, pb, kind, args, stream, precision=prec)
        s.rk3_step(dt, n)
        solo.append(s.get_state().cpu().numpy())
        s.close()
    batch = bgk.Batch(stream, 8)
    members = []
    for pb, kind, args, n, prec in cases:
        s, dt = _solver(torch, pb, kind, args, stream, precision=prec)
        batch.add(s, dt, n)
        members.append(s)
    got = {}
    for _ in range(20):
        batch.step(3)
        for s, err in batch.poll():
            assert err is None
            got[members.index(s)] = s.get_state().cpu().numpy()
        if batch.size() == 0:
            break
    assert len(got) == len(cases)
    for i in range(len(cases)):
        assert np.array_equal(got[i], solo[i]), i
    for pb, prec in ((wl.tgv3d(n=2, order=1, nv1=8), bgk.FP64),
                     (wl.box2d(n=4, order=2, nv1=8), bgk.BF16)):
        s = bgk.Solver(pb, precision=prec, stream=stream)
        s.set_maxwellian(wl.PRIM["tgv3d" if pb["dim"] == 3 else "box2d"](s.node_coords()))
        with pytest.raises(bgk.BGKError) as exc:
            batch.add(s, 1e-3, 2)
        assert exc.value.status == 2  # BGK_ERR_UNSUPPORTED
        s.close()
    batch.close()


def test_batch_poll_without_waiting_matches_solo(torch):
    """Non-blocking polls (bgk_batch_poll_ready) hand back a member only once
    the device has executed its last replay; members released that way (no
    stream synchronisation) end bitwise equal to their solo runs, and the
    queue of replays ahead of the device stays bounded."""
    from paper_2308_06196_amd import bgk
    _say("batch poll without waiting")
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
    for _ in range(200):
        batch.step(1)
        for s, err in batch.poll(block=batch.size() == 0):
            assert err is None
            got[members.index(s)] = s.get_state().cpu().numpy()
        if len(got) == len(MIX):
            break
    assert len(got) == len(MIX)
    for i in range(len(MIX)):
        assert np.array_equal(got[i], solo[i]), i
    batch.close()
