"""Serving scheduler logic against a CPU stand-in executor on a virtual clock:
admission by footprint, FIFO order, continuous admission while others run,
memory never over-committed, failures isolated to their request."""
import numpy as np
import pytest

from paper_2308_06196_amd import serve
from paper_2308_06196_amd import workloads as wl


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class FakeExecutor(serve.Executor):
    """Members advance together; a step costs dof / rate seconds of virtual time
    per member (the device is shared)."""

    def __init__(self, clock, rate=1e9, fail_admit=(), fail_run=()):
        self.clock, self.rate = clock, rate
        self.fail_admit, self.fail_run = set(fail_admit), set(fail_run)
        self.members = {}
        self.used = 0
        self.max_used = 0
        self.order = []

    def footprint(self, r):
        return r.dof * 8 * 3

    def admit(self, r):
        if r.id in self.fail_admit:
            raise RuntimeError("injected admission failure")
        self.members[r.id] = [r, r.steps]
        self.used += self.footprint(r)
        self.max_used = max(self.max_used, self.used)
        self.order.append(r.id)
        return r.id

    def step(self, n):
        cost = 0.0
        for h, m in self.members.items():
            k = min(n, m[1])
            m[1] -= k
            cost += k * m[0].dof / self.rate
        self.clock.t += cost

    def poll(self):
        out = []
        for h, (r, left) in list(self.members.items()):
            if left == 0:
                out.append((h, "injected member failure" if h in self.fail_run else None))
        return out

    def release(self, h):
        r, _ = self.members.pop(h)
        self.used -= self.footprint(r)


def _requests(n=40, rate=50.0, seed=0):
    return serve.make_requests(wl.serving_requests(n=n, seed=seed, rate=rate,
                                                   nv_choices=(8, 16), steps=20))


def test_all_complete_and_memory_bounded():
    clk = Clock()
    ex = FakeExecutor(clk)
    reqs = _requests()
    cap = int(2.5 * max(ex.footprint(r) for r in reqs))
    m = serve.Server(ex, cap, max_members=8, quantum=5, clock=clk, sleep=clk.sleep).run(reqs)
    assert m["completed"] == len(reqs) and m["failed"] == 0
    assert ex.max_used <= cap
    assert m["p99_s"] >= m["p50_s"] > 0
    for r in reqs:
        assert r.done >= r.admitted >= r.arrival
        assert r.done - r.arrival >= r.steps * r.dof / ex.rate * 0.999


def test_fifo_admission_order():
    clk = Clock()
    ex = FakeExecutor(clk)
    reqs = _requests(seed=3)
    serve.Server(ex, 10 ** 15, max_members=4, quantum=5, clock=clk, sleep=clk.sleep).run(reqs)
    by_arrival = [r.id for r in sorted(reqs, key=lambda r: (r.arrival, r.id))]
    assert ex.order == by_arrival


def test_requests_join_while_others_run():
    clk = Clock()
    ex = FakeExecutor(clk, rate=1e7)
    reqs = _requests(n=20, rate=1000.0, seed=5)
    serve.Server(ex, 10 ** 15, max_members=64, quantum=2, clock=clk, sleep=clk.sleep).run(reqs)
    # some request is admitted after another one started but before it finished
    spans = [(r.admitted, r.done) for r in reqs]
    overlap = any(a1 < a2 < d1 for (a1, d1) in spans for (a2, _) in spans)
    assert overlap


def test_oversized_and_failing_requests_are_isolated():
    clk = Clock()
    reqs = _requests(n=12, seed=7)
    ex = FakeExecutor(clk, fail_admit={reqs[2].id}, fail_run={reqs[5].id})
    big = max(reqs, key=lambda r: r.dof)
    cap = ex.footprint(big) - 1  # the largest request cannot fit at all
    m = serve.Server(ex, cap, max_members=8, quantum=5, clock=clk, sleep=clk.sleep).run(reqs)
    failed = {r.id for r in reqs if r.failed}
    assert {reqs[2].id, reqs[5].id, big.id} <= failed
    assert m["completed"] == len(reqs) - len(failed)
    assert ex.used == 0 and not ex.members


def test_metrics_percentiles():
    rs = []
    for i, lat in enumerate([1.0, 2.0, 3.0, 4.0]):
        r = serve.Request(id=i, problem={}, kind="x", prim_args={}, arrival=0.0, steps=1, dof=10)
        r.admitted, r.done = 0.0, lat
        rs.append(r)
    m = serve.metrics(rs)
    assert m["p50_s"] == pytest.approx(2.5)
    assert m["p99_s"] == pytest.approx(np.percentile([1, 2, 3, 4], 99))
    assert m["dof_updates_per_s"] == pytest.approx(40 / 4.0)


def test_sjf_admits_least_work_first():
    clk = Clock()
    ex = FakeExecutor(clk)
    reqs = _requests(n=16, rate=None, seed=4)  # all arrive at t = 0
    serve.Server(ex, 10 ** 15, max_members=1, quantum=5, clock=clk, sleep=clk.sleep,
                 policy="sjf").run(reqs)
    work = {r.id: r.dof * r.steps for r in reqs}
    order = [work[i] for i in ex.order]
    assert order == sorted(order)


def test_sjf_lowers_median_latency_under_saturation():
    res = {}
    for policy in ("fifo", "sjf"):
        clk = Clock()
        ex = FakeExecutor(clk)
        reqs = _requests(n=24, rate=None, seed=6)
        res[policy] = serve.Server(ex, 10 ** 15, max_members=2, quantum=5, clock=clk,
                                   sleep=clk.sleep, policy=policy).run(reqs)
    assert res["sjf"]["p50_s"] < res["fifo"]["p50_s"]
    assert res["sjf"]["completed"] == res["fifo"]["completed"] == 24


def test_arena_first_fit_merge_and_reuse():
    """The workspace arena (on a host tensor here): first fit, offsets on the
    alignment, released ranges merged with free neighbours, the whole arena
    one free range again once everything is released."""
    a = serve.DeviceArena(64 * 1024, device="cpu", align=1024)
    assert a.fits(64 * 1024) and not a.fits(64 * 1024 + 1)
    offs = [a.alloc(n) for n in (1000, 3000, 1024, 5000)]
    assert [o for o, _ in offs] == [0, 1024, 4096, 5120]
    assert [v.numel() for _, v in offs] == [1000, 3000, 1024, 5000]
    assert a.in_use() == 1024 + 3072 + 1024 + 5120
    # views are disjoint slices of the one buffer
    for (o, v) in offs:
        assert v.data_ptr() == a.buf.data_ptr() + o
    a.release(1024, 3000)          # hole of 3072 between two ranges
    assert a.free[0] == (1024, 3072)
    o, _ = a.alloc(2048)           # first fit takes the hole
    assert o == 1024
    a.release(0, 1000)
    a.release(1024, 2048)          # merges with both free neighbours
    assert a.free[0] == (0, 4096)
    a.release(4096, 1024)          # merges across: 0 .. 5120 free
    assert a.free[0] == (0, 5120)
    a.release(5120, 5000)
    assert a.free == [(0, 64 * 1024)] and a.in_use() == 0
    with pytest.raises(MemoryError):
        a.alloc(64 * 1024 + 1)


def test_arena_fragmentation_defers_admission():
    """A request that fits the pool's total but no free range of the arena
    waits for a completion instead of failing."""
    clk = Clock()

    class ArenaFake(FakeExecutor):
        def __init__(self, *a, **k):
            super().__init__(*a, **k)
            self.arena = serve.DeviceArena(1 << 16, device="cpu", align=1 << 10)
            self.rng = {}

        def footprint(self, r):
            return r.footprint_bytes

        def fits(self, r):
            return self.arena.fits(r.footprint_bytes)

        def admit(self, r):
            off, _ = self.arena.alloc(r.footprint_bytes)
            self.rng[r.id] = (off, r.footprint_bytes)
            return super().admit(r)

        def release(self, h):
            self.arena.release(*self.rng.pop(h))
            super().release(h)

    ex = ArenaFake(clk, rate=1e6)
    reqs = []
    # A, B, C fill the arena; A and C finish early, leaving two 16 KiB holes:
    # D (32 KiB) fits the total but no hole until B is done
    for i, (kb, steps) in enumerate([(16, 1), (32, 50), (16, 1), (32, 1)]):
        r = serve.Request(id=i, problem={}, kind="x", prim_args={}, arrival=0.0, steps=steps,
                          dof=1000)
        r.footprint_bytes = kb << 10
        reqs.append(r)
    m = serve.Server(ex, 1 << 16, max_members=4, quantum=1, clock=clk, sleep=clk.sleep,
                     policy="fifo").run(reqs)
    assert m["completed"] == 4 and m["failed"] == 0
    assert ex.order == [0, 1, 2, 3]
    d = reqs[3]
    assert d.admitted >= reqs[1].done  # waited for B's range
    assert ex.arena.in_use() == 0


def test_large_requests_run_one_at_a_time_beside_small_ones():
    """With a large-request limit no two requests of large_dof DOF or more are
    resident together, small requests are admitted while a large one runs, and
    everything completes."""
    clk = Clock()

    class Watch(FakeExecutor):
        def __init__(self, *a, **k):
            super().__init__(*a, **k)
            self.max_large = 0
            self.small_beside_large = 0

        def admit(self, r):
            h = super().admit(r)
            large = [m for m in self.members.values() if m[0].dof >= 5000]
            self.max_large = max(self.max_large, len(large))
            if large and r.dof < 5000:
                self.small_beside_large += 1
            return h

    reqs = []
    for i in range(12):
        dof = 8000 if i % 3 == 0 else 500
        r = serve.Request(id=i, problem={}, kind="x", prim_args={}, arrival=0.01 * i,
                          steps=10 if dof > 1000 else 3, dof=dof)
        reqs.append(r)
    ex = Watch(clk, rate=1e6)
    m = serve.Server(ex, 10 ** 15, max_members=4, quantum=1, clock=clk, sleep=clk.sleep,
                     policy="sjf", large_dof=5000).run(reqs)
    assert m["completed"] == 12 and m["failed"] == 0
    assert ex.max_large == 1
    assert ex.small_beside_large > 0
    # without the limit the large ones share the device
    clk2 = Clock()
    ex2 = Watch(clk2, rate=1e6)
    for r in reqs:
        r.admitted = r.done = None
    serve.Server(ex2, 10 ** 15, max_members=4, quantum=1, clock=clk2, sleep=clk2.sleep,
                 policy="sjf").run(reqs)
    assert ex2.max_large > 1


def test_sjf_max_wait_admits_the_oldest():
    """Under sjf a large request waits while smaller ones keep arriving; past
    max_wait the oldest arrived request goes first."""
    def run(max_wait):
        clk = Clock()
        ex = FakeExecutor(clk, rate=1e6)
        reqs = [serve.Request(id=0, problem={}, kind="x", prim_args={}, arrival=0.0001,
                              steps=5, dof=10000)]
        # small requests (0.0005 s each) arriving every 0.0001 s
        reqs += [serve.Request(id=i, problem={}, kind="x", prim_args={},
                               arrival=0.0 if i == 1 else 0.0001 * i, steps=5, dof=100)
                 for i in range(1, 30)]
        serve.Server(ex, 10 ** 15, max_members=1, quantum=5, clock=clk, sleep=clk.sleep,
                     policy="sjf", max_wait=max_wait).run(reqs)
        return ex.order.index(0)
    assert run(None) == 29          # passed over until the stream ends
    assert 0 < run(0.002) < 10
