"""Continuous-batching request loop for BGK solves (serving pattern).

Requests (shock tubes, periodic boxes, channels) arrive over time. The server
admits them (oldest first, or least work first) as soon as their device-memory
footprint fits the pool and a member slot is free; admitted requests stay resident and advance
together: every launch of a quantum covers all members of one kernel family
(descriptor tables in device memory), so small members' work fills the device
beside the large ones'. Finished requests free their memory and slot for waiting ones.
Latency = completion - arrival; p50/p99 and aggregate DOF-updates/s are
reported.

The scheduling logic is independent of the device: `Server` drives any object
with the `Executor` interface. `BatchExecutor` is the GPU one (libbgk batch
C-ABI); tests drive `Server` with a CPU stand-in.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import Callable, List, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    id: int
    problem: dict
    kind: str
    prim_args: dict
    arrival: float
    steps: int
    precision: int = 0
    # filled by the server
    footprint: int = 0
    dof: int = 0
    admitted: Optional[float] = None
    done: Optional[float] = None
    failed: Optional[str] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


class Executor:
    """Device side of the server. `admit` allocates and initialises one request
    and makes it a batch member; `step(n)` advances every member by up to n
    steps (members stop at their own step count); `poll` returns the handles
    of members that have completed (after waiting for queued work) as pairs
    (handle, error or None); `release` frees a completed member."""

    def footprint(self, req: Request) -> int: ...
    def admit(self, req: Request): ...
    def step(self, n: int) -> None: ...
    def poll(self) -> list: ...
    def release(self, handle) -> None: ...

    def fits(self, req: Request) -> bool:
        """Whether `admit` can place the request now (beyond the pool total:
        an executor with its own arena may be fragmented)."""
        return True


class DeviceArena:
    """One device allocation that the workspaces of admitted requests are cut
    from: first fit over the free ranges, a released range merged with its free
    neighbours, offsets rounded to `align` bytes. Admitting a request then
    calls no device allocator: a caching allocator that has to return cached
    blocks to the device to place a large workspace synchronises the device
    and frees and maps memory while the resident members' queued work runs
    out. A range is released only once the device has executed every launch
    that names it (the executors release members after their completion)."""

    def __init__(self, nbytes: int, device="cuda:0", align: int = 1 << 21):
        import torch

        self.align = int(align)
        self.nbytes = int(nbytes) // self.align * self.align
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        self.free = [(0, self.nbytes)]  # (offset, size), sorted by offset, never adjacent

    def _size(self, n: int) -> int:
        return -(-int(n) // self.align) * self.align

    def fits(self, n: int) -> bool:
        need = self._size(n)
        return any(sz >= need for _, sz in self.free)

    def alloc(self, n: int):
        """(offset, uint8 view of n bytes) of the first free range that holds n."""
        need = self._size(n)
        for k, (off, sz) in enumerate(self.free):
            if sz >= need:
                if sz == need:
                    del self.free[k]
                else:
                    self.free[k] = (off + need, sz - need)
                return off, self.buf.narrow(0, off, int(n))
        raise MemoryError(f"arena: no free range of {need} bytes")

    def release(self, off: int, n: int) -> None:
        need = self._size(n)
        k = 0
        while k < len(self.free) and self.free[k][0] < off:
            k += 1
        self.free.insert(k, (off, need))
        # merge with the following, then with the preceding range
        if k + 1 < len(self.free) and off + need == self.free[k + 1][0]:
            self.free[k] = (off, need + self.free[k + 1][1])
            del self.free[k + 1]
        if k > 0 and self.free[k - 1][0] + self.free[k - 1][1] == off:
            self.free[k - 1] = (self.free[k - 1][0], self.free[k - 1][1] + self.free[k][1])
            del self.free[k]

    def in_use(self) -> int:
        return self.nbytes - sum(sz for _, sz in self.free)


class Server:
    """policy: "fifo" admits arrived requests in arrival order; "sjf" admits the
    arrived request with the least work (DOF x steps) first, which lowers the
    median latency when the pool or the member slots are the bottleneck.
    large_dof / max_large: requests of large_dof phase-space DOF or more are
    resident at most max_large at a time (the others wait, small requests go
    past them); shared by several large solves the device would stretch each
    one's time to solution by their number."""

    def __init__(self, executor: Executor, capacity_bytes: int, max_members: int = 64,
                 quantum: int = 10, clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep, policy: str = "fifo",
                 max_wait: Optional[float] = None, large_dof: Optional[int] = None,
                 max_large: int = 1):
        if policy not in ("fifo", "sjf"):
            raise ValueError(policy)
        # sjf: a request that has waited longer than max_wait seconds goes
        # first (oldest first), so large requests are not passed over forever
        self.max_wait = max_wait
        # at most max_large requests of large_dof phase-space DOF or more are
        # resident at once: large solves then do not share the device with
        # each other (each runs at close to its solo speed, which bounds the
        # tail), while small ones keep joining beside them
        self.large_dof = large_dof
        self.max_large = int(max_large)
        self.n_large = 0
        self.ex = executor
        self.capacity = int(capacity_bytes)
        self.max_members = int(max_members)
        self.quantum = int(quantum)
        self.clock = clock
        self.sleep = sleep
        self.policy = policy
        self.used = 0
        self.active = {}  # handle -> Request

    def _large(self, r) -> int:
        return int(self.large_dof is not None and r.dof >= self.large_dof)

    def _next(self, pending, t):
        """Index of the next request to admit among those arrived by t (or
        None): the oldest (fifo, or sjf past max_wait) or the least work (sjf),
        among the requests the large-request limit lets in now."""
        full = self.n_large >= self.max_large
        best = None
        for i, r in enumerate(pending):
            if r.arrival > t:
                break
            if full and self._large(r):
                continue
            if self.policy == "fifo":
                return i
            if self.max_wait is not None and t - r.arrival > self.max_wait:
                return i
            if best is None or r.dof * r.steps < pending[best].dof * pending[best].steps:
                best = i
        return best

    def run(self, requests: List[Request]) -> dict:
        pending = sorted(requests, key=lambda r: (r.arrival, r.id))
        for r in pending:
            r.footprint = int(self.ex.footprint(r))
            if r.footprint > self.capacity:
                r.failed = "footprint exceeds the pool"
        pending = [r for r in pending if r.failed is None]
        t0 = self.clock()
        now = lambda: self.clock() - t0
        finished: List[Request] = []
        while pending or self.active:
            t = now()
            # admission by the policy, while memory and slots allow
            while len(self.active) < self.max_members:
                i = self._next(pending, t)
                if (i is None or self.used + pending[i].footprint > self.capacity
                        or not self.ex.fits(pending[i])):
                    break
                r = pending.pop(i)
                try:
                    h = self.ex.admit(r)
                except Exception as exc:  # a request that cannot start fails alone
                    r.failed = f"admit: {exc}"
                    finished.append(r)
                    continue
                r.admitted = now()
                self.used += r.footprint
                self.n_large += self._large(r)
                self.active[h] = r
            if not self.active:
                if pending:
                    wait = pending[0].arrival - now()
                    if wait > 0:
                        self.sleep(wait)
                continue
            self.ex.step(self.quantum)
            for h, err in self.ex.poll():
                r = self.active.pop(h)
                r.done = now()
                if err:
                    r.failed = str(err)
                self.used -= r.footprint
                self.n_large -= self._large(r)
                self.ex.release(h)
                finished.append(r)
        return metrics(finished + [r for r in requests if r.failed and r not in finished])


def metrics(reqs: List[Request]) -> dict:
    ok = [r for r in reqs if r.failed is None and r.done is not None]
    lat = np.array([r.latency for r in ok]) if ok else np.zeros(0)
    work = float(sum(r.dof * r.steps for r in ok))
    span = (max(r.done for r in ok) - min(r.arrival for r in ok)) if ok else 0.0
    waits = np.array([r.admitted - r.arrival for r in ok]) if ok else np.zeros(0)
    return {
        "requests": len(reqs), "completed": len(ok), "failed": len(reqs) - len(ok),
        "p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
        "p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
        "mean_admission_wait_s": float(waits.mean()) if len(waits) else None,
        "dof_updates": work, "span_s": span,
        "dof_updates_per_s": work / span if span > 0 else None,
    }


def make_requests(descs, precision: int = 0) -> List[Request]:
    """Request objects from workloads.serving_requests descriptors."""
    out = []
    for d in descs:
        pb = d["problem"]
        ne = int(np.prod(pb["nelem"][: pb["dim"]]))
        dof = ne * (pb["order"] + 1) ** pb["dim"] * int(np.prod(pb["nvel"]))
        out.append(Request(id=d["id"], problem=pb, kind=d["kind"], prim_args=d["prim_args"],
                           arrival=d["arrival"], steps=d["steps"], precision=precision, dof=dof))
    return out


class BatchExecutor(Executor):
    """GPU executor over the libbgk batch C-ABI. Each member owns a torch
    workspace; all members run on the batch's stream, each launch covering
    every member of one kernel family."""

    def __init__(self, device="cuda:0", max_members: int = 64, cfl: float = 0.1,
                 arena_bytes: Optional[int] = None):
        import torch

        from . import bgk
        from . import workloads as wl
        self.torch, self.bgk, self.wl = torch, bgk, wl
        self.stream = torch.cuda.Stream(device=device)  # default priority
        self.init_stream = torch.cuda.Stream(device=device)
        self.device = device
        self.cfl = cfl
        self.batch = bgk.Batch(self.stream, max_members)
        self.members = {}
        # workspaces from one arena (arena_bytes) or from torch's allocator
        self.arena = DeviceArena(arena_bytes, device) if arena_bytes else None
        self.ranges = {}  # handle -> (arena offset, bytes)

    def footprint(self, req: Request) -> int:
        return self.bgk.footprint(req.problem, req.precision)[0]

    def fits(self, req: Request) -> bool:
        return self.arena is None or self.arena.fits(self.footprint(req))

    def admit(self, req: Request):
        # initialise on a side stream (its synchronisation does not wait for
        # the members already running), then move to the batch stream
        ws, rng = None, None
        if self.arena is not None:
            nbytes = self.footprint(req)
            off, ws = self.arena.alloc(nbytes)
            rng = (off, nbytes)
        s = None
        try:
            s = self.bgk.Solver(req.problem, precision=req.precision, device=self.device,
                                stream=self.init_stream, workspace=ws)
            s.set_maxwellian(self.wl.PRIM[req.kind](s.node_coords(), **req.prim_args))
            dt = s.stable_dt(self.cfl)
            s.set_stream(self.stream)
            self.batch.add(s, dt, req.steps)
        except Exception:
            # nothing of this request stays queued once its range is reused
            if s is not None:
                s.close()
            self.init_stream.synchronize()
            if rng is not None:
                self.arena.release(*rng)
            raise
        self.members[id(s)] = s
        if rng is not None:
            self.ranges[id(s)] = rng
        return id(s)

    def step(self, n: int) -> None:
        self.batch.step(n)

    def poll(self) -> list:
        # without waiting while members are still stepping (the device keeps
        # working on the queued replays while the server admits new requests);
        # once none is, wait for the finished ones
        out = []
        for s, err in self.batch.poll(block=self.batch.size() == 0):
            out.append((id(s), err))
        return out

    def release(self, handle) -> None:
        # handed back by poll: the device has executed all of its work, and
        # later replays no longer name it, so its memory is free without
        # waiting for the batch stream
        s = self.members.pop(handle)
        s.close(sync=False)
        rng = self.ranges.pop(handle, None)
        if rng is not None:
            self.arena.release(*rng)

    def close(self):
        self.batch.close()
        # the arena's memory back to the device for whatever runs next
        self.arena = None
        self.ranges.clear()
        self.torch.cuda.synchronize(self.device)
        self.torch.cuda.empty_cache()


class SequentialExecutor(Executor):
    """The plain path: one request at a time on one stream, its kernels
    launched by bgk_rk3_step for that request alone (no overlap), with the same
    set-up work per request as BatchExecutor (solver creation, Maxwellian
    initial state, stable time step). Driven by a Server with one member slot
    and first-come-first-served admission, so its latencies are wall-clock
    times like the batched server's."""

    def __init__(self, device="cuda:0", cfl: float = 0.1, arena_bytes: Optional[int] = None):
        import torch

        from . import bgk
        from . import workloads as wl
        self.torch, self.bgk, self.wl = torch, bgk, wl
        self.device = device
        self.cfl = cfl
        self.stream = torch.cuda.Stream(device=device)  # default priority
        self.members = {}  # handle -> [solver, dt, remaining steps]
        # one request at a time: its workspace is the start of the arena
        self.arena = DeviceArena(arena_bytes, device) if arena_bytes else None

    def footprint(self, req: Request) -> int:
        return self.bgk.footprint(req.problem, req.precision)[0]

    def admit(self, req: Request):
        ws = None
        if self.arena is not None:
            ws = self.arena.buf.narrow(0, 0, self.footprint(req))
        s = self.bgk.Solver(req.problem, precision=req.precision, device=self.device,
                            stream=self.stream, workspace=ws)
        s.set_maxwellian(self.wl.PRIM[req.kind](s.node_coords(), **req.prim_args))
        dt = s.stable_dt(self.cfl)
        self.members[id(s)] = [s, dt, req.steps]
        return id(s)

    def step(self, n: int) -> None:
        for m in self.members.values():
            k = min(n, m[2])
            if k:
                m[0].rk3_step(m[1], k)
                m[2] -= k

    def poll(self) -> list:
        out = []
        for h, (s, _, left) in self.members.items():
            if left == 0:
                try:
                    s.synchronize()
                    out.append((h, None))
                except self.bgk.BGKError as exc:
                    out.append((h, self.bgk.STATUS.get(exc.status, str(exc))))
        return out

    def release(self, handle) -> None:
        s = self.members.pop(handle)[0]
        s.close()

    def close(self):
        for s, _, _ in self.members.values():
            s.close()
        self.members.clear()
        if self.arena is not None:
            self.arena = None
            self.torch.cuda.empty_cache()


def run_sequential(requests: List[Request], capacity_bytes: int, device="cuda:0",
                   cfl: float = 0.1, quantum: int = 10, arena: bool = False) -> dict:
    """The plain path for comparison: requests run one at a time in arrival
    order on the wall clock (set-up included), through the same Server loop;
    with arena, their workspaces come from one allocation of capacity_bytes."""
    ex = SequentialExecutor(device=device, cfl=cfl,
                            arena_bytes=capacity_bytes if arena else None)
    try:
        return Server(ex, capacity_bytes, max_members=1, quantum=quantum,
                      policy="fifo").run(requests)
    finally:
        ex.close()


def main(argv=None) -> None:
    """Run the serving mix once on cuda:0 and print its metrics as JSON:
    `python -m paper_2308_06196_amd.serve --path batched|plain [--rate R]`
    (rate: Poisson arrivals per second; all requests at t = 0 without it)."""
    import argparse
    import json

    from . import workloads as wl
    ap = argparse.ArgumentParser()
    ap.add_argument("--path", choices=["batched", "plain"], default="batched")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--rate", type=float, default=None)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--pool-gb", type=float, default=200.0)
    ap.add_argument("--members", type=int, default=8)
    ap.add_argument("--large-dof", type=float, default=2.5e8)
    a = ap.parse_args(argv)
    pool = int(a.pool_gb * (1 << 30))
    reqs = make_requests(wl.serving_requests(n=a.requests, seed=a.seed, rate=a.rate,
                                             steps=a.steps))
    if a.path == "batched":
        ex = BatchExecutor(max_members=a.members, arena_bytes=pool)
        try:
            m = Server(ex, pool, max_members=a.members, quantum=4, policy="sjf",
                       large_dof=a.large_dof or None).run(reqs)
        finally:
            ex.close()
    else:
        m = run_sequential(reqs, pool, arena=True)
    print(json.dumps({"path": a.path, "rate": a.rate, **m}), flush=True)


if __name__ == "__main__":
    main()
