"""The continuous-batching scheduler.

CPU: the scheduler against a backend built on the oracle (admission by slots
and memory, arrivals while others run, every result equal to its run alone).
GPU: a small served stream on the HIP backend, each result equal to the same
request run alone through the single-lattice path.
"""
import collections
import os

import numpy as np
import pytest

from paper_2305_12161_amd import serve, workloads as wl


class OracleBackend:
    """CPU stand-in with the GPU backend's interface; at most `slots` live lattices."""

    def __init__(self, orc, slots, every, chunk):
        self.orc, self.slots, self.every, self.chunk = orc, slots, every, chunk
        self.live = {}
        self.max_live = 0
        self.admit_order = []

    def can_admit(self, L):
        return len(self.live) < self.slots

    def admit(self, req):
        s = self.orc.init(req.L, req.seed)
        self.live[req.idx] = {"s": s, "seed": req.seed, "t": 0, "t_max": req.t_max, "trace": []}
        self.max_live = max(self.max_live, len(self.live))
        self.admit_order.append(req.idx)

    def advance(self):
        for p in self.live.values():
            tr = self.orc.run(p["s"], p["seed"], p["t"], self.chunk, self.every)
            p["trace"].extend(int(v) for v in tr)
            p["t"] += self.chunk

    def sync(self):
        pass

    def finished(self):
        return [i for i, p in self.live.items() if p["t"] >= p["t_max"]]

    def retire(self, idx):
        p = self.live.pop(idx)
        return {"trace": np.array(p["trace"], dtype=np.int64),
                "final_B": int(self.orc.bonds(p["s"]).sum())}

    def cancel(self, idx):
        self.live.pop(idx, None)

    discard = cancel


class FailingOracleBackend(OracleBackend):
    """Injects a failing step: the chunk that would take request `victim`
    past t = `at` raises, naming that request, before any lattice of the
    round is touched; the round is then retried without it."""

    def __init__(self, orc, slots, every, chunk, victim, at):
        super().__init__(orc, slots, every, chunk)
        self.victim, self.at = victim, at

    def advance(self):
        p = self.live.get(self.victim)
        if p is not None and p["t"] + self.chunk > self.at:
            raise serve.StepError(self.victim, "injected failure in a sweep chunk")
        super().advance()


def test_scheduler_with_oracle_backend(orc):
    reqs = wl.request_stream(n=24, rate_per_s=400.0, master_seed=9, sizes=(4, 6, 8),
                             t_maxes=(20, 40))
    be = OracleBackend(orc, slots=5, every=5, chunk=10)
    srv = serve.Server(be, chunk=10)
    res = srv.serve(reqs)
    assert len(res) == len(reqs)
    assert be.max_live <= 5
    assert be.admit_order == sorted(be.admit_order)       # one size class here: FIFO
    for r in res:
        s = orc.init(r.L, r.seed)
        want = orc.run(s, r.seed, 0, r.t_max, 5)
        assert np.array_equal(r.trace, want)
        assert r.final_B == int(orc.bonds(s).sum())
        assert r.done_s >= r.admitted_s >= r.arrival_s - 1e-9
    stats = serve.summarize(res, wall_s=1.0)
    assert stats["requests"] == len(reqs) and stats["p99_latency_s"] >= stats["p50_latency_s"]


class AsyncOracleBackend(OracleBackend):
    """The asynchronous protocol on the CPU: start() queues a request's whole
    quench, kick() runs at most one queued quench, poll() reports finished
    ones once -- so requests finish out of step with each other."""

    def __init__(self, orc, slots, every):
        super().__init__(orc, slots, every, chunk=None)
        self.queue = collections.deque()
        self.done = []

    def start(self, idx):
        self.queue.append(idx)

    def kick(self):
        if self.queue:
            idx = self.queue.popleft()
            p = self.live[idx]
            tr = self.orc.run(p["s"], p["seed"], 0, p["t_max"], self.every)
            p["trace"] = [int(v) for v in tr]
            p["t"] = p["t_max"]
            self.done.append(idx)

    def poll(self):
        out, self.done = self.done, []
        return out

    def cancel(self, idx):
        self.live.pop(idx, None)
        if idx in self.queue:
            self.queue.remove(idx)

    discard = cancel


def test_scheduler_asynchronous_protocol(orc):
    reqs = wl.request_stream(n=20, rate_per_s=300.0, master_seed=11, sizes=(4, 6, 8),
                             t_maxes=(10, 30))
    be = AsyncOracleBackend(orc, slots=4, every=5)
    res = serve.Server(be, chunk=10).serve(reqs)
    assert len(res) == len(reqs) and be.max_live <= 4
    for r in res:
        s = orc.init(r.L, r.seed)
        assert np.array_equal(r.trace, orc.run(s, r.seed, 0, r.t_max, 5))
        assert r.final_B == int(orc.bonds(s).sum())
        assert r.done_s >= r.admitted_s >= r.arrival_s - 1e-9


def _check_alone(orc, r, every):
    s = orc.init(r.L, r.seed)
    assert np.array_equal(r.trace, orc.run(s, r.seed, 0, r.t_max, every)), r.idx
    assert r.final_B == int(orc.bonds(s).sum())


def test_cancel_mid_flight_frees_the_slot(orc):
    """One slot: request 0 (long) is cancelled after two chunks; request 1,
    queued behind it, is admitted into the freed slot at once, and every
    other result is the request's run alone.  A cancel of a request still
    waiting drops it; a cancel of an answered request changes nothing."""
    reqs = [wl.Request(0, 6, 200, 101, 0.0), wl.Request(1, 4, 20, 102, 0.0),
            wl.Request(2, 8, 20, 103, 0.0), wl.Request(3, 4, 20, 104, 0.0)]
    be = OracleBackend(orc, slots=1, every=5, chunk=10)
    srv = serve.Server(be, chunk=10)
    seen = {}

    def tick(server, rnd):
        seen[rnd] = {i: p["t"] for i, p in be.live.items()}
        if rnd == 2:
            assert seen[rnd] == {0: 20}           # request 0 mid-flight
            server.cancel(0)
            server.cancel(2)                      # still waiting
        if rnd == 6:
            server.cancel(1)                      # already answered
    res = srv.serve(reqs, tick=tick)
    assert [r.status for r in res] == ["cancelled", "ok", "cancelled", "ok"]
    assert res[0].trace is None and res[2].admitted_s == 0.0
    assert be.admit_order == [0, 1, 3]
    assert seen[3] == {1: 10}                    # admitted and stepped in the round of the cancel
    for r in (res[1], res[3]):
        _check_alone(orc, r, 5)
    st = serve.summarize(res, wall_s=1.0)
    assert st["cancelled"] == 2 and st["failed"] == 0


def test_failing_step_answers_that_request_only(orc):
    reqs = wl.request_stream(n=16, rate_per_s=500.0, master_seed=13, sizes=(4, 6, 8),
                             t_maxes=(20, 40))
    victim = reqs[3].idx
    be = FailingOracleBackend(orc, slots=3, every=5, chunk=10, victim=victim, at=10)
    res = serve.Server(be, chunk=10).serve(reqs)
    assert len(res) == len(reqs) and be.max_live <= 3
    assert be.admit_order == sorted(be.admit_order)
    for r in res:
        if r.idx == victim:
            assert r.status == "failed" and "injected" in r.error and r.trace is None
        else:
            assert r.status == "ok"
            _check_alone(orc, r, 5)
    assert serve.summarize(res, wall_s=1.0)["failed"] == 1


class FailingAsyncBackend(AsyncOracleBackend):
    """The asynchronous protocol with a failing quench, reported through
    failures() as the GPU backend reports a failed library call."""

    def __init__(self, orc, slots, every, victim):
        super().__init__(orc, slots, every)
        self.victim = victim
        self.failed = {}

    def kick(self):
        if self.queue and self.queue[0] == self.victim:
            self.queue.popleft()
            self.failed[self.victim] = "QuenchError: injected device failure"
            return
        super().kick()

    def failures(self):
        out, self.failed = self.failed, {}
        return out


def test_asynchronous_failure_and_cancel(orc):
    reqs = wl.request_stream(n=12, rate_per_s=500.0, master_seed=17, sizes=(4, 6),
                             t_maxes=(10, 30))
    victim, cancelled = reqs[2].idx, reqs[5].idx
    be = FailingAsyncBackend(orc, slots=2, every=5, victim=victim)

    def tick(server, rnd):
        if cancelled in be.live and cancelled in be.queue:
            server.cancel(cancelled)              # admitted, its quench not yet run
    res = serve.Server(be, chunk=10).serve(reqs, tick=tick)
    assert len(res) == len(reqs) and be.max_live <= 2
    for r in res:
        if r.idx == victim:
            assert r.status == "failed" and "injected" in r.error
        elif r.idx == cancelled:
            assert r.status == "cancelled" and r.trace is None
        else:
            assert r.status == "ok"
            _check_alone(orc, r, 5)


def test_request_stream_is_seeded():
    a = wl.request_stream(n=50, rate_per_s=10.0)
    b = wl.request_stream(n=50, rate_per_s=10.0)
    assert [(r.L, r.t_max, r.seed, r.arrival_s) for r in a] == \
           [(r.L, r.t_max, r.seed, r.arrival_s) for r in b]
    assert all(r.L in wl.SERVE_SIZES and r.t_max in wl.SERVE_TMAX for r in a)
    assert all(y.arrival_s >= x.arrival_s for x, y in zip(a, a[1:]))
    assert a[0].arrival_s == 0.0


@pytest.mark.gpu
def test_served_results_equal_alone():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_12161_amd import binding
    reqs = wl.request_stream(n=30, rate_per_s=200.0, master_seed=7,
                             sizes=(64, 96, 128, 192, 256, 384), t_maxes=(100, 300))
    every, chunk = 50, 50
    be = serve.GpuBackend(budget_bytes=256 << 20, batch_slots={64: 4, 128: 3, 192: 2, 256: 2},
                          every=every, chunk=chunk, t_max_cap=300)
    srv = serve.Server(be, chunk=chunk)
    res = srv.serve(reqs)
    assert len(res) == len(reqs)
    for r in res:
        print("served", r.idx, r.L, r.t_max, flush=True)
        layout = "bit" if r.L % 64 == 0 else "i8"
        lat = binding.Lattice(r.L, r.seed, layout)
        tr = lat.run(r.t_max, every).astype(np.int64)
        assert np.array_equal(r.trace, tr), (r.idx, r.L)
        assert r.final_B == int(lat.bonds().sum())


@pytest.mark.gpu
def test_served_cancel_mid_flight_gpu():
    """Cancel one batch-slot request and one single-lattice request while they
    run: the batch slot goes back to the free list at once, the single
    lattice's memory comes back once its queued work has drained, and every
    other result equals its run alone."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_12161_amd import binding
    reqs = wl.request_stream(n=24, rate_per_s=200.0, master_seed=23, sizes=(64, 96, 128, 384),
                             t_maxes=(200, 400))
    every, chunk = 50, 50
    be = serve.GpuBackend(budget_bytes=256 << 20, batch_slots={64: 2, 128: 2}, every=every,
                          chunk=chunk, t_max_cap=400)
    cancelled = {}

    def tick(server, rnd):
        for kind in ("batch", "single"):
            if kind in cancelled:
                continue
            for i, p in be.live.items():
                if p["kind"] == kind and (kind == "single" or p["t"] > 0):
                    cancelled[kind] = i
                    server.cancel(i)
                    break
    res = serve.Server(be, chunk=chunk).serve(reqs, tick=tick)
    assert len(res) == len(reqs) and set(cancelled) == {"batch", "single"}
    for r in res:
        print("served", r.idx, r.L, r.t_max, r.status, flush=True)
        if r.idx in cancelled.values():
            assert r.status == "cancelled" and r.trace is None
            continue
        assert r.status == "ok"
        layout = "bit" if r.L % 64 == 0 else "i8"
        lat = binding.Lattice(r.L, r.seed, layout)
        assert np.array_equal(r.trace, lat.run(r.t_max, every).astype(np.int64)), (r.idx, r.L)
        assert r.final_B == int(lat.bonds().sum())
    torch.cuda.synchronize()
    be.poll()
    assert be.single_used == 0 and not be.live
    assert sorted(len(v) for v in be.free_batch.values()) == [2, 2]


@pytest.mark.gpu
def test_served_stream_prefix(orc):
    """The first 120 requests of the served stream (L uniform in {64, 96, 128,
    192, 256, 384, 512}, t_max in {1e3, 1e4}, seeds 0x50000000 + idx), all
    queued at once on the configured memory budget and batch slots: every
    result equals the request run alone, and 20 of those with L <= 128 equal
    the oracle."""
    import os
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_12161_amd import binding
    orc.set_threads(min(16, os.cpu_count() or 1))
    reqs = wl.request_stream(n=2000, rate_per_s=wl.SERVE_RATE_PER_S)[:120]
    every, chunk = 100, 100
    be = serve.GpuBackend(budget_bytes=wl.SERVE_BUDGET_BYTES, batch_slots=wl.SERVE_BATCH_SLOTS,
                          every=every, chunk=chunk)
    res = serve.Server(be, chunk=chunk).serve(reqs, time_scale=0.0)
    assert [r.idx for r in res] == [q.idx for q in reqs]
    small = []
    for r in res:
        layout = "bit" if r.L % 64 == 0 else "i8"
        lat = binding.Lattice(r.L, r.seed, layout)
        tr = lat.run(r.t_max, every).astype(np.int64)
        assert np.array_equal(r.trace, tr), (r.idx, r.L)
        assert r.final_B == int(lat.bonds().sum()), r.idx
        if r.L <= 128 and len(small) < 20:
            small.append(r)
        del lat
    print("served prefix: oracle on", len(small), "requests", flush=True)
    for r in small:
        s = orc.init(r.L, r.seed)
        want = orc.run(s, r.seed, 0, r.t_max, every)
        assert np.array_equal(r.trace, want), (r.idx, r.L)
        assert r.final_B == int(orc.bonds(s).sum()), r.idx
