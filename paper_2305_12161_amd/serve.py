"""Continuous-batching service for quench requests.

A request asks for the quench of one lattice (L, seed) up to t_max sweeps; it
is answered with its bond-count trace (every `every` sweeps) and its final
bond count.  Requests arrive over time; the server admits them into device
slots as memory and slots allow, advances every admitted lattice together in
chunks of `chunk` sweeps, and retires finished ones at chunk boundaries, so
new work joins while earlier work is still on the GPU.

Backends:
  * GpuBackend -- the HIP library: lattice sizes the batched engine takes
    (L % 64 == 0, L <= 256) live in fixed batch slots advanced by one graph
    replay per chunk; other sizes run as single lattices (the 1-bit layout when
    L % 64 == 0, else int8) spread over a few streams, each quenched to its
    t_max in one enqueue as soon as it is admitted.  Completions are noticed
    through events: nothing waits for the whole device.
  * Any object with the lock-step methods (tests use a CPU one).

Results never depend on what else is running: every lattice follows exactly
its own (L, seed) trajectory.
"""
import collections
import concurrent.futures
import threading
import time
from dataclasses import dataclass
from typing import Dict, List, Optional

import numpy as np


class StepError(RuntimeError):
    """A backend's work for one request failed; the server answers that
    request as failed and goes on with the others."""

    def __init__(self, idx: int, message: str):
        super().__init__(message)
        self.idx = idx


@dataclass
class Result:
    idx: int
    L: int
    seed: int
    t_max: int
    arrival_s: float
    admitted_s: float = 0.0
    done_s: float = 0.0
    trace: Optional[np.ndarray] = None   # B(0), B(every), ..., B(t_max - every)
    final_B: int = -1
    status: str = "ok"                   # "ok", "cancelled" or "failed"
    error: Optional[str] = None          # the failure's message

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


class GpuBackend:
    """Device slots for served quenches.

    budget_bytes caps the device memory of lattice state held at once.  The
    batch slots are pre-allocated: `batch_slots` maps L -> number of slots.
    Single lattices are allocated per request from the remaining budget.
    """

    def __init__(self, budget_bytes: int, batch_slots: Dict[int, int], every: int, chunk: int,
                 t_max_cap: int = 10_000, device=None, graph_sweeps: Optional[int] = None,
                 single_streams: int = 8, single_pass: int = 2):
        import torch
        from . import binding
        if every <= 0 or chunk <= 0 or chunk % every:
            raise ValueError("chunk must be a positive multiple of every")
        self.qz = binding
        self.torch = torch
        self.every, self.chunk = every, chunk
        self.device = torch.device("cuda") if device is None else torch.device(device)
        # the batch's own stream (default priority): synchronising it never
        # waits for the single lattices' streams
        self.stream = torch.cuda.Stream(device=self.device)
        # single lattices are spread over a few streams (default priority) so
        # that the short sweeps of mid-size lattices overlap on the GPU
        self.single_streams = [torch.cuda.Stream(device=self.device) for _ in range(single_streams)]
        self._next_stream = 0
        # one host thread per stream enqueues the single lattices' runs: a run
        # is thousands of launches, and the library call releases the
        # interpreter lock, so the streams are fed in parallel while the
        # serving loop goes on
        self._feeders = [concurrent.futures.ThreadPoolExecutor(max_workers=1)
                         for _ in self.single_streams]
        # sweeps per pass of the single bit lattices (two halves the launches
        # per chunk; the trajectories are the same)
        self.single_pass = single_pass
        specs = []
        for L in sorted(batch_slots):
            for _ in range(batch_slots[L]):
                specs.append((L, 0))
        self.batch = None
        self.batch_bytes = 0
        self.free_batch: Dict[int, List[int]] = collections.defaultdict(list)
        if specs:
            cap = t_max_cap // every + 2
            self.batch_bytes = binding.batch_state_bytes(specs, cap)
            # the autotuner's stored launch shape with one graph per chunk, or,
            # for sizes never tuned, the library's own autotune at creation
            import json
            from . import tune
            gs = chunk if graph_sweeps is None else graph_sweeps
            tuning = tune.batch_tuning_json(sorted(batch_slots))
            if tuning is not None:
                tuning = dict(json.loads(tuning), graph_sweeps=gs)
            self.batch = binding.Batch(specs, trace_every=every, trace_cap=cap, device=self.device,
                                       stream=self.stream, tuning=tuning)
            if tuning is None:
                self.batch.set_tuning(min(batch_slots), 0, gs)
            for slot, (L, _) in enumerate(specs):
                self.batch.set_active(slot, False)
                self.free_batch[L].append(slot)
        self._tuned: Dict[int, Optional[tuple]] = {}   # side -> stored two-sweep tile
        self.single_budget = budget_bytes - self.batch_bytes
        if self.single_budget < 0:
            raise ValueError("batch slots exceed the memory budget")
        self.single_used = 0
        self.live: Dict[int, dict] = {}          # request idx -> placement
        self._batch_event = None                 # completion of the batch's chunk in flight
        # cancelled or failed single lattices whose queued work has not
        # drained yet: their memory stays booked until it has
        self._zombies: List[dict] = []
        self._failed: Dict[int, str] = {}

    @staticmethod
    def layout_for(L: int) -> str:
        return "bit" if L % 64 == 0 else "i8"

    def single_bytes(self, L: int) -> int:
        return self.qz.state_bytes(L, self.layout_for(L)) + 8 * (10_000 // self.every + 2)

    def can_admit(self, L: int) -> bool:
        if self.batch is not None and self.free_batch.get(L):
            return True
        if self.batch is not None and L in self.free_batch and not self.free_batch[L]:
            return False            # a batch size with all slots busy waits for a slot
        return self.single_used + self.single_bytes(L) <= self.single_budget

    def admit(self, req) -> None:
        if req.t_max % self.chunk:
            raise ValueError("t_max must be a multiple of the chunk")
        if self.batch is not None and self.free_batch.get(req.L):
            slot = self.free_batch[req.L].pop()
            # the slot stops by itself at t_max, on the device
            self.batch.replace(slot, req.L, req.seed, req.t_max)
            self.live[req.idx] = {"kind": "batch", "slot": slot, "t": 0, "t_max": req.t_max}
            return
        wi = self._next_stream % len(self.single_streams) if self.single_streams else -1
        st = self.single_streams[wi] if self.single_streams else self.stream
        self._next_stream += 1
        # the memory is booked here; the lattice itself is made by whoever
        # enqueues its work (a feeder thread in the asynchronous protocol),
        # since its first kernel may have to wait for room in a busy queue
        self.single_used += self.single_bytes(req.L)
        self.live[req.idx] = {"kind": "single", "L": req.L, "seed": req.seed, "t": 0,
                              "t_max": req.t_max, "bytes": self.single_bytes(req.L),
                              "stream": st, "feeder": wi}

    def _materialize(self, p) -> None:
        """Device state of a single lattice: the lattice and its trace buffer
        (the trace, then the three final bond counts; the library zeroes each
        part on the lattice's stream before writing it), both from the pool of
        the lattice's stream."""
        if "lat" in p:
            return
        with self.torch.cuda.device(self.device), self.torch.cuda.stream(p["stream"]):
            p["trace"] = self.torch.empty(p["t_max"] // self.every + 3, dtype=self.torch.int64,
                                          device=self.device)
            lat = self.qz.Lattice(p["L"], p["seed"], self.layout_for(p["L"]), device=self.device,
                                  stream=p["stream"])
        if self.layout_for(p["L"]) == "bit" and self.single_pass:
            lat.set_pass(self.single_pass)
            # the autotuner's stored tile for this side, if it has one
            if p["L"] not in self._tuned:
                from . import tune
                self._tuned[p["L"]] = tune.best_pass2(p["L"])
            stored = self._tuned[p["L"]]
            if stored is not None and self.single_pass == 2:
                lat.set_pass(2, *stored)
        p["lat"] = lat

    def advance(self) -> None:
        """One chunk of sweeps for every live lattice (asynchronous); the
        lock-step protocol, kept for callers that step the backend by hand."""
        if self.batch is not None and any(p["kind"] == "batch" for p in self.live.values()):
            self.batch.run(self.chunk)
        for p in self.live.values():
            if p["kind"] == "single" and p["t"] < p["t_max"]:
                self._materialize(p)
                t = p["t"]
                sl = p["trace"][t // self.every: (t + self.chunk) // self.every]
                p["lat"].run_device(self.chunk, self.every, sl)
        for p in self.live.values():
            p["t"] = min(p["t"] + self.chunk, p["t_max"])

    def sync(self) -> None:
        self.torch.cuda.synchronize(self.device)

    def finished(self) -> List[int]:
        return [i for i, p in self.live.items() if p["t"] >= p["t_max"]]

    # ---- the asynchronous protocol: no device-wide synchronisation --------
    # A single lattice gets its whole run enqueued on its own stream at
    # admission, followed by an event; the batch advances one chunk (one
    # graph replay) at a time, followed by an event.  poll() reports the
    # requests whose work has completed, kick() starts the batch's next chunk.
    def start(self, idx: int) -> None:
        p = self.live[idx]
        if p["kind"] != "single":
            return
        torch, device = self.torch, self.device

        n = p["t_max"] // self.every

        def feed():
            # the lattice, its whole quench, the final bond counts and the
            # download of both into pinned memory, then the event: retiring the
            # request reads host memory only, and never waits for later work
            # that other lattices have queued on the same stream
            self._materialize(p)
            with torch.cuda.device(device):
                p["lat"].run_device(p["t_max"], self.every, p["trace"][:n])
                p["lat"].bonds_device(p["trace"][n:])
                host = torch.empty(n + 3, dtype=torch.int64, pin_memory=True)
                with torch.cuda.stream(p["stream"]):
                    host.copy_(p["trace"], non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(p["stream"])
            p["host"] = host
            return ev

        if p["feeder"] >= 0:
            p["future"] = self._feeders[p["feeder"]].submit(feed)
        else:
            p["event"] = feed()

    def poll(self) -> List[int]:
        self._reap()
        out = []
        for i, p in list(self.live.items()):
            if p["kind"] != "single":
                continue
            fut = p.get("future")
            if fut is not None and fut.done():
                p["future"] = None
                try:
                    p["event"] = fut.result()
                except Exception as e:            # the feeder's library call failed
                    self._failed[i] = f"{type(e).__name__}: {e}"
                    self.discard(i)
                    continue
            if p.get("event") is not None and p["event"].query():
                p["t"] = p["t_max"]
                out.append(i)
        if self._batch_event is not None and self._batch_event.query():
            self._batch_event = None
            for i, p in self.live.items():
                if p["kind"] == "batch" and p["t"] < p["t_max"] and p.get("running"):
                    p["t"] = min(p["t"] + self.chunk, p["t_max"])
                    p["running"] = False
                    if p["t"] >= p["t_max"]:
                        out.append(i)
        return out

    def kick(self) -> None:
        if self.batch is None or self._batch_event is not None:
            return
        todo = [p for p in self.live.values() if p["kind"] == "batch" and p["t"] < p["t_max"]]
        if not todo:
            return
        self.batch.run(self.chunk)
        for p in todo:
            p["running"] = True
        ev = self.torch.cuda.Event()
        ev.record(self.stream)
        self._batch_event = ev

    def busy(self) -> bool:
        return bool(self.live)

    # ---- cancellation and failures ---------------------------------------
    def cancel(self, idx: int) -> None:
        """Stop serving request idx and free its slot.  A batch slot stops at
        once (the device skips inactive slots; a chunk in flight ends first,
        stream-ordered before any reuse).  A single lattice's work is already
        queued on its stream and cannot be taken back: its memory is released
        once that work has drained."""
        p = self.live.pop(idx, None)
        if p is None:
            return
        if p["kind"] == "batch":
            self.batch.set_active(p["slot"], False)
            self.free_batch[self.batch.specs[p["slot"]][0]].append(p["slot"])
            return
        self._zombies.append(p)
        self._reap()

    discard = cancel

    def failures(self) -> Dict[int, str]:
        """Requests whose work failed since the last call (idx -> message);
        their resources are already released or queued for release."""
        out, self._failed = self._failed, {}
        return out

    def _reap(self) -> None:
        keep = []
        for p in self._zombies:
            fut = p.get("future")
            if fut is not None:
                if not fut.done():
                    keep.append(p)
                    continue
                try:
                    p["event"] = fut.result()
                except Exception:
                    p["event"] = None
                p["future"] = None
            ev = p.get("event")
            if ev is not None and not ev.query():
                keep.append(p)
                continue
            if p.get("lat") is not None:
                p["lat"].close()
            self.single_used -= p["bytes"]
        self._zombies = keep

    def retire(self, idx: int) -> dict:
        p = self.live.pop(idx)
        n = p["t_max"] // self.every
        if p.get("host") is not None:
            # filled on the lattice's stream before the event that finished
            # it: no device call here
            out = p["host"].numpy()
            p["lat"].close()
            self.single_used -= p["bytes"]
            return {"trace": out[:n].astype(np.int64), "final_B": int(out[n:n + 3].sum())}
        if p["kind"] == "batch":
            slot = p["slot"]
            trace = self.batch.trace(slot, 0, n).astype(np.int64)
            final_B = int(self.batch.bonds(slot).sum())
            self.batch.set_active(slot, False)
            L = self.batch.specs[slot][0]
            self.free_batch[L].append(slot)
        else:
            # an asynchronous copy into pinned memory on the lattice's own
            # stream, whose work is complete: a plain copy to pageable memory
            # would wait for every stream on the device
            host = self.torch.empty(n, dtype=p["trace"].dtype, pin_memory=True)
            with self.torch.cuda.stream(p["stream"]):
                host.copy_(p["trace"][:n], non_blocking=True)
            p["stream"].synchronize()
            trace = host.numpy().astype(np.int64)
            final_B = int(p["lat"].bonds().sum())
            p["lat"].close()
            self.single_used -= p["bytes"]
        return {"trace": trace, "final_B": final_B}

class Server:
    """Event loop: admit arrivals as room frees up, keep the device busy,
    retire finished requests.

    With a backend that offers poll()/kick()/start() (the GPU backend) the
    loop never waits for the whole device: single lattices run their whole
    quench on their own streams as soon as they are admitted, the batch runs
    chunk after chunk, and each completion (an event) is noticed and answered
    on its own.  Other backends (a CPU one in the tests) are stepped in lock
    step, one chunk for every live lattice per round."""

    def __init__(self, backend, chunk: int):
        self.backend = backend
        self.chunk = chunk
        self._cancel_lock = threading.Lock()
        self._cancels: List[int] = []

    def cancel(self, idx: int) -> None:
        """Ask for request idx to be cancelled (from any thread, or from the
        serve loop's callbacks).  It is dropped if it has not been admitted,
        else stopped and its slot freed; a request already answered is left
        as it is."""
        with self._cancel_lock:
            self._cancels.append(idx)

    def _take_cancels(self) -> List[int]:
        with self._cancel_lock:
            out, self._cancels = self._cancels, []
        return out

    def serve(self, requests, clock=time.perf_counter, time_scale: float = 1.0,
              progress=None, tick=None) -> List[Result]:
        """Serve `requests` (objects with idx, L, seed, t_max, arrival_s), arrivals
        replayed in real time (arrival_s * time_scale after the start).
        progress(done, total, seconds) is called after each answer (finished,
        cancelled or failed); tick(server, round) once per round of the loop.
        A backend step that fails for one request (StepError, or an entry in
        the backend's failures()) answers that request as failed; the others
        go on."""
        be = self.backend
        asynchronous = all(hasattr(be, k) for k in ("poll", "kick", "start"))
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival_s))
        waiting: collections.deque = collections.deque()
        results: Dict[int, Result] = {}
        live: set = set()
        t_start = clock()
        done = 0
        total = len(pending)

        def answered(res):
            nonlocal done
            res.done_s = clock() - t_start
            done += 1
            if progress is not None:
                progress(done, total, res.done_s)

        def finish(idx):
            if idx not in live:
                return
            live.discard(idx)
            out = be.retire(idx)
            res = results[idx]
            res.trace = out["trace"]
            res.final_B = out["final_B"]
            answered(res)

        def fail(idx, message):
            if idx not in live:
                return
            live.discard(idx)
            if hasattr(be, "discard"):
                be.discard(idx)
            res = results[idx]
            res.status, res.error = "failed", message
            answered(res)

        def collect_failures():
            if hasattr(be, "failures"):
                for idx, message in be.failures().items():
                    fail(idx, message)

        def guarded(step):
            try:
                return step()
            except StepError as e:
                fail(e.idx, str(e))
                return None

        def cancel_requested():
            for idx in self._take_cancels():
                res = results.get(idx)
                if res is not None and (res.status != "ok" or res.trace is not None):
                    continue                          # already answered
                if idx in live:
                    live.discard(idx)
                    be.cancel(idx)
                else:
                    r = next((x for x in waiting if x.idx == idx), None)
                    if r is not None:
                        waiting.remove(r)
                    else:
                        r = next((x for x in pending if x.idx == idx), None)
                        if r is None:
                            continue                  # unknown request
                        pending.remove(r)
                        res = results[idx] = Result(r.idx, r.L, r.seed, r.t_max,
                                                    r.arrival_s * time_scale)
                res = results[idx]
                res.status = "cancelled"
                answered(res)

        rounds = 0
        while done < total:
            if tick is not None:
                tick(self, rounds)
            rounds += 1
            now = clock() - t_start
            while pending and pending[0].arrival_s * time_scale <= now:
                r = pending.popleft()
                waiting.append(r)
                results[r.idx] = Result(r.idx, r.L, r.seed, r.t_max, r.arrival_s * time_scale)
            cancel_requested()
            if done >= total:
                break
            if asynchronous:
                for idx in guarded(be.poll) or []:
                    finish(idx)
                collect_failures()
            # admit in arrival order, skipping requests whose size has no room yet
            still = collections.deque()
            while waiting:
                r = waiting.popleft()
                if be.can_admit(r.L):
                    be.admit(r)
                    live.add(r.idx)
                    results[r.idx].admitted_s = clock() - t_start
                    if asynchronous:
                        guarded(lambda: be.start(r.idx))
                else:
                    still.append(r)
            waiting = still
            if not live:
                if pending:
                    # idle until the next arrival
                    wait = pending[0].arrival_s * time_scale - (clock() - t_start)
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
                continue
            if asynchronous:
                guarded(be.kick)
                collect_failures()
                time.sleep(0.0002)        # the device is busy; look again shortly
                continue
            guarded(be.advance)
            be.sync()
            collect_failures()
            for idx in be.finished():
                finish(idx)
        return [results[k] for k in sorted(results)]


def summarize(results: List[Result], wall_s: float) -> dict:
    """Latency and throughput over the requests answered with a result;
    cancelled and failed ones are counted apart."""
    ok = [r for r in results if r.status == "ok"]
    lat = np.array([r.latency_s for r in ok]) if ok else np.zeros(1)
    attempts = float(sum(r.L ** 3 * r.t_max for r in ok))
    return {
        "requests": len(results),
        "cancelled": sum(r.status == "cancelled" for r in results),
        "failed": sum(r.status == "failed" for r in results),
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "attempts_per_ns": attempts / (wall_s * 1e9),
        "wall_s": wall_s,
    }
