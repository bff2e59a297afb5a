"""Continuous-batching server for scan runs of the ion step on one GPU.

A request is one independent run (its own parameters, particle count and
seed) of a fixed number of steps.  The server keeps every admitted run's
state on the device from admission to retirement and works like this:

* arrivals enter a FIFO queue at their scheduled time;
* the head of the queue is admitted as soon as a run slot is free and its
  device footprint (ecr_footprint) fits the HBM budget next to the runs
  already resident; a request that can never fit, or whose parameters the
  library rejects, is answered at once with its error;
* each slot owns a HIP stream (default priority); an admitted run is
  created and initialised on its slot's stream and then advanced one sort
  period at a time with ecr_step_graph, i.e. one graph launch per period;
* the host loop polls one event per run: a run whose period has finished
  gets its next period queued, or, when done, its tallies and density read
  back and its slot and memory released, after which the queue head may be
  admitted;
* a request may ask for a warm-up: its first `warmup` steps are run, the
  tallies read at that point, and the result reports the tallies of the
  remaining steps only (the stationary window the paper's outputs refer to);
* a request may start from a given particle state (a checkpoint, as
  ecr_set_state takes it) instead of the initial ions;
* a run whose tallies report anomalies (a non-finite particle state, or a
  per-step collision probability above the first-order limit) at any read is
  answered with an error naming them, the tallies still attached; the
  anomaly count in the result is the run's total, never a windowed
  difference, so an anomaly of the warm-up is not hidden.

Runs on different slots overlap on the device (their streams map to
separate hardware queues); a run's result depends only on its own
parameters, so it is the same alone and in any mix (tallies and state bit
for bit, density within FP64 atomic rounding).

With batch_max_n (0, off, by default), requests of at most that many
particles are not given a slot of their own: they join one of n_batches
batches, each of which shares a stream and is advanced with ecr_step_batch,
so that each step of all its runs is one kernel launch (a batch's common
sort periods replay as one captured graph).  A batch takes new members (a request joins the idle batch
with the fewest members) and retires finished ones between its launches, up
to max_batch runs; several batches keep the GPU busy while one of them turns
around on the host.  Members' results are the same as alone.  Measured on
one MI355X: a flood of 10k-100k requests is served 15-17% faster batched
(batch_max_n = 100 000), while the scan trace of 10k-2M requests, whose work
is mostly in large runs with slots of their own, is served as fast either
way, and above capacity with a lower median latency without batches (a
small request waits for a batch's launch to end before it joins).
"""
from __future__ import annotations

import collections
import dataclasses
import time

import numpy as np

from . import EcrError, Run, footprint, step_batch


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float      # seconds after the start of the serving loop
    params: dict
    steps: int
    warmup: int = 0     # leading steps left out of the reported tallies
    state: dict | None = None  # initial particle state (Run.set_state) instead of init_ions
    step0: int = 0      # step counter of that state


@dataclasses.dataclass
class Result:
    rid: int
    n: int
    arrival: float
    admitted: float = float("nan")
    finished: float = float("nan")
    nbytes: int = 0
    steps_run: int = 0
    tallies: dict | None = None
    density: dict | None = None
    error: str | None = None

    @property
    def latency(self):
        return self.finished - self.arrival


@dataclasses.dataclass
class _Active:
    req: Request
    res: Result
    run: Run
    slot: int
    done: int = 0
    event: object = None
    base: dict | None = None  # tallies at the end of the warm-up
    halt: bool = False        # retire at the next poll: the run failed


class Server:
    """Admission by HBM footprint into at most max_active slots.

    hbm_budget: device bytes the resident runs may hold together.
    period: steps per launch (None: each run's sort_every, the unit that
    ecr_step_graph replays as one graph).
    batch_max_n: requests of at most this many particles are batched (0: every
    request gets a slot of its own); max_batch runs per batch, n_batches batches.
    density_fields: density grids to read back at retirement.
    """

    def __init__(self, hbm_budget, max_active=8, period=None, density_fields=(), device="cuda", batch_max_n=0,
                 max_batch=32, n_batches=4):
        import torch
        if max_active < 1:
            raise ValueError("max_active must be >= 1")
        self.budget = int(hbm_budget)
        self.max_active = max_active
        self.period = period
        self.fields = tuple(density_fields)
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(max_active)]
        self.batch_max_n = int(batch_max_n)
        self.max_batch = int(max_batch)
        self.batch_streams = ([torch.cuda.Stream(device=self.device) for _ in range(max(1, n_batches))]
                              if self.batch_max_n > 0 else [])
        self.log = []  # (t, event, rid, active runs, resident bytes)

    def serve(self, requests, poll_s=0.0002):
        import torch
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        waiting = collections.deque()
        active = {}   # slot -> _Active
        batches = [{} for _ in self.batch_streams]  # per batch: rid -> _Active
        bevent = [None for _ in self.batch_streams]
        free = list(range(self.max_active))[::-1]
        used = 0
        results = {}
        t0 = time.monotonic()

        def now():
            return time.monotonic() - t0

        def note(ev, rid):
            self.log.append((now(), ev, rid, len(active) + sum(len(b) for b in batches), used))

        def batch_idle(g):
            return bevent[g] is None or bevent[g].query()

        def batch_for_new():
            """The idle batch with room and the fewest members, or None."""
            best = None
            for g, b in enumerate(batches):
                if len(b) < self.max_batch and batch_idle(g) and (best is None or len(b) < len(batches[best])):
                    best = g
            return best

        def reject(req, res, msg):
            res.error, res.finished = msg, now()
            results[req.rid] = res
            note("reject", req.rid)

        def release(a):
            nonlocal used
            a.res.finished = now()
            a.res.steps_run = a.done
            results[a.req.rid] = a.res
            a.run.close()
            used -= a.res.nbytes

        def checkpoint(a):
            """Warm-up read and retirement of an idle run; True when it retired."""
            if a.req.warmup > 0 and a.base is None and a.done >= a.req.warmup:
                try:
                    a.base = a.run.tallies()
                except EcrError as e:
                    a.res.error = str(e)
                    a.halt = True
                else:
                    if a.base["anomalies"] > 0:
                        a.res.error = _anomaly_error(a.run, a.base, "warm-up")
                        a.halt = True
            if a.done >= a.req.steps or a.halt:
                try:
                    t = a.run.tallies()
                    a.res.tallies = tallies_window(t, a.base) if a.base is not None else t
                    a.res.density = {f: a.run.density(f)[0] for f in self.fields}
                    if t["anomalies"] > 0 and a.res.error is None:
                        a.res.error = _anomaly_error(a.run, t, "run")
                except EcrError as e:
                    a.res.error = str(e)
                release(a)
                return True
            return False

        def next_steps(a):
            k = self.period or int(a.req.params["sort_every"])
            stop = a.req.warmup if a.base is None and a.done < a.req.warmup else a.req.steps
            return min(k, stop - a.done)

        while pending or waiting or active or any(batches):
            t = now()
            while pending and pending[0].arrival <= t:
                waiting.append(pending.popleft())
            # admission, in arrival order
            while waiting:
                req = waiting[0]
                small = bool(self.batch_streams) and int(req.params["n"]) <= self.batch_max_n
                grp = batch_for_new() if small else None
                if small and grp is None:
                    break
                if not small and not free:
                    break
                res = Result(rid=req.rid, n=int(req.params["n"]), arrival=req.arrival)
                if not 0 <= req.warmup < req.steps:
                    waiting.popleft()
                    reject(req, res, f"warmup {req.warmup} must be in [0, steps {req.steps})")
                    continue
                try:
                    nb = footprint(req.params)
                except EcrError as e:
                    waiting.popleft()
                    reject(req, res, str(e))
                    continue
                if nb > self.budget:
                    waiting.popleft()
                    reject(req, res, f"footprint {nb} B exceeds the HBM budget {self.budget} B")
                    continue
                if used + nb > self.budget:
                    break
                waiting.popleft()
                slot = -1 if small else free.pop()
                stream = self.batch_streams[grp] if small else self.streams[slot]
                try:
                    run = Run(req.params, stream=stream, device=self.device)
                    if req.state is not None:
                        run.set_state(req.state, step=req.step0)
                    else:
                        run.init_ions()
                except EcrError as e:
                    if not small:
                        free.append(slot)
                    reject(req, res, str(e))
                    continue
                used += nb
                res.admitted, res.nbytes = now(), nb
                if small:
                    batches[grp][req.rid] = _Active(req, res, run, slot)
                else:
                    active[slot] = _Active(req, res, run, slot)
                note("admit", req.rid)
            # progress of the runs with a slot of their own
            moved = False
            for slot in list(active):
                a = active[slot]
                if a.event is not None and not a.event.query():
                    continue
                moved = True
                if checkpoint(a):
                    del active[slot]
                    free.append(slot)
                    note("finish", a.req.rid)
                    continue
                n = next_steps(a)
                try:
                    a.run.step_graph(n)
                except EcrError as e:
                    a.res.error = str(e)
                    self.streams[slot].synchronize()  # nothing may still use the arena
                    release(a)
                    del active[slot]
                    free.append(slot)
                    note("evict", a.req.rid)
                    continue
                a.done += n
                a.event = torch.cuda.Event()
                a.event.record(self.streams[slot])
            # progress of each batch: all its members at once, when idle
            for g, batch in enumerate(batches):
                if not batch or not batch_idle(g):
                    continue
                moved = True
                for rid in list(batch):
                    if checkpoint(batch[rid]):
                        del batch[rid]
                        note("finish", rid)
                if not batch:
                    bevent[g] = None
                    continue
                members = list(batch.values())
                n = min(next_steps(a) for a in members)
                try:
                    step_batch([a.run for a in members], n, self.batch_streams[g])
                except EcrError as e:
                    self.batch_streams[g].synchronize()
                    batch.clear()
                    bevent[g] = None
                    for a in members:
                        a.res.error = f"batch step failed: {e}"
                        release(a)
                        note("evict", a.req.rid)
                else:
                    for a in members:
                        a.done += n
                    bevent[g] = torch.cuda.Event()
                    bevent[g].record(self.batch_streams[g])
            if not moved:
                time.sleep(poll_s)
        return [results[r.rid] for r in sorted(requests, key=lambda r: r.rid)]


def tallies_window(t, base):
    """Tallies accumulated between two reads of one run (t later than base).
    The anomaly count stays the run's total: anomalies are never windowed."""
    out = {}
    for k, v in t.items():
        out[k] = v if k == "anomalies" else v - base[k]
    return out


def _anomaly_error(run, t, where):
    from . import lib
    msg = lib().ecr_last_error(run.h)
    detail = msg.decode() if msg else ""
    return (f"ECR_ENUMERIC: {t['anomalies']} anomalies by the end of the {where} "
            f"({detail or 'non-finite state or per-step collision probability above 0.1'})")


def summary(results):
    """p50/p99 latency (s) and throughput (particle-steps/s) of served results."""
    ok = [r for r in results if r.error is None]
    lat = np.array([r.latency for r in ok])
    work = sum(r.n * r.steps_run for r in ok)
    span = max(r.finished for r in ok) - min(r.arrival for r in ok) if ok else float("nan")
    return dict(requests=len(results), completed=len(ok),
                p50_s=float(np.percentile(lat, 50)) if len(lat) else None,
                p99_s=float(np.percentile(lat, 99)) if len(lat) else None,
                throughput=work / span if ok else None, span_s=span, particle_steps=work)
