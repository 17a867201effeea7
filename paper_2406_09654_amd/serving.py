"""Serving form: continuous batching of world-simulation requests.

A request carries a seeded initial world (state + genome table) and a number
of steps.  The server admits queued requests while a slot of its batch table
and enough HBM (the world's ``coralai_world_bytes`` footprint) are free,
keeps every admitted world resident on the device, advances all resident
worlds together with batched steps (one captured graph over a device-side
world table, so the set can change between steps), and retires each world as
soon as its own steps are done.  Requests that arrive while others run join
the next batched step.

Each world's result does not depend on which other worlds shared its steps:
the batched kernels give every world the same per-cell arithmetic as a world
stepped alone.

Metrics: per-step latency of a world = GPU duration (HIP events on the step
stream) of each batched step it took part in; time to completion = finish -
arrival; aggregate cell-updates/s over the wall-clock span of the run.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import binding as B
from .world import Batch, World, desc_from_spec


class Admission:
    """FIFO admission by free slots and free bytes, with bounded backfill.

    The head of the queue is admitted as soon as it fits.  While it does not
    fit, later requests that do fit may pass it, at most ``max_bypass`` times
    in a row; after that nothing passes until the head is admitted, so a large
    request cannot starve behind a stream of small ones."""

    def __init__(self, budget_bytes: int, max_worlds: int, max_bypass: int = 8):
        if budget_bytes <= 0 or max_worlds <= 0:
            raise ValueError("budget and slot count must be positive")
        self.budget = int(budget_bytes)
        self.max_worlds = int(max_worlds)
        self.max_bypass = int(max_bypass)
        self.used_bytes = 0
        self.used_slots = 0
        self.bypass = 0
        self.queue: collections.deque = collections.deque()

    def push(self, key, nbytes: int) -> None:
        if nbytes > self.budget:
            raise ValueError("request %r needs %d bytes, more than the whole budget (%d)"
                             % (key, nbytes, self.budget))
        self.queue.append((key, int(nbytes)))

    def _fits(self, nbytes: int) -> bool:
        return self.used_slots < self.max_worlds and self.used_bytes + nbytes <= self.budget

    def pop_admissible(self) -> list:
        out = []
        i = 0
        while i < len(self.queue) and self.used_slots < self.max_worlds:
            if i > 0 and self.bypass >= self.max_bypass:
                break
            key, nb = self.queue[i]
            if self._fits(nb):
                del self.queue[i]
                self.used_bytes += nb
                self.used_slots += 1
                out.append(key)
                if i == 0:
                    self.bypass = 0
                else:
                    self.bypass += 1
                continue
            i += 1
        return out

    def release(self, nbytes: int) -> None:
        self.used_bytes -= int(nbytes)
        self.used_slots -= 1
        assert self.used_bytes >= 0 and self.used_slots >= 0


@dataclass
class RequestResult:
    rid: int
    arrival_s: float
    admitted_s: float = 0.0
    finished_s: float = 0.0
    n_steps: int = 0
    cells: int = 0
    step_ids: list = field(default_factory=list)
    step_ms: list = field(default_factory=list)
    state: dict | None = None

    @property
    def time_to_completion_s(self) -> float:
        return self.finished_s - self.arrival_s


@dataclass
class _Live:
    res: RequestResult
    world: World
    remaining: int


def _pct(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


class Server:
    """Continuous-batching server for worlds of one network shape and precision.

    ``hbm_budget`` bounds the summed world footprints (default: half of the
    device memory free at construction).  ``max_chunk`` bounds how many
    batched steps are queued between two admission checks."""

    def __init__(self, precision: int = 0, n_weight_layers: int = 2, hidden: int = 32,
                 max_worlds: int = 64, hbm_budget: int | None = None, max_chunk: int = 4,
                 max_bypass: int = 8, tuning: tuple[int, int, int] | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("the serving loop needs the GPU")
        self.precision = int(precision)
        self.shape = (int(n_weight_layers), int(hidden))
        self.max_worlds = int(max_worlds)
        if hbm_budget is None:
            free, _total = torch.cuda.mem_get_info()
            hbm_budget = free // 2
        self.hbm_budget = int(hbm_budget)
        self.max_chunk = max(1, int(max_chunk))
        self.max_bypass = max_bypass
        self.step_stream = torch.cuda.Stream()
        self.admit_stream = torch.cuda.Stream()
        self.batch = Batch(self.max_worlds, self.step_stream)
        self.tuning = tuning

    def footprint(self, init) -> int:
        d = desc_from_spec(init.spec)
        d.precision = self.precision
        return int(B.coralai_world_bytes(d))

    def run(self, requests, inits: dict, arrivals: str = "time", keep_states: bool = False) -> dict:
        """Serve ``requests`` (objects with rid, arrival_s, n_steps); ``inits``
        maps rid -> initial world.  arrivals="time": a request arrives when
        the wall clock since the start passes its arrival_s; "step": when the
        number of batched steps issued reaches it (deterministic, for tests)."""
        for r in requests:
            sp = inits[r.rid].spec
            if (sp.n_weight_layers, sp.hidden) != self.shape:
                raise ValueError("request %d: network shape differs from the server's" % r.rid)
            if r.n_steps < 1:
                raise ValueError("request %d: n_steps must be >= 1" % r.rid)
        adm = Admission(self.hbm_budget, self.max_worlds, self.max_bypass)
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival_s, r.rid)))
        by_id = {r.rid: r for r in requests}
        results: dict[int, RequestResult] = {}
        resident: list[_Live] = []
        events = []
        n_resident_per_step = []
        t0 = time.perf_counter()
        clock = lambda: time.perf_counter() - t0
        steps_issued = 0
        changed = False
        tuned = False

        def now_marker():
            return clock() if arrivals == "time" else float(steps_issued)

        while pending or adm.queue or resident:
            mark = now_marker()
            while pending and pending[0].arrival_s <= mark:
                r = pending.popleft()
                results[r.rid] = RequestResult(r.rid, r.arrival_s, n_steps=int(r.n_steps))
                adm.push(r.rid, self.footprint(inits[r.rid]))
            for rid in adm.pop_admissible():
                init = inits[rid]
                w = World.from_init(init, stream=self.admit_stream, precision=self.precision,
                                    sync=False)
                res = results[rid]
                res.admitted_s = clock()
                res.cells = w.N
                resident.append(_Live(res, w, int(by_id[rid].n_steps)))
                changed = True
            if not resident:
                if pending:
                    if arrivals == "time":
                        time.sleep(max(0.0, pending[0].arrival_s - clock()))
                    else:
                        steps_issued = int(np.ceil(pending[0].arrival_s))
                    continue
                if adm.queue:
                    raise RuntimeError("queued requests cannot be admitted with nothing resident")
                break
            if changed:
                self.batch.set_worlds([lv.world for lv in resident])
                if not tuned:
                    if self.tuning is not None:
                        self.batch.set_tuning(*self.tuning)
                    tuned = True
                changed = False
            n = min(self.max_chunk, min(lv.remaining for lv in resident))
            if pending and arrivals == "step":
                n = max(1, min(n, int(np.ceil(pending[0].arrival_s)) - steps_issued))
            for _ in range(n):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(self.step_stream)
                self.batch.step(1)
                e1.record(self.step_stream)
                sid = len(events)
                events.append((e0, e1))
                n_resident_per_step.append(len(resident))
                for lv in resident:
                    lv.res.step_ids.append(sid)
            steps_issued += n
            for lv in resident:
                lv.remaining -= n
            done = [lv for lv in resident if lv.remaining == 0]
            if done:
                resident = [lv for lv in resident if lv.remaining > 0]
                # leave the batch first (this waits for the queued steps)
                self.batch.set_worlds([lv.world for lv in resident])
                for lv in done:
                    if keep_states:
                        lv.res.state = lv.world.get_state_device()
                    lv.world.sync()
                    lv.res.finished_s = clock()
                    lv.world.close()
                    adm.release(lv.world.nbytes)
                    lv.world = None
        torch.cuda.synchronize()
        dur = [e0.elapsed_time(e1) for e0, e1 in events]
        lat = []
        for res in results.values():
            res.step_ms = [dur[s] for s in res.step_ids]
            lat.extend(res.step_ms)
        ttc = [res.time_to_completion_s for res in results.values()]
        updates = sum(res.cells * res.n_steps for res in results.values())
        span = (max(res.finished_s for res in results.values())
                - min(res.arrival_s for res in results.values())) if arrivals == "time" else clock()
        busy_s = sum(dur) * 1e-3
        return {
            "results": results,
            "n_requests": len(results),
            "batched_steps": len(events),
            "mean_resident": float(np.mean(n_resident_per_step)) if n_resident_per_step else 0.0,
            "step_latency_ms_p50": _pct(lat, 50),
            "step_latency_ms_p99": _pct(lat, 99),
            "time_to_completion_s_p50": _pct(ttc, 50),
            "time_to_completion_s_p99": _pct(ttc, 99),
            "cell_updates": int(updates),
            "wall_s": float(span),
            "cell_updates_per_s": updates / span if span > 0 else None,
            "gpu_busy_s": busy_s,
            "cell_updates_per_gpu_busy_s": updates / busy_s if busy_s > 0 else None,
        }

    def close(self) -> None:
        self.batch.close()
