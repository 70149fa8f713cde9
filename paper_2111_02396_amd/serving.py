"""Continuous-batching request loop over the C ABI.

Requests arrive over time (each a circuit, trajectory count, seed and
request id).  A request is admitted when its device footprint, 16 * 2^n
bytes (the state plus room for a second state), fits the free budget, and
runs on one of two lanes:

* the batch lane takes every admitted request with at most 18 qubits whose
  channels are all mixtures of unitaries and packs whatever is waiting into
  one persistent launch (``qs_run_batched``); requests that arrive while a
  launch runs join the next one;
* the slot lane runs larger requests (or any other noise) with
  ``qs_run_trajectories``, each on its own stream and state, several at
  once, so their work overlaps on the device.

The lane depends only on the request, never on what else is queued, and all
randomness is counter-based per (seed, request id, trajectory), so a
request's results are the same alone and in the mix.
"""

from __future__ import annotations

import math
import threading
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import (QsError, State, load, qs_kraus_bounds, qs_run_batched, qs_run_trajectories)

BATCH_MAX_QUBITS = 18


def footprint_bytes(n: int) -> int:
    return 16 * (1 << n)


def batchable(circuit) -> bool:
    """At most 18 qubits and every channel a mixture of unitaries (each
    K_i^dag K_i a multiple of I, as qs_kraus_bounds reports): Algorithm 2
    then picks every Kraus operator from the bounds, which the persistent
    launch requires."""
    if circuit.n > BATCH_MAX_QUBITS:
        return False
    seen = {}
    for op in circuit.ops:
        if op.kind != 0:
            key = id(op.mats)
            if key not in seen:
                seen[key] = qs_kraus_bounds(op.mats)[1]
            if not seen[key]:
                return False
    return True


@dataclass
class RequestResult:
    rid: int
    lane: str
    arrival_s: float
    admitted_s: float = 0.0
    done_s: float = 0.0
    samples: Optional[np.ndarray] = None
    choices: Optional[np.ndarray] = None
    error: Optional[str] = None

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


@dataclass
class ServeStats:
    wall_s: float
    trajectories: int
    latencies_s: List[float] = field(default_factory=list)

    def percentile(self, q: float) -> float:
        return float(np.percentile(np.asarray(self.latencies_s), q)) if self.latencies_s else 0.0

    def as_dict(self) -> Dict:
        return {"wall_s": self.wall_s, "trajectories": self.trajectories,
                "trajectories_per_s": self.trajectories / self.wall_s if self.wall_s else 0.0,
                "p50_s": self.percentile(50), "p99_s": self.percentile(99),
                "requests": len(self.latencies_s)}


class Server:
    """Runs a list of workloads.configs.Request objects in (scaled) real time."""

    def __init__(self, budget_bytes: Optional[int] = None, slot_workers: int = 4,
                 max_fuse_batch: int = 3, max_fuse_slot: int = 4, max_batch: int = 512,
                 time_scale: float = 1.0):
        load()
        if budget_bytes is None:
            import torch

            free, _total = torch.cuda.mem_get_info()
            budget_bytes = int(min(free * 0.9, 288e9))
        self.budget = budget_bytes
        self.used = 0
        self.peak_used = 0  # the most footprint admitted at once
        self.slot_workers = slot_workers
        self.max_fuse_batch = max_fuse_batch
        self.max_fuse_slot = max_fuse_slot
        self.max_batch = max_batch
        self.time_scale = time_scale
        self.lock = threading.Condition()
        self.batch_q: List = []
        self.slot_q: List = []
        self.results: Dict[int, RequestResult] = {}
        self.closed = False
        self.t0 = 0.0

    # -- admission -------------------------------------------------------
    def _admit(self, req) -> bool:
        need = footprint_bytes(req.workload.circuit.n)
        if need > self.budget:
            self.results[req.rid].error = "footprint exceeds the device budget"
            self.results[req.rid].done_s = self._now()
            return True
        if self.used + need > self.budget:
            return False
        self.used += need
        self.peak_used = max(self.peak_used, self.used)
        self.results[req.rid].admitted_s = self._now()
        return True

    def _release(self, req):
        with self.lock:
            self.used -= footprint_bytes(req.workload.circuit.n)
            self.lock.notify_all()

    def _now(self) -> float:
        return time.perf_counter() - self.t0

    # -- lanes -----------------------------------------------------------
    def _batch_lane(self):
        while True:
            with self.lock:
                while not self.batch_q and not self.closed:
                    self.lock.wait()
                if not self.batch_q and self.closed:
                    return
                take = []
                rest = []
                for req in self.batch_q:
                    if len(take) < self.max_batch and self._admit(req):
                        take.append(req)
                    else:
                        rest.append(req)
                self.batch_q = rest
                if not take:
                    self.lock.wait(0.001)
                    continue
            ok = [r for r in take if self.results[r.rid].error is None]
            try:
                res, _ = qs_run_batched([r.workload for r in ok], max_fuse=self.max_fuse_batch)
                for r, out in zip(ok, res):
                    rr = self.results[r.rid]
                    rr.samples, rr.choices = out["samples"], out.get("choices")
            except QsError as e:
                for r in ok:
                    self.results[r.rid].error = str(e)
            now = self._now()
            for r in take:
                self.results[r.rid].done_s = now
                if self.results[r.rid].error is None or r in ok:
                    self._release(r)

    def _slot_lane(self):
        while True:
            with self.lock:
                req = None
                while req is None:
                    for i, cand in enumerate(self.slot_q):
                        if self._admit(cand):
                            req = self.slot_q.pop(i)
                            break
                    if req is None:
                        if self.closed and not self.slot_q:
                            return
                        self.lock.wait()
            rr = self.results[req.rid]
            if rr.error is not None:
                continue
            w = req.workload
            try:
                import torch

                stream = torch.cuda.Stream()
                with State(w.circuit.n, hip_stream=stream.cuda_stream) as st:
                    out = qs_run_trajectories(st.h, w.circuit, w.n_traj, seed=w.seed,
                                              circuit_id=w.circuit_id, n_samples=w.n_samples,
                                              p0to1=w.e0, p1to0=w.e1, max_fuse=self.max_fuse_slot)
                rr.samples, rr.choices = out["samples"], out.get("choices")
            except QsError as e:
                rr.error = str(e)
            rr.done_s = self._now()
            self._release(req)

    # -- driver ----------------------------------------------------------
    def run(self, requests) -> ServeStats:
        self.t0 = time.perf_counter()
        for r in requests:
            lane = "batch" if batchable(r.workload.circuit) else "slot"
            self.results[r.rid] = RequestResult(r.rid, lane, r.arrival_s * self.time_scale)
        workers = [threading.Thread(target=self._batch_lane, daemon=True)]
        workers += [threading.Thread(target=self._slot_lane, daemon=True)
                    for _ in range(self.slot_workers)]
        for t in workers:
            t.start()
        for r in sorted(requests, key=lambda x: x.arrival_s):
            delay = r.arrival_s * self.time_scale - self._now()
            if delay > 0:
                time.sleep(delay)
            with self.lock:
                (self.batch_q if self.results[r.rid].lane == "batch" else self.slot_q).append(r)
                self.lock.notify_all()
        with self.lock:
            self.closed = True
            self.lock.notify_all()
        for t in workers:
            t.join()
        wall = self._now()
        traj = sum(r.workload.n_traj for r in requests if self.results[r.rid].error is None)
        lat = [self.results[r.rid].latency_s for r in requests if self.results[r.rid].error is None]
        return ServeStats(wall, traj, lat)


def run_alone(req, max_fuse_batch: int = 3, max_fuse_slot: int = 4) -> RequestResult:
    """The same request through the same lane with nothing else queued."""
    srv = Server(budget_bytes=footprint_bytes(req.workload.circuit.n) * 2, slot_workers=1,
                 max_fuse_batch=max_fuse_batch, max_fuse_slot=max_fuse_slot)
    srv.run([type(req)(req.rid, 0.0, req.workload)])
    return srv.results[req.rid]
