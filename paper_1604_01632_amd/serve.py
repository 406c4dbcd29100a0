"""Served form: continuous batching of FSLBM simulations on one GPU.

Requests arrive over time, each with a scene and a horizon of steps.  The
server admits the oldest waiting request as soon as its device workspace
(``fslbm_workspace_bytes``) fits into the HBM budget and a slot is free,
keeps every admitted lattice resident on the device, and advances all
admitted domains together as one batch (one graph launch per step) in
quanta of steps.  A domain that reaches its horizon is read out (bubble
table and scalars) and released, and its memory goes to the next request;
requests arriving while others run join at the next quantum boundary, so
their work overlaps on the device.  Scenes are built, and domains uploaded
on a side stream, by host threads while the device runs; the batch is
kept for the whole run and its members are replaced in place.

The plain baseline (``run_fifo``) serves the same arrival trace one domain
at a time, first come first served, with the same kernels.

Scheduling only: every step runs in the library's HIP kernels through the
C ABI (``fslbm_batch_step`` / ``fslbm_step``).
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import time
from dataclasses import dataclass, field

import numpy as np

from . import Batch, Domain, fslbm_batch_workspace_bytes, fslbm_workspace_bytes, PRECISIONS


@dataclass
class Request:
    """One simulation: `build()` returns its scene (a ``scenes.Scene``);
    `arrival` is seconds after the start of the trace."""
    id: int
    arrival: float
    horizon: int
    build: object
    meta: dict = field(default_factory=dict)


@dataclass
class Result:
    id: int
    arrival: float
    admitted: float
    done: float
    cells: int
    steps: int
    bubbles: dict
    scalars: dict
    error: str = ""  # set when the request was rejected (never admitted)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def _finish(slot, t_done) -> Result:
    """Read out a domain whose steps the device has finished (the caller
    synchronises before taking t_done)."""
    dom = slot["dom"]
    b = dom.bubbles()
    s = dom.read(())["scalars"]
    return Result(slot["req"].id, slot["req"].arrival, slot["admitted"], t_done, dom.N,
                  slot["req"].horizon, b, s)


def summary(results, wall: float) -> dict:
    rejected = sum(1 for r in results if r.error)
    results = [r for r in results if not r.error]
    lat = np.array([r.latency for r in results])
    updates = float(sum(r.cells * r.steps for r in results))
    span = max(r.done for r in results) - min(r.arrival for r in results)
    return dict(requests=len(results), rejected=rejected, p50_s=float(np.percentile(lat, 50)),
                p99_s=float(np.percentile(lat, 99)), mean_s=float(lat.mean()),
                mlups=updates / span / 1e6, span_s=span, wall_s=wall)


class Server:
    """Continuous-batching request loop.

    budget_bytes: device memory the admitted workspaces and the batch
    tables may use (default: 80 % of the free device memory at start); a
    request that could never fit is rejected (a Result with `error` set)
    and the others keep running; max_active: slots; quantum: steps between
    scheduling decisions (a domain never runs past its horizon: a quantum
    ends at the next horizon).

    One batch lives for the whole run: admissions and completions replace
    its members in place (``fslbm_batch_reset``), with no new batch, graph
    or stream.  A request's scene is built on a host thread as soon as it
    arrives; once admitted (memory reserved), its domain is created and
    uploaded on a side stream by another host thread while the batch keeps
    stepping, and it joins the batch at the next quantum boundary after its
    upload finished.
    """

    def __init__(self, precision="fp32", budget_bytes=None, max_active=64, quantum=100,
                 build_threads=4, overrides=None):
        import torch

        self.precision = precision
        if budget_bytes is None:
            free, _ = torch.cuda.mem_get_info()
            budget_bytes = int(0.8 * free)
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.quantum = int(quantum)
        self.build_threads = int(build_threads)
        self.overrides = dict(overrides or {})

    def _need(self, sc) -> int:
        p = sc.params(precision=PRECISIONS[self.precision], **self.overrides)
        return fslbm_workspace_bytes(p)

    def run(self, requests, clock=time.perf_counter, log=None) -> list:
        import threading

        import torch

        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting = collections.deque()   # arrived: (request, future scene)
        creating = []                   # admitted: slots whose domain is being uploaded
        active, results = [], []
        tables = fslbm_batch_workspace_bytes(self.max_active)
        used = tables
        batch = None
        pool = cf.ThreadPoolExecutor(max_workers=self.build_threads)
        uploader = cf.ThreadPoolExecutor(max_workers=1)
        side = {}
        lock = threading.Lock()

        def create(sc):
            # one side stream per upload thread, default priority
            tid = threading.get_ident()
            with lock:
                if tid not in side:
                    side[tid] = torch.cuda.Stream()
                st = side[tid]
            with torch.cuda.stream(st):
                return Domain.from_scene(sc, self.precision, stream=st, **self.overrides)

        t0 = clock()
        try:
            while pending or waiting or creating or active:
                now = clock() - t0
                while pending and pending[0].arrival <= now:
                    r = pending.popleft()
                    waiting.append((r, pool.submit(r.build)))
                # admission by memory and slots, oldest first
                while waiting and len(active) + len(creating) < self.max_active:
                    r, fut = waiting[0]
                    if not fut.done() and (active or creating):
                        break  # keep the device busy while the scene is built
                    sc = fut.result()
                    need = self._need(sc)
                    if need == 0 or need + tables > self.budget:
                        waiting.popleft()
                        t = clock() - t0
                        why = ("invalid parameters" if need == 0 else
                               f"needs {need} B of device memory, budget {self.budget} B")
                        results.append(Result(r.id, r.arrival, t, t, sc.n, 0, {}, {},
                                              error=f"rejected: {why}"))
                        if log:
                            log(f"[serve] request {r.id} rejected: {why}")
                        continue
                    if used + need > self.budget:
                        break
                    waiting.popleft()
                    used += need
                    creating.append(dict(req=r, fut=uploader.submit(create, sc), need=need,
                                         admitted=clock() - t0, left=r.horizon))
                # uploads that finished join the batch
                joined = [s for s in creating if s["fut"].done()]
                if not active and not joined and creating:
                    creating[0]["fut"].result()  # nothing to step: wait for the next upload
                    joined = [s for s in creating if s["fut"].done()]
                for s in joined:
                    s["dom"] = s.pop("fut").result()
                    creating.remove(s)
                    active.append(s)
                if not active:
                    if waiting:
                        waiting[0][1].result()
                    elif pending:
                        time.sleep(max(0.0, pending[0].arrival - (clock() - t0)))
                    continue
                doms = [s["dom"] for s in active]
                if batch is None:
                    batch = Batch(doms, tuning_cache_path="", capacity=self.max_active)
                elif joined or batch.domains != doms:
                    batch.reset(doms)
                q = min(self.quantum, min(s["left"] for s in active))
                batch.step(q)
                for s in active:
                    s["left"] -= q
                done = [s for s in active if s["left"] == 0]
                for s in done:
                    s["dom"].sync()  # its last quantum has finished on the device
                    res = _finish(s, clock() - t0)
                    results.append(res)
                    if log:
                        log(f"[serve] request {res.id} done: latency {res.latency:.2f} s, "
                            f"{res.cells} cells x {res.steps} steps")
                active = [s for s in active if s["left"] > 0]
                if done:
                    # the batch no longer holds the finished domains before
                    # their memory goes back
                    if active:
                        batch.reset([s["dom"] for s in active])
                    for s in done:
                        s["dom"].close()
                        used -= s["need"]
                if not done:
                    active[0]["dom"].sync()  # bound the queue ahead of the clock
        finally:
            if batch is not None:
                batch.close()
            for s in creating:
                try:
                    s["fut"].result().close()
                except Exception:
                    pass
            pool.shutdown(wait=True)
            uploader.shutdown(wait=True)
        return results


def run_fifo(requests, precision="fp32", clock=time.perf_counter, overrides=None, log=None) -> list:
    """Plain baseline: one domain at a time in arrival order, each stepped
    to its horizon alone (scenes built on a host thread ahead of time)."""
    reqs = sorted(requests, key=lambda r: r.arrival)
    overrides = dict(overrides or {})
    results = []
    pool = cf.ThreadPoolExecutor(max_workers=2)
    futs = collections.deque()
    k = 0
    t0 = clock()
    try:
        for r in reqs:
            while k < len(reqs) and (len(futs) < 2 or reqs[k].arrival <= clock() - t0):
                futs.append(pool.submit(reqs[k].build))
                k += 1
            now = clock() - t0
            if r.arrival > now:
                time.sleep(r.arrival - now)
            sc = futs.popleft().result()
            dom = Domain.from_scene(sc, precision, **overrides)
            admitted = clock() - t0
            left = r.horizon
            while left > 0:
                q = min(500, left)
                dom.step(q)
                dom.sync()
                left -= q
            dom.sync()
            res = _finish(dict(req=r, dom=dom, admitted=admitted), clock() - t0)
            results.append(res)
            dom.close()
            if log:
                log(f"[fifo] request {res.id} done: latency {res.latency:.2f} s")
    finally:
        pool.shutdown(wait=True)
    return results
