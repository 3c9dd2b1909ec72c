"""Continuous-batching triangle-count server on one GPU.

Requests (a symmetric CSR in host memory) arrive at any time.  A scheduler
thread
  * admits waiting requests in arrival order while their estimated device
    footprint fits the free part of the HBM budget (a request that could never
    fit is failed with BBTC_EBUDGET instead of waiting forever);
  * partitions each admitted request on its own stream (upload, degree order,
    cut, block index: bbtc_partition), which overlaps with counting already in
    flight on the other streams;
  * launches everything partitioned since the last launch as ONE shared
    persistent kernel (bbtc_count_multi) on a free compute stream, so requests
    that arrive while others are on the GPU join the next launch and their
    work overlaps on the device;
  * completes a request when its launch's event has fired and its results
    are on the host, then frees its plan and budget.

Latency = time the result is on the host - arrival time.  The plain baseline
(`serve_plain`) runs the same requests first-come first-served, one at a
time, with one kernel launch per task.
"""
from __future__ import annotations

import collections
import concurrent.futures
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import (BBTC_EBUDGET, BBTC_MODE_PERSISTENT, BBTC_MODE_PLAIN_INTERSECT, BbtcError, bbtc_count,
               bbtc_count_multi, bbtc_options_default, bbtc_partition)


def footprint_estimate(n: int, nnz: int, p: int) -> int:
    """Upper bound of a plan's device bytes (the layout of bbtc_partition):
    out/in rows and active columns 12 B per edge, per-vertex arrays, the two
    block row indices (at most p+1 entries per vertex each), tasks and items."""
    m = nnz // 2
    ntasks = p * (p + 1) * (p + 2) // 6
    return 12 * m + 4 * nnz + 64 * n + 8 * (p + 1) * n + 64 * ntasks + (1 << 20)


@dataclass
class Result:
    rid: int
    total: int
    per_task: np.ndarray
    tasks: np.ndarray
    arrival: float
    done: float

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class _Req:
    rid: int
    n: int
    rowptr: np.ndarray
    colidx: np.ndarray
    p: int
    arrival: float
    future: concurrent.futures.Future
    need: int = 0
    plan: object = None
    per_task: object = None
    tasks: object = None


@dataclass
class _Batch:
    reqs: list
    stream: object
    event: object
    totals_host: object
    per_host: list = field(default_factory=list)


class Server:
    def __init__(self, hbm_budget_bytes: int, compute_streams: int = 2, p: int = 0, max_batch: int = 256,
                 options=None):
        import torch
        self.torch = torch
        self.budget = int(hbm_budget_bytes)
        self.p = p
        self.max_batch = max_batch
        self.options = options
        self.part_stream = torch.cuda.Stream()
        self.free_streams = collections.deque(torch.cuda.Stream() for _ in range(compute_streams))
        self.waiting = collections.deque()
        self.ready = []
        self.inflight = []
        self.in_use = 0
        self.cv = threading.Condition()
        self.stop_flag = False
        self.next_id = 0
        self.launches = 0
        self.thread = threading.Thread(target=self._loop, name="bbtc-server", daemon=True)
        self.thread.start()

    # ------------------------------------------------------------ client side
    def submit(self, n, rowptr, colidx, p: int | None = None) -> concurrent.futures.Future:
        fut = concurrent.futures.Future()
        with self.cv:
            rid = self.next_id
            self.next_id += 1
            pp = self.p if p is None else p
            if pp <= 0:
                pp = max(1, min(int(n), int(round(len(colidx) / max(int(n), 1)))))
            req = _Req(rid, int(n), np.ascontiguousarray(rowptr), np.ascontiguousarray(colidx, dtype=np.int32), pp,
                       time.perf_counter(), fut)
            req.need = footprint_estimate(req.n, len(req.colidx), pp)
            self.waiting.append(req)
            self.cv.notify()
        return fut

    def close(self):
        with self.cv:
            self.stop_flag = True
            self.cv.notify()
        self.thread.join()

    # ------------------------------------------------------------ scheduler
    def _admit_one(self):
        with self.cv:
            if not self.waiting:
                return False
            req = self.waiting[0]
            if req.need > self.budget:
                self.waiting.popleft()
                req.future.set_exception(BbtcError(BBTC_EBUDGET, f"request {req.rid} needs {req.need} B, "
                                                                 f"budget {self.budget} B"))
                return True
            if self.in_use + req.need > self.budget:
                return False
            self.waiting.popleft()
            self.in_use += req.need
        opt = bbtc_options_default(p=req.p, mode=BBTC_MODE_PERSISTENT)
        if self.options is not None:
            for f, _ in type(opt)._fields_:
                if f not in ("p", "mode"):
                    setattr(opt, f, getattr(self.options, f))
        try:
            req.plan = bbtc_partition(req.n, req.rowptr, req.colidx, options=opt, stream=self.part_stream,
                                      trusted=True)
            req.tasks = req.plan.tasks()
            self.ready.append(req)
        except Exception as e:  # invalid input etc.: fail this request only
            with self.cv:
                self.in_use -= req.need
            req.future.set_exception(e)
        return True

    def _launch(self):
        torch = self.torch
        if not self.ready or not self.free_streams:
            return False
        reqs, self.ready = self.ready[:self.max_batch], self.ready[self.max_batch:]
        stream = self.free_streams.popleft()
        # the plans were built on part_stream: make the compute stream wait for it
        stream.wait_stream(self.part_stream)
        with torch.cuda.stream(stream):
            pers = [torch.empty(max(r.plan.ntasks, 1), dtype=torch.int64, device="cuda") for r in reqs]
            totals = torch.empty(len(reqs), dtype=torch.int64, device="cuda")
            bbtc_count_multi([r.plan for r in reqs], pers, totals, stream=stream)
            totals_host = torch.empty(len(reqs), dtype=torch.int64, pin_memory=True)
            totals_host.copy_(totals, non_blocking=True)
            per_host = []
            for t in pers:
                h = torch.empty(t.shape, dtype=torch.int64, pin_memory=True)
                h.copy_(t, non_blocking=True)
                per_host.append(h)
            ev = torch.cuda.Event()
            ev.record(stream)
        self.inflight.append(_Batch(reqs, stream, ev, totals_host, per_host))
        self.launches += 1
        return True

    def _complete(self):
        done_any = False
        still = []
        for b in self.inflight:
            if b.event.query():
                now = time.perf_counter()
                tot = b.totals_host.numpy()
                for q, r in enumerate(b.reqs):
                    per = b.per_host[q].numpy().view(np.uint64)[:r.plan.ntasks].copy()
                    res = Result(r.rid, int(tot[q]), per, r.tasks, r.arrival, now)
                    r.plan.destroy()
                    r.plan = None
                    with self.cv:
                        self.in_use -= r.need
                    r.future.set_result(res)
                self.free_streams.append(b.stream)
                done_any = True
            else:
                still.append(b)
        self.inflight = still
        return done_any

    def _loop(self):
        while True:
            progressed = self._complete()
            while self._admit_one():
                progressed = True
                self._complete()  # keep completions flowing while partitioning
            if self._launch():
                progressed = True
            with self.cv:
                if self.stop_flag and not self.waiting and not self.ready and not self.inflight:
                    return
                if not progressed:
                    self.cv.wait(timeout=0.0002)


def serve_plain(requests, p_of=None):
    """First-come first-served, one request at a time, one launch per task.
    `requests` = list of (arrival_offset_s, n, rowptr, colidx); returns Results
    with latencies measured against the same arrival schedule."""
    import torch
    results = []
    t0 = time.perf_counter()
    for rid, (off, n, rp, ci) in enumerate(requests):
        arrival = t0 + off
        now = time.perf_counter()
        if now < arrival:
            time.sleep(arrival - now)
        p = p_of(n, len(ci)) if p_of else max(1, min(n, int(round(len(ci) / max(n, 1)))))
        plan = bbtc_partition(n, rp, ci, options=bbtc_options_default(p=p, mode=BBTC_MODE_PLAIN_INTERSECT),
                              trusted=True)
        per, tot = bbtc_count(plan)
        torch.cuda.synchronize()
        res = Result(rid, int(tot.item()), per.cpu().numpy().view(np.uint64)[:plan.ntasks].copy(), plan.tasks(),
                     arrival, time.perf_counter())
        plan.destroy()
        results.append(res)
    return results


def run_trace(server: Server, requests):
    """Submits (arrival_offset_s, n, rowptr, colidx) requests at their arrival
    times (open loop) and returns the Results in request order."""
    futs = []
    t0 = time.perf_counter()
    for off, n, rp, ci in requests:
        now = time.perf_counter()
        if now < t0 + off:
            time.sleep(t0 + off - now)
        futs.append(server.submit(n, rp, ci))
    out = []
    for f in futs:
        out.append(f.result())
    return out


def latency_summary(results, warmup: int = 0):
    lat = np.array([r.latency for r in results[warmup:]]) * 1e3
    if len(lat) == 0:
        return {}
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "requests": int(len(lat))}
