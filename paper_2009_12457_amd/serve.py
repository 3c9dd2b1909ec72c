"""Continuous-batching triangle-count server on one GPU.

Requests (a symmetric CSR in host memory) arrive at any time.  The server
  * admits waiting requests in arrival order while their device footprint
    fits the free part of the HBM budget (a request that could never fit is
    failed with BBTC_EBUDGET instead of waiting forever);
  * partitions admitted requests on a few worker threads, each with its own
    stream (upload, degree order, cut, block index: bbtc_partition), so that
    partitions overlap each other and the counting already in flight;
  * launches everything partitioned since the last launch as ONE shared
    persistent kernel (bbtc_count_multi) on a free compute stream: requests
    that arrive while others are on the GPU join the next launch and their
    work overlaps on the device;
  * completes a request when its launch's event has fired and its results are
    on the host.

Device memory is recycled: a finished request's plan goes back to a pool and
the next admitted request re-partitions into it (best fit by held bytes), so
the steady state allocates and frees no device memory; freeing would wait for
the whole device and stall every stream.  The budget counts the bytes held by
pooled plans as well as those of requests in flight; idle plans are released
only when an admission needs their room.

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
    the uploaded input and the rank of each of its entries (16 B per edge),
    out-rows, in-rows, active columns, in-slice offsets and sources,
    block-major in-slices (24 B per edge) and the 16-bit out-rows (2 B per
    edge), per-vertex arrays, the stored block
    boundaries (at most p+1 entries per stored row; the automatic threshold
    keeps them within the 4 B per edge of the out-rows unless even rows of
    degree above 32, at most nnz/33 of them, need more), tasks and items."""
    m = nnz // 2
    ntasks = p * (p + 1) * (p + 2) // 6
    stored = min(int(n), int(nnz) // 33)
    bounds = max(4 * (p + 1) * stored, 4 * m)
    return 42 * m + 72 * n + bounds + 64 * ntasks + (1 << 20)


def default_p(n: int, nnz: int) -> int:
    """Block count for a request, by edge count: 4 below 4M edges, 8 below
    24M, else 16 (measured partition + count time over R-MAT scale 12-22 and
    Erdos-Renyi n = 1e4-1e6 graphs on MI355X; the paper's prior, p near the
    average degree, was up to 3x slower on the small and medium graphs of
    this mix)."""
    m = int(nnz) // 2
    p = 4 if m < (4 << 20) else 8 if m < (24 << 20) else 16
    return max(1, min(int(n), p))


@dataclass
class Result:
    rid: int
    total: int
    per_task: np.ndarray
    tasks: np.ndarray
    arrival: float
    done: float
    stamps: dict = field(default_factory=dict)  # admitted / partitioned / launched (perf_counter seconds)

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
    charge: int = 0  # bytes counted against the budget while in flight
    stamps: dict = field(default_factory=dict)
    plan: object = None
    event: object = None
    tasks: object = None


@dataclass
class _Batch:
    reqs: list
    stream: object
    event: object
    totals_host: object
    per_host: list = field(default_factory=list)


class PlanPool:
    """Device bytes of the server: requests in flight plus plans pooled for
    reuse, kept within a budget.  A plan object only needs `destroy()`.

    take(need) finds room for a request of at most `need` bytes: the smallest
    pooled plan that already holds `need` is reused as it is; otherwise the
    largest pooled plan is reused and may grow (its old and new buffers can
    coexist for a moment, so it is charged both), and other pooled plans are
    released, largest first, until the charge fits.  Returns (plan or None,
    charge), or None when the request has to wait for running ones."""

    def __init__(self, budget: int):
        self.budget = int(budget)
        self.idle = []  # [plan, held bytes]
        self.in_use = 0
        self.released = 0

    def take(self, need: int):
        fit = [q for q, (_, held) in enumerate(self.idle) if held >= need]
        if fit:
            q = min(fit, key=lambda q: self.idle[q][1])
            plan, held = self.idle.pop(q)
            return plan, held  # already counted
        grow = max(self.idle, key=lambda e: e[1]) if self.idle else None
        others = sorted((e for e in self.idle if e is not grow), key=lambda e: -e[1])
        for e in others:
            if self.in_use + need <= self.budget:
                break
            self._release(e)
        if self.in_use + need > self.budget and grow is not None:
            self._release(grow)
            grow = None
        if self.in_use + need > self.budget:
            return None
        self.in_use += need
        if grow is None:
            return None, need
        self.idle.remove(grow)
        return grow[0], grow[1] + need

    def settle(self, charge: int, held: int) -> int:
        """A request's plan now holds `held` bytes (was charged `charge`)."""
        self.in_use += held - charge
        return held

    def give_back(self, plan, held: int):
        self.idle.append([plan, held])  # stays counted

    def drop(self, plan, charge: int):
        if plan is not None:
            plan.destroy()
            self.released += 1
        self.in_use -= charge

    def clear(self):
        for e in list(self.idle):
            self._release(e)

    def _release(self, e):
        self.idle.remove(e)
        e[0].destroy()
        self.released += 1
        self.in_use -= e[1]


class Server:
    def __init__(self, hbm_budget_bytes: int, compute_streams: int = 2, partition_workers: int = 8, p: int = 0,
                 max_batch: int = 256, options=None):
        import torch
        self.torch = torch
        self.pool = PlanPool(hbm_budget_bytes)
        self.p = p
        self.max_batch = max_batch
        self.options = options
        self.free_streams = collections.deque(torch.cuda.Stream() for _ in range(compute_streams))
        self.waiting = collections.deque()   # submitted, not admitted
        self.admitted = collections.deque()  # admitted, waiting for a partition worker
        self.ready = []                      # partitioned, waiting for a launch
        self.inflight = []
        self.cv = threading.Condition()
        self.stop_flag = False
        self.next_id = 0
        self.launches = 0
        self.plans_created = 0
        self.thread = threading.Thread(target=self._loop, name="bbtc-server", daemon=True)
        self.workers = [threading.Thread(target=self._worker, args=(torch.cuda.Stream(),), daemon=True,
                                         name=f"bbtc-partition-{q}") for q in range(max(1, partition_workers))]
        self.busy_workers = 0
        for w in self.workers:
            w.start()
        self.thread.start()

    # ------------------------------------------------------------ client side
    def submit(self, n, rowptr, colidx, p: int | None = None) -> concurrent.futures.Future:
        fut = concurrent.futures.Future()
        with self.cv:
            rid = self.next_id
            self.next_id += 1
            pp = self.p if p is None else p
            if pp <= 0:
                pp = default_p(n, len(colidx))
            req = _Req(rid, int(n), np.ascontiguousarray(rowptr), np.ascontiguousarray(colidx, dtype=np.int32), pp,
                       time.perf_counter(), fut)
            req.need = footprint_estimate(req.n, len(req.colidx), pp)
            self.waiting.append(req)
            self.cv.notify_all()
        return fut

    @property
    def in_use(self) -> int:
        return self.pool.in_use

    @property
    def budget(self) -> int:
        return self.pool.budget

    def close(self):
        with self.cv:
            self.stop_flag = True
            self.cv.notify_all()
        self.thread.join()
        for w in self.workers:
            w.join()
        with self.cv:
            self.pool.clear()

    # ------------------------------------------------------------ scheduler
    def _options(self, p):
        opt = bbtc_options_default(p=p, mode=BBTC_MODE_PERSISTENT)
        if self.options is not None:
            for f, _ in type(opt)._fields_:
                if f not in ("p", "mode"):
                    setattr(opt, f, getattr(self.options, f))
        return opt

    def _admit_one(self):
        """Admits the head of the queue if its bytes fit (caller holds cv)."""
        if not self.waiting:
            return False
        req = self.waiting[0]
        if req.need > self.pool.budget:
            self.waiting.popleft()
            req.future.set_exception(BbtcError(BBTC_EBUDGET, f"request {req.rid} needs {req.need} B, "
                                                             f"budget {self.pool.budget} B"))
            return True
        got = self.pool.take(req.need)
        if got is None:
            return False
        req.plan, req.charge = got
        req.stamps["admitted"] = time.perf_counter()
        self.waiting.popleft()
        self.admitted.append(req)
        self.cv.notify_all()
        return True

    def _worker(self, stream):
        while True:
            with self.cv:
                while not self.admitted and not (self.stop_flag and not self.waiting):
                    self.cv.wait()
                if not self.admitted:
                    return
                req = self.admitted.popleft()
                self.busy_workers += 1
            err = None
            try:
                if req.plan is None:
                    self.plans_created += 1
                req.plan = bbtc_partition(req.n, req.rowptr, req.colidx, options=self._options(req.p),
                                          stream=stream, plan=req.plan, trusted=True)
                req.tasks = req.plan.tasks()
                held = int(req.plan.stats()["footprint"])
                req.event = self.torch.cuda.Event()
                req.event.record(stream)
                req.stamps["partitioned"] = time.perf_counter()
            except Exception as e:  # invalid input etc.: fail this request only
                err = e
            with self.cv:
                self.busy_workers -= 1
                if err is None:
                    req.charge = self.pool.settle(req.charge, held)
                    self.ready.append(req)
                else:
                    self.pool.drop(req.plan, req.charge)
                    req.future.set_exception(err)
                self.cv.notify_all()

    def _launch(self):
        torch = self.torch
        with self.cv:
            if not self.ready or not self.free_streams:
                return False
            reqs, self.ready = self.ready[:self.max_batch], self.ready[self.max_batch:]
            stream = self.free_streams.popleft()
        now = time.perf_counter()
        for r in reqs:  # plans were built on the workers' streams
            stream.wait_event(r.event)
            r.stamps["launched"] = now
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
                finished = []
                for q, r in enumerate(b.reqs):
                    per = b.per_host[q].numpy().view(np.uint64)[:r.plan.ntasks].copy()
                    finished.append((r, Result(r.rid, int(tot[q]), per, r.tasks, r.arrival, now, r.stamps)))
                with self.cv:
                    for r, _ in finished:
                        self.pool.give_back(r.plan, r.charge)
                        r.plan = None
                    self.free_streams.append(b.stream)
                    self.cv.notify_all()
                for r, res in finished:
                    r.future.set_result(res)
                done_any = True
            else:
                still.append(b)
        self.inflight = still
        return done_any

    def _loop(self):
        while True:
            progressed = self._complete()
            with self.cv:
                while self._admit_one():
                    progressed = True
            if self._launch():
                progressed = True
            with self.cv:
                if (self.stop_flag and not self.waiting and not self.admitted and not self.ready
                        and not self.inflight and self.busy_workers == 0):
                    self.cv.notify_all()
                    return
                if not progressed:
                    self.cv.wait(timeout=0.0002)


def serve_plain(requests, p_of=None):
    """First-come first-served, one request at a time, one launch per task.
    `requests` = list of (arrival_offset_s, n, rowptr, colidx); returns Results
    with latencies measured against the same arrival schedule.  One plan is
    re-partitioned for every request, so no device memory is allocated or
    freed in the steady state here either."""
    import torch
    results = []
    plan = None
    t0 = time.perf_counter()
    try:
        for rid, (off, n, rp, ci) in enumerate(requests):
            arrival = t0 + off
            now = time.perf_counter()
            if now < arrival:
                time.sleep(arrival - now)
            p = p_of(n, len(ci)) if p_of else default_p(n, len(ci))
            plan = bbtc_partition(n, rp, ci, options=bbtc_options_default(p=p, mode=BBTC_MODE_PLAIN_INTERSECT),
                                  plan=plan, trusted=True)
            per, tot = bbtc_count(plan)
            torch.cuda.synchronize()
            res = Result(rid, int(tot.item()), per.cpu().numpy().view(np.uint64)[:plan.ntasks].copy(),
                         plan.tasks(), arrival, time.perf_counter())
            results.append(res)
    finally:
        if plan is not None:
            plan.destroy()
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
    return [f.result() for f in futs]


def latency_summary(results, warmup: int = 0):
    lat = np.array([r.latency for r in results[warmup:]]) * 1e3
    if len(lat) == 0:
        return {}
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "requests": int(len(lat))}


def stage_summary(results, warmup: int = 0):
    """Mean time (ms) a served request spends waiting for admission, being
    partitioned, waiting for its launch, and on the GPU until its results are
    on the host."""
    keys = ("admitted", "partitioned", "launched")
    rs = [r for r in results[warmup:] if all(k in r.stamps for k in keys)]
    if not rs:
        return {}
    def mean(f):
        return float(np.mean([f(r) for r in rs]) * 1e3)
    return {"admission_wait_ms": mean(lambda r: r.stamps["admitted"] - r.arrival),
            "partition_ms": mean(lambda r: r.stamps["partitioned"] - r.stamps["admitted"]),
            "launch_wait_ms": mean(lambda r: r.stamps["launched"] - r.stamps["partitioned"]),
            "count_ms": mean(lambda r: r.done - r.stamps["launched"])}
