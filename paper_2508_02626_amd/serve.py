"""Serving loop: continuous batching of FMM solves on one GPU.

Requests (points, charges, requested relative error) arrive at any time.  A
dispatcher admits them in arrival order while (a) a worker slot is free and
(b) the predicted device footprint of everything in flight stays within the
HBM budget (fmm_plan_estimate plus inputs and outputs).  Each slot owns a HIP
stream (default priority) and a worker thread; when it takes a request it
also takes the other waiting small requests that fit, builds their plans on
its stream (concurrently, with fmm_plan_batch) and evaluates them together
with one fmm_evaluate_batch call (one launch per pipeline stage for all of
them).  Slots run concurrently, so
requests that arrive while others are on the GPU overlap with them.  Every
kernel is deterministic and a batched evaluation equals the single one bit
for bit, so a result does not depend on what it was served with.

Latency of a request = completion time - arrival time (host wall clock).
"""
import threading
import time
from collections import deque
from concurrent.futures import Future

import numpy as np

# requested relative error -> truncation order
ERR_TO_ORDER = {1e-4: 4, 1e-7: 8, 1e-9: 12}


# The mixed path (FP32 P2P terms, FP32 M2L at orders <= 8) deviates from the
# FP64 path by a few 1e-7 in relative L2 (measured: 2.3e-7 on 1e6 uniform
# points at p = 8), so it is chosen only for requests looser than ten times
# that; tighter requests run in FP64.
MIXED_MIN_REL_ERR = 1e-5


def precision_for(rel_err):
    return "mixed" if rel_err >= MIXED_MIN_REL_ERR else "fp64"


def order_for(rel_err):
    for e in sorted(ERR_TO_ORDER):
        if rel_err <= e:
            return ERR_TO_ORDER[e]
    return ERR_TO_ORDER[max(ERR_TO_ORDER)]


class Admission:
    """Footprint accounting (host only).  admit() either reserves the bytes of
    a request or says it must wait; requests larger than the whole budget are
    refused outright."""

    def __init__(self, budget_bytes):
        self.budget = int(budget_bytes)
        self.in_flight = 0
        self.lock = threading.Lock()

    def fits_alone(self, nbytes):
        return nbytes <= self.budget

    def try_reserve(self, nbytes):
        with self.lock:
            if self.in_flight + nbytes <= self.budget:
                self.in_flight += nbytes
                return True
            return False

    def release(self, nbytes):
        with self.lock:
            self.in_flight -= nbytes
            assert self.in_flight >= 0


class Request:
    __slots__ = ("x", "q", "rel_err", "order", "n", "nbytes", "arrival", "future", "precision",
                 "leaf_size", "done")

    def __init__(self, x, q, rel_err, precision, leaf_size):
        self.x = np.ascontiguousarray(x, dtype=np.float64)
        self.q = np.ascontiguousarray(q, dtype=np.float64)
        self.n = len(self.q)
        self.rel_err = rel_err
        self.order = order_for(rel_err)
        self.precision = precision if precision else precision_for(rel_err)
        self.leaf_size = leaf_size
        self.arrival = time.perf_counter()
        self.future = Future()
        self.nbytes = 0
        self.done = None


class Server:
    """Continuous-batching FMM server for one GPU."""

    def __init__(self, hbm_budget_bytes=32 << 30, slots=4, pack_threshold=200_000, max_pack=32,
                 leaf_size=64, precision=None, device="cuda:0", build_threads=4):
        import torch
        from . import fmm
        self.torch, self.fmm = torch, fmm
        self.device = torch.device(device)
        self.adm = Admission(hbm_budget_bytes)
        self.pack_threshold = pack_threshold
        self.max_pack = max_pack
        self.build_threads = build_threads
        self.leaf_size = leaf_size
        self.precision = precision
        self.pending = deque()
        self.cv = threading.Condition()
        self.stop = False
        self.completed = []
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self.workers = [threading.Thread(target=self._worker, args=(s,), daemon=True) for s in self.streams]
        for w in self.workers:
            w.start()

    # ---- public API ----
    def submit(self, x, q, rel_err=1e-7):
        """Queue a solve; returns a Future of (phi, field, latency_s)."""
        r = Request(x, q, rel_err, self.precision, self.leaf_size)
        r.nbytes = self.fmm.estimate(r.n, r.order, r.leaf_size) + 80 * r.n
        if not self.adm.fits_alone(r.nbytes):
            r.future.set_exception(MemoryError("request needs %d bytes, budget is %d" % (r.nbytes, self.adm.budget)))
            return r.future
        with self.cv:
            self.pending.append(r)
            self.cv.notify_all()
        return r.future

    def close(self):
        with self.cv:
            self.stop = True
            self.cv.notify_all()
        for w in self.workers:
            w.join()

    # ---- internals ----
    def _take(self):
        """Under the lock: the oldest admissible request plus waiting small
        requests that also fit (arrival order is kept: a request that does not
        fit blocks the ones behind it)."""
        if not self.pending:
            return None
        head = self.pending[0]
        if not self.adm.try_reserve(head.nbytes):
            return None
        self.pending.popleft()
        group = [head]
        if head.n <= self.pack_threshold:
            while self.pending and len(group) < self.max_pack:
                nx = self.pending[0]
                if nx.n > self.pack_threshold or not self.adm.try_reserve(nx.nbytes):
                    break
                group.append(self.pending.popleft())
        return group

    def _worker(self, stream):
        torch = self.torch
        while True:
            with self.cv:
                group = self._take()
                while group is None and not self.stop:
                    self.cv.wait(0.01)
                    group = self._take()
                if group is None:
                    return
            try:
                self._run_group(group, stream)
            except Exception as e:  # a failed solve frees its slot and memory
                for r in group:
                    if not r.future.done():
                        r.future.set_exception(e)
            finally:
                for r in group:
                    self.adm.release(r.nbytes)
                with self.cv:
                    self.cv.notify_all()

    def _run_group(self, group, stream):
        torch, fmm = self.torch, self.fmm
        with torch.cuda.stream(stream):
            xs, qs, outs = [], [], []
            for r in group:
                xs.append(torch.from_numpy(r.x).pin_memory().to(self.device, non_blocking=True))
                qs.append(torch.from_numpy(r.q).pin_memory().to(self.device, non_blocking=True))
            if len(group) == 1:
                r = group[0]
                plans = [fmm.Plan(xs[0], r.order, leaf_size=r.leaf_size, precision=r.precision, stream=stream)]
            else:
                plans = fmm.plan_batch(xs, [r.order for r in group], leaf_size=[r.leaf_size for r in group],
                                       precision=[r.precision for r in group], threads=self.build_threads,
                                       stream=stream)
            if len(group) == 1:
                outs.append(plans[0].evaluate(qs[0], stream=stream))
            else:
                outs = fmm.evaluate_batch(plans, qs, stream=stream)
            host = [(p.to("cpu", non_blocking=True), f.to("cpu", non_blocking=True)) for p, f in outs]
            stream.synchronize()
            t = time.perf_counter()
            for r, (p, f), pl in zip(group, host, plans):
                pl.close()
                r.done = t
                lat = t - r.arrival
                self.completed.append((r.n, r.order, lat))
                r.future.set_result((p.numpy(), f.numpy(), lat))


def solve_alone(x, q, rel_err=1e-7, leaf_size=64, precision=None):
    """The same solve as the server would run, on its own (for comparisons)."""
    import torch
    from . import fmm
    order = order_for(rel_err)
    prec = precision if precision else precision_for(rel_err)
    pl = fmm.Plan(torch.tensor(x, device="cuda:0"), order, leaf_size=leaf_size, precision=prec)
    phi, fld = pl.evaluate(torch.tensor(q, device="cuda:0"))
    out = (phi.cpu().numpy(), fld.cpu().numpy())
    pl.close()
    return out


def latency_stats(lat):
    a = np.sort(np.asarray(lat))
    return {"p50_ms": 1e3 * float(np.percentile(a, 50)), "p99_ms": 1e3 * float(np.percentile(a, 99)),
            "mean_ms": 1e3 * float(a.mean()), "count": int(len(a))}
