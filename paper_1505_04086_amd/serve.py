"""Request loop with continuous batching over the librsoc pool.

Colouring requests (host CSR graphs) arrive over time; a request may instead
be a recolouring after topology edits (the colouring from before the edits and
the touched vertices), which joins the pool the same way.  The server keeps an
HBM budget: a request is admitted when its CSR, colour array and pool
scratch fit; its CSR is copied to the device on a copy stream while the
compute stream keeps running pool steps, then it joins the pool, whose every
step is one fused round over all live graphs (new graphs run their first
round in the same launch in which older ones run later rounds).  Finished
graphs are copied back, their memory is released, and the request completes
with its latency (completion - arrival, host monotonic clock).

PyTorch provides device memory and streams only; all colouring work runs in
the library's kernels.  :class:`PlainServer` is the one-launch-per-request
comparator: requests are coloured one at a time in arrival order with the
single-graph entry point.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

import paper_1505_04086_amd as rsoc

torch = rsoc.torch


def csr_bytes(n: int, nnz: int, resident: bool = False, touched: int = 0) -> int:
    """Device bytes the server holds for one request: row_ptr, col_idx and
    colours, or only the colours when the CSR is already on the device (plus
    the touched list of a recolouring)."""
    if resident:
        return 4 * max(n, 1) + 4 * touched
    return 4 * (n + 1) + 4 * max(nnz, 1) + 4 * max(n, 1) + 4 * touched


def _n_touched(req) -> int:
    return 0 if req.touched is None else len(req.touched)


def _on_device(t) -> bool:
    return hasattr(t, "is_cuda") and t.is_cuda


@dataclass
class Request:
    rid: int
    row_ptr: object          # host int32 (numpy or pinned torch tensor)
    col_idx: object
    arrival: float           # monotonic seconds
    n: int = 0
    nnz: int = 0
    options: object = None
    # a recolouring after topology edits: the colouring before the edits
    # (int32[n], negative = none) and the touched vertices (int32), host or
    # device; None for a colouring request
    prev_colors: object = None
    touched: object = None
    # filled by the server
    admitted: float = 0.0
    done: float = 0.0
    colors: object = None
    k: int = -1
    stats: dict = field(default_factory=dict)

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class BudgetLedger:
    """Host-side HBM accounting for CSR + colour tensors (no device calls)."""

    def __init__(self, budget: int):
        self.budget = int(budget)
        self.used = 0

    def fits(self, nbytes: int) -> bool:
        return self.used + nbytes <= self.budget

    def take(self, nbytes: int):
        if not self.fits(nbytes):
            raise RuntimeError("budget exceeded")
        self.used += nbytes

    def give(self, nbytes: int):
        self.used -= nbytes
        assert self.used >= 0


def slot_scratch_bytes(n: int, deterministic: bool) -> int:
    """Pool scratch of one slot (worklists, hub lists, colour shadow, staging),
    as the library reserves it."""
    al = lambda x: (x + 255) // 256 * 256  # noqa: E731
    L = al(4 * (n + 1))
    return 4 * L + al(n + 64) + (L if deterministic else al(4 * (n // 8 + 2)) + al(16 * (n + 2)))


def admit_fifo(queue: collections.deque, ledger: BudgetLedger, scratch_cap: int = 1 << 62):
    """Pops requests from the head of the queue, in arrival order, while their
    device bytes fit in what the ledger has left (the first one that does not
    fit blocks the ones behind it, so no request starves).  Yields
    (request, nbytes); the caller takes the bytes before asking for the next.
    A request that could never fit (larger than the whole budget, or whose
    pool scratch exceeds scratch_cap) is yielded with nbytes = -1: reject it."""
    while queue:
        req = queue[0]
        nbytes = csr_bytes(req.n, req.nnz, _on_device(req.row_ptr), _n_touched(req))
        det = req.options is not None and req.options.mode != rsoc.RSOC_MODE_OPTIMISTIC
        if nbytes > ledger.budget or slot_scratch_bytes(req.n, det) > scratch_cap:
            queue.popleft()
            yield req, -1
            continue
        if not ledger.fits(nbytes):
            break
        queue.popleft()
        yield req, nbytes


def _colour_tensors(req, dev):
    """The request's colour tensor on the device (the previous colouring for a
    recolouring, else uninitialised) and its touched list (or None); enqueued
    on the current stream."""
    if req.prev_colors is None:
        return torch.empty(max(req.n, 1), dtype=torch.int32, device=dev), None
    col = torch.as_tensor(req.prev_colors).to(dev, non_blocking=True).to(torch.int32).clone()
    tch = None
    if _n_touched(req):
        tch = torch.as_tensor(req.touched).to(dev, non_blocking=True).to(torch.int32)
    return col, tch


class Server:
    """Continuous-batching server.

    hbm_budget: device bytes the server may hold; scratch_share of it is the
    pool's scratch arena (worklists, staging), the rest holds CSR and colours.
    """

    def __init__(self, ctx: rsoc.Context, hbm_budget: int = 16 << 30, scratch_share: float = 0.35,
                 max_slots: int = 512, options=None, device: int = 0, admit_per_poll: int = 32,
                 solo_when_idle: bool = True, solo_backlog: int = 32, idle_spin_s: float = 2e-4):
        self.ctx = ctx
        self.dev = torch.device("cuda", device)
        self.scratch_cap = int(hbm_budget * scratch_share)
        self.pool = rsoc.Pool(ctx, self.scratch_cap, max_slots)
        self.ledger = BudgetLedger(int(hbm_budget * (1 - scratch_share)))
        self.options = options if options is not None else rsoc.make_options()
        self.compute = torch.cuda.Stream(device=self.dev)
        self.copy = torch.cuda.Stream(device=self.dev)
        self.queue: collections.deque = collections.deque()   # arrived, not yet copied
        self.staging = []          # (req, tensors, event): H2D in flight
        self.live = {}             # slot -> (req, tensors)
        self.draining = []         # (req, host colours, event, nbytes): D2H in flight
        self.finished = []
        self.steps = 0
        # admissions per loop iteration: each costs host work (slot set-up
        # launches), so a burst of arrivals is admitted a few dozen at a time
        # between pool steps, which keeps the device busy with rounds meanwhile
        self.admit_per_poll = admit_per_poll
        # while the pool holds nothing and at most solo_backlog requests wait,
        # the first goes straight to the single-graph entry point (_run_alone);
        # solo counts those runs.  Measured on the served workload (p50 / p99
        # ms): at half the plain capacity plain 0.94 / 4.09, backlog 2 1.00 /
        # 5.61, 6 1.00 / 4.49, 16 0.97 / 4.12, 32 0.95 / 3.98; at the plain
        # capacity plain 8.1 / 17.8, backlog 6 2.3 / 15.4, 32 5.5 / 12.3; at
        # twice it plain 155 / 315, backlog 32 10.7 / 23.3
        self.solo_when_idle = solo_when_idle
        self.solo_backlog = solo_backlog
        self.solo = 0
        # an idle server sleeps until idle_spin_s before the next arrival and
        # polls from there on: a sleep ends tens of microseconds past its
        # deadline, which a request arriving at the deadline would wait out
        self.idle_spin_s = idle_spin_s
        self.inflight = False  # a pool round launched and not yet waited for

    # -- admission ------------------------------------------------------
    def submit(self, req: Request):
        req.n = len(req.row_ptr) - 1
        req.nnz = int(req.row_ptr[-1])
        self.queue.append(req)

    def _start_copies(self):
        if len(self.staging) >= self.admit_per_poll:
            return
        for req, nbytes in admit_fifo(self.queue, self.ledger, self.scratch_cap):
            if nbytes < 0:  # can never fit: complete it with the budget error
                req.k, req.done = rsoc.RSOC_EBUDGET, time.monotonic()
                self.finished.append(req)
                continue
            self.ledger.take(nbytes)
            if _on_device(req.row_ptr) and req.prev_colors is None:
                # CSR already resident and no colouring to copy in: the request
                # is ready at once (its colour array is only written by the
                # library's kernels)
                col = torch.empty(max(req.n, 1), dtype=torch.int32, device=self.dev)
                self.staging.append((req, (req.row_ptr, req.col_idx, col, None), None, nbytes))
                if len(self.staging) >= self.admit_per_poll:
                    break
                continue
            with torch.cuda.stream(self.copy):
                if _on_device(req.row_ptr):  # CSR already resident: nothing to copy
                    rp, ci = req.row_ptr, req.col_idx
                else:
                    rp = torch.as_tensor(req.row_ptr).to(self.dev, non_blocking=True)
                    ci = torch.as_tensor(req.col_idx if req.nnz else np.zeros(1, np.int32)).to(self.dev,
                                                                                             non_blocking=True)
                col, tch = _colour_tensors(req, self.dev)
                ev = torch.cuda.Event()
                ev.record(self.copy)
            self.staging.append((req, (rp, ci, col, tch), ev, nbytes))
            if len(self.staging) >= self.admit_per_poll:
                break

    def _run_alone(self):
        """The first waiting request, when the pool holds nothing and at most
        solo_backlog requests wait, is coloured at once with the single-graph
        entry point instead of through pool steps: the pool's per-round host
        round trips only pay off when many graphs share them, and for a few
        graphs the single-graph driver (captured rounds, one host check per
        few rounds) has the lower latency.  Requests arriving meanwhile
        wait for it, as they would in the one-call-per-request form."""
        req, tens, ev, nbytes = self.staging.pop(0)
        rp, ci, col, tch = tens
        opts = req.options or self.options
        req.admitted = time.monotonic()
        try:
            with torch.cuda.stream(self.compute):
                if req.prev_colors is not None:
                    req.k, req.stats = rsoc.rsoc_recolor_device(self.ctx, rp, ci, req.n, col, tch, opts,
                                                                stream=self.compute)
                else:
                    req.k, req.stats = rsoc.rsoc_color_device(self.ctx, rp, ci, req.n, col, opts, stream=self.compute)
        except rsoc.RsocError as e:
            req.k, req.stats = e.code, {}
        self.solo += 1
        self.live[-1 - self.solo] = (req, tens, nbytes)
        self._retire_result(-1 - self.solo, req.k, req.stats)

    def _admit_copied(self):
        if (self.solo_when_idle and not self.live and self.staging
                and len(self.staging) + len(self.queue) <= self.solo_backlog):
            ev = self.staging[0][2]
            if ev is None or ev.query():
                self._run_alone()
            # else: its copy is still in flight; the loop waits for it and the
            # next poll runs it alone
            return
        keep = []
        admitted = 0
        for req, tens, ev, nbytes in self.staging:
            if admitted >= self.admit_per_poll or (ev is not None and not ev.query()):
                keep.append((req, tens, ev, nbytes))
                continue
            rp, ci, col, tch = tens
            if req.prev_colors is not None:
                slot = self.pool.try_admit_recolor(rp, ci, req.n, col, tch, req.options or self.options)
            else:
                slot = self.pool.try_admit(rp, ci, req.n, col, req.options or self.options)
            if slot == rsoc.RSOC_EBUDGET:
                keep.append((req, tens, ev, nbytes))
                continue
            req.admitted = time.monotonic()
            self.live[slot] = (req, tens, nbytes)
            admitted += 1
        self.staging = keep

    # -- completion -----------------------------------------------------
    def _retire(self, slots):
        for slot in slots:
            try:
                k, stats = self.pool.result(slot)
            except rsoc.RsocError as e:
                k, stats = e.code, {}
            self._retire_result(slot, k, stats)

    def _retire_result(self, slot, k, stats):
        req, (rp, ci, col, tch), nbytes = self.live.pop(slot)
        req.k, req.stats = k, stats
        if _on_device(req.row_ptr):
            # resident request: the colours stay on the device (the caller
            # owns the result tensor; it stays accounted until dropped here)
            req.colors = col[:req.n]
            req.done = time.monotonic()
            self.ledger.give(nbytes)
            self.finished.append(req)
            return
        # the colours are final: the pool step that finished the slot, or the
        # single-graph call, has synchronised the compute stream
        with torch.cuda.stream(self.copy):
            host = torch.empty(max(req.n, 1), dtype=torch.int32, pin_memory=True)
            host.copy_(col, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(self.copy)
        # the device tensors stay referenced until the copy has completed
        self.draining.append((req, host, ev, nbytes, (rp, ci, col, tch)))

    def _drain(self, block=False):
        keep = []
        for item in self.draining:
            req, host, ev, nbytes, tens = item
            if block:
                ev.synchronize()
            if ev.query():
                req.colors = host.numpy()[:req.n]
                req.done = time.monotonic()
                self.ledger.give(nbytes)
                self.finished.append(req)
            else:
                keep.append(item)
        self.draining = keep

    # -- loop -----------------------------------------------------------
    def idle(self) -> bool:
        return not (self.queue or self.staging or self.live or self.draining or self.inflight)

    def poll(self):
        """One loop iteration: wait for the round launched by the previous
        one, launch the next round at once, and, while it runs, hand out the
        finished graphs, start copies and admit copied requests (they join a
        later round)."""
        fin = []
        if self.inflight:
            fin = self.pool.step_finish()
            self.inflight = False
            self.steps += 1
        if len(self.live) > len(fin):  # slots still running or in set-up
            self.pool.step_launch(stream=self.compute)
            self.inflight = True
        if fin:
            self._retire(fin)
        self._start_copies()
        self._admit_copied()
        if not self.inflight and not self.live and self.staging and self.staging[0][2] is not None:
            self.staging[0][2].synchronize()
        self._drain(block=not self.inflight and not self.live and not self.staging and not self.queue)

    def run(self, requests, clock0=None):
        """Serve `requests` (sorted by arrival, offsets in seconds from clock0)."""
        t0 = time.monotonic() if clock0 is None else clock0
        pending = collections.deque(requests)
        for r in pending:
            r.arrival = t0 + r.arrival
        while pending or not self.idle():
            now = time.monotonic()
            while pending and pending[0].arrival <= now:
                self.submit(pending.popleft())
            if self.idle() and pending:
                wait = pending[0].arrival - now
                if wait > self.idle_spin_s:
                    time.sleep(min(wait - self.idle_spin_s, 0.001))
                continue
            self.poll()
        return self.finished

    def close(self):
        self.pool.close()


class PlainServer:
    """One request at a time, in arrival order, with rsoc_color_device."""

    def __init__(self, ctx: rsoc.Context, options=None, device: int = 0):
        self.ctx = ctx
        self.dev = torch.device("cuda", device)
        self.options = options if options is not None else rsoc.make_options()
        self.stream = torch.cuda.Stream(device=self.dev)

    def run(self, requests, clock0=None):
        t0 = time.monotonic() if clock0 is None else clock0
        out = []
        for req in requests:
            req.arrival = t0 + req.arrival
            req.n = len(req.row_ptr) - 1
            req.nnz = int(req.row_ptr[-1])
            now = time.monotonic()
            if req.arrival > now:
                time.sleep(req.arrival - now)
            resident = _on_device(req.row_ptr)
            with torch.cuda.stream(self.stream):
                if resident:
                    rp, ci = req.row_ptr, req.col_idx
                else:
                    rp = torch.as_tensor(req.row_ptr).to(self.dev, non_blocking=True)
                    ci = torch.as_tensor(req.col_idx if req.nnz else np.zeros(1, np.int32)).to(self.dev,
                                                                                             non_blocking=True)
                col, tch = _colour_tensors(req, self.dev)
                req.admitted = time.monotonic()
                if req.prev_colors is not None:
                    req.k, req.stats = rsoc.rsoc_recolor_device(self.ctx, rp, ci, req.n, col, tch,
                                                                req.options or self.options, stream=self.stream)
                else:
                    req.k, req.stats = rsoc.rsoc_color_device(self.ctx, rp, ci, req.n, col,
                                                              req.options or self.options, stream=self.stream)
                req.colors = col[:req.n] if resident else col.cpu().numpy()[:req.n]
            req.done = time.monotonic()
            out.append(req)
        return out


def latency_summary(reqs):
    lat = np.array([r.latency for r in reqs])
    if len(lat) == 0:
        return {}
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "max_ms": float(lat.max() * 1e3)}
