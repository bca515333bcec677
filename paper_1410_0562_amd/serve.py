"""Serving form: many tenant indices on one GPU, with continuous batching.

Each tenant owns one incremental index (a ``BwtSet``).  Append requests
arrive over time; a tenant's appends are applied in arrival order (the order
fixes the terminator numbering, so it fixes the result), while appends of
different tenants are batched: a worker takes the queued requests of up to
``max_batch`` idle tenants that fit the device memory budget and runs them as
one ``bwt_set_append_many`` call, whose blocks hold the reads of several
tenants at once (each ranked against and merged into its own index).  A pool
of workers runs such batches side by side.  Every worker leads its batches
with a handle of its own that holds no strings, so a batch runs on that
handle's workspace and HIP stream: tenant handles hold only their index
buffers, and trimming them frees nothing a later batch has to allocate
again.  To make room,
idle tenants are first trimmed (workspace and spare buffers freed) and then
spilled: the index is exported to pinned host memory and the device copy
released; the next request of a spilled tenant restores it with
``import_bwt`` before appending.  Every step of the BWT work runs in the
library's kernels; this module only schedules.

A failed append leaves its index unchanged.  The tenant is then marked
failed, and its later requests fail too (with ``TenantFailed``) instead of
being applied without the failed one, which would renumber their strings;
``resume(tenant)`` accepts requests again.

Latency of a request = completion time - arrival time.
"""
from __future__ import annotations

import collections
import threading
import time
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import bwtset


@dataclass
class Request:
    tenant: int
    reads: object          # packed reads (numpy or device tensor)
    offsets: object        # offsets (numpy uint64 or device int64 tensor)
    bases: int
    arrival: float = 0.0
    start: float = 0.0
    finish: float = 0.0
    error: Optional[BaseException] = None
    reserved: int = 0
    done: threading.Event = field(default_factory=threading.Event)

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


class TenantFailed(RuntimeError):
    """A request not applied because an earlier request of its tenant failed."""


class _Tenant:
    def __init__(self, tid: int):
        self.tid = tid
        self.index: Optional[bwtset.BwtSet] = None
        self.spill = None            # pinned host copy of B while spilled
        self.busy = False
        self.last_used = 0.0
        self.trimmed = True
        self.failed: Optional[BaseException] = None   # first failure, until resume()


class BwtService:
    """Continuous-batching append service over `tenants` indices.

    budget_bytes: device memory the tenants' handles may hold together.
    workers: batches in flight at once.
    max_batch: tenants whose queued requests one batch may take (one request
    per tenant, the oldest, so that each tenant's order is kept).
    """

    def __init__(self, tenants: int, budget_bytes: int, workers: int = 4,
                 block_size: int = 1 << 26, per_append_bytes: Optional[int] = None,
                 max_batch: int = 8):
        import torch
        self.torch = torch
        self.tenants = [_Tenant(t) for t in range(tenants)]
        self.budget = int(budget_bytes)
        self.block_size = int(block_size)
        self.max_batch = max(1, int(max_batch))
        # device bytes an append needs beyond the resident index: the block
        # workspace (about 90 bytes per suffix of a block) plus staging; a
        # batch shares one workspace
        self.per_append = int(per_append_bytes or 96 * min(self.block_size, 1 << 26))
        # every worker leads its batches with a handle of its own that holds no
        # strings (its input is empty): the batch runs on that handle's
        # workspace, so tenant handles only ever hold their index buffers and
        # trimming them frees no workspace that the next batch must allocate
        # again; the workers' workspaces count against the budget throughout
        self._leaders = []
        for _ in range(workers):
            h = bwtset.BwtSet(block_size=self.block_size)
            h.set_param(bwtset.BWT_PARAM_BATCH_LANES, 1)
            self._leaders.append(h)
        self._empty_reads = np.zeros(1, dtype=np.uint8)
        self._empty_offs = np.zeros(1, dtype=np.uint64)
        self._free_leaders = list(self._leaders)
        # device bytes each leader holds, as of the end of its last batch
        self._leader_bytes = [h.memory() for h in self._leaders]
        self.lock = threading.Condition()
        self.queue = collections.deque()      # arrival order
        self.reserved = 0                     # bytes promised to batches in flight
        self.stats = collections.Counter()
        self.completed = []
        self._stop = False
        self._workers = [threading.Thread(target=self._worker, daemon=True, name="bwt-serve-%d" % i)
                         for i in range(workers)]
        self._device = torch.cuda.current_device()
        for w in self._workers:
            w.start()

    # ---------------------------------------------------------------- client
    def submit(self, tenant: int, reads, offsets) -> Request:
        offs = offsets
        if isinstance(offs, np.ndarray):
            bases = int(offs[-1]) - int(offs[0])
        else:
            bases = int(offs[-1].item()) - int(offs[0].item())
        req = Request(tenant, reads, offsets, bases, arrival=time.perf_counter())
        with self.lock:
            self.queue.append(req)
            self.stats["submitted"] += 1
            self.lock.notify_all()
        return req

    def drain(self, timeout: Optional[float] = None) -> None:
        """Wait until every submitted request has finished."""
        t_end = None if timeout is None else time.perf_counter() + timeout
        with self.lock:
            while self.queue or any(t.busy for t in self.tenants):
                left = None if t_end is None else t_end - time.perf_counter()
                if left is not None and left <= 0:
                    raise TimeoutError("requests still pending")
                self.lock.wait(timeout=left if left is not None else 0.5)

    def close(self) -> None:
        with self.lock:
            self._stop = True
            self.lock.notify_all()
        for w in self._workers:
            w.join(timeout=60)
        for t in self.tenants:
            if t.index is not None:
                t.index.close()
                t.index = None
        for h in self._leaders:
            h.close()
        self._leaders = []

    def export(self, tenant: int) -> bytes:
        """The tenant's BWT (waits for its pending appends)."""
        t = self.tenants[tenant]
        with self.lock:
            while t.busy or any(r.tenant == tenant for r in self.queue):
                self.lock.wait(timeout=0.5)
            if t.index is not None:
                return t.index.export()
            if t.spill is not None:
                return bytes(t.spill.numpy().tobytes())
            return b""

    def failure(self, tenant: int) -> Optional[BaseException]:
        """The error that stopped the tenant's requests, or None."""
        with self.lock:
            return self.tenants[tenant].failed

    def resume(self, tenant: int) -> None:
        """Accept the tenant's requests again after a failure; its index is
        the one left by its last successful append."""
        with self.lock:
            self.tenants[tenant].failed = None
            self.lock.notify_all()

    # ----------------------------------------------------------- scheduling
    def _resident_bytes(self) -> int:
        return (self.reserved + sum(self._leader_bytes) +
                sum(t.index.memory() for t in self.tenants
                    if t.index is not None and not t.busy))

    def _make_room(self, need: int, keep) -> bool:
        """Trim, then spill, idle tenants (least recently used first, none in
        `keep`) until `need` more bytes fit the budget.  Called with the lock
        held."""
        if self._resident_bytes() + need <= self.budget:
            return True
        idle = sorted((t for t in self.tenants
                       if t not in keep and not t.busy and t.index is not None),
                      key=lambda t: t.last_used)
        for t in idle:
            if not t.trimmed:
                t.index.trim()
                t.trimmed = True
                self.stats["trims"] += 1
                if self._resident_bytes() + need <= self.budget:
                    return True
        for t in idle:
            self._spill(t)
            if self._resident_bytes() + need <= self.budget:
                return True
        return self._resident_bytes() + need <= self.budget

    def _spill(self, t: _Tenant) -> None:
        n, _ = t.index.size()
        host = self.torch.empty(max(n, 1), dtype=self.torch.uint8, pin_memory=True)
        if n:
            t.index.export(host.numpy()[:n])
        t.spill = host[:n]
        t.index.close()
        t.index = None
        self.stats["spills"] += 1

    def _restore(self, t: _Tenant) -> None:
        """Bring a spilled (or never used) tenant's index onto the device.  The
        tenant keeps its spill copy until the import has succeeded."""
        idx = bwtset.BwtSet(block_size=self.block_size)
        try:
            if t.spill is not None and len(t.spill):
                idx.import_bwt(t.spill.numpy())
        except BaseException:
            idx.close()
            raise
        if t.spill is not None:
            self.stats["restores"] += 1
        t.index = idx
        t.spill = None
        t.trimmed = False

    def _finish(self, req: Request, err: Optional[BaseException]) -> None:
        """Record a request as done.  Called with the lock held."""
        req.error = err
        req.finish = time.perf_counter()
        self.stats["completed"] += 1
        self.completed.append(req)
        req.done.set()

    def _admit(self, lk: int) -> list:
        """The oldest queued request of each idle tenant, in arrival order, up
        to max_batch of them and as long as they fit the budget together (the
        batch shares the workspace of worker lk's leading handle, which the
        first request also reserves while that handle has not yet grown it).
        Requests of a failed tenant are failed here.  Called with the lock
        held."""
        batch = []
        keep = set()
        seen = set()
        i = 0
        while i < len(self.queue) and len(batch) < self.max_batch:
            req = self.queue[i]
            t = self.tenants[req.tenant]
            if req.tenant in seen or t.busy:
                seen.add(req.tenant)       # keep per-tenant order
                i += 1
                continue
            seen.add(req.tenant)
            if t.failed is not None:
                del self.queue[i]
                self._finish(req, TenantFailed("tenant %d: an earlier request failed: %s"
                                               % (req.tenant, t.failed)))
                self.stats["failed_after"] += 1
                continue
            grow = 2 * (req.bases + 2 * len(req.offsets))  # index growth, 3 buffers
            resident = 0 if t.index is None else t.index.memory()
            restore = 0 if t.index is not None else (
                int(len(t.spill) * 1.6) if t.spill is not None else 0)
            need = grow + restore + (
                0 if batch else max(0, self.per_append - self._leader_bytes[lk]))
            if t.index is not None and not t.trimmed:
                need = max(0, need - resident)
            fits = self._make_room(need, keep | {t})
            if not fits and not batch and not any(x.busy for x in self.tenants):
                # larger than the whole budget: run it alone rather than never
                fits = True
                self.stats["oversize"] += 1
            if not fits:
                if not batch:
                    self.stats["deferred"] += 1
                break
            del self.queue[i]
            req.reserved = need + (resident if t.index is not None else 0)
            self.reserved += req.reserved
            t.busy = True
            keep.add(t)
            batch.append(req)
        return batch

    def _run_batch(self, batch: list, leader) -> None:
        """Restore, then append every request of the batch (one call, led by
        the worker's own handle).  Outside the lock; the batch's tenants are
        marked busy."""
        ready = []
        for req in batch:
            t = self.tenants[req.tenant]
            req.start = time.perf_counter()
            if t.index is None:
                try:
                    self._restore(t)
                except BaseException as e:  # noqa: BLE001
                    req.error = e
                    continue
            ready.append(req)
        if not ready:
            return
        idx = [leader] + [self.tenants[r.tenant].index for r in ready]
        try:
            bwtset.append_many(idx, [self._empty_reads] + [r.reads for r in ready],
                               [self._empty_offs] + [r.offsets for r in ready])
        except BaseException as e:  # noqa: BLE001
            for r in ready:
                r.error = e
            return
        for r in ready:
            self.tenants[r.tenant].trimmed = False

    def _worker(self) -> None:
        torch = self.torch
        torch.cuda.set_device(self._device)
        with self.lock:
            leader = self._free_leaders.pop()
            lk = self._leaders.index(leader)
        while True:
            with self.lock:
                batch = []
                while not self._stop:
                    batch = self._admit(lk)
                    if batch:
                        break
                    self.lock.wait(timeout=0.05)
                if not batch:
                    return
                self.stats["batches"] += 1
                self.stats["batched_requests"] += len(batch)
            # outside the lock: other workers keep admitting meanwhile
            self._run_batch(batch, leader)
            leader_bytes = leader.memory()
            with self.lock:
                self._leader_bytes[lk] = leader_bytes
                for req in batch:
                    t = self.tenants[req.tenant]
                    self.reserved -= req.reserved
                    t.busy = False
                    t.last_used = time.perf_counter()
                    if req.error is not None and t.failed is None:
                        t.failed = req.error
                    self._finish(req, req.error)
                self.lock.notify_all()

    # -------------------------------------------------------------- reports
    def latency_summary(self) -> dict:
        lat = np.array([r.latency for r in self.completed if r.error is None])
        bases = sum(r.bases for r in self.completed if r.error is None)
        if len(lat) == 0:
            return {"requests": 0}
        t0 = min(r.arrival for r in self.completed)
        t1 = max(r.finish for r in self.completed)
        return {"requests": int(len(lat)), "bases": int(bases),
                "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_ms": float(lat.mean() * 1e3),
                "bases_per_s": bases / (t1 - t0) if t1 > t0 else 0.0,
                "spills": int(self.stats["spills"]), "restores": int(self.stats["restores"]),
                "trims": int(self.stats["trims"]),
                "batches": int(self.stats["batches"]),
                "mean_batch": (self.stats["batched_requests"] / self.stats["batches"]
                               if self.stats["batches"] else 0.0),
                "errors": sum(1 for r in self.completed if r.error is not None)}
