"""Continuous-batching merge server for one GPU.

Clients submit merge requests (two sorted device arrays, optionally with
payloads); each returns a concurrent.futures.Future.  One scheduler thread:

- admits pending requests in arrival order while their HBM footprint fits
  the remaining budget and a slot is free (a request larger than the whole
  budget is refused with BudgetError; a cancelled request is dropped);
- launches the admitted requests as one batch (one cm_stable_merge_batch
  call: every merge cut into equal blocks, all blocks in one kernel) as soon
  as fewer than `max_inflight` batches are on the GPU, so requests that
  arrive while a batch runs go into the next one and the two overlap on the
  device (the executor alternates streams);
- completes a batch when its event has fired: results go to the futures,
  the budget is released, latency (arrival to completion seen) is recorded.

The executor is pluggable: GpuExecutor runs batches through the library;
tests drive the same scheduler with a CPU executor.  An executor that
raises in launch() or reports a failed batch makes every future of that
batch fail and releases its budget.
"""
from __future__ import annotations

import collections
import concurrent.futures
import ctypes
import threading
import time
from dataclasses import dataclass, field
from typing import Any, Callable, Optional


class BudgetError(RuntimeError):
    """The request can never fit the server's HBM budget."""


@dataclass
class MergeRequest:
    rid: int
    A: Any
    B: Any
    A_val: Any
    B_val: Any
    nbytes: int
    outputs: int
    arrival: float
    ready: Any = None  # executor token: the inputs are ready (e.g. a GPU event)
    future: concurrent.futures.Future = field(default_factory=concurrent.futures.Future)
    launched: float = 0.0
    done: float = 0.0


class Budget:
    """Bytes of HBM the server may hold for admitted requests."""

    def __init__(self, total: int):
        if total <= 0:
            raise ValueError("budget must be positive")
        self.total = total
        self.used = 0
        self.peak = 0

    def try_reserve(self, n: int) -> bool:
        if self.used + n > self.total:
            return False
        self.used += n
        self.peak = max(self.peak, self.used)
        return True

    def release(self, n: int):
        if n > self.used:
            raise RuntimeError("budget released more than reserved")
        self.used -= n


class GpuExecutor:
    """Runs a batch with one cm_stable_merge_batch call; completion is a HIP
    event query.  Streams alternate so consecutive batches can overlap.
    Each batch's outputs are views into one key slab and one payload slab
    (two allocations per batch), and its descriptors are filled with
    vectorised numpy, so the host cost per request stays small."""

    def __init__(self, device="cuda:0", num_streams: int = 2):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(num_streams)]
        self._next = 0

    def footprint(self, A, B, A_val, B_val) -> int:
        """Inputs plus outputs of one request, in bytes (after checking it once)."""
        torch = self.torch
        for t in (A, B) + ((A_val, B_val) if A_val is not None else ()):
            if not isinstance(t, torch.Tensor) or t.device != self.device or t.dim() != 1 \
                    or not t.is_contiguous():
                raise ValueError("request arrays must be contiguous 1-D tensors on the "
                                 "server's device")
        if B.dtype != A.dtype or A.dtype not in (torch.uint32, torch.uint64, torch.float32):
            raise TypeError("keys must be uint32, uint64 or float32, the same for A and B")
        if (A_val is None) != (B_val is None):
            raise ValueError("give payloads for both inputs or neither")
        if A_val is not None and (A_val.dtype != torch.uint32 or B_val.dtype != torch.uint32
                                  or A_val.numel() != A.numel() or B_val.numel() != B.numel()):
            raise ValueError("payloads must be uint32 and as long as their keys")
        n = A.numel() + B.numel()
        per = A.element_size() + (4 if A_val is not None else 0)
        return 2 * n * per

    def ready_token(self):
        """Event on the submitting thread's current stream: the request's
        inputs are ready once it has fired (called in submit)."""
        ev = self.torch.cuda.Event()
        ev.record(self.torch.cuda.current_stream(self.device))
        return ev

    def launch(self, batch):
        import numpy as np
        from . import batch_descriptors, launch_batch
        torch = self.torch
        s = self.streams[self._next]
        self._next = (self._next + 1) % len(self.streams)
        groups = {}
        for i, r in enumerate(batch):  # one launch per (key dtype, payload mode)
            groups.setdefault((r.A.dtype, r.A_val is not None), []).append(i)
        outs = [None] * len(batch)
        keep = []
        with torch.cuda.stream(s):
            for r in batch:  # inputs were produced on the submitters' streams
                if r.ready is not None:
                    s.wait_event(r.ready)
            for (dtype, with_val), idx in groups.items():
                reqs = [batch[i] for i in idx]
                m = np.array([r.A.numel() for r in reqs], dtype=np.uint64)
                n = np.array([r.B.numel() for r in reqs], dtype=np.uint64)
                N = m + n
                # each request's outputs start 16-byte aligned (4 elements), so the
                # kernel can use 16-byte accesses when the inputs are aligned too
                padded = (N + np.uint64(3)) // np.uint64(4) * np.uint64(4)
                off = np.concatenate([[0], np.cumsum(padded)]).astype(np.uint64)
                keys = torch.empty(int(off[-1]), dtype=dtype, device=self.device)
                vals = torch.empty(int(off[-1]), dtype=torch.uint32, device=self.device) \
                    if with_val else None
                ks = keys.element_size()
                d = batch_descriptors(len(reqs))
                d["A"] = [r.A.data_ptr() for r in reqs]
                d["B"] = [r.B.data_ptr() for r in reqs]
                d["m"], d["n"] = m, n
                d["C"] = np.where(N > 0, keys.data_ptr() + off[:-1] * ks, 0)
                if with_val:
                    d["A_val"] = [r.A_val.data_ptr() for r in reqs]
                    d["B_val"] = [r.B_val.data_ptr() for r in reqs]
                    d["C_val"] = np.where(N > 0, vals.data_ptr() + off[:-1] * 4, 0)
                keep.append(launch_batch(dtype, with_val, d, self.device, s))
                for k, i in enumerate(idx):
                    a, b = int(off[k]), int(off[k] + N[k])
                    outs[i] = (keys[a:b], vals[a:b]) if with_val else keys[a:b]
            ev = torch.cuda.Event()
            ev.record(s)
        return (ev, outs, keep)

    def done(self, handle) -> bool:
        return handle[0].query()

    def results(self, handle):
        return handle[1]


class Server:
    def __init__(self, executor, budget_bytes: int, max_slots: int = 256, max_batch: int = 64,
                 max_inflight: int = 2, clock: Callable[[], float] = time.perf_counter,
                 idle_wait: float = 50e-6):
        self.executor = executor
        self.budget = Budget(budget_bytes)
        self.max_slots = max_slots
        self.max_batch = max_batch
        self.max_inflight = max_inflight
        self.clock = clock
        self.idle_wait = idle_wait
        self._lock = threading.Lock()
        self._wake = threading.Condition(self._lock)
        self._incoming: collections.deque = collections.deque()
        self._pending: collections.deque = collections.deque()
        self._admitted: list = []
        self._inflight: list = []
        self._stop = False
        self._thread: Optional[threading.Thread] = None
        self._rid = 0
        self.latencies: list = []
        self.completed_outputs = 0
        self.failed = 0
        self.rejected = 0
        self.batches = 0
        self.batch_sizes: list = []
        self.max_concurrent_batches = 0
        self.first_arrival = None
        self.last_done = None

    # -- client side
    def submit(self, A, B, A_val=None, B_val=None, arrival: Optional[float] = None):
        nbytes = self.executor.footprint(A, B, A_val, B_val)
        outputs = len(A) + len(B) if not hasattr(A, "numel") else A.numel() + B.numel()
        token = self.executor.ready_token() if hasattr(self.executor, "ready_token") else None
        with self._lock:
            req = MergeRequest(self._rid, A, B, A_val, B_val, nbytes, outputs,
                               self.clock() if arrival is None else arrival, token)
            self._rid += 1
            if self.first_arrival is None:
                self.first_arrival = req.arrival
            self._incoming.append(req)
            self._wake.notify()
        return req.future

    def start(self):
        if self._thread is not None:
            raise RuntimeError("server already started")
        self._stop = False
        self._thread = threading.Thread(target=self._loop, name="merge-scheduler", daemon=True)
        self._thread.start()
        return self

    def stop(self, timeout: float = 60.0):
        """Finish every request already submitted, then stop the thread."""
        with self._lock:
            self._stop = True
            self._wake.notify()
        if self._thread is not None:
            self._thread.join(timeout)
            if self._thread.is_alive():
                raise RuntimeError("scheduler did not drain in time")
            self._thread = None

    def __enter__(self):
        return self.start()

    def __exit__(self, *exc):
        self.stop()

    # -- scheduler
    def _busy(self):
        return bool(self._incoming or self._pending or self._admitted or self._inflight)

    def _admit(self):
        while self._pending and len(self._admitted) + self._inflight_count() < self.max_slots:
            req = self._pending[0]
            if req.future.cancelled():
                self._pending.popleft()
                continue
            if req.nbytes > self.budget.total:
                self._pending.popleft()
                self.rejected += 1
                req.future.set_exception(BudgetError(
                    f"request {req.rid} needs {req.nbytes} bytes; budget is {self.budget.total}"))
                continue
            if not self.budget.try_reserve(req.nbytes):
                break  # wait for memory (arrival order is kept)
            req.future.set_running_or_notify_cancel()
            self._admitted.append(self._pending.popleft())

    def _inflight_count(self):
        return sum(len(b) for _, b in self._inflight)

    def _launch(self):
        while self._admitted and len(self._inflight) < self.max_inflight:
            batch = self._admitted[:self.max_batch]
            del self._admitted[:len(batch)]
            now = self.clock()
            for r in batch:
                r.launched = now
            try:
                handle = self.executor.launch(batch)
            except Exception as exc:  # a failed launch fails its requests only
                self._fail(batch, exc)
                continue
            self._inflight.append((handle, batch))
            self.batches += 1
            self.batch_sizes.append(len(batch))
            self.max_concurrent_batches = max(self.max_concurrent_batches, len(self._inflight))

    def _fail(self, batch, exc):
        for r in batch:
            self.budget.release(r.nbytes)
            self.failed += 1
            if not r.future.done():
                r.future.set_exception(exc)

    def _complete(self):
        progressed = False
        still = []
        for handle, batch in self._inflight:
            try:
                finished = self.executor.done(handle)
            except Exception as exc:
                self._fail(batch, exc)
                progressed = True
                continue
            if not finished:
                still.append((handle, batch))
                continue
            progressed = True
            try:
                outs = self.executor.results(handle)
            except Exception as exc:
                self._fail(batch, exc)
                continue
            now = self.clock()
            for r, out in zip(batch, outs):
                r.done = now
                self.budget.release(r.nbytes)
                self.latencies.append(now - r.arrival)
                self.completed_outputs += r.outputs
                r.future.set_result(out)
            self.last_done = now
        self._inflight = still
        return progressed

    def _loop(self):
        while True:
            with self._lock:
                while self._incoming:
                    self._pending.append(self._incoming.popleft())
                if self._stop and not self._busy():
                    return
                self._admit()
                self._launch()
            progressed = self._complete()
            if not progressed:
                with self._lock:
                    if not self._incoming and not (self._stop and not self._busy()):
                        self._wake.wait(self.idle_wait if (self._inflight or self._admitted)
                                        else 0.01)

    # -- reporting
    def stats(self) -> dict:
        lat = sorted(self.latencies)

        def pct(p):
            if not lat:
                return None
            k = min(len(lat) - 1, max(0, int(round(p / 100.0 * (len(lat) - 1)))))
            return lat[k]

        span = (self.last_done - self.first_arrival) if lat else None
        return {
            "completed": len(lat),
            "failed": self.failed,
            "rejected": self.rejected,
            "batches": self.batches,
            "mean_batch": (sum(self.batch_sizes) / len(self.batch_sizes)) if self.batch_sizes else 0,
            "max_concurrent_batches": self.max_concurrent_batches,
            "p50_s": pct(50),
            "p99_s": pct(99),
            "keys_per_s": (self.completed_outputs / span) if span else None,
            "budget_peak_bytes": self.budget.peak,
        }


class ServerDone(ctypes.Structure):
    """cm_server_done (80 bytes)."""
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("C", ctypes.c_void_p), ("C_val", ctypes.c_void_p),
                ("keys_offset", ctypes.c_uint64), ("vals_offset", ctypes.c_uint64),
                ("queued_ns", ctypes.c_uint64), ("latency_ns", ctypes.c_uint64),
                ("ended_ns", ctypes.c_uint64), ("device_ns", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    """cm_server_stats (80 bytes)."""
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("failed", ctypes.c_uint64), ("canceled", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("max_batch_seen", ctypes.c_uint64),
                ("arena_bytes", ctypes.c_uint64), ("arena_peak_bytes", ctypes.c_uint64),
                ("busy_ms", ctypes.c_double), ("span_ms", ctypes.c_double)]


class NativeServer:
    """The library's own serving runtime (cm_server_*): a scheduler thread in
    the library admits requests in arrival order against an output arena in
    HBM (a torch buffer owned here), launches the admitted ones as one batch
    per step on up to `max_inflight` streams, and reports finished merges to
    poll().  A finished merge's outputs stay in the arena until release().
    Python does argument marshalling only."""

    def __init__(self, key_dtype="uint32", with_payload=True, arena_bytes=32 << 30,
                 max_batch=64, max_inflight=2, max_requests=4096, device="cuda:0", arena=None,
                 descending=False):
        import torch
        from . import KEY_DESC_OFFSET, KEY_TYPES, load
        self.torch = torch
        self.device = torch.device(device)
        self.key_dtype = getattr(torch, str(key_dtype).replace("torch.", ""))
        self.with_payload = bool(with_payload)
        self.arena = arena if arena is not None else torch.empty(
            arena_bytes, dtype=torch.uint8, device=self.device)
        if self.arena.dtype != torch.uint8 or self.arena.device != self.device \
                or not self.arena.is_contiguous():
            raise ValueError("the arena must be a contiguous uint8 tensor on the server's device")
        self.lib = load()
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            kt = KEY_TYPES[str(self.key_dtype).replace("torch.", "")]
            rc = self.lib.cm_server_create(kt + (KEY_DESC_OFFSET if descending else 0),
                                           int(self.with_payload), self.arena.data_ptr(),
                                           self.arena.numel(), max_batch, max_inflight,
                                           max_requests, ctypes.byref(h))
        self._check(rc, "cm_server_create")
        self._h = h
        self._ticket = ctypes.c_uint64()
        self._host = {}  # ticket -> host tensors of a host request (kept alive until release)
        self._cap = 256
        self._done = (ServerDone * self._cap)()
        self._count = ctypes.c_uint32()

    def _check(self, rc, where):
        if rc != 0:
            from . import CMError
            raise CMError(rc, where)

    def _check_inputs(self, A, B, A_val, B_val):
        # the runtime reads m (n) keys and payloads from these addresses: a
        # shorter payload array would be read past its end
        if A.dtype != self.key_dtype or B.dtype != self.key_dtype:
            raise TypeError(f"keys must be {self.key_dtype}")
        if not self.with_payload:
            if A_val is not None or B_val is not None:
                raise ValueError("this server has no payloads")
            return
        if A_val.dtype != self.torch.uint32 or B_val.dtype != self.torch.uint32 \
                or A_val.numel() != A.numel() or B_val.numel() != B.numel():
            raise ValueError("payloads must be uint32 and as long as their keys")

    def submit_ptrs(self, A, A_val, m, B, B_val, n, stream=None, pending=False):
        """Raw form (device addresses and sizes); returns the status and
        sets self.last_ticket on success (CM_EBUSY = -9: no slot free)."""
        rc = self.lib.cm_server_submit(self._h, A, A_val, m, B, B_val, n, stream,
                                       1 if pending else 0, ctypes.byref(self._ticket))
        self.last_ticket = self._ticket.value
        return rc

    def submit(self, A, B, A_val=None, B_val=None, stream=None):
        """Queue a merge of device tensors; it waits for the work enqueued so
        far on `stream` (default: the current stream), which produced them.
        Returns the ticket."""
        torch = self.torch
        for t in (A, B) + ((A_val, B_val) if self.with_payload else ()):
            if t is None or t.device != self.device or t.dim() != 1 or not t.is_contiguous():
                raise ValueError("inputs must be contiguous 1-D tensors on the server's device")
        self._check_inputs(A, B, A_val, B_val)
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        rc = self.submit_ptrs(A.data_ptr() if A.numel() else None,
                              A_val.data_ptr() if self.with_payload and A.numel() else None,
                              A.numel(), B.data_ptr() if B.numel() else None,
                              B_val.data_ptr() if self.with_payload and B.numel() else None,
                              B.numel(), s.cuda_stream, pending=True)
        self._check(rc, "cm_server_submit")
        return self.last_ticket

    def submit_host(self, A, B, A_val=None, B_val=None, C=None, C_val=None):
        """Queue a merge of host (CPU) tensors: the runtime copies the inputs
        to its arena on a copy stream of its own, merges them in a batch and
        copies the outputs back into C / C_val (pinned CPU tensors allocated
        here unless given) on a second copy stream; the request is reported
        by poll() once the outputs are in host memory.  Pinned inputs
        (tensor.pin_memory()) let the copies overlap.  The tensors are kept
        referenced here until release().  Returns the ticket; the outputs
        are host_outputs(ticket)."""
        torch = self.torch
        ins = (A, B) + ((A_val, B_val) if self.with_payload else ())
        for t in ins:
            if t is None or not isinstance(t, torch.Tensor) or t.device.type != "cpu" \
                    or t.dim() != 1 or not t.is_contiguous():
                raise ValueError("inputs must be contiguous 1-D CPU tensors")
        self._check_inputs(A, B, A_val, B_val)
        N = A.numel() + B.numel()
        if C is None:
            C = torch.empty(N, dtype=self.key_dtype).pin_memory()
        if self.with_payload and C_val is None:
            C_val = torch.empty(N, dtype=torch.uint32).pin_memory()
        outs = ((C, self.key_dtype),) + (((C_val, torch.uint32),) if self.with_payload else ())
        for t, dtype in outs:
            if not isinstance(t, torch.Tensor) or t.device.type != "cpu" or not t.is_contiguous() \
                    or t.numel() != N or t.dtype != dtype:
                raise ValueError("outputs must be contiguous CPU tensors of m + n elements "
                                 "(keys of the server's key type, uint32 payloads)")

        def ptr(t):
            return t.data_ptr() if t is not None and t.numel() else None
        rc = self.lib.cm_server_submit_host(
            self._h, ptr(A), ptr(A_val) if self.with_payload else None, A.numel(), ptr(B),
            ptr(B_val) if self.with_payload else None, B.numel(), ptr(C),
            ptr(C_val) if self.with_payload else None, ctypes.byref(self._ticket))
        self._check(rc, "cm_server_submit_host")
        t = self._ticket.value
        self._host[t] = (ins, C, C_val)
        return t

    def host_outputs(self, ticket):
        """The host output tensors of a host request: C, or (C, C_val)."""
        _, C, C_val = self._host[ticket]
        return (C, C_val) if self.with_payload else C

    def poll(self, wait_us=0):
        """Finished merges (cm_server_done entries), at most 256 per call."""
        self._check(self.lib.cm_server_poll(self._h, self._done, self._cap,
                                            ctypes.byref(self._count), int(wait_us)),
                    "cm_server_poll")
        return [self._done[k] for k in range(self._count.value)]

    def outputs(self, done, num_outputs):
        """Views of a finished merge's keys (and payloads) in the arena."""
        ks = self.torch.empty(0, dtype=self.key_dtype).element_size()
        keys = self.arena[done.keys_offset:done.keys_offset + num_outputs * ks].view(
            self.key_dtype)
        if not self.with_payload:
            return keys
        vals = self.arena[done.vals_offset:done.vals_offset + num_outputs * 4].view(
            self.torch.uint32)
        return keys, vals

    def release(self, ticket):
        self._check(self.lib.cm_server_release(self._h, ticket), "cm_server_release")
        self._host.pop(ticket, None)

    def stats(self) -> dict:
        st = ServerStats()
        self._check(self.lib.cm_server_get_stats(self._h, ctypes.byref(st)),
                    "cm_server_get_stats")
        return {name: getattr(st, name) for name, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._check(self.lib.cm_server_destroy(self._h), "cm_server_destroy")
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
