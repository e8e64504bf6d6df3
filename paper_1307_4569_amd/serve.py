"""Continuous-batching request loop for DGT requests of mixed lattices.

Requests (signal of length L on the device, lattice (L, a, M, lam1, lam2))
queue per lattice plan.  Each call of ``Server.pump()``

1. retires finished batches (a HIP event per batch) and releases their HBM
   footprint,
2. admits new batches while stream slots and the HBM budget allow: the plan
   whose oldest request waited longest goes first, up to ``max_batch``
   requests of that plan form one list-batched launch
   (``dgtns_forward_batch``: no staging copies), its footprint is the output
   coefficients plus the workspace of that batch, and a batch that does not
   fit waits (or shrinks) until memory frees up.

Plans and their windows stay resident on the device.  Batches run on a pool
of streams of default priority, so requests admitted while others run
overlap on the GPU.  Latency is measured from a request's arrival time to
the moment the loop observes its batch's completion event.

Stream ordering: a batch's stream first waits for the work the submitting
thread's current stream had enqueued when the batch was launched, so a
signal produced asynchronously before submit() is complete when it is read.
The request keeps its signal tensor alive until the batch completes.  The
coefficient tensors handed out are recorded on the stream that is current
when the loop retires the batch (the consumer's), so the caching allocator
does not reuse their memory on a pool stream while the consumer's work on
them is pending.  Each stream slot owns one workspace buffer, sized for the
largest plan at max_batch and reused by every launch on that slot's stream.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional, Tuple

Key = Tuple[int, int, int, int, int]


@dataclasses.dataclass
class Request:
    rid: int
    key: Key
    f: object                       # device tensor (L,) in the server's precision
    arrival: float                  # seconds, on the server clock
    done_time: Optional[float] = None
    c: object = None                # (N, M) coefficients once done
    error: Optional[BaseException] = None
    batch_size: int = 0

    @property
    def latency(self) -> Optional[float]:
        return None if self.done_time is None else self.done_time - self.arrival


class GpuExecutor:
    """Launches list-batched forward transforms through libdgtns.  Plans use
    `algorithm` ("auto" by default: the shear algorithm, or the multiwindow
    one for lattices whose shear needs a frequency shear)."""

    def __init__(self, window_fn: Callable[[Key], object], dtype=None, streams: int = 4, max_batch: int = 8,
                 device=None, algorithm: str = "auto"):
        import torch

        from . import _binding as B
        self.torch, self.B = torch, B
        self.dtype = dtype or torch.complex64
        self.device = torch.device(device if device is not None else "cuda")
        self.streams = [torch.cuda.Stream(self.device) for _ in range(streams)]
        self.max_batch = min(max_batch, B.DGTNS_MAX_LIST_BATCH)
        self.window_fn = window_fn
        self.plans: Dict[Key, object] = {}
        self.es = 8 if self.dtype == torch.complex64 else 16
        self.ws = [None] * streams          # per-slot workspace, grown as plans are added
        self.algorithm = algorithm

    def plan(self, key: Key):
        p = self.plans.get(key)
        if p is None:
            from .api import Plan
            p = Plan(*key, dtype=self.dtype, max_batch=self.max_batch, device=self.device, algorithm=self.algorithm)
            p.set_window(self.window_fn(key))
            need = self.B.dgtns_workspace_bytes(p._h, self.B.DGTNS_OP_FORWARD, self.max_batch)
            self.torch.cuda.synchronize(self.device)
            for i in range(len(self.ws)):
                if self.ws[i] is None or self.ws[i].numel() < need:
                    self.ws[i] = self.torch.empty(need, dtype=self.torch.uint8, device=self.device)
            self.plans[key] = p
        return p

    def prepare(self, keys):
        """Create the plans (tables and windows resident) before serving."""
        for k in keys:
            self.plan(k)

    def footprint(self, key: Key, nb: int) -> int:
        p = self.plan(key)
        return nb * p.N * p.M * self.es + self.B.dgtns_workspace_bytes(p._h, self.B.DGTNS_OP_FORWARD, nb)

    def launch(self, key: Key, reqs: List[Request], slot: int):
        torch = self.torch
        p = self.plan(key)
        st = self.streams[slot]
        nb = len(reqs)
        # the signals were produced on the submitter's stream
        st.wait_stream(torch.cuda.current_stream(self.device))
        ws = self.ws[slot]
        with torch.cuda.stream(st):
            c = torch.empty((nb, p.N, p.M), dtype=self.dtype, device=self.device)
            base, stride = c.data_ptr(), p.N * p.M * self.es
            self.B.dgtns_forward_batch(p._h, [r.f.data_ptr() for r in reqs], 0,
                                       [base + i * stride for i in range(nb)], ws.data_ptr(), ws.numel(),
                                       st.cuda_stream)
            ev = torch.cuda.Event()
            ev.record(st)
        return (ev, c)

    @staticmethod
    def done(handle) -> bool:
        return handle[0].query()

    def outputs(self, handle):
        c = handle[1]
        # the consumer uses the coefficients on its own (current) stream
        c.record_stream(self.torch.cuda.current_stream(self.device))
        return [c[i] for i in range(c.shape[0])]

    @property
    def nslots(self) -> int:
        return len(self.streams)


class Server:
    def __init__(self, executor, hbm_budget: int, max_inflight_per_slot: int = 2, max_batch: Optional[int] = None,
                 clock: Callable[[], float] = time.perf_counter, keep_outputs: bool = True):
        self.ex = executor
        self.keep_outputs = keep_outputs
        self.budget = int(hbm_budget)
        self.max_inflight_per_slot = max_inflight_per_slot
        self.max_batch = max_batch or getattr(executor, "max_batch", 8)
        self.clock = clock
        self.t0 = clock()
        self.queues: Dict[Key, collections.deque] = collections.OrderedDict()
        self.inflight: List[tuple] = []          # (handle, reqs, bytes, slot)
        self.slot_load = [0] * executor.nslots
        self.bytes_inflight = 0
        self.peak_bytes = 0
        self.completed: List[Request] = []
        self.npending = 0
        self.batches = 0

    def now(self) -> float:
        return self.clock() - self.t0

    def submit(self, req: Request) -> Request:
        self.queues.setdefault(req.key, collections.deque()).append(req)
        self.npending += 1
        return req

    def _retire(self):
        keep = []
        for item in self.inflight:
            handle, reqs, nbytes, slot = item
            if self.ex.done(handle):
                t = self.now()
                try:
                    outs = self.ex.outputs(handle) if self.keep_outputs else [None] * len(reqs)
                    for r, c in zip(reqs, outs):
                        r.c, r.done_time = c, t
                except BaseException as e:     # a failed batch fails only its own requests
                    for r in reqs:
                        r.error, r.done_time = e, t
                self.completed.extend(reqs)
                self.bytes_inflight -= nbytes
                self.slot_load[slot] -= 1
            else:
                keep.append(item)
        self.inflight = keep

    def _admit(self):
        while self.npending:
            slot = min(range(len(self.slot_load)), key=lambda i: self.slot_load[i])
            if self.slot_load[slot] >= self.max_inflight_per_slot:
                return
            # plan whose oldest request has waited longest
            key = min((k for k, q in self.queues.items() if q), key=lambda k: self.queues[k][0].arrival)
            q = self.queues[key]
            nb = min(len(q), self.max_batch)
            free = self.budget - self.bytes_inflight
            fp = self.ex.footprint(key, nb)
            while nb > 1 and fp > free:
                nb -= 1
                fp = self.ex.footprint(key, nb)
            if fp > free:
                if self.bytes_inflight == 0:
                    # cannot fit even alone: fail the request instead of waiting forever
                    r = q.popleft()
                    self.npending -= 1
                    r.error = MemoryError(f"request footprint {fp} B exceeds the HBM budget {self.budget} B")
                    r.done_time = self.now()
                    self.completed.append(r)
                    continue
                return
            reqs = [q.popleft() for _ in range(nb)]
            self.npending -= nb
            for r in reqs:
                r.batch_size = nb
            try:
                handle = self.ex.launch(key, reqs, slot)
            except BaseException as e:
                t = self.now()
                for r in reqs:
                    r.error, r.done_time = e, t
                self.completed.extend(reqs)
                continue
            self.inflight.append((handle, reqs, fp, slot))
            self.slot_load[slot] += 1
            self.bytes_inflight += fp
            self.peak_bytes = max(self.peak_bytes, self.bytes_inflight)
            self.batches += 1

    def pump(self):
        self._retire()
        self._admit()

    def idle(self) -> bool:
        return self.npending == 0 and not self.inflight

    def run(self, requests: List[Request], arrivals: Optional[List[float]] = None) -> List[Request]:
        """Feed requests at their arrival times (seconds from now; None: all at
        once) and pump until every request has completed."""
        n = len(requests)
        self.t0 = self.clock()
        i = 0
        while i < n or not self.idle():
            t = self.now()
            while i < n and (arrivals is None or arrivals[i] <= t):
                requests[i].arrival = arrivals[i] if arrivals is not None else t
                self.submit(requests[i])
                i += 1
            self.pump()
        return requests


def latency_stats(reqs: List[Request], coeffs: Callable[[Request], int]) -> dict:
    import numpy as np
    ok = [r for r in reqs if r.error is None]
    lat = np.array([r.latency for r in ok]) * 1e3
    span = max(r.done_time for r in reqs) - min(r.arrival for r in reqs)
    tot = sum(coeffs(r) for r in ok)
    return {"requests": len(reqs), "failed": len(reqs) - len(ok),
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "makespan_s": span, "req_per_s": len(ok) / span,
            "coeffs_per_s": tot / span,
            "mean_batch": float(np.mean([r.batch_size for r in ok]))}
