"""Request loop for force/energy solves of many independent slab systems.

Each registered system (for instance one Brownian-dynamics trajectory) keeps
a resident plan on the device: its tables (Chebyshev nodes, quadrature
weights, twiddles and the per-mode solver coefficients) are built once. The
per-solve workspace is not resident: it is taken from the device allocator
when a request is admitted and given back when it finishes, so the number of
requests on the GPU at once is bounded by an HBM budget instead of by the
number of systems. A bounded queue sheds requests beyond its length
(Overloaded) instead of letting the backlog grow without limit.

Scheduling is continuous batching: a request is admitted as soon as an
execution slot (a HIP stream) is free and its footprint (workspace plus
outputs) fits in what is left of the budget; requests on different slots run
concurrently on the device, and a finished request frees its slot and memory
for the next one at once, without waiting for the others. Requests are taken
in arrival order; a request whose system already has one in flight waits
(the plan of a system runs one solve at a time) while later requests of other
systems may pass it. A request larger than the whole budget is rejected.

The GPU work is done by libdpse (the kernels of dpse_solve); this module only
schedules. The backend is pluggable so that the scheduling logic can be
tested without a GPU.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field
from typing import Any, Callable, Dict, List, Optional


class Rejected(RuntimeError):
    """A request that can never be admitted (larger than the budget)."""


class Overloaded(RuntimeError):
    """The queue is full: the request is shed instead of queued."""


@dataclass
class Request:
    key: Any
    pos: Any
    q: Any
    n: int
    footprint: int
    arrival: float
    ready_event: Any = None
    admitted: float = 0.0
    finished: float = 0.0
    status: int = -1
    result: Any = None
    slot: int = -1
    ticket: Any = None
    callbacks: List[Callable] = field(default_factory=list)

    # Future-like interface
    def done(self) -> bool:
        return self.status >= 0

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class DpseBackend:
    """Runs admitted requests with libdpse on a set of HIP streams.

    With autotune, the first request of every grid shape (Nx, Ny, Nz,
    support) tunes the launch shapes of spreading, interpolation and the
    column kernel on its own charges (dpse_plan_autotune, synchronous, before
    its solve is queued); every later plan of that shape takes the stored
    choice once."""

    def __init__(self, precision: int, device=None, autotune: bool = True):
        import torch
        from . import native
        self.torch = torch
        self.native = native
        self.precision = precision
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.autotune = autotune
        self.tiles = {}        # grid shape -> tuned choice

    def make_streams(self, n: int):
        return [self.torch.cuda.Stream(device=self.device) for _ in range(n)]

    def new_plan(self, params, max_n: int):
        return self.native.Plan(params, max_n=max_n, precision=self.precision, own_workspace=False)

    def footprint(self, plan, n: int) -> int:
        return plan.info["workspace_bytes"] + 8 * (4 * n + 1)

    def launch(self, plan, stream, req: Request):
        torch = self.torch
        with torch.cuda.stream(stream):
            if req.ready_event is not None:
                stream.wait_event(req.ready_event)
            ws = torch.empty(plan.info["workspace_bytes"], dtype=torch.uint8, device=self.device)
            E = torch.empty(1, dtype=torch.float64, device=self.device)
            PH = torch.empty(req.n, dtype=torch.float64, device=self.device)
            F = torch.empty((req.n, 3), dtype=torch.float64, device=self.device)
            plan.bind(ws, stream)
            if self.autotune and not getattr(plan, "_serve_tuned", False):
                p = plan.params
                key = (p.Nx, p.Ny, p.Nz, plan.info["support"])
                if key in self.tiles:
                    plan.set_tiles(self.tiles[key])
                else:
                    self.tiles[key], _ = plan.autotune(req.pos, req.q, reps=2)
                plan._serve_tuned = True
            plan.solve(req.pos, req.q, E, PH, F)
            ev = torch.cuda.Event()
            ev.record(stream)
        # the inputs are read on this stream: keep the allocator from reusing them early
        req.pos.record_stream(stream)
        req.q.record_stream(stream)
        return (ev, ws, (E, PH, F))

    def is_done(self, ticket) -> bool:
        return ticket[0].query()

    def finish(self, plan, ticket):
        st = plan.sync_status()
        plan.workspace = None  # the workspace goes back to the allocator (stream ordered)
        E, PH, F = ticket[2]
        cur = self.torch.cuda.current_stream(self.device)
        for t in (E, PH, F):
            t.record_stream(cur)
        return st, (E, PH, F)


class Server:
    """Continuous-batching request loop (see the module docstring)."""

    def __init__(self, budget_bytes: int, n_slots: int = 8, backend=None, precision: Optional[int] = None,
                 clock: Callable[[], float] = time.perf_counter, max_queue: int = 1 << 30, autotune: bool = True):
        if backend is None:
            from .native import DPSE_MIXED
            backend = DpseBackend(DPSE_MIXED if precision is None else precision, autotune=autotune)
        self.backend = backend
        self.budget = int(budget_bytes)
        self.clock = clock
        self.streams = backend.make_streams(n_slots)
        self.free_slots = list(range(n_slots))[::-1]
        self.plans: Dict[Any, Any] = {}
        self.queue: "collections.deque[Request]" = collections.deque()
        self.active: List[Request] = []
        self.busy_keys = set()
        self.in_use = 0
        self.max_queue = int(max_queue)
        self.stats = dict(submitted=0, admitted=0, completed=0, failed=0, shed=0, peak_bytes=0, peak_active=0)

    # systems -------------------------------------------------------------
    def register(self, key, params, max_n: int):
        """Creates the resident plan of a system (tables only)."""
        if key in self.plans:
            raise KeyError(f"system {key!r} already registered")
        self.plans[key] = self.backend.new_plan(params, int(max_n))

    def unregister(self, key):
        if key in self.busy_keys or any(r.key == key for r in self.queue):
            raise RuntimeError(f"system {key!r} has requests pending")
        plan = self.plans.pop(key)
        close = getattr(plan, "close", None)
        if close:
            close()

    # requests ------------------------------------------------------------
    def submit(self, key, pos, q, ready_event=None, arrival: Optional[float] = None) -> Request:
        plan = self.plans[key]
        n = int(q.shape[0])
        if n > plan.max_n:
            raise ValueError(f"{n} charges exceed the plan's max_n {plan.max_n}")
        fp = self.backend.footprint(plan, n)
        if fp > self.budget:
            raise Rejected(f"request footprint {fp} B exceeds the budget {self.budget} B")
        if len(self.queue) >= self.max_queue:
            self.stats["shed"] += 1
            raise Overloaded(f"queue full ({self.max_queue} requests)")
        r = Request(key=key, pos=pos, q=q, n=n, footprint=fp, ready_event=ready_event,
                    arrival=self.clock() if arrival is None else arrival)
        self.queue.append(r)
        self.stats["submitted"] += 1
        return r

    def _admit(self):
        if not self.queue or not self.free_slots:
            return
        kept = collections.deque()
        while self.queue and self.free_slots:
            r = self.queue.popleft()
            if r.key in self.busy_keys:
                kept.append(r)
                continue
            if self.in_use + r.footprint > self.budget:
                # the oldest admissible request waits for memory; nothing behind it passes
                kept.append(r)
                break
            slot = self.free_slots.pop()
            r.slot = slot
            r.admitted = self.clock()
            self.in_use += r.footprint
            self.busy_keys.add(r.key)
            r.ticket = self.backend.launch(self.plans[r.key], self.streams[slot], r)
            self.active.append(r)
            self.stats["admitted"] += 1
        kept.extend(self.queue)
        self.queue = kept
        self.stats["peak_bytes"] = max(self.stats["peak_bytes"], self.in_use)
        self.stats["peak_active"] = max(self.stats["peak_active"], len(self.active))

    def _retire(self) -> int:
        done = 0
        still = []
        for r in self.active:
            if self.backend.is_done(r.ticket):
                st, res = self.backend.finish(self.plans[r.key], r.ticket)
                r.finished = self.clock()
                r.status, r.result, r.ticket = st, res, None
                self.in_use -= r.footprint
                self.busy_keys.discard(r.key)
                self.free_slots.append(r.slot)
                self.stats["completed" if st == 0 else "failed"] += 1
                for cb in r.callbacks:
                    cb(r)
                done += 1
            else:
                still.append(r)
        self.active = still
        return done

    def step(self) -> int:
        """One pass of the loop: retire finished requests, admit queued ones.
        Returns the number of requests on the device."""
        self._retire()
        self._admit()
        return len(self.active)

    def pending(self) -> int:
        return len(self.queue) + len(self.active)

    def drain(self, poll_s: float = 0.0):
        while self.pending():
            if not self.step() and self.queue:
                raise RuntimeError("queue cannot make progress")
            if poll_s:
                time.sleep(poll_s)

    def close(self):
        self.drain()
        for k in list(self.plans):
            self.unregister(k)
