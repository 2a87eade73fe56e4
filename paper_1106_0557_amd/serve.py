"""Continuous-batching serving loop for isolated Poisson solves.

Requests of different mesh sizes arrive over time.  Plans (twiddles and the
Green's-function spectrum, computed once per size as in Sec. 2.2.2 of the paper)
stay resident in device memory and are shared by every request of that size;
workspaces are pooled.  A request is admitted when its device footprint
(workspace + output) fits the memory budget and an in-flight slot is free.

Scheduling is at pass granularity.  Each scheduler step issues, for every
in-flight request, the next of its passes (five, or three for a plan that fuses
the x and y transforms of each plane); requests of one mesh size at the same
pass are grouped into one batched launch (``pspfft_pass_batched``), and the
launches of a step go to different streams.  A launch waits (by events) only for
the launches its own requests were last in, so small meshes move through their
passes while a large mesh's pass runs beside them, and a step retires when its
own launches are done, in whatever order steps finish.  A request admitted while
others are in flight starts its first pass in the next step, so a solve never
waits for a whole batch to finish.  Results do not depend on the mix: each
problem is tiled the same way whatever shares its launch.

The executor interface (plans and byte counts, workspace pool, output
allocation, ``begin_step``/``run_pass``/``end_step`` and ``is_done``/``wait`` on
the step tokens) lets tests drive the same scheduler without a GPU.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass
from typing import Any, Callable, Dict, List, Optional, Sequence, Tuple

NUM_PASSES = 5


@dataclass
class Request:
    index: int
    n: Tuple[int, int, int]      # (nx, ny, nz)
    h: Tuple[float, float, float]
    S: Any                       # source, resident on the device
    arrival: float = 0.0         # seconds, on the scheduler's clock
    phi: Any = None              # output, allocated at admission
    next_pass: int = -1          # -1 waiting, 0..4 next pass to issue, 5 all issued
    passes: Tuple[int, ...] = tuple(range(NUM_PASSES))  # passes with work for this request's plan
    done: bool = False
    rejected: bool = False
    error: Optional[str] = None
    t_admit: float = math.nan
    t_done: float = math.nan
    _ws: Any = None
    _ptrs: Any = None            # executor's cached launch arguments while admitted
    _dep: Any = None             # executor's record of the launch this request was last in
    _ready: Any = None           # executor's mark, at admission, of the caller's work before the first pass

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


NUM_STREAMS = 8


class GpuExecutor:
    """Executor over the HIP library: plan cache, workspace pool, a pool of streams."""

    def __init__(self, dtype=None, device: int = 0):
        import torch

        import paper_1106_0557_amd as ps

        self.torch = torch
        self.ps = ps
        self.dtype = dtype or torch.float32
        self.device = device
        self.plans: Dict[Any, Any] = {}
        self.pool: Dict[Any, List[Any]] = collections.defaultdict(list)
        # default priority streams only
        self.streams = [torch.cuda.Stream(device=device) for _ in range(NUM_STREAMS)]
        # first work on a stream sets up its queue; do that now rather than
        # inside the first steps that happen to use it
        for s in self.streams:
            with torch.cuda.stream(s):
                torch.zeros(1, device=f"cuda:{device}")
            s.synchronize()
        self._step = 0                  # index of the step being built
        self._pending: set = set()      # steps issued and not yet seen complete
        self._launches = 0              # launches of the step being built
        self._step_events: List[Any] = []
        self._step_ready: List[Any] = []  # admission marks of the step being built
        self._events: List[Any] = []  # recycled events
        self._ws_bytes: Dict[Any, int] = {}  # workspace bytes per mesh

    # ------------------------------------------------------------- plans
    def key(self, req: Request):
        return (req.n, req.h, self.dtype)

    def plan(self, req: Request):
        k = self.key(req)
        p = self.plans.get(k)
        if p is None:
            nx, ny, nz = req.n
            p = self.ps.Plan(nx, ny, nz, h=req.h, dtype=self.dtype)
            self.plans[k] = p
        return p

    def workspace_bytes(self, req: Request) -> int:
        k = req.n
        b = self._ws_bytes.get(k)
        if b is None:
            nx, ny, nz = k
            b = self._ws_bytes[k] = self.ps.workspace_bytes(nx, ny, nz, self.dtype)
        return b

    def active_passes(self, req: Request) -> Tuple[int, ...]:
        return self.plan(req).active_passes

    def output_bytes(self, req: Request) -> int:
        nx, ny, nz = req.n
        return nx * ny * nz * (4 if self.dtype == self.torch.float32 else 8)

    def resident_bytes(self) -> int:
        return sum(p.resident_bytes for p in self.plans.values())

    def has_plan(self, req: Request) -> bool:
        return self.key(req) in self.plans

    def plan_bytes(self, req: Request) -> int:
        """Device bytes the plan of this request's mesh keeps resident (spectrum,
        twiddles, tables), known before the plan is created."""
        nx, ny, nz = req.n
        return self.ps.plan_resident_bytes(nx, ny, nz, self.dtype)

    # ------------------------------------------------ workspaces, outputs
    def acquire(self, req: Request):
        k = self.key(req)
        if self.pool[k]:
            return self.pool[k].pop()
        # memory from torch's caching allocator, wrapped as a workspace: creating
        # and trimming pooled workspaces then costs no device allocation calls
        plan = self.plan(req)
        mem = self.torch.empty(plan.workspace_bytes, dtype=self.torch.uint8, device=f"cuda:{self.device}")
        return self.ps.Workspace(plan, memory=mem)

    def release(self, req: Request, ws) -> None:
        self.pool[self.key(req)].append(ws)

    def trim_pool(self) -> int:
        """Free every pooled (idle) workspace; returns bytes released."""
        freed = 0
        for k, lst in self.pool.items():
            for ws in lst:
                freed += ws.plan.workspace_bytes
                ws.close()
            lst.clear()
        return freed

    def pooled_bytes(self) -> int:
        return sum(ws.plan.workspace_bytes for lst in self.pool.values() for ws in lst)

    def has_pooled(self, req: Request) -> bool:
        return bool(self.pool[self.key(req)])

    def alloc_output(self, req: Request):
        return self.torch.empty(req.S.shape, dtype=self.dtype, device=req.S.device)

    def admitted(self, reqs: Sequence[Request]) -> None:
        """Mark the caller's stream once the requests admitted in one scheduler
        step have their workspaces and outputs (allocated there) and their
        sources (produced there before submission).  Their first launches, on
        streams of the pool, wait for this one mark."""
        ev = self._event()
        ev.record(self.torch.cuda.current_stream(self.device))
        self._step_ready.append(ev)
        for r in reqs:
            r._ready = ev

    # ------------------------------------------------------------ launches
    def begin_step(self) -> None:
        self._launches = 0
        self._step_events = self._step_ready  # the admission marks retire with this step
        self._step_ready = []

    def _pointers(self, req: Request):
        """Launch arguments of an admitted request, checked once."""
        plan = req._ws.plan
        plan.check_field(req.S, "S")
        plan.check_field(req.phi, "Phi")
        return plan.handle, req._ws.handle, req.S.data_ptr(), req.phi.data_ptr()

    def run_pass(self, p: int, reqs: Sequence[Request]) -> None:
        # the k-th launch of a step goes to stream k (mod the pool); it waits
        # only for the launches its requests were last in, unless their steps
        # are already known complete
        s = self.streams[self._launches % len(self.streams)]
        self._launches += 1
        waited = set()
        cols = ([], [], [], [])
        for r in reqs:
            if r._ready is not None:  # first launch: after the caller's work on its stream
                if id(r._ready) not in waited:
                    waited.add(id(r._ready))
                    s.wait_event(r._ready)
                r._ready = None
            if r._dep is not None:
                ev, step = r._dep
                if step in self._pending and id(ev) not in waited:
                    waited.add(id(ev))
                    s.wait_event(ev)  # takes the event as recorded now
            if r._ptrs is None:
                r._ptrs = self._pointers(r)
            for c, v in zip(cols, r._ptrs):
                c.append(v)
        self.ps.pass_batched_ptrs(p, cols[0], cols[1], cols[2], cols[3], s.cuda_stream)
        ev = self._event()
        ev.record(s)
        self._step_events.append(ev)
        for r in reqs:
            r._dep = (ev, self._step)

    def _event(self):
        return self._events.pop() if self._events else self.torch.cuda.Event()

    def end_step(self):
        """The step's token: its index and the events of its launches."""
        token = (self._step, tuple(self._step_events))
        self._pending.add(self._step)
        self._step += 1
        return token

    def release_token(self, token) -> None:
        """A retired step: its launches are complete, so no later launch needs
        to wait on its events, which go back to the pool."""
        step, events = token
        self._pending.discard(step)
        self._events.extend(events)

    @staticmethod
    def is_done(token) -> bool:
        return all(ev.query() for ev in token[1])

    @staticmethod
    def wait(token) -> None:
        for ev in token[1]:
            ev.synchronize()

    def synchronize(self) -> None:
        self.torch.cuda.synchronize(self.device)


class Server:
    """Admission by memory footprint + pass-level continuous batching.

    ``budget_bytes`` bounds the device memory of in-flight requests (workspace
    and output), idle pooled workspaces and the resident plans (spectrum and
    twiddles, one per mesh size, kept once created).  ``max_inflight`` bounds the
    requests on the device, ``max_steps_ahead`` the scheduler steps enqueued but
    not finished.
    """

    def __init__(self, executor, budget_bytes: int, max_inflight: int = 64, max_steps_ahead: int = 16,
                 clock: Callable[[], float] = time.perf_counter):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_inflight = max_inflight
        self.max_steps_ahead = max_steps_ahead
        self.clock = clock
        self.waiting: collections.deque = collections.deque()
        self.inflight: List[Request] = []
        self.finished: List[Request] = []
        # idle workspaces and plans already held by the executor
        self.used = executor.pooled_bytes() + executor.resident_bytes()
        self.steps: collections.deque = collections.deque()  # (token, requests completing in it)
        self.t0 = clock()
        self.launches = 0
        self.max_batch = 0
        self.max_used = 0

    def now(self) -> float:
        return self.clock() - self.t0

    # ------------------------------------------------------------ requests
    def footprint(self, req: Request) -> int:
        return self.ex.workspace_bytes(req) + self.ex.output_bytes(req)

    def _plan_need(self, req: Request) -> int:
        return 0 if self.ex.has_plan(req) else self.ex.plan_bytes(req)

    def submit(self, req: Request) -> None:
        if self.footprint(req) + self._plan_need(req) > self.budget:
            req.rejected = True
            req.done = True
            req.error = "footprint exceeds the memory budget"
            req.t_done = self.now()
            self.finished.append(req)
            return
        self.waiting.append(req)

    def _admit(self) -> None:
        new = []
        while self.waiting and len(self.inflight) < self.max_inflight:
            req = self.waiting[0]
            reuse = self.ex.has_pooled(req)
            need = self.ex.output_bytes(req) + (0 if reuse else self.ex.workspace_bytes(req)) + self._plan_need(req)
            if self.used + need > self.budget:
                # idle pooled workspaces of other sizes give way to a waiting request
                pooled = self.ex.pooled_bytes()
                if pooled and not reuse and self.used - pooled + need <= self.budget:
                    self.used -= self.ex.trim_pool()
                else:
                    break
            self.waiting.popleft()
            req._ws = self.ex.acquire(req)  # creates the plan if it is new; it stays counted in `used`
            req.phi = self.ex.alloc_output(req)
            new.append(req)
            self.used += need
            self.max_used = max(self.max_used, self.used)
            active = getattr(self.ex, "active_passes", None)
            req.passes = tuple(active(req)) if active else tuple(range(NUM_PASSES))
            req.next_pass = req.passes[0]
            req.t_admit = self.now()
            self.inflight.append(req)
        admitted = getattr(self.ex, "admitted", None)
        if new and admitted is not None:
            admitted(new)

    # -------------------------------------------------------------- stepping
    def _finish(self, token, reqs) -> None:
        release = getattr(self.ex, "release_token", None)
        if release is not None:
            release(token)
        t = self.now()
        for r in reqs:
            r.done = True
            r.t_done = t
            self.ex.release(r, r._ws)  # back to the pool, still counted in `used`
            r._ws = None
            r._ptrs = None
            r._dep = None
            self.used -= self.ex.output_bytes(r)  # the output now belongs to the caller
            self.finished.append(r)

    def _retire(self, block: bool = False) -> None:
        """Retire every finished step, in whatever order they finish; with
        ``block``, wait for the oldest one if none has."""
        while self.steps:
            keep = collections.deque()
            retired = False
            for token, reqs in self.steps:
                if self.ex.is_done(token):
                    self._finish(token, reqs)
                    retired = True
                else:
                    keep.append((token, reqs))
            self.steps = keep
            if retired or not block or not self.steps:
                return
            self.ex.wait(self.steps[0][0])

    def step(self) -> bool:
        """One scheduler iteration; returns False when there is nothing to do."""
        self._retire(block=False)
        while len(self.steps) >= self.max_steps_ahead:
            self._retire(block=True)
        self._admit()
        if not self.inflight:
            return bool(self.waiting) or bool(self.steps)
        groups: Dict[Tuple[int, Tuple[int, int, int]], List[Request]] = collections.defaultdict(list)
        for r in self.inflight:
            groups[(r.next_pass, r.n)].append(r)
        self.ex.begin_step()
        for key in sorted(groups):
            self.ex.run_pass(key[0], groups[key])
            self.launches += 1
            self.max_batch = max(self.max_batch, len(groups[key]))
        token = self.ex.end_step()
        completing = []
        still = []
        for r in self.inflight:
            later = [p for p in r.passes if p > r.next_pass]
            r.next_pass = later[0] if later else NUM_PASSES
            (completing if r.next_pass == NUM_PASSES else still).append(r)
        self.inflight = still
        self.steps.append((token, completing))
        return True

    def drain(self) -> None:
        while self.inflight or self.waiting:
            self.step()
        self._retire(block=True)

    # ---------------------------------------------------------- trace replay
    def run_trace(self, requests: Sequence[Request], realtime: bool = True) -> List[Request]:
        """Replay arrivals (``Request.arrival`` seconds after start) and serve them."""
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        self.t0 = self.clock()
        while pending or self.inflight or self.waiting or self.steps:
            now = self.now()
            while pending and (pending[0].arrival <= now or not realtime):
                self.submit(pending.popleft())
            if self.inflight or self.waiting:
                self.step()
            else:
                self._retire(block=False)
                if not self.steps and pending and realtime:
                    time.sleep(min(1e-4, max(0.0, pending[0].arrival - self.now())))
        return self.finished


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q / 100.0
    f = math.floor(k)
    c = min(f + 1, len(xs) - 1)
    return xs[f] + (xs[c] - xs[f]) * (k - f)


def summarize(finished: Sequence[Request], wall: float) -> dict:
    ok = [r for r in finished if not r.rejected]
    lat = [r.latency * 1e3 for r in ok]
    return {
        "requests": len(finished),
        "served": len(ok),
        "rejected": len(finished) - len(ok),
        "solves_per_s": len(ok) / wall if wall > 0 else float("nan"),
        "latency_ms_p50": percentile(lat, 50),
        "latency_ms_p99": percentile(lat, 99),
        "latency_ms_max": max(lat) if lat else float("nan"),
        "wall_s": wall,
    }


def trace_sources(trace, dtype, device="cuda"):
    """Each trace request's own Gaussian-blob source on its n^3 unit-box mesh,
    generated on the device before any timing starts."""
    from . import sources

    return [sources.blob_field(r.n, r.blobs, device=device).to(dtype) for r in trace]


def replay_plain(sizes_arrivals, srcs, dtype=None, realtime=True, log=print):
    """The plain path under the same load: the requests' solves issued one after
    another with ``pspfft_solve`` (one plan and its default workspace per mesh
    size) as they arrive, on one stream.  Latency is arrival to completion; a
    solve starts when it has arrived and the one before it is enqueued."""
    import torch

    import paper_1106_0557_amd as ps

    dtype = dtype or torch.float64
    plans, outs = {}, {}
    for (n, _), S in zip(sizes_arrivals, srcs):
        if n not in plans:
            plans[n] = ps.Plan(n, n, n, h=1.0 / n, dtype=dtype)
            outs[n] = torch.empty_like(S)
            plans[n].solve(S, out=outs[n])  # warm: kernels, default workspace
    torch.cuda.synchronize()
    pool = [torch.cuda.Event() for _ in range(256)]
    pending = collections.deque()
    lat = []
    t0 = time.perf_counter()

    def poll():
        while pending and pending[0][1].query():
            _, ev, arrival = pending.popleft()
            lat.append(time.perf_counter() - t0 - arrival)
            pool.append(ev)

    for i, ((n, arrival), S) in enumerate(zip(sizes_arrivals, srcs)):
        while realtime and time.perf_counter() - t0 < arrival:
            poll()
        plans[n].solve(S, out=outs[n])
        ev = pool.pop() if pool else torch.cuda.Event()
        ev.record()
        pending.append((i, ev, arrival if realtime else 0.0))
        poll()
    while pending:
        pending[0][1].synchronize()
        poll()
    wall = time.perf_counter() - t0
    for p in plans.values():
        p.close()
    lat_ms = [v * 1e3 for v in lat]
    return {"requests": len(lat), "solves_per_s": len(lat) / wall, "latency_ms_p50": percentile(lat_ms, 50),
            "latency_ms_p99": percentile(lat_ms, 99), "latency_ms_max": max(lat_ms), "wall_s": wall}


class _NoGC:
    """Python's cyclic garbage collector paused over a timed trace (collected
    just before), as a serving process tunes it: a full collection over the
    trace's thousands of request objects stalls the scheduler for milliseconds."""

    def __enter__(self):
        import gc

        gc.collect()
        self._was = gc.isenabled()
        gc.disable()
        return self

    def __exit__(self, *exc):
        import gc

        if self._was:
            gc.enable()
        return False


def bench_served(n: int = 128, dtype=None, log=print, sizes=None, weights=None, count: int = 2000,
                 budget_frac: float = 0.8, max_inflight: int = 64, small_budget: int = 2 << 30,
                 plain_dtype=None):
    """Served-path measurement on two request streams, the n^3 stream and the
    mixed-size stream of ``sizes`` (weights ``weights``, seed 4), each request
    with its own Gaussian-blob source:

    * closed-loop saturation (every request present at t = 0);
    * Poisson arrivals at 0.7 x saturation: solves/s and p50/p99 arrival-to-
      completion latency;
    * the same arrivals under a forced small memory budget (``small_budget``
      bytes), so that admission defers requests;
    * the same arrivals through the plain path in ``plain_dtype`` (FP64), one
      ``pspfft_solve`` after another;
    * the potential of one request per size against the FP64 GPU solve.

    64 requests in flight keep about 20 per pass launch (three passes per fused
    plan); measured, 32 gives 4 % (single size) and 10 % (config-4 mix) less, 96
    no more."""
    import torch

    from . import sources

    dtype = dtype or torch.float32
    plain_dtype = plain_dtype or torch.float64
    results = {}
    streams = {"single": ((n,), (1.0,)),
               "mix": (tuple(sizes or sources.CONFIG4_SIZES), tuple(weights or sources.CONFIG4_WEIGHTS))}
    for name, (szs, wts) in streams.items():
        # sizes, blobs and unit-rate gaps: scaling the gaps by 1 / rate gives the
        # Poisson arrivals at that rate (same draws)
        trace = sources.config4_trace(rate_hz=1.0, count=count, sizes=szs, weights=wts)
        srcs = trace_sources(trace, dtype)
        torch.cuda.synchronize()
        free, _ = torch.cuda.mem_get_info()
        budget = int(budget_frac * free)
        ex = GpuExecutor(dtype=dtype)

        def make(scale, idx=None):
            idx = range(len(trace)) if idx is None else idx
            return [Request(i, (trace[i].n,) * 3, (1.0 / trace[i].n,) * 3, srcs[i], arrival=trace[i].arrival * scale)
                    for i in idx]

        # warm plans, kernels and the workspace pool (a server does this at start-up)
        first = {}
        for i, r in enumerate(trace):
            first.setdefault(r.n, i)
        warm = Server(ex, budget, max_inflight=max_inflight)
        warm.run_trace(make(0.0, [first[s] for _ in range(4 * max_inflight // len(szs) + 1) for s in szs]),
                       realtime=False)
        ex.synchronize()
        # closed loop: all requests present at t = 0
        srv = Server(ex, budget, max_inflight=max_inflight)
        reqs = make(0.0)  # the clients' side, before the clock starts
        with _NoGC():
            t0 = time.perf_counter()
            fin = srv.run_trace(reqs, realtime=False)
            ex.synchronize()
            wall = time.perf_counter() - t0
        sat = summarize(fin, wall)
        # accuracy: the first request of each size against the FP64 GPU solve
        import paper_1106_0557_amd as ps

        acc = {}
        for s, i in sorted(first.items()):
            r = next(q for q in fin if q.index == i)
            p64 = ps.Plan(s, s, s, h=1.0 / s, dtype=torch.float64)
            ref = p64.solve(srcs[i].to(torch.float64))
            d = r.phi.double() - ref
            acc[str(s)] = {"rel_l2_vs_gpu_fp64": float(d.norm() / ref.norm()),
                           "rel_max_vs_gpu_fp64": float(d.abs().max() / ref.abs().max())}
            p64.close()
            del ref, d
        del fin, reqs
        log(f"[serve] {name}: saturation {sat['solves_per_s']:.0f} solves/s, {srv.launches} launches, "
            f"max batch {srv.max_batch}")
        # open loop: Poisson arrivals at 0.7 x saturation
        rate = 0.7 * sat["solves_per_s"]
        srv = Server(ex, budget, max_inflight=max_inflight)
        reqs = make(1.0 / rate)
        with _NoGC():
            t0 = time.perf_counter()
            fin = srv.run_trace(reqs, realtime=True)
            ex.synchronize()
            op = summarize(fin, time.perf_counter() - t0)
        del fin, reqs
        log(f"[serve] {name}: Poisson {rate:.0f}/s: p50 {op['latency_ms_p50']:.3f} ms, "
            f"p99 {op['latency_ms_p99']:.3f} ms")
        # the same arrivals under a small memory budget (idle pooled workspaces
        # beyond it are released first)
        ex.trim_pool()
        torch.cuda.synchronize()
        srv = Server(ex, small_budget, max_inflight=max_inflight)
        reqs = make(1.0 / rate)
        with _NoGC():
            t0 = time.perf_counter()
            fin = srv.run_trace(reqs, realtime=True)
            ex.synchronize()
            small = summarize(fin, time.perf_counter() - t0)
        small.update({"budget_bytes": small_budget, "max_used_bytes": srv.max_used})
        del fin, reqs
        log(f"[serve] {name}: budget {small_budget >> 20} MiB: {small['solves_per_s']:.0f} solves/s, "
            f"p50 {small['latency_ms_p50']:.3f} ms, p99 {small['latency_ms_p99']:.3f} ms, "
            f"max used {srv.max_used >> 20} MiB")
        for lst in ex.pool.values():
            for ws in lst:
                ws.close()
        ex.pool.clear()
        for p in ex.plans.values():
            p.close()
        ex.plans.clear()
        # the plain path (FP64, one solve after another) under the same arrivals
        srcs64 = [S.to(plain_dtype) for S in srcs]
        del srcs
        torch.cuda.synchronize()
        arrivals = [(r.n, r.arrival / rate) for r in trace]
        with _NoGC():
            plain = replay_plain(arrivals, srcs64, dtype=plain_dtype, realtime=True)
        log(f"[serve] {name}: plain {str(plain_dtype).split('.')[-1]} at {rate:.0f}/s: "
            f"{plain['solves_per_s']:.0f} solves/s, p50 {plain['latency_ms_p50']:.3f} ms, "
            f"p99 {plain['latency_ms_p99']:.3f} ms")
        del srcs64
        torch.cuda.empty_cache()
        results[name] = {"sizes": list(szs), "weights": list(wts), "requests": count,
                         "sources": "each request's own 8 Gaussian blobs (seed 4 trace)",
                         "saturation": sat, "poisson_rate_hz": rate, "poisson": op,
                         "small_budget": small, "plain_fp64_same_arrivals": plain,
                         "accuracy_first_of_each_size": acc, "budget_bytes": budget,
                         "max_inflight": max_inflight}
    return results
