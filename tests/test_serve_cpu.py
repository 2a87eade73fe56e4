"""Serving scheduler logic on the CPU, driven by a test double executor.

The fake executor records every pass issued to every request and completes a
step's token after a fixed number of polls; at the last pass it computes the
potential with the FP64 oracle, so the whole request path is exercised without
a GPU.  This double exists only in the tests; the product scheduler always runs
on the HIP library.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import norms
from paper_1106_0557_amd import sources
from paper_1106_0557_amd.serve import NUM_PASSES, Request, Server, summarize


class FakeToken:
    def __init__(self, polls):
        self.left = polls

    def query(self):
        self.left -= 1
        return self.left < 0


class FakeExecutor:
    def __init__(self, polls=2, compute=False, fused_sizes=()):
        self.polls = polls
        self.compute = compute
        self.fused_sizes = set(fused_sizes)  # meshes whose plans skip the y passes
        self.pool = {}
        self.log = []          # (step, pass, request index)
        self.events = []       # ("admit" | "pass", request index), in call order
        self.step_no = 0
        self.created = 0
        self.plans = set()     # meshes with a resident plan
        self.admissions = 0    # calls of admitted(): one per scheduler step that admits

    def plan_bytes(self, req):
        nx, ny, nz = req.n
        return 32 * (nx + 1) * (ny + 1) * (nz + 1)

    def has_plan(self, req):
        return self.key(req) in self.plans

    def resident_bytes(self):
        return sum(32 * (n[0] + 1) * (n[1] + 1) * (n[2] + 1) for (n, _) in self.plans)

    def admitted(self, reqs):
        self.admissions += 1
        for r in reqs:
            self.events.append(("admit", r.index))

    def workspace_bytes(self, req):
        nx, ny, nz = req.n
        return 2 * ny * nz * (nx + 1) * 8

    def output_bytes(self, req):
        nx, ny, nz = req.n
        return nx * ny * nz * 4

    def key(self, req):
        return (req.n, req.h)

    def active_passes(self, req):
        return (0, 2, 4) if req.n[0] in self.fused_sizes else tuple(range(NUM_PASSES))

    def has_pooled(self, req):
        return bool(self.pool.get(self.key(req)))

    def pooled_bytes(self):
        return sum(b for lst in self.pool.values() for (_, b) in lst)

    def acquire(self, req):
        self.plans.add(self.key(req))
        lst = self.pool.get(self.key(req))
        if lst:
            return lst.pop()
        self.created += 1
        return (self.created, self.workspace_bytes(req))

    def release(self, req, ws):
        self.pool.setdefault(self.key(req), []).append(ws)

    def trim_pool(self):
        freed = self.pooled_bytes()
        self.pool.clear()
        return freed

    def alloc_output(self, req):
        return None

    def begin_step(self):
        self.step_no += 1

    def run_pass(self, p, reqs):
        for r in reqs:
            self.log.append((self.step_no, p, r.index))
            self.events.append(("pass", r.index))
            if p == NUM_PASSES - 1 and self.compute:
                r.phi = oracle.solve_fft(r.S, r.h)

    def end_step(self):
        return FakeToken(self.polls)

    @staticmethod
    def is_done(token):
        return token.query()

    @staticmethod
    def wait(token):
        while not token.query():
            pass


def _reqs(sizes, arrivals=None):
    arrivals = arrivals or [0.0] * len(sizes)
    return [Request(i, (n, n, n), (1.0 / n,) * 3, None, arrival=a) for i, (n, a) in enumerate(zip(sizes, arrivals))]


def test_every_request_gets_each_pass_once_in_order():
    ex = FakeExecutor()
    srv = Server(ex, budget_bytes=1 << 40, max_inflight=7)
    sizes = [16, 24, 32, 16, 48, 24, 32, 16, 16, 24, 64, 32]
    fin = srv.run_trace(_reqs(sizes), realtime=False)
    assert len(fin) == len(sizes) and all(r.done and not r.rejected for r in fin)
    for i in range(len(sizes)):
        seq = [(s, p) for (s, p, r) in ex.log if r == i]
        assert [p for _, p in seq] == list(range(NUM_PASSES))
        steps = [s for s, _ in seq]
        assert steps == sorted(steps) and len(set(steps)) == NUM_PASSES  # one pass per step


def test_fused_requests_skip_the_y_passes_beside_five_pass_ones():
    ex = FakeExecutor(fused_sizes=(16, 32))
    srv = Server(ex, budget_bytes=1 << 40, max_inflight=5)
    sizes = [16, 24, 32, 48, 16, 24, 32, 16, 48, 24]
    fin = srv.run_trace(_reqs(sizes), realtime=False)
    assert len(fin) == len(sizes) and all(r.done and not r.rejected for r in fin)
    for i, n in enumerate(sizes):
        seq = [(s, p) for (s, p, r) in ex.log if r == i]
        want = [0, 2, 4] if n in (16, 32) else [0, 1, 2, 3, 4]
        assert [p for _, p in seq] == want, (i, n, seq)
        steps = [s for s, _ in seq]
        assert steps == list(range(steps[0], steps[0] + len(want)))  # one pass per step, no gaps
    # steps mix fused and five-pass requests at the same pass
    by_step = {}
    for s, p, r in ex.log:
        by_step.setdefault((s, p), set()).add(sizes[r] in (16, 32))
    assert any(len(v) == 2 for v in by_step.values())


def test_admission_respects_budget_and_slots():
    ex = FakeExecutor()
    r32 = _reqs([32])[0]
    one = ex.workspace_bytes(r32) + ex.output_bytes(r32)
    srv = Server(ex, budget_bytes=3 * one + ex.plan_bytes(r32) + 10, max_inflight=8)
    fin = srv.run_trace(_reqs([32] * 10), realtime=False)
    assert all(r.done for r in fin)
    assert srv.max_used <= srv.budget
    # never more than 3 requests of this size in flight at once
    by_step = {}
    for s, p, r in ex.log:
        by_step.setdefault(s, set()).add(r)
    assert max(len(v) for v in by_step.values()) <= 3
    # slot limit
    ex2 = FakeExecutor()
    srv2 = Server(ex2, budget_bytes=1 << 40, max_inflight=2)
    srv2.run_trace(_reqs([16] * 6), realtime=False)
    by_step = {}
    for s, p, r in ex2.log:
        by_step.setdefault(s, set()).add(r)
    assert max(len(v) for v in by_step.values()) <= 2


def test_oversized_request_is_rejected_not_deadlocked():
    ex = FakeExecutor()
    small = _reqs([16])[0]
    budget = ex.workspace_bytes(small) + ex.output_bytes(small) + ex.plan_bytes(small)
    srv = Server(ex, budget_bytes=budget, max_inflight=4)
    fin = srv.run_trace(_reqs([16, 64, 16]), realtime=False)
    rej = [r for r in fin if r.rejected]
    assert [r.index for r in rej] == [1] and rej[0].error
    assert sum(not r.rejected for r in fin) == 2


def test_requests_join_while_others_are_in_flight():
    """Continuous batching: a late arrival starts before earlier requests finish."""
    ex = FakeExecutor(polls=0)
    clock = itertools.count()
    srv = Server(ex, budget_bytes=1 << 40, max_inflight=8, clock=lambda: next(clock) * 1e-3)
    reqs = _reqs([16, 16, 16], arrivals=[0.0, 0.0, 0.004])
    srv.run_trace(reqs, realtime=True)
    first_pass_late = min(s for s, p, r in ex.log if r == 2)
    last_pass_early = max(s for s, p, r in ex.log if r == 0)
    assert first_pass_late <= last_pass_early
    # and in that step the batch mixes requests at different passes
    mixed = [s for s in set(x[0] for x in ex.log) if len({p for (t, p, _) in ex.log if t == s}) > 1]
    assert mixed


class SizedExecutor(FakeExecutor):
    """A step's token takes more polls when the step holds a large mesh."""

    def __init__(self, slow_polls=40, **kw):
        super().__init__(**kw)
        self.slow_polls = slow_polls
        self._big = False

    def begin_step(self):
        super().begin_step()
        self._big = False

    def run_pass(self, p, reqs):
        super().run_pass(p, reqs)
        self._big |= any(r.n[0] >= 64 for r in reqs)

    def end_step(self):
        return FakeToken(self.slow_polls if self._big else 0)


def test_steps_retire_in_the_order_they_finish():
    """A step of small meshes that finishes retires before an earlier step that
    holds a large mesh's pass (the executor orders launches per request, not per
    step), and launches group requests by pass and mesh size."""
    ex = SizedExecutor(fused_sizes=(16,))
    clock = itertools.count()
    srv = Server(ex, budget_bytes=1 << 40, max_inflight=2, clock=lambda: next(clock) * 1e-3)
    reqs = _reqs([64, 16, 16, 16, 16])
    fin = srv.run_trace(reqs, realtime=False)
    assert all(r.done and not r.rejected for r in fin)
    big = reqs[0]
    done_step = {i: max(s for s, _, r in ex.log if r == i) for i in range(len(reqs))}
    later_small = [r for r in reqs[1:] if done_step[r.index] > done_step[0]]
    assert later_small, "a small request completes in a step after the large one's last"
    assert any(r.t_done < big.t_done for r in later_small)
    # one launch per (pass, size): a step's log holds each request once
    for s in set(x[0] for x in ex.log):
        rs = [r for t, _, r in ex.log if t == s]
        assert len(rs) == len(set(rs))


def test_pool_reuse_and_trim():
    ex = FakeExecutor()
    srv = Server(ex, budget_bytes=1 << 40, max_inflight=2, max_steps_ahead=2)
    srv.run_trace(_reqs([16] * 6), realtime=False)
    # two slots; a finished request keeps its workspace until its step's token
    # completes, so at most slots x (1 + steps ahead) exist, and they are reused
    assert ex.created <= 2 * (1 + srv.max_steps_ahead) and ex.created < 6
    # a budget that only fits after idle workspaces of another size are released
    r64 = _reqs([64])[0]
    budget = ex.workspace_bytes(r64) + ex.output_bytes(r64) + ex.plan_bytes(r64) + ex.resident_bytes() + 1
    srv2 = Server(ex, budget_bytes=budget, max_inflight=2)
    assert srv2.used == ex.pooled_bytes() + ex.resident_bytes() and ex.pooled_bytes() > 0
    fin = srv2.run_trace([Request(9, (64, 64, 64), (1 / 64,) * 3, None)], realtime=False)
    assert fin[0].done and not fin[0].rejected


def test_results_through_the_scheduler_match_the_oracle():
    ex = FakeExecutor(compute=True)
    srv = Server(ex, budget_bytes=1 << 40, max_inflight=3)
    reqs = []
    for i, n in enumerate([16, 24, 16, 20]):
        S = sources.random_field(n, seed=i).numpy()
        reqs.append(Request(i, (n, n, n), (1.0 / n,) * 3, S))
    fin = srv.run_trace(reqs, realtime=False)
    for r in fin:
        want = oracle.direct(r.S, r.h) if r.n[0] <= 16 else oracle.solve_fft(r.S, r.h)
        assert norms.rel_l2(r.phi, want) < 1e-12
    s = summarize(fin, 1.0)
    assert s["served"] == 4 and s["rejected"] == 0 and np.isfinite(s["latency_ms_p99"])


def test_plan_bytes_count_in_the_budget():
    """A plan (spectrum and twiddles) is resident from its first request on and
    takes budget like any other device memory."""
    ex = FakeExecutor()
    r = _reqs([32])[0]
    one = ex.workspace_bytes(r) + ex.output_bytes(r)
    P = ex.plan_bytes(r)
    assert P > one  # so that the test tells the two accountings apart
    # room for the plan and two requests: never three in flight
    srv = Server(ex, budget_bytes=P + 2 * one + 10, max_inflight=8)
    fin = srv.run_trace(_reqs([32] * 8), realtime=False)
    assert all(r.done and not r.rejected for r in fin)
    assert srv.max_used <= srv.budget and srv.max_used >= P + one
    by_step = {}
    for st, p, i in ex.log:
        by_step.setdefault(st, set()).add(i)
    assert max(len(v) for v in by_step.values()) == 2
    # a request whose plan alone would overflow the budget is rejected up front
    ex2 = FakeExecutor()
    srv2 = Server(ex2, budget_bytes=one + P - 1, max_inflight=8)
    fin2 = srv2.run_trace(_reqs([32]), realtime=False)
    assert fin2[0].rejected and not ex2.plans
    # a server starting on an executor that already holds plans counts them
    srv3 = Server(ex, budget_bytes=1 << 40)
    assert srv3.used == ex.resident_bytes() + ex.pooled_bytes() >= P


def test_each_request_is_marked_at_admission_before_its_first_pass():
    """The executor marks the caller's stream when a request is admitted (its
    source, workspace and output are ready there); the first pass comes after."""
    ex = FakeExecutor(fused_sizes=(16,))
    srv = Server(ex, budget_bytes=1 << 40, max_inflight=3)
    fin = srv.run_trace(_reqs([16, 24, 16, 32, 16, 24]), realtime=False)
    assert all(r.done for r in fin)
    for i in range(6):
        seq = [k for k, (what, r) in enumerate(ex.events) if r == i]
        kinds = [ex.events[k][0] for k in seq]
        assert kinds[0] == "admit" and kinds.count("admit") == 1 and "pass" in kinds[1:]
    # one mark per admitting step, not per request (3 admitted at once at the start)
    assert ex.admissions < 6
