"""Grouped (batched) launches and the serving loop on the GPU.

* config 3 layout: 64 Gaussian-blob sources with n drawn from {32,48,64,96,128},
  solved in grouped launches; every result is bit-identical to the same source
  solved alone, and matches the FP64 oracle within the FP32 bar.
* the serving loop: requests of mixed sizes admitted as slots and memory free
  up give, bit for bit, the result of solving each alone; a small memory budget
  still serves everything without exceeding it.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import norms
from paper_1106_0557_amd import sources

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_1106_0557_amd import _lib

    _lib.load()
    yield


def test_config3_grouped_launches_match_single_solves_and_oracle():
    import paper_1106_0557_amd as ps

    say("[config3] 64 sources, grouped launches")
    batch = sources.config3(device="cuda")
    plans = {}
    ws, S, P = [], [], []
    for n, src in batch:
        if n not in plans:
            plans[n] = ps.Plan(n, n, n, h=1.0 / n, dtype=torch.float32)
        ws.append(plans[n].workspace())
        S.append(src.to(torch.float32).contiguous())
        P.append(torch.empty_like(S[-1]))
    ps.solve_batched(ws, S, P)
    torch.cuda.synchronize()
    checked = set()
    for i, (n, src) in enumerate(batch):
        alone = plans[n].solve(S[i])
        torch.cuda.synchronize()
        assert torch.equal(alone, P[i]), f"problem {i} (n={n}) differs between batch and single solve"
        if n not in checked or i % 16 == 0:  # oracle check on each size and a few more
            checked.add(n)
            ref = oracle.solve_fft(src.cpu().numpy(), 1.0 / n)
            r = norms.report(P[i].double().cpu().numpy(), ref)
            say(f"  problem {i} n={n}: {r}")
            assert r["rel_l2"] <= 1e-5
    for w in ws:
        w.close()
    for p in plans.values():
        p.close()


def test_mixed_precision_batch_matches_single():
    import paper_1106_0557_amd as ps

    say("[mixed precision batch]")
    # (16, 8, 512): spectrum kz-fastest, z lines by wavefront
    cases = [((32, 24, 16), torch.float32), ((32, 24, 16), torch.float64), ((48, 48, 48), torch.float64),
             ((16, 36, 20), torch.float32), ((16, 8, 512), torch.float32), ((16, 8, 512), torch.float64),
             ((16, 8, 256), torch.float32)]
    ws, S, P, plans = [], [], [], []
    for k, (n, dt) in enumerate(cases):
        pl = ps.Plan(*n, h=(0.1, 0.2, 0.3), dtype=dt)
        plans.append(pl)
        ws.append(pl.workspace())
        S.append(sources.random_field(n, seed=k).to("cuda", dt))
        P.append(torch.empty_like(S[-1]))
    ps.solve_batched(ws, S, P)
    torch.cuda.synchronize()
    for k, (n, dt) in enumerate(cases):
        alone = plans[k].solve(S[k])
        torch.cuda.synchronize()
        assert torch.equal(alone, P[k])
        ref = oracle.solve_fft(S[k].double().cpu().numpy(), (0.1, 0.2, 0.3))
        tol = 1e-12 if dt == torch.float64 else 1e-5
        assert norms.rel_l2(P[k].double().cpu().numpy(), ref) <= tol


def _serve(reqs, budget, max_inflight):
    from paper_1106_0557_amd.serve import GpuExecutor, Server

    ex = GpuExecutor(dtype=torch.float32)
    srv = Server(ex, budget_bytes=budget, max_inflight=max_inflight)
    fin = srv.run_trace(reqs, realtime=False)
    ex.synchronize()
    return ex, srv, fin


def test_served_results_equal_alone_in_the_mix():
    import paper_1106_0557_amd as ps
    from paper_1106_0557_amd.serve import Request

    say("[serve] mixed sizes (fused and five-pass plans), results alone vs in the mix")
    rng = np.random.default_rng(41)
    sizes = [int(rng.choice([32, 48, 64, 96, 144])) for _ in range(40)]
    reqs = []
    for i, n in enumerate(sizes):
        S = sources.blob_field(n, sources.draw_blobs(rng, 8), device="cuda").to(torch.float32)
        reqs.append(Request(i, (n, n, n), (1.0 / n,) * 3, S))
    ex, srv, fin = _serve(reqs, budget=1 << 34, max_inflight=7)
    assert len(fin) == len(reqs) and all(r.done and not r.rejected for r in fin)
    fused = {n: ex.plans[ex.key(r)].fused for r in fin for n in [r.n[0]]}
    say(f"  fused plans by size: {fused}")
    assert fused[144] is False and fused[64] is True
    say(f"  {srv.launches} launches, max group {srv.max_batch}")
    for r in fin:
        alone = ex.plans[ex.key(r)].solve(r.S)
        torch.cuda.synchronize()
        assert torch.equal(alone, r.phi), f"request {r.index} (n={r.n[0]}) differs in the mix"
    r = fin[3]
    ref = oracle.solve_fft(r.S.double().cpu().numpy(), r.h)
    assert norms.rel_l2(r.phi.double().cpu().numpy(), ref) <= 1e-5


def test_served_small_budget_defers_but_serves_all():
    from paper_1106_0557_amd.serve import Request

    say("[serve] small memory budget")
    import paper_1106_0557_amd as ps

    n = 64
    one = ps.workspace_bytes(n, n, n, torch.float32) + n**3 * 4
    reqs = [Request(i, (n, n, n), (1.0 / n,) * 3, sources.random_field(n, seed=i).to("cuda", torch.float32))
            for i in range(12)]
    big = Request(99, (128, 128, 128), (1 / 128,) * 3, torch.zeros((128, 128, 128), device="cuda"))
    ex, srv, fin = _serve(reqs + [big], budget=2 * one + 1024, max_inflight=8)
    assert srv.max_used <= srv.budget
    assert [r.index for r in fin if r.rejected] == [99]
    served = [r for r in fin if not r.rejected]
    assert len(served) == 12
    for r in served[:3]:
        ref = oracle.solve_fft(r.S.double().cpu().numpy(), r.h)
        assert norms.rel_l2(r.phi.double().cpu().numpy(), ref) <= 1e-5


def test_warm_server_waits_for_a_source_produced_just_before_submit():
    """A server whose plans, workspaces and streams are warm takes a source that
    the caller's stream is still producing (a long chain of kernels queued just
    before submit): the first pass must wait for it."""
    from paper_1106_0557_amd.serve import GpuExecutor, Request, Server

    say("[serve] fresh source into a warm server")
    n = 64
    ex = GpuExecutor(dtype=torch.float32)
    warm = [Request(i, (n, n, n), (1.0 / n,) * 3, torch.zeros((n, n, n), device="cuda")) for i in range(4)]
    Server(ex, budget_bytes=1 << 34, max_inflight=4).run_trace(warm, realtime=False)
    ex.synchronize()
    base = sources.random_field(n, seed=77).to("cuda", torch.float32)
    reqs = []
    for i in range(3):
        S = torch.zeros_like(base)
        # queue enough work on the current stream that the source is still being
        # written when the request's first pass could start
        big = torch.randn(2048, 2048, device="cuda")
        for _ in range(20):
            big = big @ big
            big = big / big.norm()
        S += base * (i + 1) + 0.0 * big[0, 0]
        reqs.append(Request(i, (n, n, n), (1.0 / n,) * 3, S))
    fin = Server(ex, budget_bytes=1 << 34, max_inflight=4).run_trace(reqs, realtime=False)
    ex.synchronize()
    ref = oracle.solve_fft(base.double().cpu().numpy(), 1.0 / n)
    for r in sorted(fin, key=lambda q: q.index):
        got = r.phi.double().cpu().numpy() / (r.index + 1)
        assert norms.rel_l2(got, ref) <= 1e-5, f"request {r.index} read its source before it was written"


def test_plan_bytes_before_and_after_the_first_solve():
    """pspfft_plan_resident_bytes tells the plan's bytes before it exists; the
    default workspace is allocated by the first pspfft_solve and counted then."""
    import paper_1106_0557_amd as ps

    for n, dt in (((64, 64, 64), torch.float32), ((60, 48, 30), torch.float64), ((16, 8, 512), torch.float32)):
        want = ps.plan_resident_bytes(*n, dt)
        p = ps.Plan(*n, h=0.1, dtype=dt)
        assert p.resident_bytes == want
        p.solve(torch.zeros(n[::-1], dtype=dt, device="cuda"))
        torch.cuda.synchronize()
        assert p.resident_bytes == want + p.workspace_bytes
        p.close()


def test_batch_of_several_plans_keeps_the_callers_stream_order():
    """A batch of several plans runs its groups on the library's own streams; it
    must still start after the caller's earlier work on the stream (sources
    written by a long chain of kernels just before the call) and end before the
    caller's later work (copies of the potentials queued just after it)."""
    import paper_1106_0557_amd as ps

    say("[batch fork] stream order")
    meshes = [(32, 32, 32), (48, 48, 48), (24, 20, 16), (64, 64, 64), (60, 30, 15)]
    plans = [ps.Plan(*n, h=(0.1, 0.2, 0.3), dtype=torch.float32) for n in meshes]
    ws = [p.workspace() for p in plans]
    base = [sources.random_field(n, seed=200 + k).to("cuda", torch.float32) for k, n in enumerate(meshes)]
    torch.cuda.synchronize()
    big = torch.randn(2048, 2048, device="cuda")
    for _ in range(20):
        big = big @ big
        big = big / big.norm()
    S = [b + 0.0 * big[0, 0] for b in base]  # written only after the chain
    P = [torch.empty_like(s) for s in S]
    ps.solve_batched(ws, S, P)
    copies = [p.clone() for p in P]  # queued right after the batch on the same stream
    torch.cuda.synchronize()
    for k, n in enumerate(meshes):
        alone = plans[k].solve(base[k])
        torch.cuda.synchronize()
        assert torch.equal(copies[k], alone), f"problem {k} {n}: batch not ordered with the caller's stream"
    for w in ws:
        w.close()
    for p in plans:
        p.close()
