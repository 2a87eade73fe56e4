"""Parity at the mesh sizes of the served mix {64, 96, 128, 192, 256}^3 (Gaussian-blob
sources), element by element against the FP64 oracle (Sec. 2.1, Eq. (greens_function)
defines the result).

* cheap meshes that reach each line instance those sizes use: x rows of 144
  (36*4), 192 (24*8) and 256 (16*16), y lines of 512 points (16*16*2);
* the whole 192^3 and 256^3 meshes in both precisions;
* the serving loop on a trace of those sizes, each request's own source: every
  result equals, bit for bit, the same request solved alone, and one request of
  each size matches the oracle.

Bars: FP64 <= 1e-12 relative L2 and relative max; FP32 <= 1e-5 relative L2.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import norms
from paper_1106_0557_amd import sources

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5


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


def gpu_solve(n, h, S, dtype):
    from paper_1106_0557_amd import Plan

    plan = Plan(*n, h=h, dtype=dtype)
    phi = plan.solve(torch.as_tensor(S).to("cuda", dtype))
    torch.cuda.synchronize()
    out = phi.double().cpu().numpy()
    plan.close()
    return out


def check_both(n, h, S, ref):
    got64 = gpu_solve(n, h, S, torch.float64)
    got32 = gpu_solve(n, h, S, torch.float32)
    r64, r32 = norms.report(got64, ref), norms.report(got32, ref)
    say(f"  fp64 {r64}\n  fp32 {r32}")
    assert r64["rel_l2"] <= FP64_TOL and r64["rel_max"] <= FP64_TOL
    assert r32["rel_l2"] <= FP32_TOL


# x rows of 144, 192, 256; y lines of 512 points; z lines of 384 and 512 beside them
@pytest.mark.parametrize("n", [(144, 8, 8), (192, 8, 8), (256, 8, 8), (16, 256, 8), (192, 16, 192),
                               (256, 16, 256)])
def test_config4_line_instances_match_oracle(n):
    say(f"[config4 lines] n={n}")
    h = (0.011, 0.013, 0.017)
    S = sources.random_field(n, seed=sum(n) + 11).numpy()
    check_both(n, h, S, oracle.solve_fft(S, h))


def _first_of_size(size):
    for r in sources.config4_trace(rate_hz=0, count=200):
        if r.n == size:
            return r
    raise AssertionError(f"no request of size {size}")


@pytest.mark.parametrize("size", [192, 256])
def test_config4_whole_mesh_matches_oracle(size):
    """The whole 192^3 / 256^3 mesh (384^3 / 512^3 padded) with the trace's first
    Gaussian-blob source of that size."""
    say(f"[config4 mesh] n={size}")
    r = _first_of_size(size)
    S = sources.blob_field(size, r.blobs).numpy()
    h = (1.0 / size,) * 3
    check_both((size,) * 3, h, S, oracle.solve_fft(S, h))


def test_config4_served_trace_matches_alone_and_oracle():
    """The first 40 requests of the served trace (sizes {64, 96, 128, 192, 256},
    weights 0.3/0.25/0.2/0.15/0.1, seed 4), each with its own blobs, through the
    serving loop with 12 in flight."""
    from paper_1106_0557_amd.serve import GpuExecutor, Request, Server

    trace = sources.config4_trace(rate_hz=0, count=40)
    say(f"[config4 served] sizes {sorted(set(r.n for r in trace))}")
    reqs = [Request(r.index, (r.n,) * 3, (1.0 / r.n,) * 3,
                    sources.blob_field(r.n, r.blobs, device="cuda").to(torch.float32))
            for r in trace]
    ex = GpuExecutor(dtype=torch.float32)
    srv = Server(ex, budget_bytes=1 << 36, max_inflight=12)
    fin = srv.run_trace(reqs, realtime=False)
    ex.synchronize()
    assert len(fin) == len(reqs) and all(r.done and not r.rejected for r in fin)
    checked = set()
    for r in sorted(fin, key=lambda q: q.index):
        alone = ex.plans[ex.key(r)].solve(r.S)
        torch.cuda.synchronize()
        assert torch.equal(alone, r.phi), f"request {r.index} (n={r.n[0]}) differs in the mix"
        if r.n[0] not in checked:
            checked.add(r.n[0])
            ref = oracle.solve_fft(r.S.double().cpu().numpy(), r.h)
            rep = norms.report(r.phi.double().cpu().numpy(), ref)
            say(f"  request {r.index} n={r.n[0]}: {rep}")
            assert rep["rel_l2"] <= FP32_TOL
    assert checked == {64, 96, 128, 192, 256}
    for lst in ex.pool.values():
        for ws in lst:
            ws.close()
    for p in ex.plans.values():
        p.close()
