"""pspfft_solve_noalloc (the allocation-free solve, workspace in the library's
static device array) against pspfft_solve_ws (the same solve on a caller
workspace), through the C ABI: bit-identical potentials on two calls in a row,
the second on a smaller mesh, in both precisions, and both within the oracle's
bar; a mesh whose workspace exceeds the array is refused.
"""
import ctypes
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
    yield


def _noalloc(lib, plan, S, out):
    stream = torch.cuda.current_stream().cuda_stream
    return lib.pspfft_solve_noalloc(plan.handle, S.data_ptr(), out.data_ptr(), stream)


@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-5), (torch.float64, 1e-12)])
def test_noalloc_matches_workspace_solve_on_two_calls(dtype, tol):
    import paper_1106_0557_amd as ps
    from paper_1106_0557_amd import _lib

    lib = _lib.load()
    # a fused 128^3 plan, then a smaller five-pass mesh with a generic axis
    for k, n in enumerate(((128, 128, 128), (48, 40, 30))):
        say(f"[noalloc] call {k}: n={n} {dtype}")
        h = tuple(1.0 / v for v in n)
        plan = ps.Plan(*n, h=h, dtype=dtype)
        assert plan.workspace_bytes <= _lib.NOALLOC_MAX_BYTES
        S = sources.random_field(n, seed=31 + k).to("cuda", dtype)
        want = plan.workspace().solve(S)  # pspfft_solve_ws on an allocated workspace
        got = torch.full_like(S, float("nan"))
        _lib.check(_noalloc(lib, plan, S, got), "pspfft_solve_noalloc")
        torch.cuda.synchronize()
        assert torch.equal(got, want), f"call {k}: noalloc differs from the workspace solve"
        ref = oracle.solve_fft(S.double().cpu().numpy(), h)
        err = norms.rel_l2(got.double().cpu().numpy(), ref)
        say(f"  rel l2 vs oracle {err:.3e}")
        assert err <= tol
        plan.close()


def test_noalloc_refuses_meshes_beyond_its_array():
    import paper_1106_0557_amd as ps
    from paper_1106_0557_amd import _lib

    lib = _lib.load()
    n = (256, 256, 256)
    plan = ps.Plan(*n, h=1 / 256, dtype=torch.float32)
    assert plan.workspace_bytes > _lib.NOALLOC_MAX_BYTES
    S = torch.zeros(n[::-1], dtype=torch.float32, device="cuda")
    assert _noalloc(lib, plan, S, S) == 2  # PSPFFT_ERR_UNSUPPORTED_SIZE, nothing enqueued
    assert lib.pspfft_solve_noalloc(None, None, None, None) == 1
    plan.close()


def test_noalloc_solve_replays_from_a_captured_graph():
    """The use the allocation-free solve is for: captured once into a HIP graph
    (after one eager call, which looks up the array's address and sets kernel
    attributes), then replayed on new sources written between the replays; every
    replay equals the eager workspace solve of the same source, bit for bit."""
    import paper_1106_0557_amd as ps
    from paper_1106_0557_amd import _lib

    lib = _lib.load()
    n = (64, 64, 48)
    h = tuple(1.0 / v for v in n)
    plan = ps.Plan(*n, h=h, dtype=torch.float32)
    S = sources.random_field(n, seed=90).to("cuda", torch.float32)
    out = torch.empty_like(S)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        _lib.check(_noalloc(lib, plan, S, out), "pspfft_solve_noalloc")  # eager first call
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        _lib.check(_noalloc(lib, plan, S, out), "pspfft_solve_noalloc (captured)")
    ws = plan.workspace()
    for k in range(3):
        S.copy_(sources.random_field(n, seed=91 + k).to("cuda", torch.float32))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        want = ws.solve(S)
        torch.cuda.synchronize()
        say(f"[noalloc graph] replay {k}")
        assert torch.equal(out, want), f"replay {k} differs from the eager solve"
    ref = oracle.solve_fft(S.double().cpu().numpy(), h)
    assert norms.rel_l2(out.double().cpu().numpy(), ref) <= 1e-5
    del g
    ws.close()
    plan.close()
