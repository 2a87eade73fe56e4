"""Fused x-y plane kernels (nx == ny, plane in LDS) against the FP64 oracle.

* every fusable size in both precisions: the fused plan's potential matches the
  oracle (FP64 <= 1e-12, FP32 <= 1e-5 relative L2) and the five-pass plan of
  the same mesh to the same bar;
* the workspace after the fused forward pass equals the oracle's x-then-y
  transform on all 2ny rows (including the Nyquist column split off from the
  packed kx = 0 column), the y passes leave it untouched, and the fused inverse
  gives the oracle's potential;
* fused and five-pass problems share grouped launches with results bit-identical
  to solving alone, in place (S == Phi) included;
* a batch whose workspaces pass the streaming threshold (nontemporal line
  accesses in the z pass and the inverse plane pass) gives the bits of the
  same problems solved alone, which stream nothing.
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

# n = E*K with at most two stages; FP64 keeps n*K <= 256
FUSED_FP32 = [16, 20, 24, 32, 36, 40, 48, 64, 72, 80, 96, 128]
FUSED_FP64 = [16, 20, 24, 32, 36, 40, 48, 64, 72]
NOT_FUSED = [((144, 144, 16), torch.float32), ((256, 256, 8), torch.float32), ((80, 80, 10), torch.float64),
             ((96, 96, 12), torch.float64), ((128, 128, 8), torch.float64), ((64, 32, 16), torch.float32)]


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


def _nz_for(n):
    return {16: 24, 20: 16, 24: 10, 32: 20, 36: 12, 40: 18, 48: 16, 64: 24, 72: 8, 80: 12, 96: 10, 128: 12}[n]


def _solve(plan, S):
    phi = plan.solve(S)
    torch.cuda.synchronize()
    return phi


@pytest.mark.parametrize("dtype,n", [(torch.float32, n) for n in FUSED_FP32] +
                         [(torch.float64, n) for n in FUSED_FP64])
def test_fused_plan_matches_oracle_and_five_pass(dtype, n):
    from paper_1106_0557_amd import Plan

    nz = _nz_for(n)
    mesh = (n, n, nz)
    h = (0.02, 0.02 * 1.5, 0.03)
    tol = FP64_TOL if dtype == torch.float64 else FP32_TOL
    say(f"[fused] {dtype} mesh {mesh}")
    S = sources.random_field(mesh, seed=n).to("cuda", dtype)
    fused = Plan(*mesh, h=h, dtype=dtype)
    five = Plan(*mesh, h=h, dtype=dtype, five_pass=True)
    assert fused.fused and not five.fused
    assert fused.active_passes == (0, 2, 4) and five.active_passes == (0, 1, 2, 3, 4)
    got = _solve(fused, S).double().cpu().numpy()
    ref5 = _solve(five, S).double().cpu().numpy()
    want = oracle.solve_fft(S.double().cpu().numpy(), h)
    r = norms.report(got, want)
    r5 = norms.rel_l2(got, ref5)
    say(f"  vs oracle {r}, vs five-pass rel_l2 {r5:.2e}")
    assert r["rel_l2"] <= tol
    if dtype == torch.float64:
        assert r["rel_max"] <= tol
    assert r5 <= tol
    fused.close()
    five.close()


@pytest.mark.parametrize("mesh,dtype", NOT_FUSED)
def test_plans_outside_the_fused_set_run_five_passes(mesh, dtype):
    from paper_1106_0557_amd import Plan

    plan = Plan(*mesh, h=1.0 / mesh[0], dtype=dtype)
    say(f"[not fused] {dtype} mesh {mesh}: fused={plan.fused}")
    assert not plan.fused and plan.active_passes == (0, 1, 2, 3, 4)
    plan.close()


@pytest.mark.parametrize("mesh", [(32, 32, 20), (24, 24, 16), (36, 36, 10)])
def test_fused_passes_match_oracle_stages(mesh):
    from paper_1106_0557_amd import (PASS_X_FWD, PASS_X_INV, PASS_Y_FWD, PASS_Y_INV, PASS_Z_CONV, Plan,
                                     Workspace, pass_batched)

    nx, ny, nz = mesh
    h = (0.3, 0.2, 0.5)
    say(f"[fused stages] mesh {mesh}")
    S = sources.random_field(mesh, seed=7).numpy()
    plan = Plan(*mesh, h=h, dtype=torch.float64)
    assert plan.fused
    mem = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    ws = Workspace(plan, memory=mem)
    csz = 16
    main = nz * 2 * ny * nx * csz
    off = (main + 255) // 256 * 256
    B = plan.ztile  # W is [nz/B][2ny][B][nx] (pspfft_workspace_ztile)
    W = mem[:main].view(torch.complex128).view(nz // B, 2 * ny, B, nx).permute(0, 2, 1, 3)
    Wn = mem[off:off + nz * 2 * ny * csz].view(torch.complex128).view(nz, 2 * ny)
    Sd = torch.from_numpy(S).cuda()
    Phi = torch.empty_like(Sd)

    A = np.zeros((2 * nz, 2 * ny, 2 * nx), complex)
    A[:nz, :ny, :nx] = S
    A = oracle.fft_axis(oracle.fft_axis(A, 0), 1)
    pass_batched(PASS_X_FWD, [ws], S=[Sd], Phi=[Phi])
    torch.cuda.synchronize()
    got, gotn = W.reshape(nz, 2 * ny, nx).cpu().numpy(), Wn.cpu().numpy()
    ref = A[:nz, :, : nx + 1]
    scale = np.abs(ref).max()
    e = max(np.abs(got - ref[:, :, :nx]).max(), np.abs(gotn - ref[:, :, nx]).max()) / scale
    say(f"  fused x+y forward err {e:.2e}")
    assert e <= FP64_TOL

    before = mem.clone()
    pass_batched(PASS_Y_FWD, [ws], S=[Sd], Phi=[Phi])
    pass_batched(PASS_Y_INV, [ws], S=[Sd], Phi=[Phi])
    torch.cuda.synchronize()
    assert torch.equal(before, mem), "the y passes of a fused plan must not touch the workspace"

    pass_batched(PASS_Z_CONV, [ws], S=[Sd], Phi=[Phi])
    pass_batched(PASS_X_INV, [ws], S=[Sd], Phi=[Phi])
    torch.cuda.synchronize()
    want = oracle.solve_fft(S, h)
    r = norms.report(Phi.cpu().numpy(), want)
    say(f"  potential {r}")
    assert r["rel_l2"] <= FP64_TOL and r["rel_max"] <= FP64_TOL
    ws.close()
    plan.close()


def test_fused_and_five_pass_problems_in_one_batch():
    import paper_1106_0557_amd as ps

    say("[fused batch] mixed fused / five-pass / sizes, in place")
    cases = [((64, 64, 24), False), ((64, 64, 24), True), ((48, 48, 16), False), ((32, 32, 32), False),
             ((48, 48, 16), True), ((128, 128, 8), False), ((40, 24, 16), False), ((64, 64, 24), False)]
    plans = {}
    ws, S, P = [], [], []
    for k, (mesh, five) in enumerate(cases):
        key = (mesh, five)
        if key not in plans:
            plans[key] = ps.Plan(*mesh, h=(0.1, 0.1, 0.2), dtype=torch.float32, five_pass=five)
        ws.append(plans[key].workspace())
        S.append(sources.random_field(mesh, seed=100 + k).to("cuda", torch.float32))
        P.append(S[-1].clone() if k % 3 == 0 else torch.empty_like(S[-1]))  # k % 3 == 0: in place
    srcs = [s.clone() for s in S]
    ps.solve_batched(ws, [P[k] if k % 3 == 0 else S[k] for k in range(len(cases))], P)
    torch.cuda.synchronize()
    for k, (mesh, five) in enumerate(cases):
        plan = plans[(mesh, five)]
        alone = plan.solve(srcs[k])
        torch.cuda.synchronize()
        assert torch.equal(alone, P[k]), f"case {k} {mesh} five_pass={five} differs in the batch"
        want = oracle.solve_fft(srcs[k].double().cpu().numpy(), (0.1, 0.1, 0.2))
        assert norms.rel_l2(P[k].double().cpu().numpy(), want) <= FP32_TOL
    for w in ws:
        w.close()
    for p in plans.values():
        p.close()


@pytest.mark.parametrize("mesh,dtype,five,count", [((128, 128, 128), torch.float32, False, 8),
                                                    ((128, 128, 128), torch.float32, True, 8),
                                                    ((128, 128, 128), torch.float64, False, 4),
                                                    ((128, 128, 256), torch.float32, False, 4)])
def test_streaming_batch_equals_alone(mesh, dtype, five, count):
    """Problems whose workspaces together pass the 256 MB streaming threshold
    (eight FP32 or four FP64 128^3 meshes; four 128x128x256 meshes, whose z
    lines of 512 points lie within one wavefront) in one batched call, against
    each solved alone (below the threshold)."""
    import paper_1106_0557_amd as ps

    say(f"[streaming batch] {count} x {mesh} {dtype}, five_pass={five}")
    h = tuple(1.0 / m for m in mesh)
    plan = ps.Plan(*mesh, h=h, dtype=dtype, five_pass=five)
    assert count * plan.workspace_bytes > 256 * 2**20 >= plan.workspace_bytes
    if mesh[2] == 256:
        assert plan.spectrum_kz_fastest  # wavefront-owned z lines
    ws = [plan.workspace() for _ in range(count)]
    S = [sources.random_field(mesh, seed=300 + k).to("cuda", dtype) for k in range(count)]
    P = [torch.empty_like(s) for s in S]
    ps.solve_batched(ws, S, P)
    torch.cuda.synchronize()
    for k in range(count):
        alone = plan.solve(S[k])
        torch.cuda.synchronize()
        assert torch.equal(alone, P[k]), f"problem {k} differs between the streaming batch and alone"
    want = oracle.solve_fft(S[0].double().cpu().numpy(), h)
    err = norms.rel_l2(P[0].double().cpu().numpy(), want)
    say(f"  rel l2 vs oracle {err:.3e}")
    assert err <= (FP32_TOL if dtype == torch.float32 else FP64_TOL)
    for w in ws:
        w.close()
    plan.close()
