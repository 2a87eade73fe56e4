"""Mesh sizes on the generic line kernel: every n = 2^a 3^b 5^c with 2n <= 4096 that
no radix family takes (odd parts 15, 25, 27, 45, 75, 81, 125, 135, ...; lines
shorter than a family's element count; FP64 lines beyond 2 * 1152), alone, mixed
with family axes in one plan, and in batches (Sec. 2.1 defines the result, Sec.
2.2.2 the sequence of 1D transforms).

Bars: FP64 <= 1e-12 relative L2 and relative max against the FP64 oracle; FP32
<= 1e-5 relative L2; batched results bit-identical to the same problem alone.
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


def check(n, h=(0.021, 0.017, 0.013), seed=0, fp64=True, fp32=True):
    S = sources.random_field(n, seed=sum(n) + seed).numpy()
    ref = oracle.solve_fft(S, h)
    if fp64:
        r64 = norms.report(gpu_solve(n, h, S, torch.float64), ref)
        say(f"  fp64 {r64}")
        assert r64["rel_l2"] <= FP64_TOL and r64["rel_max"] <= FP64_TOL
    if fp32:
        r32 = norms.report(gpu_solve(n, h, S, torch.float32), ref)
        say(f"  fp32 {r32}")
        assert r32["rel_l2"] <= FP32_TOL


# the sizes the size contract asked for, as cubes or slabs that keep the oracle quick
CONTRACT = [(60, 60, 60), (100, 100, 100), (120, 120, 120), (135, 135, 135), (240, 24, 20), (24, 240, 20),
            (20, 24, 240)]


@pytest.mark.parametrize("n", CONTRACT)
def test_generic_sizes_match_oracle(n):
    say(f"[generic] n={n}")
    check(n)


# every axis below a family's element count, odd and one-cell axes, odd parts of
# 25, 27, 45, 75, 81, 125 and 3^5, and lines of 2 * 5^4 = 1250 points
SMALL_AND_ODD = [(1, 1, 1), (1, 2, 3), (2, 1, 1), (3, 5, 6), (5, 4, 2), (8, 9, 4), (15, 16, 16),
                 (16, 15, 16), (16, 16, 15), (25, 27, 45), (75, 81, 9), (125, 6, 10), (243, 5, 3),
                 (30, 625, 3), (45, 18, 50)]


@pytest.mark.parametrize("n", SMALL_AND_ODD)
def test_small_and_odd_meshes_match_oracle(n):
    say(f"[generic small/odd] n={n}")
    check(n, seed=1)


# FP64 lines beyond the family limit (2 * 1152): y and z lines of 3072 and 4096
# points (two LDS buffers of one line per workgroup), the largest the contract takes
@pytest.mark.parametrize("n", [(16, 1536, 8), (16, 8, 1536), (16, 2048, 8), (16, 8, 2048), (2048, 3, 2)])
def test_longest_fp64_lines_match_oracle(n):
    say(f"[generic fp64 long] n={n}")
    check(n, seed=2, fp32=False)


def test_fp64_generic_long_lines_sampled_direct_sum():
    """A 24 x 1536 x 24 mesh in FP64 (generic y lines of 3072 points) against the
    oracle's direct sum at sampled cells."""
    from paper_1106_0557_amd import Plan

    n = (24, 1536, 24)
    h = (0.01, 0.003, 0.02)
    S = sources.random_field(n, seed=99)
    size = n[0] * n[1] * n[2]
    rng = np.random.default_rng(99)
    targets = np.unique(np.concatenate([rng.integers(0, size, size=40), [0, size - 1]]))
    want = oracle.direct(S.numpy(), h, targets)
    plan = Plan(*n, h=h, dtype=torch.float64)
    got = plan.solve(S.to("cuda")).reshape(-1)[torch.from_numpy(targets).cuda()].cpu().numpy()
    plan.close()
    err = np.abs(got - want).max() / np.abs(want).max()
    say(f"[generic fp64 sampled] n={n}: rel max {err:.3e}")
    assert err <= FP64_TOL


def test_impulse_response_on_generic_axes():
    """S = delta at a cell gives Phi = G(i - c) exactly (Eq. greens_function), on a
    mesh whose three axes all run on the generic kernel."""
    n = (15, 25, 27)
    h = (0.3, 0.2, 0.5)
    c = (7, 3, 20)
    S = np.zeros(n[::-1])
    S[c[2], c[1], c[0]] = 1.0
    got = gpu_solve(n, h, S, torch.float64)
    want = np.empty_like(S)
    for z in range(n[2]):
        for y in range(n[1]):
            for x in range(n[0]):
                want[z, y, x] = oracle.green_value(abs(x - c[0]), abs(y - c[1]), abs(z - c[2]), h)
    assert np.abs(got - want).max() <= FP64_TOL * np.abs(want).max()


def test_generic_and_family_problems_batched_equal_alone():
    import paper_1106_0557_amd as ps

    cases = [((60, 64, 64), torch.float32), ((64, 60, 64), torch.float32), ((64, 64, 60), torch.float32),
             ((135, 16, 8), torch.float64), ((32, 32, 32), torch.float32), ((15, 25, 27), torch.float32),
             ((15, 25, 27), torch.float64), ((32, 32, 32), torch.float64)]
    say("[generic batch]")
    ws, S, P, plans = [], [], [], []
    for k, (n, dt) in enumerate(cases):
        pl = ps.Plan(*n, h=(0.1, 0.2, 0.3), dtype=dt)
        plans.append(pl)
        ws.append(pl.workspace())
        S.append(sources.random_field(n, seed=k + 50).to("cuda", dt))
        P.append(torch.empty_like(S[-1]))
    ps.solve_batched(ws, S, P)
    torch.cuda.synchronize()
    for k, (n, dt) in enumerate(cases):
        alone = plans[k].solve(S[k])
        torch.cuda.synchronize()
        assert torch.equal(alone, P[k]), f"case {k} {n} differs between batch and alone"
        ref = oracle.solve_fft(S[k].double().cpu().numpy(), (0.1, 0.2, 0.3))
        tol = FP64_TOL if dt == torch.float64 else FP32_TOL
        assert norms.rel_l2(P[k].double().cpu().numpy(), ref) <= tol
    for w in ws:
        w.close()
    for p in plans:
        p.close()


@pytest.mark.parametrize("n,h", [((16, 8, 15), (0.02, 0.03, 0.025)), ((20, 12, 60), (0.05, 0.04, 0.03))])
def test_generic_z_plans_keep_the_spectrum_kz_fastest(n, h):
    """Plans whose z lines run on the generic kernel store the spectrum kz-fastest (the
    lanes of a line read consecutive values) and still export the canonical octant
    (Eq. greens_function transformed, checked against the oracle's)."""
    from paper_1106_0557_amd import Plan

    say(f"[generic z spectrum] n={n}")
    want, _, abs_max = oracle.green_hat_octant(n, h)
    for dtype, tol in ((torch.float64, FP64_TOL), (torch.float32, 1e-7)):
        plan = Plan(*n, h=h, dtype=dtype)
        assert plan.spectrum_kz_fastest
        got = plan.green().double().cpu().numpy()
        plan.close()
        err = np.abs(got - want).max() / abs_max
        say(f"  {dtype}: max err / max|G~| = {err:.3e}")
        assert err <= tol
    check(n, h)
