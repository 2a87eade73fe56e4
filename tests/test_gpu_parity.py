"""Parity of the HIP path against the FP64 CPU oracle (needs a gfx950 GPU).

Bars: FP64 <= 1e-12 relative L2 and relative max against the oracle; FP32 <=
1e-5 relative L2 against the FP64 oracle (max error reported).  Integer-like
checks (batched == single) are bit-exact.
"""
import math
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
    import paper_1106_0557_amd  # noqa: F401
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


# ---------------------------------------------------------------- spectrum --

# z sizes whose three-stage z lines are kept within one wavefront (spectrum kz-fastest);
# lines of 1536 (24*8*8) take a smaller tile
WAVE_Z = (256, 288, 384, 512, 768)
# z sizes whose four-stage FP32 z lines are kept within one wavefront (arrays below 4 GB):
# 2nz = 1152 and 2304 (36*4*4*2, 36*4*4*4), 640 and 1280 (20*4*4*2, 20*4*4*4)
WAVE_Z4 = (576, 1152, 320, 640)


# z sizes whose FP32 z lines go to the 32-family, within one wavefront: 2048 = 32*32*2
WAVE_Z32 = (1024,)


def kz_fastest_expected(nz, dtype):
    return nz in WAVE_Z or (dtype == torch.float32 and (nz in WAVE_Z4 or nz in WAVE_Z32))


# (16, 8, 512): z lines of 1024 = 16*16*4, kept kz-fastest
@pytest.mark.parametrize("n,h", [((16, 16, 16), (1 / 16,) * 3), ((24, 10, 16), (0.3, 0.2, 0.5)),
                                 ((24, 18, 20), (0.05, 0.07, 0.06)), ((36, 8, 40), (1.0, 1.0, 2.0)),
                                 ((16, 8, 512), (0.02, 0.03, 0.025)), ((16, 8, 576), (0.02, 0.03, 0.025))])
def test_green_spectrum_matches_oracle(n, h):
    from paper_1106_0557_amd import Plan

    say(f"[spectrum] n={n} h={h}")
    want, imag_max, abs_max = oracle.green_hat_octant(n, h)
    for dtype, tol in ((torch.float64, FP64_TOL), (torch.float32, 1e-7)):
        plan = Plan(*n, h=h, dtype=dtype)
        assert plan.spectrum_kz_fastest == kz_fastest_expected(n[2], dtype)
        got = plan.green().double().cpu().numpy()
        plan.close()
        err = np.abs(got - want).max() / abs_max
        say(f"  {dtype}: max err / max|G~| = {err:.3e}")
        assert err <= tol


# ---------------------------------------------------------- per-pass stages --

def _workspace_views(plan, mem):
    nx, ny, nz = plan.n
    csz = 16 if plan.dtype == torch.float64 else 8
    main = nz * 2 * ny * nx * csz
    off = (main + 255) // 256 * 256
    cdt = torch.complex128 if plan.dtype == torch.float64 else torch.complex64
    B = plan.ztile  # W is [nz/B][2ny][B][nx] (pspfft_workspace_ztile)
    Wt = mem[:main].view(cdt).view(nz // B, 2 * ny, B, nx)
    Wn = mem[off:off + nz * 2 * ny * csz].view(cdt).view(nz, 2 * ny)
    return (lambda: Wt.permute(0, 2, 1, 3).reshape(nz, 2 * ny, nx)), Wn


@pytest.mark.parametrize("n,ztile", [((24, 20, 16), None), ((16, 36, 24), None), ((40, 16, 18), None),
                                     ((24, 20, 32), "4"), ((16, 12, 128), "16")])
def test_each_pass_matches_oracle_stage(n, ztile, monkeypatch):
    """Run the passes one at a time and compare the workspace with the oracle's stages.

    With ``ztile`` the workspace is forced into tiles of z planes (PSPFFT_ZTILE),
    which large meshes get by themselves, and read back through the documented layout."""
    if ztile is not None:
        monkeypatch.setenv("PSPFFT_ZTILE", ztile)
    from paper_1106_0557_amd import (PASS_X_FWD, PASS_Y_FWD, PASS_Z_CONV, PASS_Y_INV, PASS_X_INV, Plan,
                                     Workspace, pass_batched)

    say(f"[passes] n={n} ztile={ztile}")
    nx, ny, nz = n
    h = (0.3, 0.2, 0.5)
    S = sources.random_field(n, seed=11).numpy()
    plan = Plan(*n, h=h, dtype=torch.float64)
    if ztile is not None:
        assert plan.ztile == int(ztile), plan.ztile
    mem = torch.empty(plan.workspace_bytes, dtype=torch.uint8, device="cuda")
    ws = Workspace(plan, memory=mem)
    W, Wn = _workspace_views(plan, mem)
    Sd = torch.from_numpy(S).cuda()
    Phi = torch.empty_like(Sd)

    def spectrum_rows(A, zmax, ymax):
        """Compare W (kx < nx) and Wn (kx = nx) with A[z<zmax, y<ymax, kx<=nx]."""
        torch.cuda.synchronize()
        got = W().cpu().numpy()[:zmax, :ymax, :]
        gotn = Wn.cpu().numpy()[:zmax, :ymax]
        ref = A[:zmax, :ymax, : nx + 1]
        scale = np.abs(ref).max()
        e1 = np.abs(got - ref[:, :, :nx]).max() / scale
        e2 = np.abs(gotn - ref[:, :, nx]).max() / scale
        return max(e1, e2)

    A = np.zeros((2 * nz, 2 * ny, 2 * nx), complex)
    A[:nz, :ny, :nx] = S
    A = oracle.fft_axis(A, 0)
    pass_batched(PASS_X_FWD, [ws], S=[Sd], Phi=[Phi])
    e = spectrum_rows(A, nz, ny)
    say(f"  x_fwd err {e:.2e}")
    assert e <= FP64_TOL

    A = oracle.fft_axis(A, 1)
    pass_batched(PASS_Y_FWD, [ws], S=[Sd], Phi=[Phi])
    e = spectrum_rows(A, nz, 2 * ny)
    say(f"  y_fwd err {e:.2e}")
    assert e <= FP64_TOL

    g = oracle.green_doubled(n, h)
    ghat = np.fft.fftn(g).real / g.size  # an independent transform of the doubled G
    A[nz:] = 0.0  # the z pass reads only z < nz (the rest is zero padding)
    A = oracle.fft_axis(oracle.fft_axis(A, 2) * ghat, 2, +1)
    pass_batched(PASS_Z_CONV, [ws], S=[Sd], Phi=[Phi])
    e = spectrum_rows(A, nz, 2 * ny)
    say(f"  z_conv err {e:.2e}")
    assert e <= FP64_TOL

    A[nz:] = 0.0
    A = oracle.fft_axis(A, 1, +1)
    pass_batched(PASS_Y_INV, [ws], S=[Sd], Phi=[Phi])
    e = spectrum_rows(A, nz, ny)
    say(f"  y_inv err {e:.2e}")
    assert e <= FP64_TOL

    A[:, ny:] = 0.0
    A = oracle.fft_axis(A, 0, +1)
    pass_batched(PASS_X_INV, [ws], S=[Sd], Phi=[Phi])
    torch.cuda.synchronize()
    ref = A[:nz, :ny, :nx].real
    e = norms.rel_max(Phi.cpu().numpy(), ref)
    say(f"  x_inv err {e:.2e}")
    assert e <= FP64_TOL
    # and the whole thing equals the oracle solve
    assert norms.rel_l2(Phi.cpu().numpy(), oracle.solve_fft(S, h)) <= FP64_TOL
    ws.close()
    plan.close()


# ------------------------------------------------------------ whole solve --

SIZES = [
    (16, 8, 8), (16, 16, 16), (32, 32, 32), (24, 24, 24), (20, 20, 20), (36, 36, 36), (48, 32, 24),
    (40, 12, 18), (20, 12, 10), (64, 48, 40), (96, 96, 96), (72, 18, 144),
]


@pytest.mark.parametrize("n", SIZES)
def test_solve_matches_oracle(n):
    say(f"[solve] n={n}")
    h = tuple(1.0 / v for v in n)
    S = sources.random_field(n, seed=sum(n)).numpy()
    ref = oracle.solve_fft(S, h)
    got64 = gpu_solve(n, h, S, torch.float64)
    r64 = norms.report(got64, ref)
    got32 = gpu_solve(n, h, S, torch.float32)
    r32 = norms.report(got32, ref)
    say(f"  fp64 {r64}\n  fp32 {r32}")
    assert r64["rel_l2"] <= FP64_TOL and r64["rel_max"] <= FP64_TOL
    assert r32["rel_l2"] <= FP32_TOL


# Lines of three stages (radices E, M, K) with compile-time geometry: z lines of
# 512 (16*16*2), 1024 (16*16*4), 768 (24*8*4) and 576 (36*4*4), each kept within
# one wavefront, 384 (24*8*2), 320 (20*4*4); y lines of 1024 (16*16*4) and 768
# (24*8*4), each kept within one wavefront, 384 (24*8*2), 288 (36*4*2), 160
# (20*4*2); x rows of 512, 384 and 576 (36*4*4, stage tables in global memory; (576, 20, 18)
# spans several row tiles with a partial last one).
THREE_STAGE = [(16, 8, 256), (16, 8, 512), (16, 8, 384), (16, 8, 192), (16, 8, 288), (16, 512, 8),
               (16, 384, 8), (16, 192, 8), (16, 144, 8), (20, 80, 160), (512, 8, 8), (384, 8, 8),
               (16, 384, 288), (576, 8, 8), (576, 20, 18)]


@pytest.mark.parametrize("n", THREE_STAGE)
def test_three_stage_lines_match_oracle(n):
    say(f"[three-stage] n={n}")
    from paper_1106_0557_amd import Plan

    for dt in (torch.float32, torch.float64):
        p = Plan(*n, h=0.1, dtype=dt)
        assert p.spectrum_kz_fastest == (n[2] in WAVE_Z)
        p.close()
    h = (0.02, 0.03, 0.025)
    S = sources.random_field(n, seed=sum(n) + 1).numpy()
    ref = oracle.solve_fft(S, h)
    got64 = gpu_solve(n, h, S, torch.float64)
    got32 = gpu_solve(n, h, S, torch.float32)
    r64, r32 = norms.report(got64, ref), norms.report(got32, ref)
    say(f"  fp64 {r64}\n  fp32 {r32}")
    assert r64["rel_l2"] <= FP64_TOL and r64["rel_max"] <= FP64_TOL
    assert r32["rel_l2"] <= FP32_TOL


# Long lines whose default tile does not fit (the workgroup limit of the family
# or the LDS), so their compile-time geometry takes a smaller tile: y and z lines
# of 1536 (24*8*8) and 2048 (16*16*8, lines of 128 threads, two wavefronts), x
# rows of 768 (24*8*4), 1024 (16*16*4) and 2048 (16*16*8, whose split-step
# partners go through LDS rather than the mirror lane).  Their z passes fill a
# CU with one workgroup and run persistently, as do their y passes; (80, 18,
# 768) and (40, 18, 1024) give z workgroups several tiles each (more tiles than
# CUs) and a partial last Nyquist tile (36 lines), whose spare lanes repeat the
# set's last line, and (80, 768, 36) does the same for the y passes.
# FP32 z lines of 2048 points go to the 32-family (32*32*2, within one wavefront):
# (48, 36, 1024) gives its persistent workgroups several tiles; (80, 36, 512) does the
# same for the 16-family's 1024-point lines.
LONG_LINES = [(16, 768, 8), (16, 8, 768), (768, 8, 8), (16, 1024, 8), (16, 8, 1024), (1024, 8, 8), (2048, 8, 8),
              (80, 18, 768), (40, 18, 1024), (80, 768, 36), (80, 36, 512), (48, 36, 1024)]


@pytest.mark.parametrize("n", LONG_LINES)
def test_long_lines_match_oracle(n):
    say(f"[long lines] n={n}")
    from paper_1106_0557_amd import Plan

    for dt in (torch.float32, torch.float64):
        p = Plan(*n, h=0.1, dtype=dt)
        assert p.spectrum_kz_fastest == kz_fastest_expected(n[2], dt)
        p.close()
    h = (0.02, 0.03, 0.025)
    S = sources.random_field(n, seed=sum(n) + 3).numpy()
    ref = oracle.solve_fft(S, h)
    got64 = gpu_solve(n, h, S, torch.float64)
    got32 = gpu_solve(n, h, S, torch.float32)
    r64, r32 = norms.report(got64, ref), norms.report(got32, ref)
    say(f"  fp64 {r64}\n  fp32 {r32}")
    assert r64["rel_l2"] <= FP64_TOL and r64["rel_max"] <= FP64_TOL
    assert r32["rel_l2"] <= FP32_TOL


# Lines of four stages (radices E, M, M, K) with compile-time geometry: z lines
# of 1152 (36*4*4*2), 2304 (36*4*4*4), 640 (20*4*4*2), 1280 (20*4*4*4) and 3072
# (24*8*8*2, FP32 only: FP64 meshes stop at 1152), y lines of 1152 and 1280, x
# rows of 1152 and 640.  In FP32 the z lines of 1152, 2304, 640 and 1280 points
# (and the y lines of 1152 and 1280) are kept within one wavefront; (20, 18, 576)
# ends on partial tiles, and (80, 18, 576) and (40, 18, 1152) give the
# persistent z workgroups several tiles each.
FOUR_STAGE = [(16, 8, 576), (16, 8, 1152), (16, 8, 320), (16, 8, 640), (16, 8, 1536), (16, 576, 8), (16, 640, 8),
              (1152, 8, 8), (640, 8, 8), (20, 18, 576), (80, 18, 576), (40, 18, 1152)]


@pytest.mark.parametrize("n", FOUR_STAGE)
def test_four_stage_lines_match_oracle(n):
    say(f"[four-stage] n={n}")
    from paper_1106_0557_amd import Plan

    for dt in (torch.float32, torch.float64):
        if dt == torch.float64 and max(n) > 1152:
            continue
        p = Plan(*n, h=0.1, dtype=dt)
        assert p.spectrum_kz_fastest == kz_fastest_expected(n[2], dt)
        p.close()
    h = (0.02, 0.03, 0.025)
    S = sources.random_field(n, seed=sum(n) + 7).numpy()
    ref = oracle.solve_fft(S, h)
    if max(n) <= 1152:
        got64 = gpu_solve(n, h, S, torch.float64)
        r64 = norms.report(got64, ref)
        say(f"  fp64 {r64}")
        assert r64["rel_l2"] <= FP64_TOL and r64["rel_max"] <= FP64_TOL
    got32 = gpu_solve(n, h, S, torch.float32)
    r32 = norms.report(got32, ref)
    say(f"  fp32 {r32}")
    assert r32["rel_l2"] <= FP32_TOL


def test_zero_source_gives_zero_potential():
    say("[zero source]")
    n = (24, 16, 20)
    for dtype in (torch.float32, torch.float64):
        got = gpu_solve(n, 0.1, np.zeros(n[::-1]), dtype)
        assert np.all(got == 0.0)


@pytest.mark.parametrize("c", [(0, 0, 0), (5, 3, 7), (15, 11, 9)])
def test_impulse_response_is_green_function(c):
    say(f"[impulse] c={c}")
    n = (16, 12, 10)
    h = (0.3, 0.2, 0.5)
    S = np.zeros(n[::-1])
    S[c[2], c[1], c[0]] = 1.0
    got = gpu_solve(n, h, S, torch.float64)
    want = np.empty_like(S)
    for z in range(n[2]):
        for y in range(n[1]):
            for x in range(n[0]):
                want[z, y, x] = oracle.green_value(abs(x - c[0]), abs(y - c[1]), abs(z - c[2]), h)
    assert np.abs(got - want).max() <= FP64_TOL * np.abs(want).max()


def test_config1_matches_full_direct_sum():
    say("[config1] n=32 sphere vs direct sum")
    n, h, S = sources.config1()
    S = S.numpy()
    want = oracle.direct(S, h)
    got64 = gpu_solve((n,) * 3, h, S, torch.float64)
    got32 = gpu_solve((n,) * 3, h, S, torch.float32)
    r64, r32 = norms.report(got64, want), norms.report(got32, want)
    say(f"  fp64 {r64}\n  fp32 {r32}")
    assert r64["rel_l2"] <= FP64_TOL and r64["rel_max"] <= FP64_TOL
    assert r32["rel_l2"] <= FP32_TOL


def test_config2_spheroid_n128():
    from oracle import closed_forms as cf

    say("[config2] n=128 spheroid")
    n, h, S = sources.config2()
    S = S.numpy()
    ref = oracle.solve_fft(S, h)
    got64 = gpu_solve((n,) * 3, h, S, torch.float64)
    got32 = gpu_solve((n,) * 3, h, S, torch.float32)
    r64, r32 = norms.report(got64, ref), norms.report(got32, ref)
    r32_64 = norms.report(got32, got64)
    say(f"  fp64 vs oracle {r64}\n  fp32 vs oracle {r32}\n  fp32 vs gpu fp64 {r32_64}")
    assert r64["rel_l2"] <= FP64_TOL and r64["rel_max"] <= FP64_TOL
    assert r32["rel_l2"] <= FP32_TOL and r32_64["rel_l2"] <= FP32_TOL
    x = (np.arange(n) + 0.5) * h - 0.5
    analytic = cf.phi_spheroid(x[None, None, :], x[None, :, None], x[:, None, None], 0.3, 0.15, 1.0)
    l1 = norms.l1(got64, analytic)
    say(f"  L1 vs analytic spheroid: {l1:.3e}")
    assert l1 < 5e-3


def test_in_place_solve():
    from paper_1106_0557_amd import Plan

    say("[in place]")
    n = (32, 24, 16)
    S = sources.random_field(n, seed=3)
    ref = oracle.solve_fft(S.numpy(), 0.1)
    for dtype, tol in ((torch.float64, FP64_TOL), (torch.float32, FP32_TOL)):
        plan = Plan(*n, h=0.1, dtype=dtype)
        buf = S.to("cuda", dtype)
        plan.solve(buf, out=buf)
        torch.cuda.synchronize()
        assert norms.rel_l2(buf.double().cpu().numpy(), ref) <= tol
        plan.close()


@pytest.mark.parametrize("n", [(2048, 8, 8), (16, 8, 1152)])
def test_longest_lines(n):
    """The longest transform lengths the kernels accept (x: L = 2048 FP32; z: L = 2304 FP64)."""
    say(f"[longest] n={n}")
    h = (0.01, 0.02, 0.03)
    S = sources.random_field(n, seed=5).numpy()
    ref = oracle.solve_fft(S, h)
    got64 = gpu_solve(n, h, S, torch.float64) if max(n) <= 1152 else None
    got32 = gpu_solve(n, h, S, torch.float32)
    if got64 is not None:
        r64 = norms.report(got64, ref)
        say(f"  fp64 {r64}")
        assert r64["rel_l2"] <= FP64_TOL and r64["rel_max"] <= FP64_TOL
    r32 = norms.report(got32, ref)
    say(f"  fp32 {r32}")
    assert r32["rel_l2"] <= FP32_TOL


# ------------------------------------------------------------- large sizes --

_CONFIG5 = {}


def _config5_direct():
    """Config 5 (512^3, 64 blobs plus a sphere) and the oracle's direct sum at 256
    sampled cells (the three corners of interest among them), computed once."""
    if not _CONFIG5:
        n, h, S = sources.config5(device="cuda")
        S = S.cpu()
        rng = np.random.default_rng(55)
        targets = np.unique(np.concatenate([rng.integers(0, n**3, size=253),
                                            [0, n**3 - 1, (n // 2) * (n * n + n + 1)]]))
        while targets.size < 256:
            targets = np.unique(np.concatenate([targets, rng.integers(0, n**3, size=256 - targets.size)]))
        _CONFIG5.update(n=n, h=h, S=S, targets=targets, want=oracle.direct(S.numpy(), h, targets))
    c = _CONFIG5
    return c["n"], c["h"], c["S"], c["targets"], c["want"]


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_config5_n512_sampled_direct_sum(dtype):
    """Full-size 512^3 (1024^3 padded) solve checked at 256 sampled targets by the direct sum."""
    from paper_1106_0557_amd import Plan

    say(f"[config5] n=512 {dtype}")
    n, h, S, targets, want = _config5_direct()
    assert targets.size == 256
    plan = Plan(n, n, n, h=h, dtype=dtype)
    # z lines of 1024 within one wavefront (FP64: the 64-bit form, its workspace passes 4 GB)
    assert plan.spectrum_kz_fastest
    phi = plan.solve(S.to("cuda", dtype))
    torch.cuda.synchronize()
    got = phi.reshape(-1)[torch.from_numpy(targets).cuda()].double().cpu().numpy()
    plan.close()
    del phi
    err = np.abs(got - want).max() / np.abs(want).max()
    say(f"  sampled rel max err {err:.3e}")
    assert err <= (FP64_TOL if dtype == torch.float64 else FP32_TOL)


def test_config5_fp64_and_fp32_agree_on_every_cell():
    """The 512^3 solve in both precisions: the FP64 workspace passes 4 GB (64-bit
    addressing), the FP32 one does not; the two potentials agree to the FP32
    tolerance over the whole field."""
    from paper_1106_0557_amd import Plan, workspace_bytes

    say("[config5] n=512 fp64 vs fp32, whole field")
    n, h, S = sources.config5(device="cuda")
    assert workspace_bytes(n, n, n, torch.float64) >= 1 << 32 > workspace_bytes(n, n, n, torch.float32)
    out = {}
    for dt in (torch.float64, torch.float32):
        plan = Plan(n, n, n, h=h, dtype=dt)
        out[dt] = plan.solve(S.to(dt)).double()
        torch.cuda.synchronize()
        plan.close()
    d = (torch.linalg.vector_norm(out[torch.float32] - out[torch.float64])
         / torch.linalg.vector_norm(out[torch.float64])).item()
    say(f"  rel l2 {d:.3e}")
    assert d <= FP32_TOL


# FP32 meshes whose workspace passes 4 GB (64-bit addressing): x rows of 768 = 24*8*4,
# y lines of 1536 = 24*8*8 and z lines of 1024 = 16*16*4; then y lines of 1152 =
# 36*4*4*2 and z lines of 1280 = 20*4*4*4; z lines of 2048 (the 32-family, 32*32*2)
# and of 1536 (24*8*8, a halved tile), the z lines always kept within one
# wavefront (64-bit bases per block of positions).
@pytest.mark.parametrize("n", [(768, 768, 512), (768, 576, 640), (512, 512, 1024), (640, 576, 768)])
def test_fp32_arrays_above_4gb_sampled_direct_sum(n):
    """An FP32 mesh whose workspace passes 4 GB, checked at sampled targets by the direct sum."""
    from paper_1106_0557_amd import Plan, workspace_bytes

    h = (0.011, 0.009, 0.013)
    say(f"[above_4gb] n={n} fp32")
    assert workspace_bytes(*n, torch.float32) >= 1 << 32
    S = sources.random_field(n, seed=57) + 1.0
    size = n[0] * n[1] * n[2]
    rng = np.random.default_rng(57)
    targets = np.concatenate([np.unique(rng.integers(0, size, size=24)), [0, size - 1, size // 2 + n[0] // 2]])
    want = oracle.direct(S.numpy(), h, targets)
    plan = Plan(*n, h=h, dtype=torch.float32)
    assert plan.spectrum_kz_fastest  # z lines within one wavefront, 64-bit block bases
    phi = plan.solve(S.to("cuda", torch.float32))
    torch.cuda.synchronize()
    got = phi.reshape(-1)[torch.from_numpy(targets).cuda()].double().cpu().numpy()
    plan.close()
    del phi
    err = np.abs(got - want).max() / np.abs(want).max()
    say(f"  sampled rel max err {err:.3e}")
    assert err <= FP32_TOL
