"""The C ABI library loads and exports every symbol include/pspfft.h declares.

No compute calls: only host-side validation paths that return before any HIP
call, plus pure size queries.  Runs without a GPU.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pspfft.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pspfft_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1106_0557_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        from paper_1106_0557_amd import build

        build.build(verbose=False)
    return _lib.load()


def test_library_exports_every_declared_symbol(lib):
    from paper_1106_0557_amd import _lib

    declared = _declared_functions()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), f"libpspfft.so does not export {name}"
    assert sorted(_lib.EXPORTS) == declared


def test_status_strings(lib):
    for code in range(6):
        s = lib.pspfft_status_string(code)
        assert s and s.decode() != "unknown status"
    assert lib.pspfft_status_string(99).decode() == "unknown status"


def _smooth(n):
    """n = 2^a 3^b 5^c"""
    if n < 1:
        return False
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


def _odd_part(n):
    while n % 2 == 0:
        n //= 2
    return n


def test_supported_sizes_y_z(lib):
    """Every n = 2^a 3^b 5^c with 2n <= 4096, in both precisions, and nothing else."""
    for n in list(range(-2, 2100)) + [2160, 2304, 3072, 4096]:
        ok = _smooth(n) and n <= 2048
        for prec in (0, 1):
            assert (lib.pspfft_workspace_bytes(16, n, 16, prec) > 0) == ok, (n, prec)
            assert (lib.pspfft_workspace_bytes(16, 16, n, prec) > 0) == ok, (n, prec)


def test_supported_sizes_x(lib):
    """x: every 2^a 3^b 5^c up to 2048 as for y and z; the packed real transform of
    length n also takes longer rows whose odd part is 1, 3, 5 or 9 (up to 4096 in
    FP32, 2304 in FP64)."""
    for n in list(range(-2, 2100)) + [2160, 2304, 2400, 2560, 3072, 3200, 4096, 4608, 8192]:
        for prec, lim in ((0, 4096), (1, 2304)):
            ok = _smooth(n) and (n <= 2048 or (_odd_part(n) in (1, 3, 5, 9) and n <= lim))
            assert (lib.pspfft_workspace_bytes(n, 16, 16, prec) > 0) == ok, (n, prec)


def test_workspace_bytes_formula(lib):
    for (nx, ny, nz) in [(128, 128, 128), (32, 48, 64), (16, 8, 24)]:
        for prec, c in ((0, 8), (1, 16)):
            main = nz * 2 * ny * nx * c
            nyq = nz * 2 * ny * c
            want = (main + 255) // 256 * 256 + (nyq + 255) // 256 * 256
            assert lib.pspfft_workspace_bytes(nx, ny, nz, prec) == want
    assert lib.pspfft_workspace_bytes(16, 16, 16, 7) == 0
    # odd sizes, and the largest rows per precision
    assert lib.pspfft_workspace_bytes(15, 1, 27, 1) == ((27 * 2 * 15 * 16 + 255) // 256 + (27 * 2 * 16 + 255) // 256) * 256
    assert lib.pspfft_workspace_bytes(16, 2048, 8, 1) > 0
    assert lib.pspfft_workspace_bytes(2304, 8, 8, 1) > 0
    assert lib.pspfft_workspace_bytes(4096, 8, 8, 0) > 0
    assert lib.pspfft_workspace_bytes(4096, 8, 8, 1) == 0


def _create(lib, n, h, prec=0):
    handle = ctypes.c_void_p()
    h3 = None if h is None else (ctypes.c_double * 3)(*h)
    st = lib.pspfft_plan_create(n[0], n[1], n[2], h3, prec, ctypes.byref(handle))
    return st, handle.value


def test_plan_create_rejects_bad_arguments_before_device_work(lib):
    bad_h = [(0.0, 1.0, 1.0), (-1.0, 1.0, 1.0), (float("nan"), 1.0, 1.0), (1.0, float("inf"), 1.0)]
    for h in bad_h:
        st, handle = _create(lib, (16, 16, 16), h)
        assert st == 1 and handle is None
    st, handle = _create(lib, (16, 16, 16), None)
    assert st == 1
    st, handle = _create(lib, (16, 16, 16), (1, 1, 1), prec=3)
    assert st == 1
    st, handle = _create(lib, (0, 16, 16), (1, 1, 1))
    assert st == 1
    for n in [(7, 16, 16), (16, 7, 16), (16, 16, 4096), (22, 16, 16), (16, 16, 2049), (16, 14, 16)]:
        st, handle = _create(lib, n, (1, 1, 1))
        assert st == 2 and handle is None
    # null out-pointer
    h3 = (ctypes.c_double * 3)(1, 1, 1)
    assert lib.pspfft_plan_create(16, 16, 16, h3, 0, None) == 1


def test_plan_create_ex_rejects_unknown_flags_before_device_work(lib):
    h3 = (ctypes.c_double * 3)(1, 1, 1)
    handle = ctypes.c_void_p()
    for flags in (2, 4, 0x80000000, 3):
        assert lib.pspfft_plan_create_ex(16, 16, 16, h3, 0, flags, ctypes.byref(handle)) == 1
        assert handle.value is None
    assert lib.pspfft_plan_create_ex(16, 16, 16, h3, 0, 0, None) == 1
    assert lib.pspfft_plan_create_ex(16, 16, 16, None, 0, 1, ctypes.byref(handle)) == 1
    assert lib.pspfft_plan_create_ex(16, 16, 14, h3, 0, 1, ctypes.byref(handle)) == 2


def test_null_handles(lib):
    assert lib.pspfft_destroy(None) == 1
    assert lib.pspfft_workspace_destroy(None) == 1
    assert lib.pspfft_solve(None, None, None, None) == 1
    assert lib.pspfft_solve_ws(None, None, None, None, None) == 1
    assert lib.pspfft_plan_bytes(None) == 0
    assert lib.pspfft_pass_bytes(None, 0) == 0
    assert lib.pspfft_plan_info(None, None, None, None) == 1
    assert lib.pspfft_plan_green(None, None, None) == 1
    assert lib.pspfft_plan_fused(None) == 0
    assert lib.pspfft_plan_spectrum_kz_fastest(None) == 0
    assert lib.pspfft_workspace_ztile(None) == 0
    # an empty batch is a no-op; a negative count is an error
    assert lib.pspfft_solve_batched(0, None, None, None, None, None) == 0
    assert lib.pspfft_solve_batched(-1, None, None, None, None, None) == 1
    assert lib.pspfft_pass_batched(0, 0, None, None, None, None, None) == 0
    assert lib.pspfft_pass_batched(9, 0, None, None, None, None, None) == 1


def test_python_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1106_0557_amd import _lib

    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _lib.load()
