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


@pytest.mark.parametrize("n,ok", [(8, True), (16, True), (128, True), (10, True), (12, True), (18, True),
                                  (24, True), (36, True), (40, True), (48, True), (96, True), (144, True),
                                  (1152, True), (2048, True), (4, False), (6, False), (9, False), (15, False),
                                  (7, False), (27, False), (4096, False), (0, False), (-8, False)])
def test_supported_sizes_y_z(lib, n, ok):
    assert (lib.pspfft_workspace_bytes(16, n, 16, 0) > 0) == ok
    assert (lib.pspfft_workspace_bytes(16, 16, n, 0) > 0) == ok


@pytest.mark.parametrize("n,ok", [(16, True), (20, True), (24, True), (36, True), (32, True), (40, True),
                                  (48, True), (72, True), (128, True), (2048, True), (4096, True), (2304, True),
                                  (8, False), (10, False), (12, False), (18, False), (6, False), (8192, False)])
def test_supported_sizes_x(lib, n, ok):
    """x uses the packed real transform of length n, so its minimum sizes are twice those of y, z."""
    assert (lib.pspfft_workspace_bytes(n, 16, 16, 0) > 0) == ok


def test_workspace_bytes_formula(lib):
    for (nx, ny, nz) in [(128, 128, 128), (32, 48, 64), (16, 8, 24)]:
        for prec, c in ((0, 8), (1, 16)):
            main = nz * 2 * ny * nx * c
            nyq = nz * 2 * ny * c
            want = (main + 255) // 256 * 256 + (nyq + 255) // 256 * 256
            assert lib.pspfft_workspace_bytes(nx, ny, nz, prec) == want
    assert lib.pspfft_workspace_bytes(16, 16, 16, 7) == 0
    # FP64 has a smaller maximum size
    assert lib.pspfft_workspace_bytes(16, 2048, 8, 0) > 0
    assert lib.pspfft_workspace_bytes(16, 2048, 8, 1) == 0
    assert lib.pspfft_workspace_bytes(2304, 8, 8, 1) > 0
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
    for n in [(15, 16, 16), (16, 7, 16), (16, 16, 4096), (4, 16, 16), (8, 16, 16)]:
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
    assert lib.pspfft_plan_create_ex(16, 16, 15, h3, 0, 1, ctypes.byref(handle)) == 2


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
