"""FP64 CPU oracle for the isolated Poisson solve of arXiv:1106.0557 (PSPFFT).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this package; the product library never
does.  It shares no code with the HIP path.

Contents
  * ``liboracle.so`` (from ``oracle.c``, plain C, FP64): textbook DFT, naive
    recursive mixed-radix FFT, 3D transform, the discrete Green's function with
    its self-cell value (Sec. 2.1, Eqs. greens2 and greens_function), the doubled
    mesh by the explicit reflection rules, Hockney's mesh-doubling FFT
    convolution, and the direct O(N^2) sum.
  * :mod:`oracle.closed_forms` -- analytic potentials of the uniform sphere
    (Sec. 4.1) and homogeneous oblate spheroid (Sec. 4.2, 4.3).
  * :mod:`oracle.norms` -- the L1 error norm of Eq. (L1-Norm_Error), relative L2
    and relative max errors.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC_PATH = os.path.join(_HERE, "oracle.c")
_lib = None


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc and OpenMP."""
    if force or not os.path.exists(_LIB_PATH) or (
        os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC_PATH)
    ):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", _LIB_PATH, _SRC_PATH, "-lm"]
        subprocess.check_call(cmd)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    lp = ctypes.POINTER(ctypes.c_long)
    lib.oracle_threads.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_dft_1d.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int]
    lib.oracle_fft_1d.argtypes = [ctypes.c_int, dp, dp, ctypes.c_int]
    lib.oracle_fft_3d.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int]
    lib.oracle_fft_axis.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, ctypes.c_int]
    lib.oracle_green_value.argtypes = [ctypes.c_long, ctypes.c_long, ctypes.c_long, dp]
    lib.oracle_green_value.restype = ctypes.c_double
    lib.oracle_green_doubled.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, dp, dp]
    lib.oracle_green_hat_octant.argtypes = [ctypes.c_int] * 3 + [dp, dp, dp, dp]
    lib.oracle_solve_fft.argtypes = [ctypes.c_int] * 3 + [dp, dp, dp]
    lib.oracle_solve_fft.restype = ctypes.c_int
    lib.oracle_direct.argtypes = [ctypes.c_int] * 3 + [dp, dp, ctypes.c_long, lp, dp]
    lib.oracle_direct.restype = ctypes.c_int
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _h3(h) -> np.ndarray:
    h = np.broadcast_to(np.asarray(h, dtype=np.float64), (3,))
    return np.ascontiguousarray(h, dtype=np.float64)


def threads() -> int:
    return _load().oracle_threads()


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def dft_1d(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """Textbook O(L^2) DFT, ``sum_j x[j] exp(sign 2 pi i j k / L)``."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    out = np.empty_like(x)
    _load().oracle_dft_1d(x.size, _dptr(x.view(np.float64)), _dptr(out.view(np.float64)), sign)
    return out


def fft_1d(x: np.ndarray, sign: int = -1) -> np.ndarray:
    """Naive recursive mixed-radix FFT (same convention as :func:`dft_1d`)."""
    x = np.ascontiguousarray(x, dtype=np.complex128)
    out = np.empty_like(x)
    _load().oracle_fft_1d(x.size, _dptr(x.view(np.float64)), _dptr(out.view(np.float64)), sign)
    return out


def fft_3d(a: np.ndarray, sign: int = -1) -> np.ndarray:
    """3D transform of a complex array of shape (nz, ny, nx); returns a new array."""
    a = np.array(a, dtype=np.complex128, order="C", copy=True)
    nz, ny, nx = a.shape
    _load().oracle_fft_3d(nx, ny, nz, _dptr(a.view(np.float64)), sign)
    return a


def fft_axis(a: np.ndarray, axis: int, sign: int = -1) -> np.ndarray:
    """1D transforms along ``axis`` (0 = x, the last array axis; 2 = z, the first) of a
    complex (nz, ny, nx) array; returns a new array."""
    a = np.array(a, dtype=np.complex128, order="C", copy=True)
    nz, ny, nx = a.shape
    _load().oracle_fft_axis(nx, ny, nz, _dptr(a.view(np.float64)), int(axis), sign)
    return a


def green_value(p: int, q: int, r: int, h) -> float:
    """Discrete Green's function at index offset (p, q, r), Eq. (greens2) plus self cell."""
    return _load().oracle_green_value(int(p), int(q), int(r), _dptr(_h3(h)))


def green_doubled(n, h) -> np.ndarray:
    """Doubled-mesh Green's function of shape (2nz, 2ny, 2nx), reflection rules of Eq. (greens_function)."""
    nx, ny, nz = n
    g = np.empty((2 * nz, 2 * ny, 2 * nx), dtype=np.float64)
    _load().oracle_green_doubled(nx, ny, nz, _dptr(_h3(h)), _dptr(g))
    return g


def green_hat_octant(n, h):
    """Octant (kz<=nz, ky<=ny, kx<=nx) of DFT(doubled G) / ((2nx)(2ny)(2nz)).

    Returns ``(ghat, imag_max, abs_max)`` where ``ghat`` has shape (nz+1, ny+1, nx+1).
    """
    nx, ny, nz = n
    out = np.empty((nz + 1, ny + 1, nx + 1), dtype=np.float64)
    im = np.zeros(1)
    ab = np.zeros(1)
    _load().oracle_green_hat_octant(nx, ny, nz, _dptr(_h3(h)), _dptr(out), _dptr(im), _dptr(ab))
    return out, float(im[0]), float(ab[0])


def solve_fft(S: np.ndarray, h) -> np.ndarray:
    """Hockney mesh-doubling FFT solve (Sec. 2.1); S has shape (nz, ny, nx)."""
    S = np.ascontiguousarray(S, dtype=np.float64)
    nz, ny, nx = S.shape
    phi = np.empty_like(S)
    rc = _load().oracle_solve_fft(nx, ny, nz, _dptr(_h3(h)), _dptr(S), _dptr(phi))
    if rc != 0:
        raise MemoryError("oracle_solve_fft: allocation failed")
    return phi


def direct(S: np.ndarray, h, targets=None) -> np.ndarray:
    """Direct O(N^2) sum at flat target indices (all cells if ``targets`` is None)."""
    S = np.ascontiguousarray(S, dtype=np.float64)
    nz, ny, nx = S.shape
    if targets is None:
        targets = np.arange(S.size, dtype=np.int64)
    targets = np.ascontiguousarray(targets, dtype=np.int64)
    out = np.empty(targets.size, dtype=np.float64)
    rc = _load().oracle_direct(
        nx, ny, nz, _dptr(_h3(h)), _dptr(S), targets.size,
        targets.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _dptr(out),
    )
    if rc != 0:
        raise MemoryError("oracle_direct: allocation failed")
    return out if targets.size != S.size else out.reshape(S.shape)
