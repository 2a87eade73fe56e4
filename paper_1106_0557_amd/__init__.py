"""MI355X (gfx950) isolated Poisson solver after Budiardja & Cardall,
arXiv:1106.0557 (PSPFFT): Hockney's mesh-doubling FFT convolution with the
discrete free-space Green's function (Sec. 2.1), as hand-written HIP kernels
behind the C ABI in ``include/pspfft.h``.

Python layer = argument marshalling over that ABI; torch supplies device memory
and streams.  The library is loaded on first use and there is no CPU fallback.

    plan = Plan(128, 128, 128, h=1/128, dtype=torch.float32)
    phi = plan.solve(S)               # S: (nz, ny, nx) cuda tensor of plan dtype
"""
from __future__ import annotations

import ctypes
from typing import Sequence

import torch

from . import _lib
from ._lib import (PASS_NAMES, PASS_X_FWD, PASS_Y_FWD, PASS_Z_CONV, PASS_Y_INV, PASS_X_INV,  # noqa: F401
                   PspfftError)

from ._lib import CONSOLE_ERROR, CONSOLE_WARNING, CONSOLE_INFO_1, CONSOLE_INFO_2  # noqa: F401

__all__ = ["Plan", "Workspace", "solve_batched", "pass_batched", "workspace_bytes", "plan_resident_bytes",
           "PspfftError",
           "PASS_NAMES", "PASS_X_FWD", "PASS_Y_FWD", "PASS_Z_CONV", "PASS_Y_INV", "PASS_X_INV",
           "set_verbosity", "get_verbosity", "set_log_callback",
           "CONSOLE_ERROR", "CONSOLE_WARNING", "CONSOLE_INFO_1", "CONSOLE_INFO_2"]


def _prec(dtype) -> int:
    if dtype == torch.float32:
        return _lib.PSPFFT_FP32
    if dtype == torch.float64:
        return _lib.PSPFFT_FP64
    raise TypeError(f"unsupported dtype {dtype}; use torch.float32 or torch.float64")


def _stream_handle(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def workspace_bytes(nx: int, ny: int, nz: int, dtype=torch.float32) -> int:
    return int(_lib.load().pspfft_workspace_bytes(nx, ny, nz, _prec(dtype)))


def plan_resident_bytes(nx: int, ny: int, nz: int, dtype=torch.float32) -> int:
    """``pspfft_plan_resident_bytes``: device bytes a plan of this size keeps."""
    return int(_lib.load().pspfft_plan_resident_bytes(nx, ny, nz, _prec(dtype)))


PLAN_FIVE_PASS = 1  # pspfft_plan_flags


def set_verbosity(level: int) -> None:
    """``pspfft_set_verbosity``: process-wide message level (Sec. 3.2, VerbosityOption)."""
    _lib.check(_lib.load().pspfft_set_verbosity(int(level)), "pspfft_set_verbosity")


def get_verbosity() -> int:
    return int(_lib.load().pspfft_get_verbosity())


_log_cb = None  # keeps the ctypes callback alive while the library holds it


def set_log_callback(fn) -> None:
    """``pspfft_set_log_callback``: ``fn(level, message)`` receives the library's
    messages instead of stderr; ``None`` goes back to stderr."""
    global _log_cb
    lib = _lib.load()
    if fn is None:
        _lib.check(lib.pspfft_set_log_callback(ctypes.cast(None, _lib.LOG_FN), None), "pspfft_set_log_callback")
        _log_cb = None
        return
    cb = _lib.LOG_FN(lambda level, msg, _user: fn(int(level), msg.decode(errors="replace")))
    _lib.check(lib.pspfft_set_log_callback(cb, None), "pspfft_set_log_callback")
    _log_cb = cb


class Plan:
    """``pspfft_plan_create_ex`` / ``pspfft_destroy`` (the paper's Create / Destroy).

    ``five_pass=True`` keeps the five separate passes where the x and y
    transforms of a plane could otherwise share one kernel (``fused``).
    ``verbosity`` (one of the CONSOLE_* levels) is the plan's own message level,
    the paper's VerbosityOption of Create; by default the process-wide level.
    """

    def __init__(self, nx: int, ny: int, nz: int, h, dtype=torch.float32, five_pass: bool = False,
                 verbosity: int | None = None):
        lib = _lib.load()
        if isinstance(h, (int, float)):
            h = (float(h),) * 3
        self.shape = (int(nz), int(ny), int(nx))
        self.n = (int(nx), int(ny), int(nz))
        self.h = tuple(float(v) for v in h)
        self.dtype = dtype
        handle = ctypes.c_void_p()
        h3 = (ctypes.c_double * 3)(*self.h)
        flags = PLAN_FIVE_PASS if five_pass else 0
        if verbosity is not None:
            flags |= (int(verbosity) + 1) << _lib.PLAN_VERBOSITY_SHIFT
        _lib.check(lib.pspfft_plan_create_ex(int(nx), int(ny), int(nz), h3, _prec(dtype), flags,
                                             ctypes.byref(handle)),
                   f"pspfft_plan_create_ex({nx},{ny},{nz})")
        self._handle = handle.value
        self._lib = lib
        self.fused = bool(lib.pspfft_plan_fused(self._handle))
        self.spectrum_kz_fastest = bool(lib.pspfft_plan_spectrum_kz_fastest(self._handle))
        self.ztile = int(lib.pspfft_workspace_ztile(self._handle))  # z planes per workspace tile
        # passes that launch work for this plan (a fused plan skips the y passes)
        self.active_passes = tuple(p for p in range(5) if lib.pspfft_pass_bytes(self._handle, p) > 0)

    @property
    def handle(self) -> int:
        if not self._handle:
            raise RuntimeError("plan already destroyed")
        return self._handle

    def close(self) -> None:
        if getattr(self, "_handle", None):
            _lib.check(self._lib.pspfft_destroy(self._handle), "pspfft_destroy")
            self._handle = None

    def __del__(self):  # pragma: no cover - interpreter teardown order varies
        try:
            self.close()
        except Exception:
            pass

    @property
    def resident_bytes(self) -> int:
        return int(self._lib.pspfft_plan_bytes(self.handle))

    @property
    def workspace_bytes(self) -> int:
        nx, ny, nz = self.n
        return int(self._lib.pspfft_workspace_bytes(nx, ny, nz, _prec(self.dtype)))

    def pass_bytes(self, which: int) -> int:
        return int(self._lib.pspfft_pass_bytes(self.handle, int(which)))

    def solve_bytes(self) -> int:
        return sum(self.pass_bytes(p) for p in range(5))

    def check_field(self, t: torch.Tensor, name: str) -> None:
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
            raise TypeError(f"{name} must be a cuda tensor")
        if t.dtype != self.dtype:
            raise TypeError(f"{name} has dtype {t.dtype}, plan uses {self.dtype}")
        if tuple(t.shape) != self.shape or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {self.shape}, got {tuple(t.shape)}")

    def solve(self, S: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """``pspfft_solve``: potential of S; ``out`` may be S itself (in place)."""
        self.check_field(S, "S")
        if out is None:
            out = torch.empty_like(S)
        self.check_field(out, "out")
        _lib.check(self._lib.pspfft_solve(self.handle, S.data_ptr(), out.data_ptr(), _stream_handle(stream)),
                   "pspfft_solve")
        return out

    def workspace(self) -> "Workspace":
        return Workspace(self)

    def green(self, stream=None) -> torch.Tensor:
        """The resident spectrum octant, shape (nz+1, ny+1, nx+1), plan dtype."""
        nx, ny, nz = self.n
        dst = torch.empty((nz + 1, ny + 1, nx + 1), dtype=self.dtype, device="cuda")
        _lib.check(self._lib.pspfft_plan_green(self.handle, dst.data_ptr(), _stream_handle(stream)),
                   "pspfft_plan_green")
        return dst


class Workspace:
    """One in-flight solve's buffer (``pspfft_workspace_create`` / ``_wrap``).

    With ``memory`` (a cuda tensor of at least ``plan.workspace_bytes`` bytes,
    256-byte aligned) the workspace wraps caller memory and the tensor is kept
    alive by this object.
    """

    def __init__(self, plan: Plan, memory: torch.Tensor | None = None):
        self.plan = plan
        self._lib = plan._lib
        handle = ctypes.c_void_p()
        self.memory = memory
        if memory is None:
            _lib.check(self._lib.pspfft_workspace_create(plan.handle, ctypes.byref(handle)),
                       "pspfft_workspace_create")
        else:
            nbytes = memory.numel() * memory.element_size()
            _lib.check(self._lib.pspfft_workspace_wrap(plan.handle, memory.data_ptr(), nbytes,
                                                       ctypes.byref(handle)), "pspfft_workspace_wrap")
        self._handle = handle.value

    @property
    def handle(self) -> int:
        if not self._handle:
            raise RuntimeError("workspace already destroyed")
        return self._handle

    def close(self) -> None:
        if getattr(self, "_handle", None):
            _lib.check(self._lib.pspfft_workspace_destroy(self._handle), "pspfft_workspace_destroy")
            self._handle = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def solve(self, S: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        self.plan.check_field(S, "S")
        if out is None:
            out = torch.empty_like(S)
        self.plan.check_field(out, "out")
        _lib.check(self._lib.pspfft_solve_ws(self.plan.handle, self.handle, S.data_ptr(), out.data_ptr(),
                                             _stream_handle(stream)), "pspfft_solve_ws")
        return out


def _batch_args(workspaces: Sequence[Workspace], S, Phi):
    if S is not None and len(S) != len(workspaces):
        raise ValueError("S and workspaces differ in length")
    if Phi is not None and len(Phi) != len(workspaces):
        raise ValueError("Phi and workspaces differ in length")
    plans = _lib.ptr_array([w.plan.handle for w in workspaces])
    ws = _lib.ptr_array([w.handle for w in workspaces])
    s_arr = _lib.ptr_array([t.data_ptr() for t in S]) if S is not None else None
    p_arr = _lib.ptr_array([t.data_ptr() for t in Phi]) if Phi is not None else None
    return plans, ws, s_arr, p_arr


def solve_batched(workspaces: Sequence[Workspace], S: Sequence[torch.Tensor], Phi: Sequence[torch.Tensor],
                  stream=None) -> None:
    """``pspfft_solve_batched``: problem i uses workspaces[i] (and its plan), S[i], Phi[i]."""
    for w, s, p in zip(workspaces, S, Phi):
        w.plan.check_field(s, "S")
        w.plan.check_field(p, "Phi")
    plans, ws, s_arr, p_arr = _batch_args(workspaces, S, Phi)
    lib = _lib.load()
    _lib.check(lib.pspfft_solve_batched(len(workspaces), plans, ws, s_arr, p_arr, _stream_handle(stream)),
               "pspfft_solve_batched")


def pass_batched_ptrs(which: int, plans: Sequence[int], workspaces: Sequence[int], S: Sequence[int] | None,
                      Phi: Sequence[int] | None, stream_handle: int = 0) -> None:
    """``pspfft_pass_batched`` on raw handles and device pointers, for callers
    (the serving loop) that validated their tensors once when they took them."""
    lib = _lib.load()
    n = len(workspaces)
    _lib.check(lib.pspfft_pass_batched(int(which), n, _lib.ptr_array(plans), _lib.ptr_array(workspaces),
                                       _lib.ptr_array(S) if S is not None else None,
                                       _lib.ptr_array(Phi) if Phi is not None else None, stream_handle),
               f"pspfft_pass_batched({which})")


def pass_batched(which: int, workspaces: Sequence[Workspace], S=None, Phi=None, stream=None) -> None:
    """``pspfft_pass_batched``: one pass of the solve for every listed problem."""
    if which == PASS_X_FWD:
        for w, s in zip(workspaces, S):
            w.plan.check_field(s, "S")
    if which == PASS_X_INV:
        for w, p in zip(workspaces, Phi):
            w.plan.check_field(p, "Phi")
    plans, ws, s_arr, p_arr = _batch_args(workspaces, S, Phi)
    lib = _lib.load()
    _lib.check(lib.pspfft_pass_batched(int(which), len(workspaces), plans, ws, s_arr, p_arr,
                                       _stream_handle(stream)), f"pspfft_pass_batched({which})")
