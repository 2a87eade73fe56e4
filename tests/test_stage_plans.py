"""Stage plans of the host runtime, read from the INFO_2 messages that
pspfft_plan_create_ex prints before any device work (no GPU needed).

Every length 2^a 3^b 5^c gets a plan whose radices multiply to the line length:
the radix families (odd part 1, 3, 5, 9) split a doubled line of 2n points into
stages that all divide the family's element count (FP32 z lines of 2048 points
take the 32-family); the generic kernel takes the
largest of its radices that divides what is left (Sec. 2.2.2: the 1D transforms
of every axis; the stage plan is this implementation's)."""
import ctypes
import math
import re

import pytest

import paper_1106_0557_amd as ps
from paper_1106_0557_amd import _lib


def _plans(n, prec=0):
    lib = _lib.load()
    msgs = []
    ps.set_log_callback(lambda level, text: msgs.append(text))
    try:
        h3 = (ctypes.c_double * 3)(0.1, 0.1, 0.1)
        handle = ctypes.c_void_p()
        flags = (ps.CONSOLE_INFO_2 + 1) << _lib.PLAN_VERBOSITY_SHIFT
        st = lib.pspfft_plan_create_ex(n[0], n[1], n[2], h3, prec, flags, ctypes.byref(handle))
        if st == 0:
            lib.pspfft_destroy(handle.value)
    finally:
        ps.set_log_callback(None)
    out = {}
    for t in msgs:
        mt = re.match(r"\s*axis ([xyz]): n = (\d+), line of (\d+) points, stages (.+), (radix-family kernels|generic line kernel)", t)
        if mt:
            radices = [] if mt.group(4) == "none" else [int(v) for v in mt.group(4).split(" x ")]
            out[mt.group(1)] = (int(mt.group(2)), int(mt.group(3)), radices, mt.group(5).startswith("radix"))
    return out


def _smooth(n):
    for p in (2, 3, 5):
        while n % p == 0:
            n //= p
    return n == 1


@pytest.mark.parametrize("prec", [0, 1])
def test_every_size_gets_a_plan_whose_radices_multiply_to_the_line(prec):
    sizes = [n for n in range(1, 2049) if _smooth(n)]
    for k in range(0, len(sizes), 3):
        trio = tuple(sizes[k:k + 3]) + (1,) * (3 - len(sizes[k:k + 3]))
        plans = _plans(trio, prec)
        assert set(plans) == {"x", "y", "z"}, trio
        for axis, n in zip("xyz", trio):
            nn, L, radices, family = plans[axis]
            assert nn == n and L == (n if axis == "x" else 2 * n)
            assert math.prod(radices) == L, (axis, n, radices)
            assert len(radices) <= 10


def test_family_and_generic_stage_choices():
    p = _plans((240, 120, 60))
    assert p["x"] == (240, 240, [16, 15], False)       # generic: largest radix first
    assert p["y"] == (120, 240, [16, 15], False)
    assert p["z"] == (60, 120, [15, 8], False)
    p = _plans((128, 96, 576))
    assert p["x"] == (128, 128, [16, 8], True)          # family E = 16: radices divide 16
    assert p["y"] == (96, 192, [24, 8], True)           # family E = 24
    assert p["z"] == (576, 1152, [36, 4, 4, 2], True)   # family E = 36: 36, then 4s, then 2
    p = _plans((15, 1, 2), prec=1)
    assert p["x"] == (15, 15, [15], False)
    assert p["y"] == (1, 2, [2], False)                 # below every family's element count
    assert p["z"] == (2, 4, [4], False)
    # FP64 lines beyond the family limit (2 * 1152 points) run on the generic kernel
    p = _plans((16, 2048, 1536), prec=1)
    assert p["y"] == (2048, 4096, [16, 16, 16], False)
    assert p["z"] == (1536, 3072, [16, 16, 12], False)
    p = _plans((16, 2048, 1536), prec=0)
    assert p["y"][3] and p["z"][3]                       # FP32: families up to 2048
    # FP32 z lines of 2048 points: the 32-family (lines within one wavefront)
    assert _plans((16, 8, 512))["z"] == (512, 1024, [16, 16, 4], True)
    assert _plans((16, 8, 1024))["z"] == (1024, 2048, [32, 32, 2], True)
    assert _plans((16, 8, 512), prec=1)["z"] == (512, 1024, [16, 16, 4], True)
    assert _plans((16, 512, 8))["y"] == (512, 1024, [16, 16, 4], True)  # y lines keep the 16-family
    # unless a z line's block of 64 positions (64 * 2ny * nx values) reaches 4 GB
    assert _plans((2048, 2048, 1024))["z"] == (1024, 2048, [16, 16, 8], True)
