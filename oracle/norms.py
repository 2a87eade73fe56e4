"""Error measures (test infrastructure only).

``l1`` is the paper's L1 error norm, Eq. (L1-Norm_Error) of Sec. 4.1: the sum of
absolute differences over all cells divided by the sum of absolute reference
values.  ``rel_l2`` and ``rel_max`` are normwise: max|d| / max|ref|, so that cells
where the reference is near zero do not dominate.
"""
from __future__ import annotations

import numpy as np


def l1(phi, ref) -> float:
    phi = np.asarray(phi, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(phi - ref).sum() / np.abs(ref).sum())


def rel_l2(phi, ref) -> float:
    phi = np.asarray(phi, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm((phi - ref).ravel()) / np.linalg.norm(ref.ravel()))


def rel_max(phi, ref) -> float:
    phi = np.asarray(phi, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(phi - ref).max() / np.abs(ref).max())


def report(phi, ref) -> dict:
    return {"l1": l1(phi, ref), "rel_l2": rel_l2(phi, ref), "rel_max": rel_max(phi, ref)}
