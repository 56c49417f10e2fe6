"""Brute-force maximum-likelihood detection for tiny instances.

TEST INFRASTRUCTURE ONLY.

x_ML = argmin over s in O^U of ||y - H s||^2 (the problem that equalization-based
detection approximates, Section III-A), by enumerating all |O|^U candidates.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def alphabet(M: int) -> np.ndarray:
    L = int(round(math.sqrt(M)))
    kappa = math.sqrt(2.0 * (M - 1) / 3.0)
    lv = (2.0 * np.arange(L) - (L - 1)) / kappa
    return np.array([a + 1j * b for a in lv for b in lv])


def ml_detect(H, y, M: int) -> np.ndarray:
    H = np.asarray(H, dtype=np.complex128)
    y = np.asarray(y, dtype=np.complex128)
    U = H.shape[1]
    pts = alphabet(M)
    if len(pts) ** U > 70000:
        raise ValueError("instance too large for enumeration")
    best, arg = math.inf, None
    for cand in itertools.product(pts, repeat=U):
        s = np.array(cand)
        d = y - H @ s
        v = float(np.real(np.vdot(d, d)))
        if v < best:
            best, arg = v, s
    return arg
