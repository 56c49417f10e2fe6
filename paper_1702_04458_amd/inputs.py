"""Seeded synthetic inputs for massive MU-MIMO uplink detection and downlink precoding.

This module holds only the input recipe, shared by the GPU path, its tests and the
CPU oracle. It contains none of the detection or precoding arithmetic.

Recipe (system model of Section II, with synthetic statistics in place of the
paper's WINNER-II channels, which are not available):

* Channel ``H`` (uplink layout ``[n_sc][B][U]``): i.i.d. CN(0, 1) entries, i.e.
  real and imaginary parts N(0, 1/2), independent across antennas, users and
  subcarriers.  Optional base-station-side exponential correlation with
  coefficient ``a``: along the antenna index, per user column,
  ``h_1 = w_1`` and ``h_i = a h_{i-1} + sqrt(1 - a^2) w_i``, which gives
  ``E[h_i conj(h_j)] = a^|i-j|``.
* Symbols ``s``: uniform over the unit-energy square Gray M-QAM alphabet
  (``Es = 1``).  Levels per dimension are ``(2 i - (L - 1)) / kappa`` with
  ``L = sqrt(M)`` and ``kappa = sqrt(2 (M - 1) / 3)``.
* Noise: CN(0, N0) per receive antenna with ``N0 = U * Es / SNR`` (the SNR is
  the average receive SNR per antenna: with E|h|^2 = 1 the per-antenna receive
  power is ``U * Es``).
* Uplink receive vector ``y = H s + n`` (Section II-A, uplink model).
* Downlink targets: 64-QAM (or any M-QAM) symbols ``s`` per subcarrier, no noise.

Everything is produced by ``numpy.random.Generator(PCG64(seed))`` so the same
seed gives the same arrays on every machine.  Arrays handed to both sides are
complex64; the oracle upcasts them to complex128 itself.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

QAM_ORDERS = (4, 16, 64)


def frame_seed(config_id: int, frame_id: int = 0, snr_db: float = 0.0) -> int:
    """Seed formula used by the tests and the bench: distinct per config, frame and SNR."""
    return 1_000_003 * int(config_id) + 7919 * int(frame_id) + int(round(snr_db))


def qam_side(M: int) -> int:
    if M not in QAM_ORDERS:
        raise ValueError(f"unsupported QAM order {M}")
    return int(round(math.sqrt(M)))


def qam_kappa(M: int) -> float:
    """Normalisation that makes the square M-QAM alphabet unit-energy."""
    return math.sqrt(2.0 * (M - 1) / 3.0)


def qam_points(iI: np.ndarray, iQ: np.ndarray, M: int) -> np.ndarray:
    """Map per-dimension level indices to complex constellation points (complex128)."""
    L = qam_side(M)
    k = qam_kappa(M)
    return ((2 * iI - (L - 1)) + 1j * (2 * iQ - (L - 1))) / k


def _cn(rng: np.random.Generator, shape, var: float = 1.0) -> np.ndarray:
    sd = math.sqrt(var / 2.0)
    return sd * rng.standard_normal(shape) + 1j * sd * rng.standard_normal(shape)


def rayleigh_channel(rng: np.random.Generator, n_sc: int, B: int, U: int,
                     corr: float = 0.0) -> np.ndarray:
    """[n_sc][B][U] complex128 channel; ``corr`` > 0 adds antenna-side AR(1) correlation."""
    W = _cn(rng, (n_sc, B, U))
    if corr == 0.0:
        return W
    a = float(corr)
    H = np.empty_like(W)
    H[:, 0, :] = W[:, 0, :]
    g = math.sqrt(1.0 - a * a)
    for i in range(1, B):
        H[:, i, :] = a * H[:, i - 1, :] + g * W[:, i, :]
    return H


@dataclass
class UplinkFrame:
    H: np.ndarray        # [n_sc][B][U] complex64
    y: np.ndarray        # [n_sc][n_sym][B] complex64
    s: np.ndarray        # [n_sc][n_sym][U] complex128 transmitted symbols
    idx: np.ndarray      # [n_sc][n_sym][U] uint8 transmitted QAM index iI + L*iQ
    N0: float
    Es: float
    qam: int
    snr_db: float


@dataclass
class DownlinkFrame:
    H: np.ndarray        # [n_sc][B][U] complex64, uplink layout (H^d = H^T by reciprocity)
    s: np.ndarray        # [n_sc][n_sym][U] complex64 precoder targets
    qam: int


def uplink_frame(seed: int, n_sc: int, B: int, U: int, qam: int, snr_db: float,
                 n_sym: int = 1, corr: float = 0.0) -> UplinkFrame:
    rng = np.random.Generator(np.random.PCG64(seed))
    H = rayleigh_channel(rng, n_sc, B, U, corr).astype(np.complex64)
    L = qam_side(qam)
    iI = rng.integers(0, L, size=(n_sc, n_sym, U))
    iQ = rng.integers(0, L, size=(n_sc, n_sym, U))
    s = qam_points(iI, iQ, qam)
    Es = 1.0
    N0 = U * Es / (10.0 ** (snr_db / 10.0))
    n = _cn(rng, (n_sc, n_sym, B), N0)
    Hd = H.astype(np.complex128)
    y = np.einsum("kbu,knu->knb", Hd, s) + n
    idx = (iI + L * iQ).astype(np.uint8)
    return UplinkFrame(H=H, y=y.astype(np.complex64), s=s, idx=idx, N0=float(N0),
                       Es=Es, qam=qam, snr_db=float(snr_db))


def downlink_frame(seed: int, n_sc: int, B: int, U: int, qam: int = 64,
                   n_sym: int = 1, corr: float = 0.0) -> DownlinkFrame:
    rng = np.random.Generator(np.random.PCG64(seed))
    H = rayleigh_channel(rng, n_sc, B, U, corr).astype(np.complex64)
    L = qam_side(qam)
    iI = rng.integers(0, L, size=(n_sc, n_sym, U))
    iQ = rng.integers(0, L, size=(n_sc, n_sym, U))
    s = qam_points(iI, iQ, qam).astype(np.complex64)
    return DownlinkFrame(H=H, s=s, qam=qam)


# Valid serving shapes: (B, U, C) with B in {64,128,256,512}, U in {8,16,32,64},
# C in {4,8,16} and U <= S = B / C.
def serving_shapes():
    out = []
    for B in (64, 128, 256, 512):
        for U in (8, 16, 32, 64):
            for C in (4, 8, 16):
                if B % C == 0 and U <= B // C:
                    out.append((B, U, C))
    return out
