"""Accuracy metrics in FP64.

Infidelity is the normalised form 1 - |<a|b>|^2 / (|a|^2 |b|^2), evaluated
without cancellation: with unit vectors a^, b^ and phi = arg <a^|b^>,
D = || b^ - e^{i phi} a^ ||^2 = 2 - 2 |<a^|b^>|, hence
1 - F = 1 - (1 - D/2)^2 = D (1 - D/4).  D is a sum of small squares, so it
stays accurate far below 1e-16 (needed for the complex128 comparison).  The
paper's complex64 QFT check reports an unnormalised value dominated by norm
drift (Section "Independent complex128 validation"); norm drift is therefore
reported separately.
"""
from __future__ import annotations

import cmath
import math

import numpy as np

_CHUNK = 1 << 20


def _fsum_sq(v: np.ndarray) -> float:
    """Compensated sum of |v|^2: pairwise numpy sums per chunk, exact fsum
    across chunks."""
    parts = []
    for s in range(0, v.size, _CHUNK):
        c = v[s:s + _CHUNK]
        parts.append(float(np.sum(c.real * c.real + c.imag * c.imag)))
    return math.fsum(parts)


def norm2(a: np.ndarray) -> float:
    return _fsum_sq(np.asarray(a, dtype=np.complex128))


def infidelity(a: np.ndarray, b: np.ndarray) -> float:
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    na, nb = math.sqrt(norm2(a)), math.sqrt(norm2(b))
    ah, bh = a / na, b / nb
    ov = np.vdot(ah, bh)
    ph = cmath.exp(1j * cmath.phase(ov)) if abs(ov) > 0 else 1.0
    D = _fsum_sq(bh - ph * ah)
    return max(0.0, D * (1.0 - D / 4.0))


def norm_drift(a: np.ndarray) -> float:
    return abs(norm2(a) - 1.0)


def l2(a: np.ndarray, b: np.ndarray) -> float:
    """|| a - b || without phase alignment."""
    return math.sqrt(_fsum_sq(np.asarray(a, np.complex128) - np.asarray(b, np.complex128)))


def prob_mae(a: np.ndarray, b: np.ndarray) -> float:
    return float(np.mean(np.abs(np.abs(a) ** 2 - np.abs(b) ** 2)))
