"""Read-out of a state: marginal distributions and inverse-CDF shot sampling.

TEST INFRASTRUCTURE ONLY (see the package header).

Measurement in the computational basis (paper, Sections "State Management"
and "Algorithm Implementations", where sampling and marginal probabilities
are read from the final state) draws index i with probability
p_i = |psi_i|^2 / ||psi||^2.  For a uniform number u in [0, 1) the inverse
CDF picks the first i whose cumulative mass sum_{j <= i} |psi_j|^2 exceeds
u ||psi||^2; a marginal over a subset S of the qubits sums p over every
assignment of the other qubits.  Both are written here as those definitions:
a sequential FP64 cumulative sum and a sum over tensor axes.
"""
from __future__ import annotations

from typing import Sequence

import numpy as np


def cumulative_mass(psi: np.ndarray) -> np.ndarray:
    """C_i = sum_{j <= i} |psi_j|^2, in FP64, in index order."""
    p = np.abs(np.asarray(psi, dtype=np.complex128)) ** 2
    return np.cumsum(p)


def inverse_cdf_sample(psi: np.ndarray, u: Sequence[float]) -> np.ndarray:
    """For each u in [0, 1): the first index i with C_i > u C_{N-1}."""
    C = cumulative_mass(psi)
    t = np.asarray(u, dtype=np.float64) * C[-1]
    return np.searchsorted(C, t, side="right").astype(np.uint64)


def marginal(psi: np.ndarray, n: int, qubits: Sequence[int]) -> np.ndarray:
    """Unnormalised marginal sum of |psi|^2 over the qubits not listed.

    Qubit q is axis q of the C-order tensor view (MSB-first); the result is
    indexed by the listed qubits in increasing order, the lowest-numbered one
    most significant."""
    sel = sorted(set(int(q) for q in qubits))
    p = (np.abs(np.asarray(psi, dtype=np.complex128)) ** 2).reshape((2,) * n)
    other = tuple(a for a in range(n) if a not in sel)
    return np.sum(p, axis=other).reshape(-1) if other else p.reshape(-1)
