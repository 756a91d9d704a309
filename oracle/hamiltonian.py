"""Dense Pauli-sum Hamiltonians and exact time evolution (small n only).

Used for the Trotter-error reference of the paper (Section "Trotter Error":
dense complex128 evolution with scipy.linalg.expm) and for exact
diagonalisation checks at <= 12 qubits.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import gates as _g


def pauli_matrix(n: int, x_mask: int, z_mask: int) -> np.ndarray:
    """Dense 2^n x 2^n matrix of a Pauli string (bit q of the masks = qubit q).
    Qubit 0 is the leftmost Kronecker factor (MSB-first)."""
    M = np.ones((1, 1), dtype=np.complex128)
    for q in range(n):
        xb, zb = (x_mask >> q) & 1, (z_mask >> q) & 1
        f = _g.Y if (xb and zb) else _g.X if xb else _g.Z if zb else _g.I2
        M = np.kron(M, f)
    return M


def dense(n: int, terms) -> np.ndarray:
    Hm = np.zeros((1 << n, 1 << n), dtype=np.complex128)
    for c, xm, zm in terms:
        Hm += c * pauli_matrix(n, xm, zm)
    return Hm


def tfim_terms(n: int, J: float, h: float):
    """H = -J sum_{i<n-1} Z_i Z_{i+1} + h sum_i X_i (open chain)."""
    out = [(-J, 0, (1 << i) | (1 << (i + 1))) for i in range(n - 1)]
    out += [(h, 1 << i, 0) for i in range(n)]
    return out


def evolve(n: int, terms, t: float, psi0: np.ndarray) -> np.ndarray:
    """exp(-i H t) psi0 with a dense matrix exponential."""
    U = scipy.linalg.expm(-1j * t * dense(n, terms))
    return U @ np.asarray(psi0, dtype=np.complex128)


def ground_energy(n: int, terms) -> float:
    return float(np.linalg.eigvalsh(dense(n, terms))[0])
