"""Gate matrices of the oracle (complex128).

Rotations follow exp(-i theta P / 2); P(lambda) = diag(1, e^{i lambda});
CPHASE(theta) = diag(1, 1, 1, e^{i theta}) (OpenQASM cu1/cp, as used by the
QFT ladder of the paper, Section "Quantum Fourier Transform").  Multi-qubit
matrices index rows with the first listed wire as the most significant bit.
"""
from __future__ import annotations

import cmath
import math

import numpy as np

I2 = np.eye(2, dtype=np.complex128)
X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
Z = np.array([[1, 0], [0, -1]], dtype=np.complex128)
H = np.array([[1, 1], [1, -1]], dtype=np.complex128) / math.sqrt(2.0)
S = np.array([[1, 0], [0, 1j]], dtype=np.complex128)
T = np.array([[1, 0], [0, cmath.exp(1j * math.pi / 4)]], dtype=np.complex128)
SX = np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]], dtype=np.complex128) / 2.0

PAULI = {"X": X, "Y": Y, "Z": Z}


def rx(t):
    c, s = math.cos(t / 2), math.sin(t / 2)
    return np.array([[c, -1j * s], [-1j * s, c]], dtype=np.complex128)


def ry(t):
    c, s = math.cos(t / 2), math.sin(t / 2)
    return np.array([[c, -s], [s, c]], dtype=np.complex128)


def rz(t):
    return np.array([[cmath.exp(-0.5j * t), 0], [0, cmath.exp(0.5j * t)]], dtype=np.complex128)


def phase(t):
    return np.array([[1, 0], [0, cmath.exp(1j * t)]], dtype=np.complex128)


def _pp_rot(P, t):
    """exp(-i t P (x) P / 2) for a Pauli P: cos(t/2) I - i sin(t/2) P (x) P."""
    PP = np.kron(P, P)
    return math.cos(t / 2) * np.eye(4, dtype=np.complex128) - 1j * math.sin(t / 2) * PP


def controlled(U):
    M = np.eye(4, dtype=np.complex128)
    M[2:, 2:] = U
    return M


CNOT = controlled(X)
CZ = np.diag([1, 1, 1, -1]).astype(np.complex128)
SWAP = np.array([[1, 0, 0, 0], [0, 0, 1, 0], [0, 1, 0, 0], [0, 0, 0, 1]], dtype=np.complex128)


def matrix(gate, params=None) -> np.ndarray:
    """Matrix of a :class:`workloads.Gate` (2^k x 2^k, wires in listed order)."""
    name = gate.name
    k = len(gate.wires)
    if name in ("MCZ", "MCP"):
        t = math.pi if name == "MCZ" else gate.angle(params)
        d = np.ones(1 << k, dtype=np.complex128)
        d[-1] = cmath.exp(1j * t)
        return np.diag(d)
    fixed = {"I": I2, "H": H, "X": X, "Y": Y, "Z": Z, "S": S, "SDG": S.conj().T,
             "T": T, "TDG": T.conj().T, "SX": SX, "CNOT": CNOT, "CZ": CZ, "SWAP": SWAP}
    if name in fixed:
        return fixed[name].copy()
    if name in ("U", "UNITARY"):
        d = 1 << k
        return np.asarray(gate.mat, dtype=np.complex128).reshape(d, d)
    if name == "CU":
        return controlled(np.asarray(gate.mat, dtype=np.complex128).reshape(2, 2))
    t = gate.angle(params)
    if name == "RX":
        return rx(t)
    if name == "RY":
        return ry(t)
    if name == "RZ":
        return rz(t)
    if name == "P":
        return phase(t)
    if name == "CPHASE":
        return np.diag([1, 1, 1, cmath.exp(1j * t)]).astype(np.complex128)
    if name == "RZZ":
        return _pp_rot(Z, t)
    if name == "RXX":
        return _pp_rot(X, t)
    if name == "RYY":
        return _pp_rot(Y, t)
    raise ValueError(f"unknown gate {name}")


def generator(gate):
    """Hermitian G with d/dtheta U(theta) = -i/2 * scale * G U (rotation gates),
    or None when the gate has no single-Pauli generator."""
    name = gate.name
    if name in ("RX", "RY", "RZ"):
        return PAULI[name[1]]
    if name in ("RZZ", "RXX", "RYY"):
        P = PAULI[name[1]]
        return np.kron(P, P)
    return None
