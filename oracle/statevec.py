"""One-gate-at-a-time complex128 state-vector evaluation.

A state of n qubits is a flat complex128 array of length 2^n; qubit q is
index bit n-1-q (MSB-first), so the C-order tensor view of shape (2,)*n has
qubit q on axis q.  Single-qubit gates use the (A, 2, B) slice update of the
paper's pure tier (Appendix A, "The pure-MLX path"); diagonal gates multiply
by a broadcast phase tensor; other multi-qubit gates are contracted with
numpy.tensordot (Section "Gate Operations": reshape, contract, flatten).
"""
from __future__ import annotations

from typing import Iterable, List, Optional, Sequence

import numpy as np

from . import gates as _g

DIAGONAL = {"I", "Z", "S", "SDG", "T", "TDG", "RZ", "P", "CZ", "CPHASE", "RZZ", "MCZ", "MCP"}


def basis(n: int, index: int) -> np.ndarray:
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[index] = 1.0
    return psi


def plus(n: int) -> np.ndarray:
    return np.full(1 << n, (1 << n) ** -0.5, dtype=np.complex128)


def apply_1q(psi: np.ndarray, n: int, U: np.ndarray, q: int) -> np.ndarray:
    """In place: view the state as (2^q, 2, 2^(n-1-q)); axis 1 is qubit q."""
    v = psi.reshape(1 << q, 2, 1 << (n - 1 - q))
    s0 = v[:, 0, :].copy()
    s1 = v[:, 1, :].copy()
    v[:, 0, :] = U[0, 0] * s0 + U[0, 1] * s1
    v[:, 1, :] = U[1, 0] * s0 + U[1, 1] * s1
    return psi


def apply_diag(psi: np.ndarray, n: int, d: np.ndarray, wires: Sequence[int]) -> np.ndarray:
    """In place: multiply by a diagonal given on the listed wires."""
    k = len(wires)
    dd = np.asarray(d, dtype=np.complex128).reshape((2,) * k)
    order = np.argsort(np.asarray(wires))
    dd = np.transpose(dd, order)
    shape = [1] * n
    for w in wires:
        shape[w] = 2
    t = psi.reshape((2,) * n)
    t *= dd.reshape(shape)
    return psi


def apply_kq(psi: np.ndarray, n: int, U: np.ndarray, wires: Sequence[int]) -> np.ndarray:
    """Contract a 2^k x 2^k matrix with the listed axes; returns a new array."""
    k = len(wires)
    t = psi.reshape((2,) * n)
    Ut = np.asarray(U, dtype=np.complex128).reshape((2,) * (2 * k))
    out = np.tensordot(Ut, t, axes=(list(range(k, 2 * k)), list(wires)))
    out = np.moveaxis(out, list(range(k)), list(wires))
    return np.ascontiguousarray(out).reshape(-1)


def check_wires(n: int, wires: Sequence[int]) -> None:
    if len(set(wires)) != len(wires) or any(w < 0 or w >= n for w in wires):
        raise ValueError(f"bad wires {tuple(wires)} for n={n}")


def apply_gate(psi: np.ndarray, n: int, gate, params=None) -> np.ndarray:
    """Apply one gate; returns the (possibly new) state array."""
    check_wires(n, gate.wires)
    U = _g.matrix(gate, params)
    if gate.name in DIAGONAL:
        return apply_diag(psi, n, np.diagonal(U), gate.wires)
    if len(gate.wires) == 1:
        return apply_1q(psi, n, U, gate.wires[0])
    return apply_kq(psi, n, U, gate.wires)


def run(psi0: np.ndarray, n: int, stream: Iterable, params=None) -> np.ndarray:
    """U_G ... U_1 psi0 (copy of psi0, upcast to complex128)."""
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    for g in stream:
        psi = apply_gate(psi, n, g, params)
    return psi


def apply_pauli(psi: np.ndarray, n: int, x_mask: int, z_mask: int) -> np.ndarray:
    """P psi for P = prod_q sigma_q with sigma = X (x bit), Z (z bit), Y (both);
    masks use qubit numbering (bit q = qubit q)."""
    out = np.array(psi, dtype=np.complex128, copy=True)
    for q in range(n):
        xb, zb = (x_mask >> q) & 1, (z_mask >> q) & 1
        if xb and zb:
            out = apply_1q(out, n, _g.Y, q)
        elif xb:
            out = apply_1q(out, n, _g.X, q)
        elif zb:
            out = apply_1q(out, n, _g.Z, q)
    return out


def expect_terms(psi: np.ndarray, n: int, terms) -> np.ndarray:
    """Per-term c_t <psi|P_t|psi> (real part; P_t Hermitian)."""
    out = np.empty(len(terms), dtype=np.float64)
    for i, (c, xm, zm) in enumerate(terms):
        out[i] = c * np.vdot(psi, apply_pauli(psi, n, xm, zm)).real
    return out


def expect(psi: np.ndarray, n: int, terms) -> float:
    return float(np.sum(expect_terms(psi, n, terms)))


def apply_pauli_sum(psi: np.ndarray, n: int, terms) -> np.ndarray:
    """sum_t c_t P_t psi."""
    out = np.zeros_like(psi, dtype=np.complex128)
    for c, xm, zm in terms:
        out += c * apply_pauli(psi, n, xm, zm)
    return out


def probabilities(psi: np.ndarray) -> np.ndarray:
    return np.abs(psi) ** 2


def norm2(psi: np.ndarray) -> float:
    return float(np.vdot(psi, psi).real)


def inverse_stream(stream: Sequence, params=None) -> List:
    """Adjoint stream: reversed order, each gate replaced by its inverse given
    as an explicit matrix gate (used for the plan-then-inverse invariant)."""
    from workloads import G
    out = []
    for g in reversed(list(stream)):
        U = _g.matrix(g, params)
        Ud = U.conj().T
        name = "U" if len(g.wires) == 1 else "UNITARY"
        out.append(G(name, *g.wires, mat=Ud))
    return out
