"""Per-amplitude definitions for sampled checks at full size.

At 30 qubits a dense host reference is impractical, but three of the path's
layers have plain per-output definitions that cost O(k) for a k-sparse input:

* QFT (Section "Quantum Fourier Transform"): QFT|j> = N^{-1/2} sum_k
  e^{2 pi i j k / N} |k>; the gate stream carries no final swaps, so the
  amplitude of k appears at index rev_n(k).
* Walsh layer H^{(x)n} (Appendix A, the H^{(x)4} closed form extended to n
  qubits): <y|H^n|j> = N^{-1/2} (-1)^{popcount(j AND y)}.
* QFT followed by the Walsh layer (the composed circuit of the state-vector
  benchmark): with u = rev_n(y), <y|H^n QFT|j> = N^{-1} sum_k
  (-1)^{popcount(u AND k)} e^{2 pi i j k / N}, and the sum over the bits of k
  factorises into prod_b (1 + (-1)^{u_b} e^{2 pi i j 2^b / N}).
* X/CNOT/SWAP blocks (Section "Kernel Taxonomy", GF(2) affine gathers): the
  output amplitude at y is the input amplitude at the index obtained by
  pushing y back through the gates in reverse order (each is an
  involution), one gate at a time on the integer index.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np


def bit_reverse(x: np.ndarray, n: int) -> np.ndarray:
    x = np.asarray(x, dtype=np.uint64)
    r = np.zeros_like(x)
    for b in range(n):
        r |= ((x >> np.uint64(b)) & np.uint64(1)) << np.uint64(n - 1 - b)
    return r


def qft_sparse(n: int, idx: np.ndarray, coeffs: np.ndarray, ys: np.ndarray) -> np.ndarray:
    """Output amplitudes at indices ``ys`` of the QFT stream applied to
    sum_k coeffs[k] |idx[k]>."""
    N = 1 << n
    ks = bit_reverse(ys, n)
    out = np.zeros(len(ys), dtype=np.complex128)
    for j, c in zip(np.asarray(idx, dtype=np.uint64), coeffs):
        # (j * k) mod N exactly, in integers (N <= 2^32, products < 2^64)
        m = (np.uint64(j) * ks) & np.uint64(N - 1)
        ang = (2.0 * math.pi / N) * m.astype(np.float64)
        out += c * np.exp(1j * ang)
    return out / math.sqrt(N)


def popcount_parity(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.uint64).copy()
    p = np.zeros_like(x)
    while np.any(x):
        p ^= x & np.uint64(1)
        x >>= np.uint64(1)
    return p


def wht_sparse(n: int, idx: np.ndarray, coeffs: np.ndarray, ys: np.ndarray) -> np.ndarray:
    out = np.zeros(len(ys), dtype=np.complex128)
    ys = np.asarray(ys, dtype=np.uint64)
    for j, c in zip(np.asarray(idx, dtype=np.uint64), coeffs):
        sign = 1.0 - 2.0 * popcount_parity(ys & np.uint64(j)).astype(np.float64)
        out += c * sign
    return out / math.sqrt(1 << n)


def qft_wht_sparse(n: int, idx: np.ndarray, coeffs: np.ndarray, ys: np.ndarray) -> np.ndarray:
    """Output amplitudes at ``ys`` of the QFT stream followed by the Walsh
    layer, applied to sum_k coeffs[k] |idx[k]> (product form above)."""
    N = 1 << n
    u = bit_reverse(ys, n)
    out = np.zeros(len(ys), dtype=np.complex128)
    for j, c in zip(np.asarray(idx, dtype=np.uint64), coeffs):
        prod = np.ones(len(ys), dtype=np.complex128)
        for b in range(n):
            # (j * 2^b) mod N exactly in integers
            m = (int(j) << b) & (N - 1)
            e = np.exp(2j * math.pi * m / N)
            sign = 1.0 - 2.0 * ((u >> np.uint64(b)) & np.uint64(1)).astype(np.float64)
            prod *= 1.0 + sign * e
        out += c * prod
    return out / N


def perm_source(n: int, stream: Sequence, ys: np.ndarray) -> np.ndarray:
    """Source index src(y) with out[y] = in[src(y)] for an X/CNOT/SWAP stream.

    Qubit q is bit n-1-q.  Gates are replayed on the index in reverse order.
    """
    y = np.array(ys, dtype=np.uint64, copy=True)
    one = np.uint64(1)
    for g in reversed(list(stream)):
        if g.name == "X":
            y ^= one << np.uint64(n - 1 - g.wires[0])
        elif g.name == "CNOT":
            c, t = (np.uint64(n - 1 - w) for w in g.wires)
            y ^= ((y >> c) & one) << t
        elif g.name == "SWAP":
            a, b = (np.uint64(n - 1 - w) for w in g.wires)
            d = ((y >> a) ^ (y >> b)) & one
            y ^= (d << a) | (d << b)
        else:
            raise ValueError(f"{g.name} is not a permutation gate")
    return y
