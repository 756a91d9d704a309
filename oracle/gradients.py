"""Reference gradients of E(params) = <psi(params)|H|psi(params)>.

Parameter shift (Section "Algorithm Implementations": the variational
workload uses parameter-shift gradients) for gates whose generator has two
eigenvalues one apart in units of the angle (RX, RY, RZ, P, RZZ, RXX, RYY,
CPHASE, MCP): dE/dangle = [E(angle + pi/2) - E(angle - pi/2)] / 2, applied
per occurrence and multiplied by the occurrence's ``scale``.  Central finite
differences serve as a second, independent check.
"""
from __future__ import annotations

import math

import numpy as np

from workloads import Gate
from . import statevec as sv

SHIFTABLE = {"RX", "RY", "RZ", "P", "RZZ", "RXX", "RYY", "CPHASE", "MCP"}


def energy(n, stream, params, terms, psi0=None) -> float:
    psi0 = sv.basis(n, 0) if psi0 is None else psi0
    return sv.expect(sv.run(psi0, n, stream, params), n, terms)


def parameter_shift(n, stream, params, terms, psi0=None) -> np.ndarray:
    params = np.asarray(params, dtype=np.float64)
    stream = list(stream)
    grad = np.zeros(len(params))
    for pos, g in enumerate(stream):
        if g.param < 0:
            continue
        if g.name not in SHIFTABLE:
            raise ValueError(f"no shift rule for {g.name}")
        a = g.angle(params)
        vals = []
        for s in (+0.5 * math.pi, -0.5 * math.pi):
            mod = list(stream)
            mod[pos] = Gate(g.name, g.wires, a + s, -1, 1.0, g.mat)
            vals.append(energy(n, mod, params, terms, psi0))
        grad[g.param] += g.scale * 0.5 * (vals[0] - vals[1])
    return grad


def finite_differences(n, stream, params, terms, psi0=None, h: float = 1e-5) -> np.ndarray:
    params = np.asarray(params, dtype=np.float64)
    grad = np.zeros(len(params))
    for j in range(len(params)):
        p = params.copy()
        p[j] += h
        ep = energy(n, stream, p, terms, psi0)
        p[j] -= 2 * h
        em = energy(n, stream, p, terms, psi0)
        grad[j] = (ep - em) / (2 * h)
    return grad
