"""Test-side numpy interpreter of a described plan (``Plan.describe()``).

Applies the layers exactly as the plan states them -- tile passes round by
round, diagonal layers from their FP64 lookup tables, GF(2) gathers from
their row masks -- so the planner's rewrite can be checked against the
one-gate-at-a-time oracle on the CPU, without a GPU.  A QFT stage is a
butterfly on bit p, then a twiddle on the bit-p = 1 half; the twiddle is
formed the way the tile kernel forms it: a group factor (the index with the
round's four bits cleared) times the plan's in-round coefficient E[k] (k =
the round bits below the stage's register bit).  The group factor is
exp(i pi low / 2^p), low = the group index bits in [base, p), or, where the
plan flags the stage ``square``, the square of the previous stage's group
factor -- so a wrong flag, or a wrong E table, shows up here as a wrong
state.  Dense layers apply the matrix the plan carries; plain layers call the
oracle's gate application.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import statevec as sv


def _popc(x):
    return np.bitwise_count(x).astype(np.int64)


def diag_phase(d, n):
    I = np.arange(1 << n, dtype=np.uint64)
    lut = np.array([complex(a, b) for a, b in d["lut"]])
    ph = np.ones(1 << n, dtype=np.complex128)
    terms = d["lut_terms"]
    for tb, te, lb, ll in d["lut_groups"]:
        cnt = np.zeros(1 << n, dtype=np.int64)
        for form, shift, mask in terms[tb:te]:
            m = np.uint64(mask)
            s = np.uint64(shift)
            if form == 0:
                cnt += _popc(I & m)
            elif form == 1:
                cnt += _popc((I ^ (I >> s)) & m)
            elif form == 2:
                cnt += _popc((I & (I >> s)) & m)
            elif form == 3:
                cnt += _popc(I & m) & 1
            else:
                cnt += ((I & m) == m).astype(np.int64)
        assert cnt.max() < ll
        ph *= lut[lb + cnt]
    return ph


def apply_bit_2x2(psi, n, b, U):
    v = psi.reshape(1 << (n - 1 - b), 2, 1 << b)
    x = v[:, 0, :].copy()
    y = v[:, 1, :].copy()
    v[:, 0, :] = U[0][0] * x + U[0][1] * y
    v[:, 1, :] = U[1][0] * x + U[1][1] * y


def apply_dense(psi, n, bits, U):
    idx = np.arange(1 << n, dtype=np.int64)
    tmask = sum(1 << b for b in bits)
    base = idx[(idx & tmask) == 0]
    offs = np.array([sum(((r >> u) & 1) << b for u, b in enumerate(bits)) for r in range(len(U))], np.int64)
    pos = base[None, :] + offs[:, None]
    out = psi.copy()
    out[pos] = U @ psi[pos]
    return out


def apply_layer(psi, n, L, stream, params):
    k = L["kind"]
    if k == "diag":
        ph = diag_phase(L["diag"], n)
        return psi * (np.conj(ph) if L.get("inverse") else ph)
    if k == "gf2":
        rows = [np.uint64(r) for r in L["rows"]]
        y = np.arange(1 << n, dtype=np.uint64)
        src = np.zeros_like(y)
        for r, row in enumerate(rows):
            src |= (_popc(y & row) & 1).astype(np.uint64) << np.uint64(r)
        src ^= np.uint64(L["cprime"])
        return psi[src.astype(np.int64)]
    if k == "dense":
        # the plan's own matrix: index bit u of rows and columns on bits[u]
        U = np.array([complex(a, b) for a, b in L["mat"]])
        K = int(round(math.sqrt(U.size)))
        return apply_dense(psi, n, L["bits"], U.reshape(K, K))
    if k == "plain":
        g = stream[L["gate"]]
        if L.get("inverse"):
            from oracle import gates as og
            U = og.matrix(g, params).conj().T
            from workloads import G
            g = G("U" if len(g.wires) == 1 else "UNITARY", *g.wires, mat=U)
        return sv.apply_gate(psi, n, g, params)
    assert k == "tile"
    psi = psi.copy()
    r2 = 1 / math.sqrt(2)
    i = np.arange(1 << n, dtype=np.int64)
    for R in L["rounds"]:
        if R["diag"] >= 0:
            ph = diag_phase(L["diags"][R["diag"]], n)
            psi *= np.conj(ph) if L.get("inverse") else ph
        sbits = [tb if tb < L["L"] else L["a"] + (tb - L["L"]) for tb in R["tbits"]]
        g = i & ~sum(1 << sb for sb in sbits)
        w_prev = None
        for op in L["ops"][R["ops"][0]:R["ops"][1]]:
            b = op["bit"]
            c = [complex(a, bb) for a, bb in op.get("coef", [])]
            if op["kind"] == 0:
                apply_bit_2x2(psi, n, b, [[c[0], c[1]], [c[2], c[3]]])
            elif op["kind"] == 3:
                apply_bit_2x2(psi, n, b, [[c[0], 0], [0, c[1]]])
            elif op["kind"] == 1:
                apply_bit_2x2(psi, n, b, [[r2, r2], [r2, -r2]])
            elif op["kind"] in (2, 4):
                base = op.get("base", 0)
                sel = ((i >> b) & 1) == 1
                if c:
                    if op["square"]:
                        assert w_prev is not None, "square flag on a round's first stage"
                        w = w_prev * w_prev
                    else:
                        w = np.exp(1j * math.pi * (g & ((1 << b) - 1) & ~((1 << base) - 1)) / (1 << b))
                    w_prev = w
                    kk = np.zeros_like(i)
                    for r in range(op["rbit"]):
                        kk |= ((i >> sbits[r]) & 1) << r
                    tw = w * np.array(c)[kk]
                else:  # unbound plan: the plain stage definition
                    tw = np.exp(1j * math.pi * (i & ((1 << b) - 1) & ~((1 << base) - 1)) / (1 << b))
                if op["kind"] == 2:
                    apply_bit_2x2(psi, n, b, [[r2, r2], [r2, -r2]])
                    psi[sel] *= tw[sel]
                else:  # inverse QFT stage: undo the twiddle, then the butterfly
                    psi[sel] *= np.conj(tw[sel])
                    apply_bit_2x2(psi, n, b, [[r2, r2], [r2, -r2]])
            else:
                raise AssertionError(f"unexpected op kind {op['kind']}")
    return psi


def run_plan(desc, psi0, stream, params=None):
    n = desc["n"]
    psi = np.array(psi0, dtype=np.complex128, copy=True)
    for L in desc["layers"]:
        psi = apply_layer(psi, n, L, stream, params)
    return psi
